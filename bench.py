#!/usr/bin/env python3
"""Throughput of the LJ velocity-Verlet step at one million atoms on one GPU.

Workload: LJ fluid, N = 1,000,000 on a jittered 100^3 lattice, rho = 0.8442,
T = 1, r_cut = 2.5 sigma (truncated), Verlet skin 0.3 sigma with rebuilds when
the largest displacement exceeds skin/2, dt = 0.005, periodic cube.  Inputs
are synthetic (seeded) and resident in device memory before timing starts.

One timed step = fused kick/drift with the displacement check, gated cell-list
and Verlet-list rebuild, LJ force/energy/virial, closing kick with kinetic
energy; all graph-launched.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "LJ atom-steps/s at 1M particles, %HBM roofline; batched & adjoint vs plain"
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "lj_step_lj1m_counters.txt")
# the sources the force kernel is compiled from
LJ_SOURCES = [os.path.join(ROOT, "paper_1804_07598_amd", "csrc", f)
              for f in ("lj.hip", "geom.h", "fpm_internal.h")]


def log(msg: str, quiet: bool):
    if not quiet:
        print(msg, file=sys.stderr, flush=True)


def source_hash(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(n_launch_atoms: int, unroll: int):
    """HBM bytes per launch of the fused step kernel with `unroll` list entries
    in flight, from the committed rocprofv3 counter summary, or None when the
    summary is missing, holds no figure for that unroll or atom count, or the
    kernel source changed since."""
    if not os.path.exists(PROFILE_COUNTERS):
        return None
    kv = {}
    for line in open(PROFILE_COUNTERS):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        if kv.get("kernel_source_sha256_16") != source_hash(LJ_SOURCES):
            return None
        if int(kv.get("atoms", "0")) != n_launch_atoms:
            return None
        return float(kv[f"hbm_bytes_per_launch_unroll{unroll}"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pos, box, target_s: float, quiet: bool):
    """The FP64 O(N^2) oracle on a bounded sample: forces of R random atoms
    against all N atoms, timed on the host's cores (median of three timings of
    the same sample), plus the small configurations in full: the 4096-atom
    liquid's force evaluation and 10 velocity-Verlet steps, and one force
    evaluation of the 32,768-atom mixture."""
    import numpy as np
    import oracle as O
    from paper_1804_07598_amd import inputs
    rc2 = O.radius2(2.5)
    rng = np.random.default_rng(0)
    R = 64
    O.lj(pos, box, (1, 1, 1), rc2, rows=rng.choice(len(pos), R, replace=False))  # warm
    per_run = target_s / 3.0
    while True:
        rows = rng.choice(len(pos), R, replace=False)
        t0 = time.perf_counter()
        O.lj(pos, box, (1, 1, 1), rc2, rows=rows)
        dt = time.perf_counter() - t0
        if dt >= per_run or R >= len(pos):
            break
        R = min(len(pos), max(R * 2, int(R * per_run / max(dt, 1e-3) * 1.1)))
        log(f"cpu baseline: trying {R} rows", quiet)
    times = [dt]
    for _ in range(2):
        t0 = time.perf_counter()
        O.lj(pos, box, (1, 1, 1), rc2, rows=rows)
        times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    # the 4096-atom case in full: one evaluation and 10 steps (11 evaluations)
    s1 = inputs.lj_config("lj4096")
    t0 = time.perf_counter()
    O.lj_traj(s1.pos, s1.vel, s1.box, (1, 1, 1), 2.5, 0.005, 10)
    t_cfg1 = time.perf_counter() - t0
    s5 = inputs.lj_lattice(32768, 1.2, 1.0, 5, mixture=True)
    M = inputs.LJ_MIXTURE
    t0 = time.perf_counter()
    O.lj(s5.pos, s5.box, (1, 1, 1), rc2, M["eps"], M["sig"], s5.typ)
    t_cfg5 = time.perf_counter() - t0
    return {"value": R / med, "unit": "atom-steps/s", "cores": O.num_threads(), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{R} random atoms' LJ forces against all {len(pos)} atoms (FP32 predicate, "
                      f"FP64 physics) at the initial configuration; median of 3 timings "
                      f"({', '.join(f'{t:.1f}' for t in times)} s)",
            "full_cases": {
                "lj4k_1_eval_10_steps_s": t_cfg1,
                "lj4k_atom_steps_per_s": s1.n * 11 / t_cfg1,
                "mix32k_1_eval_s": t_cfg5,
                "mix32k_pair_tests_per_s": 32768.0 * 32768.0 / t_cfg5}}


def dem_cpu_baseline(s, oprm, target_s: float, quiet: bool):
    """The FP64 O(N^2) DEM oracle on a bounded sample: forces and torques of R
    random grains against all N grains (no contact history), on the host's
    cores."""
    import numpy as np
    import oracle as O
    rng = np.random.default_rng(1)
    x, v, w = s.pos.astype(np.float64), s.vel, s.omega
    R = 64
    O.dem_forces_rows(x, v, w, s.L, s.periodic, oprm, rng.choice(len(x), R, replace=False))
    while True:
        rows = rng.choice(len(x), R, replace=False)
        t0 = time.perf_counter()
        O.dem_forces_rows(x, v, w, s.L, s.periodic, oprm, rows)
        dt = time.perf_counter() - t0
        if dt >= target_s or R >= len(x):
            break
        R = min(len(x), max(R * 2, int(R * target_s / max(dt, 1e-3) * 1.1)))
        log(f"dem cpu baseline: trying {R} rows", quiet)
    return {"value": R / dt, "unit": "grain-steps/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{R} random grains' contact forces and torques against all {len(x)} "
                      f"grains (FP64) at the initial configuration; {dt:.1f} s"}


def copy_rate(dev, mib: int = 1024) -> float:
    """Achievable HBM rate: GB/s (read + written bytes) of a device-to-device
    copy of `mib` MiB, the best of five, HIP events."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    return 2.0 * 4 * n / (best / 1e3) / 1e9


def timed_steps(sim, nsteps, dt, warmup, eps=(1.0,) * 3, sig=(1.0,) * 3, n_types=1):
    """Milliseconds of nsteps graph-launched steps after warmup steps (HIP events
    on the stream the library launches on)."""
    import torch
    sim.step(warmup, dt, eps, sig, n_types)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.step(nsteps, dt, eps, sig, n_types)
    e1.record()
    torch.cuda.synchronize()
    sim.check()
    return e0.elapsed_time(e1)


def bench_symmetric(dev, nsteps: int, quiet: bool, plain_value: float):
    """The 1M-atom liquid with symmetric half lists (each pair evaluated once,
    reactions gathered in a second pass): step rate and both passes' time."""
    from paper_1804_07598_amd import _lib as F
    from paper_1804_07598_amd import inputs
    from paper_1804_07598_amd.sim import ParticleSim
    s = inputs.lj_config("lj1m")
    sim = ParticleSim(s.pos, s.box, (1, 1, 1), vel=s.vel, r_cut=2.5, skin=0.3, device=dev,
                      symmetric=True)
    ms = timed_steps(sim, nsteps, 0.005, 20)
    F.fpm_set_profiling(sim.ctx, True)
    for _ in range(20):
        sim.lj_forces()
    f_ms, _ = F.fpm_kernel_time(sim.ctx, "lj_force")
    F.fpm_kernel_time(sim.ctx, "cell_build")
    F.fpm_kernel_time(sim.ctx, "verlet_build")
    F.fpm_set_profiling(sim.ctx, False)
    sim.check()
    sim.close()
    value = s.n * nsteps / (ms / 1e3)
    log(f"symmetric lists: {ms / nsteps * 1e3:.1f} us/step ({value:.3g} atom-steps/s), "
        f"both passes {f_ms * 1e3:.1f} us", quiet)
    return {"workload": "lj1m with symmetric half lists (each pair once, reactions gathered)",
            "steps": nsteps, "value": value, "unit": "atom-steps/s",
            "ms_per_step": ms / nsteps, "force_passes_us": f_ms * 1e3,
            "vs_full_lists": value / plain_value}


def bench_batched(dev, nsteps: int, quiet: bool, tuning=None):
    """512 independent boxes of 256..8192 atoms stepped together, against one
    box holding the same total number of atoms (launch shapes from the
    autotuner, or `tuning` for both)."""
    import numpy as np
    from paper_1804_07598_amd import inputs
    from paper_1804_07598_amd.sim import BatchSim, ParticleSim
    ns, rhos, Ts = inputs.batched_table()
    systems = [inputs.batched_system(k, ns, rhos, Ts) for k in range(len(ns))]
    n = int(ns.sum())
    sim = BatchSim([s.pos for s in systems], [s.box for s in systems], (1, 1, 1),
                   vel_list=[s.vel for s in systems], r_cut=2.5, skin=0.3, device=dev)
    from paper_1804_07598_amd.tune import tune
    if tuning:
        knobs = tuning
        sim.set_tuning(*knobs)
    else:
        knobs, _ = tune(sim, float(np.mean(rhos)), cache=None)
    sim.step(20, 0.005)  # warm-up
    reb0 = sim.counters()[0]
    ms_b = timed_steps(sim, nsteps, 0.005, 0)
    reb_b = sim.counters()[0] - reb0  # over the timed steps, all systems
    sim.close()
    one = inputs.lj_lattice(n, float(np.mean(rhos)), float(np.mean(Ts)), 6)
    sim = ParticleSim(one.pos, one.box, (1, 1, 1), vel=one.vel, r_cut=2.5, skin=0.3,
                      max_nbr=184, device=dev)
    if tuning:
        sim.set_tuning(*tuning)
    else:
        tune(sim, float(np.mean(rhos)), cache=None)
    ms_p = timed_steps(sim, nsteps, 0.005, 20)
    sim.close()
    vb, vp = n * nsteps / (ms_b / 1e3), n * nsteps / (ms_p / 1e3)
    log(f"batched: {len(ns)} systems, {n} atoms, {ms_b / nsteps * 1e3:.1f} us/step "
        f"({vb:.3g} atom-steps/s); one box of {n}: {ms_p / nsteps * 1e3:.1f} us/step", quiet)
    return {"workload": f"{len(ns)} periodic LJ boxes, N_s uniform in [256, 8192], rho_s in "
                        "[0.6, 0.9], T_s in [0.8, 1.5], r_cut=2.5, skin=0.3, dt=0.005",
            "systems": len(ns), "atoms": n, "steps": nsteps, "value": vb, "unit": "atom-steps/s",
            "ms_per_step": ms_b / nsteps, "rebuilds": reb_b, "tuning": list(knobs),
            "plain_value": vp, "plain_workload": f"one box of {n} atoms at the mean rho and T",
            "vs_plain": vb / vp}


def bench_sph(dev, nsteps: int, quiet: bool):
    """Weakly compressible SPH water column: 128 x 128 x 128 fluid particles at
    dx = 0.01 on a 3-layer floor (N = 2,146,304), Wendland C2 with h = 1.3 dx,
    Tait EOS (c0 = 20 sqrt(g H), gamma = 7), alpha = 0.1, CFL 0.2."""
    import math
    import numpy as np
    import torch
    from paper_1804_07598_amd import _lib as F
    from paper_1804_07598_amd import inputs
    from paper_1804_07598_amd.sim import ParticleSim
    s = inputs.sph_column(128, 128)
    dx, H, g = s.dx, s.H, 9.81
    h = 1.3 * dx
    c0 = 20.0 * math.sqrt(g * H)
    prm = F.sph_params(h, 1000.0 * dx ** 3, 1000.0, c0, 7.0, 0.1, 0.01 * h * h, (0, 0, -g), 0.2)
    r_cut = float(np.float32(2 * h))
    sim = ParticleSim(s.pos, s.L, (1, 1, 0), vel=s.vel, typ=s.kind, r_cut=r_cut, skin=0.1 * h,
                      max_nbr=160, device=dev)
    sim.set_density(s.rho)
    sim.sph_step(20, prm)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    hist = sim.sph_step(nsteps, prm)
    e1.record()
    torch.cuda.synchronize()
    sim.check()
    ms = e0.elapsed_time(e1)
    F.fpm_set_profiling(sim.ctx, True)
    for _ in range(10):
        sim.sph_rates(prm)
    r_ms, _ = F.fpm_kernel_time(sim.ctx, "sph_rates")
    F.fpm_set_profiling(sim.ctx, False)
    reb, _, total = sim.counters()
    sim.close()
    n = len(s.pos)
    nbar = total / n
    bytes_rates = n * (52.0 + 4.0 * nbar)
    achieved = bytes_rates / (r_ms / 1e3) / 1e9
    t_sim = float(hist[-1, 0].item())
    log(f"sph: {n} particles, {ms / nsteps * 1e3:.1f} us/step, rates kernel {r_ms * 1e3:.1f} us "
        f"({achieved:.0f} GB/s), mean list {nbar:.1f}, simulated {t_sim:.4g} s", quiet)
    return {"workload": "SPH water column 128^3 fluid + 3-layer floor, N=2,146,304, dx=0.01, "
                        "Wendland C2 h=1.3dx, Tait gamma=7, c0=20 sqrt(gH), alpha=0.1, CFL 0.2",
            "particles": n, "steps": nsteps, "value": n * nsteps / (ms / 1e3),
            "unit": "particle-steps/s", "ms_per_step": ms / nsteps, "simulated_s": t_sim,
            "rates_kernel_us": r_ms * 1e3, "mean_list": nbar, "rebuilds": reb,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "bytes_model": "N*(52 + 4*nbar): pos, vel 32, count 4, list, out 16"}}


def bench_dambreak(dev, quiet: bool, t_end: float = 1.5, chunk: int = 2000,
                   max_steps: int = 60000):
    """Section 4.2's dam break with the paper's SPH choices (cubic spline kernel
    with support 2 sqrt(3) dp, Eq. 5 viscosity with sqrt(g h_swl), Verlet time
    stepping with an Euler-form step every 40 and the CFL step) on the
    synthetic walled tank with obstacle (179,154 particles, dp = 0.01), run to
    t_end of simulated time as the paper does."""
    import math
    import numpy as np
    import torch
    from paper_1804_07598_amd import _lib as F
    from paper_1804_07598_amd import inputs
    from paper_1804_07598_amd.sim import ParticleSim
    s = inputs.sph_dambreak()
    dx, H, g = s.dx, s.H, 9.81
    h = math.sqrt(3.0) * dx
    c0, cbar = 20.0 * math.sqrt(g * H), math.sqrt(g * H)
    prm = F.sph_params(h, 1000.0 * dx ** 3, 1000.0, c0, 7.0, 0.1, 0.01 * h * h, (0, 0, -g), 0.2,
                       kernel=1, cbar=cbar, scheme=1, verlet_every=40)
    r_cut = float(np.float32(2 * h))
    sim = ParticleSim(s.pos, s.L, (0, 0, 0), vel=s.vel, typ=s.kind, r_cut=r_cut, skin=0.1 * h,
                      max_nbr=320, device=dev)
    sim.set_density(s.rho)
    hist = torch.zeros((chunk, 4), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    steps, t, dt = 0, 0.0, 0.0
    while t < t_end and steps < max_steps:
        # the last chunk is sized from the latest step to end just past t_end
        k = chunk if dt == 0.0 else max(1, min(chunk, math.ceil((t_end - t) / dt)))
        sim.sph_step(k, prm, hist)
        steps += k
        t, dt = (float(x) for x in hist[k - 1, :2].tolist())
        log(f"dam break: {steps} steps, t = {t:.4f} s", quiet)
    e1.record()
    torch.cuda.synchronize()
    sim.check()
    ms = e0.elapsed_time(e1)
    F.fpm_set_profiling(sim.ctx, True)
    for _ in range(10):
        sim.sph_rates(prm)
    r_ms, _ = F.fpm_kernel_time(sim.ctx, "sph_rates")
    F.fpm_set_profiling(sim.ctx, False)
    reb, _, total = sim.counters()
    sim.close()
    n = len(s.pos)
    log(f"dam break: {n} particles to t = {t:.3f} s in {steps} steps, {ms / 1e3:.2f} s "
        f"({ms / steps * 1e3:.1f} us/step), rates kernel {r_ms * 1e3:.1f} us", quiet)
    return {"workload": "SPH dam break, synthetic walled tank 1.6 x 0.67 x 0.4 with obstacle, "
                        "water column 0.4 x 0.67 x 0.3, dp=0.01, N=179,154; cubic spline "
                        "h=sqrt(3) dp, Verlet (Euler every 40), CFL 0.2, c0=20 sqrt(g h_swl), "
                        "cbar=sqrt(g h_swl), alpha=0.1",
            "particles": n, "steps": steps, "simulated_s": t, "wall_s": ms / 1e3,
            "value": n * steps / (ms / 1e3), "unit": "particle-steps/s",
            "ms_per_step": ms / steps, "rates_kernel_us": r_ms * 1e3,
            "mean_list": total / n, "rebuilds": reb}


def bench_dem(dev, quiet: bool, steps: int = 2000, warmup: int = 200, scale: float = 4.2,
              cpu_seconds: float = 0.0):
    """Section 4.5's granular avalanche: the Silbert grain model with Hertzian
    contacts, tangential history and Coulomb cap, x walls, periodic y and a
    floor, gravity tilted by 30 degrees; the block at scale 4.2 holds 688,380
    grains (the paper's single-core figure is for 677,310)."""
    import torch
    from paper_1804_07598_amd import _lib as F
    from paper_1804_07598_amd import inputs
    from paper_1804_07598_amd.sim import ParticleSim
    A = inputs.DEM_AVALANCHE
    s = inputs.dem_avalanche(scale)
    R = A["R"]
    prm = F.dem_params(R, A["mass"], A["inertia"], A["kn"], A["kt"], A["gn"], A["gt"], A["mu"],
                       inputs.dem_avalanche_gravity(), A["dt"], A["walls"])
    sim = ParticleSim(s.pos, s.L, s.periodic, vel=s.vel, r_cut=2 * R, skin=0.1 * R, max_nbr=32,
                      device=dev, dem_contacts=16)
    sim.set_omega(s.omega)
    sim.dem_step(warmup, prm)
    torch.cuda.synchronize()
    sim.check()
    reb0, _, _ = sim.counters()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.dem_step(steps, prm)
    e1.record()
    torch.cuda.synchronize()
    sim.check()
    ms = e0.elapsed_time(e1)
    reb1, _, total = sim.counters()
    _, _, nc = sim.get_dem()
    cbar = float(nc.double().mean())
    F.fpm_set_profiling(sim.ctx, True)
    for _ in range(20):
        sim.dem_forces(prm)
    f_ms, _ = F.fpm_kernel_time(sim.ctx, "dem_forces")
    F.fpm_set_profiling(sim.ctx, False)
    sim.close()
    n = len(s.pos)
    nbar = total / n
    # per grain: pos, vel, omega, id, list count 56 B; list 4 nbar; history
    # entries read 16 nbar and written for the contacts 16 cbar; force, torque
    # 32 B; contact count 4 B (neighbour state gathered from cache)
    bytes_f = n * (92.0 + 20.0 * nbar + 16.0 * cbar)
    achieved = bytes_f / (f_ms / 1e3) / 1e9
    cpu = None
    if cpu_seconds > 0:
        import oracle as O
        oprm = O.dem_params_array(R, A["mass"], A["inertia"], A["kn"], A["kt"], A["gn"], A["gt"],
                                  A["mu"], inputs.dem_avalanche_gravity(), A["dt"], A["walls"])
        cpu = dem_cpu_baseline(s, oprm, cpu_seconds, quiet)
    log(f"DEM avalanche: {n} grains, {steps} steps in {ms:.1f} ms ({ms / steps * 1e3:.1f} us/step), "
        f"forces kernel {f_ms * 1e3:.1f} us, mean list {nbar:.2f}, mean contacts {cbar:.2f}, "
        f"rebuilds {reb1 - reb0}", quiet)
    return {"workload": "DEM avalanche (Silbert model), synthetic block 149 x 105 x 44 grains "
                        "R=0.06 at spacing 2R in a 35.28 x 12.6 x 13.356 domain, x walls, "
                        "periodic y, floor, |g|=5e-4 tilted 30 deg, dt=0.01, N=688,380",
            "grains": n, "steps": steps, "value": n * steps / (ms / 1e3),
            "unit": "grain-steps/s", "ms_per_step": ms / steps,
            "paper_single_core_ms_per_step": 320.0,
            "forces_kernel_us": f_ms * 1e3, "mean_list": nbar, "mean_contacts": cbar,
            "rebuilds": reb1 - reb0,
            "cpu_baseline": cpu,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "bytes_per_launch": bytes_f,
                         "bytes_model": "N*(92 + 20*nbar + 16*cbar): own state 56, list and "
                                        "history entries 20 per entry, history of contacts "
                                        "16, outputs 36"}}


def bench_adjoint(dev, quiet: bool):
    """Gradient of a force-matching loss through a 200-step trajectory of the
    N = 32768 binary mixture (checkpoints and loss frames every 20 steps), and
    the single-evaluation force VJP, each against the plain forward."""
    import numpy as np
    import torch
    from paper_1804_07598_amd import _lib as F
    from paper_1804_07598_amd import inputs
    from paper_1804_07598_amd.adjoint import LJTrajFn
    from paper_1804_07598_amd.sim import ParticleSim
    s = inputs.lj_config("mix32k")
    mix = inputs.LJ_MIXTURE
    theta = np.float32(np.array(mix["eps"] + mix["sig"])).astype(np.float64)
    sim = ParticleSim(s.pos, s.box, (1, 1, 1), vel=s.vel, typ=s.typ, r_cut=2.5, skin=0.3,
                      device=dev)
    K, every = 200, 20
    ms_plain = timed_steps(sim, K, 0.005, 20, mix["eps"], mix["sig"], 2)
    # single evaluation: force kernel against VJP kernel
    lam = torch.randn((s.n, 3), dtype=torch.float64, device=dev)
    F.fpm_set_profiling(sim.ctx, True)
    for _ in range(20):
        sim.lj_forces(mix["eps"], mix["sig"], 2)
        sim.force_vjp(lam, mix["eps"], mix["sig"], 2)
    f_ms, _ = F.fpm_kernel_time(sim.ctx, "lj_force")
    v_ms, _ = F.fpm_kernel_time(sim.ctx, "lj_vjp")
    F.fpm_set_profiling(sim.ctx, False)
    res = []
    for rep in range(2):  # the first call captures the step graphs
        x0 = torch.tensor(s.pos, dtype=torch.float64, device=dev, requires_grad=True)
        v0 = torch.tensor(s.vel, dtype=torch.float64, device=dev, requires_grad=True)
        th = torch.tensor(theta, device=dev, requires_grad=True)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record()
        Fk = LJTrajFn.apply(x0, v0, th, sim, 0.005, K, every, every, 2)
        loss = (Fk ** 2).mean()
        ev[1].record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        ev[2].record()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res.append((ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), (t1 - t0) * 1e3,
                    (t2 - t1) * 1e3))
    sim.check()
    sim.close()
    fwd, bwd, fwd_wall, bwd_wall = res[-1]
    log(f"adjoint: plain {K} steps {ms_plain:.1f} ms, forward {fwd:.1f} ms, backward "
        f"{bwd:.1f} ms (wall {fwd_wall:.1f} + {bwd_wall:.1f}); force {f_ms * 1e3:.1f} us, "
        f"VJP {v_ms * 1e3:.1f} us", quiet)
    return {"workload": "LJ binary mixture N=32768, rho=1.2, T=1, 200 steps dt=0.005, "
                        "checkpoints and force-matching frames every 20 steps",
            "steps": K, "plain_ms": ms_plain, "forward_ms": fwd, "backward_ms": bwd,
            "forward_wall_ms": fwd_wall, "backward_wall_ms": bwd_wall,
            "value": s.n * K / ((fwd + bwd) / 1e3), "unit": "atom-steps/s (forward + backward)",
            "vs_plain": ms_plain / (fwd + bwd),
            "total_over_plain": (fwd + bwd) / ms_plain,
            "backward_over_forward": bwd / fwd,
            "force_kernel_us": f_ms * 1e3, "vjp_kernel_us": v_ms * 1e3,
            "vjp_over_force": v_ms / f_ms,
            "timing": "HIP events on the context's stream (forward and backward include any "
                      "gaps while the host queues work); wall clock beside them"}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning", type=str, default="",
                    help="fixed launch shapes 'path,zblock,unroll' instead of the tuner (headline and --form batched)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the library's default launch shapes")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched and adjoint measurements")
    ap.add_argument("--form", choices=["batched", "sph", "sph_dambreak", "adjoint", "dem",
                                       "symmetric"],
                    help="run only this form's measurement and print its JSON (for profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer 5 times (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--quiet", action="store_true")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {a.gpus}).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1804_07598_amd import _lib as F
    from paper_1804_07598_amd import inputs
    from paper_1804_07598_amd.sim import ParticleSim

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if a.copy_calibration:
        n = a.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}), flush=True)
        return 0
    if a.form:
        fixed = tuple(int(x) for x in a.tuning.split(",")) if a.tuning else None
        legs = {"batched": lambda: bench_batched(dev, 100, a.quiet, fixed),
                "symmetric": lambda: bench_symmetric(dev, 200, a.quiet, float("nan")),
                "sph": lambda: bench_sph(dev, 500, a.quiet),
                "sph_dambreak": lambda: bench_dambreak(dev, a.quiet),
                "adjoint": lambda: bench_adjoint(dev, a.quiet),
                "dem": lambda: bench_dem(dev, a.quiet,
                                         cpu_seconds=0.0 if a.no_cpu_baseline else a.cpu_seconds / 2)}
        print(json.dumps({a.form: legs[a.form]()}), flush=True)
        return 0
    s = inputs.lj_config("lj1m")
    log(f"workload lj1m: N={s.n} L={s.L:.5f}", a.quiet)
    sim = ParticleSim(s.pos, s.box, (1, 1, 1), vel=s.vel, r_cut=2.5, skin=0.3, device=dev)
    knobs = (0, 0, 0)
    if a.tuning:
        knobs = tuple(int(x) for x in a.tuning.split(","))
        sim.set_tuning(*knobs)
    elif not a.no_tune:
        from paper_1804_07598_amd.tune import tune
        knobs, table = tune(sim, s.rho, cache=None)
        for k, f_ms, b_ms, cost in table:
            log(f"tune {k}: force {f_ms * 1e3:.1f} us, rebuild {b_ms * 1e3:.1f} us, "
                f"cost {cost * 1e3:.1f} us", a.quiet)
    dt = 0.005
    thermo = torch.zeros((max(a.steps, a.warmup, 1), 8), dtype=torch.float64, device=dev)

    sim.step(a.warmup, dt=dt, thermo=thermo)
    torch.cuda.synchronize()
    sim.check()
    reb0, _, _ = sim.counters()
    log(f"warmup done ({a.warmup} steps)", a.quiet)

    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(a.steps, dt=dt, thermo=thermo)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    sim.check()
    reb1, longest, total = sim.counters()
    th = thermo[:a.steps].cpu().numpy()
    assert np.isfinite(th).all(), "non-finite thermo"
    rebuilds = reb1 - reb0
    nbar = total / s.n
    kbar = a.steps / max(rebuilds, 1)
    value = s.n * a.steps / (ms / 1e3)
    log(f"timed {a.steps} steps: {ms:.2f} ms (wall {wall * 1e3:.1f} ms), rebuilds {rebuilds}, "
        f"mean list {nbar:.2f}", a.quiet)

    # dominant kernel: LJ force, timed with HIP events around each launch on the
    # stream it runs on
    F.fpm_set_profiling(sim.ctx, True)
    for _ in range(a.kernel_reps):
        sim.lj_forces()
    f_ms, f_n = F.fpm_kernel_time(sim.ctx, "lj_force")
    # drop the records of the gated (no-op) list refreshes made by the force calls
    F.fpm_kernel_time(sim.ctx, "cell_build")
    F.fpm_kernel_time(sim.ctx, "verlet_build")
    for _ in range(5):
        sim.build_verlet()
    c_ms, _ = F.fpm_kernel_time(sim.ctx, "cell_build")
    v_ms, _ = F.fpm_kernel_time(sim.ctx, "verlet_build")
    F.fpm_set_profiling(sim.ctx, False)
    sim.check()
    _, _, total2 = sim.counters()
    nbar_k = total2 / s.n
    bytes_force = s.n * (36.0 + 4.0 * nbar_k)
    achieved = bytes_force / (f_ms / 1e3) / 1e9
    log(f"force kernel {f_ms * 1e3:.1f} us over {f_n} launches -> {achieved:.0f} GB/s; "
        f"cell build {c_ms * 1e3:.1f} us, Verlet build {v_ms * 1e3:.1f} us", a.quiet)

    # the step's own force kernel (forces fused with the kicks and the drift):
    # the same steps issued without graphs, each launch timed with events
    F.fpm_set_profiling(sim.ctx, True)
    sim.step(a.kernel_reps, dt=dt, thermo=thermo)
    s_ms, s_n = F.fpm_kernel_time(sim.ctx, "lj_step")
    F.fpm_kernel_time(sim.ctx, "cell_build")
    F.fpm_kernel_time(sim.ctx, "verlet_build")
    F.fpm_set_profiling(sim.ctx, False)
    sim.check()
    bytes_step = s.n * (84.0 + 4.0 * nbar_k)
    achieved_step = bytes_step / (s_ms / 1e3) / 1e9
    unroll = knobs[2] or 8  # 0 = automatic = 8
    traffic = stored_traffic(s.n, unroll)
    copy_gbs = copy_rate(dev)
    log(f"step force kernel {s_ms * 1e3:.1f} us over {s_n} launches -> {achieved_step:.0f} GB/s; "
        f"device copy {copy_gbs:.0f} GB/s", a.quiet)

    # bytes per atom-step: the fused step kernel every step, and per rebuild
    # the cell sort and the Verlet build (164 B of state, 4 B per list entry)
    B = 84.0 + 4.0 * nbar + (164.0 + 4.0 * nbar) / kbar
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "state_dtype": "f32 (positions, velocities, forces; pair arithmetic and sums in f64)",
        "data": "synthetic",
        "config": {"workload": "lj1m: LJ fluid N=1,000,000 (jittered 100^3 lattice), rho=0.8442, "
                               "T=1, r_cut=2.5, skin=0.3, dt=0.005, periodic",
                   "n": s.n, "dt": dt, "r_cut": 2.5, "skin": 0.3,
                   "tuning": {"verlet_path": knobs[0], "zblock": knobs[1], "unroll": knobs[2]}},
        "roofline": {"bound": "hbm", "achieved": achieved_step, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved_step / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"lj_step (k_lj<1, {unroll}, 1>: forces, closing kick, next "
                               "opening kick and drift)", "kernel_ms": s_ms,
                     "bytes_per_launch": bytes_step,
                     "bytes_model": "N*(84 + 4*nbar): pos_i 16, count 4, list 4*nbar, "
                                    "vel 16 + 16, build position 16, drifted position 16",
                     "measured_copy_gbs": copy_gbs,
                     "step_hbm_frac": B * value / (HBM_PEAK_GBS * 1e9)},
        "force_kernel": {"kernel": f"lj_force (k_lj<1, {unroll}, 0>, forces only)", "ms": f_ms,
                         "bytes_per_launch": bytes_force, "achieved_gbs": achieved,
                         "frac": achieved / HBM_PEAK_GBS,
                         "bytes_model": "N*(36 + 4*nbar): pos_i 16, count 4, list 4*nbar, "
                                        "force 16"},
        "step_model": {"mean_list": nbar, "rebuilds": rebuilds, "rebuild_interval": kbar,
                       "bytes_per_atom_step": B,
                       "hbm_frac": B * value / (HBM_PEAK_GBS * 1e9),
                       "cell_build_ms": c_ms, "verlet_build_ms": v_ms},
        "cpu_baseline": None,
    }
    sim.close()
    if not a.no_forms:
        result["symmetric"] = bench_symmetric(dev, 200, a.quiet, value)
        result["batched"] = bench_batched(dev, 100, a.quiet)
        result["sph"] = bench_sph(dev, 500, a.quiet)
        result["sph_dambreak"] = bench_dambreak(dev, a.quiet)
        result["adjoint"] = bench_adjoint(dev, a.quiet)
        result["dem"] = bench_dem(dev, a.quiet,
                                  cpu_seconds=0.0 if a.no_cpu_baseline else a.cpu_seconds / 2)
    if not a.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(s.pos, s.box, a.cpu_seconds, a.quiet)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
