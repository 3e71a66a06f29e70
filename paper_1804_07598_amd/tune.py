"""Launch-shape autotuner.

The library exposes three knobs through fpm_set_tuning: how Verlet lists are
built (particle by particle over whole neighbour cells or over candidate
windows, by column workgroups that stage the 3 x 3 neighbouring cell columns
in LDS, or by lane groups that stage rows of lists in LDS), how many z-cells a
column workgroup takes (lanes per particle for lane groups), and how many list
entries each lane of the force kernel keeps in flight.  None of them changes a result.  `tune()` times every candidate on
the caller's own system (or batch) with the library's event timing and keeps
the one with the smallest cost per step,

    cost = t_force + t_build / k,

k being the number of steps between list rebuilds of a system, measured on
the caller's own system by a short trajectory from its current state (which
is restored afterwards), unless the caller gives it.  Results are cached in a
JSON file keyed by device, particle-count bucket (log2 of N) and density
bucket (steps of 0.05), so later runs of similar systems skip the search.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import _lib as F

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_1804_07598_amd",
                             "tuning.json")

# (verlet_path, zblock, unroll); zblock 0 lets the library size the column blocks,
# for path 4 it is the number of lanes per particle
CANDIDATES = [(5, 0, 8), (5, 0, 4), (4, 8, 8), (4, 8, 4), (4, 4, 8), (3, 0, 8), (2, 0, 8),
              (1, 0, 8)]


def _device_key(device) -> str:
    p = torch.cuda.get_device_properties(device)
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|{p.multi_processor_count}"


def bucket(n: int, density: float) -> str:
    return f"n2^{int(round(math.log2(max(n, 1))))}|rho{round(density * 20) / 20:.2f}"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path: str, data: dict):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _measure(sim, reps: int, eps, sig, n_types):
    """(force ms, rebuild ms): mean event-timed durations."""
    F.fpm_set_profiling(sim.ctx, True)
    for _ in range(reps):
        sim.lj_forces(eps, sig, n_types)
    f_ms, _ = F.fpm_kernel_time(sim.ctx, "lj_force")
    F.fpm_kernel_time(sim.ctx, "verlet_build")  # the force calls' skipped (gated) refreshes
    F.fpm_kernel_time(sim.ctx, "cell_build")
    for _ in range(reps):
        sim.build_verlet()
    v_ms, _ = F.fpm_kernel_time(sim.ctx, "verlet_build")
    c_ms, _ = F.fpm_kernel_time(sim.ctx, "cell_build")
    F.fpm_set_profiling(sim.ctx, False)
    return f_ms, v_ms + c_ms


def measure_rebuild_interval(sim, steps: int = 100, dt: float = 0.005, eps=(1.0, 1.0, 1.0),
                     sig=(1.0, 1.0, 1.0), n_types: int = 1) -> float:
    """Mean number of steps between list rebuilds of a system of `sim` over
    `steps` steps from its current state; the state is restored afterwards."""
    p, v, _ = sim.get()
    r0 = sim.counters()[0]
    sim.step(steps, dt, eps, sig, n_types)
    r = sim.counters()[0] - r0
    sim.set_particles(p, v)
    return steps * sim.nsys / max(r, 1)


def tune(sim, density: float, *, rebuild_interval: float | None = None, dt: float = 0.005,
         reps: int = 5, eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0), n_types: int = 1,
         cache: str | None = DEFAULT_CACHE, force: bool = False, candidates=None):
    """Pick and apply the fastest launch shapes for `sim` (a ParticleSim or
    BatchSim).  rebuild_interval None measures it (100 steps of size dt).
    Returns (knobs, table of (knobs, force ms, build ms, cost))."""
    key_dev = _device_key(sim.device)
    key = bucket(sim.n, density)
    data = _load(cache) if cache else {}
    hit = data.get(key_dev, {}).get(key)
    if hit is not None and not force:
        knobs = tuple(hit["knobs"])
        sim.set_tuning(*knobs)
        return knobs, []
    k = rebuild_interval
    if k is None:
        k = measure_rebuild_interval(sim, dt=dt, eps=eps, sig=sig, n_types=n_types)
    raw = []
    for knobs in candidates or CANDIDATES:
        sim.set_tuning(*knobs)
        f_ms, b_ms = _measure(sim, 1, eps, sig, n_types)  # warm (graphs, caches)
        f_ms, b_ms = _measure(sim, reps, eps, sig, n_types)
        raw.append((knobs, f_ms, b_ms))
    # the force kernel's time depends on the build path too (the order of the
    # entries it writes decides how many cache lines a gather touches), so each
    # candidate keeps its own force timing
    table = [(knobs, f_ms, b_ms, f_ms + b_ms / k) for knobs, f_ms, b_ms in raw]
    best = min(table, key=lambda r: r[3])
    sim.set_tuning(*best[0])
    if cache:
        data = _load(cache)
        data.setdefault(key_dev, {})[key] = {"knobs": list(best[0]), "force_ms": best[1],
                                             "build_ms": best[2], "cost_ms": best[3],
                                             "rebuild_interval": k, "n": sim.n}
        _save(cache, data)
    return best[0], table
