"""Runs the library's paths through its debug build (libfpm_checked.so: the
cell list and the Verlet lists validated after every rebuild, list entries
range-checked where the LJ force and VJP kernels read them) and stops at the
first FPM_EBADINDEX that fpm_check reports.  Started in a process of its own
by tests/test_gpu_checked.py, since a process loads one build of the library.
Prints one line per case, naming it before it starts."""
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import oracle as O  # noqa: E402
from paper_1804_07598_amd import _lib as F  # noqa: E402
from paper_1804_07598_amd import inputs  # noqa: E402

F.LIB_PATH = os.path.join(ROOT, "paper_1804_07598_amd", "libfpm_checked.so")
from paper_1804_07598_amd.sim import BatchSim, ParticleSim  # noqa: E402

PER = (1, 1, 1)


def case(name):
    print(f"case {name}", flush=True)


def lj_cases():
    s = inputs.lj_lattice(4096, 0.8442, 1.0, seed=1)
    for tuning in (None, (5, 0, 8), (4, 8, 8), (3, 0, 8), (2, 0, 8), (1, 0, 8)):
        case(f"lj 4096 tuning {tuning}")
        sim = ParticleSim(s.pos, s.box, PER, vel=s.vel, r_cut=2.5, skin=0.3, tuning=tuning)
        sim.lj_forces()
        _, _, f = sim.get()
        F64 = O.lj(s.pos, s.box, PER, O.radius2(2.5))[0]
        err = np.abs(f.cpu().numpy().astype(np.float64) - F64).max() / math.sqrt((F64 ** 2).mean())
        assert err <= 1e-5, err
        sim.step(60, dt=0.005)  # several automatic rebuilds
        sim.check()
        sim.close()
    case("lj mixture 4096 with the force VJP")
    m = inputs.LJ_MIXTURE
    s = inputs.lj_lattice(4096, 1.2, 1.0, seed=5, mixture=True)
    sim = ParticleSim(s.pos, s.box, PER, vel=s.vel, typ=s.typ, r_cut=2.5, skin=0.3)
    sim.lj_forces(m["eps"], m["sig"], 2)
    lam = torch.from_numpy(np.random.default_rng(6).normal(size=(s.n, 3))).cuda()
    sim.force_vjp(lam, m["eps"], m["sig"], 2)
    sim.step(40, 0.005, m["eps"], m["sig"], 2)
    sim.check()
    sim.close()
    case("lj 4096 symmetric half lists")
    s = inputs.lj_lattice(4096, 0.8442, 1.0, seed=2)
    sim = ParticleSim(s.pos, s.box, PER, vel=s.vel, r_cut=2.5, skin=0.3, symmetric=True)
    sim.step(40, dt=0.005)
    sim.check()
    sim.close()


def batch_cases():
    ns, rhos, Ts = inputs.batched_table()
    systems = [inputs.batched_system(k, ns, rhos, Ts) for k in list(range(10)) + [72, 130]]
    for tuning in (None, (5, 0, 4)):
        case(f"batch of {len(systems)} tuning {tuning}")
        sim = BatchSim([x.pos for x in systems], [x.box for x in systems], PER,
                       vel_list=[x.vel for x in systems], r_cut=2.5, skin=0.3, tuning=tuning)
        sim.step(60, 0.005)
        sim.check()
        sim.close()


def sph_case():
    case("sph column 16 x 16")
    s = inputs.sph_column(16, 16)
    h = 1.3 * s.dx
    c0 = 20.0 * math.sqrt(9.81 * s.H)
    sim = ParticleSim(s.pos, s.L, (1, 1, 0), vel=s.vel, typ=s.kind,
                      r_cut=float(np.float32(2 * h)), skin=0.1 * h, max_nbr=160)
    sim.set_density(s.rho)
    prm = F.sph_params(h, 1000.0 * s.dx ** 3, 1000.0, c0, 7.0, 0.1, 0.01 * h * h,
                       (0, 0, -9.81), 0.2)
    sim.sph_step(40, prm)
    sim.check()
    sim.close()


def dem_case():
    case("dem packing 10 x 10 x 10")
    R, M, I = 0.06, 1.0, 1.44e-3
    L = [10 * 1.9 * R] * 3
    s = inputs.dem_block((10, 10, 10), R, 1.9 * R, L, PER, seed=1, jitter=0.005,
                         vel_sigma=0.3, omega_sigma=3.0)
    sim = ParticleSim(s.pos, s.L, s.periodic, vel=s.vel, r_cut=2 * R, skin=0.02, max_nbr=48,
                      dem_contacts=16)
    sim.set_omega(s.omega)
    prm = F.dem_params(R, M, I, 7.849, 2.243, 3.401, 1.0, 0.5, (0.0, 0.0, 0.0), 2e-4, 0)
    sim.dem_step(100, prm)
    sim.check()
    sim.close()


def main():
    torch.cuda.set_device(0)
    assert F.lib()._name.endswith("libfpm_checked.so")
    lj_cases()
    batch_cases()
    sph_case()
    dem_case()
    print("all cases ok", flush=True)


if __name__ == "__main__":
    main()
