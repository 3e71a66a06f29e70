"""Symmetric half lists (the section 4.1 listing's getCellListSym and
applyKernel_in_sym): every pair evaluated once at its lower slot, the
reaction added to the partner in a second pass.  Through the C ABI against
the FP64 oracle (forces within 1e-5 of the RMS force, energy 1e-6, virial
1e-6 of sum |r.F|), against the full-list path, bit-for-bit repeatability
(no atomics), neighbour sets unchanged, and trajectories with rebuilds."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1804_07598_amd import inputs

pytestmark = pytest.mark.gpu

PER = (1, 1, 1)
RC, SKIN = 2.5, 0.3
MIX = inputs.LJ_MIXTURE


def np_(t):
    return t.detach().cpu().numpy()


def make(s, sym=True, **kw):
    from paper_1804_07598_amd.sim import ParticleSim
    return ParticleSim(s.pos, s.box, PER, vel=s.vel, typ=s.typ, r_cut=RC, skin=SKIN,
                       symmetric=sym, **kw)


def check(sim, s, eps=(1.0,) * 3, sig=(1.0,) * 3, nt=1, typ=None, rows=None):
    out = np_(sim.lj_forces(eps, sig, nt))
    _, _, f = sim.get()
    f = np_(f).astype(np.float64)
    F64, U64, W64, _, _ = O.lj(s.pos, s.box, PER, O.radius2(RC), eps, sig, typ, rows=rows)
    if rows is not None:
        f = f[rows]
    assert np.abs(f - F64).max() <= 1e-5 * math.sqrt((F64 ** 2).mean())
    if rows is None:
        assert abs(out[0] - U64) <= 1e-6 * abs(U64)
        scale = O.lj_virial_scale(s.pos, s.box, PER, O.radius2(RC), eps, sig, typ)
        assert np.abs(out[2:] - W64).max() <= 1e-6 * scale
    return out, f


@pytest.mark.parametrize("n,rho,seed", [(4096, 0.8442, 1), (1000, 0.8442, 7), (300, 0.6, 4001)])
def test_symmetric_forces_match_oracle(n, rho, seed):
    s = inputs.lj_lattice(n, rho, 1.0, seed)
    sim = make(s)
    sim.check()
    check(sim, s)
    # the sets are the FP32-predicate sets, whatever the list order
    counts, cols = (np_(t) for t in sim.neighbors())
    ocnt, ocols = O.neighbors(s.pos, s.box, PER, O.radius2(RC, SKIN), cap=sim.max_nbr)
    assert np.array_equal(counts, ocnt)
    for i in range(s.n):
        assert set(cols[i, :counts[i]].tolist()) == set(ocols[i, :ocnt[i]].tolist())
    sim.close()


def test_symmetric_mixture_and_repeatability():
    s = inputs.lj_lattice(4096, 1.2, 1.0, 5, mixture=True)
    sim = make(s)
    out1, f1 = check(sim, s, MIX["eps"], MIX["sig"], 2, s.typ)
    out2, f2 = check(sim, s, MIX["eps"], MIX["sig"], 2, s.typ)
    sim2 = make(s)
    out3, f3 = check(sim2, s, MIX["eps"], MIX["sig"], 2, s.typ)
    assert np.array_equal(f1, f2) and np.array_equal(out1, out2)
    assert np.array_equal(f1, f3) and np.array_equal(out1, out3)
    # against the full-list path on the same state
    full = make(s, sym=False)
    outf, ff = check(full, s, MIX["eps"], MIX["sig"], 2, s.typ)
    rms = math.sqrt((ff ** 2).mean())
    assert np.abs(f1 - ff).max() <= 1e-6 * rms
    assert abs(out1[0] - outf[0]) <= 1e-9 * abs(outf[0])
    for x in (sim, sim2, full):
        x.close()


def test_symmetric_batch():
    from paper_1804_07598_amd.sim import BatchSim
    ns, rhos, Ts = inputs.batched_table()
    systems = [inputs.batched_system(k, ns, rhos, Ts) for k in (0, 3, 72)]
    sim = BatchSim([x.pos for x in systems], [x.box for x in systems], PER, r_cut=RC, skin=SKIN,
                   symmetric=True)
    out = np_(sim.lj_forces())
    _, _, f = sim.get()
    f = np_(f).astype(np.float64)
    for k, x in enumerate(systems):
        a, b = sim.offsets[k], sim.offsets[k + 1]
        F64, U64, _, _, _ = O.lj(x.pos, x.box, PER, O.radius2(RC))
        assert np.abs(f[a:b] - F64).max() <= 1e-5 * math.sqrt((F64 ** 2).mean()), k
        assert abs(out[k, 0] - U64) <= 1e-6 * abs(U64), k


def test_symmetric_steps_match_full_list_and_oracle():
    """40 steps with rebuilds: the symmetric and full-list step loops follow
    the oracle's FP32-state trajectory, and forces at the reached state match
    the oracle; repeated runs are identical bit for bit."""
    s = inputs.lj_lattice(4096, 0.8442, 1.0, 1)
    K = 40
    thr = np.float32((0.5 * float(np.float32(SKIN))) ** 2)
    xs, vs, Fs, nb = O.lj_traj_f32(s.pos, s.vel, s.box, PER, O.radius2(RC), np.float32(0.005),
                                   K, thr)
    res = []
    for sym in (True, True, False):
        sim = make(s, sym=sym)
        th = np_(sim.step(K, dt=0.005))
        sim.check()
        p, v, f = (np_(t) for t in sim.get())
        res.append((p, v, f, th, sim.counters()[0]))
        sim.close()
    assert nb >= 2 and res[0][4] == nb
    (p, v, f, th, _), (p2, v2, f2, th2, _), (pf, vf, ff, thf, _) = res
    assert np.array_equal(p, p2) and np.array_equal(f, f2) and np.array_equal(th, th2)
    rms = math.sqrt((Fs[K].astype(np.float64) ** 2).mean())
    assert np.abs(f.astype(np.float64) - Fs[K]).max() <= 1e-5 * rms
    assert np.abs(p - xs[K]).max() <= 1e-4
    assert np.abs(ff.astype(np.float64) - f).max() <= 1e-5 * rms
    E, Ef = th[:, 0] + th[:, 1], thf[:, 0] + thf[:, 1]
    assert np.abs(E - Ef).max() <= 1e-6 * abs(Ef[0])


def test_symmetric_1m_sampled_rows():
    s = inputs.lj_config("lj1m")
    sim = make(s)
    rows = np.random.default_rng(7).choice(s.n, 2048, replace=False)
    check(sim, s, rows=rows)
    sim.step(20, dt=0.005)
    sim.check()
    p, _, f = (np_(t) for t in sim.get())
    F64, _, _, _, _ = O.lj(p, s.box, PER, O.radius2(RC), rows=rows)
    assert np.abs(f[rows].astype(np.float64) - F64).max() <= 1e-5 * math.sqrt((F64 ** 2).mean())
    sim.close()
