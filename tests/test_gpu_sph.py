"""Parity of the HIP SPH path (section 4.2, Eqs. 1-5) with the FP64 oracle:
rates (acceleration and density rate) within 1e-5 of their RMS, the CFL time
step, multi-step runs against the oracle's own trajectory, and the
2.1M-particle column on sampled rows."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1804_07598_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-5
RHO0, G = 1000.0, 9.81


def setup(nf, nz, seed=None, vel_sigma=0.0, rho_noise=0.0):
    from paper_1804_07598_amd import _lib as F
    from paper_1804_07598_amd.sim import ParticleSim
    s = inputs.sph_column(nf, nz)
    dx, H = s.dx, s.H
    h = 1.3 * dx
    c0 = 20.0 * math.sqrt(G * H)
    vel, rho = s.vel.copy(), s.rho.copy()
    if seed is not None:
        rng = np.random.default_rng(seed)
        fl = s.kind == 0
        vel[fl] = rng.normal(0, vel_sigma, (fl.sum(), 3)).astype(np.float32)
        rho = (rho * (1 + rng.uniform(-rho_noise, rho_noise, len(rho)))).astype(np.float32)
    r_cut = float(np.float32(2 * h))
    sim = ParticleSim(s.pos, s.L, (1, 1, 0), vel=vel, typ=s.kind, r_cut=r_cut, skin=0.1 * h,
                      max_nbr=160)
    sim.set_density(rho)
    prm = F.sph_params(h, RHO0 * dx ** 3, RHO0, c0, 7.0, 0.1, 0.01 * h * h, (0, 0, -G), 0.2)
    oprm = O.sph_params_array(h, RHO0 * dx ** 3, RHO0, c0, 7.0, 0.1, 0.01 * h * h, (0, 0, -G))
    return s, sim, prm, oprm, r_cut, vel, rho


def np_(t):
    return t.detach().cpu().numpy()


def compare_rates(sim, s, pos, vel, rho, oprm, r_cut, rows=None):
    _, _, a = sim.get()
    _, dr = sim.get_sph()
    a, dr = np_(a).astype(np.float64), np_(dr).astype(np.float64)
    acc, drho, mu = O.sph_rates(pos, vel, rho, s.kind, s.L, (1, 1, 0), O.radius2(r_cut), oprm,
                                rows=rows)
    if rows is not None:
        a, dr = a[rows], dr[rows]
    ea = np.abs(a - acc).max() / math.sqrt((acc ** 2).mean())
    assert ea <= TOL, ea
    rms_d = math.sqrt((drho ** 2).mean())
    if rms_d > 0:
        ed = np.abs(dr - drho).max() / rms_d
        assert ed <= TOL, ed
    else:
        assert np.all(dr == 0)
    return acc, drho, mu


def test_rates_column_at_rest():
    s, sim, prm, oprm, r_cut, vel, rho = setup(16, 16)
    dt = float(np_(sim.sph_rates(prm))[0])
    acc, drho, mu = compare_rates(sim, s, s.pos, vel, rho, oprm, r_cut)
    assert np.all(drho == 0)
    assert dt == pytest.approx(O.sph_dt(acc, s.kind, mu, oprm, 0.2), rel=1e-5)


def test_rates_with_motion_and_noise():
    s, sim, prm, oprm, r_cut, vel, rho = setup(16, 12, seed=3, vel_sigma=0.05, rho_noise=0.01)
    dt = float(np_(sim.sph_rates(prm))[0])
    acc, drho, mu = compare_rates(sim, s, s.pos, vel, rho, oprm, r_cut)
    assert dt == pytest.approx(O.sph_dt(acc, s.kind, mu, oprm, 0.2), rel=1e-5)


def test_steps_match_oracle_trajectory():
    s, sim, prm, oprm, r_cut, vel, rho = setup(16, 16, seed=4, vel_sigma=0.02)
    K = 30
    hist = np_(sim.sph_step(K, prm))
    sim.check()
    p, v, _ = (np_(t) for t in sim.get())
    r, _ = sim.get_sph()
    r = np_(r).astype(np.float64)
    # boundary particles never move
    fb = s.kind == 1
    assert np.array_equal(p[fb], s.pos[fb]) and np.all(v[fb] == 0)
    # time is the sum of the device time steps, each positive
    assert np.all(hist[:, 1] > 0)
    assert hist[-1, 0] == pytest.approx(hist[:, 1].sum(), rel=1e-12)
    # the oracle's KDK trajectory from the same start.  Per step the FP32 state
    # updates round x (|x| < 0.5), v (|v| < 0.2) and rho (~1000) by at most half
    # an ulp: after 30 steps < 30 * 0.5 ulp, i.e. 1e-6, 1e-7 and 2e-3.  The
    # fluid is stiff: a position error dx excites acoustic motion with velocity
    # ~ (c0 / h) dx, and c0 / h = 5.4e3 / s turns one half-ulp position rounding
    # (7.5e-9 at x = 0.25) into 4e-5 of velocity, which bounds v instead.
    x64, v64, r64, h64 = O.sph_kdk(s.pos, vel, rho, s.kind, s.L, (1, 1, 0), O.radius2(r_cut),
                                   oprm, 0.2, K)
    d = p.astype(np.float64) - x64
    for a in range(2):
        d[:, a] -= float(s.L[a]) * np.round(d[:, a] / float(s.L[a]))
    assert np.abs(d).max() <= 4e-6
    assert np.abs(v.astype(np.float64) - v64).max() <= 5e-5
    assert np.abs(r - r64).max() <= 1e-2
    assert np.abs(hist[:, 1] / h64[:, 1] - 1).max() <= 1e-5


def test_full_column_sampled_rows():
    s, sim, prm, oprm, r_cut, vel, rho = setup(128, 128)
    sim.sph_rates(prm)
    rows = np.random.default_rng(0).choice(len(s.pos), 96, replace=False)
    compare_rates(sim, s, s.pos, vel, rho, oprm, r_cut, rows=rows)


def test_isolated_particles():
    # no neighbours within 2h: a fluid particle feels gravity alone, its
    # density does not change, and a boundary particle gets nothing
    from paper_1804_07598_amd import _lib as F
    from paper_1804_07598_amd.sim import ParticleSim
    pos = np.array([[0.1, 0.1, 0.1], [0.5, 0.5, 0.5], [0.9, 0.2, 0.3], [0.3, 0.7, 0.05]],
                   np.float32)
    kind = np.array([0, 0, 0, 1], np.int32)
    vel = np.array([[0.1, 0.0, 0.0], [0.0, -0.2, 0.0], [0.0, 0.0, 0.3], [0.0, 0.0, 0.0]],
                   np.float32)
    dx = 0.01
    h = 1.3 * dx
    r_cut = float(np.float32(2 * h))
    sim = ParticleSim(pos, np.array([1.0, 1.0, 1.0], np.float32), (1, 1, 0), vel=vel, typ=kind,
                      r_cut=r_cut, skin=0.1 * h, max_nbr=16)
    sim.set_density(np.full(4, RHO0, np.float32))
    prm = F.sph_params(h, RHO0 * dx ** 3, RHO0, 20.0 * math.sqrt(G * 0.3), 7.0, 0.1,
                       0.01 * h * h, (0, 0, -G), 0.2)
    sim.sph_rates(prm)
    sim.check()
    _, _, a = sim.get()
    _, dr = sim.get_sph()
    a, dr = np_(a), np_(dr)
    assert np.array_equal(a[:3], np.tile(np.array([0, 0, -G], np.float32), (3, 1)))
    assert np.all(a[3] == 0) and np.all(dr == 0)
