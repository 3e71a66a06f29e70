"""Parity of the paper-faithful SPH variant (section 4.2) with the FP64
oracle: the classic cubic spline kernel with support 2 sqrt(3) dp, Eq. 5's
viscosity with the sound speed sqrt(g h_swl), and the Verlet time stepping
with a dynamic step and periodic Euler-form steps; the walled dam-break tank
(closed box, obstacle, mostly empty cells) at small and full size."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1804_07598_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-5
RHO0, G = 1000.0, 9.81


def np_(t):
    return t.detach().cpu().numpy()


def make(s, per, seed=None, vel_sigma=0.0, rho_noise=0.0, every=40):
    """Simulation and parameters for system s with the paper's SPH choices."""
    from paper_1804_07598_amd import _lib as F
    from paper_1804_07598_amd.sim import ParticleSim
    dx, H = s.dx, s.H
    h = math.sqrt(3.0) * dx
    c0, cbar = 20.0 * math.sqrt(G * H), math.sqrt(G * H)
    vel, rho = s.vel.copy(), s.rho.copy()
    if seed is not None:
        rng = np.random.default_rng(seed)
        fl = s.kind == 0
        vel[fl] = rng.normal(0, vel_sigma, (fl.sum(), 3)).astype(np.float32)
        rho = (rho * (1 + rng.uniform(-rho_noise, rho_noise, len(rho)))).astype(np.float32)
    r_cut = float(np.float32(2 * h))
    sim = ParticleSim(s.pos, s.L, per, vel=vel, typ=s.kind, r_cut=r_cut, skin=0.1 * h,
                      max_nbr=320)
    sim.set_density(rho)
    m = RHO0 * dx ** 3
    prm = F.sph_params(h, m, RHO0, c0, 7.0, 0.1, 0.01 * h * h, (0, 0, -G), 0.2, kernel=1,
                       cbar=cbar, scheme=1, verlet_every=every)
    oprm = O.sph_params_array(h, m, RHO0, c0, 7.0, 0.1, 0.01 * h * h, (0, 0, -G), kernel=1,
                              cbar=cbar)
    return sim, prm, oprm, r_cut, vel, rho


def compare_rates(sim, s, per, vel, rho, oprm, r_cut, rows=None):
    _, _, a = sim.get()
    _, dr = sim.get_sph()
    a, dr = np_(a).astype(np.float64), np_(dr).astype(np.float64)
    acc, drho, mu = O.sph_rates(s.pos, vel, rho, s.kind, s.L, per, O.radius2(r_cut), oprm,
                                rows=rows)
    if rows is not None:
        a, dr = a[rows], dr[rows]
    assert np.abs(a - acc).max() / math.sqrt((acc ** 2).mean()) <= TOL
    rms_d = math.sqrt((drho ** 2).mean())
    if rms_d > 0:
        assert np.abs(dr - drho).max() / rms_d <= TOL
    else:  # a state at rest: no density rate anywhere
        assert np.all(dr == 0)
    return acc, drho, mu


def test_cubic_rates_with_motion_and_noise():
    s = inputs.sph_column(14, 10, dx=0.0085)
    per = (1, 1, 0)
    sim, prm, oprm, r_cut, vel, rho = make(s, per, seed=3, vel_sigma=0.05, rho_noise=0.01)
    dt = float(np_(sim.sph_rates(prm))[0])
    acc, drho, mu = compare_rates(sim, s, per, vel, rho, oprm, r_cut)
    assert dt == pytest.approx(O.sph_dt(acc, s.kind, mu, oprm, 0.2), rel=1e-5)


def check_trajectory(s, per, sim, prm, oprm, r_cut, vel, rho, K, every):
    hist = np_(sim.sph_step(K, prm))
    sim.check()
    p, v, _ = (np_(t) for t in sim.get())
    r, _ = sim.get_sph()
    r = np_(r).astype(np.float64)
    fb = s.kind == 1
    assert np.array_equal(p[fb], s.pos[fb]) and np.all(v[fb] == 0)
    assert np.all(hist[:, 1] > 0)
    assert hist[-1, 0] == pytest.approx(hist[:, 1].sum(), rel=1e-12)
    # the oracle's own Verlet trajectory from the same start; the bounds are
    # those of the kick-drift-kick comparison (FP32 rounding of the state per
    # step, amplified in v by the acoustic stiffness c0 / h)
    x64, v64, r64, h64 = O.sph_verlet(s.pos, vel, rho, s.kind, s.L, per, O.radius2(r_cut),
                                      oprm, 0.2, K, every)
    d = p.astype(np.float64) - x64
    for a in range(3):
        if per[a]:
            d[:, a] -= float(s.L[a]) * np.round(d[:, a] / float(s.L[a]))
    assert np.abs(d).max() <= 4e-6
    assert np.abs(v.astype(np.float64) - v64).max() <= 5e-5
    assert np.abs(r - r64).max() <= 1e-2
    assert np.abs(hist[:, 1] / h64[:, 1] - 1).max() <= 1e-5
    return hist


def test_verlet_steps_match_oracle_trajectory():
    # 30 steps with an Euler-form step every 8: steps 0, 8, 16 and 24
    s = inputs.sph_column(12, 12, dx=0.0085)
    per = (1, 1, 0)
    sim, prm, oprm, r_cut, vel, rho = make(s, per, seed=4, vel_sigma=0.02, every=8)
    check_trajectory(s, per, sim, prm, oprm, r_cut, vel, rho, 30, 8)


def test_verlet_continues_across_calls():
    # two calls of 12 and 18 steps are the same 30 steps (the Verlet state and
    # the Euler-step count carry over); setting the density restarts the count
    s = inputs.sph_column(10, 8, dx=0.0085)
    per = (1, 1, 0)
    sim, prm, oprm, r_cut, vel, rho = make(s, per, seed=5, vel_sigma=0.02, every=7)
    sim.sph_step(12, prm)
    sim.sph_step(18, prm)
    p1, v1, _ = (np_(t) for t in sim.get())
    sim2, _, _, _, _, _ = make(s, per, seed=5, vel_sigma=0.02, every=7)
    sim2.sph_step(30, prm)
    p2, v2, _ = (np_(t) for t in sim2.get())
    assert np.array_equal(p1, p2) and np.array_equal(v1, v2)


def test_small_dambreak_trajectory():
    # closed tank with walls, obstacle and mostly empty cells, coarse spacing
    s = inputs.sph_dambreak(0.04)
    per = (0, 0, 0)
    sim, prm, oprm, r_cut, vel, rho = make(s, per, every=10)
    check_trajectory(s, per, sim, prm, oprm, r_cut, vel, rho, 25, 10)


def test_full_dambreak_sampled_rates_and_run():
    s = inputs.sph_dambreak()  # 179,154 particles, dp = 0.01
    per = (0, 0, 0)
    sim, prm, oprm, r_cut, vel, rho = make(s, per)
    sim.sph_rates(prm)
    rows = np.random.default_rng(0).choice(len(s.pos), 96, replace=False)
    fluid_rows = np.flatnonzero(s.kind == 0)[::4000]
    compare_rates(sim, s, per, vel, rho, oprm, r_cut, rows=np.concatenate([rows, fluid_rows]))
    # 300 Verlet steps: the column starts to collapse; state stays finite, the
    # walls hold, densities stay near rho0 and time advances by the device dt
    hist = np_(sim.sph_step(300, prm))
    sim.check()
    p, v, _ = (np_(t) for t in sim.get())
    r, _ = sim.get_sph()
    r = np_(r)
    fl = s.kind == 0
    assert np.isfinite(p).all() and np.isfinite(v).all() and np.isfinite(r).all()
    assert hist[-1, 0] == pytest.approx(hist[:, 1].sum(), rel=1e-12) and hist[-1, 0] > 0
    w = 3 * s.dx
    assert p[fl, 0].min() > w - 0.5 * s.dx and p[fl, 2].min() > w - 0.5 * s.dx
    assert np.abs(r[fl] / RHO0 - 1).max() < 0.05
    assert v[fl, 0].max() > 0.1  # the front moves into the tank
