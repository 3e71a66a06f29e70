"""Pins of the SPH oracle (section 4.2, Eqs. 1-5) against facts that do not
come from the oracle: kernel normalisation, the kernel's derivative, two-body
closed forms built from them, lattice symmetry, momentum conservation and the
sign of viscous dissipation."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle as O

H = 0.013
DX = 0.01
RHO0 = 1000.0
C0 = 20.0 * math.sqrt(9.81 * 1.28)
M = RHO0 * DX ** 3


def prm(g=(0.0, 0.0, -9.81), alpha=0.1):
    return O.sph_params_array(H, M, RHO0, C0, 7.0, alpha, 0.01 * H * H, g)


def tait(rho):
    B = C0 * C0 * RHO0 / 7.0
    return B * ((rho / RHO0) ** 7 - 1.0)


def test_kernel_normalised():
    val, err = quad(lambda r: O.sph_kernel_w(r, H) * 4 * math.pi * r * r, 0, 2 * H, epsabs=0,
                    epsrel=1e-13)
    assert val == pytest.approx(1.0, abs=1e-12)
    assert O.sph_kernel_w(2 * H, H) == 0.0
    assert O.sph_kernel_w(2.5 * H, H) == 0.0


def dwdr_numeric(r):
    e = 1e-9 * H
    return (O.sph_kernel_w(r + e, H) - O.sph_kernel_w(r - e, H)) / (2 * e)


def two_body(r, rho_a, rho_b, va=(0, 0, 0), vb=(0, 0, 0), g=(0, 0, 0), alpha=0.1):
    L = np.array([1.0, 1.0, 1.0], np.float32)
    pos = np.array([[0.5, 0.5, 0.5], [0.5 + r, 0.5, 0.5]], np.float32)
    rr = float(pos[1, 0]) - float(pos[0, 0])
    vel = np.array([va, vb], np.float32)
    rho = np.array([rho_a, rho_b], np.float32)
    kind = np.zeros(2, np.int32)
    acc, drho, mu = O.sph_rates(pos, vel, rho, kind, L, (1, 1, 1), O.radius2(2 * H),
                                prm(g, alpha))
    return acc, drho, mu, rr, rho


def test_two_body_pressure_closed_form():
    acc, drho, mu, r, rho = two_body(0.011, 1010.0, 1020.0)
    ra, rb = float(rho[0]), float(rho[1])
    # particle a sits at smaller x; grad_a W = W'(r) (x_a - x_b)/r = -W'(r) e_x
    grad_ax = -dwdr_numeric(r)
    expect = -M * (tait(ra) + tait(rb)) / (ra * rb) * grad_ax
    assert acc[0, 0] == pytest.approx(expect, rel=1e-6)
    assert expect < 0  # compressed pair pushes a away from b (towards -x)
    assert acc[1, 0] == pytest.approx(-expect * 1.0, rel=1e-6)  # equal masses: opposite
    assert np.all(acc[:, 1:] == 0) and np.all(drho == 0)


def test_two_body_continuity_and_viscosity():
    u = float(np.float32(0.3))  # the value the FP32 velocity array holds
    acc, drho, mu, r, rho = two_body(0.012, RHO0, RHO0, va=(u, 0, 0))
    wp = dwdr_numeric(r)
    # approaching pair: density grows, d rho_a/dt = m v_ab . grad_a W = -m u W'(r) > 0
    assert drho[0] == pytest.approx(-M * u * wp, rel=1e-6)
    assert drho[0] > 0 and drho[1] == pytest.approx(drho[0], rel=1e-12)
    # P = 0 at rho0, so only Eq. 5's viscosity acts; it decelerates the pair
    mu_ab = H * (u * -float(r)) / (r * r + 0.01 * H * H)
    Pi = -0.1 * C0 * mu_ab / RHO0
    assert Pi > 0
    assert acc[0, 0] == pytest.approx(-M * Pi * (-wp), rel=1e-6)
    assert acc[0, 0] < 0 and mu[0] == pytest.approx(abs(mu_ab), rel=1e-9)
    # receding pair: no artificial viscosity
    acc2, _, _, _, _ = two_body(0.012, RHO0, RHO0, va=(-u, 0, 0))
    assert np.all(acc2 == 0)


def lattice(n, dx, jitter=0.0, seed=0):
    idx = np.indices((n, n, n)).reshape(3, -1).T
    pos = (idx + 0.5) * dx
    if jitter:
        pos += np.random.default_rng(seed).uniform(-jitter, jitter, pos.shape)
    return pos.astype(np.float32), np.full(3, n * dx, np.float32)


def test_uniform_lattice_at_rest():
    # symmetric neighbourhoods: pressure gradients cancel, a = g, drho = 0.
    # A dyadic spacing keeps every lattice site exact in FP32.
    dx = 2.0 ** -7
    h = 1.3 * dx
    pos, L = lattice(12, dx)
    n = len(pos)
    rho = np.full(n, 1010.0, np.float32)
    p = O.sph_params_array(h, RHO0 * dx ** 3, RHO0, C0, 7.0, 0.1, 0.01 * h * h, (0, 0, -9.81))
    acc, drho, _ = O.sph_rates(pos, np.zeros_like(pos), rho, np.zeros(n, np.int32), L,
                               (1, 1, 1), O.radius2(2 * h), p)
    scale = M * 2 * tait(1010.0) / 1010.0 ** 2 * abs(dwdr_numeric(DX))
    assert np.abs(acc - np.array([0, 0, -9.81])).max() < 1e-10 * scale
    assert np.all(drho == 0)


def test_momentum_conservation_and_dissipation():
    pos, L = lattice(10, DX, jitter=0.002, seed=1)
    n = len(pos)
    rng = np.random.default_rng(2)
    vel = rng.normal(0, 0.2, (n, 3)).astype(np.float32)
    rho = rng.uniform(990, 1030, n).astype(np.float32)
    kind = np.zeros(n, np.int32)
    acc, drho, _ = O.sph_rates(pos, vel, rho, kind, L, (1, 1, 1), O.radius2(2 * H), prm())
    f = acc - np.array([0, 0, -9.81])
    scale = np.abs(f).max()
    assert np.abs(f.sum(axis=0)).max() < 1e-10 * scale * n
    # viscosity alone (rho = rho0 so P = 0) never adds kinetic energy
    rho0 = np.full(n, RHO0, np.float32)
    acc0, _, _ = O.sph_rates(pos, vel, rho0, kind, L, (1, 1, 1), O.radius2(2 * H), prm())
    power = float((vel.astype(np.float64) * (acc0 - np.array([0, 0, -9.81]))).sum()) * M
    assert power < 0


def test_boundary_particles_have_no_acceleration():
    pos, L = lattice(8, DX, jitter=0.001, seed=3)
    n = len(pos)
    kind = (pos[:, 2] < 2 * DX).astype(np.int32)
    rho = np.full(n, 1005.0, np.float32)
    vel = np.zeros_like(pos)
    vel[kind == 0, 2] = -0.1
    acc, drho, _ = O.sph_rates(pos, vel, rho, kind, L, (1, 1, 0), O.radius2(2 * H), prm())
    assert np.all(acc[kind == 1] == 0)
    assert np.any(drho[kind == 1] != 0)


def test_dt_rule():
    acc = np.array([[0, 0, -9.81], [0, 0, -40.0], [0, 0, -1000.0]])
    kind = np.array([0, 0, 1])
    p = prm()
    dt = O.sph_dt(acc, kind, np.array([0.5, 0.1, 0.0]), p, 0.2)
    assert dt == pytest.approx(0.2 * min(math.sqrt(H / 40.0), H / (C0 + 0.5)))
