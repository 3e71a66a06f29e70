"""Pins of the DEM oracle (Silbert grain model, Eqs. 9-13) against closed
forms and invariants it does not share: the two-body Hertz force, normal
damping, the tangential spring and its torque, rotation in the contact
velocity, the Coulomb cap, loss of contact, conservation of linear and angular
momentum, the leapfrog's free-fall sequence and the wall force."""
import math

import numpy as np
import pytest

import oracle as O

R, M, INERTIA = 0.06, 1.0, 1.44e-3
KN, KT, GN = 7.849, 2.243, 3.401
L = np.array([10.0, 10.0, 10.0], np.float32)


def prm(gt=0.0, mu=0.5, g=(0.0, 0.0, 0.0), dt=1e-3, walls=0):
    return O.dem_params_array(R, M, INERTIA, KN, KT, GN, gt, mu, g, dt, walls)


def pair(d, vp=(0, 0, 0), vq=(0, 0, 0), wp=(0, 0, 0), wq=(0, 0, 0), p=None, hist=None):
    """Grains p at (5 + d, 5, 5) and q at (5, 5, 5): n = +x, |r| = d."""
    x = np.array([[5.0 + d, 5.0, 5.0], [5.0, 5.0, 5.0]])
    v = np.array([vp, vq], np.float64)
    w = np.array([wp, wq], np.float64)
    return O.dem_forces(x, v, w, L, (1, 1, 1), prm() if p is None else p, hist)


def test_two_body_hertz_force():
    d = 0.1
    F, T, (hid, hu), nc = pair(d)
    delta = 2 * R - d
    fn = math.sqrt(delta / (2 * R)) * KN * delta
    assert F[0] == pytest.approx([fn, 0, 0], rel=1e-14)
    assert F[1] == pytest.approx([-fn, 0, 0], rel=1e-14)
    assert np.all(T == 0) and list(nc) == [1, 1]
    assert hid[0, 0] == 1 and hid[1, 0] == 0 and np.all(hu[:, 0] == 0)
    # beyond contact: nothing
    F2, _, (hid2, _), nc2 = pair(2 * R + 1e-9)
    assert np.all(F2 == 0) and list(nc2) == [0, 0] and np.all(hid2 == -1)


def test_normal_damping():
    d, u = 0.11, 0.3
    F, _, _, _ = pair(d, vp=(-u, 0, 0))  # p moves towards q: v_n = -u along +x
    delta = 2 * R - d
    s = math.sqrt(delta / (2 * R))
    expect = s * (KN * delta - GN * (M / 2) * (-u))
    assert F[0, 0] == pytest.approx(expect, rel=1e-14) and F[1, 0] == pytest.approx(-expect)


def test_tangential_spring_and_torque():
    d, vy, dt, gt = 0.1, 0.2, 1e-3, 0.7
    p = prm(gt=gt, dt=dt, mu=100.0)
    F, T, (hid, hu), _ = pair(d, vp=(0, vy, 0), p=p)
    delta = 2 * R - d
    s = math.sqrt(delta / (2 * R))
    u = np.array([0, vy * dt, 0])
    ft = s * (-KT * u - gt * (M / 2) * np.array([0, vy, 0]))
    assert hu[0, 0] == pytest.approx(u, abs=1e-18) and hu[1, 0] == pytest.approx(-u, abs=1e-18)
    assert F[0, 1] == pytest.approx(ft[1], rel=1e-13) and F[1, 1] == pytest.approx(-ft[1], rel=1e-13)
    # torque (-a n) x F_t, a = d / 2, n = +x: (-a, 0, 0) x (0, ft_y, 0) = (0, 0, -a ft_y),
    # equal on both grains
    assert T[0] == pytest.approx([0, 0, -0.5 * d * ft[1]], rel=1e-13)
    assert T[1] == pytest.approx(T[0], rel=1e-13)


def test_rotation_enters_the_contact_velocity():
    d, wz, dt = 0.1, 5.0, 1e-3
    _, _, (hid, hu), _ = pair(d, wp=(0, 0, wz), p=prm(dt=dt, mu=100.0))
    # v_pq = -a (w_p x n) = -a (0, 0, wz) x (1, 0, 0) = -a (0, wz, 0), a = d / 2
    assert hu[0, 0] == pytest.approx([0, -0.5 * d * wz * dt, 0], rel=1e-14)


def test_coulomb_cap_and_rescaled_history():
    d, mu = 0.1, 0.5
    hid = np.full((2, 16), -1, np.int64)
    hu = np.zeros((2, 16, 3))
    hid[0, 0], hid[1, 0] = 1, 0
    hu[0, 0], hu[1, 0] = (0, 0.05, 0), (0, -0.05, 0)  # a large tangential stretch
    F, _, (hid2, hu2), _ = pair(d, p=prm(mu=mu), hist=(hid, hu))
    delta = 2 * R - d
    s = math.sqrt(delta / (2 * R))
    fn = s * KN * delta
    assert abs(F[0, 1]) == pytest.approx(mu * fn, rel=1e-13) and F[0, 1] < 0
    assert hu2[0, 0, 1] == pytest.approx(mu * fn / (s * KT), rel=1e-13)
    assert hu2[1, 0] == pytest.approx(-hu2[0, 0], rel=1e-13)


def test_lost_contact_forgets_history():
    hid = np.full((2, 16), -1, np.int64)
    hu = np.zeros((2, 16, 3))
    hid[0, 0], hid[1, 0] = 1, 0
    hu[0, 0], hu[1, 0] = (0, 0.01, 0), (0, -0.01, 0)
    F, _, (hid2, _), nc = pair(2 * R + 0.01, hist=(hid, hu))
    assert np.all(hid2 == -1) and np.all(nc == 0) and np.all(F == 0)


def cluster(n, seed):
    rng = np.random.default_rng(seed)
    side = int(round(n ** (1 / 3)))
    idx = np.indices((side, side, side)).reshape(3, -1).T[:n]
    x = 4.0 + idx * 1.9 * R + rng.uniform(-0.01, 0.01, (n, 3))
    v = rng.normal(0, 0.3, (n, 3))
    w = rng.normal(0, 3.0, (n, 3))
    return x, v, w


def test_momentum_and_angular_momentum_conserved():
    x, v, w = cluster(64, 3)
    p = prm(gt=0.5, dt=2e-4)
    P0 = M * v.sum(axis=0)
    J0 = (M * np.cross(x, v)).sum(axis=0) + INERTIA * w.sum(axis=0)
    x1, v1, w1, hist, F, T, nc = O.dem_steps(x, v, w, L, (0, 0, 0), p, 200)
    assert nc.max() > 0  # collisions happened
    P1 = M * v1.sum(axis=0)
    J1 = (M * np.cross(x1, v1)).sum(axis=0) + INERTIA * w1.sum(axis=0)
    scale = M * np.abs(v).sum()
    assert np.abs(P1 - P0).max() < 1e-12 * scale
    assert np.abs(J1 - J0).max() < 1e-10 * (scale * 5.0)


def test_leapfrog_free_fall_sequence():
    x0 = np.array([[1.0, 2.0, 3.0], [6.0, 6.0, 6.0]])
    v0 = np.array([[0.1, 0.0, 0.2], [0.0, -0.3, 0.0]])
    w0 = np.array([[1.0, 2.0, 3.0], [0.0, 0.0, 0.0]])
    g, dt, k = (0.0, 0.0, -9.81), 1e-3, 50
    x, v, w, _, _, _, _ = O.dem_steps(x0, v0, w0, L, (0, 0, 0), prm(g=g, dt=dt), k)
    gv = np.array(g)
    # v first, then x with the new v: x_k = x0 + k dt v0 + dt^2 g k (k + 1) / 2
    assert np.allclose(v, v0 + k * dt * gv, rtol=0, atol=1e-12)
    assert np.allclose(x, x0 + k * dt * v0 + dt * dt * gv * k * (k + 1) / 2, rtol=0, atol=1e-12)
    assert np.array_equal(w, w0)


def test_floor_and_side_walls():
    x = np.array([[5.0, 5.0, 0.05], [0.02, 5.0, 5.0], [9.97, 5.0, 5.0]])
    v = np.array([[0.0, 0.0, -0.1], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    F, T, _, nc = O.dem_forces(x, v, np.zeros((3, 3)), L, (0, 0, 0), prm(walls=3))
    d0 = R - 0.05
    f0 = math.sqrt(d0 / (2 * R)) * (KN * d0 - GN * M * (-0.1))
    assert F[0] == pytest.approx([0, 0, f0], rel=1e-13)
    d1 = R - 0.02
    assert F[1] == pytest.approx([math.sqrt(d1 / (2 * R)) * KN * d1, 0, 0], rel=1e-13)
    d2 = R - (10.0 - 9.97)
    assert F[2, 0] == pytest.approx(-math.sqrt(d2 / (2 * R)) * KN * d2, rel=1e-10)
    assert np.all(T == 0) and np.all(nc == 0)
    # the floor only with bit 2, the x walls only with bit 1
    F2, _, _, _ = O.dem_forces(x, v, np.zeros((3, 3)), L, (0, 0, 0), prm(walls=1))
    assert F2[0, 2] == 0 and F2[1, 0] > 0


def test_rows_evaluation_equals_full_evaluation():
    # the sampled-rows entry (used to time the oracle on large systems) gives
    # the full evaluation's rows bit for bit, walls and gravity included
    x, v, w = cluster(125, 4)
    x[:, 2] -= 3.97  # the bottom layer touches the floor
    p = prm(gt=0.5, g=(0.3, 0.0, -9.81), walls=3)
    F, T, _, nc = O.dem_forces(x, v, w, L, (0, 1, 0), p)
    rows = np.array([0, 7, 31, 64, 99, 124])
    Fr, Tr, ncr = O.dem_forces_rows(x, v, w, L, (0, 1, 0), p, rows)
    assert np.array_equal(Fr, F[rows]) and np.array_equal(Tr, T[rows])
    assert np.array_equal(ncr, nc[rows]) and nc.max() > 0
