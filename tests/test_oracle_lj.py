"""Pins of the FP64 CPU oracle (LJ, neighbour sets, cell sort, velocity Verlet)
against facts fixed by the paper and by mathematics, not by the oracle itself:
closed forms of the LJ potential of section 4.1, hand-built neighbour cases,
symmetry (Newton's third law, perfect-lattice forces, lattice sums),
translation/permutation invariance, and the convergence order and time
reversibility of velocity Verlet."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from paper_1804_07598_amd import inputs

PER = (1, 1, 1)


def pair_system(r, L=20.0, axis=np.array([1.0, 0.0, 0.0])):
    """Two particles at separation r along `axis`, centred in a periodic box."""
    c = np.full(3, L / 2)
    u = axis / np.linalg.norm(axis)
    pos = np.stack([c - 0.5 * r * u, c + 0.5 * r * u]).astype(np.float32)
    return pos


def pair_energy_force(r, rc=2.5, eps=1.0, sig=1.0):
    """(U, F_x on particle 0) for two particles at FP64-exact separation r.

    r is represented exactly because the positions are chosen as FP32 values."""
    L = 20.0
    pos = np.array([[0.0, 5.0, 5.0], [r, 5.0, 5.0]], dtype=np.float32)
    rr = float(pos[1, 0]) - float(pos[0, 0])
    F, U, W, _, _ = O.lj(pos, np.full(3, L, np.float32), PER, O.radius2(rc),
                         eps=(eps,) * 3, sig=(sig,) * 3)
    return U, F[0, 0], rr


# ---------------------------------------------------------------- LJ closed forms

def test_lj_zero_force_at_minimum():
    # F(2^(1/6) sigma) = 0 and V there equals -eps (section 4.1 potential).
    for sig, eps in [(1.0, 1.0), (0.8, 1.5), (0.88, 0.5)]:
        rmin = 2 ** (1 / 6) * sig
        pos = np.array([[3.0, 3, 3], [3.0 + rmin, 3, 3]], dtype=np.float32)
        rr = float(pos[1, 0]) - 3.0
        F, U, W, _, _ = O.lj(pos, np.full(3, 20, np.float32), PER, O.radius2(2.5),
                             eps=(eps,) * 3, sig=(sig,) * 3)
        # FP32 rounding of rmin moves r by < 1e-7, so F is O(1e-5 eps/sig)
        assert abs(F[0, 0]) < 1e-4 * eps / sig
        assert U == pytest.approx(-eps, rel=1e-10, abs=1e-10) or abs(U + eps) < 1e-10
        assert abs(rr - rmin) < 1e-6


def test_lj_zero_energy_at_sigma():
    U, F, rr = pair_energy_force(1.0)
    assert rr == 1.0
    assert abs(U) < 1e-15
    # at r = sigma the pair repels with |F| = 24 eps / sigma
    assert F == pytest.approx(-24.0, rel=1e-14)


def test_lj_force_is_minus_gradient():
    # central difference of the pair energy against the pair force
    for r in [0.95, 1.1, 1.5, 2.0, 2.4]:
        h = 2 ** -20
        Up, _, rp = pair_energy_force(r + h)
        Um, _, rm = pair_energy_force(r - h)
        _, F, r0 = pair_energy_force(r)
        dVdr = (Up - Um) / (rp - rm)
        # force on particle 0 (at smaller x) is -dV/dr along -x: F0x = dV/dr
        assert F == pytest.approx(dVdr, rel=1e-7, abs=1e-9), r


def test_lj_truncation_tie_and_beyond():
    # The listing keeps a pair unless rn > r_cut^2: at exactly r_cut it is kept.
    U_in, F_in, r_in = pair_energy_force(2.5)
    assert r_in == 2.5
    assert U_in == pytest.approx(4 * (2.5 ** -12 - 2.5 ** -6), rel=1e-14)
    U_out, F_out, r_out = pair_energy_force(float(np.nextafter(np.float32(2.5), np.float32(3))))
    assert r_out > 2.5 and U_out == 0.0 and F_out == 0.0


def test_lj_mixture_table_order():
    # AA, AB, BB entries are picked by the pair of types (upper-triangular order)
    pos = np.array([[2.0, 2, 2], [3.0, 2, 2], [2.0, 8, 2], [3.0, 8, 2], [2.0, 2, 8], [3.0, 2, 8]],
                   dtype=np.float32)
    typ = np.array([0, 0, 0, 1, 1, 1], dtype=np.int32)
    eps, sig = (1.0, 1.5, 0.5), (1.0, 0.8, 0.88)
    F, U, W, Ur, _ = O.lj(pos, np.full(3, 20, np.float32), PER, O.radius2(2.5), eps, sig, typ)

    def V(r, e, s):
        return 4 * e * ((s / r) ** 12 - (s / r) ** 6)
    assert 2 * Ur[0] == pytest.approx(V(1.0, 1.0, 1.0), rel=1e-13)
    assert 2 * Ur[2] == pytest.approx(V(1.0, 1.5, 0.8), rel=1e-13)
    assert 2 * Ur[4] == pytest.approx(V(1.0, 0.5, 0.88), rel=1e-13)


# ---------------------------------------------------------------- neighbour sets by hand

def test_neighbors_hand_cases():
    L = np.full(3, 10.0, np.float32)
    pos = np.array([
        [0.5, 5.0, 5.0],   # 0
        [9.0, 5.0, 5.0],   # 1: 1.5 from 0 across the x face
        [3.0, 5.0, 5.0],   # 2: exactly 2.5 from 0 (6.25 is exact in FP32)
        [0.2, 0.2, 0.2],   # 3
        [9.8, 9.8, 9.8],   # 4: across the corner from 3, d = sqrt(0.48)
        [5.0, 5.0, 5.0],   # 5: 2.0 from 2, 4.5 from 0 (excluded)
        [3.0, 7.5, 5.0],   # 6: 2.5 from 2 exactly, 3.54 from 0
    ], dtype=np.float32)
    sets = O.neighbor_sets(pos, L, PER, O.radius2(2.5))
    assert sets[0] == (1, 2)
    assert sets[1] == (0,)
    assert sets[2] == (0, 5, 6)
    assert sets[3] == (4,)
    assert sets[4] == (3,)
    assert sets[5] == (2,)
    assert sets[6] == (2,)
    # non-periodic x: the face-crossing pair disappears
    sets_np = O.neighbor_sets(pos, L, (0, 1, 1), O.radius2(2.5))
    assert 1 not in sets_np[0]
    assert 4 not in sets_np[3]  # corner pair needs the x image too


def test_neighbors_symmetric_and_no_self():
    s = inputs.lj_lattice(500, 0.8442, 1.0, seed=11)
    cnt, cols = O.neighbors(s.pos, s.box, PER, O.radius2(2.5, 0.3))
    sets = [set(cols[i, :cnt[i]].tolist()) for i in range(s.n)]
    for i in range(s.n):
        assert i not in sets[i]
        for j in sets[i]:
            assert i in sets[j]


def test_image_separation_is_rounded_once_and_symmetric():
    # pairs across the x face at separations within a few ulp of R: the image
    # separation must be the exact separation rounded once to FP32 (the larger
    # coordinate minus L is exact), so membership is symmetric in i and j
    rng = np.random.default_rng(21)
    R2 = O.radius2(2.5, 0.3)
    R = float(np.sqrt(np.float64(R2)))
    L = np.array([20.0, 240.0, 240.0], np.float32)
    g = np.stack(np.meshgrid(np.arange(40), np.arange(40), indexing="ij"), -1).reshape(-1, 2)
    npair = len(g)
    u = rng.uniform(0.01, 1.5, npair)                       # a near x = 0
    ang = rng.uniform(0.0, 0.6, npair)                      # pair direction off the x axis
    dx = R * np.cos(ang) * (1 + rng.uniform(-3e-7, 3e-7, npair))
    a = np.zeros((npair, 3))
    a[:, 0] = u
    a[:, 1:] = g * 6.0 + 1.0
    b = a.copy()
    b[:, 0] = u - dx + L[0]                                 # b near x = L, image at u - dx
    b[:, 1] += R * np.sin(ang)
    pos = np.concatenate([a, b]).astype(np.float32)
    sets = O.neighbor_sets(pos, L, PER, R2, cap=4)
    p32 = pos.astype(np.float64)
    hits = 0
    for k in range(npair):
        i, j = k, k + npair
        assert (j in sets[i]) == (i in sets[j]), k
        d = (p32[j] - p32[i]).copy()
        d[0] -= L[0] * (1.0 if d[0] > L[0] / 2 else 0.0)    # exact in FP64
        d32 = d.astype(np.float32)                          # exact separation, rounded once
        d2 = np.float32(np.float32(d32[0] * d32[0]) + np.float32(d32[1] * d32[1]))
        d2 = np.float32(d2 + np.float32(d32[2] * d32[2]))
        assert (j in sets[i]) == bool(d2 <= R2), k
        hits += j in sets[i]
    assert 0 < hits < npair  # the ties really straddle R


def test_neighbors_translation_and_permutation_invariant():
    s = inputs.lj_lattice(700, 0.8442, 1.0, seed=12)
    L = s.box
    base = O.neighbor_sets(s.pos, L, PER, O.radius2(2.5, 0.3))
    rng = np.random.default_rng(0)
    perm = rng.permutation(s.n)
    inv = np.argsort(perm)
    sets_p = O.neighbor_sets(s.pos[perm], L, PER, O.radius2(2.5, 0.3))
    for i in range(s.n):
        assert tuple(sorted(perm[list(sets_p[inv[i]])].tolist())) == base[i]
    # a translation by 1.0 (then wrapped) moves coordinates only by their FP32
    # rounding, so energy and forces agree to that rounding
    F0, U0, W0, _, _ = O.lj(s.pos, L, PER, O.radius2(2.5))
    shifted = s.pos + np.float32(0.0)
    shifted[:, 0] = np.where(shifted[:, 0] + 1.0 >= L[0], shifted[:, 0] + 1.0 - L[0],
                             shifted[:, 0] + 1.0).astype(np.float32)
    F1, U1, W1, _, _ = O.lj(shifted, L, PER, O.radius2(2.5))
    assert U1 == pytest.approx(U0, rel=1e-6)
    assert np.abs(F1 - F0).max() < 1e-4 * np.sqrt((F0 ** 2).mean())


# ---------------------------------------------------------------- cell sort

def test_cell_sort_invariants():
    s = inputs.lj_config("lj4096")
    nc = O.cell_grid(s.box, 2.5, 0.3)
    assert tuple(nc) == (6, 6, 6)  # 16.93 / 2.8 -> 6 cells of side 2.82 >= 2.8
    cid = O.cell_index(s.pos, s.box, nc)
    ncells = int(np.prod(nc))
    counts, offsets, order = O.cell_sort(cid, ncells)
    assert counts.sum() == s.n
    assert np.array_equal(offsets, np.concatenate([[0], np.cumsum(counts)]))
    assert np.array_equal(np.sort(order), np.arange(s.n))
    for c in range(ncells):
        members = order[offsets[c]:offsets[c + 1]]
        assert np.all(cid[members] == c)
        assert np.all(np.diff(members) > 0)
    # with the z key: same cells and offsets, each cell ordered by (z, index),
    # which makes every column of cells one run sorted by z
    z = s.pos[:, 2]
    counts_z, offsets_z, order_z = O.cell_sort(cid, ncells, z)
    assert np.array_equal(offsets_z, offsets)
    assert np.array_equal(order_z, np.lexsort((np.arange(s.n), z, cid)))  # cell, z, index
    col = nc[2]
    for c0 in range(0, ncells, col):
        run = order_z[offsets_z[c0]:offsets_z[c0 + col]]
        assert np.all(np.diff(z[run]) >= 0)
    zt = z.copy()
    zt[::2] = zt[1::2]  # pairs of equal keys, broken by index
    _, _, order_t = O.cell_sort(cid, ncells, zt)
    assert np.array_equal(order_t, np.lexsort((np.arange(s.n), zt, cid)))
    # each particle lies in (or within rounding of) its cell's geometric bounds
    side = s.box.astype(np.float64) / nc
    ijk = np.stack([cid // (nc[1] * nc[2]), (cid // nc[2]) % nc[1], cid % nc[2]], axis=1)
    lo = ijk * side - 1e-5
    hi = (ijk + 1) * side + 1e-5
    assert np.all((s.pos >= lo) & (s.pos <= hi))


def test_cell_index_faces():
    L = np.full(3, 9.0, np.float32)
    nc = O.cell_grid(L, 2.5, 0.3)
    assert tuple(nc) == (3, 3, 3)
    pos = np.array([[0.0, 0.0, 0.0], [3.0, 3.0, 3.0], [8.999999, 6.0, 5.9999995]],
                   dtype=np.float32)
    cid = O.cell_index(pos, L, nc)
    assert cid[0] == 0
    assert cid[1] == (1 * 3 + 1) * 3 + 1
    assert cid[2] == (2 * 3 + 2) * 3 + 1


# ---------------------------------------------------------------- sums over pairs

def test_newton_third_law():
    s = inputs.lj_config("lj4096")
    F, U, W, _, _ = O.lj(s.pos, s.box, PER, O.radius2(2.5))
    rms = math.sqrt((F ** 2).mean())
    assert np.abs(F.sum(axis=0)).max() <= 1e-12 * rms * math.sqrt(s.n)


def lattice_energy_per_atom(a, rc):
    """1/2 sum over lattice vectors 0 < |n| a <= rc of V(|n| a)."""
    m = int(math.ceil(rc / a)) + 1
    tot = 0.0
    for n in itertools.product(range(-m, m + 1), repeat=3):
        r2 = (n[0] ** 2 + n[1] ** 2 + n[2] ** 2) * a * a
        if 0 < r2 <= rc * rc:
            tot += 4 * (r2 ** -6 - r2 ** -3)
    return 0.5 * tot


def test_perfect_lattice_forces_and_energy():
    # spacing 17/16: every site (i + 1/2) a is exact in FP32
    s = inputs.lj_lattice(4096, 4096 / 17.0 ** 3, 1.0, seed=1, jitter=0.0)
    assert float(s.box[0]) == 17.0
    F, U, W, _, _ = O.lj(s.pos, s.box, PER, O.radius2(2.5))
    a = float(s.box[0]) / 16
    # symmetry: no net force on any site
    assert np.abs(F).max() < 1e-12
    assert U / s.n == pytest.approx(lattice_energy_per_atom(a, 2.5), rel=1e-6)
    # isotropic virial: W is diagonal with equal entries
    assert abs(W[0] - W[1]) < 1e-6 * abs(W[0]) and abs(W[0] - W[2]) < 1e-6 * abs(W[0])
    assert np.abs(W[3:]).max() < 1e-6 * abs(W[0])


def test_rows_match_full():
    s = inputs.lj_lattice(1000, 0.8442, 1.0, seed=3)
    F, U, W, Ur, Wr = O.lj(s.pos, s.box, PER, O.radius2(2.5))
    rows = np.array([0, 17, 999, 500])
    Fs, Us, Ws, Urs, Wrs = O.lj(s.pos, s.box, PER, O.radius2(2.5), rows=rows)
    assert np.array_equal(Fs, F[rows])
    assert np.array_equal(Urs, Ur[rows])


# ---------------------------------------------------------------- velocity Verlet

def diatomic(dt, T):
    """Two atoms oscillating about the LJ minimum; returns the max |E - E0|."""
    x = np.array([[5.0, 5, 5], [6.2, 5, 5]])
    v = np.array([[-0.3, 0, 0], [0.3, 0, 0]])
    n = int(round(T / dt))
    _, _, th = O.vv(x, v, np.full(3, 20.0), PER, 2.5, dt, n)
    E = th[:, 0] + th[:, 1]
    return np.abs(E - E[0]).max()


def test_verlet_second_order():
    e1 = diatomic(0.004, 2.0)
    e2 = diatomic(0.002, 2.0)
    e3 = diatomic(0.001, 2.0)
    assert 3.5 < e1 / e2 < 4.5
    assert 3.5 < e2 / e3 < 4.5


def test_verlet_time_reversible_and_momentum():
    s = inputs.lj_lattice(512, 0.8442, 1.0, seed=4)
    x0 = s.pos.astype(np.float64)
    v0 = s.vel.astype(np.float64)
    x1, v1, _ = O.vv(x0, v0, s.box, PER, 2.5, 0.005, 20)
    x2, v2, _ = O.vv(x1, -v1, s.box, PER, 2.5, 0.005, 20)
    d = x2 - x0
    d -= float(s.box[0]) * np.round(d / float(s.box[0]))
    assert np.abs(d).max() < 1e-9
    # total momentum is conserved (the FP32 start is zero-mean only to rounding)
    assert np.abs(v1.sum(axis=0) - v0.sum(axis=0)).max() < 1e-10


# ---------------------------------------------------------------- virial and rebuild criterion

def pair_virial_closed_form(d):
    """W_ab = r_a (s r_b) for one pair with separation d (each pair once),
    s = 24 (2 u^-7 - u^-4), u = |d|^2 (sigma = eps = 1), i.e. the outer
    product of the separation with the pair force; tr W = r F(r)."""
    u = float(np.dot(d, d))
    s = 24.0 * (2.0 * u ** -7 - u ** -4)
    return np.array([s * d[0] * d[0], s * d[1] * d[1], s * d[2] * d[2],
                     s * d[0] * d[1], s * d[0] * d[2], s * d[1] * d[2]])


def test_virial_two_particles_closed_form():
    # Along x: W_xx = r F(r) with F = -dV/dr from the section 4.1 potential,
    # every other component 0.  A dropped factor 1/2 (the pair is seen from
    # both rows) doubles it, a sign slip flips it.
    L = np.full(3, 20.0, np.float32)
    for r in [0.9, 1.0, 2.0 ** (1 / 6), 1.5, 2.4]:
        pos = np.array([[4.0, 5.0, 5.0], [4.0 + r, 5.0, 5.0]], dtype=np.float32)
        rr = float(pos[1, 0]) - float(pos[0, 0])
        F, U, W, _, Wr = O.lj(pos, L, PER, O.radius2(2.5))
        dVdr = -24.0 * (2.0 * rr ** -13 - rr ** -7)       # derivative of 4 (r^-12 - r^-6)
        assert W[0] == pytest.approx(-rr * dVdr, rel=1e-12, abs=1e-12), r
        assert np.abs(W[1:]).max() == 0.0
        # each row carries half of the pair's virial
        assert Wr[0, 0] == pytest.approx(Wr[1, 0], rel=1e-15)
    # an oblique pair across the x and y faces (image separation) gets the
    # full outer product, off-diagonal terms included
    pos = np.array([[0.25, 19.5, 7.0], [19.5, 0.5, 7.75]], dtype=np.float32)
    F, U, W, _, _ = O.lj(pos, L, PER, O.radius2(2.5))
    d = np.array([0.25 - (19.5 - 20.0), (19.5 - 20.0) - 0.5, 7.0 - 7.75])  # x_0 - x_1 (image)
    assert np.allclose(W, pair_virial_closed_form(d), rtol=1e-12, atol=1e-12)
    # the pair force itself: F_0 = s d
    u = float(np.dot(d, d))
    s = 24.0 * (2.0 * u ** -7 - u ** -4)
    assert np.allclose(F[0], s * d, rtol=1e-12, atol=1e-12)
    assert np.allclose(F[1], -s * d, rtol=1e-12, atol=1e-12)


def lattice_virial_trace(n_atoms, a, rc):
    """tr W = sum over pairs of r F(r) = 1/2 N sum over lattice vectors
    0 < |n| a <= rc of 24 (2 r^-12 - r^-6) (sigma = eps = 1)."""
    m = int(math.ceil(rc / a)) + 1
    tot = 0.0
    for n in itertools.product(range(-m, m + 1), repeat=3):
        r2 = (n[0] ** 2 + n[1] ** 2 + n[2] ** 2) * a * a
        if 0 < r2 <= rc * rc:
            tot += 24.0 * (2.0 * r2 ** -6 - r2 ** -3)
    return 0.5 * n_atoms * tot


def test_virial_trace_perfect_lattice():
    s = inputs.lj_lattice(4096, 4096 / 17.0 ** 3, 1.0, seed=1, jitter=0.0)
    F, U, W, _, _ = O.lj(s.pos, s.box, PER, O.radius2(2.5))
    a = float(s.box[0]) / 16
    tr = W[0] + W[1] + W[2]
    assert tr == pytest.approx(lattice_virial_trace(s.n, a, 2.5), rel=1e-9)
    # isotropy of a cubic lattice: each diagonal entry is a third of the trace
    for k in range(3):
        assert W[k] == pytest.approx(tr / 3, rel=1e-9)


def test_max_disp2_hand_cases():
    # minimum-image displacement in the predicate's FP32 arithmetic; all
    # coordinates are exact binary fractions, so every value is exact
    L = np.full(3, 16.0, np.float32)
    ref = np.array([[0.25, 8.0, 8.0],     # crosses the x face downwards: 15.5 is 0.75 away
                    [4.0, 4.0, 4.0],      # moves 0.5 in y
                    [15.75, 15.75, 8.0],  # crosses the x and y faces upwards
                    [8.0, 8.0, 8.0]], dtype=np.float32)
    pos = np.array([[15.5, 8.0, 8.0],
                    [4.0, 4.5, 4.0],
                    [0.25, 0.125, 8.0],
                    [8.0, 8.0, 8.0]], dtype=np.float32)
    per_row = [0.5625, 0.25, 0.25 + 0.140625, 0.0]
    for k in range(4):
        assert float(O.max_disp2(pos[k:k + 1], ref[k:k + 1], L, PER)) == per_row[k]
    assert float(O.max_disp2(pos, ref, L, PER)) == 0.5625
    # a corner crossing on all three axes
    r3 = np.array([[0.25, 0.25, 0.25]], np.float32)
    p3 = np.array([[15.75, 15.75, 15.75]], np.float32)
    assert float(O.max_disp2(p3, r3, L, PER)) == 0.75
    # without periodic x the face crossing is a long move
    assert float(O.max_disp2(pos[:1], ref[:1], L, (0, 1, 1))) == 15.25 ** 2


def test_rebuild_criterion_is_strict():
    # One free particle (no pairs) moves 1/32 per step: after two steps its
    # squared displacement equals the threshold exactly and no rebuild is due
    # (the rule is "exceeds"); the third step rebuilds, and the count restarts
    # from the new reference.  A non-strict rule would rebuild at 2, 4, 6.
    L = np.full(3, 16.0, np.float32)
    x0 = np.array([[15.9375, 8.0, 8.0]], np.float32)
    v0 = np.array([[0.25, 0.0, 0.0]], np.float32)
    dt = np.float32(0.125)
    thr = np.float32(0.0625 ** 2)
    xs, vs, Fs, nb = O.lj_traj_f32(x0, v0, L, PER, O.radius2(2.5), dt, 7, thr)
    assert nb == 1 + 2  # the initial build, then steps 3 and 6
    assert np.all(Fs == 0.0) and np.all(vs[:, 0, 0] == 0.25)
    # positions are wrapped into [0, L) at rebuilds only: the particle is at
    # 16.0 after step 2 (not wrapped, no rebuild), back at 0.03125 after step 3
    assert xs[2, 0, 0] == np.float32(16.0)
    assert xs[3, 0, 0] == np.float32(0.03125)
    assert xs[6, 0, 0] == np.float32(0.125)
    assert float(O.max_disp2(xs[2], xs[0], L, PER)) == float(thr)
