"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle for the
LJ hot path: cell lists and Verlet sets bit-exact, forces within 1e-5 of the
RMS force (max norm), energy and virial within 1e-6, velocity-Verlet steps,
edge cases and error paths."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1804_07598_amd import inputs

pytestmark = pytest.mark.gpu

PER = (1, 1, 1)
RC, SKIN = 2.5, 0.3
FORCE_TOL = 1e-5
ENERGY_TOL = 1e-6


def make_sim(s, **kw):
    from paper_1804_07598_amd.sim import ParticleSim
    return ParticleSim(s.pos, s.box, PER, vel=s.vel, typ=s.typ, r_cut=kw.pop("r_cut", RC),
                       skin=kw.pop("skin", SKIN), **kw)


def np_(t):
    return t.detach().cpu().numpy()


def force_error(Fg, F64):
    rms = math.sqrt((F64 ** 2).mean())
    e = np.abs(Fg.astype(np.float64) - F64) / rms
    return float(e.max()), rms


def check_lj(sim, pos, L, eps=(1.0,) * 3, sig=(1.0,) * 3, typ=None, n_types=1, rows=None):
    """Evaluate forces on the GPU and compare with the oracle at the same positions."""
    out = np_(sim.lj_forces(eps, sig, n_types))
    _, _, Fg = sim.get()
    Fg = np_(Fg)
    F64, U64, W64, Ur, _ = O.lj(pos, L, PER, O.radius2(RC), eps, sig, typ, rows=rows)
    if rows is not None:
        Fg = Fg[rows]
    err, rms = force_error(Fg, F64)
    assert err <= FORCE_TOL, (err, rms)
    if rows is None:
        assert abs(out[0] - U64) <= ENERGY_TOL * abs(U64), (out[0], U64)
        scale = O.lj_virial_scale(pos, L, PER, O.radius2(RC), eps, sig, typ)
        assert np.abs(out[2:] - W64).max() <= ENERGY_TOL * scale, (out[2:], W64)
    return out, F64


# ---------------------------------------------------------------- cell list

# the two sparse cases have 85,184 and 17,373,979 cells: the scan then runs
# over the whole device, in 21 and 4242 tiles of 4096 cells
@pytest.mark.parametrize("n,rho,seed", [(4096, 0.8442, 1), (1000, 0.8442, 7), (256, 0.6, 4001),
                                        (20000, 0.01, 12), (50000, 1.3e-4, 13)])
def test_cell_list_bit_exact(n, rho, seed):
    s = inputs.lj_lattice(n, rho, 1.0, seed)
    sim = make_sim(s)
    sim.build_cell_list()
    ncell, off, order = sim.cell_list()
    nc = O.cell_grid(s.box, RC, SKIN)
    assert tuple(ncell) == tuple(nc)
    cid = O.cell_index(s.pos, s.box, nc)
    counts, offsets, order64 = O.cell_sort(cid, int(np.prod(nc)), s.pos[:, 2])
    assert np.array_equal(np_(off), offsets)
    assert np.array_equal(np_(order), order64)


# ---------------------------------------------------------------- Verlet sets

def compare_sets(sim, pos, L, R2, rows=None):
    counts, cols = sim.neighbors()
    counts, cols = np_(counts), np_(cols)
    ocnt, ocols = O.neighbors(pos, L, PER, R2, rows=rows, cap=sim.max_nbr)
    idx = range(len(pos)) if rows is None else rows
    for r, i in enumerate(idx):
        got = np.sort(cols[i, :counts[i]])
        exp = ocols[r, :ocnt[r]]
        assert counts[i] == ocnt[r] and np.array_equal(got, exp), i


@pytest.mark.parametrize("n,rho,seed", [(4096, 0.8442, 1), (1000, 0.8442, 7), (256, 0.6, 4001),
                                        (4097, 0.8442, 9)])
def test_verlet_sets_bit_exact(n, rho, seed):
    s = inputs.lj_lattice(n, rho, 1.0, seed)
    sim = make_sim(s)
    compare_sets(sim, s.pos, s.box, O.radius2(RC, SKIN))


# ---------------------------------------------------------------- forces

@pytest.mark.parametrize("n,rho,seed", [(4096, 0.8442, 1), (1000, 0.8442, 7), (256, 0.6, 4001),
                                        (4097, 0.8442, 9)])
def test_lj_forces_match_oracle(n, rho, seed):
    s = inputs.lj_lattice(n, rho, 1.0, seed)
    sim = make_sim(s)
    check_lj(sim, s.pos, s.box)


def test_lj_mixture_forces():
    s = inputs.lj_lattice(4096, 1.2, 1.0, seed=5, mixture=True)
    sim = make_sim(s)
    m = inputs.LJ_MIXTURE
    check_lj(sim, s.pos, s.box, m["eps"], m["sig"], s.typ, n_types=2)


def test_lj_deterministic_and_permutation_invariant():
    import torch
    s = inputs.lj_config("lj4096")
    a = make_sim(s)
    a.lj_forces()
    _, _, Fa = a.get()
    b = make_sim(s)
    b.lj_forces()
    _, _, Fb = b.get()
    assert torch.equal(Fa, Fb)  # bitwise run-to-run
    perm = np.random.default_rng(3).permutation(s.n)
    sp = inputs.LJSystem(s.pos[perm], s.vel[perm], s.typ[perm], s.L, s.seed, s.rho, s.T)
    c = make_sim(sp)
    c.lj_forces()
    _, _, Fc = c.get()
    Fc = np_(Fc)
    back = np.empty_like(Fc)
    back[perm] = Fc
    err, _ = force_error(back, np_(Fa).astype(np.float64))
    assert err < 1e-6


# ---------------------------------------------------------------- time stepping

def test_velocity_verlet_steps():
    s = inputs.lj_config("lj4096")
    sim = make_sim(s)
    th = np_(sim.step(10, dt=0.005))
    sim.check()
    p, v, f = (np_(t) for t in sim.get())
    ke = 0.5 * float((v.astype(np.float64) ** 2).sum())
    assert th[-1, 1] == pytest.approx(ke, rel=1e-6)
    # the oracle's own FP64 trajectory from the same start: FP32 storage of x, v
    # and F perturbs each step by ~1e-7 relative, far below these bounds
    x64, v64, th64 = O.vv(s.pos.astype(np.float64), s.vel.astype(np.float64), s.box, PER, RC,
                          0.005, 10)
    d = p.astype(np.float64) - x64
    d -= float(s.box[0]) * np.round(d / float(s.box[0]))
    assert np.abs(d).max() < 1e-4
    assert np.abs(v.astype(np.float64) - v64).max() < 1e-4
    E64 = th64[1:, 0] + th64[1:, 1]
    assert np.abs(th[:, 0] - th64[1:, 0]).max() < 1e-5 * abs(E64[0])
    assert np.abs(th[:, 1] - th64[1:, 1]).max() < 1e-5 * abs(E64[0])


def kept_lists_cover(sim, L, rows=None):
    """The lists the step loop left behind hold every pair within r_cut now."""
    from list_coverage import assert_lists_cover
    counts, cols = (np_(t) for t in sim.neighbors())
    p, _, _ = sim.get()
    return assert_lists_cover(counts, cols, np_(p), L, RC, rows=rows)


def test_rebuilds_follow_displacement():
    s = inputs.lj_config("lj4096")
    sim = make_sim(s)
    for _ in range(6):
        sim.step(10, dt=0.005)
        kept_lists_cover(sim, s.box)
    rebuilds, longest, total = sim.counters()
    assert rebuilds >= 2  # the initial build plus at least one automatic rebuild


def test_nve_energy_bounded():
    s = inputs.lj_config("lj4096")
    sim = make_sim(s)
    th = np_(sim.step(400, dt=0.005))
    E = th[:, 0] + th[:, 1]
    ref = O.vv(s.pos.astype(np.float64), s.vel.astype(np.float64), s.box, PER, RC, 0.005, 400)[2]
    E64 = ref[1:, 0] + ref[1:, 1]
    # same drift as the FP64 trajectory (truncated LJ drifts while the lattice melts)
    assert abs((E[-1] - E[0]) - (E64[-1] - E64[0])) < 2e-3 * abs(E64[0])


# ---------------------------------------------------------------- edges and errors

def test_small_box_two_cells():
    s = inputs.lj_lattice(256, 0.6, 1.0, seed=4000)
    sim = make_sim(s)
    assert sim.cell_list()[0] == (2, 2, 2)
    compare_sets(sim, s.pos, s.box, O.radius2(RC, SKIN))
    check_lj(sim, s.pos, s.box)


def test_particles_on_faces_and_empty_cells():
    rng = np.random.default_rng(5)
    L = np.float32(16.0)
    # half of the box empty, particles exactly on cell faces and on x = 0
    pts = rng.uniform(0, 8.0, size=(900, 3)).astype(np.float32)
    pts[:30, 0] = 0.0
    pts[30:60, 1] = np.float32(16.0 / 5)  # a cell face (5 cells of 3.2)
    pts = np.unique(pts, axis=0)
    s = inputs.LJSystem(pts, np.zeros_like(pts), np.zeros(len(pts), np.int32), float(L), 0, 0, 0)
    # lists longer than the lane-group build keeps in LDS (128) occur here
    sim = make_sim(s, max_nbr=512)
    assert sim.counters()[1] > 128
    compare_sets(sim, s.pos, s.box, O.radius2(RC, SKIN))


def test_set_positions_moved_by_whole_periods():
    # a small move plus a whole-period shift is a small move of the periodic
    # system: the forces must be those of the wrapped positions
    s = inputs.lj_lattice(4096, 0.8442, 1.0, seed=21)
    sim = make_sim(s)
    check_lj(sim, s.pos, s.box)
    rng = np.random.default_rng(22)
    moved = (s.pos + rng.uniform(-0.02, 0.02, s.pos.shape)).astype(np.float32)
    moved = np.mod(moved, np.float32(s.box)).astype(np.float32)
    shifted = moved.copy()
    k = rng.choice(len(moved), 300, replace=False)
    shifted[k] += (rng.integers(-1, 2, (300, 3)) * s.box).astype(np.float32)
    sim.set_positions(shifted)
    sim.lj_forces()
    pg = np_(sim.get()[0])
    # wrapped back into the box, up to the FP32 rounding of (x +- L) -+ L
    assert pg.min() >= 0 and (pg < s.box).all()
    d = pg - moved
    d -= s.box * np.round(d / s.box)
    assert np.abs(d).max() <= 4e-6 * s.box.max()
    check_lj(sim, pg, s.box)


@pytest.mark.parametrize("tuning", [None, (5, 0, 8)])
def test_set_particles_again_equals_a_fresh_context(tuning):
    # a second fpm_set_particles with the same count keeps the layout and the
    # captured step graphs; the state must be that of a fresh context
    import torch
    a = inputs.lj_lattice(4096, 0.8442, 1.0, seed=31)
    b = inputs.lj_lattice(4096, 0.8442, 1.2, seed=32)
    sim = make_sim(a, tuning=tuning)
    sim.step(30, dt=0.005)  # graphs captured, lists rebuilt on the way
    sim.set_particles(b.pos, b.vel)
    th = np_(sim.step(25, dt=0.005))
    ref = make_sim(b, tuning=tuning)
    th_ref = np_(ref.step(25, dt=0.005))
    for x, y in zip(sim.get(), ref.get()):
        assert torch.equal(x, y)
    assert np.array_equal(th, th_ref)
    assert sim.counters() == ref.counters()
    sim.check()


@pytest.mark.parametrize("tuning", [None, (3, 0, 8), (4, 8, 8), (5, 0, 8)])
def test_overflow_is_reported(tuning):
    from paper_1804_07598_amd._lib import FpmError, FPM_EOVERFLOW
    s = inputs.lj_lattice(1000, 0.8442, 1.0, seed=7)
    sim = make_sim(s, max_nbr=8, tuning=tuning)
    with pytest.raises(FpmError) as e:
        sim.check()
    assert e.value.code == FPM_EOVERFLOW
    with pytest.raises(FpmError):
        sim.neighbors()
    # a larger capacity gives the exact sets again
    sim2 = make_sim(s, max_nbr=160, tuning=tuning)
    compare_sets(sim2, s.pos, s.box, O.radius2(RC, SKIN))


@pytest.mark.parametrize("n", [1, 2])
def test_degenerate_systems(n):
    # one particle, or two beyond the list radius: empty lists, zero forces and
    # energy, and free flight under velocity Verlet
    pos = np.array([[1.0, 2.0, 3.0], [7.0, 8.0, 9.0]], np.float32)[:n]
    vel = np.array([[0.5, -0.25, 0.125], [-1.0, 0.0, 2.0]], np.float32)[:n]
    s = inputs.LJSystem(pos, vel, np.zeros(n, np.int32), 12.0, 0, 0, 0)
    sim = make_sim(s)
    counts, _ = sim.neighbors()
    assert np.all(np_(counts) == 0)
    out = np_(sim.lj_forces())
    _, _, f = sim.get()
    assert np.all(np_(f) == 0) and np.all(out == 0)
    sim.step(4, dt=0.25)
    sim.check()
    p, v, _ = (np_(t) for t in sim.get())
    assert np.array_equal(v, vel)
    assert np.allclose(p, pos + 4 * 0.25 * vel, rtol=0, atol=1e-6)


def test_cutoff_error():
    from paper_1804_07598_amd._lib import FpmError, FPM_ECUTOFF
    s = inputs.lj_lattice(64, 0.8442, 1.0, seed=2)  # L = 4.2 < 2 * 2.8
    with pytest.raises(FpmError) as e:
        make_sim(s)
    assert e.value.code == FPM_ECUTOFF


# ---------------------------------------------------------------- 1M atoms, sampled

def sampled_rows(pos, L, seed, n_face=1024, n_rand=3072):
    """Rows for full-size checks: n_face particles within the list radius of a
    periodic face (their lists hold image pairs) and n_rand random ones."""
    rng = np.random.default_rng(seed)
    near = np.nonzero(((pos < RC + SKIN) | (pos > L - (RC + SKIN))).any(axis=1))[0]
    face = rng.choice(near, n_face, replace=False)
    rest = rng.choice(np.setdiff1d(np.arange(len(pos)), face), n_rand, replace=False)
    return np.sort(np.concatenate([face, rest]))


def test_lj_1m_sampled_rows():
    s = inputs.lj_config("lj1m")
    sim = make_sim(s)
    rows = sampled_rows(s.pos, s.box, 2)
    sim.lj_forces()
    compare_sets(sim, s.pos, s.box, O.radius2(RC, SKIN), rows=rows)
    check_lj(sim, s.pos, s.box, rows=rows)
    # after steps with rebuilds (the step loop's fused force kernels, the launch
    # configuration the bench times) the kept lists still cover the force set,
    # the forces at the reached positions match the oracle on sampled rows, and
    # the total energy stays put (truncated LJ, 40 steps)
    th = np_(sim.step(40, dt=0.005))
    sim.check()
    assert sim.counters()[0] >= 2
    kept_lists_cover(sim, s.box, rows=np.random.default_rng(3).choice(s.n, 4096, replace=False))
    p, _, f = (np_(t) for t in sim.get())
    rows2 = sampled_rows(p, s.box, 4)
    F64, _, _, _, _ = O.lj(p, s.box, PER, O.radius2(RC), rows=rows2)
    err, _ = force_error(f[rows2], F64)
    assert err <= FORCE_TOL
    E = th[:, 0] + th[:, 1]
    assert abs(E[-1] - E[0]) < 1e-3 * abs(E[0])
