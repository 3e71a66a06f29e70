"""FP64 CPU oracle for the OpenFPM particle hot path (arXiv 1804.07598).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the bench's
CPU-baseline leg, never by the product package.  The C sources next to this
file are compiled with gcc (see build.py) and loaded with ctypes.  Nothing here
shares code with the HIP library.

Functions take numpy arrays in the caller's particle order:
positions (n, 3) float32 (the FP32 values the GPU sees, promoted exactly) or
float64 for the oracle's own FP64 trajectories; box L (3,) float32 with origin
0; per (3,) int periodic flags; pair tables eps/sig of 3 entries (AA, AB, BB).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")


def _opt(ptype):
    """ndpointer that also accepts None (NULL)."""
    class _P(ptype):  # type: ignore[misc, valid-type]
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return ptype.from_param(obj)
    return _P


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.oracle_radius2_f32.restype = C.c_float
        L.oracle_radius2_f32.argtypes = [C.c_float, C.c_float]
        L.oracle_cell_grid.argtypes = [f32p, C.c_float, C.c_float, i32p]
        L.oracle_cell_index.argtypes = [C.c_int64, f32p, f32p, i32p, i32p]
        L.oracle_cell_sort.argtypes = [C.c_int64, i32p, _opt(f32p), C.c_int32, i32p, i32p, i32p]
        L.oracle_neighbors.restype = C.c_int
        L.oracle_neighbors.argtypes = [C.c_int64, f32p, f32p, i32p, C.c_float, _opt(i64p),
                                       C.c_int64, i32p, i32p, C.c_int64]
        L.oracle_max_disp2.restype = C.c_float
        L.oracle_max_disp2.argtypes = [C.c_int64, f32p, f32p, f32p, i32p]
        L.oracle_lj_rows.argtypes = [C.c_int64, f32p, _opt(i32p), f32p, i32p, C.c_float, f64p,
                                     f64p, _opt(i64p), C.c_int64, f64p, _opt(f64p), _opt(f64p)]
        L.oracle_lj_virial_scale.restype = C.c_double
        L.oracle_lj_virial_scale.argtypes = [C.c_int64, f32p, _opt(i32p), f32p, i32p, C.c_float,
                                             f64p, f64p]
        L.oracle_vv.argtypes = [C.c_int64, f64p, f64p, _opt(i32p), f64p, i32p, C.c_double, f64p,
                                f64p, C.c_double, C.c_double, C.c_int32, _opt(f64p)]
        L.oracle_lj_forces_f64.argtypes = [C.c_int64, f64p, _opt(i32p), f64p, i32p, C.c_double,
                                           f64p, f64p, f64p, f64p]
        L.oracle_num_threads.restype = C.c_int
        L.oracle_num_threads.argtypes = []
        if hasattr(L, "oracle_sph_rows"):
            L.oracle_sph_rows.argtypes = [C.c_int64, f32p, f32p, f32p, i32p, f32p, i32p, C.c_float,
                                          f64p, _opt(i64p), C.c_int64, f64p, f64p, f64p]
            L.oracle_sph_kernel_w.restype = C.c_double
            L.oracle_sph_kernel_w.argtypes = [C.c_double, C.c_double]
            L.oracle_sph_cubic_w.restype = C.c_double
            L.oracle_sph_cubic_w.argtypes = [C.c_double, C.c_double]
            L.oracle_sph_kernel_dwdr.restype = C.c_double
            L.oracle_sph_kernel_dwdr.argtypes = [C.c_double, C.c_double, C.c_int]
        if hasattr(L, "oracle_dem_forces"):
            L.oracle_dem_forces.restype = C.c_int
            L.oracle_dem_forces.argtypes = [C.c_int64, f64p, f64p, f64p, f32p, i32p, f64p, C.c_int,
                                            i64p, f64p, f64p, f64p, i64p, f64p, i32p]
            L.oracle_dem_leapfrog.argtypes = [C.c_int64, f64p, f64p, f64p, f64p, f64p, f64p]
            L.oracle_dem_forces_rows.argtypes = [C.c_int64, f64p, f64p, f64p, f32p, i32p, f64p,
                                                 i64p, C.c_int64, f64p, f64p, i32p]
        if hasattr(L, "oracle_lj_vjp"):
            L.oracle_lj_vjp.argtypes = [C.c_int64, f32p, _opt(i32p), f32p, i32p, C.c_float, f64p,
                                        f64p, f64p, f64p, f64p]
            L.oracle_lj_vjp_f64.argtypes = [C.c_int64, f64p, _opt(i32p), f64p, i32p, C.c_double,
                                            f64p, f64p, f64p, f64p, f64p]
            L.oracle_lj_traj.argtypes = [C.c_int64, f64p, f64p, _opt(i32p), f64p, i32p,
                                         C.c_double, f64p, f64p, C.c_double, C.c_int32, f64p,
                                         f64p, _opt(f64p)]
            L.oracle_lj_traj_adjoint.argtypes = [C.c_int64, f64p, _opt(i32p), f64p, i32p,
                                                 C.c_double, f64p, f64p, C.c_double, C.c_int32,
                                                 f64p, f64p, f64p, f64p]
            L.oracle_lj_traj_f32.restype = C.c_int32
            L.oracle_lj_traj_f32.argtypes = [C.c_int64, f32p, f32p, _opt(i32p), f32p, i32p,
                                             C.c_float, f64p, f64p, C.c_float, C.c_float,
                                             C.c_int32, C.c_int32, f32p, f32p, f32p]
            L.oracle_lj_traj_adjoint_f32.argtypes = [C.c_int64, f32p, _opt(i32p), f32p, i32p,
                                                     C.c_float, f64p, f64p, C.c_double,
                                                     C.c_int32, f64p, f64p, f64p, f64p]
        _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _per(per):
    return _i32(np.broadcast_to(np.asarray(per, dtype=np.int32), (3,)))


def _box(L):
    return _f32(np.broadcast_to(np.asarray(L, dtype=np.float32), (3,)))


def radius2(r_cut: float, skin: float = 0.0) -> np.float32:
    """R^2 rounded once to FP32 from (r_cut + skin) in FP64."""
    return np.float32(lib().oracle_radius2_f32(float(np.float32(r_cut)), float(np.float32(skin))))


def cell_grid(L, r_cut: float, skin: float = 0.0) -> np.ndarray:
    out = np.zeros(3, np.int32)
    lib().oracle_cell_grid(_box(L), float(np.float32(r_cut)), float(np.float32(skin)), out)
    return out


def cell_index(pos, L, ncell) -> np.ndarray:
    pos = _f32(pos)
    out = np.empty(len(pos), np.int32)
    lib().oracle_cell_index(len(pos), pos, _box(L), _i32(ncell), out)
    return out


def cell_sort(cid, ncells: int, z=None):
    """(counts, offsets, order) of a counting sort by cell; inside a cell by z
    then particle index (by particle index alone when z is None)."""
    cid = _i32(cid)
    counts = np.empty(ncells, np.int32)
    offsets = np.empty(ncells + 1, np.int32)
    order = np.empty(len(cid), np.int32)
    lib().oracle_cell_sort(len(cid), cid, None if z is None else _f32(z), int(ncells), counts,
                           offsets, order)
    return counts, offsets, order


def neighbors(pos, L, per, R2, rows=None, cap: int = 512):
    """Brute-force neighbour sets: (counts, cols (nrows, cap)) in ascending j.

    Raises OverflowError if a row has more than cap neighbours."""
    pos = _f32(pos)
    nr = len(pos) if rows is None else len(rows)
    rows_a = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    counts = np.empty(nr, np.int32)
    cols = np.full((nr, cap), -1, np.int32)
    rc = lib().oracle_neighbors(len(pos), pos, _box(L), _per(per), float(np.float32(R2)), rows_a,
                                nr, counts, cols, cap)
    if rc != 0:
        raise OverflowError("neighbour cap exceeded")
    return counts, cols


def neighbor_sets(pos, L, per, R2, rows=None, cap: int = 512):
    counts, cols = neighbors(pos, L, per, R2, rows, cap)
    return [tuple(cols[r, :counts[r]].tolist()) for r in range(len(counts))]


def max_disp2(pos, ref, L, per) -> np.float32:
    pos, ref = _f32(pos), _f32(ref)
    return np.float32(lib().oracle_max_disp2(len(pos), pos, ref, _box(L), _per(per)))


def lj(pos, L, per, rc2, eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0), typ=None, rows=None):
    """FP64 LJ on the FP32 pair set.  Returns (F rows x 3, U total, W total (6,),
    U per row, W per row).  Totals cover the requested rows only."""
    pos = _f32(pos)
    nr = len(pos) if rows is None else len(rows)
    rows_a = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    F = np.empty((nr, 3), np.float64)
    U = np.empty(nr, np.float64)
    W = np.empty((nr, 6), np.float64)
    lib().oracle_lj_rows(len(pos), pos, None if typ is None else _i32(typ), _box(L), _per(per),
                         float(np.float32(rc2)), _f64(eps), _f64(sig), rows_a, nr, F, U, W)
    return F, float(U.sum()), W.sum(axis=0), U, W


def lj_virial_scale(pos, L, per, rc2, eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0), typ=None) -> float:
    pos = _f32(pos)
    return float(lib().oracle_lj_virial_scale(len(pos), pos, None if typ is None else _i32(typ),
                                              _box(L), _per(per), float(np.float32(rc2)),
                                              _f64(eps), _f64(sig)))


def lj_forces_f64(x, L, per, rc, eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0), typ=None):
    """FP64 forces of FP64 positions with an FP64 cut-off test: (F, U)."""
    x = _f64(x)
    F = np.empty_like(x)
    U = np.zeros(1, np.float64)
    lib().oracle_lj_forces_f64(len(x), x, None if typ is None else _i32(typ),
                               _f64(np.broadcast_to(np.asarray(L, np.float64), (3,))), _per(per),
                               float(rc), _f64(eps), _f64(sig), F, U)
    return F, float(U[0])


def vv(x, v, L, per, rc, dt, nsteps, eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0), typ=None,
       mass: float = 1.0):
    """FP64 velocity-Verlet trajectory.  Returns (x, v, thermo (nsteps+1, 2) = [U, KE])."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    thermo = np.empty((nsteps + 1, 2), np.float64)
    lib().oracle_vv(len(x), x, v, None if typ is None else _i32(typ),
                    _f64(np.broadcast_to(np.asarray(L, np.float64), (3,))), _per(per), float(rc),
                    _f64(eps), _f64(sig), float(mass), float(dt), int(nsteps), thermo)
    return x, v, thermo


def _box64(L):
    return _f64(np.broadcast_to(np.asarray(L, np.float64), (3,)))


def lj_vjp(pos, L, per, rc2, lam, eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0), typ=None):
    """Vector-Jacobian product of the forces at FP32 positions on the FP32 pair
    set: (dL/dx (n, 3), dL/dtheta (6,) = eps AA, AB, BB, sig AA, AB, BB) for
    lam = dL/dF."""
    pos = _f32(pos)
    gx = np.empty((len(pos), 3), np.float64)
    gt = np.empty(6, np.float64)
    lib().oracle_lj_vjp(len(pos), pos, None if typ is None else _i32(typ), _box(L), _per(per),
                        float(np.float32(rc2)), _f64(eps), _f64(sig), _f64(lam), gx, gt)
    return gx, gt


def lj_vjp_f64(x, L, per, rc, lam, eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0), typ=None):
    """The same at FP64 positions with the FP64 cut-off test u <= rc^2."""
    x = _f64(x)
    gx = np.empty_like(x)
    gt = np.empty(6, np.float64)
    lib().oracle_lj_vjp_f64(len(x), x, None if typ is None else _i32(typ), _box64(L), _per(per),
                            float(rc), _f64(eps), _f64(sig), _f64(lam), gx, gt)
    return gx, gt


def lj_traj(x0, v0, L, per, rc, dt, nsteps, eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0), typ=None):
    """FP64 velocity-Verlet trajectory: (xs, Fs, vs), each (nsteps + 1, n, 3)."""
    x0 = _f64(x0)
    n = len(x0)
    xs = np.empty((nsteps + 1, n, 3), np.float64)
    Fs = np.empty_like(xs)
    vs = np.empty_like(xs)
    lib().oracle_lj_traj(n, x0, _f64(v0), None if typ is None else _i32(typ), _box64(L),
                         _per(per), float(rc), _f64(eps), _f64(sig), float(dt), int(nsteps), xs,
                         Fs, vs)
    return xs, Fs, vs


def lj_traj_adjoint(xs, L, per, rc, dt, fbar, eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0),
                    typ=None):
    """Reverse-mode derivative through an FP64 trajectory xs (K + 1, n, 3) of a
    loss with dL/dF_k = fbar (K + 1, n, 3): (dL/dx0, dL/dv0, dL/dtheta (6,))."""
    xs = _f64(xs)
    K = xs.shape[0] - 1
    n = xs.shape[1]
    xb = np.empty((n, 3), np.float64)
    vb = np.empty((n, 3), np.float64)
    gt = np.empty(6, np.float64)
    lib().oracle_lj_traj_adjoint(n, xs, None if typ is None else _i32(typ), _box64(L), _per(per),
                                 float(rc), _f64(eps), _f64(sig), float(dt), int(K), _f64(fbar),
                                 xb, vb, gt)
    return xb, vb, gt


def lj_traj_f32(x0, v0, L, per, rc2, dt, nsteps, disp2_thr, rebuild_every=0,
                eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0), typ=None):
    """Velocity-Verlet trajectory with FP32 particle state (see oracle_adjoint.c):
    (xs, vs, Fs) float32 (nsteps + 1, n, 3) and the number of rebuilds."""
    x0 = _f32(x0)
    n = len(x0)
    xs = np.empty((nsteps + 1, n, 3), np.float32)
    vs = np.empty_like(xs)
    Fs = np.empty_like(xs)
    nb = lib().oracle_lj_traj_f32(n, x0, _f32(v0), None if typ is None else _i32(typ), _box(L),
                                  _per(per), float(np.float32(rc2)), _f64(eps), _f64(sig),
                                  float(np.float32(dt)), float(np.float32(disp2_thr)),
                                  int(rebuild_every), int(nsteps), xs, vs, Fs)
    return xs, vs, Fs, int(nb)


def lj_traj_adjoint_f32(xs, L, per, rc2, dt, fbar, eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0),
                        typ=None):
    """lj_traj_adjoint over FP32 states with the FP32 pair set of each state."""
    xs = _f32(xs)
    K = xs.shape[0] - 1
    n = xs.shape[1]
    xb = np.empty((n, 3), np.float64)
    vb = np.empty((n, 3), np.float64)
    gt = np.empty(6, np.float64)
    lib().oracle_lj_traj_adjoint_f32(n, xs, None if typ is None else _i32(typ), _box(L),
                                     _per(per), float(np.float32(rc2)), _f64(eps), _f64(sig),
                                     float(dt), int(K), _f64(fbar), xb, vb, gt)
    return xb, vb, gt


def sph_kernel_w(r: float, h: float) -> float:
    """Wendland C2 kernel value W(r) with support 2h."""
    return float(lib().oracle_sph_kernel_w(float(r), float(h)))


def sph_cubic_w(r: float, h: float) -> float:
    """Cubic spline kernel value W(r) with support 2h (section 4.2's kernel)."""
    return float(lib().oracle_sph_cubic_w(float(r), float(h)))


def sph_kernel_dwdr(r: float, h: float, kernel: int) -> float:
    """dW/dr of the Wendland C2 (kernel 0) or cubic spline (kernel 1) kernel."""
    return float(lib().oracle_sph_kernel_dwdr(float(r), float(h), int(kernel)))


def sph_params_array(h, mass, rho0, c0, gamma=7.0, alpha=0.1, eta2=None, g=(0.0, 0.0, -9.81),
                     kernel=0, cbar=0.0):
    """The oracle's SPH parameter vector {h, m, rho0, c0, gamma, alpha, eta2, gx, gy, gz,
    kernel, cbar}: kernel 0 Wendland C2, 1 cubic spline; cbar the sound speed of
    Eq. 5's viscosity (0: c0)."""
    if eta2 is None:
        eta2 = 0.01 * h * h
    return np.array([h, mass, rho0, c0, gamma, alpha, eta2, g[0], g[1], g[2], kernel, cbar],
                    dtype=np.float64)


def sph_rates(pos, vel, rho, kind, L, per, R2, prm, rows=None):
    """FP64 SPH rates (Eqs. 1-2) on the FP32 pair set.

    Returns (acc (rows, 3), drho (rows,), mumax (rows,))."""
    pos, vel, rho = _f32(pos), _f32(vel), _f32(rho)
    nr = len(pos) if rows is None else len(rows)
    rows_a = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    acc = np.empty((nr, 3), np.float64)
    drho = np.empty(nr, np.float64)
    mu = np.empty(nr, np.float64)
    lib().oracle_sph_rows(len(pos), pos, vel, rho, _i32(kind), _box(L), _per(per),
                          float(np.float32(R2)), _f64(prm), rows_a, nr, acc, drho, mu)
    return acc, drho, mu


def sph_dt(acc, kind, mumax, prm, cfl):
    """CFL time step from full-system rates: cfl * min(min_a sqrt(h/|a_a|), h/(c0 + max mu))."""
    h, c0 = float(prm[0]), float(prm[3])
    fl = np.asarray(kind) == 0
    am = np.sqrt((np.asarray(acc)[fl] ** 2).sum(axis=1))
    t1 = np.sqrt(h / am[am > 0].max()) if np.any(am > 0) else np.inf
    t2 = h / (c0 + float(np.max(mumax)))
    return cfl * min(t1, t2)


def sph_kdk(pos, vel, rho, kind, L, per, R2, prm, cfl, nsteps):
    """nsteps kick-drift-kick steps on (x, v, rho) with the CFL time step of the
    latest rates (section 4.2 names the dynamic step but not the scheme; this is
    the reading used throughout): with rates (a, D) and dt at step n,
      rho += dt/2 D;  v += dt/2 a (fluid);  x += dt v (fluid);
      rates at the new (x, v, rho);  rho += dt/2 D;  v += dt/2 a (fluid);
      t += dt;  dt = CFL step of the new rates.
    Boundary particles (kind 1) keep x and v; their density evolves.  The state
    is kept in FP64; rates see it rounded to FP32 (the precision the particle
    arrays have).  Returns (x, v, rho, hist (nsteps, 2) = [t, dt])."""
    x = np.asarray(pos, np.float64).copy()
    v = np.asarray(vel, np.float64).copy()
    r = np.asarray(rho, np.float64).copy()
    fl = np.asarray(kind) == 0

    def rates():
        return sph_rates(x.astype(np.float32), v.astype(np.float32), r.astype(np.float32),
                         kind, L, per, R2, prm)

    a, D, mu = rates()
    dt = sph_dt(a, kind, mu, prm, cfl)
    t = 0.0
    hist = np.empty((nsteps, 2), np.float64)
    for k in range(nsteps):
        r += 0.5 * dt * D
        v[fl] += 0.5 * dt * a[fl]
        x[fl] += dt * v[fl]
        a, D, mu = rates()
        r += 0.5 * dt * D
        v[fl] += 0.5 * dt * a[fl]
        t += dt
        hist[k] = (t, dt)
        dt = sph_dt(a, kind, mu, prm, cfl)
    return x, v, r, hist


def verlet_steps(x, v, rho, fluid, rates, dt_of, nsteps, every):
    """The Verlet scheme of section 4.2 (ref. [46]) with a dynamic step, on FP64
    state: at step n with rates (a, D) of the state n and time step dt,
      x^{n+1} = x^n + dt v^n + dt^2/2 a^n                      (fluid only)
      v^{n+1} = v^{n-1} + 2 dt a^n,  rho^{n+1} = rho^{n-1} + 2 dt D^n,
    except on every `every`-th step counted from 0, which takes the Euler form
      v^{n+1} = v^n + dt a^n,  rho^{n+1} = rho^n + dt D^n
    (step 0 has no previous state).  Boundary particles (fluid False) keep x
    and v; their density evolves.  `rates(x, v, rho)` returns (a, D, extra)
    and `dt_of(a, extra)` the step for those rates.  Returns (x, v, rho,
    hist (nsteps, 2) = [t, dt])."""
    x, v, r = (np.asarray(q, np.float64).copy() for q in (x, v, rho))
    fl = np.asarray(fluid, bool)
    vp, rp = v.copy(), r.copy()
    a, D, extra = rates(x, v, r)
    t = 0.0
    hist = np.empty((nsteps, 2), np.float64)
    for n in range(nsteps):
        dt = dt_of(a, extra)
        euler = n % every == 0
        bv, br, f = (v, r, dt) if euler else (vp, rp, 2.0 * dt)
        xn = x.copy()
        xn[fl] = x[fl] + dt * v[fl] + 0.5 * dt * dt * a[fl]
        vn = v.copy()
        vn[fl] = bv[fl] + f * a[fl]
        rn = br + f * D
        vp, rp = v, r
        x, v, r = xn, vn, rn
        a, D, extra = rates(x, v, r)
        t += dt
        hist[n] = (t, dt)
    return x, v, r, hist


def sph_verlet(pos, vel, rho, kind, L, per, R2, prm, cfl, nsteps, every):
    """nsteps of the Verlet scheme (verlet_steps) with SPH rates (Eqs. 1-5) and
    the CFL time step of the current rates.  Rates see the FP64 state rounded
    to FP32 (the precision the particle arrays have)."""
    def rates(x, v, r):
        a, D, mu = sph_rates(x.astype(np.float32), v.astype(np.float32), r.astype(np.float32),
                             kind, L, per, R2, prm)
        return a, D, mu

    return verlet_steps(pos, vel, rho, np.asarray(kind) == 0, rates,
                        lambda a, mu: sph_dt(a, kind, mu, prm, cfl), nsteps, every)


def dem_params_array(R, m, I, kn, kt, gn, gt=0.0, mu=0.5, g=(0.0, 0.0, 0.0), dt=1e-4, walls=0):
    """The oracle's DEM parameter vector {R, m, I, kn, kt, gn, gt, mu, gx, gy, gz, dt, walls}."""
    return np.array([R, m, I, kn, kt, gn, gt, mu, g[0], g[1], g[2], dt, walls], np.float64)


def dem_empty_history(n, C=16):
    return np.full((n, C), -1, np.int64), np.zeros((n, C, 3), np.float64)


def dem_forces(x, v, w, L, per, prm, hist=None, C=16):
    """Forces and torques of the Silbert grain model (Eqs. 9-12) at (x, v, w)
    with contact history `hist` = (ids (n, C), u_t (n, C, 3)); returns
    (F, T, new history, contact counts)."""
    x, v, w = (np.ascontiguousarray(q, np.float64) for q in (x, v, w))
    n = len(x)
    hid, hu = dem_empty_history(n, C) if hist is None else (np.ascontiguousarray(hist[0], np.int64),
                                                           np.ascontiguousarray(hist[1], np.float64))
    F = np.empty((n, 3)); T = np.empty((n, 3))
    hid2, hu2 = dem_empty_history(n, C)
    nc = np.empty(n, np.int32)
    lib().oracle_dem_forces(n, x, v, w, _box(L), _per(per), _f64(prm), int(C), hid, hu, F, T,
                            hid2, hu2, nc)
    return F, T, (hid2, hu2), nc


def dem_forces_rows(x, v, w, L, per, prm, rows):
    """Forces and torques (dem_forces) of the grains `rows` only, against all
    grains, with no contact history; returns (F, T, contact counts)."""
    x, v, w = (np.ascontiguousarray(q, np.float64) for q in (x, v, w))
    rows = np.ascontiguousarray(rows, np.int64)
    F = np.empty((len(rows), 3)); T = np.empty((len(rows), 3))
    nc = np.empty(len(rows), np.int32)
    lib().oracle_dem_forces_rows(len(x), x, v, w, _box(L), _per(per), _f64(prm), rows,
                                 len(rows), F, T, nc)
    return F, T, nc


def dem_steps(x, v, w, L, per, prm, nsteps, hist=None, C=16):
    """nsteps of forces (dem_forces) and the leapfrog of Eq. 13 on FP64 state.
    Returns (x, v, w, history, F, T, contact counts) after the last step."""
    x, v, w = (np.array(q, np.float64) for q in (x, v, w))
    F = T = nc = None
    for _ in range(nsteps):
        F, T, hist, nc = dem_forces(x, v, w, L, per, prm, hist, C)
        lib().oracle_dem_leapfrog(len(x), x, v, w, F, T, _f64(prm))
    return x, v, w, hist, F, T, nc


def num_threads() -> int:
    """OpenMP threads used by the oracle's loops."""
    return int(lib().oracle_num_threads())
