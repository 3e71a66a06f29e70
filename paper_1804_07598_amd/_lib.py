"""ctypes binding of libfpm.so (include/fpm.h).  Argument marshalling only.

Every function here has the name of the C entry point it calls and raises
FpmError on a non-zero return code.  Device pointers are passed as integers
(torch.Tensor.data_ptr()).  There is no fallback: if the library is not built,
loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfpm.so")

FPM_OK = 0
FPM_EINVAL = -1
FPM_EHIP = -2
FPM_ECUTOFF = -3
FPM_EOVERFLOW = -4
FPM_ENOWS = -5
FPM_ENONFINITE = -6
FPM_EBADINDEX = -7
_NAMES = {FPM_EINVAL: "FPM_EINVAL", FPM_EHIP: "FPM_EHIP", FPM_ECUTOFF: "FPM_ECUTOFF",
          FPM_EOVERFLOW: "FPM_EOVERFLOW", FPM_ENOWS: "FPM_ENOWS",
          FPM_ENONFINITE: "FPM_ENONFINITE", FPM_EBADINDEX: "FPM_EBADINDEX"}


class FpmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class fpm_lj_params(C.Structure):
    _fields_ = [("n_types", C.c_int32), ("eps", C.c_float * 3), ("sig", C.c_float * 3)]


class fpm_sph_params(C.Structure):
    _fields_ = [("h", C.c_float), ("mass", C.c_float), ("rho0", C.c_float), ("c0", C.c_float),
                ("gamma", C.c_float), ("alpha", C.c_float), ("eta2", C.c_float),
                ("g", C.c_float * 3), ("cfl", C.c_float), ("kernel", C.c_int32),
                ("cbar", C.c_float), ("scheme", C.c_int32), ("verlet_every", C.c_int32)]


class fpm_dem_params(C.Structure):
    _fields_ = [("R", C.c_float), ("mass", C.c_float), ("inertia", C.c_float),
                ("kn", C.c_float), ("kt", C.c_float), ("gn", C.c_float), ("gt", C.c_float),
                ("mu", C.c_float), ("g", C.c_float * 3), ("dt", C.c_float), ("walls", C.c_int32)]


_P = C.c_void_p
_SIGS = {
    "fpm_create": [C.POINTER(_P), _P],
    "fpm_destroy": [_P],
    "fpm_set_box": [_P, C.POINTER(C.c_float), C.POINTER(C.c_int32)],
    "fpm_set_systems": [_P, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_int32),
                        C.POINTER(C.c_int64)],
    "fpm_set_tuning": [_P, C.c_int32, C.c_int32, C.c_int32],
    "fpm_set_neighbor_params": [_P, C.c_float, C.c_float, C.c_int32],
    "fpm_workspace_size": [_P, C.c_int64, C.POINTER(C.c_size_t)],
    "fpm_set_workspace": [_P, _P, C.c_size_t],
    "fpm_set_particles": [_P, C.c_int64, _P, _P, _P],
    "fpm_set_positions": [_P, _P],
    "fpm_system_info": [_P, C.c_int32, C.POINTER(C.c_int64)],
    "fpm_set_density": [_P, _P],
    "fpm_get_particles": [_P, _P, _P, _P],
    "fpm_get_sph": [_P, _P, _P],
    "fpm_build_cell_list": [_P],
    "fpm_get_cell_list": [_P, C.POINTER(C.c_int32), _P, _P],
    "fpm_build_verlet": [_P],
    "fpm_get_neighbors": [_P, _P, _P],
    "fpm_lj_forces": [_P, C.POINTER(fpm_lj_params), _P],
    "fpm_lj_forces_static": [_P, C.POINTER(fpm_lj_params), C.c_int64, _P, _P, _P, _P],
    "fpm_lj_force_vjp": [_P, C.POINTER(fpm_lj_params), _P, _P, _P],
    "fpm_lj_adjoint_step": [_P, C.POINTER(fpm_lj_params), C.c_float, _P, _P, _P, _P, _P,
                            C.c_int32],
    "fpm_lj_adjoint_sweep": [_P, C.POINTER(fpm_lj_params), C.c_float, C.c_int32, _P, _P, _P,
                             _P, _P, _P],
    "fpm_step_record": [_P, C.POINTER(fpm_lj_params), C.c_float, C.c_int32, _P],
    "fpm_integrate": [_P, C.c_float, C.c_int32],
    "fpm_step": [_P, C.POINTER(fpm_lj_params), C.c_float, C.c_int32, _P],
    "fpm_sph_rates": [_P, C.POINTER(fpm_sph_params), _P],
    "fpm_sph_step": [_P, C.POINTER(fpm_sph_params), C.c_int32, _P],
    "fpm_set_dem": [_P, C.c_int32],
    "fpm_set_symmetric": [_P, C.c_int32],
    "fpm_set_omega": [_P, _P],
    "fpm_dem_forces": [_P, C.POINTER(fpm_dem_params)],
    "fpm_dem_step": [_P, C.POINTER(fpm_dem_params), C.c_int32],
    "fpm_get_dem": [_P, _P, _P, _P],
    "fpm_get_contacts": [_P, _P, _P],
    "fpm_check": [_P],
    "fpm_read_counters": [_P, C.POINTER(C.c_int64)],
    "fpm_set_profiling": [_P, C.c_int32],
    "fpm_kernel_time": [_P, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)],
}

_lib = None


def lib() -> C.CDLL:
    """Load libfpm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run "
                              "python paper_1804_07598_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            if not hasattr(L, name):
                continue
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.fpm_last_error.argtypes = [_P]
        L.fpm_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def exported_symbols(L=None):
    L = L or lib()
    return [n for n in list(_SIGS) + ["fpm_last_error"] if hasattr(L, n)]


def _call(name: str, ctx, *args) -> int:
    L = lib()
    rc = getattr(L, name)(ctx, *args)
    if rc != FPM_OK:
        msg = L.fpm_last_error(ctx).decode() if ctx else "null context"
        raise FpmError(rc, f"{name}: {msg}")
    return rc


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def fpm_create(stream: int = 0):
    ctx = _P()
    rc = lib().fpm_create(C.byref(ctx), _P(stream) if stream else None)
    if rc != FPM_OK:
        raise FpmError(rc, "fpm_create")
    return ctx


def fpm_destroy(ctx):
    lib().fpm_destroy(ctx)


def fpm_last_error(ctx) -> str:
    return lib().fpm_last_error(ctx).decode()


def fpm_set_box(ctx, L, periodic):
    Lc = (C.c_float * 3)(*[float(x) for x in L])
    pc = (C.c_int32 * 3)(*[int(x) for x in periodic])
    _call("fpm_set_box", ctx, Lc, pc)


def fpm_set_systems(ctx, L, periodic, counts):
    """L, periodic: (nsys, 3); counts: (nsys,) particles per system."""
    nsys = len(counts)
    Lc = (C.c_float * (3 * nsys))(*[float(x) for row in L for x in row])
    pc = (C.c_int32 * (3 * nsys))(*[int(x) for row in periodic for x in row])
    cc = (C.c_int64 * nsys)(*[int(x) for x in counts])
    _call("fpm_set_systems", ctx, int(nsys), Lc, pc, cc)


def fpm_set_tuning(ctx, verlet_path: int = 0, zblock: int = 0, unroll: int = 0):
    _call("fpm_set_tuning", ctx, int(verlet_path), int(zblock), int(unroll))


def fpm_set_neighbor_params(ctx, r_cut: float, skin: float, max_nbr: int):
    _call("fpm_set_neighbor_params", ctx, float(r_cut), float(skin), int(max_nbr))


def fpm_workspace_size(ctx, n: int) -> int:
    out = C.c_size_t(0)
    _call("fpm_workspace_size", ctx, int(n), C.byref(out))
    return int(out.value)


def fpm_set_workspace(ctx, ws):
    _call("fpm_set_workspace", ctx, _ptr(ws), ws.numel() * ws.element_size())


def fpm_set_particles(ctx, pos, vel=None, typ=None):
    _call("fpm_set_particles", ctx, int(pos.shape[0]), _ptr(pos), _ptr(vel), _ptr(typ))


def fpm_set_positions(ctx, pos):
    _call("fpm_set_positions", ctx, _ptr(pos))


def fpm_system_info(ctx, s: int):
    out = (C.c_int64 * 8)()
    _call("fpm_system_info", ctx, int(s), out)
    return tuple(int(x) for x in out)


def fpm_set_density(ctx, rho):
    _call("fpm_set_density", ctx, _ptr(rho))


def fpm_get_particles(ctx, pos=None, vel=None, frc=None):
    _call("fpm_get_particles", ctx, _ptr(pos), _ptr(vel), _ptr(frc))


def fpm_get_sph(ctx, rho=None, drho=None):
    _call("fpm_get_sph", ctx, _ptr(rho), _ptr(drho))


def fpm_build_cell_list(ctx):
    _call("fpm_build_cell_list", ctx)


def fpm_get_cell_list(ctx, offsets=None, order=None):
    nc = (C.c_int32 * 3)()
    _call("fpm_get_cell_list", ctx, nc, _ptr(offsets), _ptr(order))
    return tuple(nc)


def fpm_build_verlet(ctx):
    _call("fpm_build_verlet", ctx)


def fpm_get_neighbors(ctx, counts, cols):
    _call("fpm_get_neighbors", ctx, _ptr(counts), _ptr(cols))


def lj_params(eps=(1.0, 1.0, 1.0), sig=(1.0, 1.0, 1.0), n_types: int = 1) -> fpm_lj_params:
    p = fpm_lj_params()
    p.n_types = int(n_types)
    for k in range(3):
        p.eps[k] = float(eps[k])
        p.sig[k] = float(sig[k])
    return p


def sph_params(h, mass, rho0, c0, gamma=7.0, alpha=0.1, eta2=None, g=(0.0, 0.0, -9.81),
               cfl=0.2, *, kernel=0, cbar=0.0, scheme=0, verlet_every=40) -> fpm_sph_params:
    p = fpm_sph_params()
    p.kernel, p.cbar, p.scheme, p.verlet_every = int(kernel), float(cbar), int(scheme), \
        int(verlet_every)
    p.h, p.mass, p.rho0, p.c0, p.gamma, p.alpha = (float(h), float(mass), float(rho0),
                                                    float(c0), float(gamma), float(alpha))
    p.eta2 = float(0.01 * h * h if eta2 is None else eta2)
    for k in range(3):
        p.g[k] = float(g[k])
    p.cfl = float(cfl)
    return p


def dem_params(R, mass, inertia, kn, kt, gn, gt=0.0, mu=0.5, g=(0.0, 0.0, 0.0), dt=1e-4,
               walls=0) -> fpm_dem_params:
    p = fpm_dem_params()
    p.R, p.mass, p.inertia, p.kn, p.kt, p.gn, p.gt, p.mu = (float(x) for x in
                                                          (R, mass, inertia, kn, kt, gn, gt, mu))
    for k in range(3):
        p.g[k] = float(g[k])
    p.dt, p.walls = float(dt), int(walls)
    return p


def fpm_set_symmetric(ctx, on: bool):
    _call("fpm_set_symmetric", ctx, 1 if on else 0)


def fpm_set_dem(ctx, max_contacts: int):
    _call("fpm_set_dem", ctx, int(max_contacts))


def fpm_set_omega(ctx, omega=None):
    _call("fpm_set_omega", ctx, _ptr(omega))


def fpm_dem_forces(ctx, prm: fpm_dem_params):
    _call("fpm_dem_forces", ctx, C.byref(prm))


def fpm_dem_step(ctx, prm: fpm_dem_params, nsteps: int):
    _call("fpm_dem_step", ctx, C.byref(prm), int(nsteps))


def fpm_get_dem(ctx, omega=None, torque=None, ncontact=None):
    _call("fpm_get_dem", ctx, _ptr(omega), _ptr(torque), _ptr(ncontact))


def fpm_get_contacts(ctx, ids=None, ut=None):
    _call("fpm_get_contacts", ctx, _ptr(ids), _ptr(ut))


def fpm_lj_forces(ctx, prm: fpm_lj_params, out=None):
    _call("fpm_lj_forces", ctx, C.byref(prm), _ptr(out))


def fpm_lj_forces_static(ctx, prm: fpm_lj_params, pos, frc, typ=None, out=None):
    _call("fpm_lj_forces_static", ctx, C.byref(prm), int(pos.shape[0]), _ptr(pos), _ptr(typ),
          _ptr(frc), _ptr(out))


def fpm_lj_force_vjp(ctx, prm: fpm_lj_params, lam, gx, gtheta=None):
    _call("fpm_lj_force_vjp", ctx, C.byref(prm), _ptr(lam), _ptr(gx), _ptr(gtheta))


def fpm_lj_adjoint_step(ctx, prm: fpm_lj_params, dt: float, floss, xbar, vbar, fbar,
                        gtheta=None, last: int = 0):
    _call("fpm_lj_adjoint_step", ctx, C.byref(prm), float(dt), _ptr(floss), _ptr(xbar),
          _ptr(vbar), _ptr(fbar), _ptr(gtheta), int(last))


def fpm_lj_adjoint_sweep(ctx, prm: fpm_lj_params, dt: float, nsteps: int, xs, floss, xbar,
                         vbar, fbar, gtheta=None):
    """floss: a sequence of nsteps device tensors or None (per step)."""
    tab = (C.c_void_p * max(int(nsteps), 1))(*[_ptr(f) for f in floss])
    _call("fpm_lj_adjoint_sweep", ctx, C.byref(prm), float(dt), int(nsteps), _ptr(xs), tab,
          _ptr(xbar), _ptr(vbar), _ptr(fbar), _ptr(gtheta))


def fpm_step_record(ctx, prm: fpm_lj_params, dt: float, nsteps: int, xs):
    _call("fpm_step_record", ctx, C.byref(prm), float(dt), int(nsteps), _ptr(xs))


def fpm_integrate(ctx, dt: float, half: int):
    _call("fpm_integrate", ctx, float(dt), int(half))


def fpm_step(ctx, prm: fpm_lj_params, dt: float, nsteps: int, thermo=None):
    _call("fpm_step", ctx, C.byref(prm), float(dt), int(nsteps), _ptr(thermo))


def fpm_sph_rates(ctx, prm: fpm_sph_params, dt_out=None):
    _call("fpm_sph_rates", ctx, C.byref(prm), _ptr(dt_out))


def fpm_sph_step(ctx, prm: fpm_sph_params, nsteps: int, hist=None):
    _call("fpm_sph_step", ctx, C.byref(prm), int(nsteps), _ptr(hist))


def fpm_check(ctx):
    _call("fpm_check", ctx)


def fpm_read_counters(ctx):
    out = (C.c_int64 * 3)()
    _call("fpm_read_counters", ctx, out)
    return tuple(int(x) for x in out)


def fpm_set_profiling(ctx, on: bool):
    _call("fpm_set_profiling", ctx, 1 if on else 0)


def fpm_kernel_time(ctx, kernel: str):
    """(mean ms, count) of the event-timed launches of `kernel` (records consumed)."""
    ms = C.c_double(0)
    n = C.c_int64(0)
    _call("fpm_kernel_time", ctx, kernel.encode(), C.byref(ms), C.byref(n))
    return float(ms.value), int(n.value)
