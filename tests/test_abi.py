"""The C-ABI library loads on the host and exports every entry point that
include/*.h declares (no device work is started here)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(fpm_\w+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ["fpm_create", "fpm_destroy", "fpm_set_box", "fpm_set_neighbor_params",
                     "fpm_set_particles", "fpm_build_cell_list", "fpm_build_verlet",
                     "fpm_lj_forces", "fpm_integrate", "fpm_step"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1804_07598_amd import _lib
    L = _lib.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_debug_build_exports_the_same_symbols():
    path = os.path.join(ROOT, "paper_1804_07598_amd", "libfpm_checked.so")
    L = ctypes.CDLL(path)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_1804_07598_amd import _lib
    bound = set(_lib._SIGS) | {"fpm_last_error"}
    assert set(declared_functions()) <= bound


def test_host_side_errors_without_device():
    """Argument checks that return before any HIP call."""
    from paper_1804_07598_amd import _lib as F
    L = F.lib()
    ctx = ctypes.c_void_p()
    assert L.fpm_create(ctypes.byref(ctx), None) == 0
    try:
        bad = (ctypes.c_float * 3)(10.0, -1.0, 10.0)
        per = (ctypes.c_int32 * 3)(1, 1, 1)
        assert L.fpm_set_box(ctx, bad, per) == F.FPM_EINVAL
        good = (ctypes.c_float * 3)(10.0, 10.0, 10.0)
        assert L.fpm_set_box(ctx, good, per) == 0
        # r_cut + skin must stay below L/2 on periodic axes
        assert L.fpm_set_neighbor_params(ctx, 4.9, 0.3, 128) == F.FPM_ECUTOFF
        assert b"half" in L.fpm_last_error(ctx)
        assert L.fpm_set_neighbor_params(ctx, 2.5, 0.3, 0) == F.FPM_EINVAL
        assert L.fpm_set_neighbor_params(ctx, 2.5, 0.3, 128) == 0
        sz = ctypes.c_size_t()
        assert L.fpm_workspace_size(ctx, 1000, ctypes.byref(sz)) == 0
        assert sz.value > 1000 * 128 * 4
        assert L.fpm_workspace_size(ctx, 0, ctypes.byref(sz)) == F.FPM_EINVAL
        # calls that need particles fail cleanly
        assert L.fpm_build_verlet(ctx) == F.FPM_EINVAL
        assert L.fpm_step(ctx, None, ctypes.c_float(0.005), 1, None) == F.FPM_EINVAL
        lj = F.lj_params((1.0,) * 3, (1.0,) * 3, 1)
        assert L.fpm_step_record(ctx, ctypes.byref(lj), ctypes.c_float(0.005), 1,
                                 None) == F.FPM_EINVAL
        assert L.fpm_lj_adjoint_sweep(ctx, ctypes.byref(lj), ctypes.c_float(0.005), 1, None,
                                      None, None, None, None, None) == F.FPM_EINVAL
        # size limits: n at most 2^26 - 1, list capacity at most 4096
        assert L.fpm_workspace_size(ctx, 1 << 26, ctypes.byref(sz)) == F.FPM_EINVAL
        assert L.fpm_workspace_size(ctx, (1 << 26) - 1, ctypes.byref(sz)) == 0
        assert L.fpm_set_neighbor_params(ctx, 2.5, 0.3, 4097) == F.FPM_EINVAL
        # launch-shape knobs outside their ranges
        assert L.fpm_set_tuning(ctx, 6, 0, 0) == F.FPM_EINVAL
        assert L.fpm_set_tuning(ctx, 5, 0, 0) == 0
        assert L.fpm_set_tuning(ctx, 4, 5, 0) == F.FPM_EINVAL
        assert L.fpm_set_tuning(ctx, 2, 65, 0) == F.FPM_EINVAL
        assert L.fpm_set_tuning(ctx, 0, 0, 6) == F.FPM_EINVAL
        assert L.fpm_set_tuning(ctx, 4, 16, 4) == 0
        # DEM: capacity range, and the DEM calls need DEM storage and particles
        assert L.fpm_set_dem(ctx, 0) == F.FPM_EINVAL
        assert L.fpm_set_dem(ctx, 65) == F.FPM_EINVAL
        prm = F.dem_params(0.06, 1.0, 1.44e-3, 7.849, 2.243, 3.401)
        assert L.fpm_dem_forces(ctx, ctypes.byref(prm)) == F.FPM_EINVAL
        base = ctypes.c_size_t()
        assert L.fpm_workspace_size(ctx, 1000, ctypes.byref(base)) == 0
        assert L.fpm_set_dem(ctx, 16) == 0
        dem_size = ctypes.c_size_t()
        assert L.fpm_workspace_size(ctx, 1000, ctypes.byref(dem_size)) == 0
        # the history: 16 B per list slot (capacity 128) plus 20 B per contact
        # slot (16 per grain)
        assert dem_size.value >= base.value + 1000 * (128 * 16 + 16 * 20)
        assert L.fpm_dem_step(ctx, ctypes.byref(prm), 1) == F.FPM_EINVAL
    finally:
        L.fpm_destroy(ctx)
