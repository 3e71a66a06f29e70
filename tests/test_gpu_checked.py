"""The library's debug build (libfpm_checked.so) on the paths the parity tests
cover: LJ forces and steps under every Verlet build, the two-type mixture with
the force VJP, symmetric half lists, a batch, SPH and DEM.  Every rebuild's
cell list and Verlet lists are validated on the device and every list entry
the LJ kernels read is range-checked; fpm_check must report nothing.  The
cases run in a process of their own (tests/checked_cases.py), which loads the
debug build in place of libfpm.so."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_debug_build_finds_no_bad_index():
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "checked_cases.py")],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    print(r.stdout[-3000:])
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-3000:])
    assert "all cases ok" in r.stdout
