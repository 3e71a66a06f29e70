"""MI355X-native particle hot path of OpenFPM (arXiv 1804.07598).

Hand-written HIP kernels for gfx950 behind the C ABI in include/fpm.h:
cell lists, Verlet lists, Lennard-Jones forces/energy/virial, weakly
compressible SPH sums and velocity-Verlet stepping.  Importing the package does
not load the library; `lib()` or the simulation classes do, and fail loudly if
libfpm.so has not been built.
"""
from ._lib import FpmError, lib  # noqa: F401

__all__ = ["FpmError", "lib"]
