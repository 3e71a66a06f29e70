"""Compile the HIP library libfpm.so for gfx950 in-tree, and its debug build
libfpm_checked.so (FPM_CHECKED=1: cell and Verlet lists validated after every
rebuild, list entries range-checked where the LJ kernels read them).

Every .hip file under csrc/ is compiled separately (in parallel) with hipcc and
linked into the library.  Packed FP32 instructions are disabled for all device
code.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfpm.so")
OBJ_CHECKED = os.path.join(HERE, "_build", "checked")
LIB_CHECKED = os.path.join(HERE, "libfpm_checked.so")
ARCH = os.environ.get("FPM_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I", os.path.join(HERE, "..", "include"),
]


def _compile(src: str, verbose: bool, checked: bool = False) -> str:
    obj = os.path.join(OBJ_CHECKED if checked else OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *(["-DFPM_CHECKED=1"] if checked else []), "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = (r.stdout + r.stderr)
    # the host pass does not know the packed-fp32 feature; that warning is expected
    out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{out}")
    if out and verbose:
        print(out, flush=True)
    return obj


def build(verbose: bool = False) -> str:
    """Both libraries; returns the path of libfpm.so."""
    os.makedirs(OBJ_CHECKED, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = [(src, checked) for checked in (False, True) for src in srcs]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        objs = list(ex.map(lambda j: _compile(j[0], verbose, j[1]), jobs))
    for lib, part in ((LIB, objs[:len(srcs)]), (LIB_CHECKED, objs[len(srcs):])):
        tmp = lib + ".tmp"
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *part]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
