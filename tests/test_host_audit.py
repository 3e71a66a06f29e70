"""Host-side audit of the C ABI's workspace layout under AddressSanitizer and
UndefinedBehaviorSanitizer (host pass only; no GPU needed): tests/host/
plan_audit.cpp compiles in the library's api.hip and checks, for the 1M-atom
LJ liquid, the 688,380-grain DEM avalanche (16 and 64 contact slots), a batch
and the SPH column, that every array the kernels index lies inside the
workspace without overlap and holds its kernels' extent."""
import concurrent.futures as cf
import glob
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "host_audit")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         "-Xarch_host", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include")]


def _compile(src):
    obj = os.path.join(OUT, os.path.basename(src) + ".o")
    r = subprocess.run([HIPCC, *FLAGS, "-c", src, "-o", obj], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return obj


def test_workspace_layout_audit_under_sanitizers():
    os.makedirs(OUT, exist_ok=True)
    csrc = os.path.join(ROOT, "paper_1804_07598_amd", "csrc")
    srcs = [os.path.join(ROOT, "tests", "host", "plan_audit.cpp")]
    srcs += [p for p in sorted(glob.glob(os.path.join(csrc, "*.hip")))
             if os.path.basename(p) != "api.hip"]  # api.hip is compiled into the audit
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, srcs))
    exe = os.path.join(OUT, "plan_audit")
    r = subprocess.run([HIPCC, *FLAGS, *objs, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    for cfg in ("lj1m", "dem688k", "dem688k-C64", "batch64", "sph2m"):
        assert f"ok [{cfg}]" in r.stderr, r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
