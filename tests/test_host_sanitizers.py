"""The C-ABI library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The library is built a second time with both sanitizers on its host code only
(the device code is unchanged) and loaded in a child process that preloads
the sanitizer runtime.  Without a GPU the child drives every host path that
needs none: the capacity and footprint queries, the error strings, every entry
point's argument checks and the failing context creation; any report ends the
child.  (In a process that uses the GPU the sanitizer runtime's interceptor of
the HSA memory-pool allocation refuses the runtime's first device allocation,
so the device paths are not run this way.)
"""
import glob
import os
import subprocess
import sys

import pytest

from paper_2401_10462_amd import build as lib_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ASAN_RT = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))

SCRIPT = r"""
import ctypes, os, sys
from paper_2401_10462_amd import _lib
_lib.LIB_PATH = os.environ["SASA_SAN_LIB"]
L = _lib.load()
assert list(_lib.sasa_capacity()) == [512, 128]
assert _lib.sasa_footprint(5000) > 0
for code in range(0, -9, -1):
    assert L.sasa_strerror(code)
n = ctypes.c_int64(0)
cnt = (ctypes.c_int64 * 8)()
assert L.sasa_compute(None, 10, None, None, 1.4, None, None, 0, None) == _lib.SASA_E_INVAL
assert L.sasa_compute_batch(None, 1, None, None, None, 1.4, None, None, 0, None) == _lib.SASA_E_INVAL
assert L.sasa_backward(None, None, None, 0, None) == _lib.SASA_E_INVAL
assert L.sasa_triangles_by_sort(None, None, None, 0, ctypes.byref(n), None) == _lib.SASA_E_INVAL
assert L.sasa_edges_vertices_by_sort(None, None, None, 0, None, None, None, 0, None, None) == _lib.SASA_E_INVAL
assert L.sasa_complex_counts(None, cnt) == _lib.SASA_E_INVAL
assert L.sasa_status(None) == _lib.SASA_E_INVAL
assert L.sasa_curvature(None, None, None, 0, None) == _lib.SASA_E_INVAL
assert L.sasa_curvature_backward(None, None, None, 0, None) == _lib.SASA_E_INVAL
h = ctypes.c_void_p()
bad = _lib.sasa_options(0, 0, 0, 1 << 10, 0)
assert L.sasa_create(ctypes.byref(bad), ctypes.byref(h)) == _lib.SASA_E_INVAL and not h.value
opts = _lib.sasa_options(0, 0, 1000, 0, 0)
rc = L.sasa_create(ctypes.byref(opts), ctypes.byref(h))
assert rc != 0 and not h.value, rc  # no GPU in this process
L.sasa_destroy(None)
maps = open("/proc/self/maps").read()
assert "libclang_rt.asan" in maps and os.path.basename(os.environ["SASA_SAN_LIB"]) in maps
print("sanitized host paths ok", flush=True)
"""


@pytest.mark.skipif(not ASAN_RT or not os.path.exists(HIPCC), reason="no hipcc or clang AddressSanitizer runtime")
def test_host_code_clean_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "libsasa_hip_hostsan.so")
    srcs = lib_build.SOURCES
    # sanitizers on the host compilation only
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-mcode-object-version=5",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
           *srcs, "-o", lib]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    env = dict(os.environ, LD_PRELOAD=ASAN_RT[-1], SASA_SAN_LIB=lib, PYTHONPATH=ROOT,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("HIP_VISIBLE_DEVICES", None)
    res = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=600)
    report = res.stdout[-3000:] + res.stderr[-6000:]
    assert res.returncode == 0, report
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, report
    assert "sanitized host paths ok" in res.stdout
