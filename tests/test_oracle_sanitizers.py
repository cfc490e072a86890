"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle's sources are built a second time with both sanitizers (every
report fatal) and driven, in a child process that preloads the sanitizer
runtime, through general-position clusters, a small globule, the degenerate
inputs (ties decided by exact arithmetic and the symbolic perturbation,
tangencies, coincident centres), the volume oracle and the VJPs: any
out-of-bounds access, use after free or undefined operation ends the child
with a report.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np
import oracle
from synth.globule import heavy_chain, random_cluster
from synth.degenerate import (CASES, coincident_equal, coincident_smaller, regular_tetrahedron, tangent_pair,
                              tangent_triple)

runs = 0
for seed in range(3):
    xyz, rad = random_cluster(25, seed)
    r = oracle.run(xyz, rad, 1.4)
    r.vjp(np.linspace(-1.0, 1.0, len(rad)))
    oracle.volume(xyz, rad, 1.4)
    runs += 1
xyz, rad = heavy_chain(120, 3)[:2]
r = oracle.run(xyz, rad, 1.4)
assert np.all(np.isfinite(r.area)) and np.all(np.isfinite(r.dadx))
runs += 1
inputs = [c[1] for c in CASES] + [tangent_pair(), tangent_triple(), coincident_smaller(), regular_tetrahedron(1e-3)]
for xyz, rad in inputs:
    probe = 1.5 if len(rad) in (2, 3) and rad[0] == 1.5 else 1.4
    r = oracle.run(xyz, rad, probe)
    assert np.all(np.isfinite(r.area))
    runs += 1
try:
    oracle.run(*coincident_equal(), 1.4)
except Exception:
    pass  # (two equal balls on one centre are refused)
runs += 1
maps = open("/proc/self/maps").read()
assert "libasan" in maps and "libsasa_oracle_san" in maps, "the sanitized build is not the one loaded"
print("sanitized oracle runs:", runs, flush=True)
"""


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="no gcc AddressSanitizer runtime")
def test_oracle_clean_under_asan_ubsan():
    sys.path.insert(0, ROOT)
    from oracle import build
    lib = build.build_sanitized()
    env = dict(os.environ, LD_PRELOAD=_runtime("libasan.so"), SASA_ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               PYTHONPATH=ROOT)
    res = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    report = res.stdout[-3000:] + res.stderr[-6000:]
    assert res.returncode == 0, report
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, report
    assert "sanitized oracle runs:" in res.stdout
