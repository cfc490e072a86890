"""The benchmark's secondary workloads run end to end at small sizes (the measurements themselves are not checked).

Each workload function of bench.py is called in this process with a reduced configuration, so that a mistake in
the benchmark's own code (not the library's) shows up in the test run rather than in a measurement.
"""
import argparse

import pytest

pytestmark = pytest.mark.gpu


def _args(**kw):
    base = dict(gpus=1, steps=3, warmup=1, precision="mixed", heavy=150, seed=2, batch=0, cpu_seconds=0.0,
                workload="globule", serve_requests=20, rates="200", md_atoms=600, frames=4, calibrate_copy=0)
    base.update(kw)
    return argparse.Namespace(**base)


def test_local_moves():
    import bench
    print("bench local moves, 600 atoms, 4 frames", flush=True)
    r = bench.local_moves(_args(), "mixed")
    assert r["last_frame_equal"]
    assert r["cold"]["frames_per_s"] > 0 and r["incremental"]["frames_per_s"] > 0
    assert 0.0 <= r["incremental"]["stars_kept"] <= 1.0


def test_md():
    import bench
    print("bench md, 600 atoms, 4 frames", flush=True)
    r = bench.md(_args(), "mixed")
    assert r["cold"]["frames_per_s"] > 0 and r["hinted"]["frames_per_s"] > 0


def test_small_and_gbsa():
    import bench
    print("bench small (300 heavy atoms) and gbsa (150 + 150 atoms, 10 steps)", flush=True)
    assert bench.small(_args())["atoms_per_s"] > 0
    r = bench.gbsa(_args(), "mixed")
    assert r["steps_per_s"] > 0 and r["nonpolar_kcal_mol"] > 0

