"""Oracle per-atom areas versus the independent latitude-slice integral."""
import numpy as np
import pytest

import oracle
from synth.globule import heavy_chain, random_cluster
from tests.pins.slice_area import exposed_area, exposed_areas


@pytest.mark.parametrize("n,seed,rmin,rmax", [(8, 1, 1.2, 1.8), (12, 2, 1.5, 1.8), (25, 3, 1.2, 1.8),
                                              (40, 4, 1.0, 2.0), (18, 5, 0.5, 2.5)])
def test_random_clusters(n, seed, rmin, rmax):
    xyz, rad = random_cluster(n, seed, rmin=rmin, rmax=rmax)
    r = oracle.run(xyz, rad, 1.4)
    s = exposed_areas(xyz, rad, 1.4)
    assert np.abs(r.area - s).max() < 1e-9


def test_globule_sample():
    xyz, rad, _ = heavy_chain(300, 1)
    r = oracle.run(xyz, rad, 1.4)
    R = rad + 1.4
    idx = np.random.default_rng(3).choice(len(rad), 30, replace=False)
    s = np.array([exposed_area(i, xyz, R) for i in idx])
    assert np.abs(r.area[idx] - s).max() < 1e-9


def test_hydrogen_like_mix_with_hidden_atoms():
    # small balls close to big ones: some are hidden (not in K, zero area)
    rng = np.random.default_rng(11)
    heavy = rng.uniform(0, 6, size=(10, 3))
    hyd = heavy[rng.integers(0, 10, 10)] + rng.normal(size=(10, 3)) * 0.35
    xyz = np.vstack([heavy, hyd])
    rad = np.concatenate([np.full(10, 1.7), np.full(10, 0.4)])
    r = oracle.run(xyz, rad, 1.4)
    s = exposed_areas(xyz, rad, 1.4)
    assert np.abs(r.area - s).max() < 1e-9
    assert (r.vert_in == 0).sum() >= 1
