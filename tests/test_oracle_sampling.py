"""The oracle's areas against fine-grid sphere-point sampling on tiny inputs.

Each sphere carries a Fibonacci lattice of points (near-uniform, the lattice
the point-counting methods of the Introduction use); a point is exposed when
it lies outside every other ball.  The exposed fraction times 4 pi R^2 tends
to A_i as the lattice grows; with 400,000 points per sphere the error is a
few 1e-5 of the sphere's area (tested at 2e-4), so this is a loose pin, independent of every
formula the oracle uses.
"""
import math

import numpy as np
import pytest

import oracle
from synth.globule import random_cluster


def fibonacci_sphere(n):
    k = np.arange(n) + 0.5
    z = 1.0 - 2.0 * k / n
    r = np.sqrt(1.0 - z * z)
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def sampled_areas(xyz, R, n_points=400_000):
    unit = fibonacci_sphere(n_points)
    out = np.zeros(len(R))
    for i in range(len(R)):
        pts = xyz[i] + R[i] * unit
        exposed = np.ones(n_points, dtype=bool)
        for j in range(len(R)):
            if j != i and np.linalg.norm(xyz[j] - xyz[i]) < R[i] + R[j]:
                exposed &= ((pts - xyz[j]) ** 2).sum(1) >= R[j] ** 2
        out[i] = exposed.mean() * 4.0 * math.pi * R[i] ** 2
    return out


@pytest.mark.parametrize("n,seed,rmin,rmax", [(3, 1, 1.2, 1.8), (5, 2, 1.0, 2.0), (8, 3, 1.5, 1.8)])
def test_areas_against_point_sampling(n, seed, rmin, rmax):
    xyz, rad = random_cluster(n, seed, rmin=rmin, rmax=rmax)
    R = rad + 1.4
    ref = oracle.run(xyz, rad, 1.4)
    s = sampled_areas(xyz, R)
    err = np.abs(ref.area - s) / (4.0 * math.pi * R ** 2)
    assert err.max() < 2e-4, err
    assert abs(ref.area.sum() - s.sum()) / s.sum() < 2e-4
