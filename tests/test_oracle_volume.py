"""The oracle's per-atom volumes and molecular-volume gradient, pinned.

Closed forms (one ball; two balls: the ball minus the cap beyond the radical
plane), the direct chord integral of each cell (tests/pins/volume_grid.py),
the symmetry of the flat faces, central finite differences of the summed
volume, translation / rotation / scaling invariance, and 0 <= V_i <= 4/3 pi R^3.
"""
import math

import numpy as np
import pytest

import oracle
from synth.globule import globule, random_cluster
from tests.pins.volume_grid import cell_volume


def test_one_ball():
    v, g = oracle.volume(np.zeros((1, 3)), np.array([1.7]), 1.4)
    assert abs(v[0] - 4.0 / 3.0 * math.pi * 3.1 ** 3) < 1e-12
    assert np.abs(g).max() == 0.0


@pytest.mark.parametrize("d", [0.3, 1.0, 2.5, 4.0, 5.5])
def test_two_balls_closed_form(d):
    R1, R2 = 3.0, 2.6
    x = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
    v, g = oracle.volume(x, np.array([R1, R2]) - 1.4, 1.4)
    h = (d * d + R1 * R1 - R2 * R2) / (2.0 * d)    # radical plane from centre 1

    def cap(R, hh):                                 # ball beyond a plane at distance hh from its centre
        H = R - hh
        H = min(max(H, 0.0), 2.0 * R)
        return math.pi * H * H * (3.0 * R - H) / 3.0

    ref1 = 4.0 / 3.0 * math.pi * R1 ** 3 - cap(R1, h)
    ref2 = 4.0 / 3.0 * math.pi * R2 ** 3 - cap(R2, d - h)
    assert abs(v[0] - ref1) < 1e-10 and abs(v[1] - ref2) < 1e-10
    # d(V1 + V2)/dd = area of the shared disk
    disk = math.pi * max(R1 * R1 - h * h, 0.0)
    assert abs(g[1, 0] - disk) < 1e-10 and abs(g[0, 0] + disk) < 1e-10


@pytest.mark.parametrize("n,seed,rmin,rmax", [(6, 1, 1.2, 1.8), (10, 2, 1.0, 2.0), (14, 3, 0.6, 2.4)])
def test_cells_against_direct_integral(n, seed, rmin, rmax):
    xyz, rad = random_cluster(n, seed, rmin=rmin, rmax=rmax)
    v, _ = oracle.volume(xyz, rad, 1.4)
    R = rad + 1.4
    direct = np.array([cell_volume(i, xyz, R) for i in range(n)])
    scale = 4.0 / 3.0 * math.pi * R ** 3
    assert (np.abs(v - direct) / scale).max() < 2e-6


def test_faces_are_symmetric():
    xyz, rad = random_cluster(12, 7, rmin=1.0, rmax=2.0)
    for i in range(12):
        for j in range(i + 1, 12):
            a, b = oracle.facet_area(xyz, rad, 1.4, i, j), oracle.facet_area(xyz, rad, 1.4, j, i)
            assert abs(a - b) <= 1e-10 * max(1.0, a)


def test_gradient_finite_differences():
    xyz, rad = globule(20, 4, hydrogens=True)
    _, g = oracle.volume(xyz, rad, 1.4)
    h = 1e-5
    rng = np.random.default_rng(2)
    for m in rng.choice(len(rad), 8, replace=False):
        for c in range(3):
            xp, xm = xyz.copy(), xyz.copy()
            xp[m, c] += h
            xm[m, c] -= h
            fd = (oracle.volume(xp, rad, 1.4)[0].sum() - oracle.volume(xm, rad, 1.4)[0].sum()) / (2 * h)
            assert abs(fd - g[m, c]) < 1e-5 * max(1.0, abs(g[m, c])), (m, c, fd, g[m, c])


def test_invariants():
    xyz, rad = globule(40, 6, hydrogens=True)
    v, g = oracle.volume(xyz, rad, 1.4)
    R = rad + 1.4
    assert (v >= -1e-9).all() and (v <= 4.0 / 3.0 * math.pi * R ** 3 + 1e-9).all()
    assert np.abs(g.sum(0)).max() < 1e-9                       # translation
    assert np.abs(np.cross(xyz, g).sum(0)).max() < 1e-8        # rotation
    q, _ = np.linalg.qr(np.random.default_rng(1).normal(size=(3, 3)))
    v2, g2 = oracle.volume(xyz @ q.T + 3.0, rad, 1.4)
    assert np.abs(v2 - v).max() < 1e-9 and np.abs(g2 - g @ q.T).max() < 1e-9
    v3, g3 = oracle.volume(2.0 * xyz, 2.0 * rad, 2.8)           # scaling by s = 2
    assert np.abs(v3 - 8.0 * v).max() < 1e-8 and np.abs(g3 - 4.0 * g).max() < 1e-8


def test_face_centroids():
    # a face that is a whole disk has its centre as centroid; a face is one set
    # of points, so (i, j) and (j, i) give the same centroid
    x = np.array([[0.0, 0.0, 0.0], [2.5, 0.0, 0.0]])
    f, c = oracle.facet_centroid(x, np.array([1.6, 1.2]), 1.4, 0, 1)
    h = (2.5 ** 2 + 3.0 ** 2 - 2.6 ** 2) / (2 * 2.5)
    assert abs(f - math.pi * (9.0 - h * h)) < 1e-10 and np.abs(c - [h, 0.0, 0.0]).max() < 1e-12
    xyz, rad = random_cluster(12, 7, rmin=1.0, rmax=2.0)
    for i in range(12):
        for j in range(i + 1, 12):
            fa, ca = oracle.facet_centroid(xyz, rad, 1.4, i, j)
            fb, cb = oracle.facet_centroid(xyz, rad, 1.4, j, i)
            if fa > 1e-6:
                assert np.abs(ca - cb).max() < 1e-9


def test_volume_vjp_finite_differences():
    xyz, rad = globule(15, 4, hydrogens=True)
    u = np.random.default_rng(1).uniform(-1.0, 1.0, len(rad))
    g = oracle.volume_vjp(xyz, rad, 1.4, u)
    h = 1e-5
    for m in range(len(rad)):
        for c in range(3):
            xp, xm = xyz.copy(), xyz.copy()
            xp[m, c] += h
            xm[m, c] -= h
            fd = (u @ oracle.volume(xp, rad, 1.4)[0] - u @ oracle.volume(xm, rad, 1.4)[0]) / (2 * h)
            assert abs(fd - g[m, c]) < 1e-6 * max(1.0, abs(g[m, c])), (m, c, fd, g[m, c])
    # u = 1 gives the molecular-volume gradient
    assert np.abs(oracle.volume_vjp(xyz, rad, 1.4, np.ones(len(rad))) - oracle.volume(xyz, rad, 1.4)[1]).max() < 1e-10
