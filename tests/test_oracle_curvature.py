"""Pins of the oracle's integrated mean curvature and of the Euler characteristic of the union.

C = sum_i A_i / R_i - 1/2 sum_{i<j} L_ij gamma_ij rests on the areas (pinned elsewhere), on the
exposed arc lengths L_ij and on the crease angles gamma_ij.  Those are pinned here by what fixes
them independently of the oracle's own interval arithmetic:

* one ball: C = 4 pi R;
* the arcs against dense sampling of each circle against every other ball;
* the crease angle against the two outward normals at a point of the circle;
* inflation: growing every radius by e (the probe by e) moves each sphere outwards and each arc
  along sphere i at speed tan(gamma / 2) into its patch, so
      dA/d(probe) = 2 sum_i A_i / R_i - 2 sum_{i<j} L_ij tan(gamma_ij / 2),
  the left side by central differences of the area oracle (Eq. 1), which no arc enters;
* scaling: C is a length, so scaling all coordinates, radii and the probe by s scales it by s.

The Euler characteristic V - E + T - Q of the dual complex (the nerve of the balls up to homotopy,
so the integrated Gaussian curvature of the surface is 4 pi chi by Gauss-Bonnet) is pinned by
topology: a ball 1, two disjoint clusters 2, a closed ring of balls (a solid torus) 0, a hollow
closed shell 2, and balls that all contain one point (a star-shaped, contractible union) 1.
"""
import math

import numpy as np
import pytest

import oracle
from synth.globule import globule, random_cluster


def _R(radii, probe):
    return np.asarray(radii) + probe


def test_one_ball():
    x, r = np.zeros((1, 3)), np.array([1.7])
    c, sums = oracle.mean_curvature(x, r, 1.4)
    assert abs(c[0] - 4.0 * math.pi * 3.1) < 1e-12
    assert sums == (0.0, 0.0)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_arcs_against_sampling(seed):
    """Exposed arc lengths against 200,000 evenly spaced points on each circle."""
    x, r = random_cluster(14, seed, box=6.0)
    R = _R(r, 1.4)
    m = 200000
    t = (np.arange(m) + 0.5) * (2.0 * math.pi / m)
    checked = 0
    for i in range(len(r)):
        for j in range(i + 1, len(r)):
            L, gamma, rho = oracle.exposed_arc(x, r, 1.4, i, j)
            d = np.linalg.norm(x[j] - x[i])
            if not (abs(R[i] - R[j]) < d < R[i] + R[j]):
                assert L == 0.0 and rho == 0.0
                continue
            u = (x[j] - x[i]) / d
            h = (d * d + R[i] ** 2 - R[j] ** 2) / (2 * d)
            e1 = np.cross(u, [0.3, 0.5, 0.8]); e1 /= np.linalg.norm(e1)
            e2 = np.cross(u, e1)
            c = x[i] + h * u
            pts = c + math.sqrt(R[i] ** 2 - h * h) * (np.cos(t)[:, None] * e1 + np.sin(t)[:, None] * e2)
            inside = np.zeros(m, bool)
            for k in range(len(r)):
                if k not in (i, j):
                    inside |= np.sum((pts - x[k]) ** 2, axis=1) < R[k] ** 2
            L_s = 2.0 * math.pi * math.sqrt(R[i] ** 2 - h * h) * (1.0 - inside.mean())
            assert abs(L - L_s) <= 2e-4 * max(2.0 * math.pi * rho, 1.0), (i, j, L, L_s)
            # the crease angle: between the outward normals at a point of the circle
            p = pts[0]
            ni, nj = (p - x[i]) / R[i], (p - x[j]) / R[j]
            assert abs(gamma - math.acos(np.clip(ni @ nj, -1.0, 1.0))) < 1e-6
            checked += 1
    assert checked > 10


@pytest.mark.parametrize("case", ["cluster1", "cluster2", "globule"])
def test_inflation_identity(case):
    """dA/d(probe) by central differences of Eq. 1 against 2 sum A/R - 2 sum L tan(gamma / 2)."""
    if case == "globule":
        x, r = globule(60, 4)
    else:
        x, r = random_cluster(40, int(case[-1]), box=9.0)
    probe, h = 1.4, 1e-5
    a0 = oracle.run(x, r, probe).area
    ap = oracle.run(x, r, probe + h).area.sum()
    am = oracle.run(x, r, probe - h).area.sum()
    dA = (ap - am) / (2 * h)
    _, (_, s_tan) = oracle.mean_curvature(x, r, probe, area=a0)
    rhs = 2.0 * np.sum(a0 / _R(r, probe)) - 2.0 * s_tan
    assert abs(dA - rhs) <= 1e-6 * max(abs(dA), 1.0), (dA, rhs)


def test_scaling():
    x, r = random_cluster(30, 5, box=8.0)
    c1, _ = oracle.mean_curvature(x, r, 1.4)
    c2, _ = oracle.mean_curvature(2.5 * x, 2.5 * r, 3.5)
    assert np.allclose(c2, 2.5 * c1, rtol=1e-10, atol=1e-10)


def test_two_balls_total():
    """Two equal balls: the total from the pinned pieces, C = 4 pi R + 2 pi d - pi rho gamma."""
    R, d = 3.1, 3.0
    x, r = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]]), np.array([1.7, 1.7])
    c, _ = oracle.mean_curvature(x, r, 1.4)
    rho = math.sqrt(R * R - d * d / 4)
    gamma = 2.0 * math.asin(d / (2.0 * R))  # the angle between the normals, from the isosceles triangle
    assert abs(c.sum() - (4 * math.pi * R + 2 * math.pi * d - math.pi * rho * gamma)) < 1e-11


def _ring(m=8, radius=4.0, r=0.6):
    a = 2 * math.pi * np.arange(m) / m
    return np.stack([radius * np.cos(a), radius * np.sin(a), np.zeros(m)], axis=1), np.full(m, r)


def _shell(m=100, radius=10.0, r=1.6):
    k = np.arange(m) + 0.5
    z = 1 - 2 * k / m
    phi = math.pi * (1 + math.sqrt(5)) * k
    s = np.sqrt(1 - z * z)
    return radius * np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1), np.full(m, r)


@pytest.mark.parametrize("case,chi", [("ball", 1), ("two clusters", 2), ("ring", 0), ("shell", 2), ("star", 1)])
def test_euler_characteristic(case, chi):
    if case == "ball":
        x, r = np.zeros((1, 3)), np.array([1.5])
    elif case == "two clusters":
        a, ra = random_cluster(12, 7, box=5.0)
        x, r = np.vstack([a, a + [40.0, 0.0, 0.0]]), np.concatenate([ra, ra])
        # each cluster in one piece
        assert oracle.euler_characteristic(oracle.run(a, ra, 1.4)) == 1
    elif case == "ring":
        x, r = _ring()
    elif case == "shell":
        x, r = _shell()
    else:
        # centres within 2 sqrt(3) A of the box centre, radii + probe >= 4.9 A: every ball holds it
        x, r = random_cluster(40, 3, box=4.0, rmin=3.5, rmax=4.0)
    assert oracle.euler_characteristic(oracle.run(x, r, 1.4)) == chi
