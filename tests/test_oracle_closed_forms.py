"""Oracle pins: closed forms and the paper's two-sphere experiment.

Each test fixes a value by mathematics the oracle does not use (textbook
solid angles and dihedral angles, Archimedes' cap area, the two-sphere
derivative, spherical excess), so that a dropped term, a wrong sign or a
swapped operand in the oracle fails here.
"""
import math

import numpy as np
import pytest

import oracle
from tests.pins.slice_area import exposed_area

PI = math.pi


def _golden():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")) as f:
        return json.load(f)


def test_single_sphere():
    # one ball: the whole sphere is exposed, K = {v}, no gradient
    r = oracle.run(np.array([[1.0, -2.0, 3.0]]), [1.7], 1.4)
    assert r.area[0] == pytest.approx(4 * PI * 3.1 ** 2, rel=1e-14)
    assert r.counts["vertices"] == 1 and r.counts["edges"] == 0
    assert np.all(r.dadx == 0)


def test_solid_angle_textbook_values():
    o = np.zeros(3)
    ex, ey, ez = np.eye(3)
    # octant: pi/2 sr -> 1/8 of the sphere
    assert oracle.solid_angle(o, ex, ey, ez) == pytest.approx(1 / 8, rel=1e-14)
    # regular tetrahedron vertex: arccos(23/27) sr
    P = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
    assert oracle.solid_angle(*P) == pytest.approx(math.acos(23 / 27) / (4 * PI), rel=1e-13)
    # nearly flat cone around the apex: close to a hemisphere (denominator < 0 branch)
    eps = 1e-3
    a = np.array([1, 0, -eps])
    b = np.array([-0.5, math.sqrt(3) / 2, -eps])
    c = np.array([-0.5, -math.sqrt(3) / 2, -eps])
    w = oracle.solid_angle(o, a, b, c)
    assert 0.49 < w < 0.5


def test_dihedral_textbook_values():
    o = np.zeros(3)
    ex, ey, ez = np.eye(3)
    assert oracle.dihedral(o, ex, ey, ez) == pytest.approx(0.25, rel=1e-14)
    P = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
    assert oracle.dihedral(*P) == pytest.approx(math.acos(1 / 3) / (2 * PI), rel=1e-13)
    # obtuse: faces almost opposite
    k = np.array([0.5, 1.0, 0.01])
    l = np.array([0.5, -1.0, 0.01])
    assert oracle.dihedral(o, ex, k, l) == pytest.approx((PI - 2 * math.atan2(0.01, 1.0)) / (2 * PI), rel=1e-12)


@pytest.mark.parametrize("seed", range(5))
def test_spherical_excess_links_solid_and_dihedral_angles(seed):
    # Gauss-Bonnet on the unit sphere: solid angle = sum of the three dihedral
    # angles at the apex edges - pi, i.e. omega = (phi_ij + phi_ik + phi_il)/2 - 1/4.
    rng = np.random.default_rng(seed)
    P = rng.normal(size=(4, 3))
    w = oracle.solid_angle(*P)
    s = (oracle.dihedral(P[0], P[1], P[2], P[3]) + oracle.dihedral(P[0], P[2], P[1], P[3])
         + oracle.dihedral(P[0], P[3], P[1], P[2]))
    assert w == pytest.approx(s / 2 - 0.25, abs=1e-13)


def test_octants_close_around_vertex_and_edge():
    # the 8 octant tetrahedra fill the space around the origin: solid angles sum to 1,
    # the 4 around the +x axis have dihedral fractions summing to 1
    o = np.zeros(3)
    tot = 0.0
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sz in (-1, 1):
                tot += oracle.solid_angle(o, [sx, 0, 0], [0, sy, 0], [0, 0, sz])
    assert tot == pytest.approx(1.0, abs=1e-14)
    ring = [[0, 1, 0], [0, 0, 1], [0, -1, 0], [0, 0, -1]]
    tot = sum(oracle.dihedral(o, [1, 0, 0], ring[q], ring[(q + 1) % 4]) for q in range(4))
    assert tot == pytest.approx(1.0, abs=1e-14)


def test_cap_area_archimedes():
    # two balls, cap of sphere i inside ball j vs the independent slice integral
    P = np.array([[0, 0, 0], [2.3, 1.1, -0.4]], float)
    R = np.array([3.0, 2.6])
    cap = oracle.cap_area(P[0], R[0], P[1], R[1])
    exposed = exposed_area(0, P, R)
    assert cap == pytest.approx(4 * PI * R[0] ** 2 - exposed, abs=1e-9)


@pytest.mark.parametrize("seed", range(6))
def test_triple_term_matches_slice_integral(seed):
    # S_ijk^(i) = area of sphere i inside B_j and B_k = cap_j + cap_k - (covered by j or k)
    rng = np.random.default_rng(100 + seed)
    while True:
        P = rng.uniform(-1.6, 1.6, size=(3, 3))
        R = rng.uniform(2.6, 3.2, size=3)
        d = np.linalg.norm(P[:, None] - P[None], axis=-1)
        if (d[np.triu_indices(3, 1)] > 0.8).all():
            break
    S = oracle.triple_term(P[0], R[0], P[1], R[1], P[2], R[2])
    covered = 4 * PI * R[0] ** 2 - exposed_area(0, P, R)
    caps = oracle.cap_area(P[0], R[0], P[1], R[1]) + oracle.cap_area(P[0], R[0], P[2], R[2])
    assert S == pytest.approx(caps - covered, abs=1e-8)


def test_triple_term_equal_radii_limit_is_a_120_degree_lune():
    # three coincident-size balls on a tiny equilateral triangle: the caps are
    # almost hemispheres whose planes meet at 120 degrees -> lune of 1/3 sphere
    d = 1e-4
    R = 3.0
    P = np.array([[0, 0, 0], [d, 0, 0], [d / 2, d * math.sqrt(3) / 2, 0]])
    S = oracle.triple_term(P[0], R, P[1], R, P[2], R)
    assert S == pytest.approx(4 * PI * R * R / 3, rel=1e-4)


def _two(d, r1=1.5, r2=1.7, probe=1.4):
    u = np.array([0.6, -0.48, 0.64])
    P = np.array([[0.3, 0.2, -0.1], [0.3, 0.2, -0.1]]) + np.outer([0, d], u)
    return oracle.run(P, [r1, r2], probe), u


@pytest.mark.parametrize("d", [0.1, 0.15, 0.5, 1.0, 2.5, 4.0, 5.5, 5.99, 6.01, 7.0])
def test_two_spheres_closed_form(d):
    # extended radii 2.9 and 3.1 A as in the paper's singularity study
    r, u = _two(d)
    R1, R2 = 2.9, 3.1
    w1, w2 = R1 * R1, R2 * R2
    if d >= R1 + R2:
        exp = [4 * PI * w1, 4 * PI * w2]
        g = 0.0
    elif d <= R2 - R1:
        exp = [0.0, 4 * PI * w2]  # ball 1 inside ball 2
        g = 0.0
    else:
        a1 = (d * d + w1 - w2) / (2 * d)
        a2 = (d * d + w2 - w1) / (2 * d)
        exp = [4 * PI * w1 - 2 * PI * R1 * (R1 - a1), 4 * PI * w2 - 2 * PI * R2 * (R2 - a2)]
        g = PI * (R1 + R2) * (1 - (R1 - R2) ** 2 / d ** 2)  # d(A1+A2)/dd
    assert r.area == pytest.approx(exp, abs=1e-10)
    # the total's gradient with respect to atom 2 is g along u, atom 1 gets -g u
    assert r.dadx[1] == pytest.approx(g * u, abs=1e-10)
    assert r.dadx[0] == pytest.approx(-g * u, abs=1e-10)


def test_two_sphere_study_minimum_and_leap():
    # sum of SASA is minimal (4 pi 3.1^2) once the smaller ball is inside the
    # larger (d <= 0.2), and its derivative jumps by pi (R1+R2)(1-(R1-R2)^2/d^2)
    # = 18.83 A^2/A at external tangency d = 6.0; the paper's printed bound on
    # the leap and its radii come from tests/golden/paper_values.json
    gold = _golden()["two_sphere_study"]
    assert gold["extended_radii_A"] == [2.9, 3.1]
    tot = {d: _two(d)[0].area.sum() for d in (0.05, 0.2, 0.3, 1.0, 3.0, 5.9, 6.1)}
    assert tot[0.05] == pytest.approx(4 * PI * 3.1 ** 2, rel=1e-14)
    assert tot[0.2] == pytest.approx(4 * PI * 3.1 ** 2, abs=1e-9)
    assert tot[0.3] > tot[0.2] and tot[1.0] > tot[0.3] and tot[3.0] > tot[1.0]
    inside, _ = _two(6.0 - 1e-9)
    outside, _ = _two(6.0 + 1e-9)
    leap = np.linalg.norm(inside.dadx[1]) - np.linalg.norm(outside.dadx[1])
    assert leap == pytest.approx(18.83, abs=5e-3)
    assert leap < gold["derivative_leap_upper_bound_A2"]
