"""Pins of the oracle on inputs with exact and near ties (CPU).

Ideal rings, cube corners, lattices and the like hold many weighted points on
one sphere (the weighted Delaunay tetrahedrization is not unique there) and
many radical planes through one line.  The oracle decides every predicate
exactly and breaks ties by a symbolic perturbation of the weights, so it
builds one consistent complex, and Eq. 1 over it gives the exact areas.  The
pins need no triangulation: the latitude-slice integral of each sphere's
exposed area, the limit of four coinciding balls, the two-sphere closed form
at exact tangency, hidden balls, finite differences and the complex's own
structure (closure under faces, Euler characteristic of the union of balls).
"""
import numpy as np
import pytest

import oracle
from synth.degenerate import CASES, cube, lattice, octahedron, regular_tetrahedron, ring
from tests.pins.slice_area import exposed_areas

PROBE = 1.4


@pytest.mark.parametrize("name,inp,nodes,chi", CASES, ids=[c[0] for c in CASES])
def test_areas_match_slice_integral(name, inp, nodes, chi):
    xyz, rad = inp
    r = oracle.run(xyz, rad, PROBE)
    ref = exposed_areas(xyz, rad, PROBE, nodes=nodes)
    assert np.all(r.area >= 0.0), name  # the paper's per-atom non-negativity
    assert np.all(r.area <= 4 * np.pi * (rad + PROBE) ** 2 + 1e-9)
    err = np.abs(r.area - ref) / np.maximum(ref, 1.0)
    assert err.max() <= 1e-9, (name, err.max())
    assert abs(r.area.sum() - ref.sum()) <= 1e-9 * ref.sum()


@pytest.mark.parametrize("name,inp,nodes,chi", CASES, ids=[c[0] for c in CASES])
def test_complex_is_closed_and_has_the_union_topology(name, inp, nodes, chi):
    xyz, rad = inp
    r = oracle.run(xyz, rad, PROBE)
    E = set(map(tuple, r.edges.tolist()))
    T = set(map(tuple, r.tris.tolist()))
    for q in r.tets.tolist():
        for f in ((q[1], q[2], q[3]), (q[0], q[2], q[3]), (q[0], q[1], q[3]), (q[0], q[1], q[2])):
            assert f in T
    for t in r.tris.tolist():
        for e in ((t[0], t[1]), (t[0], t[2]), (t[1], t[2])):
            assert e in E
    for e in r.edges.tolist():
        assert r.vert_in[e[0]] and r.vert_in[e[1]]
    # the dual complex is homotopy equivalent to the union of balls (nerve)
    euler = r.counts["vertices"] - r.counts["edges"] + r.counts["triangles"] - r.counts["tetrahedra"]
    assert euler == chi, (name, euler)


def test_ties_are_exercised():
    # exact coordinates: co-spherical points with exact ties the perturbation decides
    for inp in (cube(2.0), lattice(3, 3.0), octahedron(2.0)):
        assert oracle.run(*inp, PROBE).counts["ties_broken"] > 0
    # rounded ideal ring: no exact tie, but predicates the FP64 filter cannot decide
    r = oracle.run(*ring(), PROBE)
    assert r.counts["exact_predicates"] > 0


def test_regular_tetrahedron_coinciding_limit():
    """Four equal balls on a regular tetrahedron of size d -> 0: the union tends
    to one ball, and by symmetry each atom keeps the quarter of its sphere that
    faces its own vertex, a cone of pi sr, so A_i -> pi w_i, to first order in d."""
    w = (1.7 + PROBE) ** 2
    prev = None
    for d in (1e-1, 1e-2, 1e-3, 1e-4):
        r = oracle.run(*regular_tetrahedron(d), PROBE)
        assert r.counts["tetrahedra"] == 1
        assert np.allclose(r.area, r.area[0], rtol=0, atol=1e-9)
        dev = r.area[0] - np.pi * w
        assert 0 < dev < 20 * d, (d, dev)
        if prev is not None:
            assert 5 < prev / dev < 20  # first order: the deviation shrinks with d
        prev = dev
    ref = exposed_areas(*regular_tetrahedron(1e-2), PROBE)
    assert np.abs(oracle.run(*regular_tetrahedron(1e-2), PROBE).area - ref).max() < 1e-9


def test_exact_external_tangency():
    """r = 1.5, probe 1.5: R = 3 exactly and centres 6 apart, so the balls touch
    exactly (the edge's size predicate is exactly 0).  Each sphere keeps its
    whole area (a cap of height 0) whichever way the tie goes, and the gradient
    is one of the two one-sided limits of the two-sphere closed form:
    d(A_1 + A_2)/dd = pi (R_1 + R_2) (1 - (R_1 - R_2)^2 / d^2) on the overlapping
    side, 0 on the apart side."""
    xyz = np.array([[0.0, 0, 0], [6.0, 0, 0]])
    r = oracle.run(xyz, np.array([1.5, 1.5]), 1.5)
    assert np.allclose(r.area, 4 * np.pi * 9.0, rtol=0, atol=1e-12)
    dd = r.dadx[1, 0]  # d(sum A)/d x_2 = d(sum A)/dd
    assert min(abs(dd - 0.0), abs(dd - np.pi * 6.0)) < 1e-9, dd
    # three balls, pairwise exactly tangent (equilateral triangle of side 6)
    s3 = np.sqrt(27.0)
    xyz3 = np.array([[0.0, 0, 0], [6.0, 0, 0], [3.0, s3, 0]])
    r3 = oracle.run(xyz3, np.full(3, 1.5), 1.5)
    assert np.allclose(r3.area, 4 * np.pi * 9.0, rtol=0, atol=1e-9)


def test_coincident_centres():
    """A smaller ball with the same centre as a larger one has no cell: hidden,
    A = 0 and no gradient; the larger ball's area is as if it were absent.  Two
    equal balls with one centre share one cell and the input is refused."""
    xyz = np.array([[0.0, 0, 0], [0.0, 0, 0], [2.0, 0, 0]])
    rad = np.array([1.7, 1.2, 1.5])
    r = oracle.run(xyz, rad, PROBE)
    alone = oracle.run(xyz[[0, 2]], rad[[0, 2]], PROBE)
    assert r.area[1] == 0.0 and not r.vert_in[1]
    assert np.allclose(r.area[[0, 2]], alone.area, rtol=0, atol=1e-12)
    assert np.all(r.dadx[1] == 0.0)
    assert np.allclose(r.dadx[[0, 2]], alone.dadx, rtol=0, atol=1e-12)
    with pytest.raises(ValueError):
        oracle.run(np.array([[0.0, 0, 0], [0.0, 0, 0]]), np.array([1.7, 1.7]), PROBE)


@pytest.mark.parametrize("name,inp", [("C6 ring", ring()), ("cube corners s=2", cube(2.0))])
def test_gradient_at_ties_by_finite_differences(name, inp):
    """At these ties the area is C^1 but not C^2 (the complex changes on either
    side), so central differences converge to the analytic gradient at first
    order in h: checked at h = 1e-6 A, with the error falling tenfold from 1e-5."""
    xyz, rad = inp
    G = oracle.run(xyz, rad, PROBE).jacobian_dense()
    errs = {}
    for h in (1e-5, 1e-6):
        worst = 0.0
        for m in range(len(xyz)):
            for c in range(3):
                xp, xm = xyz.copy(), xyz.copy()
                xp[m, c] += h
                xm[m, c] -= h
                fd = (oracle.run(xp, rad, PROBE).area - oracle.run(xm, rad, PROBE).area) / (2 * h)
                worst = max(worst, np.abs(fd - G[:, m, c]).max())
        errs[h] = worst
    assert errs[1e-6] < 1e-5, errs
    assert errs[1e-5] > 3 * errs[1e-6], errs


def test_gradient_near_ties_rotated_lattice():
    """The 3x3x3 lattice rotated and moved off the origin: rounding turns its
    co-planar quadruples into nearly flat K-tetrahedra, whose angle terms have
    derivatives on the branch of their (tiny) orientation.  With that sign taken
    exactly, the analytic gradient matches central differences of the slice
    integral (no triangulation involved); a face-centre atom's gradient is 0
    by symmetry."""
    xyz, rad = lattice(3, 3.0)
    rng = np.random.default_rng(11)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    xyz = xyz @ q.T + np.array([10.3, -4.7, 2.2])
    r = oracle.run(xyz, rad, PROBE)
    assert np.abs(r.area - exposed_areas(xyz, rad, PROBE, nodes=200)).max() < 1e-9
    h = 1e-6
    for m in (22, 4, 0):
        fd = np.zeros(3)
        for c in range(3):
            xp, xm = xyz.copy(), xyz.copy()
            xp[m, c] += h
            xm[m, c] -= h
            fd[c] = (exposed_areas(xp, rad, PROBE, nodes=200).sum() - exposed_areas(xm, rad, PROBE, nodes=200).sum()) / (2 * h)
        assert np.abs(r.dadx[m] - fd).max() < 1e-5, (m, r.dadx[m], fd)
    assert np.linalg.norm(r.dadx[22]) < 1e-9
