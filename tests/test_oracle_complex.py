"""Oracle pins for the dual complex K and its classification.

* K versus the alpha = 0 complex built from Qhull's regular triangulation by
  the attachment rule (library routine + textbook rule, not the oracle's
  per-simplex definition tests);
* K edges versus a direct brute-force test of the definition: the disk cut
  from B_i by the radical plane of i, j, intersected with the half-planes of
  every other neighbour, is minimised over candidate points (centre,
  projections on lines, line-line intersections);
* classification identities and the simplex counts of the paper.
"""
import itertools

import numpy as np
import pytest

import oracle
from synth.globule import heavy_chain, random_cluster
from tests.pins.qhull_complex import alpha0_complex


def _sets(r):
    return (set(map(tuple, r.edges.tolist())), set(map(tuple, r.tris.tolist())), set(map(tuple, r.tets.tolist())))


@pytest.mark.parametrize("n,seed", [(12, 0), (20, 1), (40, 2), (60, 3), (80, 4)])
def test_complex_matches_qhull_random(n, seed):
    xyz, rad = random_cluster(n, seed)
    r = oracle.run(xyz, rad, 1.4)
    assert r.counts["ties_broken"] == 0  # general position: no exact tie
    K1, K2, K3 = alpha0_complex(xyz, rad, 1.4)
    E, T, Q = _sets(r)
    assert Q == K3
    assert T == K2
    assert E == K1


def test_complex_matches_qhull_globule():
    xyz, rad, _ = heavy_chain(300, 1)
    r = oracle.run(xyz, rad, 1.4)
    K1, K2, K3 = alpha0_complex(xyz, rad, 1.4)
    E, T, Q = _sets(r)
    assert (Q, T, E) == (K3, K2, K1)


def _edge_by_definition(P, w, i, j):
    """Is there x on the radical plane of i, j with pi_i(x) <= 0 and pi_m(x) >= pi_i(x) for all m?"""
    u = P[j] - P[i]
    d2 = u @ u
    y = P[i] + u * (d2 + w[i] - w[j]) / (2 * d2)
    r2 = w[i] - ((y - P[i]) @ (y - P[i]))
    if r2 < 0:
        return False
    # in-plane orthonormal basis
    a = np.cross(u, [1.0, 0.3, 0.1])
    a /= np.linalg.norm(a)
    b = np.cross(u / np.sqrt(d2), a)
    lines = []
    for m in range(len(P)):
        if m in (i, j):
            continue
        am = P[m] - P[i]
        # pi_m(x) - pi_i(x) = c0 - 2 am.(x - P_i) ; with x = y + s a + t b
        c0 = am @ am - w[m] + w[i] - 2 * am @ (y - P[i])
        lines.append((c0, -2 * am @ a, -2 * am @ b))
    if not lines:
        return True
    L = np.array(lines)

    def feasible(s, t):
        return (L[:, 0] + L[:, 1] * s + L[:, 2] * t >= -1e-12).all()

    best = np.inf
    cands = [(0.0, 0.0)]
    for c0, ca, cb in L:
        nn = ca * ca + cb * cb
        cands.append((-c0 * ca / nn, -c0 * cb / nn))
    for (p, q) in itertools.combinations(range(len(L)), 2):
        M = np.array([[L[p, 1], L[p, 2]], [L[q, 1], L[q, 2]]])
        if abs(np.linalg.det(M)) < 1e-14:
            continue
        s, t = np.linalg.solve(M, -L[[p, q], 0])
        cands.append((s, t))
    for s, t in cands:
        if feasible(s, t):
            best = min(best, s * s + t * t)
    return best <= r2


@pytest.mark.parametrize("seed", range(3))
def test_edges_match_direct_definition(seed):
    xyz, rad = random_cluster(10, 10 + seed)
    R = rad + 1.4
    w = R * R
    r = oracle.run(xyz, rad, 1.4)
    E = set(map(tuple, r.edges.tolist()))
    for i in range(len(R)):
        for j in range(i + 1, len(R)):
            if np.linalg.norm(xyz[i] - xyz[j]) >= R[i] + R[j]:
                assert (i, j) not in E
                continue
            assert ((i, j) in E) == _edge_by_definition(xyz, w, i, j), (i, j)


def test_classification_identities():
    xyz, rad, _ = heavy_chain(300, 1)
    r = oracle.run(xyz, rad, 1.4)
    # every K-tet face is a K-triangle, every K-triangle edge a K-edge
    T = set(map(tuple, r.tris.tolist()))
    E = set(map(tuple, r.edges.tolist()))
    for q in r.tets.tolist():
        for f in itertools.combinations(q, 3):
            assert f in T
    for t in r.tris.tolist():
        for e in itertools.combinations(t, 2):
            assert e in E
    # exterior triangles are exactly those with at most one K-tet
    assert np.array_equal(r.tri_ext, (r.tri_ntet <= 1).astype(np.uint8))
    # interior (non-exterior) atoms in K have zero area; exposed atoms are exterior
    inner = (r.vert_in == 1) & (r.vert_ext == 0)
    assert np.all(r.area[inner] == 0)
    assert np.all(r.vert_ext[r.area > 1e-9] == 1)
    assert inner.sum() > 10


def test_simplex_counts_per_atom():
    # the paper's counts for a 1700-atom molecule (tests/golden/paper_values.json:
    # > 11200 tets, 22600 triangles, 13000 edges, i.e. 6.6 / 13.3 / 7.6 per
    # atom).  A smaller globule has a larger surface share, so the counts per
    # atom are lower; this is a loose sanity band.
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")) as f:
        g = json.load(f)["simplex_counts"]
    ref = np.array([g["tetrahedra_more_than"], g["triangles_more_than"], g["edges_more_than"]]) / g["atoms"]
    xyz, rad, _ = heavy_chain(2000, 2)
    r = oracle.run(xyz, rad, 1.4)
    n = len(rad)
    per = np.array([r.counts["tetrahedra"], r.counts["triangles"], r.counts["edges"]]) / n
    assert 0.45 * ref[0] < per[0] < 1.3 * ref[0]
    assert 0.45 * ref[1] < per[1] < 1.3 * ref[1]
    assert 0.6 * ref[2] < per[2] < 1.3 * ref[2]
    # Euler characteristic of the dual complex of a connected molecule-like union
    chi = r.counts["vertices"] - r.counts["edges"] + r.counts["triangles"] - r.counts["tetrahedra"]
    assert abs(chi - 1) <= 50  # one component; tunnels and cavities shift it a little
