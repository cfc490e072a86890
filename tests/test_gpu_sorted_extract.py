"""The paper's sorted-face extraction of unique triangles against the stars.

The stars classify every triangle locally (n_t = end vertices of the cell edge
inside the ball); the paper's GPU section sorts the faces of all tetrahedra
and counts the runs.  Both must give the same triangles with the same n_t
(hence the same exterior ones, n_t <= 1), equal to the oracle's where it runs.
"""
import numpy as np
import pytest

import oracle
from synth.globule import globule, heavy_chain, random_cluster

pytestmark = pytest.mark.gpu


def _dict(tris, nt):
    d = {tuple(t): int(k) for t, k in zip(tris.tolist(), nt.tolist())}
    assert len(d) == len(tris), "duplicate triangles"
    return d


CASES = [
    ("one-ball", lambda: (np.zeros((1, 3)), np.array([1.7]))),
    ("two-balls", lambda: (np.array([[0.0, 0.0, 0.0], [2.5, 0.3, -0.2]]), np.array([1.6, 1.2]))),
    ("cluster-40", lambda: random_cluster(40, 2)),
    ("globule-300", lambda: heavy_chain(300, 1)[:2]),
    ("globule-5000H", lambda: globule(2500, 2, hydrogens=True)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_sorted_faces_equal_stars(name, make):
    from paper_2401_10462_amd import SasaContext
    xyz, rad = make()
    print(f"sorted extraction {name} n={len(rad)}", flush=True)
    ctx = SasaContext(precision="mixed")
    ctx.compute(xyz, rad, 1.4)
    tris, nt, ms = ctx.triangles_by_sort()
    _, t_star, nt_star, _, _ = ctx.export()
    d_sort, d_star = _dict(tris, nt), _dict(t_star, nt_star)
    assert d_sort == d_star
    n_faces = int((nt > 0).sum())
    keys = [tuple(t) for t in tris[:n_faces].tolist()]
    assert keys == sorted(keys)                       # the tetrahedron faces come out sorted
    assert (nt[n_faces:] == 0).all()
    if len(rad) <= 300:
        ref = oracle.run(xyz, rad, 1.4)
        assert d_sort == _dict(ref.tris, ref.tri_ntet)
    print(f"{len(tris)} triangles, {ms:.3f} ms", flush=True)
    ctx.close()


def _classify(n, edges, tris, tri_ntet):
    """The classification read from the paper, from a complex: an edge is
    exterior iff it lies on an exterior triangle (n_t <= 1) or on none; a
    vertex iff it has an exterior edge or none."""
    on_tri, on_ext = set(), set()
    for (a, b, c), k in zip(tris.tolist(), tri_ntet.tolist()):
        for e in ((a, b), (a, c), (b, c)):
            on_tri.add(e)
            if k <= 1:
                on_ext.add(e)
    e_ext = {tuple(e): (tuple(e) not in on_tri) or (tuple(e) in on_ext) for e in edges.tolist()}
    has_e, has_ext = set(), set()
    for e, x in e_ext.items():
        has_e.update(e)
        if x:
            has_ext.update(e)
    return e_ext, has_e, has_ext


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_sorted_edges_vertices_equal_stars(name, make):
    """The other half of the paper's extraction: unique edges and vertices by
    sorting, classified from the runs, against the stars' own classification
    (exterior vertices) and against the rule applied to the complex (the
    star kernel's, and the oracle's where it runs)."""
    from paper_2401_10462_amd import SasaContext
    xyz, rad = make()
    print(f"sorted edges/vertices {name} n={len(rad)}", flush=True)
    ctx = SasaContext(precision="mixed")
    ctx.compute(xyz, rad, 1.4)
    edges, e_ext, verts, v_ext, ms = ctx.edges_vertices_by_sort()
    e_star, t_star, nt_star, _, vf = ctx.export()
    keys = [tuple(e) for e in edges.tolist()]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    assert all(a < b for a, b in keys)
    assert set(keys) == set(map(tuple, e_star.tolist()))
    assert verts.tolist() == sorted(np.nonzero(vf & 1)[0].tolist())
    # exterior vertices: the star kernel's flag
    assert np.array_equal(v_ext, (vf[verts] & 2) != 0)
    # exterior edges and vertices: the rule on the star kernel's complex
    rule_e, has_e, has_ext = _classify(len(rad), e_star, t_star, nt_star)
    assert {k: bool(x) for k, x in zip(keys, e_ext.tolist())} == rule_e
    assert [bool(x) for x in v_ext.tolist()] == [(v not in has_e) or (v in has_ext) for v in verts.tolist()]
    if len(rad) <= 300:
        ref = oracle.run(xyz, rad, 1.4)
        ref_e, _, _ = _classify(len(rad), ref.edges, ref.tris, ref.tri_ntet)
        assert {k: bool(x) for k, x in zip(keys, e_ext.tolist())} == ref_e
    print(f"{len(edges)} edges ({int(e_ext.sum())} exterior), {len(verts)} vertices ({int(v_ext.sum())} exterior), "
          f"{ms:.3f} ms", flush=True)
    ctx.close()
