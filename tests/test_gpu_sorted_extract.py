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
