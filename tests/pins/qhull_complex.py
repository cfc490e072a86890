"""The alpha = 0 dual complex from Qhull -- an independent pin for the oracle.

The regular (weighted Delaunay) tetrahedrization is the lower convex hull of
the lifted points (p, |p|^2 - w) (a library routine: scipy's Qhull).  From it
the dual complex follows by the standard attachment rule of alpha complexes at
alpha = 0: a simplex belongs iff it is a face of a member, or its smallest
orthosphere has non-positive power and is power-empty (unattached).
"""
import itertools

import numpy as np
from scipy.spatial import ConvexHull


def regular_tetrahedra(xyz, w):
    lifted = np.column_stack([xyz, (xyz * xyz).sum(1) - w])
    hull = ConvexHull(lifted, qhull_options="Qt")
    lower = hull.equations[:, 3] < 0  # outward normal points down in the lifted axis
    tets = np.sort(hull.simplices[lower], axis=1)
    return tets


def _ortho_power(P, w, idx):
    """Orthocentre (in the affine hull of the centres) and its power for a simplex."""
    p0 = P[idx[0]]
    A = P[list(idx[1:])] - p0
    b = (A * A).sum(1) - w[list(idx[1:])] + w[idx[0]]
    # y = p0 + A^T c with 2 A A^T c = b
    G = 2 * A @ A.T
    c = np.linalg.solve(G, b)
    y = p0 + A.T @ c
    return y, ((y - p0) ** 2).sum() - w[idx[0]]


def power_empty(P, w, idx, y):
    pw = ((P - y) ** 2).sum(1) - w
    ref = pw[idx[0]]
    mask = np.ones(len(P), bool)
    mask[list(idx)] = False
    return bool((pw[mask] >= ref).all())


def alpha0_complex(xyz, radii, probe=1.4):
    P = np.asarray(xyz, float)
    R = np.asarray(radii, float) + probe
    w = R * R
    tets = regular_tetrahedra(P, w)
    K3 = set()
    for t in map(tuple, tets):
        _, s = _ortho_power(P, w, t)
        if s <= 0:
            K3.add(t)
    tris = set()
    for t in map(tuple, tets):
        for f in itertools.combinations(t, 3):
            tris.add(f)
    K2 = set(f for t in K3 for f in itertools.combinations(t, 3))
    for f in tris:
        if f in K2:
            continue
        y, s = _ortho_power(P, w, f)
        if s <= 0 and power_empty(P, w, f, y):
            K2.add(f)
    edges = set(e for t in map(tuple, tets) for e in itertools.combinations(t, 2))
    K1 = set(e for f in K2 for e in itertools.combinations(f, 2))
    for e in edges:
        if e in K1:
            continue
        y, s = _ortho_power(P, w, e)
        if s <= 0 and power_empty(P, w, e, y):
            K1.add(e)
    return K1, K2, K3
