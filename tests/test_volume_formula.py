"""The face inclusion-exclusion used by the GPU volumes, checked on the CPU.

The GPU kernel computes each flat face of a cell from the dual complex alone:
2F = rho^2 theta + sum_t delta_t l_t with theta / 2pi = Phi - sum over exterior
triangles of c_t 2 phi(T_x), and the edge lengths as chords less the parts cut
off at K-tetrahedra.  For the per-atom volume derivatives it also forms each
face's first moment, 3 M = rho int_arcs (x - c) ds + sum_t delta_t int_t (x - c) ds,
with the arcs' integral from their end points (the exposed triple points) and
the edges' integrals from the same chord-less-cuts decomposition.  This is a reading written for the volume extension (the
paper gives no volume formula), so it is checked here, written out plainly
over the oracle's complex, against the oracle's volumes whose faces are
clipped from their definition.
"""
import math

import numpy as np
import pytest

import oracle
from synth.globule import globule, random_cluster

TWO_PI = 2.0 * math.pi


def dihedral_frac(e, u, v):
    """Dihedral angle along axis e between the half-planes through u and v, over 2 pi."""
    n1, n2 = np.cross(e, u), np.cross(e, v)
    return math.atan2(np.linalg.norm(np.cross(n1, n2)), n1 @ n2) / TWO_PI


def orthocentre2(a, b, ra, rb):
    """y in span(a, b) with 2 a.y = ra and 2 b.y = rb."""
    aa, bb, ab = a @ a, b @ b, a @ b
    det = 2.0 * (aa * bb - ab * ab)
    return (ra * bb - rb * ab) / det * a + (aa * rb - ab * ra) / det * b


def face_distance(aj, ak, y, hj):
    """Signed distance, in plane j, from the disk centre to the cell edge (i, j, k) through y."""
    nj = aj / np.linalg.norm(aj)
    m = ak - nj * (ak @ nj)
    return (y - nj * hj) @ m / np.linalg.norm(m)


def volumes_from_complex(xyz, rad, probe=1.4):
    r = oracle.run(xyz, rad, probe)
    R = rad + probe
    w = R * R
    n = len(R)
    edges = [tuple(e) for e in r.edges.tolist()]
    vol = np.zeros(n)
    grad = np.zeros((n, 3))
    for i in range(n):
        if not r.vert_in[i]:
            continue
        nb = sorted({b for a, b in edges if a == i} | {a for a, b in edges if b == i})
        P = {j: xyz[j] - xyz[i] for j in nb}
        h = {j: (P[j] @ P[j] + w[i] - w[j]) / (2.0 * np.linalg.norm(P[j])) for j in nb}
        rr = {j: P[j] @ P[j] - w[j] + w[i] for j in nb}
        phi = dict.fromkeys(nb, 0.0)
        arc = dict.fromkeys(nb, 0.0)
        seg = dict.fromkeys(nb, 0.0)
        for q in r.tets.tolist():
            if i not in q:
                continue
            ks = [v for v in q if v != i]
            PP = [P[k] for k in ks]
            z = np.linalg.solve(2.0 * np.array(PP), np.array([rr[k] for k in ks]))
            for c in range(3):
                phi[ks[c]] += dihedral_frac(PP[c], PP[(c + 1) % 3], PP[(c + 2) % 3])
            for o in range(3):
                e, f = (o + 1) % 3, (o + 2) % 3
                y = orthocentre2(PP[e], PP[f], rr[ks[e]], rr[ks[f]])
                u = np.cross(PP[e], PP[f])
                zeta = (z - y) @ u / np.linalg.norm(u)
                sz = zeta if PP[o] @ u > 0.0 else -zeta
                seg[ks[e]] += face_distance(PP[e], PP[f], y, h[ks[e]]) * sz
                seg[ks[f]] += face_distance(PP[f], PP[e], y, h[ks[f]]) * sz
        for t, nt in zip(r.tris.tolist(), r.tri_ntet.tolist()):
            if i not in t or nt > 1:
                continue
            a, b = [v for v in t if v != i]
            ct = 1.0 - 0.5 * nt
            A, B = P[a], P[b]
            y = orthocentre2(A, B, rr[a], rr[b])
            half = math.sqrt(max(w[i] - y @ y, 0.0))
            u = np.cross(A, B)
            x = y + u * half / np.linalg.norm(u)
            arc[a] += ct * 2.0 * dihedral_frac(A, B, x)
            arc[b] += ct * 2.0 * dihedral_frac(B, A, x)
            seg[a] += ct * face_distance(A, B, y, h[a]) * 2.0 * half
            seg[b] += ct * face_distance(B, A, y, h[b]) * 2.0 * half
        hv = 0.0
        for j in nb:
            rho2 = max(w[i] - h[j] ** 2, 0.0)
            F = 0.5 * (rho2 * TWO_PI * (1.0 - phi[j] - arc[j]) + seg[j])
            hv += h[j] * F
            grad[i] -= F * P[j] / np.linalg.norm(P[j])
        vol[i] = (R[i] * r.area[i] + hv) / 3.0
    return vol, grad


def volume_vjp_from_complex(xyz, rad, u, probe=1.4):
    """sum_i u_i dV_i/dp_m from the faces' areas and first moments, written out over the complex."""
    r = oracle.run(xyz, rad, probe)
    R = rad + probe
    w = R * R
    n = len(R)
    edges = [tuple(e) for e in r.edges.tolist()]
    out = np.zeros((n, 3))
    for i in range(n):
        if not r.vert_in[i]:
            continue
        nb = sorted({b for a, b in edges if a == i} | {a for a, b in edges if b == i})
        P = {j: xyz[j] - xyz[i] for j in nb}
        dist = {j: np.linalg.norm(P[j]) for j in nb}
        nh = {j: P[j] / dist[j] for j in nb}
        h = {j: (P[j] @ P[j] + w[i] - w[j]) / (2.0 * dist[j]) for j in nb}
        cen = {j: nh[j] * h[j] for j in nb}
        rr = {j: P[j] @ P[j] - w[j] + w[i] for j in nb}
        phi = dict.fromkeys(nb, 0.0)
        arc = dict.fromkeys(nb, 0.0)
        seg = dict.fromkeys(nb, 0.0)
        mom = {j: np.zeros(3) for j in nb}
        itets = [[v for v in q if v != i] for q in r.tets.tolist() if i in q]
        for ks in itets:
            PP = [P[k] for k in ks]
            z = np.linalg.solve(2.0 * np.array(PP), np.array([rr[k] for k in ks]))
            for c in range(3):
                phi[ks[c]] += dihedral_frac(PP[c], PP[(c + 1) % 3], PP[(c + 2) % 3])
            for o in range(3):
                e, f = (o + 1) % 3, (o + 2) % 3
                y = orthocentre2(PP[e], PP[f], rr[ks[e]], rr[ks[f]])
                ud = np.cross(PP[e], PP[f])
                ud /= np.linalg.norm(ud)
                a = math.sqrt(max(w[i] - y @ y, 0.0))
                zeta = (z - y) @ ud
                sg = 1.0 if PP[o] @ ud > 0.0 else -1.0
                cut = a - sg * zeta                  # the chord's part beyond the tetrahedron's plane
                mid = 0.5 * (zeta + sg * a)          # its middle, along the line
                for pl, other in ((ks[e], ks[f]), (ks[f], ks[e])):
                    dl = face_distance(P[pl], P[other], y, h[pl])
                    seg[pl] += dl * sg * zeta
                    mom[pl] += dl * (a * (y - cen[pl]) - cut * (y + mid * ud - cen[pl])) / 3.0
        for t, nt in zip(r.tris.tolist(), r.tri_ntet.tolist()):
            if i not in t or nt > 1:
                continue
            ka, kb = [v for v in t if v != i]
            ct = 1.0 - 0.5 * nt
            A, B = P[ka], P[kb]
            y = orthocentre2(A, B, rr[ka], rr[kb])
            a = math.sqrt(max(w[i] - y @ y, 0.0))
            ud = np.cross(A, B)
            ud /= np.linalg.norm(ud)
            xs = [y + a * ud, y - a * ud]
            arc[ka] += ct * 2.0 * dihedral_frac(A, B, xs[0])
            arc[kb] += ct * 2.0 * dihedral_frac(B, A, xs[0])
            if nt == 1:  # only the triple point inside the tetrahedron's fourth half-space is exposed
                l = next(v for q in itets if ka in q and kb in q for v in q if v not in (ka, kb))
                xs = [x for x in xs if 2.0 * P[l] @ x <= rr[l]]
            for pl, other in ((ka, B), (kb, A)):
                dl = face_distance(P[pl], other, y, h[pl])
                seg[pl] += ct * dl * 2.0 * a
                mom[pl] += ct * dl * 2.0 * a * (y - cen[pl]) / 3.0
                rho2 = max(w[i] - h[pl] ** 2, 0.0)
                toward = other - nh[pl] * (other @ nh[pl])
                for x in xs:  # an exposed arc ends (+) or starts (-) here, going round n
                    s = 1.0 if np.cross(nh[pl], x - cen[pl]) @ toward > 0.0 else -1.0
                    mom[pl] += rho2 * s * np.cross(x - cen[pl], nh[pl]) / 3.0
        for j in nb:
            rho2 = max(w[i] - h[j] ** 2, 0.0)
            F = 0.5 * (rho2 * TWO_PI * (1.0 - phi[j] - arc[j]) + seg[j])
            out[i] += (u[i] - u[j]) * (F * cen[j] + mom[j]) / dist[j] - u[i] * F * nh[j]
    return out


@pytest.mark.parametrize("make", [lambda: random_cluster(12, 0), lambda: random_cluster(40, 2),
                                  lambda: random_cluster(80, 4, rmin=0.6, rmax=2.4),
                                  lambda: globule(60, 3, hydrogens=True)])
def test_face_moments_from_complex(make):
    xyz, rad = make()
    u = np.random.default_rng(4).uniform(-1.0, 1.0, len(rad))
    g = volume_vjp_from_complex(xyz, rad, u)
    ref = oracle.volume_vjp(xyz, rad, 1.4, u)
    assert np.abs(g - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("make", [lambda: random_cluster(12, 0), lambda: random_cluster(40, 2),
                                  lambda: random_cluster(80, 4, rmin=0.6, rmax=2.4),
                                  lambda: globule(100, 3, hydrogens=True)])
def test_faces_from_complex(make):
    xyz, rad = make()
    v, g = volumes_from_complex(xyz, rad)
    rv, rg = oracle.volume(xyz, rad, 1.4)
    assert np.abs(v - rv).max() <= 1e-11 * max(1.0, rv.max())
    assert np.abs(g - rg).max() <= 1e-11 * max(1.0, np.abs(rg).max())
