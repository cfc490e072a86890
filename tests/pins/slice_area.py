"""Exposed sphere area by latitude slicing -- an independent pin for the oracle.

It uses no triangulation and none of the paper's formulas.  On a sphere of
radius R the area element is R dphi dz (Archimedes), so the exposed area of
sphere i is R times the integral over the height z of the angular measure of
the latitude circle at z that no other ball covers.  Each other ball covers an
arc of that circle; the exposed measure is 2 pi minus the measure of the union
of arcs.  The integrand is smooth between breakpoints (heights where an arc
appears or vanishes, and heights of points where two cap circles cross); at a
breakpoint it has square-root behaviour, which the substitution
z = m - h cos(t) removes, so Gauss-Legendre in t converges geometrically.
"""
import numpy as np

_GL = {96: np.polynomial.legendre.leggauss(96)}


def _gauss(nodes):
    if nodes not in _GL:
        _GL[nodes] = np.polynomial.legendre.leggauss(nodes)
    return _GL[nodes]


def _frame(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q  # columns e1, e2, e3 (e3 is the slicing axis)


def _union_measure(lo, hi):
    """Measure of the union of arcs [lo, hi] (rows: nodes, cols: arcs) on the circle."""
    two_pi = 2 * np.pi
    width = hi - lo
    start = np.mod(lo, two_pi)
    end = start + width
    wrap = end > two_pi
    s2 = np.where(wrap, 0.0, 0.0)
    e2 = np.where(wrap, end - two_pi, 0.0)
    end = np.minimum(end, two_pi)
    S = np.concatenate([start, s2], axis=1)
    E = np.concatenate([end, e2], axis=1)
    E = np.where(E > S, E, S)  # empty intervals
    order = np.argsort(S, axis=1)
    S = np.take_along_axis(S, order, axis=1)
    E = np.take_along_axis(E, order, axis=1)
    prev = np.maximum.accumulate(E, axis=1)
    prev = np.concatenate([np.zeros((S.shape[0], 1)), prev[:, :-1]], axis=1)
    return np.maximum(0.0, E - np.maximum(S, prev)).sum(axis=1)


def exposed_area(i, xyz, R, frame_seed=12345, nodes=96):
    """Exposed area of sphere i among balls (xyz, R) (radii already probe-inflated).

    ``nodes`` Gauss-Legendre nodes per interval between breakpoints; where three
    or more cap circles cross at one point the integrand is less smooth there
    and converges more slowly (400 nodes reach 1e-12 on such inputs).
    """
    xyz = np.asarray(xyz, float)
    R = np.asarray(R, float)
    c, Ri = xyz[i], R[i]
    F = _frame(frame_seed + i)
    d_all = np.linalg.norm(xyz - c, axis=1)
    nb = [j for j in range(len(xyz)) if j != i and d_all[j] < Ri + R[j]]
    caps = []
    for j in nb:
        d = d_all[j]
        if d == 0.0:  # same centre: the larger ball covers the smaller one
            if R[j] == Ri:
                raise ValueError("two equal balls with one centre")
            if R[j] > Ri:
                return 0.0
            continue
        a = (d * d + Ri * Ri - R[j] * R[j]) / (2 * d)  # cap plane offset along u
        if a <= -Ri:
            return 0.0  # sphere i inside ball j
        if a >= Ri:
            continue  # ball j inside sphere i (or touching): covers nothing
        u = (xyz[j] - c) / d
        caps.append((u @ F[:, 0], u @ F[:, 1], u @ F[:, 2], a, u))
    if not caps:
        return 4 * np.pi * Ri * Ri
    al = np.array([cp[0] for cp in caps])
    be = np.array([cp[1] for cp in caps])
    ga = np.array([cp[2] for cp in caps])
    aa = np.array([cp[3] for cp in caps])
    s = np.sqrt(al * al + be * be)
    th = np.arctan2(be, al)
    # breakpoints: z-extent of every cap circle, z of every pair of crossing cap circles
    zb = [-Ri, Ri]
    rc = np.sqrt(np.maximum(Ri * Ri - aa * aa, 0.0))
    zb += list(aa * ga + s * rc)
    zb += list(aa * ga - s * rc)
    U = np.array([cp[4] for cp in caps])
    for p in range(len(caps)):
        for q in range(p + 1, len(caps)):
            n = np.cross(U[p], U[q])
            nn = n @ n
            if nn < 1e-30:
                continue
            # point on both planes: x = alpha U_p + beta U_q
            g = U[p] @ U[q]
            det = 1 - g * g
            alpha = (aa[p] - aa[q] * g) / det
            beta = (aa[q] - aa[p] * g) / det
            x0 = alpha * U[p] + beta * U[q]
            rem = Ri * Ri - x0 @ x0
            if rem < 0:
                continue
            t = np.sqrt(rem / nn)
            for sgn in (-1, 1):
                x = x0 + sgn * t * n
                zb.append(x @ F[:, 2])
    zb = np.unique(np.clip(np.array(zb), -Ri, Ri))
    zb = zb[np.concatenate([[True], np.diff(zb) > 1e-13])]
    # nodes
    m = 0.5 * (zb[1:] + zb[:-1])
    h = 0.5 * (zb[1:] - zb[:-1])
    gl_t, gl_w = _gauss(nodes)
    t = 0.5 * np.pi * (gl_t + 1)  # t in [0, pi]
    w = 0.5 * np.pi * gl_w
    Z = (m[:, None] - h[:, None] * np.cos(t)[None, :]).reshape(-1)
    Wz = (h[:, None] * np.sin(t)[None, :] * w[None, :]).reshape(-1)
    rho = np.sqrt(np.maximum(Ri * Ri - Z * Z, 0.0))
    # arc of cap j on the circle at height z: rho s cos(phi - th) >= a - z ga
    with np.errstate(divide="ignore", invalid="ignore"):
        qv = (aa[None, :] - Z[:, None] * ga[None, :]) / (rho[:, None] * s[None, :])
    full = (qv <= -1).any(axis=1)
    qc = np.clip(qv, -1, 1)
    hw = np.where(qv >= 1, 0.0, np.arccos(qc))
    lo = th[None, :] - hw
    hi = th[None, :] + hw
    covered = _union_measure(lo, hi)
    expo = np.where(full, 0.0, np.maximum(0.0, 2 * np.pi - covered))
    return Ri * float((expo * Wz).sum())


def exposed_areas(xyz, radii, probe=1.4, nodes=96):
    """Exposed area of every sphere (radii are van der Waals; the probe is added)."""
    R = np.asarray(radii, float) + probe
    return np.array([exposed_area(i, xyz, R, nodes=nodes) for i in range(len(R))])
