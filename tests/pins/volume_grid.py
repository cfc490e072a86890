"""Independent pin of the per-atom volumes: the cell B_i ∩ L_i integrated directly.

V_i = integral over the (y, z) disk of the ball of the length of the x-chord
of B_i that satisfies pi_i <= pi_k for every atom k whose ball meets B_i (each
such condition is linear in x on a chord).  Polar coordinates about the ball's
axis with r = R sin(theta) make the integrand smooth at the rim; Gauss-Legendre
in theta and in the angle does the rest.  The integrand still has kinks where a
plane becomes active, so this is accurate to about 1e-6 relative, not to
rounding: a loose but fully independent check of the divergence-theorem
volumes (no facets, no areas, no polygons).
"""
import numpy as np


def cell_volume(i, xyz, R, n_theta=400, n_phi=400):
    xyz = np.asarray(xyz, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    p = xyz[i]
    Ri = R[i]
    d = xyz - p
    dist2 = (d * d).sum(1)
    nb = [k for k in range(len(R)) if k != i and dist2[k] < (Ri + R[k]) ** 2]
    t, wt = np.polynomial.legendre.leggauss(n_theta)
    theta = 0.25 * np.pi * (t + 1.0)            # [0, pi/2]
    wt = wt * 0.25 * np.pi
    f, wf = np.polynomial.legendre.leggauss(n_phi)
    phi = np.pi * (f + 1.0)                     # [0, 2 pi]
    wf = wf * np.pi
    TH, PH = np.meshgrid(theta, phi, indexing="ij")
    r = Ri * np.sin(TH)
    y = r * np.cos(PH)
    z = r * np.sin(PH)
    half = Ri * np.cos(TH)                      # x-chord of the ball: |x| <= half
    lo, hi = -half, half.copy()
    for k in nb:
        a = d[k]
        # 2 a . (x, y, z) <= |a|^2 - w_k + w_i  with x free
        c = (a * a).sum() - R[k] ** 2 + Ri ** 2 - 2.0 * (a[1] * y + a[2] * z)
        if a[0] > 0.0:
            hi = np.minimum(hi, c / (2.0 * a[0]))
        elif a[0] < 0.0:
            lo = np.maximum(lo, c / (2.0 * a[0]))
        else:
            hi = np.where(c < 0.0, -np.inf, hi)
    length = np.maximum(hi - lo, 0.0)
    # dA = r dr dphi, dr = R cos(theta) dtheta
    jac = r * Ri * np.cos(TH)
    return float((length * jac * wt[:, None] * wf[None, :]).sum())
