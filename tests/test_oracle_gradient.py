"""Oracle pins for the analytic derivatives (Eq. 2) and the invariants.

* central finite differences of the independent slice-integral areas;
* translation and rotation invariance of every atom's area (rows of the
  Jacobian sum to zero; torques vanish);
* rigid-motion, permutation and scaling behaviour of the areas;
* 0 <= A_i <= 4 pi (r_i + probe)^2 (the paper notes dSASA atoms are never
  negative).
"""
import numpy as np
import pytest

import oracle
from synth.globule import heavy_chain, random_cluster
from tests.pins.slice_area import exposed_area


@pytest.mark.parametrize("seed", range(3))
def test_jacobian_matches_fd_of_slice_integral(seed):
    xyz, rad = random_cluster(7, 200 + seed)
    R = rad + 1.4
    r = oracle.run(xyz, rad, 1.4)
    J = r.jacobian_dense()
    h = 1e-4
    for i in range(len(R)):
        for m in range(len(R)):
            for c in range(3):
                xp = xyz.copy()
                xm = xyz.copy()
                xp[m, c] += h
                xm[m, c] -= h
                fd = (exposed_area(i, xp, R) - exposed_area(i, xm, R)) / (2 * h)
                assert J[i, m, c] == pytest.approx(fd, abs=2e-6 * max(1.0, abs(fd))), (i, m, c)


def test_jacobian_matches_fd_on_globule():
    # oracle areas under central differences, h = 1e-4 A, on a sample of
    # coordinates of a 300-atom globule (skipping any step that changes K)
    xyz, rad, _ = heavy_chain(300, 1)
    base = oracle.run(xyz, rad, 1.4)
    rng = np.random.default_rng(5)
    h = 1e-4
    skipped = 0
    for m in rng.choice(len(rad), size=25, replace=False):
        for c in range(3):
            xp = xyz.copy()
            xm = xyz.copy()
            xp[m, c] += h
            xm[m, c] -= h
            rp = oracle.run(xp, rad, 1.4)
            rm = oracle.run(xm, rad, 1.4)
            if rp.counts != base.counts or rm.counts != base.counts:
                skipped += 1
                continue
            fd = (rp.area.sum() - rm.area.sum()) / (2 * h)
            assert base.dadx[m, c] == pytest.approx(fd, abs=1e-6 * max(1.0, abs(fd)))
    assert skipped <= 3


def test_translation_and_rotation_invariance_per_atom():
    xyz, rad, _ = heavy_chain(300, 1)
    r = oracle.run(xyz, rad, 1.4)
    rows = np.zeros((len(rad), 3))
    torque = np.zeros((len(rad), 3))
    np.add.at(rows, r.jac_rows, r.jac_vals)
    np.add.at(torque, r.jac_rows, np.cross(xyz[r.jac_cols], r.jac_vals))
    scale = np.abs(r.jac_vals).max()
    assert np.abs(rows).max() < 1e-11 * scale
    assert np.abs(torque).max() < 1e-10 * scale * np.abs(xyz).max()


def test_rigid_motion_permutation_scaling():
    xyz, rad, _ = heavy_chain(300, 1)
    r = oracle.run(xyz, rad, 1.4)
    rng = np.random.default_rng(9)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    moved = xyz @ q.T + rng.normal(size=3) * 10
    r2 = oracle.run(moved, rad, 1.4)
    assert np.allclose(r2.area, r.area, rtol=0, atol=1e-9)
    assert np.allclose(r2.dadx, r.dadx @ q.T, rtol=0, atol=1e-8)
    perm = rng.permutation(len(rad))
    r3 = oracle.run(xyz[perm], rad[perm], 1.4)
    assert np.allclose(r3.area, r.area[perm], rtol=0, atol=1e-9)
    assert np.allclose(r3.dadx, r.dadx[perm], rtol=0, atol=1e-8)
    s = 1.7
    r4 = oracle.run(xyz * s, rad * s, 1.4 * s)
    assert np.allclose(r4.area, r.area * s * s, rtol=1e-12, atol=1e-9)
    assert np.allclose(r4.dadx, r.dadx * s, rtol=1e-10, atol=1e-8)


def test_area_bounds():
    xyz, rad, _ = heavy_chain(300, 1)
    r = oracle.run(xyz, rad, 1.4)
    full = 4 * np.pi * (rad + 1.4) ** 2
    assert (r.area >= -1e-9).all()
    assert (r.area <= full + 1e-9).all()
    assert (r.area == 0).sum() > 0 and (r.area > 0).sum() > 0


def test_vjp_is_weighted_jacobian():
    xyz, rad = random_cluster(30, 7)
    r = oracle.run(xyz, rad, 1.4)
    u = np.random.default_rng(1).uniform(-1, 1, len(rad))
    J = r.jacobian_dense()
    assert np.allclose(r.vjp(u), np.einsum("i,imc->mc", u, J), atol=1e-12)
    assert np.allclose(r.dadx, J.sum(0), atol=1e-12)
