"""sasa_compute_noalloc (the entry point with the library's fixed work space)
against sasa_compute on the same device buffers, through the C-ABI: two calls
in a row, the second with a smaller molecule, in both precisions."""
import numpy as np
import pytest

import oracle
from synth.globule import globule, random_cluster

pytestmark = pytest.mark.gpu


def _dev(xyz, rad):
    import torch
    X = torch.tensor(np.ascontiguousarray(xyz), dtype=torch.float64, device="cuda:0")
    R = torch.tensor(np.ascontiguousarray(rad), dtype=torch.float64, device="cuda:0")
    return X, R


def _noalloc(X, R, prec):
    import torch
    from paper_2401_10462_amd import _lib
    n = R.shape[0]
    a = torch.full((n,), -1.0, dtype=torch.float64, device="cuda:0")
    g = torch.full((n, 3), -1.0, dtype=torch.float64, device="cuda:0")
    _lib.sasa_compute_noalloc(0, n, X, R, 1.4, a, g, precision=_lib.SASA_FP64 if prec == "fp64" else _lib.SASA_MIXED)
    torch.cuda.synchronize()
    return a.cpu().numpy(), g.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_equals_compute_two_calls(prec):
    import torch
    from paper_2401_10462_amd import SasaContext, _lib
    big = globule(2048, 7, hydrogens=True)  # 4096 atoms: the entry point's maximum
    assert len(big[1]) == _lib.SASA_NOALLOC_MAX_ATOMS
    small = random_cluster(300, 5)
    ctx = SasaContext(precision=prec)
    try:
        for xyz, rad in (big, small):
            X, R = _dev(xyz, rad)
            a0, g0 = ctx.compute(X, R, 1.4)
            torch.cuda.synchronize()
            a0, g0 = a0.cpu().numpy(), g0.cpu().numpy()
            a1, g1 = _noalloc(X, R, prec)
            # the same kernels on the same inputs
            assert np.array_equal(a0, a1) and np.array_equal(g0, g1)
        ref = oracle.run(*small, 1.4)
        tol = 1e-9 if prec == "fp64" else 1e-4
        assert np.all(np.abs(a1 - ref.area) <= tol * np.maximum(ref.area, 1.0))
        assert np.all(np.linalg.norm(g1 - ref.dadx, axis=1) <= tol * np.maximum(np.linalg.norm(ref.dadx, axis=1), 1.0))
    finally:
        ctx.close()


def test_noalloc_limits():
    from paper_2401_10462_amd import _lib
    xyz, rad = random_cluster(40, 2)
    X, R = _dev(xyz, rad)
    # no atoms: nothing to do
    _lib.sasa_compute_noalloc(0, 0, X, R, 1.4, None, None)
    # beyond the fixed work space: a clear error, nothing launched
    big = globule(2100, 3, hydrogens=True)
    XB, RB = _dev(*big)
    with pytest.raises(_lib.SasaError) as e:
        _lib.sasa_compute_noalloc(0, len(big[1]), XB, RB, 1.4, None, None)
    assert e.value.code == _lib.SASA_E_INVAL and "SASA_NOALLOC_MAX_ATOMS" in str(e.value)
    # invalid input is reported like sasa_compute's
    bad = rad.copy()
    bad[3] = -1.0
    XR, RR = _dev(xyz, bad)
    with pytest.raises(_lib.SasaError) as e:
        _lib.sasa_compute_noalloc(0, len(bad), XR, RR, 1.4, None, None)
    assert e.value.code == _lib.SASA_E_INVAL
    # and a good call after the failures
    a, g = _noalloc(X, R, "fp64")
    ref = oracle.run(xyz, rad, 1.4)
    assert np.all(np.abs(a - ref.area) <= 1e-9 * np.maximum(ref.area, 1.0))
