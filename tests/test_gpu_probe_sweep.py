"""Volumes, curvatures and their derivatives across probe radii, against the oracle.

The volume and curvature parity tests run at the usual 1.4 A probe; here the same quantities are checked at a
probe of 0 (the van der Waals surface: fewer overlaps, smaller caps, a union with many tunnels), 0.7 A and 3.0 A
(many more overlapping neighbours, larger caps), in both precisions.  Bars as in those tests:
1e-9 relative per atom (floors 1 A^3, 1 A^2, 1 A), FP64 throughout since the volume and curvature kernels are FP64.
"""
import numpy as np
import pytest

import oracle
from synth.globule import globule, random_cluster

pytestmark = pytest.mark.gpu

TOL = 1e-9
PROBES = [0.0, 0.7, 3.0]
_refs = {}


def _ref(probe):
    if probe not in _refs:
        x, r = globule(300, 1)
        res = oracle.run(x, r, probe)
        vol, vgrad = oracle.volume(x, r, probe)
        curv, _ = oracle.mean_curvature(x, r, probe, area=res.area)
        u = np.random.default_rng(11).uniform(-1.0, 1.0, len(r))
        _refs[probe] = dict(x=x, r=r, res=res, vol=vol, vgrad=vgrad, curv=curv, u=u,
                            vvjp=oracle.volume_vjp(x, r, probe, u), chi=oracle.euler_characteristic(res))
    return _refs[probe]


def _rel(a, b, floor=1.0):
    if a.ndim == 2:
        return (np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), floor)).max()
    return (np.abs(a - b) / np.maximum(np.abs(b), floor)).max()


@pytest.mark.parametrize("probe", PROBES)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_volume_and_curvature_across_probes(probe, prec):
    from paper_2401_10462_amd import SasaContext
    ref = _ref(probe)
    print(f"probe sweep: globule 300, probe {probe}, {prec}", flush=True)
    ctx = SasaContext(precision=prec)
    ctx.compute(ref["x"], ref["r"], probe)
    vol, vgrad = ctx.volume()
    assert _rel(vol, ref["vol"]) <= TOL
    assert _rel(vgrad, ref["vgrad"]) <= TOL
    assert _rel(ctx.volume_backward(ref["u"]), ref["vvjp"]) <= TOL
    curv, chi = ctx.curvature()
    assert _rel(curv, ref["curv"]) <= TOL
    assert chi == ref["chi"]
    ctx.close()


@pytest.mark.parametrize("probe", [0.0, 3.0])
def test_curvature_vjp_across_probes(probe):
    """sum_i u_i dC_i/dx against central differences of the oracle's curvature at probes 0 and 3 A."""
    from paper_2401_10462_amd import SasaContext
    x, r = random_cluster(20, 8, box=7.0)
    n = len(r)
    u = np.random.default_rng(8).uniform(-1.0, 1.0, n)
    print(f"curvature VJP, 20-atom cluster, probe {probe}", flush=True)
    ctx = SasaContext(precision="fp64")
    ctx.compute(x, r, probe)
    g = ctx.curvature_backward(u)
    ctx.close()
    h = 1e-5
    fd = np.zeros((n, 3))
    for m in range(n):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[m, a] += h
            xm[m, a] -= h
            fd[m, a] = (u @ oracle.mean_curvature(xp, r, probe)[0] - u @ oracle.mean_curvature(xm, r, probe)[0]) / (2 * h)
    assert _rel(g, fd) <= 1e-5
