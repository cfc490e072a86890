"""Curvature measures of the accessible surface (sasa_curvature) against the oracle.

Per-atom integrated mean curvature C_i = A_i / R_i - 1/4 sum_j L_ij gamma_ij: the GPU takes the
exposed crease arcs L_ij from the kept complex (the inclusion-exclusion of the volume kernel), the
oracle from the circles themselves (interval union against every other ball), so agreement checks
the arcs end to end.  The Euler characteristic of the union (integrated Gaussian curvature
4 pi chi) must equal the oracle's and the topology of the pinned shapes.
"""
import numpy as np
import pytest

import oracle
from synth.globule import globule, random_cluster
from tests.test_oracle_curvature import _ring, _shell

pytestmark = pytest.mark.gpu

TOL = 1e-9  # FP64 in both precisions, relative per atom with a 1 A floor


def _ctx(**kw):
    from paper_2401_10462_amd import SasaContext
    return SasaContext(**kw)


def _check(c, ref):
    err = np.abs(c - ref) / np.maximum(np.abs(ref), 1.0)
    assert err.max() <= TOL, f"curvature differs by {err.max():.3e} at atom {err.argmax()}"


CASES = [
    ("cluster 30", lambda: random_cluster(30, 1, box=8.0)),
    ("cluster 200", lambda: random_cluster(200, 2)),
    ("globule 300", lambda: globule(300, 1)),
    ("globule 1000 + H", lambda: globule(1000, 5, hydrogens=True)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_mean_curvature_and_euler_vs_oracle(name, make, prec):
    x, r = make()
    print(f"curvature {name} ({len(r)} atoms) {prec}", flush=True)
    ctx = _ctx(precision=prec)
    ctx.compute(x, r, 1.4)
    c, chi = ctx.curvature()
    res = oracle.run(x, r, 1.4)
    ref, _ = oracle.mean_curvature(x, r, 1.4, area=res.area)
    _check(c, ref)
    assert chi == oracle.euler_characteristic(res)
    ctx.close()


@pytest.mark.parametrize("shape,chi", [("ring", 0), ("shell", 2)])
def test_topology_pins(shape, chi):
    x, r = _ring() if shape == "ring" else _shell()
    ctx = _ctx(precision="fp64")
    ctx.compute(x, r, 1.4)
    c, e = ctx.curvature()
    assert e == chi
    ref, _ = oracle.mean_curvature(x, r, 1.4)
    _check(c, ref)
    ctx.close()


def test_device_tensors_batch_and_state():
    """Device outputs, a batch (each molecule's atoms as alone, chi summed), and no kept compute."""
    import torch
    from paper_2401_10462_amd import _lib
    a, ra = globule(300, 1)
    b, rb = random_cluster(120, 4)
    ctx = _ctx(precision="mixed")
    with pytest.raises(_lib.SasaError):
        ctx.curvature()
    dev = torch.device("cuda:0")
    ctx.compute(torch.tensor(a, device=dev), torch.tensor(ra, device=dev), 1.4)
    ca, ea = ctx.curvature()
    assert ca.is_cuda
    ctx.compute(b, rb, 1.4)
    cb, eb = ctx.curvature()
    offs = np.array([0, len(ra), len(ra) + len(rb)], dtype=np.int64)
    ctx.compute_batch(offs, np.vstack([a, b]), np.concatenate([ra, rb]), 1.4)
    cab, eab = ctx.curvature()
    assert np.array_equal(cab, np.concatenate([ca.cpu().numpy(), cb]))
    assert eab == ea + eb
    ctx.close()
