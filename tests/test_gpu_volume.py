"""Cell volumes and the molecular-volume gradient: HIP path vs the FP64 oracle.

Per atom i: |V - V_ref| <= 1e-9 max(V_ref, 1 A^3) and |g - g_ref| <=
1e-9 max(|g_ref|, 1 A^2), through the C-ABI, for device and host buffers, one
molecule or a batch, contexts of either precision (the volumes are FP64).
"""
import numpy as np
import pytest

import oracle
from synth.globule import globule, heavy_chain, random_cluster

pytestmark = pytest.mark.gpu

TOL = 1e-9


def _check(vol, grad, xyz, rad):
    ref_v, ref_g = oracle.volume(xyz, rad, 1.4)
    ev = np.abs(vol - ref_v) / np.maximum(ref_v, 1.0)
    eg = np.linalg.norm(grad - ref_g, axis=1) / np.maximum(np.linalg.norm(ref_g, axis=1), 1.0)
    assert ev.max() <= TOL, f"volume rel err {ev.max():.3e} at atom {ev.argmax()}"
    assert eg.max() <= TOL, f"gradient rel err {eg.max():.3e} at atom {eg.argmax()}"
    assert np.abs(grad.sum(0)).max() < 1e-8 * max(1.0, np.abs(grad).max())


CASES = [
    ("one-ball", lambda: (np.zeros((1, 3)), np.array([1.7]))),
    ("two-balls", lambda: (np.array([[0.0, 0.0, 0.0], [2.5, 0.3, -0.2]]), np.array([1.6, 1.2]))),
    ("cluster-12", lambda: random_cluster(12, 0)),
    ("cluster-40", lambda: random_cluster(40, 2)),
    ("cluster-80-wide-radii", lambda: random_cluster(80, 4, rmin=0.6, rmax=2.4)),
    ("globule-300", lambda: heavy_chain(300, 1)[:2]),
    ("globule-1000H", lambda: globule(500, 3, hydrogens=True)),
    ("globule-5000H-benchmark", lambda: globule(2500, 2, hydrogens=True)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_volume_parity(name, make, prec):
    from paper_2401_10462_amd import SasaContext
    xyz, rad = make()
    print(f"volume {name} {prec} n={len(rad)}", flush=True)
    ctx = SasaContext(precision=prec)
    ctx.compute(xyz, rad, 1.4)          # host buffers
    vol, grad = ctx.volume()
    _check(vol, grad, xyz, rad)
    ctx.close()


def test_volume_device_and_batch():
    import torch
    from paper_2401_10462_amd import SasaContext
    xa, ra = globule(1000, 4, hydrogens=True)
    xb, rb = heavy_chain(700, 6)[:2]
    dev = torch.device("cuda:0")
    print("volume device buffers 2000 + batch of 2000 + 700", flush=True)
    ctx = SasaContext(precision="mixed")
    ctx.compute(torch.tensor(xa, device=dev), torch.tensor(ra, device=dev), 1.4)
    vol, grad = ctx.volume()
    assert vol.is_cuda and grad.is_cuda
    _check(vol.cpu().numpy(), grad.cpu().numpy(), xa, ra)
    offs = np.array([0, len(ra), len(ra) + len(rb)], dtype=np.int64)
    X = np.vstack([xa, xb + 200.0])
    R = np.concatenate([ra, rb])
    ctx.compute_batch(offs, torch.tensor(X, device=dev), torch.tensor(R, device=dev), 1.4)
    vol, grad = ctx.volume()
    v, g = vol.cpu().numpy(), grad.cpu().numpy()
    _check(v[:len(ra)], g[:len(ra)], xa, ra)
    _check(v[len(ra):], g[len(ra):], xb, rb)
    ctx.close()


def test_volume_needs_a_compute():
    from paper_2401_10462_amd import SasaContext, SasaError
    ctx = SasaContext()
    with pytest.raises(SasaError):
        ctx.volume()
    ctx.close()
