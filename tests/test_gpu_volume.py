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


VJP_CASES = [
    ("cluster-12", lambda: random_cluster(12, 0)),
    ("cluster-80-wide-radii", lambda: random_cluster(80, 4, rmin=0.6, rmax=2.4)),
    ("globule-300", lambda: heavy_chain(300, 1)[:2]),
    ("globule-1000H", lambda: globule(500, 3, hydrogens=True)),
]


@pytest.mark.parametrize("name,make", VJP_CASES, ids=[c[0] for c in VJP_CASES])
def test_volume_vjp_parity(name, make):
    """sum_i u_i dV_i/dx against the oracle's (face areas and clipped-face centroids)."""
    from paper_2401_10462_amd import SasaContext
    xyz, rad = make()
    u = np.random.default_rng(9).uniform(-1.0, 1.0, len(rad))
    print(f"volume vjp {name} n={len(rad)}", flush=True)
    ctx = SasaContext(precision="mixed")
    ctx.compute(xyz, rad, 1.4)
    g = ctx.volume_backward(u)
    ref = oracle.volume_vjp(xyz, rad, 1.4, u)
    eg = np.linalg.norm(g - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1.0)
    assert eg.max() <= TOL, f"vjp rel err {eg.max():.3e} at atom {eg.argmax()}"
    # u = 1: the molecular-volume gradient of sasa_volume
    _, grad = ctx.volume()
    assert np.abs(ctx.volume_backward(np.ones(len(rad))) - grad).max() <= 1e-9 * max(1.0, np.abs(grad).max())
    ctx.close()


def test_volume_autograd_batch():
    """VolumeFunction over a batch of two molecules: forward and backward against the oracle."""
    import torch
    from paper_2401_10462_amd.autograd import volume
    xa, ra = globule(400, 4, hydrogens=True)
    xb, rb = heavy_chain(300, 6)[:2]
    offs = np.array([0, len(ra), len(ra) + len(rb)], dtype=np.int64)
    X = torch.tensor(np.vstack([xa, xb + 150.0]), device="cuda", requires_grad=True)
    R = torch.tensor(np.concatenate([ra, rb]), device="cuda")
    w = np.random.default_rng(3).uniform(-1.0, 1.0, len(R))
    print("volume autograd batch 800 + 300", flush=True)
    V = volume(X, R, 1.4, offsets=offs)
    (torch.tensor(w, device="cuda") * V).sum().backward()
    v, g = V.detach().cpu().numpy(), X.grad.cpu().numpy()
    for s, (x, r) in ((slice(0, len(ra)), (xa, ra)), (slice(len(ra), None), (xb, rb))):
        ref_v, _ = oracle.volume(x, r, 1.4)
        assert (np.abs(v[s] - ref_v) / np.maximum(ref_v, 1.0)).max() <= TOL
        ref_g = oracle.volume_vjp(x, r, 1.4, w[s])
        assert (np.linalg.norm(g[s] - ref_g, axis=1) / np.maximum(np.linalg.norm(ref_g, axis=1), 1.0)).max() <= TOL
