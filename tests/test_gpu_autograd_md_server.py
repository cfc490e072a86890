"""Growth patterns on the GPU: autograd backward, device-resident MD loop, serving.

* SASAFunction backward (hand-written VJP kernel) vs the oracle VJP and vs
  central finite differences of the FP64 forward (h = 1e-4 A);
* MD-like loop: per-frame SASA and forces F = -gamma dA/dx vs the oracle at
  several frames, coordinates kept on the device;
* continuous batching: every result equals the molecule computed alone.
"""
import numpy as np
import pytest

import oracle
from synth.globule import heavy_chain, random_cluster

pytestmark = pytest.mark.gpu


def _pack(mols):
    offs = np.cumsum([0] + [len(r) for _, r in mols]).astype(np.int64)
    return offs, np.vstack([x for x, _ in mols]), np.concatenate([r for _, r in mols])


def _close(g, g_ref, tol):
    err = np.linalg.norm(g - g_ref, axis=-1) / np.maximum(np.linalg.norm(g_ref, axis=-1), 1.0)
    return err.max()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-4)])
def test_autograd_batch_vs_oracle_vjp(precision, tol):
    import torch
    from paper_2401_10462_amd.autograd import sasa
    mols = [heavy_chain(300, 50_000 + m)[:2] for m in range(6)]
    offs, X, R = _pack(mols)
    w = np.random.default_rng(5).uniform(-1, 1, len(R))
    Xt = torch.tensor(X, device="cuda", requires_grad=True)
    A = sasa(Xt, torch.tensor(R, device="cuda"), 1.4, offsets=offs, precision=precision)
    (torch.tensor(w, device="cuda") * A).sum().backward()
    g = Xt.grad.cpu().numpy()
    for k, (x, r) in enumerate(mols):
        s = slice(offs[k], offs[k + 1])
        ref = oracle.run(x, r, 1.4)
        assert np.abs(A.detach().cpu().numpy()[s] - ref.area).max() <= tol * max(ref.area.max(), 1)
        assert _close(g[s], ref.vjp(w[s]), tol) <= tol


def test_autograd_vs_central_fd():
    import torch
    from paper_2401_10462_amd import SasaContext
    from paper_2401_10462_amd.autograd import sasa
    mols = [heavy_chain(300, 50_100 + m)[:2] for m in range(4)]
    offs, X, R = _pack(mols)
    rng = np.random.default_rng(55)
    w = rng.uniform(-1, 1, len(R))
    Xt = torch.tensor(X, device="cuda", requires_grad=True)
    Rt = torch.tensor(R, device="cuda")
    wt = torch.tensor(w, device="cuda")
    (wt * sasa(Xt, Rt, 1.4, offsets=offs)).sum().backward()
    g = Xt.grad.cpu().numpy()
    ctx = SasaContext(precision="fp64")
    h = 1e-4
    nmol = len(mols)

    def losses(Xh):
        a, _ = ctx.compute_batch(offs, Xh, R, 1.4, grad=False)
        c = ctx.counts()
        return np.array([np.dot(w[offs[k]:offs[k + 1]], a[offs[k]:offs[k + 1]]) for k in range(nmol)]), c

    base_counts = losses(X)[1]
    skipped = checked = 0
    for _ in range(32):
        j = rng.integers(0, 300)
        c = rng.integers(0, 3)
        idx = offs[:-1] + j
        Xp, Xm = X.copy(), X.copy()
        Xp[idx, c] += h
        Xm[idx, c] -= h
        lp, cp = losses(Xp)
        lm, cm = losses(Xm)
        if cp != base_counts or cm != base_counts:
            skipped += 1  # the complex changes within +-h of this point
            continue
        fd = (lp - lm) / (2 * h)
        an = g[idx, c]
        assert np.all(np.abs(an - fd) <= 1e-4 * np.maximum(np.abs(fd), 1.0)), (j, c, an, fd)
        checked += 1
    ctx.close()
    assert checked >= 28


def test_md_loop_forces_vs_oracle():
    import torch
    from paper_2401_10462_amd.md_loop import md_loop
    xyz, rad, _ = heavy_chain(2000, 3)
    gamma = 0.005
    lat, kept = md_loop(xyz, rad, frames=60, sigma=0.02, gamma=gamma, precision="mixed", keep_frames=(0, 30, 59))
    assert len(lat) == 60
    for f, (x, area, forces) in kept.items():
        ref = oracle.run(x, rad, 1.4)
        assert np.all(np.abs(area - ref.area) <= 1e-4 * np.maximum(ref.area, 1.0)), f
        assert _close(forces, -gamma * ref.dadx, gamma * 1e-4) <= gamma * 1e-4 + 1e-12, f
    # the coordinates really moved (cumulative noise ~ 0.02 * sqrt(60) A per component)
    assert np.abs(kept[59][0] - xyz).std() > 0.05


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_server_results_equal_alone(precision):
    from paper_2401_10462_amd import SasaContext
    from paper_2401_10462_amd.server import SasaServer, latency_stats
    rng = np.random.default_rng(3)
    mols = []
    for k in range(40):
        n = int(rng.integers(5, 120))
        mols.append(random_cluster(n, 900 + k))
    mols += [heavy_chain(300, 77)[:2], heavy_chain(300, 78)[:2]]
    alone = SasaContext(precision=precision)
    ref = [alone.compute(x, r, 1.4) for x, r in mols]
    alone.close()
    with SasaServer(precision=precision, slots=3, slot_budget_bytes=64 << 20) as srv:
        futs = [srv.submit(x, r) for x, r in mols]
        res = [f.result(timeout=120) for f in futs]
        st = latency_stats(srv.completed)
        batches = srv.batches
    assert batches < len(mols)  # requests were packed together
    for (a, g), (a0, g0) in zip(res, ref):
        assert np.array_equal(a, a0) and np.array_equal(g, g0)
    assert st["requests"] == len(mols)
