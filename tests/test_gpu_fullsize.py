"""The HIP path at the workloads' full sizes, against the FP64 oracle.

* MD-like sequence: a 20,000-atom globule (chains of 2,500 atoms), 500 frames
  of cumulative Gaussian moves (sigma 0.02 A), SASA + forces (gamma 0.005) with
  the state on the device -- areas and forces of frames 0, 100, 250 and 499 vs
  the oracle, and the dual complex of the first frame simplex for simplex;
* serving: requests from 200 to 20,000 atoms in one continuous-batching run,
  each result bitwise equal to the molecule computed alone, and 200 served
  requests of log-uniform size checked one by one against the oracle;
* differentiation: 64 conformations of 2,000 atoms (8 chains x 8 noise
  frames) through SASAFunction, loss sum w_i A_i with w ~ U(-1, 1), backward
  vs the oracle's VJP on sampled molecules and vs central differences.

Tolerances as in the other parity tests: MIXED 1e-4 relative to
max(|ref|, 1 A^2) per atom (forces scaled by gamma), FP64 1e-9.
"""
import numpy as np
import pytest

import oracle
from synth.globule import globule_complex, heavy_chains, md_frames

pytestmark = pytest.mark.gpu


def _rel(a, ref, floor=1.0):
    return np.abs(a - ref) / np.maximum(np.abs(ref), floor)


def _grad_rel(g, ref, floor=1.0):
    return np.linalg.norm(g - ref, axis=-1) / np.maximum(np.linalg.norm(ref, axis=-1), floor)


@pytest.fixture(scope="module")
def globule20k():
    print("generating the 20,000-atom globule", flush=True)
    return globule_complex(20000, 3)


def test_md_globule_20000(globule20k):
    """500 frames with the state on the device (trajectory mode), checked
    against the oracle at frames 0, 100, 250 and 499."""
    from paper_2401_10462_amd import SasaContext
    from paper_2401_10462_amd.md_loop import md_loop
    xyz, rad = globule20k
    gamma = 0.005
    keep = (0, 100, 250, 499)
    print("md loop: 500 frames", flush=True)
    lat, kept = md_loop(xyz, rad, frames=500, sigma=0.02, gamma=gamma, precision="mixed", keep_frames=keep,
                        frame_hints=True)
    print("oracle on frames", keep, flush=True)
    refs = dict(zip(keep, oracle.run_many([(kept[f][0], rad, 1.4) for f in keep], workers=4)))
    for f in keep:
        x, area, forces = kept[f]
        print(f"frame {f}: area err {_rel(area, refs[f].area).max():.2e}, "
              f"force err {_grad_rel(forces / gamma, -refs[f].dadx).max():.2e}", flush=True)
    for f in keep:
        x, area, forces = kept[f]
        assert _rel(area, refs[f].area).max() <= 1e-4, f
        assert _grad_rel(forces / gamma, -refs[f].dadx).max() <= 1e-4, f
    # the dual complex of the first frame, simplex for simplex (FP64 predicates in both precisions)
    x0 = kept[0][0]
    ref = refs[0]
    ctx = SasaContext(precision="fp64")
    area, dadx = ctx.compute(x0, rad, 1.4)
    assert _rel(area, ref.area).max() <= 1e-9
    assert _grad_rel(dadx, ref.dadx).max() <= 1e-9
    e, t, nt, q, vf = ctx.export()
    assert set(map(tuple, q.tolist())) == set(map(tuple, ref.tets.tolist()))
    assert {tuple(a): int(k) for a, k in zip(t.tolist(), nt.tolist())} == \
        {tuple(a): int(k) for a, k in zip(ref.tris.tolist(), ref.tri_ntet.tolist())}
    assert set(map(tuple, e.tolist())) == set(map(tuple, ref.edges.tolist()))
    d = ctx.diagnostics()
    assert d["overflow"] == 0 and d["lost_pairs"] == 0
    ctx.close()


def test_serving_batch_invariance_200_to_20000(globule20k):
    """Requests of 200 to 20,000 atoms in one continuous-batching run: each
    result bitwise equal to the molecule computed alone."""
    from paper_2401_10462_amd import SasaContext
    from paper_2401_10462_amd.server import SasaServer
    xyz, rad = globule20k
    rng = np.random.default_rng(4)
    mols = []
    for n in (200, 20000, 640, 2100, 7000, 350, 12000, 900):
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        mols.append((np.ascontiguousarray(xyz[:n] @ q.T), np.ascontiguousarray(rad[:n])))
    alone = SasaContext(precision="mixed")
    ref = [alone.compute(x, r, 1.4) for x, r in mols]
    alone.close()
    with SasaServer(precision="mixed", slots=3, slot_budget_bytes=256 << 20) as srv:
        res = [f.result(timeout=120) for f in [srv.submit(x, r) for x, r in mols]]
        assert srv.batches < len(mols)
    for (a, g), (a0, g0) in zip(res, ref):
        assert np.array_equal(a, a0) and np.array_equal(g, g0)


def test_served_requests_vs_oracle(globule20k):
    """200 requests of log-uniform size 200..20,000 atoms (the first n atoms of
    the globule, randomly rotated), served by the batched server, every one
    checked against the oracle (one worker process per host core)."""
    from paper_2401_10462_amd.server import SasaServer
    xyz, rad = globule20k
    rng = np.random.default_rng(40)
    mols = []
    for _ in range(200):
        n = int(round(np.exp(rng.uniform(np.log(200), np.log(20000)))))
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        mols.append((np.ascontiguousarray(xyz[:n] @ q.T + rng.normal(size=3) * 10), np.ascontiguousarray(rad[:n])))
    print(f"serving 200 requests, {sum(len(r) for _, r in mols)} atoms", flush=True)
    with SasaServer(precision="mixed", slots=3, slot_budget_bytes=512 << 20) as srv:
        res = [f.result(timeout=300) for f in [srv.submit(x, r) for x, r in mols]]
    print("oracle on all 200", flush=True)
    refs = oracle.run_many([(x, r, 1.4) for x, r in mols])
    ea = max(_rel(a, o.area).max() for (a, g), o in zip(res, refs))
    eg = max(_grad_rel(g, o.dadx).max() for (a, g), o in zip(res, refs))
    print(f"largest error over the 200 requests: area {ea:.2e}, gradient {eg:.2e}", flush=True)
    for k, ((a, g), o) in enumerate(zip(res, refs)):
        assert _rel(a, o.area).max() <= 1e-4, k
        assert _grad_rel(g, o.dadx).max() <= 1e-4, k


def test_autograd_64_conformations_of_2000():
    import torch
    from paper_2401_10462_amd import SasaContext
    from paper_2401_10462_amd.autograd import sasa
    print("generating 8 chains of 2,000 atoms", flush=True)
    base = heavy_chains([(2000, 50_000 + m) for m in range(8)])
    mols = []
    for m, (x, r, _) in enumerate(base):
        for f, xf in enumerate(md_frames(x, 500 + m, 8, sigma=0.02)):
            mols.append((xf, r))
    assert len(mols) == 64
    offs = np.cumsum([0] + [len(r) for _, r in mols]).astype(np.int64)
    X = np.vstack([x for x, _ in mols])
    R = np.concatenate([r for _, r in mols])
    w = np.random.default_rng(5).uniform(-1, 1, len(R))
    Xt = torch.tensor(X, device="cuda", requires_grad=True)
    Rt = torch.tensor(R, device="cuda")
    A = sasa(Xt, Rt, 1.4, offsets=offs, precision="mixed")
    (torch.tensor(w, device="cuda") * A).sum().backward()
    g = Xt.grad.cpu().numpy()
    a = A.detach().cpu().numpy()
    rng = np.random.default_rng(55)
    picks = rng.choice(64, size=6, replace=False)
    for k, o in zip(picks, oracle.run_many([(mols[k][0], mols[k][1], 1.4) for k in picks], workers=6)):
        s = slice(offs[k], offs[k + 1])
        assert _rel(a[s], o.area).max() <= 1e-4
        assert _grad_rel(g[s], o.vjp(w[s])).max() <= 1e-4
    # central differences of the FP64 forward on 32 atoms, moved in all 64
    # molecules at once; a molecule counts where the differences at h = 1e-4 A
    # and h/2 agree (no change of the complex within +-h there)
    ctx = SasaContext(precision="fp64")

    def losses(Xh):
        ah, _ = ctx.compute_batch(offs, Xh, R, 1.4, grad=False)
        return np.array([np.dot(w[offs[k]:offs[k + 1]], ah[offs[k]:offs[k + 1]]) for k in range(64)])

    def fd(idx, c, h):
        Xp, Xm = X.copy(), X.copy()
        Xp[idx, c] += h
        Xm[idx, c] -= h
        return (losses(Xp) - losses(Xm)) / (2 * h)

    checked = total = 0
    for _ in range(32):
        j = int(rng.integers(0, 2000))
        c = int(rng.integers(0, 3))
        idx = offs[:-1] + j
        f1, f2 = fd(idx, c, 1e-4), fd(idx, c, 5e-5)
        smooth = np.abs(f1 - f2) <= 1e-6 * np.maximum(np.abs(f1), 1.0)
        an = g[idx, c]
        assert np.all((np.abs(an - f1) <= 1e-4 * np.maximum(np.abs(f1), 1.0)) | ~smooth), (j, c)
        checked += int(smooth.sum())
        total += 64
    ctx.close()
    assert checked >= 0.8 * total
