"""Incremental calls (SASA_FLAG_INCREMENTAL): only the stars that moved atoms
can reach are rebuilt; every other atom keeps its star, area and gradient
blocks from the previous call.

A star is decided by the atom's weighted point and those of the atoms whose
balls overlap its ball (no other radical plane meets the ball), so every
result of an incremental call must equal a cold context's bit for bit, over
local moves, a radius change, moves far outside the previous grid, calls with
and without the gradient, and after whatever starts afresh (a batch, a probe
or size change, a failed call).  The mode must also do what it is for: most
stars kept when a small group moves, none when most atoms move.
"""
import numpy as np
import pytest

import oracle
from synth.globule import globule

pytestmark = pytest.mark.gpu


def _ctx(**kw):
    from paper_2401_10462_amd import SasaContext
    return SasaContext(**kw)


def _equal(a, b, what):
    (a1, g1), (a2, g2) = a, b
    assert np.array_equal(a1, a2), f"{what}: areas differ (max {np.abs(a1 - a2).max():.3e})"
    if g1 is not None or g2 is not None:
        assert np.array_equal(g1, g2), f"{what}: gradients differ (max {np.abs(g1 - g2).max():.3e})"


def _local_move(xyz, rng, radius=4.0, sigma=0.3):
    """Atoms within `radius` of a random atom, each displaced by N(0, sigma^2) A (a side-chain-like move)."""
    c = xyz[rng.integers(len(xyz))]
    sel = np.nonzero(np.linalg.norm(xyz - c, axis=1) < radius)[0]
    out = xyz.copy()
    out[sel] += rng.normal(0.0, sigma, size=(len(sel), 3))
    return out, len(sel)


def _tiled(copies):
    """`copies` globules of 2,000 atoms side by side (touching): one molecule."""
    xyz, rad = globule(1000, 5, hydrogens=True)
    xyz = xyz - xyz.mean(axis=0)
    X = np.vstack([xyz + [30.0 * k, 0.0, 0.0] for k in range(copies)])
    return X, np.tile(rad, copies)


@pytest.mark.parametrize("prec,copies", [("fp64", 1), ("mixed", 1), ("fp64", 5)])
def test_incremental_equals_cold(prec, copies):
    """Frames of local moves (one-block and multi-kernel cell list) against a cold context."""
    xyz, rad = _tiled(copies)
    n = len(rad)
    print(f"incremental {n} atoms {prec}", flush=True)
    inc, cold = _ctx(precision=prec, incremental=True), _ctx(precision=prec)
    rng = np.random.default_rng(21)

    def step(X, R, what, grad=True, probe=1.4):
        ri = inc.compute(X, R, probe, grad=grad)
        di = inc.diagnostics()
        rc = cold.compute(X, R, probe, grad=grad)
        dc = cold.diagnostics()
        _equal(ri, rc, what)
        assert di["overflow"] == 0 and dc["skipped_atoms"] == 0 and dc["moved_atoms"] == 0
        assert inc.counts() == cold.counts(), what  # the kept records still sum to the complex
        return di

    d = step(xyz, rad, "first call")
    assert d["moved_atoms"] == n and d["skipped_atoms"] == 0
    d = step(xyz, rad, "same coordinates")
    assert d["moved_atoms"] == 0 and d["skipped_atoms"] == n
    X = xyz
    kept = []
    for f in range(4):
        X, moved = _local_move(X, rng)
        d = step(X, rad, f"local move {f}")
        assert d["moved_atoms"] == moved
        assert d["skipped_atoms"] <= n - moved
        kept.append(d["skipped_atoms"] / n)
    print(f"kept stars per local move: {[round(k, 3) for k in kept]}", flush=True)
    assert min(kept) > (0.6 if copies == 1 else 0.9)
    # one radius changes
    R = rad.copy()
    R[n // 2] *= 1.1
    d = step(X, R, "radius change")
    assert d["moved_atoms"] == 1 and d["skipped_atoms"] > 0
    # areas only, then the gradient again (the blocks of kept stars are stale then)
    d = step(X, R, "areas only", grad=False)
    assert d["skipped_atoms"] == n
    X2, _ = _local_move(X, rng)
    step(X2, R, "gradient after areas only")
    X = X2
    # a group moved far outside the previous grid, and back
    sel = np.arange(0, n, max(1, n // 12))[:12]
    Xf = X.copy()
    Xf[sel] += [60.0, -45.0, 80.0]
    d = step(Xf, R, "moved far away")
    assert d["moved_atoms"] == len(sel)
    d = step(X, R, "moved back")
    assert d["moved_atoms"] == len(sel)
    # most atoms move: every star is rebuilt
    Xj = X + rng.normal(0.0, 0.01, size=X.shape)
    d = step(Xj, R, "all atoms jittered")
    assert d["skipped_atoms"] == 0
    # another probe starts afresh
    d = step(Xj, R, "probe change", probe=1.2)
    assert d["skipped_atoms"] == 0 and d["moved_atoms"] == n
    d = step(Xj, R, "same again", probe=1.2)
    assert d["skipped_atoms"] == n
    # the last frame against the oracle at the precision's bar
    if copies == 1:
        a, g = inc.compute(Xj, R, 1.2)
        ref = oracle.run(Xj, R, 1.2)
        tol = 1e-9 if prec == "fp64" else 1e-4
        assert (np.abs(a - ref.area) / np.maximum(ref.area, 1.0)).max() <= tol
        assert (np.linalg.norm(g - ref.dadx, axis=1) / np.maximum(np.linalg.norm(ref.dadx, axis=1), 1.0)).max() <= tol
    inc.close()
    cold.close()


def test_incremental_restarts():
    """A batch, a size change and a failed call in between: the next call starts afresh."""
    import torch
    xyz, rad = globule(1000, 5, hydrogens=True)
    n = len(rad)
    print(f"incremental restarts {n} atoms", flush=True)
    inc, cold = _ctx(precision="fp64", incremental=True), _ctx(precision="fp64")
    rng = np.random.default_rng(4)
    inc.compute(xyz, rad, 1.4)
    # a batch of two molecules: no star is kept, nor afterwards
    offs = np.array([0, 800, n], dtype=np.int64)
    _equal(inc.compute_batch(offs, xyz, rad, 1.4), cold.compute_batch(offs, xyz, rad, 1.4), "batch")
    assert inc.diagnostics()["skipped_atoms"] == 0
    X, _ = _local_move(xyz, rng)
    _equal(inc.compute(X, rad, 1.4), cold.compute(X, rad, 1.4), "after batch")
    assert inc.diagnostics()["skipped_atoms"] == 0
    # a smaller molecule, then the first again
    _equal(inc.compute(X[:1500], rad[:1500], 1.4), cold.compute(X[:1500], rad[:1500], 1.4), "smaller")
    assert inc.diagnostics()["skipped_atoms"] == 0
    _equal(inc.compute(X, rad, 1.4), cold.compute(X, rad, 1.4), "size back")
    assert inc.diagnostics()["skipped_atoms"] == 0
    # a call that fails on the device (NaN coordinate in device memory)
    dev = torch.device("cuda:0")
    Xd = torch.tensor(X, device=dev)
    Rd = torch.tensor(rad, device=dev)
    Xbad = Xd.clone()
    Xbad[7, 1] = float("nan")
    with pytest.raises(Exception):
        inc.compute(Xbad, Rd, 1.4)
    X3, _ = _local_move(X, rng)
    _equal(inc.compute(X3, rad, 1.4), cold.compute(X3, rad, 1.4), "after a failed call")
    assert inc.diagnostics()["skipped_atoms"] == 0
    X4, _ = _local_move(X3, rng)
    _equal(inc.compute(X4, rad, 1.4), cold.compute(X4, rad, 1.4), "kept again")
    assert inc.diagnostics()["skipped_atoms"] > n // 2
    inc.close()
    cold.close()


def test_incremental_device_forces_and_frames():
    """Device tensors and forces (the MD-like use); with SASA_FLAG_FRAMES too."""
    import torch
    xyz, rad = globule(1000, 6, hydrogens=True)
    n = len(rad)
    print(f"incremental device forces {n} atoms", flush=True)
    dev = torch.device("cuda:0")
    Rd = torch.tensor(rad, device=dev)
    inc, cold = _ctx(precision="mixed", incremental=True), _ctx(precision="mixed")
    both = _ctx(precision="mixed", incremental=True, frames=True)
    rng = np.random.default_rng(8)
    X = xyz
    for f in range(6):
        if f:
            X, _ = _local_move(X, rng, radius=5.0)
        Xd = torch.tensor(X, device=dev)
        ai, fi = inc.forces(Xd, Rd, 0.005, 1.4)
        ac, fc = cold.forces(Xd, Rd, 0.005, 1.4)
        ab, fb = both.forces(Xd, Rd, 0.005, 1.4)
        torch.cuda.synchronize()
        assert torch.equal(ai, ac) and torch.equal(fi, fc), f"frame {f}"
        # hinted clipping orders the terms differently: equal up to rounding
        assert torch.allclose(ab, ac, rtol=1e-12, atol=1e-12) and torch.allclose(fb, fc, rtol=1e-12, atol=1e-12)
        if f:
            assert inc.diagnostics()["skipped_atoms"] > n // 2
    for c in (inc, cold, both):
        c.close()


def test_incremental_with_second_pass_atoms():
    """A large probe puts many atoms past the fast pass (more than 160 overlapping neighbours):
    the kept and rebuilt stars still equal a cold context's, including the second pass's."""
    xyz, rad = globule(400, 2, hydrogens=True)
    n = len(rad)
    print(f"incremental, probe 3.0, {n} atoms", flush=True)
    inc, cold = _ctx(precision="mixed", incremental=True), _ctx(precision="mixed")
    rng = np.random.default_rng(12)
    X = xyz
    for f in range(4):
        if f:
            X, _ = _local_move(X, rng, radius=4.0)
        _equal(inc.compute(X, rad, 3.0), cold.compute(X, rad, 3.0), f"frame {f}")
        di, dc = inc.diagnostics(), cold.diagnostics()
        assert dc["second_pass_atoms"] > 0 and di["overflow"] == 0
        if f:
            assert 0 < di["skipped_atoms"] < n
            assert di["second_pass_atoms"] < dc["second_pass_atoms"]  # only rebuilt stars are queued
        assert inc.counts() == cold.counts()
    inc.close()
    cold.close()


@pytest.mark.parametrize("seed", [31, 32])
def test_incremental_random_sequence(seed):
    """A seeded random sequence of calls (moves of 1 to 400 atoms, radius changes, areas-only calls,
    probe changes, unchanged repeats) on one incremental context, each compared bit for bit with a
    cold context."""
    xyz, rad = globule(1000, 7, hydrogens=True)
    n = len(rad)
    print(f"incremental random sequence, seed {seed}, {n} atoms", flush=True)
    inc, cold = _ctx(precision="fp64", incremental=True), _ctx(precision="fp64")
    rng = np.random.default_rng(seed)
    X, R, probe = xyz.copy(), rad.copy(), 1.4
    skipped = []
    for step in range(24):
        op = rng.integers(6)
        grad = True
        if op == 0:  # a group of 1..400 atoms near a random centre
            c = X[rng.integers(n)]
            order = np.argsort(np.linalg.norm(X - c, axis=1))[: int(rng.integers(1, 400))]
            X = X.copy()
            X[order] += rng.normal(0.0, float(rng.choice([0.01, 0.3, 2.0])), size=(len(order), 3))
        elif op == 1:  # scattered single atoms
            X = X.copy()
            idx = rng.choice(n, size=int(rng.integers(1, 30)), replace=False)
            X[idx] += rng.normal(0.0, 0.5, size=(len(idx), 3))
        elif op == 2:  # radii of a few atoms
            R = R.copy()
            idx = rng.choice(n, size=int(rng.integers(1, 5)), replace=False)
            R[idx] *= rng.uniform(0.9, 1.1, size=len(idx))
        elif op == 3:
            grad = False
        elif op == 4 and rng.random() < 0.3:
            probe = float(rng.choice([1.2, 1.4, 1.6]))
        # op 5: the same input again
        _equal(inc.compute(X, R, probe, grad=grad), cold.compute(X, R, probe, grad=grad), f"step {step} (op {op})")
        skipped.append(inc.diagnostics()["skipped_atoms"])
        assert inc.counts() == cold.counts()
    print(f"kept stars per step: {skipped}", flush=True)
    assert max(skipped) > n // 2
    inc.close()
    cold.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_incremental_with_volume_and_curvature(prec):
    """Volumes, curvatures and their VJPs taken between incremental calls: bitwise those of a cold context, and the
    incremental calls after them still equal cold ones (the volume and curvature kernels recompute FP64 areas of
    every atom and must not disturb the kept stars; the curvature VJP rewrites the gradient blocks, so the next
    call starts afresh)."""
    x, r = globule(600, 4, hydrogens=True)
    n = len(r)
    rng = np.random.default_rng(21)
    u = rng.uniform(-1.0, 1.0, n)
    inc, cold = _ctx(precision=prec, incremental=True), _ctx(precision=prec)
    cur = x
    for step in range(6):
        cur, moved = _local_move(cur, rng)
        print(f"incremental + volume/curvature {prec}: step {step}, {moved} atoms moved", flush=True)
        _equal(inc.compute(cur, r, 1.4), cold.compute(cur, r, 1.4), f"step {step} compute")
        kept = inc.diagnostics()["skipped_atoms"]
        if step in (1, 2, 4):
            assert kept > n // 2, f"step {step}: only {kept} stars kept"
        else:  # the first call, and the calls after a curvature VJP
            assert kept == 0
        if step == 0:
            continue
        (v1, vg1), (v0, vg0) = inc.volume(), cold.volume()
        assert np.array_equal(v1, v0) and np.array_equal(vg1, vg0), f"step {step}: volumes differ"
        assert np.array_equal(inc.volume_backward(u), cold.volume_backward(u))
        (c1, e1), (c0, e0) = inc.curvature(), cold.curvature()
        assert np.array_equal(c1, c0) and e1 == e0, f"step {step}: curvatures differ"
        if step % 2 == 0:
            assert np.array_equal(inc.curvature_backward(u), cold.curvature_backward(u))
    inc.close()
    cold.close()
