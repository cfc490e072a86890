"""Benchmark: exact SASA + gradient throughput (atoms/s) on one MI355X.

One step is one pass of the whole hot path (weights, cell list, per-atom
power-cell star, Eq. 1 terms, Eq. 2 gradient blocks, gradient gather) over one
synthetic molecule whose coordinates are already resident in HBM.

Workload (default): a 5,000-atom globule -- 2,500 heavy atoms (compact
self-avoiding chain, C/N/O/S radii) plus 2,500 hydrogens (r = 1.20 A) --,
probe 1.4 A, MIXED precision as the workload names it (float area terms,
double predicates and accumulation), per-atom SASA and d(sum A)/dx.  The
same plain loop in FP64 is reported beside it: MI355X runs FP64 vector
arithmetic at the rate of unpacked FP32, and FP64 measures faster.

Prints one JSON line.  Extra keys: p50/p99 per-step latency, the batched
form (many molecules per launch sequence), the roofline of the dominant kernel
(HIP events around it, algorithmic FLOPs from the kernel's own work counters)
and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SASA+gradient atoms/s at 1 GPU (batched vs plain, \u22641e-4 rel err); p50/p99 latency"
FP64_PEAK_TFLOPS = 78.6  # MI355X vector FP64
HBM_PEAK = 8.0e12        # MI355X HBM3E, bytes/s
# FP64 operations per unit of star-kernel work, counted from the kernel source:
#   side test of a cell vertex against a plane: 3 mul + 3 add/sub        =  6
#   new cell vertex from three planes (cross products, det, 1 div, 3 dots) = 51
#   neighbour candidate: 3 sub, 3 mul, 2 add, (R_i + R_j)^2               = 10
FLOP_PER_TEST, FLOP_PER_VERTEX, FLOP_PER_CANDIDATE = 6, 51, 10


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=30)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    p.add_argument("--heavy", type=int, default=2500, help="heavy atoms (hydrogens double it)")
    p.add_argument("--seed", type=int, default=2)
    p.add_argument("--batch", type=int, default=32, help="molecules in the batched form (0: skip)")
    p.add_argument("--cpu-seconds", type=float, default=20.0, help="budget of the oracle CPU leg (0: skip)")
    p.add_argument("--workload", default="globule",
                   choices=["globule", "serving", "md", "local", "gbsa", "small", "autograd"],
                   help="globule: the headline line; serving: Poisson stream sweep; md: MD-like frames; "
                        "local: frames of local moves, cold against incremental calls; "
                        "gbsa: Langevin harness with SASA forces through autograd; small: one 300-heavy-atom "
                        "globule in FP64; autograd: 64 conformations of 2,000 atoms, forward + backward")
    p.add_argument("--serve-requests", type=int, default=600, help="requests per arrival rate (serving)")
    p.add_argument("--rates", default="100,500,2000,5000", help="arrival rates, req/s (serving)")
    p.add_argument("--md-atoms", type=int, default=20000)
    p.add_argument("--frames", type=int, default=500)
    p.add_argument("--calibrate-copy", type=int, default=0,
                   help="MiB: only run a device copy of this size (HBM counter calibration) and exit")
    return p.parse_args()


def pool_molecules(sizes, seed=40_000):
    """Request molecules: the first n atoms of pooled globule chains, randomly rotated."""
    from synth.globule import globule_complex
    top = max(sizes)
    levels = sorted(set(int(round(x)) for x in np.geomspace(200, top, 7)))
    levels[-1] = top
    pool = [globule_complex(n, seed + k) for k, n in enumerate(levels)]
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        k = next(k for k, m in enumerate(levels) if m >= n)
        x, r = pool[k]
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        out.append((np.ascontiguousarray(x[:n] @ q.T), np.ascontiguousarray(r[:n])))
    return out


def serving(args, precision):
    """Poisson stream of requests, batched server vs plain (one molecule per launch)."""
    from paper_2401_10462_amd.server import SasaServer, poisson_run
    rng = np.random.default_rng(4)
    nreq = args.serve_requests
    sizes = np.round(np.exp(rng.uniform(np.log(200), np.log(20000), size=nreq))).astype(int)
    reqs = pool_molecules(sizes)
    rates = [float(x) for x in args.rates.split(",")]
    res = {"requests_per_rate": nreq, "mean_atoms": float(sizes.mean()),
           "molecules": "first n atoms of 7 pooled structures (200 to 20,000 atoms; above 2,500 atoms complexes of "
                        "globules of up to 2,500 heavy atoms), randomly rotated",
           "rates": []}
    for rate in rates:
        row = {"rate_req_s": rate}
        for name, kw in (("batched", dict(slots=3, slot_budget_bytes=1 << 30)),
                         ("plain", dict(slots=1, max_requests_per_batch=1, slot_budget_bytes=1 << 30))):
            with SasaServer(precision=precision, **kw) as srv:
                srv.submit(*reqs[0]).result()  # warm-up
                st = poisson_run(srv, reqs, rate, seed=int(rate))
                st["batches"] = srv.batches - 1
            row[name] = st
            print(json.dumps({"serving_rate": rate, name: st}), file=sys.stderr, flush=True)
        res["rates"].append(row)
    return res


def md(args, precision):
    """Config: a globule, cumulative Gaussian moves, SASA + forces every frame, state on the device."""
    from paper_2401_10462_amd.md_loop import md_loop
    from synth.globule import globule_complex
    xyz, rad = globule_complex(args.md_atoms, 3)
    out = {"atoms": len(rad), "frames": args.frames, "gamma": 0.005, "sigma": 0.02,
           "structure": f"complex of {-(-len(rad) // 2500)} globules of up to 2,500 heavy atoms (seed 3)"}
    # md_loop's default (every cell clipped from scratch), then the same frames
    # in trajectory mode (each cell kept from the previous frame when it still
    # verifies, else clipped with the previous frame's facets first)
    from paper_2401_10462_amd import SasaContext
    for key, hints in (("cold", False), ("hinted", True)):
        md_loop(xyz, rad, frames=min(args.warmup, 5), precision=precision, frame_hints=hints)
        ctx = SasaContext(precision=precision, max_atoms=len(rad), frames=hints)
        lat, _ = md_loop(xyz, rad, frames=args.frames, precision=precision, ctx=ctx, frame_hints=hints)
        lat = np.array(lat)
        out[key] = {"frames_per_s": 1e3 / lat.mean(), "atoms_per_s": len(rad) * 1e3 / lat.mean(),
                    "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                    "cells_kept_last_frame": int(ctx.diagnostics()["reused_cells"])}
        ctx.close()
    return out


def local_moves(args, precision):
    """Config: the MD complex, each frame moving the atoms within 5 A of a random atom (a side-chain-like
    trial move), SASA + forces every frame; a cold context against an incremental one."""
    import torch
    from paper_2401_10462_amd import SasaContext
    from synth.globule import globule_complex
    xyz, rad = globule_complex(args.md_atoms, 3)
    n = len(rad)
    rng = np.random.default_rng(17)
    frames = args.frames
    # the moves are drawn up front (groups picked on the starting structure)
    moves = []
    for _ in range(frames + args.warmup):
        c = xyz[rng.integers(n)]
        sel = np.nonzero(np.linalg.norm(xyz - c, axis=1) < 5.0)[0]
        moves.append((sel, rng.normal(0.0, 0.3, size=(len(sel), 3))))
    dev = torch.device("cuda:0")
    R = torch.tensor(rad, device=dev)
    moves = [(torch.tensor(i, device=dev), torch.tensor(d, device=dev)) for i, d in moves]
    out = {"atoms": n, "frames": frames, "gamma": 0.005, "moved_per_frame": float(np.mean([len(i) for i, _ in moves])),
           "structure": f"complex of {-(-n // 2500)} globules of up to 2,500 heavy atoms (seed 3)",
           "move": "atoms within 5 A of a random atom, each displaced by N(0, 0.3^2) A per coordinate"}
    last = {}
    for key, inc in (("cold", False), ("incremental", True)):
        ctx = SasaContext(precision=precision, max_atoms=n, incremental=inc)
        X = torch.tensor(xyz, device=dev)
        for idx, d in moves[:args.warmup]:
            X.index_add_(0, idx, d)
            ctx.forces(X, R, 0.005, 1.4)
        torch.cuda.synchronize()
        lat, kept = [], []
        bufs = (torch.empty(n, dtype=torch.float64, device=dev), torch.empty((n, 3), dtype=torch.float64, device=dev))
        for idx, d in moves[args.warmup:]:
            t = time.perf_counter()
            X.index_add_(0, idx, d)
            a, f = ctx.forces(X, R, 0.005, 1.4, out=bufs)
            torch.cuda.synchronize()
            lat.append(1e3 * (time.perf_counter() - t))
            if inc and len(kept) < 20:
                kept.append(ctx.diagnostics()["skipped_atoms"] / n)
        lat = np.array(lat)
        out[key] = {"frames_per_s": 1e3 / lat.mean(), "p50_ms": float(np.percentile(lat, 50)),
                    "p99_ms": float(np.percentile(lat, 99))}
        if inc:
            out[key]["stars_kept"] = float(np.mean(kept))
        last[key] = (a.cpu().numpy(), f.cpu().numpy())
        ctx.close()
    # the same trajectory both ways: the last frame's results agree bit for bit
    out["last_frame_equal"] = bool(np.array_equal(last["cold"][0], last["incremental"][0])
                                   and np.array_equal(last["cold"][1], last["incremental"][1]))
    out["speedup"] = out["incremental"]["frames_per_s"] / out["cold"]["frames_per_s"]
    return out


def gbsa(args, precision):
    """Langevin steps (1 fs, 300 K) of the headline molecule, nonpolar forces through SASAFunction + bonds."""
    import torch
    from synth.globule import globule
    from paper_2401_10462_amd.gbsa_md import (NonpolarBondedModel, bonds_by_distance, langevin_baoab,
                                              masses_from_radii, thermal_velocities)
    xyz, rad = globule(args.heavy, args.seed, hydrogens=True)
    dev = torch.device("cuda:0")
    bonds, r0 = bonds_by_distance(xyz)
    m = masses_from_radii(rad).to(dev)
    g = torch.Generator().manual_seed(3)
    v0 = thermal_velocities(m.cpu(), 300.0, g).to(dev)
    model = NonpolarBondedModel(torch.tensor(rad, device=dev), bonds.to(dev), r0.to(dev), gamma=0.007,
                                precision=precision)
    x = torch.tensor(xyz, device=dev)
    x, v0, _ = langevin_baoab(model, x, v0, m, 1.0, max(args.warmup, 3), 300.0, 5.0, g)
    torch.cuda.synchronize()
    steps = max(args.steps, 10)
    t0 = time.perf_counter()
    _, _, tr = langevin_baoab(model, x, v0, m, 1.0, steps, 300.0, 5.0, g)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"atoms": len(rad), "steps": steps, "dt_fs": 1.0, "gamma": 0.007, "steps_per_s": steps / el,
            "ms_per_step": 1e3 * el / steps, "ns_per_day": steps / el * 86400 * 1e-6,
            "nonpolar_kcal_mol": tr[-1][2]}


def small(args):
    """One 300-heavy-atom globule, FP64, plain calls: atoms/s and p50/p99 latency."""
    import torch
    from paper_2401_10462_amd import SasaContext
    from synth.globule import heavy_chain
    xyz, rad, _ = heavy_chain(300, 1)
    dev = torch.device("cuda:0")
    X, R = torch.tensor(xyz, device=dev), torch.tensor(rad, device=dev)
    ctx = SasaContext(precision="fp64", max_atoms=len(rad))
    out = (torch.empty(len(rad), dtype=torch.float64, device=dev),
           torch.empty((len(rad), 3), dtype=torch.float64, device=dev))
    for _ in range(max(args.warmup, 3)):
        ctx.compute(X, R, 1.4, out=out)
    torch.cuda.synchronize()
    lat = []
    steps = max(args.steps, 100)
    t0 = time.perf_counter()
    for _ in range(steps):
        s = time.perf_counter()
        ctx.compute(X, R, 1.4, out=out)
        lat.append(time.perf_counter() - s)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    lat = np.array(lat) * 1e3
    return {"atoms": len(rad), "steps": steps, "atoms_per_s": len(rad) * steps / el, "ms_per_step": 1e3 * el / steps,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99))}


def autograd(args):
    """64 conformations of 2,000 atoms in one batch through SASAFunction: loss = sum w_i A_i, forward + backward."""
    import torch
    from paper_2401_10462_amd.autograd import sasa
    from synth.globule import heavy_chains, md_frames
    base = heavy_chains([(2000, 50_000 + m) for m in range(8)])
    mols = [(xf, r) for m, (x, r, _) in enumerate(base) for xf in md_frames(x, 500 + m, 8, sigma=0.02)]
    offs = np.cumsum([0] + [len(r) for _, r in mols]).astype(np.int64)
    dev = torch.device("cuda:0")
    X = torch.tensor(np.vstack([x for x, _ in mols]), device=dev)
    R = torch.tensor(np.concatenate([r for _, r in mols]), device=dev)
    w = torch.tensor(np.random.default_rng(5).uniform(-1, 1, len(R)), device=dev)

    def step():
        x = X.detach().requires_grad_(True)
        (w * sasa(x, R, 1.4, offsets=offs, precision=args.precision)).sum().backward()
        return x.grad

    for _ in range(max(args.warmup, 2)):
        step()
    torch.cuda.synchronize()
    steps = max(args.steps // 3, 5)
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        s = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s)
    el = time.perf_counter() - t0
    lat = np.array(lat) * 1e3
    return {"molecules": 64, "atoms": int(len(R)), "steps": steps, "atoms_per_s": len(R) * steps / el,
            "ms_per_step": 1e3 * el / steps, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99))}


def measured_traffic():
    """HBM bytes per k_star launch from the committed rocprofv3 counter runs, or
    None when kernels.hip has changed since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_star_traffic_globule5000H.json")  # k_star is precision-free
    src = os.path.join(ROOT, "paper_2401_10462_amd", "csrc", "kernels.hip")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    return rec["bytes_per_launch"] if rec.get("kernels_hip_sha256") == sha else None


def cpu_baseline(xyz, rad, budget, area=None, dadx=None, all_cores=True):
    """FP64 oracle on the host: whole molecule, repeated up to the time budget.

    The oracle is the plain brute-force reference of the tests (every candidate
    simplex of each atom's overlapping neighbours decided from its definition,
    O(n k^3), with dual-number Jacobians), built -O3 for x86-64-v3: a baseline
    of that code, not of a tuned CPU implementation of the method.  The timed
    leg also yields the oracle's result for this molecule, so the error of the
    GPU result just measured is reported beside it (per atom, relative to
    max(|ref|, 1 A^2) or max(|ref|, 1 A^2/A)).  The all-core leg runs one
    worker process per host core (at most 16, the host share of one GPU) on as
    many distinct conformations of the molecule (Gaussian moves, sigma 0.02 A):
    molecules are independent, so that is the fair multi-core form.
    """
    import oracle
    oracle.lib()
    t0 = time.perf_counter()
    runs = 0
    ref = None
    while True:
        ref = oracle.run(xyz, rad, 1.4)
        runs += 1
        el = time.perf_counter() - t0
        if el > budget or runs >= 8:
            break
    out = {"value": runs * len(rad) / el, "unit": "atoms/s", "cores": 1, "kind": "oracle",
           "sample": f"{runs} full run(s) of the {len(rad)}-atom molecule (SASA + dA/dx, FP64, one thread; "
                     "brute-force oracle)",
           "seconds": el, "host_cpus": os.cpu_count()}
    if area is not None:
        out["max_rel_err_area"] = float((np.abs(area - ref.area) / np.maximum(ref.area, 1.0)).max())
        gn = np.linalg.norm(ref.dadx, axis=1)
        out["max_rel_err_grad"] = float((np.linalg.norm(dadx - ref.dadx, axis=1) / np.maximum(gn, 1.0)).max())
    if all_cores:
        from synth.globule import md_frames
        P = max(1, min(16, os.cpu_count() or 1))
        confs = [(x, rad, 1.4) for x in md_frames(xyz, 77, P)]
        ta = time.perf_counter()
        oracle.run_many(confs, workers=P)
        ea = time.perf_counter() - ta
        out["all_cores"] = {"value": P * len(rad) / ea, "unit": "atoms/s", "cores": P, "seconds": ea,
                            "sample": f"{P} distinct conformations of the {len(rad)}-atom molecule, one worker "
                                      "process per core (process start included)"}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported (the method runs on a "
              "single device; see the sharding design notes).", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2401_10462_amd import SasaContext
    from synth.globule import globule

    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}))
        return
    if args.workload == "serving":
        print(json.dumps({"workload": "serving", "precision": args.precision, **serving(args, args.precision)}))
        return
    if args.workload == "small":
        print(json.dumps({"workload": "small", "precision": "fp64", **small(args)}))
        return
    if args.workload == "autograd":
        print(json.dumps({"workload": "autograd", "precision": args.precision, **autograd(args)}))
        return
    if args.workload == "gbsa":
        print(json.dumps({"workload": "gbsa", "precision": args.precision, **gbsa(args, args.precision)}))
        return
    if args.workload == "md":
        print(json.dumps({"workload": "md", "precision": args.precision, **md(args, args.precision)}))
        return
    if args.workload == "local":
        print(json.dumps({"workload": "local", "precision": args.precision, **local_moves(args, args.precision)}))
        return

    xyz, rad = globule(args.heavy, args.seed, hydrogens=True)
    n = len(rad)
    dev = torch.device("cuda:0")
    X = torch.tensor(xyz, device=dev)
    R = torch.tensor(rad, device=dev)
    # the headline and batched loops run without stage events (each event
    # between two kernels leaves the GPU idle for a few microseconds); a second
    # context with events times the stages for the roofline
    ctx = SasaContext(precision=args.precision, max_atoms=n * max(args.batch, 1))
    tctx = SasaContext(precision=args.precision, max_atoms=n, timing=True)

    # ---- plain form: one molecule per launch sequence (results into the same
    # device buffers every call, as a loop over frames or requests would)
    def f64(*shape):
        return torch.empty(shape, dtype=torch.float64, device=dev)

    outp = (f64(n), f64(n, 3))
    for _ in range(args.warmup):
        ctx.compute(X, R, 1.4, out=outp)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s = time.perf_counter()
        area, dadx = ctx.compute(X, R, 1.4, out=outp)
        lat.append(time.perf_counter() - s)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = n * args.steps / elapsed
    diag = ctx.diagnostics()

    # ---- stage times (HIP events on the library's stream) and work counters
    for _ in range(args.warmup):
        tctx.compute(X, R, 1.4)
    stage = {"cells": 0.0, "star": 0.0, "star_wide": 0.0, "terms": 0.0, "gather": 0.0}
    work = {"plane_tests": 0, "new_vertices": 0, "candidates": 0}
    for _ in range(args.steps):
        tctx.compute(X, R, 1.4)
        d = tctx.diagnostics()
        for k in stage:
            stage[k] += d["ms_" + k]
        for k in work:
            work[k] += d[k]
    tctx.close()

    # ---- the same molecule from host buffers (PCIe transfers inside each call)
    for _ in range(2):
        ctx.compute(xyz, rad, 1.4)
    th = time.perf_counter()
    kh = max(5, args.steps // 3)
    for _ in range(kh):
        ctx.compute(xyz, rad, 1.4)
    eh = time.perf_counter() - th
    host = {"atoms_per_s": n * kh / eh, "ms_per_call": 1e3 * eh / kh, "calls": kh}

    # ---- cell volumes and the molecular-volume gradient of the same molecule
    # (FP64: the areas are recomputed in FP64, then the faces)
    for _ in range(2):
        ctx.compute(X, R, 1.4)
        ctx.volume()
    kv = max(5, args.steps // 3)
    tv = 0.0
    for _ in range(kv):
        ctx.compute(X, R, 1.4)
        s = time.perf_counter()
        vol, _ = ctx.volume()
        tv += time.perf_counter() - s
    uv = torch.linspace(-1.0, 1.0, n, dtype=torch.float64, device=dev)
    ctx.volume_backward(uv)
    tb = 0.0
    for _ in range(kv):
        s = time.perf_counter()
        ctx.volume_backward(uv)
        tb += time.perf_counter() - s
    volume = {"ms_per_call": 1e3 * tv / kv, "atoms_per_s": n * kv / tv, "calls": kv,
              "volume_A3": float(vol.sum().item()), "vjp_ms_per_call": 1e3 * tb / kv}
    # ---- curvature measures of the same surface: per-atom integrated mean
    # curvature (FP64) and the Euler characteristic of the union
    ctx.compute(X, R, 1.4)
    ctx.curvature()
    tc = 0.0
    for _ in range(kv):
        s = time.perf_counter()
        cmean, chi = ctx.curvature()
        tc += time.perf_counter() - s
    curvature = {"ms_per_call": 1e3 * tc / kv, "calls": kv, "mean_curvature_A": float(cmean.sum().item()),
                 "euler_characteristic": chi, "gaussian_curvature": 4.0 * math.pi * chi}

    # ---- the paper's sorted extraction of the same complex (A/B against the
    # classification the star kernel does per atom): triangles, then also the
    # edges and vertices
    ctx.compute(X, R, 1.4)
    ctx.triangles_by_sort()
    sort_ms = [ctx.triangles_by_sort()[2] for _ in range(5)]
    ev = [ctx.edges_vertices_by_sort() for _ in range(3)]
    sorted_extraction = {"ms": float(np.median(sort_ms)), "triangles": int(ctx.counts()["triangles"]),
                         "with_edges_vertices_ms": float(np.median([r[4] for r in ev])),
                         "edges": int(len(ev[-1][0])), "vertices": int(len(ev[-1][2])),
                         "star_kernel_ms": stage["star"] / args.steps}

    # ---- dominant kernel roofline (VALU-bound FP64 clipping): k_star alone
    dom = max(stage, key=stage.get)
    star_s = stage["star"] / 1e3 / args.steps
    flops = (FLOP_PER_TEST * work["plane_tests"] + FLOP_PER_VERTEX * work["new_vertices"]
             + FLOP_PER_CANDIDATE * work["candidates"]) / args.steps
    achieved = flops / star_s / 1e12
    traffic = measured_traffic() if args.heavy == 2500 and args.seed == 2 else None
    roofline = {"kernel": "k_star", "dominant_stage": dom, "bound": "alu", "achieved": achieved,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                "traffic": traffic,
                "flop_per_launch": flops, "ms_per_launch": star_s * 1e3,
                "hbm_gbs": (traffic / star_s / 1e9) if traffic else None,
                "hbm_frac": (traffic / star_s / HBM_PEAK) if traffic else None,
                "stage_ms_per_step": {k: v / args.steps for k, v in stage.items()}}

    # ---- batched form: many molecules (rigid copies) in one launch sequence
    batched = None
    if args.batch > 0:
        rng = np.random.default_rng(7)
        mats = []
        for _ in range(args.batch):
            q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
            mats.append(xyz @ q.T + rng.normal(size=3) * 5)
        XB = torch.tensor(np.vstack(mats), device=dev)
        RB = torch.tensor(np.tile(rad, args.batch), device=dev)
        offs = np.arange(args.batch + 1, dtype=np.int64) * n
        outb = (f64(n * args.batch), f64(n * args.batch, 3))
        for _ in range(max(1, args.warmup)):
            ctx.compute_batch(offs, XB, RB, 1.4, out=outb)
        torch.cuda.synchronize()
        kb = max(3, args.steps // 4)
        tb = time.perf_counter()
        for _ in range(kb):
            ab, gb = ctx.compute_batch(offs, XB, RB, 1.4, out=outb)
        torch.cuda.synchronize()
        eb = time.perf_counter() - tb
        # the first molecule of the batch equals the plain result (rotated gradient aside)
        bd = ctx.diagnostics()
        batched = {"molecules": args.batch, "atoms": n * args.batch, "steps": kb,
                   "atoms_per_s": n * args.batch * kb / eb, "ms_per_step": 1e3 * eb / kb,
                   "speedup_vs_plain": (n * args.batch * kb / eb) / value,
                   "second_pass_atoms": bd["second_pass_atoms"], "exact_side_tests": bd["near_ties"]}

    # ---- the same plain loop in the other precision
    other = "fp64" if args.precision == "mixed" else "mixed"
    octx = SasaContext(precision=other, max_atoms=n)
    outo = (f64(n), f64(n, 3))  # (the plain loop's results stay in outp)
    for _ in range(args.warmup):
        octx.compute(X, R, 1.4, out=outo)
    torch.cuda.synchronize()
    to = time.perf_counter()
    for _ in range(args.steps):
        octx.compute(X, R, 1.4, out=outo)
    torch.cuda.synchronize()
    eo = time.perf_counter() - to
    other_precision = {"precision": other, "atoms_per_s": n * args.steps / eo, "ms_per_step": 1e3 * eo / args.steps}
    octx.close()

    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(xyz, rad, args.cpu_seconds, area.cpu().numpy(), dadx.cpu().numpy())

    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "atoms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-terms/f64-predicates" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"globule {args.heavy} heavy + {args.heavy} H atoms (seed {args.seed}), "
                               f"probe 1.4 A, {args.precision}, SASA + dA/dx", "atoms": n},
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "batched": batched,
        "other_precision": other_precision,
        "host_pointers": host,
        "volume": volume,
        "curvature": curvature,
        "sorted_extraction": sorted_extraction,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "gpu_over_cpu": (value / cpu["value"]) if cpu else None,
        "gpu_over_cpu_all_cores": (value / cpu["all_cores"]["value"]) if cpu and "all_cores" in cpu else None,
        "diagnostics": {k: diag[k] for k in ("max_neighbours", "max_cell_vertices", "near_ties", "lost_pairs",
                                             "overflow", "plane_tests", "new_vertices", "candidates",
                                             "planes_used", "max_planes_used", "atoms_over_64_planes",
                                             "second_pass_atoms")},
        "sasa_total": float(area.sum().item()),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
