"""Seeded synthetic molecules: compact self-avoiding chains folded into globules.

This module only draws inputs (coordinates and radii); it holds none of the
surface-area arithmetic and is shared by the tests, the oracle runs and the
benchmark.  The paper's own structures (proteins of 10-190 residues, RNAs) are
not available, so these globules stand in for them with protein-like
heavy-atom density and the paper's element radii (Methods, dSASA: C 1.7,
O 1.5 -- 1.52 here --, N 1.55, S 1.8 A; probe 1.4 A).

Recipe (all randomness from numpy PCG64 seeded by ``seed``):
  1. elements i.i.d. C/N/O/S with p = .62/.17/.19/.02;
  2. grow a self-avoiding walk inside a sphere of density 0.025 atoms/A^3:
     steps U(1.45, 1.55) A in uniform directions, rejecting positions closer
     than 3.0 A to any atom three or more bonds away or 2.2 A to atom i-2;
  3. shrink the confining sphere to density 0.058 atoms/A^3 in stages, each
     followed by projection sweeps that restore the wall, the 3.0 A and 2.2 A
     exclusions and the bond-length window;
  4. optionally add one hydrogen (r = 1.20 A) per heavy atom, U(1.0, 1.1) A
     from a uniformly chosen heavy parent, at least 1.5 A from every other atom.
"""
import math

import numpy as np
from scipy.spatial import cKDTree

ELEMENTS = ("C", "N", "O", "S")
RADII = {"C": 1.70, "N": 1.55, "O": 1.52, "S": 1.80, "H": 1.20}
PROBS = (0.62, 0.17, 0.19, 0.02)
PROBE = 1.4

BOND_MIN, BOND_MAX = 1.45, 1.55
NONBONDED_MIN = 3.0
ONE_THREE_MIN = 2.2
GROW_DENSITY = 0.025
TARGET_DENSITY = 0.058


def _unit(rng, k):
    v = rng.normal(size=(k, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


class _Grid:
    """Uniform hash grid for the growth phase (cell side = exclusion radius)."""

    def __init__(self, h):
        self.h = h
        self.cells = {}

    def key(self, p):
        return (int(math.floor(p[0] / self.h)), int(math.floor(p[1] / self.h)), int(math.floor(p[2] / self.h)))

    def add(self, idx, p):
        self.cells.setdefault(self.key(p), []).append(idx)

    def remove(self, idx, p):
        self.cells[self.key(p)].remove(idx)

    def near(self, p):
        cx, cy, cz = self.key(p)
        out = []
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    out.extend(self.cells.get((cx + dx, cy + dy, cz + dz), ()))
        return out


def _grow(n, rng, radius):
    """Self-avoiding walk of n atoms inside a sphere, with backtracking.

    Dead ends are left by backtracking; the depth grows with the number of
    consecutive failures, and a walk that makes no new progress for 20,000
    attempts retreats 32, 64, ... 1024 atoms, so that a jammed region is always
    escaped.
    """
    pos = np.zeros((n, 3))
    grid = _Grid(NONBONDED_MIN)
    pos[0] = _unit(rng, 1)[0] * rng.uniform(0, 0.3 * radius)
    grid.add(0, pos[0])
    i = 1
    stuck = 0
    best, since_best, escape = 1, 0, 0
    while i < n:
        if i > best:
            best, since_best = i, 0
        since_best += 1
        if since_best > 20000:
            # a pocket the short backtracks keep regrowing into: retreat further
            # each time (never taken while the chain keeps making progress)
            escape += 1
            since_best = 0
            for _ in range(min(i - 1, 16 << min(escape, 6))):
                i -= 1
                grid.remove(i, pos[i])
            best = i
        k = 32
        steps = rng.uniform(BOND_MIN, BOND_MAX, size=k)[:, None] * _unit(rng, k)
        cand = pos[i - 1] + steps
        ok = np.einsum("ij,ij->i", cand, cand) <= radius * radius
        near = [j for j in grid.near(pos[i - 1]) if j <= i - 3]
        if near:
            d2 = ((cand[:, None, :] - pos[near][None, :, :]) ** 2).sum(-1)
            ok &= (d2 >= NONBONDED_MIN ** 2).all(axis=1)
        if i >= 2:
            ok &= ((cand - pos[i - 2]) ** 2).sum(-1) >= ONE_THREE_MIN ** 2
        hit = np.flatnonzero(ok)
        if hit.size:
            pos[i] = cand[hit[0]]
            grid.add(i, pos[i])
            i += 1
            stuck = max(0, stuck - 1)
            continue
        stuck += 1
        if stuck % 4 == 0 and i > 1:
            back = min(i - 1, 1 + stuck // 4 + int(rng.integers(0, 3)))
            for _ in range(back):
                i -= 1
                grid.remove(i, pos[i])
    return pos


def _sweeps(pos, wall, k, slack=0.0):
    """Jacobi projection sweeps: exclusions, bond window, then the wall."""
    n = len(pos)
    for _ in range(k):
        delta = np.zeros_like(pos)
        cnt = np.zeros(n)
        pairs = cKDTree(pos).query_pairs(NONBONDED_MIN + slack, output_type="ndarray")
        if len(pairs):
            a, b = pairs[:, 0], pairs[:, 1]
            sep = np.abs(a - b)
            lim = np.where(sep >= 3, NONBONDED_MIN + slack, np.where(sep == 2, ONE_THREE_MIN + slack, 0.0))
            d = pos[b] - pos[a]
            dist = np.linalg.norm(d, axis=1)
            bad = dist < lim
            if bad.any():
                a, b, d, dist, lim = a[bad], b[bad], d[bad], dist[bad], lim[bad]
                corr = (0.5 * (lim - dist) / np.maximum(dist, 1e-9))[:, None] * d
                np.add.at(delta, a, -corr)
                np.add.at(delta, b, corr)
                np.add.at(cnt, a, 1)
                np.add.at(cnt, b, 1)
        d = pos[1:] - pos[:-1]
        dist = np.linalg.norm(d, axis=1)
        tgt = np.clip(dist, BOND_MIN + 0.002, BOND_MAX - 0.002)
        corr = (0.5 * (dist - tgt) / dist)[:, None] * d
        delta[:-1] += corr
        delta[1:] -= corr
        cnt[:-1] += 1
        cnt[1:] += 1
        pos += delta / np.maximum(cnt, 1)[:, None] * 1.6
        r = np.linalg.norm(pos, axis=1)
        out = r > wall
        pos[out] *= (wall / r[out])[:, None]
    return pos


def _violations(pos):
    n = len(pos)
    bonds = np.linalg.norm(pos[1:] - pos[:-1], axis=1)
    pairs = cKDTree(pos).query_pairs(NONBONDED_MIN, output_type="ndarray")
    worst = NONBONDED_MIN
    worst13 = ONE_THREE_MIN
    if len(pairs):
        sep = np.abs(pairs[:, 0] - pairs[:, 1])
        dist = np.linalg.norm(pos[pairs[:, 1]] - pos[pairs[:, 0]], axis=1)
        if (sep >= 3).any():
            worst = min(worst, dist[sep >= 3].min())
        if (sep == 2).any():
            worst13 = min(worst13, dist[sep == 2].min())
    return bonds.min() if n > 1 else BOND_MIN, bonds.max() if n > 1 else BOND_MAX, worst, worst13


def heavy_chain(n, seed):
    """Heavy-atom globule of n atoms: (xyz (n,3) float64, radii (n,), elements)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    elem = rng.choice(4, size=n, p=PROBS)
    radii = np.array([RADII[ELEMENTS[e]] for e in elem])
    r_grow = (3 * n / (4 * math.pi * GROW_DENSITY)) ** (1 / 3)
    r_tgt = (3 * n / (4 * math.pi * TARGET_DENSITY)) ** (1 / 3)
    pos = _grow(n, rng, r_grow)
    stages = 40
    for s in range(1, stages + 1):
        wall = r_grow + (r_tgt - r_grow) * s / stages
        pos = _sweeps(pos, wall, 8, slack=0.05)
    # polish until the exclusions and bond window hold
    for _ in range(400):
        bmin, bmax, nb, n13 = _violations(pos)
        if bmin >= BOND_MIN - 5e-3 and bmax <= BOND_MAX + 5e-3 and nb >= NONBONDED_MIN - 1e-2 and n13 >= ONE_THREE_MIN - 1e-2:
            break
        pos = _sweeps(pos, r_tgt, 4, slack=0.02)
    pos -= pos.mean(axis=0)
    # a random rigid rotation so that no structure aligns with the axes
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    pos = pos @ q.T
    return np.ascontiguousarray(pos), radii, [ELEMENTS[e] for e in elem]


def add_hydrogens(xyz, radii, elements, seed):
    """One hydrogen per heavy atom at U(1.0, 1.1) A from a random heavy parent.

    Up to 100 directions are tried per hydrogen; the first one at least 1.5 A
    from every atom other than the parent (hydrogens placed so far included)
    is kept, else the last one.
    """
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    n = len(xyz)
    tree = cKDTree(xyz)
    grid = _Grid(1.5)
    hs = np.zeros((n, 3))
    for k in range(n):
        parent = int(rng.integers(0, n))
        d = rng.uniform(1.0, 1.1, size=100)
        cand = xyz[parent] + d[:, None] * _unit(rng, 100)
        near = tree.query_ball_point(cand, 1.5)
        pick = 99
        for t in range(100):
            if any(j != parent for j in near[t]):
                continue
            hn = grid.near(cand[t])
            if hn and (np.linalg.norm(hs[hn] - cand[t], axis=1) < 1.5).any():
                continue
            pick = t
            break
        hs[k] = cand[pick]
        grid.add(k, hs[k])
    xyz2 = np.vstack([xyz, hs])
    radii2 = np.concatenate([radii, np.full(n, RADII["H"])])
    return np.ascontiguousarray(xyz2), radii2, list(elements) + ["H"] * n


def globule(n_heavy, seed, hydrogens=False):
    """G(N_heavy, seed, H): coordinates (A) and van der Waals radii (A)."""
    xyz, radii, elem = heavy_chain(n_heavy, seed)
    if hydrogens:
        xyz, radii, elem = add_hydrogens(xyz, radii, elem, seed)
    return xyz, radii


def random_cluster(n, seed, box=None, rmin=1.5, rmax=1.8):
    """Small random cluster in general position (uniform centres in a cube)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if box is None:
        box = 2.2 * n ** (1 / 3) + 2.0
    xyz = rng.uniform(0, box, size=(n, 3))
    radii = rng.uniform(rmin, rmax, size=n)
    return xyz, radii


def md_frames(xyz, seed, frames, sigma=0.02):
    """Yield cumulative Gaussian-noise frames (sigma A per component per frame)."""
    cur = xyz.copy()
    for f in range(frames):
        rng = np.random.Generator(np.random.PCG64([seed, f]))
        cur = cur + rng.normal(scale=sigma, size=cur.shape)
        yield cur


def _chain(args):
    return heavy_chain(*args)


def heavy_chains(jobs, workers=8):
    """heavy_chain(n, seed) for every (n, seed) in ``jobs``, drawn in up to
    ``workers`` spawned processes (the results do not depend on the count)."""
    jobs = list(jobs)
    if len(jobs) > 1 and workers > 1:
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=min(workers, len(jobs)), mp_context=mp.get_context("spawn")) as ex:
            return list(ex.map(_chain, jobs))
    return [_chain(j) for j in jobs]


def globule_complex(n_total, seed, chain_atoms=2500, workers=8):
    """A complex of compact globules (one chain each, recipe above).

    Large molecules are built this way because the compression step of a single
    chain stops reaching the target density with all exclusions above a few
    thousand atoms.  ceil(n_total / chain_atoms) chains are placed along
    Fibonacci-sphere directions, each moved out until it is at least 3.0 A from
    every chain placed before it.  The chains are drawn in up to ``workers``
    fresh (spawned) processes; each has its own seed, so the result does not
    depend on the worker count.
    """
    chains = max(1, -(-n_total // chain_atoms))
    sizes = [n_total // chains + (1 if k < n_total % chains else 0) for k in range(chains)]
    parts = heavy_chains([(n, seed * 101 + k) for k, n in enumerate(sizes)], workers)
    k = np.arange(chains) + 0.5
    phi = np.arccos(1 - 2 * k / chains)
    theta = np.pi * (1 + 5 ** 0.5) * k
    dirs = np.column_stack([np.cos(theta) * np.sin(phi), np.sin(theta) * np.sin(phi), np.cos(phi)])
    placed = []
    for c, (x, r, e) in enumerate(parts):
        rad = np.linalg.norm(x, axis=1).max()
        shift = 0.0 if chains == 1 else rad
        while True:
            y = x + dirs[c] * shift
            if not placed:
                break
            d, _ = cKDTree(np.vstack([p for p, _ in placed])).query(y)
            if d.min() >= NONBONDED_MIN:
                break
            shift += 1.0
        placed.append((y, r))
    xyz = np.vstack([p for p, _ in placed])
    radii = np.concatenate([r for _, r in placed])
    xyz -= xyz.mean(axis=0)
    return np.ascontiguousarray(xyz), radii
