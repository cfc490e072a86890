"""HIP path vs the FP64 oracle, element by element, through the C-ABI.

Bars (per atom i, Q17-style floors so that buried atoms are not divided by 0):
  FP64 : |A - A_ref| <= 1e-9 max(A_ref, 1 A^2);  |g - g_ref| <= 1e-9 max(|g_ref|, 1 A^2/A)
  MIXED: the same with 1e-4 (areas and gradients, the tolerance of the FP32 area terms)
  the dual complex K (edges, triangles, tetrahedra, n_tet, vertex flags) bit-exact.
"""
import numpy as np
import pytest

import oracle
from synth.globule import globule, heavy_chain, random_cluster

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "mixed": 1e-4}


@pytest.fixture(scope="module")
def ctxs():
    from paper_2401_10462_amd import SasaContext
    c = {"fp64": SasaContext(precision="fp64"), "mixed": SasaContext(precision="mixed")}
    yield c
    for v in c.values():
        v.close()


def _sets_gpu(ctx):
    e, t, nt, q, vf = ctx.export()
    E = set(map(tuple, e.tolist()))
    T = {tuple(x): int(k) for x, k in zip(t.tolist(), nt.tolist())}
    Q = set(map(tuple, q.tolist()))
    assert len(E) == len(e) and len(T) == len(t) and len(Q) == len(q), "duplicate simplices"
    # canonical order: ids ascending inside a tuple, tuples sorted
    for a in (e, t, q):
        if len(a):
            assert (np.diff(a, axis=1) > 0).all(), "ids not ascending inside a tuple"
            keys = [tuple(x) for x in a.tolist()]
            assert keys == sorted(keys), "tuples not in lexicographic order"
    return E, T, Q, vf


def _check_complex(ctx, ref):
    E, T, Q, vf = _sets_gpu(ctx)
    assert Q == set(map(tuple, ref.tets.tolist()))
    assert set(T) == set(map(tuple, ref.tris.tolist()))
    ref_nt = {tuple(x): int(k) for x, k in zip(ref.tris.tolist(), ref.tri_ntet.tolist())}
    assert T == ref_nt
    assert E == set(map(tuple, ref.edges.tolist()))
    assert np.array_equal(vf & 1, ref.vert_in)
    assert np.array_equal((vf >> 1) & 1, ref.vert_ext)


def _check_values(area, dadx, ref, tol):
    a_ref = ref.area
    err_a = np.abs(area - a_ref) / np.maximum(a_ref, 1.0)
    assert err_a.max() <= tol, f"area rel err {err_a.max():.3e} at atom {err_a.argmax()}"
    if dadx is not None:
        g_ref = ref.dadx
        err_g = np.linalg.norm(dadx - g_ref, axis=1) / np.maximum(np.linalg.norm(g_ref, axis=1), 1.0)
        assert err_g.max() <= tol, f"gradient rel err {err_g.max():.3e} at atom {err_g.argmax()}"


CASES = [
    ("tiny-12", lambda: random_cluster(12, 0)),
    ("cluster-40", lambda: random_cluster(40, 2)),
    ("cluster-80-wide-radii", lambda: random_cluster(80, 4, rmin=0.6, rmax=2.4)),
    ("globule-300", lambda: heavy_chain(300, 1)[:2]),
    ("globule-2000", lambda: heavy_chain(2000, 2)[:2]),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_parity_host_pointers(ctxs, name, make, prec):
    xyz, rad = make()
    ref = oracle.run(xyz, rad, 1.4)
    ctx = ctxs[prec]
    area, dadx = ctx.compute(xyz, rad, 1.4)
    _check_complex(ctx, ref)
    _check_values(area, dadx, ref, TOL[prec])
    d = ctx.diagnostics()
    assert d["overflow"] == 0 and d["lost_pairs"] == 0


def test_parity_hydrogens_5000(ctxs):
    # 2,500 heavy atoms + 2,500 hydrogens (hidden and partly buried small balls)
    xyz, rad = globule(2500, 2, hydrogens=True)
    ref = oracle.run(xyz, rad, 1.4)
    for prec in ("fp64", "mixed"):
        ctx = ctxs[prec]
        area, dadx = ctx.compute(xyz, rad, 1.4)
        _check_complex(ctx, ref)
        _check_values(area, dadx, ref, TOL[prec])


def test_device_pointers_and_vjp(ctxs):
    import torch
    xyz, rad, _ = heavy_chain(300, 1)
    ref = oracle.run(xyz, rad, 1.4)
    u = np.random.default_rng(5).uniform(-1, 1, len(rad))
    for prec in ("fp64", "mixed"):
        ctx = ctxs[prec]
        X = torch.tensor(xyz, device="cuda")
        R = torch.tensor(rad, device="cuda")
        area, dadx = ctx.compute(X, R, 1.4)
        torch.cuda.synchronize()
        _check_values(area.cpu().numpy(), dadx.cpu().numpy(), ref, TOL[prec])
        g = ctx.backward(torch.tensor(u, device="cuda")).cpu().numpy()
        g_ref = ref.vjp(u)
        err = np.linalg.norm(g - g_ref, axis=1) / np.maximum(np.linalg.norm(g_ref, axis=1), 1.0)
        assert err.max() <= TOL[prec]


def test_batch_equals_alone(ctxs):
    mols = [random_cluster(30, 50 + k) for k in range(3)] + [heavy_chain(300, 7)[:2], random_cluster(1, 9)]
    offs = np.cumsum([0] + [len(m[1]) for m in mols])
    X = np.vstack([m[0] for m in mols])
    R = np.concatenate([m[1] for m in mols])
    ctx = ctxs["fp64"]
    area_b, g_b = ctx.compute_batch(offs, X, R, 1.4)
    for k, (x, r) in enumerate(mols):
        a, g = ctx.compute(x, r, 1.4)
        s = slice(offs[k], offs[k + 1])
        assert np.array_equal(a, area_b[s])
        assert np.array_equal(g, g_b[s])


def test_deterministic_fp64(ctxs):
    xyz, rad, _ = heavy_chain(300, 3)
    ctx = ctxs["fp64"]
    a1, g1 = ctx.compute(xyz, rad, 1.4)
    a2, g2 = ctx.compute(xyz, rad, 1.4)
    assert np.array_equal(a1, a2) and np.array_equal(g1, g2)


def test_edge_cases(ctxs):
    from paper_2401_10462_amd import _lib
    ctx = ctxs["fp64"]
    a, g = ctx.compute(np.zeros((0, 3)), np.zeros(0), 1.4)
    assert a.shape == (0,)
    a, g = ctx.compute(np.array([[1.0, 2.0, 3.0]]), np.array([1.7]), 1.4)
    assert a[0] == pytest.approx(4 * np.pi * 3.1 ** 2, rel=1e-14) and np.all(g == 0)
    # nested and disjoint pairs, a hidden atom
    xyz = np.array([[0, 0, 0], [0.1, 0, 0], [20, 0, 0], [23, 0, 0]], float)
    rad = np.array([1.7, 0.5, 1.5, 1.7])
    ref = oracle.run(xyz, rad, 1.4)
    a, g = ctx.compute(xyz, rad, 1.4)
    _check_values(a, g, ref, 1e-9)
    assert a[1] == 0.0
    with pytest.raises(_lib.SasaError) as e:
        ctx.compute(np.array([[np.nan, 0, 0]]), np.array([1.7]), 1.4)
    assert e.value.code == _lib.SASA_E_INVAL
    with pytest.raises(_lib.SasaError) as e:
        ctx.compute(np.zeros((1, 3)), np.array([-1.0]), 1.4)
    assert e.value.code == _lib.SASA_E_INVAL
    from paper_2401_10462_amd import SasaContext
    fresh = SasaContext()
    with pytest.raises(_lib.SasaError) as e:
        fresh.backward(np.zeros(3))
    assert e.value.code == _lib.SASA_E_STATE
    fresh.close()


def _shell(n_shell, R_center=4.0, r_shell=1.5, dist=5.0, seed=0):
    """A large atom whose power cell has about 2 n_shell vertices: n_shell atoms
    on a Fibonacci shell around it (small jitter keeps general position)."""
    rng = np.random.default_rng(seed)
    k = np.arange(n_shell) + 0.5
    phi = np.arccos(1 - 2 * k / n_shell)
    th = np.pi * (1 + 5 ** 0.5) * k
    d = np.column_stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)])
    xyz = np.vstack([[0.0, 0.0, 0.0], dist * d + rng.normal(scale=0.05, size=d.shape)])
    rad = np.concatenate([[R_center], np.full(n_shell, r_shell)])
    return xyz, rad


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_large_cell_takes_the_wide_pass(ctxs, prec):
    # 48 shell atoms: the central cell has more than 64 vertices, beyond the
    # fast pass's capacity, and is computed by the wide pass
    xyz, rad = _shell(48)
    ref = oracle.run(xyz, rad, 1.4)
    ctx = ctxs[prec]
    area, dadx = ctx.compute(xyz, rad, 1.4)
    d = ctx.diagnostics()
    assert d["max_cell_vertices"] > 64 and d["overflow"] == 0
    _check_complex(ctx, ref)
    _check_values(area, dadx, ref, TOL[prec])


_LARGE_PROBE = {"600 heavy, probe 3.5": (600, False, 3.5), "400 heavy + H, probe 3.0": (400, True, 3.0)}
_large_probe_refs = {}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", list(_LARGE_PROBE))
def test_large_probe_beyond_neighbour_capacity(ctxs, case, prec):
    """Large probes on dense globules give atoms more overlapping neighbours than the kernels hold
    (up to 310 against 160): the second pass keeps the nearest planes and proves that the others
    lie beyond the cell.  Same complex and values as the oracle."""
    n, hyd, probe = _LARGE_PROBE[case]
    xyz, rad = globule(n, 2, hydrogens=hyd)
    print(f"large probe: {case} ({len(rad)} atoms) {prec}", flush=True)
    if case not in _large_probe_refs:
        _large_probe_refs[case] = oracle.run(xyz, rad, probe)
    ref = _large_probe_refs[case]
    ctx = ctxs[prec]
    area, dadx = ctx.compute(xyz, rad, probe)
    d = ctx.diagnostics()
    assert d["max_neighbours"] > 160 and d["overflow"] == 0 and d["second_pass_atoms"] > 0
    _check_complex(ctx, ref)
    _check_values(area, dadx, ref, TOL[prec])


def test_cell_beyond_every_capacity_is_an_error(ctxs):
    from paper_2401_10462_amd import _lib
    xyz, rad = _shell(90, R_center=5.0, dist=6.0)
    with pytest.raises(_lib.SasaError) as e:
        ctxs["fp64"].compute(xyz, rad, 1.4)
    assert e.value.code == _lib.SASA_E_CAPACITY


def test_reused_output_buffers(ctxs):
    """Results written into caller-given buffers, call after call, equal freshly allocated ones
    (device and host, compute, forces and batch); buffers of the wrong shape or type are refused."""
    import torch
    x, r = globule(300, 1)
    n = len(r)
    dev = torch.device("cuda:0")
    X, R = torch.tensor(x, device=dev), torch.tensor(r, device=dev)
    ctx = ctxs["fp64"]
    a0, g0 = ctx.compute(X, R, 1.4)
    f0 = ctx.forces(X, R, 0.005, 1.4)[1]
    out = (torch.empty(n, dtype=torch.float64, device=dev), torch.empty((n, 3), dtype=torch.float64, device=dev))
    for _ in range(3):
        a1, g1 = ctx.compute(X, R, 1.4, out=out)
        assert a1.data_ptr() == out[0].data_ptr() and g1.data_ptr() == out[1].data_ptr()
        assert torch.equal(a1, a0) and torch.equal(g1, g0)
        assert torch.equal(ctx.forces(X, R, 0.005, 1.4, out=out)[1], f0)
    a2, g2 = ctx.compute(X, R, 1.4, grad=False, out=(out[0], None))
    assert g2 is None and torch.equal(a2, a0)
    hout = (np.empty(n), np.empty((n, 3)))
    ha, hg = ctx.compute(x, r, 1.4, out=hout)
    assert ha is hout[0] and np.array_equal(ha, a0.cpu().numpy()) and np.array_equal(hg, g0.cpu().numpy())
    offs = np.array([0, n, 2 * n], dtype=np.int64)
    bout = (torch.empty(2 * n, dtype=torch.float64, device=dev), torch.empty((2 * n, 3), dtype=torch.float64, device=dev))
    X2 = X + 50.0  # (a translated copy rounds differently: compared with its own call alone)
    a3, g3 = ctx.compute(X2, R, 1.4)
    ab, gb = ctx.compute_batch(offs, torch.cat([X, X2]), torch.cat([R, R]), 1.4, out=bout)
    assert torch.equal(ab[:n], a0) and torch.equal(gb[:n], g0) and torch.equal(ab[n:], a3) and torch.equal(gb[n:], g3)
    for bad in ((out[0][:10], out[1]), (out[0].float(), out[1]), (out[0], None)):
        with pytest.raises(ValueError):
            ctx.compute(X, R, 1.4, out=bad)
    with pytest.raises(ValueError):  # host buffers for device inputs
        ctx.compute(X, R, 1.4, out=hout)


def test_stream_handle_is_torch_current_stream():
    """The binding hands the library torch's current stream (default and inside a stream context)."""
    import torch
    from paper_2401_10462_amd import _lib
    X = torch.zeros((4, 3), dtype=torch.float64, device="cuda:0")
    assert _lib.stream_of((X,)).value == (torch.cuda.current_stream().cuda_stream or None)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        assert _lib.stream_of((X,)).value == s.cuda_stream
    assert _lib.stream_of((np.zeros(3),)) is None
