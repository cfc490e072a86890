"""Error reporting and the on-demand counters, through the C-ABI.

A compute reports input errors and capacity failures from two words that its
terms kernel writes to pinned host memory; the size and work counts of the
star kernel are summed from its per-atom records only when diagnostics or the
complex counts ask for them.  These tests pin that bookkeeping: the counts are
summed once (asking twice gives the same numbers, in either order), an
asynchronous call's error surfaces through sasa_status, and an input error
that only the device sees (device buffers are not checked on the host) fails
the call.
"""
import numpy as np
import pytest

import oracle
from synth.globule import globule

pytestmark = pytest.mark.gpu


def _shell(n_shell, R_center, dist, seed=0):
    # one large atom ringed by n_shell small ones: its power cell has about
    # 2 n_shell vertices
    rng = np.random.default_rng(seed)
    k = np.arange(n_shell) + 0.5
    phi = np.arccos(1 - 2 * k / n_shell)
    th = np.pi * (1 + 5 ** 0.5) * k
    d = np.column_stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)])
    xyz = np.vstack([[0.0, 0.0, 0.0], dist * d + rng.normal(scale=0.05, size=d.shape)])
    rad = np.concatenate([[R_center], np.full(n_shell, 1.5)])
    return xyz, rad


def _dev(a):
    import torch
    return torch.tensor(a, dtype=torch.float64, device="cuda:0")


def test_counts_are_summed_once():
    from paper_2401_10462_amd import SasaContext
    xyz, rad = globule(150, 3, hydrogens=True)
    a = SasaContext(precision="fp64")
    b = SasaContext(precision="fp64")
    try:
        a.compute(xyz, rad, 1.4)
        b.compute(xyz, rad, 1.4)
        d1 = a.diagnostics()
        d2 = a.diagnostics()
        c_after = a.counts()
        c_first = b.counts()
        d_b = b.diagnostics()
        assert d1 == d2
        assert c_after == c_first
        for k in ("max_neighbours", "max_cell_vertices", "plane_tests", "new_vertices", "candidates",
                  "planes_used", "max_planes_used", "atoms_over_64_planes"):
            assert d1[k] == d_b[k], k
        assert d1["plane_tests"] > 0 and d1["new_vertices"] > 0 and d1["max_neighbours"] > 0
        # the counts agree with the exported complex
        e, t, nt, q, vf = a.export()
        assert (len(e), len(t), len(q)) == (c_after["edges"], c_after["triangles"], c_after["tetrahedra"])
        assert int((vf & 1).sum()) == c_after["vertices"]
        # a second compute of another molecule replaces them
        xyz2, rad2 = globule(60, 4)
        a.compute(xyz2, rad2, 1.4)
        ref = oracle.run(xyz2, rad2, 1.4)
        c2 = a.counts()
        assert (c2["edges"], c2["triangles"], c2["tetrahedra"], c2["atoms"]) == (
            len(ref.edges), len(ref.tris), len(ref.tets), len(rad2))
    finally:
        a.close()
        b.close()


def test_async_capacity_error_surfaces_in_status():
    from paper_2401_10462_amd import SasaContext, _lib
    ctx = SasaContext(precision="fp64", async_calls=True)
    try:
        xyz, rad = _shell(90, R_center=5.0, dist=6.0)
        ctx.compute(_dev(xyz), _dev(rad), 1.4)  # returns before the stream is done
        with pytest.raises(_lib.SasaError) as e:
            ctx.status()
        assert e.value.code == _lib.SASA_E_CAPACITY
        ctx.status()  # reported once
        # the context is usable again, and a good call reports no error
        xyz, rad = globule(80, 5)
        ref = oracle.run(xyz, rad, 1.4)
        area, dadx = ctx.compute(_dev(xyz), _dev(rad), 1.4)
        ctx.status()
        err = np.abs(area.cpu().numpy() - ref.area) / np.maximum(ref.area, 1.0)
        assert err.max() <= 1e-9
        assert ctx.diagnostics()["overflow"] == 0
    finally:
        ctx.close()


def test_device_side_input_error():
    from paper_2401_10462_amd import SasaContext, _lib
    ctx = SasaContext(precision="mixed")
    try:
        xyz, rad = globule(40, 6)
        y7 = xyz[7, 1]
        xyz[7, 1] = np.nan
        with pytest.raises(_lib.SasaError) as e:
            ctx.compute(_dev(xyz), _dev(rad), 1.4)
        assert e.value.code == _lib.SASA_E_INVAL
        assert ctx.diagnostics()["input_errors"] == 1
        rad[7] = -1.0
        xyz[7, 1] = y7
        with pytest.raises(_lib.SasaError) as e:
            ctx.compute(_dev(xyz), _dev(rad), 1.4)
        assert e.value.code == _lib.SASA_E_INVAL
        rad[7] = 1.7
        ref = oracle.run(xyz, rad, 1.4)
        area, _ = ctx.compute(_dev(xyz), _dev(rad), 1.4)
        err = np.abs(area.cpu().numpy() - ref.area) / np.maximum(ref.area, 1.0)
        assert err.max() <= 1e-4
    finally:
        ctx.close()
