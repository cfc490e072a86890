"""The one-block cell list against the multi-kernel one, at the sizes where the one-block kernel changes shape.

A single molecule of at most 8,192 atoms takes the one-block cell list, whose thread count and atoms per thread
depend on n (256 threads up to 512 atoms, then 1,024 threads with 1, 2, 5 or 8 atoms each); a batch always takes
the multi-kernel cell list.  The same molecule computed alone and as the first molecule of a batch (with a far
copy of its first atoms as the second) must give bitwise the same areas and gradients, at every size on either
side of each switch.  Both sides are independent of the oracle, which the parity tests cover at these shapes.
"""
import numpy as np
import pytest

from synth.globule import random_cluster

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 64, 255, 256, 511, 512, 513, 1023, 1024, 1025, 2047, 2048, 2049, 5119, 5120, 5121, 8191, 8192]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_one_block_equals_multi_kernel(prec):
    from paper_2401_10462_amd import SasaContext
    ctx = SasaContext(precision=prec, max_atoms=8192 + 8)
    for n in SIZES:
        x, r = random_cluster(n, 100 + n)
        m = min(n, 3)
        xb = np.vstack([x, x[:m] + 1000.0])
        rb = np.concatenate([r, r[:m]])
        offs = np.array([0, n, n + m], dtype=np.int64)
        print(f"cell list sizes {prec}: n = {n}", flush=True)
        a1, g1 = ctx.compute(x, r, 1.4)
        a2, g2 = ctx.compute_batch(offs, xb, rb, 1.4)
        assert np.array_equal(a1, a2[:n]), f"areas differ at n = {n}"
        assert np.array_equal(g1, g2[:n]), f"gradients differ at n = {n}"
        assert np.all(np.isfinite(a1)) and np.all(np.isfinite(g1))
    ctx.close()


@pytest.mark.parametrize("n,box", [(5000, 400.0), (8192, 500.0)])
def test_one_block_sparse_grid_counts_in_global_memory(n, box):
    """A sparse molecule whose grid has more cells than the one-block kernel keeps in LDS (32,768): the cell counts
    and cursors then live in global memory; still bitwise the multi-kernel result."""
    from paper_2401_10462_amd import SasaContext
    x, r = random_cluster(n, 7, box=box)
    xb = np.vstack([x, x[:3] + 5000.0])
    rb = np.concatenate([r, r[:3]])
    offs = np.array([0, n, n + 3], dtype=np.int64)
    # the grid rule (cell side R_max, enlarged by 1.25 until at most 8 n + 8 cells) gives more than 32,768 cells here
    ext, s = x.max(axis=0) - x.min(axis=0), r.max() + 1.4
    while np.prod(np.floor(ext / s) + 1) > 8 * n + 8:
        s *= 1.25
    assert np.prod(np.floor(ext / s) + 1) > 32768
    ctx = SasaContext(precision="fp64", max_atoms=n + 3)
    print(f"sparse cell list: n = {n}, box {box} A", flush=True)
    a1, g1 = ctx.compute(x, r, 1.4)
    a2, g2 = ctx.compute_batch(offs, xb, rb, 1.4)
    assert np.array_equal(a1, a2[:n]) and np.array_equal(g1, g2[:n])
    ctx.close()
