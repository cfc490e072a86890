"""A device allocation that fails part-way through growing a context's buffers
(injected: SASA_TEST_FAIL_ALLOC=k fails the k-th allocation) is reported as
SASA_E_NOMEM, and the context stays usable: the next call regrows the whole
group instead of writing through a buffer that was freed and not replaced."""
import numpy as np
import pytest

import oracle
from synth.globule import random_cluster

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fail_at", [1, 5, 12, 23, 25])
def test_failed_grow_leaves_a_usable_context(monkeypatch, fail_at):
    from paper_2401_10462_amd import SasaContext, _lib
    xyz, rad = random_cluster(60, 8)
    ref = oracle.run(xyz, rad, 1.4)
    ctx = SasaContext(precision="fp64")
    try:
        small = random_cluster(20, 9)
        ctx.compute(*small, 1.4)  # buffers for 20 atoms exist
        monkeypatch.setenv("SASA_TEST_FAIL_ALLOC", str(fail_at))
        with pytest.raises(_lib.SasaError) as e:
            ctx.compute(xyz, rad, 1.4)  # grows: one allocation fails
        assert e.value.code == _lib.SASA_E_NOMEM
        monkeypatch.delenv("SASA_TEST_FAIL_ALLOC")
        # a smaller call than the failed one, then the failed size again
        a, g = ctx.compute(*small, 1.4)
        r2 = oracle.run(*small, 1.4)
        assert np.abs(a - r2.area).max() <= 1e-9 * max(r2.area.max(), 1.0)
        a, g = ctx.compute(xyz, rad, 1.4)
        assert np.abs(a - ref.area).max() <= 1e-9 * max(ref.area.max(), 1.0)
        assert np.abs(g - ref.dadx).max() <= 1e-9 * max(np.abs(ref.dadx).max(), 1.0)
    finally:
        ctx.close()
