"""Scheduling logic of the continuous-batching server, on the CPU.

The GPU slot is replaced by a fake slot that computes with the oracle and
finishes after a simulated service time, so admission by footprint, FIFO order,
overlap of slots and result routing are tested without a GPU.
"""
import time

import numpy as np

import oracle
from paper_2401_10462_amd import _lib
from paper_2401_10462_amd.server import SasaServer, latency_stats
from synth.globule import random_cluster


class FakeSlot:
    log = []

    def __init__(self, service_s=0.02):
        self.reqs = []
        self.service = service_s
        self.t_end = 0.0

    def launch(self, reqs):
        self.reqs = reqs
        self.t_end = time.perf_counter() + self.service
        FakeSlot.log.append([id(r) for r in reqs])

    def done(self):
        return time.perf_counter() >= self.t_end

    def finish(self):
        out = []
        for r in self.reqs:
            res = oracle.run(r.xyz, r.radii, 1.4)
            out.append((res.area, res.dadx))
        reqs, self.reqs = self.reqs, []
        return reqs, out

    def close(self):
        pass


def _mols(k, n=12):
    return [random_cluster(n, 300 + i) for i in range(k)]


def test_results_routed_and_batched():
    FakeSlot.log = []
    mols = _mols(24)
    srv = SasaServer(slots=2, slot_budget_bytes=_lib.sasa_footprint(12 * 5), slot_factory=lambda: FakeSlot(0.03))
    with srv:
        futs = [srv.submit(x, r) for x, r in mols]
        res = [f.result(timeout=30) for f in futs]
        assert len(srv.completed) == 24  # completion is recorded before results are delivered
    for (x, r), (a, g) in zip(mols, res):
        ref = oracle.run(x, r, 1.4)
        assert np.array_equal(a, ref.area) and np.array_equal(g, ref.dadx)
    sizes = [len(b) for b in FakeSlot.log]
    assert max(sizes) > 1            # queued requests were packed together
    assert max(sizes) <= 5           # footprint budget of 5 molecules respected
    order = [i for b in FakeSlot.log for i in b]
    assert len(order) == 24
    st = latency_stats(srv.completed)
    assert st["requests"] == 24 and st["p99_ms"] >= st["p50_ms"] > 0


def test_fifo_and_plain_mode():
    FakeSlot.log = []
    mols = _mols(6)
    srv = SasaServer(slots=1, max_requests_per_batch=1, slot_factory=lambda: FakeSlot(0.005))
    with srv:
        futs = [srv.submit(x, r) for x, r in mols]
        for f in futs:
            f.result(timeout=30)
    assert all(len(b) == 1 for b in FakeSlot.log)
    arrivals = [r.arrival for r in sorted(srv.completed, key=lambda r: r.t_admit)]
    assert arrivals == sorted(arrivals)


def test_oversized_request_runs_alone():
    FakeSlot.log = []
    big = random_cluster(40, 7)
    small = _mols(3)
    srv = SasaServer(slots=1, slot_budget_bytes=_lib.sasa_footprint(20), slot_factory=lambda: FakeSlot(0.005))
    with srv:
        futs = [srv.submit(*big)] + [srv.submit(x, r) for x, r in small]
        for f in futs:
            f.result(timeout=30)
    assert [len(b) for b in FakeSlot.log][0] == 1


class PoisonSlot(FakeSlot):
    """A fake slot whose batch fails as the library would (SASA_E_INVAL from the
    finished call) when it holds a request with the marker radius 9.99, and
    whose launch fails (out of device memory) for the marker radius 8.88."""

    def launch(self, reqs):
        if any(np.any(r.radii == 8.88) for r in reqs):
            raise _lib.SasaError(_lib.SASA_E_NOMEM, "no device memory for this batch")
        super().launch(reqs)

    def finish(self):
        if any(np.any(r.radii == 9.99) for r in self.reqs):
            raise _lib.SasaError(_lib.SASA_E_INVAL, "bad input in this batch")
        return super().finish()


def test_bad_requests_fail_alone():
    mols = _mols(12)
    bad_finish = (mols[3][0], np.where(np.arange(12) == 0, 9.99, mols[3][1]))
    bad_launch = (mols[7][0], np.where(np.arange(12) == 0, 8.88, mols[7][1]))
    reqs = mols[:3] + [bad_finish] + mols[4:7] + [bad_launch] + mols[8:]
    srv = SasaServer(slots=2, slot_budget_bytes=_lib.sasa_footprint(12 * 6), slot_factory=lambda: PoisonSlot(0.01))
    with srv:
        futs = [srv.submit(x, r) for x, r in reqs]
        for k, f in enumerate(futs):
            if k in (3, 7):
                err = f.exception(timeout=30)
                assert isinstance(err, _lib.SasaError)
                assert err.code == (_lib.SASA_E_INVAL if k == 3 else _lib.SASA_E_NOMEM)
            else:
                a, g = f.result(timeout=30)
                ref = oracle.run(*reqs[k], 1.4)
                assert np.array_equal(a, ref.area)
    assert len(srv.errors) == 2


def test_invalid_request_refused_at_submit():
    x, r = _mols(1)[0]
    srv = SasaServer(slots=1, slot_factory=lambda: FakeSlot(0.0))
    for bad in (np.where(np.arange(len(r))[:, None] == 0, np.nan, x), ):
        try:
            srv.submit(bad, r)
        except ValueError:
            pass
        else:
            raise AssertionError("NaN coordinate accepted")
    for rr in (np.where(np.arange(len(r)) == 1, 0.0, r), np.where(np.arange(len(r)) == 1, -1.0, r)):
        try:
            srv.submit(x, rr)
        except ValueError:
            pass
        else:
            raise AssertionError("radius <= 0 accepted")
    srv.stop(drain=False)


def test_scheduler_failure_resolves_every_future():
    class BrokenSlot(FakeSlot):
        def done(self):
            raise RuntimeError("slot failure")

    srv = SasaServer(slots=1, slot_factory=lambda: BrokenSlot(0.0))
    srv.start()
    futs = [srv.submit(x, r) for x, r in _mols(4)]
    for f in futs:
        assert isinstance(f.exception(timeout=10), RuntimeError)
    srv.stop(drain=True)  # returns: the scheduler is gone
