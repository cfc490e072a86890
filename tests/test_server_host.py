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
