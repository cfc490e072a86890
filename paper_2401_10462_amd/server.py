"""Continuous-batching SASA + gradient server on one GPU.

Requests (one molecule each: coordinates, radii) are queued as they arrive.  A
scheduler thread owns ``slots`` library contexts, each with its own HIP stream
and device buffers.  Whenever a slot is free it admits queued requests in
arrival order while their summed device footprint (``sasa_footprint``) stays
within the slot's HBM budget, packs them into one batch (one segment per
molecule, so no atom of one request ever sees another's), and launches the
whole path asynchronously on the slot's stream.  Slots overlap on the device;
a finished slot's results are split back per request and the slot admits the
next requests right away, so requests that arrive while others run are
served as soon as a slot and memory free up.

``SasaServer(..., slots=1, max_requests_per_batch=1)`` is the plain form: one
molecule per launch sequence, first in first out.
"""
import collections
import gc
import queue
import threading
import time
from concurrent.futures import Future

import numpy as np
import torch

from . import _lib
from .context import SasaContext


class Request:
    __slots__ = ("xyz", "radii", "future", "arrival", "t_admit", "t_done", "n", "solo")

    def __init__(self, xyz, radii, arrival):
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        self.radii = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
        if self.xyz.shape[0] != self.radii.shape[0]:
            raise ValueError("xyz and radii disagree on the atom count")
        # checked here so that a bad request is refused alone, before it can
        # share a batch with others
        if not np.all(np.isfinite(self.xyz)):
            raise ValueError("non-finite coordinate")
        if not np.all(np.isfinite(self.radii) & (self.radii > 0)):
            raise ValueError("radii must be finite and > 0")
        self.n = self.radii.shape[0]
        self.solo = False  # set when a batch that held it failed: it then runs alone
        self.future = Future()
        self.arrival = arrival
        self.t_admit = None
        self.t_done = None


class _Slot:
    def __init__(self, device, precision, max_atoms, probe):
        self.ctx = SasaContext(device=device, precision=precision, max_atoms=max_atoms, async_calls=True)
        self.stream = torch.cuda.Stream(device=device)  # default priority
        self.event = torch.cuda.Event()
        self.reqs = []
        self.probe = probe
        self.device = device
        self.host_out = None
        self.area = None
        self.grad = None
        # pinned staging for a full slot, allocated once (a pinned allocation
        # of a new size can stall the device for milliseconds); a batch reuses
        # it only after the previous one has been finished
        self.cap = max(int(max_atoms), 1)
        self._pin = self._pinned(self.cap)
        # device result buffers for a full slot (a batch fills a prefix)
        self._dev = (torch.empty(self.cap, dtype=torch.float64, device=device),
                     torch.empty((self.cap, 3), dtype=torch.float64, device=device))

    @staticmethod
    def _pinned(n):
        return {"xyz": torch.empty((n, 3), dtype=torch.float64, pin_memory=True),
                "rad": torch.empty(n, dtype=torch.float64, pin_memory=True),
                "area": torch.empty(n, dtype=torch.float64, pin_memory=True),
                "grad": torch.empty((n, 3), dtype=torch.float64, pin_memory=True)}

    def launch(self, reqs):
        self.reqs = reqs
        n = sum(r.n for r in reqs)
        offs = np.zeros(len(reqs) + 1, np.int64)
        offs[1:] = np.cumsum([r.n for r in reqs])
        pin = self._pin if n <= self.cap else self._pinned(n)  # (a request above the budget, run alone)
        xyz, rad = pin["xyz"][:n], pin["rad"][:n]
        np.concatenate([r.xyz for r in reqs], out=xyz.numpy())
        np.concatenate([r.radii for r in reqs], out=rad.numpy())
        with torch.cuda.stream(self.stream):
            X = xyz.to(self.device, non_blocking=True)
            R = rad.to(self.device, non_blocking=True)
            out = (self._dev[0][:n], self._dev[1][:n]) if n <= self.cap else None
            area, grad = self.ctx.compute_batch(offs, X, R, self.probe, grad=True, out=out)
            self.host_out = (pin["area"][:n], pin["grad"][:n])
            self.host_out[0].copy_(area, non_blocking=True)
            self.host_out[1].copy_(grad, non_blocking=True)
            self.event.record(self.stream)
        # keep the staging alive until the event completes
        self._keep = (pin, X, R, area, grad, offs)

    def done(self):
        return self.event.query()

    def close(self):
        self.ctx.close()

    def finish(self):
        self.event.synchronize()
        self.ctx.status()  # raises on capacity / input errors of this batch
        a, g = self.host_out[0].numpy(), self.host_out[1].numpy()
        out, o = [], 0
        for r in self.reqs:
            out.append((a[o:o + r.n].copy(), g[o:o + r.n].copy()))
            o += r.n
        reqs, self.reqs, self._keep = self.reqs, [], None
        return reqs, out


class SasaServer:
    """Continuous batching over ``slots`` concurrent streams.

    slot_budget_bytes: HBM footprint one slot may use (admission limit); a
    request larger than the budget is run alone.
    freeze_gc: move the objects that exist when the server starts out of the
    garbage collector's reach (``gc.freeze``).  A full collection walks every
    tracked object of the process (a few hundred thousand once torch is
    imported) and, holding the interpreter lock, stalls the scheduler thread for
    about 70 ms: the one-in-a-hundred latencies of a stream.  Objects frozen
    here are never collected, so a process that creates and drops many servers
    may prefer to leave it off.
    """

    def __init__(self, device=0, precision="mixed", slots=3, slot_budget_bytes=2 << 30, probe=1.4,
                 max_requests_per_batch=None, slot_factory=None, freeze_gc=True):
        if freeze_gc:
            gc.collect()
            gc.freeze()
        self.device = device
        self.budget = slot_budget_bytes
        self.max_req = max_requests_per_batch
        per_atom = _lib.sasa_footprint(1_000_000) / 1_000_000
        self.max_atoms = int(slot_budget_bytes / per_atom)
        make = slot_factory or (lambda: _Slot(device, precision, self.max_atoms, probe))
        self._slots = [make() for _ in range(slots)]
        self._cuda = slot_factory is None
        self._q = collections.deque()
        self._inbox = queue.SimpleQueue()
        self._stop = threading.Event()
        self._wake = threading.Event()
        self._thread = None
        self.completed = []
        self.errors = []
        self.batches = 0

    # ---------------------------------------------------------------- API
    def submit(self, xyz, radii, arrival=None):
        r = Request(xyz, radii, time.perf_counter() if arrival is None else arrival)
        self._inbox.put(r)
        self._wake.set()
        return r.future

    def start(self):
        self._thread = threading.Thread(target=self._loop, name="sasa-server", daemon=True)
        self._thread.start()
        return self

    def stop(self, drain=True):
        if drain:
            while not (self._inbox.empty() and not self._q and all(not s.reqs for s in self._slots)):
                if self._thread is None or not self._thread.is_alive():
                    break
                time.sleep(1e-3)
        self._stop.set()
        self._wake.set()
        if self._thread:
            self._thread.join()
        for s in self._slots:
            s.close()

    def __enter__(self):
        return self.start()

    def __exit__(self, *exc):
        self.stop(drain=exc[0] is None)

    # ----------------------------------------------------------- scheduler
    def _admit(self):
        """Requests for one batch: FIFO while the footprint fits the slot budget
        (a request whose batch failed before runs alone)."""
        batch, atoms = [], 0
        while self._q:
            r = self._q[0]
            if r.solo or (batch and batch[0].solo):
                if not batch:
                    batch.append(self._q.popleft())
                break
            need = _lib.sasa_footprint(atoms + r.n)
            if batch and (need > self.budget or (self.max_req and len(batch) >= self.max_req)):
                break
            batch.append(self._q.popleft())
            atoms += r.n
            if self.max_req and len(batch) >= self.max_req:
                break
        return batch

    def _fail_or_split(self, reqs, err):
        """A failed batch of several requests goes back to the front of the
        queue one request at a time (only an offending request then fails); a
        request that fails alone gets the error."""
        if len(reqs) > 1:
            for r in reversed(reqs):
                r.solo = True
                self._q.appendleft(r)
        else:
            for r in reqs:
                r.future.set_exception(err)
            self.errors.append(err)

    def _loop(self):
        try:
            self._serve()
        except BaseException as e:  # never leave a caller waiting on a dead scheduler
            pending = list(self._q) + [r for s in self._slots for r in s.reqs]
            while not self._inbox.empty():
                pending.append(self._inbox.get())
            for r in pending:
                if not r.future.done():
                    r.future.set_exception(e)
            self.errors.append(e)

    def _serve(self):
        if self._cuda:
            torch.cuda.set_device(self.device)
        while not self._stop.is_set():
            while not self._inbox.empty():
                self._q.append(self._inbox.get())
            progressed = False
            for s in self._slots:
                if s.reqs and s.done():
                    try:
                        reqs, results = s.finish()
                        t = time.perf_counter()
                        for r in reqs:
                            r.t_done = t
                        self.completed.extend(reqs)  # recorded before any caller is woken
                        for r, res in zip(reqs, results):
                            r.future.set_result(res)
                    except Exception as e:
                        reqs, s.reqs = s.reqs, []
                        self._fail_or_split(reqs, e)
                    progressed = True
            for s in self._slots:
                if not s.reqs and self._q:
                    batch = self._admit()
                    now = time.perf_counter()
                    for r in batch:
                        r.t_admit = now
                    try:
                        s.launch(batch)
                    except Exception as e:  # e.g. no device memory for a request run alone
                        s.reqs = []
                        self._fail_or_split(batch, e)
                    self.batches += 1
                    progressed = True
            if not progressed:
                if any(s.reqs for s in self._slots):
                    time.sleep(2e-5)
                else:
                    self._wake.wait(timeout=1e-3)
                    self._wake.clear()


def latency_stats(reqs):
    """p50 / p99 latency (ms) from arrival to result, and atoms/s over the span."""
    lat = np.array([(r.t_done - r.arrival) * 1e3 for r in reqs])
    atoms = sum(r.n for r in reqs)
    span = max(r.t_done for r in reqs) - min(r.arrival for r in reqs)
    return {"requests": len(reqs), "atoms": atoms, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "atoms_per_s": atoms / span, "span_s": span}


def poisson_run(server, requests, rate, seed=4):
    """Open-loop load: submit ``requests`` [(xyz, radii), ...] at Poisson arrival times.

    Each request's latency runs from its scheduled arrival to its result, so
    queueing delay counts even if the submitter falls behind.  Returns the
    latency / throughput summary (``latency_stats``) of this run.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=len(requests))
    t0 = time.perf_counter() + 0.01
    arrivals = t0 + np.cumsum(gaps)
    futs = []
    for (xyz, rad), ta in zip(requests, arrivals):
        now = time.perf_counter()
        if ta > now:
            time.sleep(ta - now)
        futs.append(server.submit(xyz, rad, arrival=ta))
    for f in futs:
        f.result()
    ids = {id(f) for f in futs}
    done = [r for r in server.completed if id(r.future) in ids]
    out = latency_stats(done)
    out["rate_req_s"] = rate
    return out
