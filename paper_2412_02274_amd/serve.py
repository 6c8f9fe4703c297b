"""Serving gres queries over resident relations (continuous batching over the C ABI).

A query names a resident relation and a set of its tuples; the answer is the grid resistance
(Def. 2, via Alg. 1) of each of them in that relation, i.e. ``gres_search`` against the
relation's prepared skyline. The server keeps every relation resident on the device (its SoA
values and its skyline prepared once with ``gres_prepare``: candidates in curve order with
their tile boxes, from which every level's keys are one FP32 multiply away).

Scheduling (``Server``):
  * arrivals wait in a FIFO queue;
  * when a slot (one HIP stream with its own pinned staging buffers) is free, the oldest
    queued query is admitted together with the later queued queries for the same relation (one
    search launch over their concatenated tuples), if the batch's device memory -- target
    indices, search workspace, outputs -- fits in what is left of the HBM budget (an arena of
    ``budget_bytes`` carved first-fit); the batch shrinks to fit, and if even the oldest query
    does not fit, everything waits (the oldest query is never overtaken: no starvation);
  * a batch's upload, search and download are queued on its slot's stream, so up to ``slots``
    batches run on the device at once, overlapping each other;
  * completions are detected by polling events, which frees the slot and the arena range and
    admits more work at once.
Latency is arrival -> completion as the host observes it.

``PlainServer`` is the reference: one query at a time, in arrival order, on one stream, each
waited for before the next starts.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import gc
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from .api import _ptr, PreparedCandidates, build, ingest, check_status

__all__ = ["Resident", "Query", "Arena", "Server", "PlainServer", "poisson_trace", "latency_stats"]


class Resident:
    """One relation kept on the device: values (SoA), its skyline, the prepared candidates."""

    def __init__(self, x_rows_host: np.ndarray, device):
        dev = torch.device(device)
        self.n, self.d = (int(v) for v in x_rows_host.shape)
        x_rows = torch.from_numpy(np.ascontiguousarray(x_rows_host, dtype=np.float32)).to(dev)
        self.x_soa = ingest(x_rows)
        del x_rows
        plan = build(self.x_soa)
        plan.local_skylines()
        self.sky = plan.merge().clone()
        plan.close()
        self.s = int(self.sky.numel())
        self.sky_host = self.sky.cpu().numpy()
        self.prep = PreparedCandidates(self.x_soa, self.sky)
        torch.cuda.synchronize(dev)
        check_status(self.prep.status, "gres_prepare")

    def resident_bytes(self):
        return self.x_soa.numel() * 4 + self.sky.numel() * 8 + self.prep.prep.numel()


@dataclass
class Query:
    qid: int
    rel: int
    targets: np.ndarray          # int64 rows of the relation
    g_max: int
    arrival: float               # seconds from the start of the trace
    admitted: float = -1.0
    done: float = -1.0
    g_exit: np.ndarray | None = None
    extra: dict = field(default_factory=dict)

    @property
    def latency(self):
        return self.done - self.arrival


def poisson_trace(residents, rate, duration, seed=0, g_max=25, start=0):
    """Queries with exponential inter-arrival times (mean 1/rate) over `duration` seconds; each
    picks a relation uniformly and a uniformly random subset of its skyline of uniform size in
    1..S."""
    rng = np.random.default_rng(seed)
    t, out, q = 0.0, [], start
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        r = int(rng.integers(len(residents)))
        sky = residents[r].sky_host
        k = int(rng.integers(1, len(sky) + 1))
        tg = np.sort(rng.choice(sky, size=k, replace=False)).astype(np.int64)
        out.append(Query(q, r, tg, g_max, t))
        q += 1
    return out


class Arena:
    """First-fit ranges of one device buffer (256-byte aligned)."""

    ALIGN = 256

    def __init__(self, nbytes, device):
        self.size = int(nbytes)
        self.buf = torch.empty(self.size, dtype=torch.uint8, device=device)
        self.free = [(0, self.size)]
        self.used = 0

    def alloc(self, nbytes):
        need = -(-int(nbytes) // self.ALIGN) * self.ALIGN
        for i, (a, n) in enumerate(self.free):
            if n >= need:
                if n == need:
                    self.free.pop(i)
                else:
                    self.free[i] = (a + need, n - need)
                self.used += need
                return a, need
        return None

    def release(self, rng):
        a, n = rng
        self.used -= n
        self.free.append((a, n))
        self.free.sort()
        merged = []
        for s, k in self.free:
            if merged and merged[-1][0] + merged[-1][1] == s:
                merged[-1] = (merged[-1][0], merged[-1][1] + k)
            else:
                merged.append((s, k))
        self.free = merged

    _SIZE = {torch.int64: 8, torch.int32: 4, torch.float32: 4, torch.uint8: 1}

    def view(self, rng, dtype, count, offset=0):
        a, _ = rng
        nb = self._SIZE[dtype] * count
        return self.buf[a + offset: a + offset + nb].view(dtype)


def _query_bytes(nt, d):
    ws = int(_lib.load().gres_search_bytes(nt, d))
    return ws, [8 * nt, 4 * nt, 256, ws]  # targets, g_exit, status, workspace


class _Slot:
    def __init__(self, device, cap):
        self.stream = torch.cuda.Stream(device)
        self.h_targets = torch.empty(cap, dtype=torch.int64, pin_memory=True)
        self.h_out = torch.empty(cap + 1, dtype=torch.int32, pin_memory=True)
        self.event = torch.cuda.Event()
        self.batch = None
        self.rng = None


class Server:
    """Continuous batching of gres queries under an HBM budget (see the module docstring).

    When a slot frees, the oldest queued query is admitted together with the later queued
    queries for the same relation and g_max (up to ``max_batch`` queries and ``max_targets``
    tuples), as ONE search launch over their concatenated tuples; each query's answer is its
    slice of the result. The oldest queued query is always in the next batch admitted."""

    def __init__(self, residents, budget_bytes=64 << 20, slots=4, device="cuda", max_batch=64,
                 max_targets=1 << 16):
        self.res = residents
        self.device = torch.device(device)
        max_nt = max(r.s for r in residents)
        self.cap = max(max_nt, int(max_targets))
        self.max_batch = int(max_batch)
        self.arena = Arena(budget_bytes, self.device)
        self.slots = [_Slot(self.device, self.cap) for _ in range(slots)]
        self.queue = []
        self.completed = []
        self.peak_used = 0
        self.max_in_flight = 0
        self.admit_order = []
        self.batch_log = []   # (oldest queued qid at admission, qids of the batch)
        for r in residents:  # the largest query of any relation must fit the budget alone
            if self._footprint(r.s, r.d) > budget_bytes:
                raise ValueError("budget_bytes below the largest query's footprint")

    @staticmethod
    def _footprint(nt, d):
        _, parts = _query_bytes(nt, d)
        return sum(-(-p // Arena.ALIGN) * Arena.ALIGN for p in parts)

    def _launch(self, slot, batch, rng, now):
        lib = _lib.load()
        q0 = batch[0]
        r = self.res[q0.rel]
        nt = sum(len(q.targets) for q in batch)
        ws_bytes, parts = _query_bytes(nt, r.d)
        offs = np.cumsum([0] + [-(-p // Arena.ALIGN) * Arena.ALIGN for p in parts])
        st = slot.stream
        with torch.cuda.stream(st):
            slot.h_targets[:nt].copy_(torch.from_numpy(np.concatenate([q.targets for q in batch])))
            d_targets = self.arena.view(rng, torch.int64, nt, int(offs[0]))
            d_ge = self.arena.view(rng, torch.int32, nt, int(offs[1]))
            d_status = self.arena.view(rng, torch.int32, 1, int(offs[2]))
            d_ws = self.arena.buf[rng[0] + int(offs[3]): rng[0] + int(offs[3]) + ws_bytes]
            d_targets.copy_(slot.h_targets[:nt], non_blocking=True)
            d_status.zero_()
            opts = _lib.GresOpts(_lib.SKY_GRES_AUTO)
            _lib.check(lib.gres_search(_ptr(r.prep.prep), r.s, r.d, _ptr(r.x_soa), r.n,
                                       r.x_soa.stride(0), _ptr(d_targets), nt, q0.g_max,
                                       _ptr(d_ge), None, _ptr(d_ws), ws_bytes, _ptr(d_status),
                                       C.byref(opts), C.c_void_p(st.cuda_stream)), "gres_search")
            slot.h_out[:nt].copy_(d_ge, non_blocking=True)
            slot.h_out[nt:nt + 1].copy_(d_status, non_blocking=True)
            slot.event.record(st)
        slot.batch, slot.rng = batch, rng
        for q in batch:
            q.admitted = now

    def _retire(self, slot, now):
        batch = slot.batch
        nt = sum(len(q.targets) for q in batch)
        code = int(slot.h_out[nt])
        if code != _lib.SKY_OK:
            raise _lib.SkyError(code, f"queries {[q.qid for q in batch]}")
        out = slot.h_out[:nt].numpy()
        o = 0
        for q in batch:
            q.g_exit = out[o:o + len(q.targets)].copy()
            o += len(q.targets)
            q.done = now
            self.completed.append(q)
        self.arena.release(slot.rng)
        slot.batch, slot.rng = None, None

    def _gather(self):
        """The next batch: the oldest queued query and later ones for the same relation and
        g_max, within the batch limits."""
        head = self.queue[0]
        batch, nt = [head], len(head.targets)
        for q in self.queue[1:]:
            if len(batch) >= self.max_batch:
                break
            if q.rel == head.rel and q.g_max == head.g_max and nt + len(q.targets) <= self.cap:
                batch.append(q)
                nt += len(q.targets)
        return batch, nt

    def poll(self, now):
        """Retire finished batches, then admit queued queries while a slot and memory are free."""
        for slot in self.slots:
            if slot.batch is not None and slot.event.query():
                self._retire(slot, now)
        while self.queue:
            slot = next((s for s in self.slots if s.batch is None), None)
            if slot is None:
                break
            batch, nt = self._gather()
            d = self.res[batch[0].rel].d
            rng = self.arena.alloc(self._footprint(nt, d))
            while rng is None and len(batch) > 1:  # shrink the batch, never skip its head
                nt -= len(batch[-1].targets)
                batch.pop()
                rng = self.arena.alloc(self._footprint(nt, d))
            if rng is None:
                break  # wait for memory rather than let later queries overtake the oldest
            self.batch_log.append((self.queue[0].qid, [q.qid for q in batch]))
            taken = {id(q) for q in batch}
            self.queue = [q for q in self.queue if id(q) not in taken]
            self._launch(slot, batch, rng, now)
            self.admit_order.extend(q.qid for q in batch)
            self.peak_used = max(self.peak_used, self.arena.used)
        self.max_in_flight = max(self.max_in_flight, sum(s.batch is not None for s in self.slots))

    def busy(self):
        return bool(self.queue) or any(s.batch is not None for s in self.slots)

    def run_trace(self, queries, clock=time.perf_counter):
        """Replay arrivals in real time (queries sorted by arrival); returns completed queries."""
        self.completed = []
        with _no_gc_pauses():
            t0 = clock()
            i = 0
            while i < len(queries) or self.busy():
                now = clock() - t0
                while i < len(queries) and queries[i].arrival <= now:
                    self.queue.append(queries[i])
                    i += 1
                self.poll(now)
        return self.completed


class PlainServer:
    """One query at a time, in arrival order, each waited for before the next starts."""

    def __init__(self, residents, device="cuda"):
        self.res = residents
        self.device = torch.device(device)
        max_nt = max(r.s for r in residents)
        self.d_targets = torch.empty(max_nt, dtype=torch.int64, device=self.device)
        self.d_ge = torch.empty(max_nt, dtype=torch.int32, device=self.device)
        self.status = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.ws = torch.empty(max(int(_lib.load().gres_search_bytes(max_nt, r.d)) for r in residents),
                              dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(self.device)

    def run_one(self, q):
        lib = _lib.load()
        r = self.res[q.rel]
        nt = len(q.targets)
        st = self.stream
        with torch.cuda.stream(st):
            self.d_targets[:nt].copy_(torch.from_numpy(q.targets))
            self.status.zero_()
            ws_bytes = int(lib.gres_search_bytes(nt, r.d))
            opts = _lib.GresOpts(_lib.SKY_GRES_AUTO)
            _lib.check(lib.gres_search(_ptr(r.prep.prep), r.s, r.d, _ptr(r.x_soa), r.n,
                                       r.x_soa.stride(0), _ptr(self.d_targets), nt, q.g_max,
                                       _ptr(self.d_ge), None, _ptr(self.ws), ws_bytes,
                                       _ptr(self.status), C.byref(opts), C.c_void_p(st.cuda_stream)),
                       "gres_search")
            out = self.d_ge[:nt].cpu().numpy()
            check_status(self.status, f"query {q.qid}")
        q.g_exit = out
        return q

    def run_trace(self, queries, clock=time.perf_counter):
        done = []
        with _no_gc_pauses():
            t0 = clock()
            for q in queries:
                while clock() - t0 < q.arrival:
                    pass
                q.admitted = clock() - t0
                self.run_one(q)
                q.done = clock() - t0
                done.append(q)
        return done


@contextlib.contextmanager
def _no_gc_pauses():
    """The dispatch loop runs with Python's cyclic garbage collector off: a full collection over
    thousands of live query objects stalls every query in flight for tens of milliseconds. It
    is switched back on (and run once) when the loop ends."""
    was = gc.isenabled()
    gc.disable()
    try:
        yield
    finally:
        if was:
            gc.enable()
            gc.collect()


def latency_stats(done):
    lat = np.array([q.latency for q in done]) * 1e3
    span = max(q.done for q in done) - min(q.arrival for q in done)
    return {"requests": len(done), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "max_ms": float(lat.max()), "throughput_rps": len(done) / span,
            "tuples_per_s": sum(len(q.targets) for q in done) / span}
