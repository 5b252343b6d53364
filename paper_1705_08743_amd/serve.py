"""Continuously batched closure serving on one GPU, over the C ABI.

A request is one closure (all-pairs shortest anti-distances, or Boolean
reachability) of an n x n matrix that arrives on the host at a given time and
whose result goes back to the host.  The server:

* admits requests by HBM footprint: a request enters only while the device
  bytes of all admitted, unfinished requests plus its own stay within the
  budget, and a stream slot is free; the queue is scanned first-fit, so a
  small request can pass a large one that does not fit yet;
* keeps each admitted request's matrix resident on the device from its upload
  to its download (one H2D copy in, the closure in place, one D2H copy out);
* batches continuously: requests of one kind and of up to ``batch_n``
  vertices that are waiting when a slot frees up are closed together by one
  ``closure_batched`` launch (Boolean ones as {0, 255} anti-distance matrices
  in 16-bit working copies); larger requests each take a slot; all slots run
  concurrently on the device (one HIP stream each, default priority), and new
  arrivals are admitted as soon as slots and memory free up, while others are
  still running;
* measures latency from a request's arrival to the completion of its closure
  on the device (hipEvent timestamps on the request's stream, relative to a
  start event), and separately to the end of its download;
* isolates failures: a request whose closure call is refused by the library
  fails alone (its error is recorded, its slot and memory are released); when
  a batched call is refused, its requests are closed one by one, so only the
  bad one fails;
* cancels queued requests: ``cancel(rid)`` (from any thread) or a request's
  ``cancel_at`` time removes it from the queue if it has not been admitted
  yet; it is then never run.

``mode="serial"`` replays the same trace one solve at a time in arrival order
on one stream (no batching, no overlap): the baseline the served numbers are
compared with.  Every result is the same in both modes (integer arithmetic).
"""
import collections
import threading
import time

import numpy as np

from . import (SR_ANTIDIST_U16, SR_ANTIDIST_U8, SR_BOOL, SemiringError, closure,
               closure_batched, closure_work_bytes, empty, padded_ld)

_UNIT = {SR_BOOL: 8, SR_ANTIDIST_U8: 1, SR_ANTIDIST_U16: 2}


def footprint_bytes(kind, n, batch_n=256):
    """Device bytes a request holds while admitted: its padded matrix, plus
    the library's working memory for its closure, as the library's own query
    reports it (it follows closure()'s method rules and autotuning table).  A
    request closed in a batch needs no more: a uint8 batch's 16-bit working
    copy is smaller than closure()'s, and Boolean graphs of at most batch_n
    (<= 1024) vertices are closed on their bits."""
    del batch_n
    return n * padded_ld(n, kind) * _UNIT[kind] + closure_work_bytes(kind, n)


class Request:
    """One closure request: kind, vertex count, host matrix (uint8 / uint16
    entries, or uint64 Boolean words), arrival time in seconds.

    cancel_at: seconds from the start at which the request is withdrawn if it
    is still queued (None: never).  inject_fault: the request's closure call
    is made with a size beyond its matrix, which the library refuses (a
    failure injected for tests of failure isolation).  After a run, `result`
    holds the closure, or None with `error` (refused) or `cancelled` set."""

    __slots__ = ("rid", "kind", "n", "host", "arrival", "footprint", "result", "t_admit",
                 "t_compute_done", "t_done", "batch_size", "cancel_at", "inject_fault",
                 "error", "cancelled", "_dev", "_pin_in", "_pin_out")

    def __init__(self, rid, kind, n, host, arrival=0.0, cancel_at=None, inject_fault=False):
        self.rid = rid
        self.kind = kind
        self.n = n
        self.host = host
        self.arrival = float(arrival)
        self.footprint = footprint_bytes(kind, n)
        self.cancel_at = cancel_at
        self.inject_fault = bool(inject_fault)
        self._reset()

    def _reset(self):
        self.result = None
        self.t_admit = None
        self.t_compute_done = None
        self.t_done = None
        self.batch_size = 0
        self.error = None
        self.cancelled = False


class _Job:
    __slots__ = ("reqs", "slot", "ev_compute", "ev_done", "bytes")

    def __init__(self, reqs, slot, ev_compute, ev_done):
        self.reqs = reqs
        self.slot = slot
        self.ev_compute = ev_compute
        self.ev_done = ev_done
        self.bytes = sum(r.footprint for r in reqs)


class ClosureServer:
    def __init__(self, budget_bytes=16 << 30, slots=4, batch_n=256, batch_max=256):
        import torch
        self.torch = torch
        self.budget = int(budget_bytes)
        self.nslots = int(slots)
        self.batch_n = int(batch_n)
        self.batch_max = int(batch_max)
        self.streams = [torch.cuda.Stream() for _ in range(self.nslots)]
        self._pinned = {}
        self._cancel_lock = threading.Lock()
        self._cancel_ids = set()

    def cancel(self, rid):
        """Withdraw request `rid` if it is still queued (thread-safe; takes
        effect at the serving loop's next pass)."""
        with self._cancel_lock:
            self._cancel_ids.add(rid)

    # -- one request's buffers --------------------------------------------
    def _prepare(self, req):
        """Pinned host buffers for the upload and the result (allocated before
        the timed replay, as a client would hand them over).  The pinned copy
        of an input is cached per host array across replays."""
        torch = self.torch
        key = id(req.host)
        pin = self._pinned.get(key)
        if pin is None or pin[0] is not req.host:
            host = np.ascontiguousarray(req.host)
            if req.kind == SR_BOOL:
                words = (req.n + 63) // 64
                src = torch.from_numpy(host[:, :words].view(np.int64).copy())
            else:
                src = torch.from_numpy(host[:, :req.n].copy())
            pin = (req.host, src.pin_memory())
            self._pinned[key] = pin
        req._pin_in = pin[1]
        req._pin_out = torch.empty(pin[1].shape, dtype=pin[1].dtype, pin_memory=True)

    @staticmethod
    def _dim(r):
        # an injected fault asks for more vertices than the matrix holds
        return r.n + (1 << 20) if r.inject_fault else r.n

    def _close_one(self, r, stream):
        try:
            closure(r.kind, r._dev, D=self._dim(r), stream=stream)
        except SemiringError as e:
            r.error = str(e)

    def _launch(self, reqs, slot):
        """Upload, close and download a group of requests on one stream.  A
        refused closure call fails its request alone: the library checks
        every argument before it enqueues anything, so a refused batch is
        closed again one request at a time."""
        torch = self.torch
        stream = self.streams[slot]
        ev_compute = torch.cuda.Event(enable_timing=True)
        ev_done = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            for r in reqs:
                cols = r.n
                r._dev = empty(r.kind, r.n, cols, zero=False)
                r._dev.copy_(r._pin_in, non_blocking=True)
            if len(reqs) == 1:
                self._close_one(reqs[0], stream)
            else:
                try:
                    closure_batched(reqs[0].kind, [r._dev for r in reqs],
                                    Ds=[self._dim(r) for r in reqs], stream=stream)
                except SemiringError:
                    for r in reqs:
                        self._close_one(r, stream)
            ev_compute.record(stream)
            for r in reqs:
                if r.error is None:
                    r._pin_out.copy_(r._dev, non_blocking=True)
            ev_done.record(stream)
        for r in reqs:
            r.batch_size = len(reqs)
        return _Job(reqs, slot, ev_compute, ev_done)

    # -- admission ----------------------------------------------------------
    def _pick(self, waiting, free_bytes, allow_batch):
        """First-fit choice of the next job from the waiting queue: a batch of
        small requests of one kind, or one request."""
        for i, r in enumerate(waiting):
            if r.footprint > free_bytes:
                continue
            if allow_batch and r.n <= self.batch_n:
                group, used = [], 0
                for q in waiting:
                    if (q.kind == r.kind and q.n <= self.batch_n and used + q.footprint <= free_bytes
                            and len(group) < self.batch_max):
                        group.append(q)
                        used += q.footprint
                return group
            return [r]
        return None

    def run(self, requests, mode="served", poll_sleep=20e-6):
        """Replay `requests` (their `arrival` times are seconds from the start)
        and return a stats dict; each request's `result` holds its closure."""
        torch = self.torch
        serial = mode == "serial"
        if mode not in ("served", "serial"):
            raise ValueError("mode is 'served' or 'serial'")
        for r in requests:
            r._reset()
            r.footprint = footprint_bytes(r.kind, r.n, self.batch_n)
            if r.footprint > self.budget:
                raise ValueError("request %d needs %d bytes, above the budget" % (r.rid, r.footprint))
            self._prepare(r)
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = collections.deque()
        inflight = []
        free_slots = list(range(1 if serial else self.nslots))
        free_bytes = self.budget
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev0.record(self.streams[0])
        ev0.synchronize()
        t0 = time.perf_counter()
        while pending or waiting or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            progressed = False
            # withdrawals of queued requests, before any admission
            with self._cancel_lock:
                ids = set(self._cancel_ids)
            for r in list(waiting):
                if r.rid in ids or (r.cancel_at is not None and r.cancel_at <= now):
                    waiting.remove(r)
                    r.cancelled = True
                    r.t_done = now
                    progressed = True
            for job in list(inflight):
                if job.ev_done.query():
                    tc = ev0.elapsed_time(job.ev_compute) * 1e-3
                    td = ev0.elapsed_time(job.ev_done) * 1e-3
                    for r in job.reqs:
                        r.t_compute_done, r.t_done = tc, td
                        r.result = r._pin_out.numpy() if r.error is None else None
                        r._dev = None
                    free_bytes += job.bytes
                    free_slots.append(job.slot)
                    inflight.remove(job)
                    progressed = True
            while waiting and free_slots:
                group = self._pick(waiting, free_bytes, allow_batch=not serial)
                if group is None:
                    break
                if serial and group[0] is not waiting[0]:
                    break
                for r in group:
                    waiting.remove(r)
                    r.t_admit = time.perf_counter() - t0
                slot = free_slots.pop(0)
                free_bytes -= sum(r.footprint for r in group)
                inflight.append(self._launch(group, slot))
                progressed = True
            if not progressed:
                if pending and not waiting and not inflight:
                    wait = pending[0].arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 1e-3))
                else:
                    time.sleep(poll_sleep)
        with self._cancel_lock:
            self._cancel_ids.clear()
        return summarize(requests, mode)


def summarize(requests, mode):
    """Latency percentiles and throughput over the completed requests
    (failed and cancelled ones are counted apart)."""
    done = [r for r in requests if not r.cancelled and r.error is None]
    if not done:
        return {"mode": mode, "requests": 0,
                "failed": int(sum(1 for r in requests if r.error is not None)),
                "cancelled": int(sum(1 for r in requests if r.cancelled))}
    lat = np.array([r.t_compute_done - r.arrival for r in done])
    e2e = np.array([r.t_done - r.arrival for r in done])
    first = min(r.arrival for r in requests)
    last = max(r.t_done for r in done)
    span = last - first
    updates = float(sum(float(r.n) ** 3 for r in done))
    return {
        "mode": mode,
        "requests": len(done),
        "failed": int(sum(1 for r in requests if r.error is not None)),
        "cancelled": int(sum(1 for r in requests if r.cancelled)),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "p50_e2e_ms": float(np.percentile(e2e, 50) * 1e3),
        "p99_e2e_ms": float(np.percentile(e2e, 99) * 1e3),
        "makespan_s": span,
        "throughput_rps": len(done) / span,
        "updates_per_s": updates / span,
        "batched_requests": int(sum(1 for r in done if r.batch_size > 1)),
    }
