"""Continuous-batching check server on one GPU.

Requests (protocol text or bytecode, thread count) are compiled and planned
on arrival (host-only library calls).  The plan carries the library's upper
bound on the device scratch a check of the request takes; the part of it
beyond the fixed per-call cost is the request's footprint.  Requests wait
in an admission queue.  Each worker thread owns a libdrf context and its
own HIP stream.  Whenever a worker is free it takes waiting requests, in
arrival order, while the batch's footprint (the per-call cost plus the
requests' footprints) fits what is left of ONE device-wide budget shared by
all workers; the batch holds its footprint until it completes, then the
worker hands its context's pools back down to a small retained size.  So
the scratch held on the device stays within the budget plus the retained
pools.  A request too large for the budget runs alone once nothing else is
in flight (the library then splits its big phases into waves under the
context's limit).

Requests that arrive while batches run are admitted as soon as memory and
a worker free up, and batches of different workers overlap on the device.
A batch whose protocols are all statically small (every phase fits one
LDS tile by the plan) and that fits the worker's shape class is checked by
replaying the worker's class graph (one hipGraph launch, no host round
trip); any other batch goes through drf_check_batch.
Results stay in device memory until the batch completes; latency is
measured from submit() to the result.  A request whose future was
cancelled before admission is dropped; submit() raises Overloaded when the
queue already holds max_queue requests.  hold() pauses admission (for
maintenance; requests keep queueing) until resume().

    with Server(workers=2) as srv:
        fut = srv.submit("(seq (wr tid) (sync) (rd (mod (+ tid 1) 64)))", 64)
        print(fut.result().racy)
"""
from __future__ import annotations

import threading
import time
from collections import deque
from concurrent.futures import Future
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple, Union

import numpy as np

from . import drf

# scratch a worker's context keeps between batches (pool A of a typical
# batch: metadata and witness candidates)
RETAIN_BYTES = 64 << 20
# shape class of each worker's graph (batches beyond it use drf_check_batch)
GRAPH_CAPS = dict(max_protocols=256, max_nests=16384, max_code_words=1 << 18, max_fixed=16384,
                  max_phases=1 << 21, max_units=1 << 16)


class Overloaded(RuntimeError):
    """The admission queue is full."""


@dataclass
class Request:
    code: np.ndarray
    n: int
    plan: drf.Plan
    bytes: int                      # footprint beyond the per-call cost
    t_submit: float
    future: Future
    t_done: float = 0.0


@dataclass
class Stats:
    completed: int = 0
    cancelled: int = 0
    rejected: int = 0
    records: int = 0
    batches: int = 0
    max_batch_size: int = 0
    max_in_flight_bytes: int = 0      # largest sum of footprints held at once
    graph_batches: int = 0            # batches checked by a class graph replay
    latencies: List[float] = field(default_factory=list)

    def percentile(self, q: float) -> float:
        if not self.latencies:
            return float("nan")
        return float(np.percentile(np.array(self.latencies), q))


def admit(queue: Sequence[Request], call_bytes: int, free_bytes: int, in_flight: int,
          max_batch: int) -> int:
    """How many requests from the head of `queue` one batch takes.

    Requests join in arrival order while the per-call cost plus their
    footprints fits `free_bytes`.  When even the head request does not fit:
    it runs alone if no batch is in flight (0 is returned only when the
    queue is empty or the head must wait for memory)."""
    if not queue:
        return 0
    used = call_bytes
    k = 0
    while k < len(queue) and k < max_batch and used + queue[k].bytes <= free_bytes:
        used += queue[k].bytes
        k += 1
    if k == 0 and in_flight == 0:
        k = 1
    return k


class Server:
    def __init__(self, device: int = 0, workers: int = 2, budget_bytes: int = 16 << 30,
                 max_batch: int = 4096, max_queue: int = 1 << 20, graph_caps: Optional[dict] = None):
        import torch
        self.device = device
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.max_queue = max_queue
        self.stats = Stats()
        self._q: deque = deque()
        self._cv = threading.Condition()
        self._stop = False
        self._held = False
        self._in_flight_bytes = 0
        self._in_flight = 0
        self._threads = []
        self._checkers = []
        self._streams = []
        self._graphs = []
        # shape class of the workers' graphs (None: no graphs)
        self.graph_caps = dict(GRAPH_CAPS) if graph_caps is None else (graph_caps or None)
        # per-call scratch (what a check of the smallest protocol takes):
        # charged once per batch, not per request
        self.call_bytes = int(drf.plan("(skip)", 1).scratch_bytes)
        for w in range(workers):
            # one batch may use the whole budget when it runs alone
            chk = drf.Checker(device, scratch_limit=max(self.budget, 2 * self.call_bytes))
            self._checkers.append(chk)
            self._streams.append(torch.cuda.Stream(device=device))
            self._graphs.append(chk.graph_class(**self.graph_caps) if self.graph_caps else None)
        for w in range(workers):
            t = threading.Thread(target=self._worker, args=(w,), daemon=True)
            t.start()
            self._threads.append(t)

    # -------------------------------------------------------------- client
    def submit(self, proto: Union[str, np.ndarray], n: int) -> Future:
        t0 = time.perf_counter()
        code = drf.compile_text(proto) if isinstance(proto, str) else np.ascontiguousarray(proto, dtype=np.uint32)
        p = drf.plan(code, n)
        fut: Future = Future()
        req = Request(code, int(n), p, max(0, int(p.scratch_bytes) - self.call_bytes), t0, fut)
        with self._cv:
            if self._stop:
                raise RuntimeError("server is closed")
            if len(self._q) >= self.max_queue:
                self.stats.rejected += 1
                raise Overloaded("admission queue holds %d requests" % len(self._q))
            self._q.append(req)
            self._cv.notify()
        return fut

    def hold(self):
        """Stop admitting new batches (batches in flight finish; requests
        keep queueing up to max_queue)."""
        with self._cv:
            self._held = True

    def resume(self):
        with self._cv:
            self._held = False
            self._cv.notify_all()

    def reset_stats(self):
        """Start the statistics afresh (e.g. after a warm-up stream)."""
        with self._cv:
            self.stats = Stats()

    def close(self):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        for t in self._threads:
            t.join()
        for gr in self._graphs:
            if gr is not None:
                gr.close()
        for c in self._checkers:
            c.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -------------------------------------------------------------- worker
    def _take(self) -> Optional[Tuple[List[Request], int]]:
        with self._cv:
            while True:
                # requests cancelled while waiting are dropped
                while self._q and self._q[0].future.cancelled():
                    self._q.popleft()
                    self.stats.cancelled += 1
                if self._stop and not self._q:
                    return None
                if self._held and not self._stop:
                    self._cv.wait()
                    continue
                k = admit(self._q, self.call_bytes, self.budget - self._in_flight_bytes, self._in_flight,
                          self.max_batch)
                if k:
                    break
                self._cv.wait()
            batch = []
            for _ in range(k):
                r = self._q.popleft()
                if r.future.set_running_or_notify_cancel():
                    batch.append(r)
                else:
                    self.stats.cancelled += 1
            held = min(self.budget, self.call_bytes + sum(r.bytes for r in batch)) if batch else 0
            self._in_flight_bytes += held
            self._in_flight += 1
            st = self.stats
            st.max_in_flight_bytes = max(st.max_in_flight_bytes, self._in_flight_bytes)
            return batch, held

    def _finish(self, held: int):
        with self._cv:
            self._in_flight_bytes -= held
            self._in_flight -= 1
            self._cv.notify_all()

    def _worker(self, w: int):
        import torch
        chk = self._checkers[w]
        stream = self._streams[w]
        graph = self._graphs[w]
        tile = chk.tuning()["tile_events"]
        while True:
            got = self._take()
            if got is None:
                return
            batch, held = got
            if not batch:
                self._finish(held)
                continue
            try:
                with torch.cuda.stream(stream):
                    b = drf.Batch([(r.code, r.n) for r in batch], self.device, plans=[r.plan for r in batch])
                    static = graph is not None and len(batch) <= graph.caps.max_protocols and all(
                        r.plan.status != 0 or r.plan.max_phase_records <= tile for r in batch)
                    by_graph = static and graph.check(b, stream)
                    if not by_graph:
                        chk.run_batch(b, stream)
                    stream.synchronize()
                    res = b.collect()
                    if not by_graph:
                        chk.release(RETAIN_BYTES)
            except Exception as e:  # a failed batch fails its requests, not the server
                self._finish(held)
                for r in batch:
                    r.future.set_exception(e)
                continue
            self._finish(held)
            now = time.perf_counter()
            with self._cv:
                st = self.stats
                st.batches += 1
                st.graph_batches += 1 if by_graph else 0
                st.max_batch_size = max(st.max_batch_size, len(batch))
                for r, x in zip(batch, res):
                    r.t_done = now
                    st.completed += 1
                    st.records += x.num_records
                    st.latencies.append(now - r.t_submit)
            for r, x in zip(batch, res):
                r.future.set_result(x)


def run_stream(server: Server, requests: Sequence[Tuple[float, str, int]]):
    """Submit (arrival_s, text, n) requests at their arrival times; wait for
    all results.  The texts are encoded to bytecode before the stream starts
    (the client's side of the protocol), so submission is planning and
    admission only.  Returns (results, wall seconds from first arrival to
    last result)."""
    coded = [(at, drf.compile_text(text), n) for at, text, n, *_ in requests]
    futs = []
    t0 = time.perf_counter()
    for at, code, n in coded:
        # sleep only when the next arrival is well ahead (a short sleep
        # overshoots by tens of microseconds); otherwise catch up at once
        delay = at - (time.perf_counter() - t0)
        if delay > 2e-4:
            time.sleep(delay - 1e-4)
        futs.append(server.submit(code, n))
    out = [f.result() for f in futs]
    return out, time.perf_counter() - t0
