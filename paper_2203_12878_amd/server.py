"""Continuous-batching check server on one GPU.

Requests (protocol text or bytecode, thread count) are compiled and planned
on arrival (host-only library calls) to get their device footprint, then
wait in an admission queue.  Each worker thread owns a libdrf context and
its own HIP stream; whenever a worker is free it takes every waiting
request, in arrival order, whose footprint still fits its budget (at least
one), and checks them as one batch.  Requests that arrive while batches
run are admitted as soon as a worker frees up, and batches of different
workers overlap on the device.  Results stay in device memory until the
batch completes; latency is measured from submit() to the result.

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

# HBM bytes per access event of a phase that goes through HBM (two record
# buffers and partition metadata); phases within one LDS tile need none.
BYTES_PER_EVENT = 20
TILE_EVENTS = 8192
BASE_FOOTPRINT = 4096


def footprint(p: drf.Plan) -> int:
    """Device bytes a request may need beyond its fixed metadata."""
    if p.status != 0 or p.max_phase_records <= TILE_EVENTS:
        return BASE_FOOTPRINT
    return BASE_FOOTPRINT + BYTES_PER_EVENT * int(p.max_records)


@dataclass
class Request:
    code: np.ndarray
    n: int
    plan: drf.Plan
    bytes: int
    t_submit: float
    future: Future
    t_done: float = 0.0


@dataclass
class Stats:
    completed: int = 0
    records: int = 0
    batches: int = 0
    max_batch_bytes: int = 0          # largest footprint of a batch of two or more requests
    max_batch_size: int = 0
    latencies: List[float] = field(default_factory=list)

    def percentile(self, q: float) -> float:
        if not self.latencies:
            return float("nan")
        return float(np.percentile(np.array(self.latencies), q))


class Server:
    def __init__(self, device: int = 0, workers: int = 2, budget_bytes: int = 16 << 30,
                 max_batch: int = 4096):
        import torch
        self.device = device
        self.budget = budget_bytes
        self.max_batch = max_batch
        self.stats = Stats()
        self._q: deque = deque()
        self._cv = threading.Condition()
        self._stop = False
        self._threads = []
        self._checkers = []
        self._streams = []
        for w in range(workers):
            chk = drf.Checker(device, scratch_limit=budget_bytes + (1 << 30))
            self._checkers.append(chk)
            self._streams.append(torch.cuda.Stream(device=device))
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
        req = Request(code, int(n), p, footprint(p), t0, fut)
        with self._cv:
            if self._stop:
                raise RuntimeError("server is closed")
            self._q.append(req)
            self._cv.notify()
        return fut

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
        for c in self._checkers:
            c.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -------------------------------------------------------------- worker
    def _take(self) -> Optional[List[Request]]:
        with self._cv:
            while not self._q and not self._stop:
                self._cv.wait()
            if not self._q:
                return None
            batch = [self._q.popleft()]
            used = batch[0].bytes
            while self._q and len(batch) < self.max_batch and used + self._q[0].bytes <= self.budget:
                r = self._q.popleft()
                used += r.bytes
                batch.append(r)
            return batch

    def _worker(self, w: int):
        import torch
        chk = self._checkers[w]
        stream = self._streams[w]
        while True:
            batch = self._take()
            if batch is None:
                return
            try:
                with torch.cuda.stream(stream):
                    b = drf.Batch([(r.code, r.n) for r in batch], self.device, plans=[r.plan for r in batch])
                    chk.run_batch(b, stream)
                    stream.synchronize()
                    res = b.collect()
            except Exception as e:  # a failed batch fails its requests, not the server
                for r in batch:
                    r.future.set_exception(e)
                continue
            now = time.perf_counter()
            with self._cv:
                st = self.stats
                st.batches += 1
                st.max_batch_size = max(st.max_batch_size, len(batch))
                if len(batch) > 1:
                    st.max_batch_bytes = max(st.max_batch_bytes, sum(r.bytes for r in batch))
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
