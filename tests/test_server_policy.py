"""Admission policy of the serving loop (host logic, no GPU): requests join a
batch in arrival order while the per-call cost plus their footprints fits
the free part of the one device-wide budget; a request larger than the
budget runs alone once nothing is in flight, and otherwise waits."""
from concurrent.futures import Future
from dataclasses import dataclass

from paper_2203_12878_amd.server import admit


@dataclass
class R:
    bytes: int
    future: Future = None


def q(*sizes):
    return [R(s, Future()) for s in sizes]


def test_takes_in_arrival_order_while_it_fits():
    assert admit(q(10, 20, 30, 40), call_bytes=5, free_bytes=70, in_flight=1, max_batch=100) == 3
    # the fourth would fit alone but order is kept: nothing jumps the queue
    assert admit(q(10, 60, 1), call_bytes=5, free_bytes=70, in_flight=1, max_batch=100) == 1


def test_batch_size_cap():
    assert admit(q(*[1] * 50), call_bytes=0, free_bytes=10 ** 9, in_flight=0, max_batch=16) == 16


def test_oversized_request_waits_then_runs_alone():
    big = q(500, 1, 1)
    # memory is held by a batch in flight: wait
    assert admit(big, call_bytes=5, free_bytes=100, in_flight=1, max_batch=100) == 0
    # nothing in flight: the big request runs alone (the library splits it
    # into waves under the context's limit)
    assert admit(big, call_bytes=5, free_bytes=100, in_flight=0, max_batch=100) == 1


def test_empty_queue():
    assert admit([], call_bytes=5, free_bytes=100, in_flight=0, max_batch=100) == 0


def test_in_flight_sum_never_exceeds_budget():
    # simulate workers taking batches until memory runs out: the footprints
    # held at once stay within the budget unless a single request is larger
    budget, call = 1000, 10
    queue = q(*[37, 410, 5, 999, 120, 80, 300, 2, 2, 2, 640, 15])
    held, in_flight, peak = 0, 0, 0
    batches = []
    while queue:
        k = admit(queue, call, budget - held, in_flight, max_batch=8)
        if k == 0:      # wait: the oldest batch completes
            b = batches.pop(0)
            held -= b
            in_flight -= 1
            continue
        take, queue = queue[:k], queue[k:]
        fp = min(budget, call + sum(r.bytes for r in take))
        held += fp
        in_flight += 1
        batches.append(fp)
        peak = max(peak, held)
    assert peak <= budget
