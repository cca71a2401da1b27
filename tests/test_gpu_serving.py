"""Serving (continuous batching) on the GPU: every request's result in the
mix equals its result checked alone (exact integers, tolerance 0), the
oracle agrees on the smaller ones, admission keeps the footprints held at
once within the one device-wide budget, cancelled requests never run and a
full queue refuses new requests.  The stream is served both with the
workers' class graphs (statically small batches replayed as one graph
launch) and without them."""
import pytest

from oracle import o2
from paper_2203_12878_amd import workloads as w

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("graphs", [True, False])
def test_serving_mix_equals_alone(graphs):
    from paper_2203_12878_amd import drf
    from paper_2203_12878_amd.server import Server, run_stream
    reqs = w.gen_requests(rate=3000.0, max_requests=400, horizon_s=1.0)
    assert len(reqs) > 100
    budget = 2 << 30
    with Server(device=0, workers=2, budget_bytes=budget, graph_caps=None if graphs else {}) as srv:
        mixed, wall = run_stream(srv, reqs)
        st = srv.stats
    assert st.completed == len(reqs)
    assert st.batches < len(reqs)          # requests were batched
    assert st.max_in_flight_bytes <= budget   # a request above the budget runs alone
    assert (st.graph_batches > 0) == graphs
    chk = drf.Checker(0)
    alone = [chk.check(t, n) for _, t, n, _ in reqs]
    chk.close()
    for (at, t, n, src), a, b in zip(reqs, alone, mixed):
        assert a.key() == b.key(), (src, n)
    small = [i for i, r in enumerate(alone) if r.num_records < 2_000_000]
    want = o2.check_many([(reqs[i][1], reqs[i][2]) for i in small], jobs=16)
    for i, e in zip(small, want):
        assert mixed[i].key() == e.key(), reqs[i][3]


def test_cancel_and_overload():
    from paper_2203_12878_amd.server import Overloaded, Server
    items = [w.gen_small(s) for s in range(6)] + [w.tree_protocol(10 + s, s) for s in range(6)]
    with Server(device=0, workers=2, budget_bytes=1 << 30, max_queue=len(items)) as srv:
        srv.hold()
        futs = [srv.submit(t, n) for t, n in items]
        with pytest.raises(Overloaded):
            srv.submit(*items[0])
        cancelled = [i for i in range(len(futs)) if i % 4 == 1]
        for i in cancelled:
            assert futs[i].cancel()
        srv.resume()
        keep = [i for i in range(len(futs)) if i not in cancelled]
        got = [futs[i].result(timeout=60) for i in keep]
        st = srv.stats
    assert st.rejected == 1 and st.cancelled == len(cancelled) and st.completed == len(keep)
    assert all(futs[i].cancelled() for i in cancelled)
    want = o2.check_many([items[i] for i in keep])
    assert [g.key() for g in got] == [e.key() for e in want]
