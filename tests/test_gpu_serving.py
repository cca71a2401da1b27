"""Serving (continuous batching) on the GPU: every request's result in the
mix equals its result checked alone (exact integers, tolerance 0), the
oracle agrees on the smaller ones, and admission respects the budget."""
import pytest

from oracle import o2
from paper_2203_12878_amd import workloads as w

pytestmark = pytest.mark.gpu


def test_serving_mix_equals_alone():
    from paper_2203_12878_amd import drf
    from paper_2203_12878_amd.server import Server, run_stream
    reqs = w.gen_requests(rate=3000.0, max_requests=400, horizon_s=1.0)
    assert len(reqs) > 100
    budget = 2 << 30
    with Server(device=0, workers=2, budget_bytes=budget) as srv:
        mixed, wall = run_stream(srv, reqs)
        st = srv.stats
    assert st.completed == len(reqs)
    assert st.batches < len(reqs)          # requests were batched
    assert st.max_batch_bytes <= budget   # a request above the budget runs alone
    chk = drf.Checker(0)
    alone = [chk.check(t, n) for _, t, n, _ in reqs]
    chk.close()
    for (at, t, n, src), a, b in zip(reqs, alone, mixed):
        assert a.key() == b.key(), (src, n)
    small = [i for i, r in enumerate(alone) if r.num_records < 2_000_000]
    want = o2.check_many([(reqs[i][1], reqs[i][2]) for i in small], jobs=16)
    for i, e in zip(small, want):
        assert mixed[i].key() == e.key(), reqs[i][3]
