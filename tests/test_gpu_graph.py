"""Prepared batches (one hipGraph per batch): every replay reproduces the
oracle's results exactly, with eager checks and synchronizations between
the replays; the autotuner's tunings keep results equal to the oracle's."""
import pytest

from oracle import o2
from paper_2203_12878_amd import workloads as w

pytestmark = pytest.mark.gpu


def _items():
    items = [w.gen_small(s) for s in range(3)]
    items += [(t, n) for t, n, _ in w.gen_mixed_batch(1, 48)]
    items += [w.tree_protocol(14, None), w.tree_protocol(15, 3), w.tree_protocol(13, 12)]
    items += [(w.gen_large(1, n=4096, lo_prod=2, hi_prod=6)[0], 4096)]
    items += [("(foru x 0 3 (seq (wr 5) (rd (+ tid x))))", 9000), ("(wr (<< 1 tid))", 40)]
    return items


def test_graph_replays_match_oracle():
    import torch
    from paper_2203_12878_amd import drf
    chk = drf.Checker(0)
    items = _items()
    direct = o2.check_many(items, jobs=8)
    b = drf.Batch(items, 0)
    prep = chk.prepare(b)
    torch.cuda.synchronize()
    assert [r.key() for r in b.collect()] == [r.key() for r in direct]
    assert prep.launches > 5
    for rep in range(4):
        b.results.zero_()
        b.counts.zero_()
        prep.run()
        torch.cuda.synchronize()
        got = b.collect()
        assert [r.key() for r in got] == [r.key() for r in direct], rep
        # eager work between replays
        again = chk.check_batch(items[:5])
        assert [r.key() for r in again] == [r.key() for r in direct[:5]]
    prep.close()
    chk.close()


@pytest.mark.parametrize("tune", [dict(tile_events=2048, digit_bits=6), dict(tile_events=4096, digit_bits=10),
                                  dict(tile_events=256, digit_bits=4, unit_events=256, item_events=1024)])
def test_tunings_keep_results_exact(tune):
    from paper_2203_12878_amd import drf
    items = _items()
    ref = o2.check_many(items, jobs=8)
    chk = drf.Checker(0)
    chk.set_tuning(**tune)
    got = chk.check_batch(items)
    chk.close()
    assert [r.key() for r in got] == [r.key() for r in ref]
