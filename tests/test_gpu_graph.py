"""Graphs: a prepared batch (one hipGraph per batch) reproduces the
oracle's results on every replay, with eager checks and synchronizations
between the replays; a shape-class graph (captured once) checks several
different statically small batches exactly as the oracle does and refuses
batches outside its class without writing anything; the autotuner's
tunings keep results equal to the oracle's."""
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
                                  dict(tile_events=256, digit_bits=4, unit_events=256, item_events=1024),
                                  dict(unit_events=49152, item_events=262144),
                                  dict(unit_events=16384, item_events=262144), dict(digit_bits=8, unit_events=65536)])
def test_tunings_keep_results_exact(tune):
    from paper_2203_12878_amd import drf
    items = _items()
    ref = o2.check_many(items, jobs=8)
    chk = drf.Checker(0)
    chk.set_tuning(**tune)
    got = chk.check_batch(items)
    chk.close()
    assert [r.key() for r in got] == [r.key() for r in ref]


def _static_items():
    from paper_2203_12878_amd import drf
    mixed = [(t, n) for t, n, _ in w.gen_mixed_batch(2, 300)]
    mixed = [it for it in mixed if drf.plan(*it).max_phase_records <= 8192][:120]
    items = [w.gen_small(s) for s in range(4)]
    items += [w.tree_protocol(k, r) for k, r in ((8, None), (9, 3), (10, 9), (11, 0), (11, None))]
    items += [("(seq (if (= tid 0) (wr 1) (wr 2)) (sync) (if (= tid 1) (rd 0) (skip)) (wr 0))", 2),
              ("(foru x 0 3 (seq (wr 5) (rd (+ tid x))))", 900), ("(wr (<< 1 tid))", 40), ("(rd x)", 4)]
    return items + mixed


def test_graph_class_replays_new_batches_like_the_oracle():
    import torch
    from paper_2203_12878_amd import drf
    chk = drf.Checker(0)
    gc = chk.graph_class(max_protocols=160, max_nests=8192, max_code_words=1 << 18, max_fixed=8192,
                         max_phases=1 << 20, max_units=1 << 16)
    items = _static_items()
    want_all = o2.check_many(items, jobs=16)
    # batches of different sizes and contents through the one captured graph
    n = len(items)
    batches = [list(range(n)), list(range(40, 90)), list(range(9)), list(range(129, 4, -1)), list(range(100, n))]
    for bi, idx in enumerate(batches):
        its = [items[i] for i in idx]
        want = [want_all[i] for i in idx]
        b = drf.Batch(its, 0)
        assert gc.check(b), bi
        torch.cuda.synchronize()
        assert [r.key() for r in b.collect()] == [r.key() for r in want], bi
        # eager work between replays
        again = chk.check_batch(its[:3])
        assert [r.key() for r in again] == [r.key() for r in want[:3]]
    # outside the class: a phase above one tile, or more protocols than the capacity
    for its in ([w.tree_protocol(14, None)] + items[:4], items + items[:50]):
        b = drf.Batch(its, 0)
        b.results.fill_(7)
        assert not gc.check(b)
        torch.cuda.synchronize()
        assert int(b.results.min()) == 7 and int(b.results.max()) == 7
    gc.close()
    chk.close()
