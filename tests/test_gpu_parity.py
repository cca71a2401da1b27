"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
bit-exact on every output (status, race flag, witness, per-phase counts,
record count)."""
import os
import sys

import numpy as np
import pytest

from oracle import o2, ref
from paper_2203_12878_amd import workloads as w

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def chk():
    from paper_2203_12878_amd import drf
    c = drf.Checker(0)
    yield c
    c.close()


def _same(got, want, items):
    bad = [(t[:120], n, g, e) for (t, n), g, e in zip(items, got, want) if g.key() != e.key()]
    assert not bad, "%d mismatches, first: %r" % (len(bad), bad[:3])


def test_paper_examples(chk):
    import test_oracle as T
    golden = T.load_golden()
    items = [(c["text"], c["n"]) for c in golden]
    got = chk.check_batch(items)
    for c, g in zip(golden, got):
        e = c["expect"]
        assert g.status == e["status"], c["name"]
        if e["status"] == 0:
            assert g.racy == e["racy"] and list(g.phase_counts) == e["phase_counts"], c["name"]
            assert g.witness == (tuple(e["witness"]) if e["witness"] else None), c["name"]


def test_closed_forms(chk):
    import test_oracle as T
    cases = T.closed_form_cases()
    got = chk.check_batch([(t, n) for _, t, n, *_ in cases])
    for (name, t, n, racy, wit, counts), g in zip(cases, got):
        assert (g.status, g.racy, g.witness, list(g.phase_counts)) == (0, racy, wit, counts), name
    errs = chk.check_batch([(t, n) for t, n, _ in T.ERROR_CASES])
    for (t, n, st), g in zip(T.ERROR_CASES, errs):
        assert g.status == st, t


def test_tiny_enumeration(chk):
    items = list(w.enumerate_tiny())
    want = o2.check_many(items, jobs=16)
    got = chk.check_batch(items)
    _same(got, want, items)


def test_plain_path_equals_batch(chk):
    items = list(w.enumerate_tiny(limit_random=400, seed=3))[-400:]
    items += [w.gen_small(1), w.tree_protocol(9, 2)]
    batch = chk.check_batch(items)
    for (t, n), b in zip(items, batch):
        assert chk.check(t, n).key() == b.key(), t


def test_small_config_seeds(chk):
    items = [w.gen_small(s) for s in range(10)]
    _same(chk.check_batch(items), o2.check_many(items, jobs=10), items)


def test_big_phase_path(chk):
    # phases with more events than one LDS tile: emitted to HBM and
    # partitioned by index bits; a hot cell makes a single-index group
    items = []
    for s in range(3):
        t, _ = w.gen_large(s, n=4096, lo_prod=2, hi_prod=6)
        items.append((t, 4096))
    items += [("(foru x 0 3 (seq (wr 5) (rd (+ tid x))))", 9000),           # 27000 events on cell 5
              ("(seq (rd 77) (if (= tid 8191) (wr 77) (skip)))", 20000),    # last reader writes
              ("(seq (wr tid) (rd (mod (* tid 7) 20011)))", 20011),
              ("(rd 0)", 30000),                                           # index_bits 0, read only
              ("(seq (rd 0) (if (= tid 29999) (wr 0) (skip)))", 30000),
              ("(fors x 0 3 (seq (wr (+ (* tid 3) x)) (sync) (rd (+ (* tid 3) x))))", 12000)]
    items += [w.tree_protocol(16, r) for r in (None, 0, 3, 14, 15)]
    _same(chk.check_batch(items), o2.check_many(items, jobs=8), items)


def test_thread_limit_guards(chk):
    # leaves `if tid < e {..} else {no access}` run only the tids below e
    items = [("(if (<= tid 3) (wr (mod tid 2)) (skip))", 9),
             ("(fors l 0 5 (seq (if (> (>> 16 l) tid) (wr (+ tid 1)) (skip)) (sync)))", 20),
             ("(fors l 0 5 (if (> (>> 16 l) tid) (wr (+ tid 1)) (skip)))", 20),
             ("(if (< tid 0) (wr 0) (skip))", 300),
             ("(if (< tid 100000) (wr (mod tid 1000)) (foru x 0 3 (skip)))", 4000),
             ("(fors x 0 3 (if (>= (* x 300) tid) (rd (mod tid 7)) (skip)))", 1000),
             ("(fors x 0 40 (seq (if (< tid (* x 700)) (wr (+ (* x 100000) tid)) (skip)) (rd (+ (* x 100000) 5))))", 30000)]
    _same(chk.check_batch(items), o2.check_many(items, jobs=8), items)


def test_packed_fused_groups(chk):
    # many small phases per fused group (packed keys), racy in a late phase
    items = [("(fors x 0 500 (seq (wr (+ (* tid 4) (mod x 4))) (sync) (rd (+ (* (mod (+ tid 1) 50) 4) (mod x 4))) (sync)))", 50),
             ("(fors x 0 300 (seq (wr (+ (* tid 4) (mod x 4))) (rd (+ (* (mod (+ tid 1) 50) 4) (mod (+ x 1) 4))) (sync)))", 50),
             ("(fors x 0 300 (seq (wr (+ (* tid 4) (mod x 4))) (if (= x 277) (rd (+ (* (mod (+ tid 1) 50) 4) (mod x 4))) (skip)) (sync)))", 50)]
    _same(chk.check_batch(items), o2.check_many(items, jobs=8), items)


def test_tree_batch_closed_form(chk):
    import test_oracle as T
    batch = w.gen_tree_batch(0, count=64, kmax=16)
    got = chk.check_batch([(t, n) for t, n, _ in batch])
    for (t, n, lab), g in zip(batch, got):
        k = n.bit_length() - 1
        removed = None if lab == "drf" else int(lab.split("@")[1])
        racy, wit, counts = T.tree_expect(k, removed)
        assert (g.status, g.racy, g.witness, list(g.phase_counts)) == (0, racy, wit, counts), lab


def test_mixed_batch_subset(chk):
    batch = w.gen_mixed_batch(0, count=256)
    items = [(t, n) for t, n, _ in batch]
    got = chk.check_batch(items)
    # oracle on the ones it finishes quickly
    small = [i for i, (t, n) in enumerate(items) if got[i].num_records < 3_000_000]
    want = o2.check_many([items[i] for i in small], jobs=16)
    _same([got[i] for i in small], want, [items[i] for i in small])
    for (t, n, lab), g in zip(batch, got):
        assert g.status == 0 and g.racy == (lab != "drf"), lab


BIGCELL = "(+ (* x 33554432) (mod tid 16))"   # eight threads a cell, phases 2^25 apart


def test_decision_fallbacks(chk):
    # one group whose survivors hold more distinct cells than the LDS hash
    # table takes (each cell read twice by one thread): the survivors are
    # sorted instead; then the same with a race at cell 3
    items = [("(seq (rd (* tid 3)) (rd (* tid 3)))", 4096),
             ("(seq (rd (* tid 3)) (rd (* tid 3)) (if (= tid 0) (wr 3) (skip)))", 4000),
             # packed groups whose cells span more than 2^32 (phase above a
             # 31-bit index): repeated cells are sorted without the hash table
             ("(fors x 0 64 (seq (rd (* x 33554432)) (sync)))", 2),
             ("(fors x 0 64 (seq (if (= tid 1) (wr (* x 33554432)) (rd (* x 33554432))) (sync)))", 2),
             # the same with a full group (64 phases of 128 records, 8192
             # sorted at once), race free and racy at phase 50 only
             ("(fors x 0 64 (seq (rd %s) (sync)))" % BIGCELL, 128),
             ("(fors x 0 64 (seq (if (= x 50) (if (= tid 3) (wr %s) (rd %s)) (rd %s)) (sync)))" % (BIGCELL, BIGCELL, BIGCELL),
              128)]
    got = chk.check_batch(items)
    _same(got, o2.check_many(items, jobs=4), items)
    assert [g.racy for g in got] == [0, 1, 0, 1, 0, 1]
    assert got[5].witness == (50, 50 * 33554432 + 3, 3, 19)


def test_multi_block_items(chk):
    # leaves with a data-dependent branch (interpreted, not compiled) whose
    # count / emit items span many 256-tid blocks, through the HBM path
    # (phases of 65,536 records) and the fused path; racy and race free
    items = [("(fors x 0 4 (seq (if (< (mod tid 3) 1) (wr tid) (rd (+ tid 1))) (sync)))", 65536),
             ("(fors x 0 4 (seq (if (< (mod tid 3) 1) (wr (* tid 2)) (rd (+ (* tid 2) 1))) (sync)))", 65536),
             ("(fors x 0 3 (seq (if (= (mod tid 7) 0) (wr (+ tid x)) (skip)) (sync)))", 3000)]
    got = chk.check_batch(items)
    _same(got, o2.check_many(items, jobs=4), items)
    assert [g.racy for g in got] == [1, 0, 0]


def test_table_path_on_dense_big_phases():
    """Big phases decided by cell tables (table_bits on) against the C
    oracle: dense phases with races at the first, a middle and the last
    cell, read-only sharing, same-thread repeats, writers only, several
    table phases per protocol and several protocols per wave, and a
    protocol too sparse for a table next to them."""
    from paper_2203_12878_amd import drf
    items = [
        ("(wr (mod tid 4096))", 65536),                                   # every cell written by 16 threads
        ("(seq (rd (mod tid 8192)) (if (= tid 40000) (wr 5000) (skip)))", 65536),   # one writer in a read phase
        ("(seq (rd (mod tid 8192)) (if (= tid 8191) (wr 8191) (skip)))", 16384),    # race at the last cell
        ("(seq (rd (mod tid 2048)) (sync) (wr (mod (* tid 3) 2048)))", 20000),
        ("(foru x 0 4 (wr (+ (* (/ tid 4) 4) x)))", 65536),                # four threads write the same four cells
        ("(fors x 0 3 (seq (wr (mod (+ tid x) 4096)) (sync)))", 4096),    # own cells, DRF, three table phases
        ("(fors x 0 3 (seq (wr (mod (+ tid x) 4096)) (rd (mod (+ tid 1) 4096)) (sync)))", 4096),   # racy
        ("(rd (mod tid 1024))", 50000),                                   # read-only sharing: DRF
        ("(wr (* tid 97))", 30000),                                       # sparse: partitioned
        # values beyond 2^32 (the 64-bit evaluator) in dense phases
        ("(wr (mod (* tid 4294967311) 4096))", 65536),
        ("(seq (rd (mod (* tid 8589934597) 2048)) (if (= tid 7) (wr 5) (skip)))", 8192),
    ]
    want = o2.check_many(items, jobs=8)
    chk = drf.Checker(0)
    for bits in (255, 24, 12):
        chk.set_tuning(table_bits=bits)
        got = chk.check_batch(items)
        for it, g, e in zip(items, got, want):
            assert g.key() == e.key(), (bits, it, g, e)
    chk.close()
    assert sum(e.racy for e in want) >= 4
