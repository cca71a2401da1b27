"""The allocation-free entry point, drf_check_batch_noalloc, against
drf_check_batch on the same inputs, through the C ABI.

Two calls in a row (the second smaller, so stale contents of the fixed
scratch array from the first would show), each compared field by field
with drf_check_batch: status, race flag, witness, record total and every
per-phase count (tolerance 0: all integers).  The inputs span the fused
path, the count read-back and big phases partitioned in the fixed array
(tree instances of up to 2^17 threads: 196,608 events in their first
phase), and a protocol with one phase too large for the array, which gets
status DRF_E_NOMEM while the others stay exact.
"""
import sys

import pytest

from paper_2203_12878_amd import drf, workloads

pytestmark = pytest.mark.gpu


def _items():
    mixed = [(t, n) for t, n, _ in workloads.gen_mixed_batch(0, 400)]
    small = [it for it in mixed if drf.plan(*it).max_phase_records <= 200_000][:160]
    trees = [(t, n) for t, n, _ in workloads.gen_tree_batch(0, 200) if n <= (1 << 17)][:40]
    items = []
    for i in range(max(len(small), len(trees))):
        if i < len(small):
            items.append(small[i])
        if i < len(trees):
            items.append(trees[i])
    return items


def _run(chk, items, noalloc):
    import torch
    b = drf.Batch(items, 0)
    if noalloc:
        chk.run_batch_noalloc(b)
    else:
        chk.run_batch(b)
    torch.cuda.synchronize()
    return b.collect()


def test_noalloc_equals_batch_on_two_calls():
    items = _items()
    assert len(items) >= 150
    assert any(drf.plan(*it).max_phase_records > 8192 for it in items)   # big phases are exercised
    ref_chk = drf.Checker(0)
    chk = drf.Checker(0)
    try:
        calls = [("first call", items), ("second call, smaller", items[:37])]
        for what, its in calls:
            print("noalloc:", what, len(its), "protocols", flush=True)
            want = _run(ref_chk, its, noalloc=False)
            got = _run(chk, its, noalloc=True)
            assert len(got) == len(want)
            for i, (g, w) in enumerate(zip(got, want)):
                assert g.key() == w.key(), (what, i, g, w)
            assert sum(r.racy for r in got) > 0
    finally:
        chk.close()
        ref_chk.close()


def test_noalloc_phase_beyond_the_array_is_a_status():
    big = ("(wr tid)", 1 << 23)          # one phase of 8,388,608 events: more than the array holds
    items = _items()[:20]
    mixed = items[:10] + [big] + items[10:]
    ref_chk = drf.Checker(0)
    chk = drf.Checker(0)
    try:
        print("noalloc: one phase beyond the fixed array", flush=True)
        got = _run(chk, mixed, noalloc=True)
        want = _run(ref_chk, items, noalloc=False)
        assert got[10].status == drf.E_NOMEM
        rest = got[:10] + got[11:]
        for i, (g, w) in enumerate(zip(rest, want)):
            assert g.key() == w.key(), (i, g, w)
        # a smaller call right after still matches
        again = _run(chk, items[:5], noalloc=True)
        assert [r.key() for r in again] == [r.key() for r in want[:5]]
    finally:
        chk.close()
        ref_chk.close()


if __name__ == "__main__":
    sys.exit(pytest.main([__file__, "-v", "-m", "gpu"]))
