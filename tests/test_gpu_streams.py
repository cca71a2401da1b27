"""The second stream of a context: an ordinary checking call whose counted
small phases and big phases both hold at least 2^24 events decides the
counted small phases on the context's second stream, beside the partition
of the big phases, and folds their witnesses into the call's own before the
results are written.  Recorded (prepared) calls keep one stream.

Here two slices of the mixed batch (512 protocols each, 2.3 G and 2.5 G
access events, so both sides are far above the threshold) are

* checked by ordinary calls enqueued back to back on one stream, without a
  synchronization between them (the second call reuses the first one's
  pools and its second stream), and compared with the stored oracle
  results of the same protocols (a protocol's result does not depend on
  the batch it is checked in);
* checked again as a prepared batch (one stream, replayed graph), which
  must give the same results field for field."""
import hashlib
import json
import os

import pytest

from paper_2203_12878_amd import workloads as w

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _key(r):
    return (r.status, r.racy, tuple(r.witness) if r.witness else None, r.num_records,
            hashlib.sha256(" ".join(str(int(x)) for x in r.phase_counts).encode()).hexdigest())


def _stored(lo, hi):
    with open(os.path.join(GOLDEN, "expected_mixed.json")) as f:
        exp = json.load(f)["results"][lo:hi]
    return [(e["status"], e["racy"], tuple(e["witness"]) if e["witness"] else None, e["num_records"],
             e["phase_counts_sha256"]) for e in exp]


def test_back_to_back_calls_and_prepared_equal_stored():
    import torch
    from paper_2203_12878_amd import drf
    items = [(t, n) for t, n, _ in w.gen_mixed_batch(0, 1024)]
    slices = [(0, 512), (512, 1024)]
    chk = drf.Checker(0)
    try:
        batches = [drf.Batch(items[lo:hi], 0) for lo, hi in slices]
        print("two ordinary calls, 512 protocols each", flush=True)
        for b in batches:
            chk.run_batch(b)
        torch.cuda.synchronize()
        for (lo, hi), b in zip(slices, batches):
            got = [_key(r) for r in b.collect()]
            assert got == _stored(lo, hi), (lo, hi)
            assert sum(k[1] for k in got) > 0
        print("prepared batch of the first slice", flush=True)
        b2 = drf.Batch(items[:512], 0)
        p = drf.Prepared(chk, b2)
        p.run()
        torch.cuda.synchronize()
        assert [_key(r) for r in b2.collect()] == [_key(r) for r in batches[0].collect()]
        p.close()
    finally:
        chk.close()
