"""GPU parity at full size: the HIP path (through the C ABI) against oracle
results stored by tests/golden/make_expected.py (which calls only the CPU
oracle), on the full synthetic workloads:

* the plain large protocol (65,536 threads, three nested for^S, 2^24
  cells) for seeds whose protocol writes, through the plain and the
  batched path;
* the whole mixed batch (4096 protocols) and the whole tree-reduction
  batch (2048 instances) in one batched check each, with the big phases
  partitioned and (a second time) with the dense ones decided by tables;
* a served Poisson stream at 5k req/s (1000 requests drawn 70/30 from the
  mixed and tree generators), every request against its stored result;
* a whole mixed batch at another seed against the oracle run in the test.

Every field is compared exactly: status, race flag, witness, record
count, number of phases and the per-phase counts (in full when stored,
else by their sha256 digest)."""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_2203_12878_amd import workloads as w

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _expected(name):
    with open(os.path.join(GOLDEN, "expected_%s.json" % name)) as f:
        return json.load(f)["results"]


def _digest(counts):
    c = counts.tolist() if hasattr(counts, "tolist") else list(counts)
    return hashlib.sha256(" ".join(str(int(x)) for x in c).encode()).hexdigest()


def _mismatches(got, exp):
    assert len(got) == len(exp)
    bad = []
    for i, (g, e) in enumerate(zip(got, exp)):
        same = (g.status, g.racy, list(g.witness) if g.witness else None, g.num_records) == \
            (e["status"], e["racy"], e["witness"], e["num_records"])
        if same and g.status == 0:
            same = len(g.phase_counts) == e["num_phases"] and _digest(g.phase_counts) == e["phase_counts_sha256"]
            if same and e["phase_counts"] is not None:
                same = [int(x) for x in g.phase_counts] == e["phase_counts"]
        if not same:
            bad.append((i, g, e["status"], e["racy"], e["witness"], e["num_records"]))
    return bad


@pytest.fixture(scope="module")
def chk():
    from paper_2203_12878_amd import drf
    c = drf.Checker(0)
    yield c
    c.close()


@pytest.mark.parametrize("seed", [1, 2])
def test_large_protocol_with_writes(chk, seed):
    t, n = w.gen_large(seed)
    exp = _expected("large%d" % seed)
    assert "(wr " in t and exp[0]["num_records"] > 5 * 10 ** 7
    print("large seed %d: %d events" % (seed, exp[0]["num_records"]), flush=True)
    plain = chk.check(t, n)
    assert _mismatches([plain], exp) == []
    batched = chk.check_batch([(t, n)])
    assert _mismatches(batched, exp) == []


@pytest.mark.parametrize("table_bits", [255, 20])
def test_mixed_batch_full(chk, table_bits):
    items = [(t, n) for t, n, _ in w.gen_mixed_batch(0, 4096)]
    exp = _expected("mixed")
    chk.set_tuning(table_bits=table_bits)   # 255: partition path only; 20: dense big phases by tables
    try:
        got = chk.check_batch(items)
    finally:
        chk.set_tuning(table_bits=255)
    bad = _mismatches(got, exp)
    assert not bad, "%d of %d differ, first %r" % (len(bad), len(items), bad[:2])
    assert sum(g.racy for g in got) == sum(e["racy"] for e in exp) > 0


@pytest.mark.parametrize("table_bits", [255, 24])
def test_tree_batch_full(chk, table_bits):
    items = [(t, n) for t, n, _ in w.gen_tree_batch(0, 2048)]
    exp = _expected("tree")
    chk.set_tuning(table_bits=table_bits)
    try:
        got = chk.check_batch(items)
    finally:
        chk.set_tuning(table_bits=255)
    bad = _mismatches(got, exp)
    assert not bad, "%d of %d differ, first %r" % (len(bad), len(items), bad[:2])


def test_mixed_batch_new_seed_live_oracle(chk):
    """A whole mixed batch at a seed with no stored results: every protocol
    below 2e7 events (about 3.7e9 events in all) against the C oracle run
    now, and every protocol's verdict against the race its generator built
    in (or not)."""
    from oracle import o2
    batch = w.gen_mixed_batch(7, 4096)
    items = [(t, n) for t, n, _ in batch]
    got = chk.check_batch(items)
    sel = [i for i, r in enumerate(got) if r.num_records < 20_000_000]
    assert len(sel) > 3500
    want = o2.check_many([items[i] for i in sel], jobs=16)
    bad = [items[i][0][:80] for i, e in zip(sel, want) if got[i].key() != e.key()]
    assert not bad, "%d of %d differ, first %r" % (len(bad), len(sel), bad[:2])
    assert all(g.status == 0 and g.racy == (lab != "drf") for (t, n, lab), g in zip(batch, got))


def test_served_stream_matches_oracle():
    from paper_2203_12878_amd.server import Server, run_stream
    reqs = w.gen_requests(rate=5000.0, max_requests=1000, horizon_s=1.0)
    exp = _expected("serve5k")
    assert len(reqs) == len(exp) == 1000
    with Server(device=0, workers=4, budget_bytes=8 << 30) as srv:
        got, wall = run_stream(srv, reqs)
        st = srv.stats
    assert st.completed == len(reqs) and st.batches < len(reqs)
    bad = _mismatches(got, exp)
    assert not bad, "%d of %d differ, first %r" % (len(bad), len(reqs), bad[:2])
