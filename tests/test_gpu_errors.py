"""Error paths of the C ABI on the GPU, and the scratch limit.

* A scratch limit far below a protocol's plan still gives the oracle's
  result: the big phases are split into waves that fit.
* A phase that cannot fit the limit at all gets status DRF_E_NOMEM while
  the other protocols of the batch are checked exactly; nothing is written
  past the caller's result and count arrays.
* A limit too small for the call's metadata is a call-level DRF_E_NOMEM
  that writes nothing.
* A device that does not exist is DRF_E_HIP at context creation, and
  contexts on the real device keep working.
Expected values come from the CPU oracle (stored results or o2 on the
spot)."""
import ctypes
import json
import os

import pytest

from oracle import o2
from paper_2203_12878_amd import workloads as w

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SENT = 0xAB


def _ctx(limit):
    from paper_2203_12878_amd import drf
    h = ctypes.c_void_p()
    assert drf.lib().drf_ctx_create(0, int(limit), ctypes.byref(h)) == drf.OK
    return h


def _run_guarded(ctx, items, extra=4):
    """drf_check_batch into buffers with `extra` sentinel entries past the
    end of both arrays.  Returns (rc, results, counts, guards intact)."""
    import torch
    from paper_2203_12878_amd import drf
    b = drf.Batch(items, 0)
    res = torch.full(((b.count + extra) * 40,), SENT, dtype=torch.uint8, device="cuda")
    cnt = torch.full(((b.total_phases + extra) * 8,), SENT, dtype=torch.uint8, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = drf.lib().drf_check_batch(ctx, drf._u32p(b.code), drf._u64p(b.code_off), drf._u32p(b.nthreads), b.count,
                                   ctypes.c_void_p(res.data_ptr()), ctypes.c_void_p(cnt.data_ptr()),
                                   b.total_phases, st)
    torch.cuda.synchronize()
    r = res.cpu().numpy()
    c = cnt.cpu().numpy()
    guards = bool((r[b.count * 40:] == SENT).all() and (c[b.total_phases * 8:] == SENT).all())
    b.results.copy_(res[:b.count * 40])
    b.counts.view(torch.uint8).copy_(cnt[:max(1, b.total_phases) * 8] if b.total_phases else cnt[:8])
    return rc, b, r, guards


def test_limit_below_plan_splits_into_waves():
    """Large protocol seed 1 (plan about 2.4 GB of scratch) under a 256 MB
    limit: several waves, same result as the oracle."""
    from paper_2203_12878_amd import drf
    t, n = w.gen_large(1)
    p = drf.plan(t, n)
    assert p.scratch_bytes > 2 * 10 ** 9
    with open(os.path.join(GOLDEN, "expected_large1.json")) as f:
        e = json.load(f)["results"][0]
    ctx = _ctx(256 << 20)
    try:
        rc, b, _, guards = _run_guarded(ctx, [(t, n)])
        assert rc == drf.OK and guards
        g = b.collect()[0]
        assert (g.status, g.racy, list(g.witness), g.num_records) == \
            (e["status"], e["racy"], e["witness"], e["num_records"])
        assert len(g.phase_counts) == e["num_phases"]
    finally:
        drf.lib().drf_ctx_destroy(ctx)


def test_phase_beyond_limit_is_a_status_and_others_are_exact():
    from paper_2203_12878_amd import drf
    items = [w.gen_large(1), w.gen_small(0), w.tree_protocol(14, 5),
             ("(seq (if (= tid 0) (wr 1) (wr 2)) (sync) (if (= tid 1) (rd 0) (skip)) (wr 0))", 2)]
    call = drf.plan("(skip)", 1).scratch_bytes
    # room for the call's metadata and about a tree phase of records, far
    # from the 393,216-record phases of the large protocol
    ctx = _ctx(call + (3 << 20))
    try:
        rc, b, _, guards = _run_guarded(ctx, items)
        assert rc == drf.OK and guards
        got = b.collect()
    finally:
        drf.lib().drf_ctx_destroy(ctx)
    assert got[0].status == drf.E_NOMEM
    want = o2.check_many(items[1:])
    for g, e in zip(got[1:], want):
        assert g.key() == e.key()


def test_limit_below_metadata_is_a_call_error_that_writes_nothing():
    from paper_2203_12878_amd import drf
    items = [w.gen_small(0), w.tree_protocol(12, None)]
    ctx = _ctx(1 << 20)
    try:
        rc, b, r, guards = _run_guarded(ctx, items)
        assert rc == drf.E_NOMEM and guards
        assert (r == SENT).all()          # no result written
    finally:
        drf.lib().drf_ctx_destroy(ctx)


def test_missing_device_is_a_hip_error_and_contexts_still_work():
    import torch
    from paper_2203_12878_amd import drf
    h = ctypes.c_void_p()
    missing = torch.cuda.device_count()
    assert drf.lib().drf_ctx_create(missing, 0, ctypes.byref(h)) == drf.E_HIP and not h.value
    assert drf.lib().drf_ctx_create(-1, 0, ctypes.byref(h)) == drf.E_HIP and not h.value
    items = [w.gen_small(0), w.tree_protocol(12, 3)]
    ctx = _ctx(0)
    try:
        rc, b, _, guards = _run_guarded(ctx, items)
        assert rc == drf.OK and guards
        want = o2.check_many(items)
        assert [g.key() for g in b.collect()] == [e.key() for e in want]
    finally:
        drf.lib().drf_ctx_destroy(ctx)


def test_release_then_reuse():
    """Pools handed back after a check grow again on the next one."""
    from paper_2203_12878_amd import drf
    chk = drf.Checker(0)
    items = [w.gen_large(2, n=8192, lo_prod=4, hi_prod=8), w.gen_small(1)]
    want = o2.check_many(items)
    for _ in range(3):
        got = chk.check_batch(items)
        assert [g.key() for g in got] == [e.key() for e in want]
        chk.release(0)
    chk.close()
