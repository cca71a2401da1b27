"""C-ABI boundary on the CPU: the library loads, exports every symbol that
include/drf.h declares, and its host-only calls (text compiler, bytecode
validation and planning) agree with the oracle's static statuses."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import ref
from paper_2203_12878_amd import drf, workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "drf.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|uint64_t|const char \*)\s*(drf_\w+)\s*\(", txt, re.M)))


def test_library_exports_declared_symbols():
    L = drf.lib()
    syms = declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(L, s), s
    assert L.drf_version().startswith(b"libdrf")


def test_compile_rejects_bad_text():
    for bad in ["", "(", "(wr)", "(wr 1 2)", "(foo 1)", "(fors 1 0 2 (skip))", "(wr 18446744073709551616)",
                "(wr (+ 1))", "(if (+ 1 2) (skip) (skip))", "(skip) (skip)"]:
        with pytest.raises(drf.DrfError):
            drf.compile_text(bad)


def test_bytecode_layout():
    c = drf.compile_text("(seq (fors x 0 4 (wr (+ tid x))) (sync))")
    assert c[0] == 0x3150414D and c[1] == 1 and c[3] == len(c) - 4
    # corrupting any word either still decodes or reports E_BYTECODE, never crashes
    rng = np.random.default_rng(0)
    for _ in range(300):
        d = c.copy()
        j = int(rng.integers(0, len(d)))
        d[j] = np.uint32(rng.integers(0, 2**32))
        p = drf.plan(d, 3)
        assert p.status in (0, drf.E_BYTECODE, drf.E_UNBOUND, drf.E_SHADOW, drf.E_SYNC_IN_U,
                            drf.E_DIVERGENT, drf.E_RANGE, drf.E_LIMIT, drf.E_MULTI)
    p = drf.plan(c[:-1], 3)
    assert p.status == drf.E_BYTECODE


def test_static_status_matches_oracle():
    items = list(w.enumerate_tiny(limit_random=2000))[::7]
    import test_oracle as T
    items += [(t, n) for t, n, _ in T.ERROR_CASES]
    for t, n in items:
        o = ref.check_literal(t, n)
        p = drf.plan(t, n)
        if o.status in (0, ref.E_RANGE):
            # range overflow of leaf code is found on the device; of for^S
            # bounds already by the planner
            assert p.status in (0, ref.E_RANGE), (t, n)
            if p.status == 0:
                assert p.num_phases == len(o.phase_counts) or o.status == ref.E_RANGE
                assert p.max_records >= o.num_records
        else:
            assert p.status == o.status, (t, n, p.status, o.status)


def test_plan_of_configs():
    t, n = w.gen_small(0)
    p = drf.plan(t, n)
    assert (p.status, p.num_phases, p.wide) == (0, 17, 0)
    assert p.max_records == 65536 and p.index_bits == 11
    t, n = w.gen_large(0)
    p = drf.plan(t, n)
    assert p.status == 0 and p.wide == 0 and p.index_bits == 24
    t, n = w.tree_protocol(12, None)
    p = drf.plan(t, n)
    assert p.num_phases == 13 and p.index_bits >= 12   # interval bound: tid + s
    # limits are reported, not crashed on
    deep = "(wr 0)"
    for i in range(20):
        deep = "(foru v%d 0 1 %s)" % (i, deep)
    assert drf.plan(deep, 1).status == drf.E_LIMIT


def test_plan_batch_agrees_with_plan_protocol():
    items = [w.gen_small(0), w.gen_large(0), w.tree_protocol(12, None), ("(skip)", 1),
             ("(fors x 0 tid (wr x))", 4), ("(wr (+ tid 1))", 70000)]
    plans, total = drf.plan_batch(items)
    singles = [drf.plan(t, n) for t, n in items]
    fields = [f for f, _ in drf.Plan._fields_]
    for a, b in zip(plans, singles):
        assert [getattr(a, f) for f in fields] == [getattr(b, f) for f in fields]
    call = drf.plan("(skip)", 1).scratch_bytes
    # one call's cost once, plus every protocol's own part
    assert max(p.scratch_bytes for p in singles) <= total <= sum(p.scratch_bytes for p in singles)
    assert total >= call + 0.99 * sum(p.scratch_bytes - call for p in singles)
    # big phases need record buffers: about 20 bytes per event of the large protocol
    big = singles[1]
    assert 16 * big.max_records <= big.scratch_bytes - call <= 24 * big.max_records
    assert singles[0].scratch_bytes - call < (1 << 20)     # every phase fits one LDS tile


def test_context_without_gpu_is_a_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    assert drf.lib().drf_ctx_create(0, 0, ctypes.byref(h)) == drf.E_HIP and not h.value
