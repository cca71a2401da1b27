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
                            drf.E_DIVERGENT, drf.E_RANGE, drf.E_LIMIT)
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
