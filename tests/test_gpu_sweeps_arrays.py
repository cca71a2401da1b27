"""GPU parity for parameter sweeps and protocols over several shared arrays,
through the C ABI (drf_check_sweep, drf_check_arrays), against the oracle:

* sweeps: every instance p[M := v] against the C oracle on the text with M
  written out as the numeral (the paper's racy loop of Section 2 among
  them); instances differ in their number of phases;
* several arrays: every array's result against the multi-array oracle on
  small protocols, and against the C oracle on the text with the other
  arrays' accesses written as (skip) on generated protocols of up to 512
  threads."""
import re

import pytest

from oracle import multi, o2
from paper_2203_12878_amd import workloads as w

pytestmark = pytest.mark.gpu


def bind(text, name, v):
    return re.sub(r"(?<![\w:])%s(?![\w])" % re.escape(name), str(v), text)


@pytest.fixture(scope="module")
def chk():
    from paper_2203_12878_amd import drf
    c = drf.Checker(0)
    yield c
    c.close()


def test_sweeps_match_instances(chk):
    from paper_2203_12878_amd import drf
    for text, n in w.gen_sweep_protocols():
        slot = drf.text_slot(text, "M")
        first, count = 0, 33
        got = chk.check_sweep(text, n, slot, first, count)
        want = o2.check_many([(bind(text, "M", v), n) for v in range(first, first + count)], jobs=8)
        assert [g.key() for g in got] == [e.key() for e in want], text
    # the racy example: DRF only at M = 0
    got = chk.check_sweep("(foru x 0 M (seq (rd x) (wr x)))", 4, 1, 0, 9)
    assert [g.racy for g in got] == [0] + [1] * 8
    assert all(g.witness == (0, 0, 0, 1) for g in got[1:])


def test_sweep_from_an_offset_and_bound_parameter(chk):
    from paper_2203_12878_amd import drf
    text, n = "(fors y 0 M (seq (wr (+ (* tid M) y)) (sync)))", 16
    slot = drf.text_slot(text, "M")
    got = chk.check_sweep(text, n, slot, 1000, 5)
    want = o2.check_many([(bind(text, "M", v), n) for v in range(1000, 1005)])
    assert [g.key() for g in got] == [e.key() for e in want]
    # a slot that a loop binds is not a parameter
    with pytest.raises(drf.DrfError):
        chk.check_sweep(text, n, drf.text_slot(text, "y"), 0, 3)


SMALL_ARRAYS = [
    ("(seq (wr:A tid) (rd:B (+ tid 1)))", 4),
    ("(seq (wr:A 0) (rd:B 0))", 3),
    ("(seq (wr:A tid) (sync) (rd:B tid) (rd:B 0))", 3),
    ("(seq (rd:X tid) (wr 5))", 2),
    ("(fors x 0 2 (seq (wr:P (+ tid x)) (rd:Q (* 2 tid)) (sync) (wr:Q tid) (rd:P 3)))", 4),
    ("(seq (wr:A tid) (rd:B y))", 2),
    ("(seq (wr:A 4294967296) (rd:B tid))", 2),
    ("(seq (if (< tid 2) (wr:C 1) (rd:D tid)) (foru z 0 3 (seq (rd:C z) (wr:D (+ tid z)))))", 6),
]


def test_small_multi_array_protocols(chk):
    for text, n in SMALL_ARRAYS:
        got = chk.check_arrays(text, n)
        want = multi.check_arrays(text, n)
        assert [g.key() for g in got] == [e.key() for e in want], text


def _written_out(text):
    """One single-array text per array: the other arrays' accesses written
    as (skip) (arrays numbered in order of first appearance)."""
    heads = re.findall(r"\((rd|wr)(?::(\w+))? ", text)
    names = []
    for _, nm in heads:
        if nm not in names:
            names.append(nm)
    out = []
    for keep in names:
        def sub(m):
            mode, nm = m.group(1), m.group(2) or ""
            return "(%s " % mode if nm == keep else "(skip_acc "
        t = re.sub(r"\((rd|wr)(?::(\w+))? ", sub, text)
        # (skip_acc <expr>) -> (skip): drop the balanced expression
        while "(skip_acc " in t:
            i = t.index("(skip_acc ")
            depth, j = 0, i
            while True:
                if t[j] == "(":
                    depth += 1
                elif t[j] == ")":
                    depth -= 1
                    if depth == 0:
                        break
                j += 1
            t = t[:i] + "(skip)" + t[j + 1:]
        out.append(t)
    return out


def test_generated_multi_array_protocols(chk):
    items = w.gen_multi_array(0, 24, arrays=3)
    for text, n in items:
        got = chk.check_arrays(text, n)
        want = o2.check_many([(t, n) for t in _written_out(text)])
        assert [g.key() for g in got] == [e.key() for e in want], text[:120]
    # a race of one array is a race of the protocol with the arrays merged,
    # and on these inputs the split removes some races
    merged = o2.check_many([(re.sub(r"\((rd|wr):\w+ ", r"(\1 ", t), n) for t, n in items], jobs=8)
    split = [chk.check_arrays(t, n) for t, n in items]
    assert all(m.racy or not any(r.racy for r in s) for m, s in zip(merged, split))
    assert any(m.racy and not any(r.racy for r in s) for m, s in zip(merged, split))


def test_multi_array_status_on_the_plain_calls(chk):
    from paper_2203_12878_amd import drf
    r = chk.check("(seq (wr:A tid) (rd:B 0))", 4)
    assert r.status == drf.E_MULTI
