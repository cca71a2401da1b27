"""BabyCUDA front end (host code of the library, no GPU) and Theorem 1 as a
property test, against the oracle's interpreter of programs with data
(oracle/baby.py).

* The paper's programs (tests/golden/babycuda_examples.json): the inferred
  protocols are the types Section 4 prints; the ill-typed example is
  rejected; the data interpreter reproduces the history example of
  Section 3 exactly and finds its race.
* The data interpreter is pinned by hand-derived closed forms of rule read
  (lastwrite sees the thread's own current-phase writes, not other
  threads', and earlier phases from the most recent) and rule par.
* Theorem 1: for random well-typed programs, every phase's access values
  i:o[j] of the program's history equal those of its inferred protocol
  (per array), and the history is DRF exactly when the protocol is, with
  the same least witness.
* Every generated ill-typed program is rejected; unbound names and binders
  that are not fresh are reported."""
import json
import os
import re

import pytest

from oracle import baby, multi, ref
from paper_2203_12878_amd import drf, workloads as w

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def examples():
    with open(os.path.join(GOLDEN, "babycuda_examples.json")) as f:
        return json.load(f)["cases"]


def bind(text, params):
    for k, v in params.items():
        text = re.sub(r"(?<![\w:])%s(?![\w])" % re.escape(k), str(v), text)
    return text


@pytest.mark.parametrize("case", [c for c in examples() if "protocol" in c], ids=lambda c: c["name"])
def test_paper_programs_get_the_printed_types(case):
    st, proto = drf.infer(case["program"], case["params"])
    assert st == case["status"]
    assert proto == case["protocol"]


def test_history_example_of_section_3():
    case = [c for c in examples() if c["name"] == "history_example"][0]
    hist = baby.run(case["program"], case["n"])
    want = [{int(t): {"": (set(r), dict((j, v) for j, v in wr))} for t, (r, wr) in ph.items()}
            for ph in case["history"]]
    assert hist == want
    assert baby.racy_witness(hist) == tuple(case["witness"])
    # and its protocol agrees (Theorem 1 on this program)
    st, proto = drf.infer(case["program"])
    assert st == 0
    r = ref.check_literal(proto, case["n"])
    assert r.witness == tuple(case["witness"])


def test_lastwrite_closed_forms():
    init = [{0: {"": (set(), {0: 7, 1: 8})}}]
    # own write in the current phase is seen: thread t writes 50+t at 0,
    # then reads 0 and writes what it read at index 10+t
    h = baby.run("(seq (wr 0 (+ 50 tid)) (rd y 0 (wr (+ 10 tid) y)))", 3, initial=init)
    assert [h[0][t][""][1][10 + t] for t in range(3)] == [50, 51, 52]
    # another thread's write in the same phase is hidden (rule par): thread
    # 1 reads index 1 which thread 0 writes in this phase -> the earlier 8
    h = baby.run("(seq (if (= tid 0) (wr 1 99) (skip)) (if (= tid 1) (rd y 1 (wr 5 y)) (skip)))", 2, initial=init)
    assert h[0][1][""][1][5] == 8
    # ... but after a barrier it is seen (the most recent phase first)
    h = baby.run("(seq (if (= tid 0) (wr 1 99) (skip)) (sync) (if (= tid 1) (rd y 1 (wr 5 y)) (skip)))", 2,
                 initial=init)
    assert h[1][1][""][1][5] == 99
    # nothing ever written: undefined, and an undefined payload stays so
    h = baby.run("(rd y 3 (wr (+ 20 tid) (+ y 1)))", 2, initial=init)
    assert h[0][0][""][1][20] is None
    # a read's value never changes which accesses happen (well typed)
    h1 = baby.run("(rd y 0 (wr tid y))", 4, initial=init)
    h2 = baby.run("(rd y 0 (wr tid y))", 4, initial=[{0: {"": (set(), {0: 1234})}}])
    assert [baby.access_values(p) for p in h1] == [baby.access_values(p) for p in h2]


def test_divergent_barriers_are_rejected_by_the_interpreter():
    with pytest.raises(baby.Diverged):
        baby.run("(if (= tid 0) (sync) (skip))", 2)


def _names_in_order(proto):
    names = []
    for _, nm in re.findall(r"\((rd|wr)(?::(\w+))? ", proto):
        if nm not in names:
            names.append(nm)
    return names or [""]


INIT = [{0: {"": (set(), {i: 100 + i for i in range(8)}), "B": (set(), {i: 200 + i for i in range(8)})}}]


@pytest.mark.parametrize("chunk", range(4))
def test_theorem_1_on_random_programs(chunk):
    for seed in range(chunk * 100, chunk * 100 + 100):
        prog, n, params = w.gen_babycuda(seed)
        st, proto = drf.infer(prog, list(params))
        assert st == 0, prog
        hist = baby.run(prog, n, params, initial=INIT)
        concrete = bind(proto, params)
        stmt, na = multi.parse(concrete)
        names = _names_in_order(proto)
        assert len(names) == na
        for a, name in enumerate(names):
            pa = multi.array_protocol(stmt, a)
            phases = ref.expand(pa, n)
            assert len(phases) == len(hist), prog
            for k, (ev, ph) in enumerate(zip(phases, hist)):
                lam = {(t, o, j) for (t, o, j) in ev}
                src = {(t, o, j) for (t, o, arr, j) in baby.access_values(ph) if arr == name}
                assert lam == src, (prog, name, k)
            # DRF of the history iff DRF of the protocol, same least witness
            r = ref.check_literal(pa, n)
            assert r.witness == baby.racy_witness(hist, name), (prog, name)


def test_ill_typed_programs_are_rejected():
    for seed in range(200):
        prog, n, params = w.gen_babycuda(seed, ill_typed=True)
        st, proto = drf.infer(prog, list(params))
        assert st == drf.E_ILLTYPED and proto is None, prog


def test_other_typing_statuses_and_syntax():
    assert drf.infer("(wr k 0)")[0] == drf.E_UNBOUND                # k never bound
    assert drf.infer("(wr 0 k)")[0] == drf.E_UNBOUND                # nor in a payload
    assert drf.infer("(for x 0 2 (for x 0 2 (skip)))")[0] == drf.E_SHADOW
    assert drf.infer("(rd y 0 (rd y 1 (skip)))")[0] == drf.E_SHADOW
    assert drf.infer("(for tid 0 2 (skip))")[0] == drf.E_SHADOW
    assert drf.infer("(for x 0 M (wr x 0))", ["M"])[0] == 0
    assert drf.infer("(for x 0 M (wr x 0))")[0] == drf.E_UNBOUND
    # the first violation in program order decides
    assert drf.infer("(seq (wr k 0) (rd y 0 (wr y 1)))")[0] == drf.E_UNBOUND
    assert drf.infer("(seq (rd y 0 (wr y 1)) (wr k 0))")[0] == drf.E_ILLTYPED
    for bad in ["(wr 0)", "(rd y 0)", "(for x 0 (skip))", "(seq (wr 0 1)", "(wr 0 1) (skip)", "(foo)"]:
        with pytest.raises(drf.DrfError):
            drf.infer(bad)


def test_synchronized_loops_become_fors():
    st, proto = drf.infer("(for l 0 3 (seq (rd:A a tid (wr:B tid a)) (sync)))")
    assert st == 0 and proto.startswith("(fors l 0 3")
    st, proto = drf.infer("(for l 0 3 (wr tid l))")
    assert st == 0 and proto.startswith("(foru l 0 3")


def _theorem_1_holds(prog, n, params, proto):
    hist = baby.run(prog, n, params, initial=INIT)
    stmt, na = multi.parse(bind(proto, params))
    for a, name in enumerate(_names_in_order(proto)):
        if a >= na:
            return False
        phases = ref.expand(multi.array_protocol(stmt, a), n)
        if len(phases) != len(hist):
            return False
        for ev, ph in zip(phases, hist):
            if {(t, o, j) for (t, o, j) in ev} != {(t, o, j) for (t, o, arr, j) in baby.access_values(ph)
                                                  if arr == name}:
                return False
    return True


@pytest.mark.parametrize("mistake", ["read_dropped", "read_as_write", "loop_one_short", "guard_negated"])
def test_planted_inference_mistakes_break_theorem_1(mistake):
    # a plausible mistake in the inferred protocol is caught by the property
    mutate = {
        "read_dropped": lambda p: re.sub(r"\(rd(:\w+)? ", r"(skip_", p, count=1),
        "read_as_write": lambda p: re.sub(r"\(rd(:\w+)? ", r"(wr\1 ", p, count=1),
        "loop_one_short": lambda p: re.sub(r"\(foru (\w+) 0 (\d+) ", lambda m: "(foru %s 0 (- %s 1) " %
                                           (m.group(1), m.group(2)), p, count=1),
        "guard_negated": lambda p: re.sub(r"\(if (\([^()]*(\([^()]*\)[^()]*)*\)) ", r"(if (not \1) ", p, count=1),
    }[mistake]
    caught = 0
    for seed in range(120):
        prog, n, params = w.gen_babycuda(seed)
        st, proto = drf.infer(prog, list(params))
        bad = mutate(proto)
        if bad == proto:
            continue
        if "(skip_" in bad:       # drop the whole read access
            i = bad.index("(skip_")
            depth, j = 0, i
            while True:
                depth += bad[j] == "("
                depth -= bad[j] == ")"
                if depth == 0:
                    break
                j += 1
            bad = bad[:i] + "(skip)" + bad[j + 1:]
        assert _theorem_1_holds(prog, n, params, proto)
        caught += not _theorem_1_holds(prog, n, params, bad)
    assert caught >= 5
