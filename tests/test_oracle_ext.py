"""Oracle pins for the extensions beyond one concrete single-array protocol
(CPU only):

* several shared arrays (one behavioural type per array, Section 3,
  Syntax): closed forms derived by hand, where merging the arrays would
  change the verdict, and invariants tying the multi-array oracle to the
  single-array one;
* parameter sweeps: the paper's racy example of Section 2 (a for^U loop up
  to a parameter M over rd[x]; wr[x]) and closed forms in the parameter,
  checked instance by instance through textual substitution.

Each closed form states its derivation; planted mistakes in the oracle
(arrays merged, an access of another array kept) are caught."""
import re

import pytest

from oracle import multi, ref


def key(r):
    return (r.status, r.racy, r.witness, tuple(r.phase_counts), r.num_records)


# ------------------------------------------------------------ several arrays
def test_arrays_separate_a_race_that_one_array_would_have():
    # thread t writes A[t] and reads B[t+1]: A has one writer per cell, B is
    # only read -> both race free.  With one array, thread t-1 reads the cell
    # t writes: racy at index 1 between threads 0 and 1.
    n = 4
    got = multi.check_arrays("(seq (wr:A tid) (rd:B (+ tid 1)))", n)
    assert [key(r) for r in got] == [(0, 0, None, (4,), 4), (0, 0, None, (4,), 4)]
    one = ref.check_literal("(seq (wr tid) (rd (+ tid 1)))", n)
    assert (one.racy, one.witness) == (1, (0, 1, 0, 1))


def test_arrays_write_write_and_read_read():
    # every thread writes A[0] (write-write race, least pair 0,1) and reads
    # B[0] (reads never race)
    got = multi.check_arrays("(seq (wr:A 0) (rd:B 0))", 3)
    assert key(got[0]) == (0, 1, (0, 0, 0, 1), (3,), 3)
    assert key(got[1]) == (0, 0, None, (3,), 3)


def test_arrays_share_phases():
    # the sync splits both arrays' protocols at the same point: A has its 3
    # writes in phase 0, B its 6 reads in phase 1
    got = multi.check_arrays("(seq (wr:A tid) (sync) (rd:B tid) (rd:B 0))", 3)
    assert [tuple(r.phase_counts) for r in got] == [(3, 0), (0, 6)]
    assert [r.racy for r in got] == [0, 0]


def test_unnamed_array_is_numbered_in_order_of_appearance():
    # plain wr names the unnamed array: here it comes second
    got = multi.check_arrays("(seq (rd:X tid) (wr 5))", 2)
    assert len(got) == 2
    assert key(got[0]) == (0, 0, None, (2,), 2)
    assert key(got[1]) == (0, 1, (0, 5, 0, 1), (2,), 2)


def test_statuses_count_against_the_array_that_has_them():
    # an unbound variable in B's index: only B's protocol mentions it;
    # an index of 2^32 in A: only A's protocol evaluates it
    got = multi.check_arrays("(seq (wr:A tid) (rd:B y))", 2)
    assert got[0].status == 0 and got[1].status == ref.E_UNBOUND
    got = multi.check_arrays("(seq (wr:A 4294967296) (rd:B tid))", 2)
    assert got[0].status == ref.E_RANGE and key(got[1]) == (0, 0, None, (2,), 2)


def test_one_named_array_equals_the_single_array_oracle():
    texts = ["(fors x 0 3 (seq (wr (+ tid x)) (sync) (rd (mod (+ tid 1) 5))))",
             "(seq (if (< tid 2) (wr 0) (rd 1)) (foru y 0 2 (rd (* y tid))))",
             "(seq (wr tid) (rd (+ tid 1)))"]
    for t in texts:
        named = re.sub(r"\((rd|wr) ", r"(\1:M ", t)
        for n in (1, 2, 5):
            assert [key(r) for r in multi.check_arrays(named, n)] == [key(ref.check_literal(t, n))]


def test_array_protocols_equal_their_written_out_projection():
    # array a's result equals the single-array oracle on the text where the
    # other arrays' accesses are written as skip
    t = "(fors x 0 2 (seq (wr:P (+ tid x)) (rd:Q (* 2 tid)) (sync) (wr:Q tid) (rd:P 3)))"
    per = {"P": "(fors x 0 2 (seq (wr (+ tid x)) (skip) (sync) (skip) (rd 3)))",
           "Q": "(fors x 0 2 (seq (skip) (rd (* 2 tid)) (sync) (wr tid) (skip)))"}
    for n in (2, 3, 4):
        got = multi.check_arrays(t, n)
        assert key(got[0]) == key(ref.check_literal(per["P"], n))
        assert key(got[1]) == key(ref.check_literal(per["Q"], n))


def test_planted_array_mistakes_are_caught(monkeypatch):
    # merging every array into one would report the A/B closed form racy
    orig = multi.array_protocol
    monkeypatch.setattr(multi, "array_protocol", lambda s, a: orig(_merged(s), 0))
    assert multi.check_arrays("(seq (wr:A tid) (rd:B (+ tid 1)))", 4)[1].racy == 1
    monkeypatch.setattr(multi, "array_protocol", orig)
    # keeping another array's accesses (as reads) would add B's events to A
    def keep_all(s, a):
        if s[0] == "acc":
            return (s[1], s[3])
        return orig(s, a) if s[0] != "seq" else ("seq",) + tuple(keep_all(c, a) for c in s[1:])
    monkeypatch.setattr(multi, "array_protocol", keep_all)
    assert multi.check_arrays("(seq (wr:A tid) (sync) (rd:B tid) (rd:B 0))", 3)[0].phase_counts != [3, 0]


def _merged(s):
    if s[0] == "acc":
        return ("acc", s[1], 0, s[3])
    if s[0] == "seq":
        return ("seq",) + tuple(_merged(c) for c in s[1:])
    if s[0] == "if":
        return ("if", s[1], _merged(s[2]), _merged(s[3]))
    if s[0] in ("foru", "fors"):
        return s[:4] + (_merged(s[4]),)
    return s


# ----------------------------------------------------------- parameter sweeps
def bind(text: str, name: str, v: int) -> str:
    """Textual substitution of a parameter by a numeral (whole tokens)."""
    return re.sub(r"(?<![\w:])%s(?![\w])" % re.escape(name), str(v), text)


RACY_EXAMPLE = "(foru x 0 M (seq (rd x) (wr x)))"


@pytest.mark.parametrize("n", [1, 2, 3, 8])
def test_paper_racy_example_for_every_m(n):
    # Section 2: every thread reads and writes A[x] for x < M.  With two or
    # more threads and M >= 1 threads 0 and 1 both write index 0 (the least
    # index, phase 0); with M = 0 nothing is accessed; one thread never races.
    for m in range(0, 17):
        r = ref.check_literal(bind(RACY_EXAMPLE, "M", m), n)
        assert r.phase_counts == [2 * m * n]
        if m >= 1 and n >= 2:
            assert (r.racy, r.witness) == (1, (0, 0, 0, 1))
        else:
            assert (r.racy, r.witness) == (0, None)


def test_sweep_closed_forms():
    # own cells: thread t writes t*M + x for x < M -> disjoint for every M
    for m in range(0, 12):
        r = ref.check_literal(bind("(foru x 0 M (wr (+ (* tid M) x)))", "M", m), 5)
        assert (r.racy, r.num_records) == (0, 5 * m)
    # one cell past the slot: t writes t*M .. t*M + M, so t and t+1 share
    # t*M + M; least is index M between threads 0 and 1 (M = 0: all write 0)
    for m in range(0, 12):
        r = ref.check_literal(bind("(foru x 0 (+ M 1) (wr (+ (* tid M) x)))", "M", m), 4)
        assert (r.racy, r.witness) == (1, (0, m, 0, 1))
    # a parameter in a for^S bound sets the number of phases: M iterations
    # of (write own cell; sync) -> M + 1 phases, n events in each but the last
    for m in range(0, 9):
        r = ref.check_literal(bind("(fors y 0 M (seq (wr (+ tid y)) (sync)))", "M", m), 3)
        assert r.phase_counts == [3] * m + [0] and r.racy == 0
