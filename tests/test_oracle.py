"""Pins for the CPU oracle: it is checked against things other than itself.

* the paper's worked examples (tests/golden/paper_examples.json);
* closed forms derived by hand from Definition 1 (tree reduction, constant
  write, own-slot write, write/read ring with and without a barrier);
* natural-number conventions observed through race verdicts;
* the three formulations O1 (pairwise, direct interpreter), O2 (C
  aggregate) and O3 (split into unsynchronized fragments by substitution)
  agree on an exhaustive enumeration of small protocols;
* metamorphic invariants of Definition 1;
* planted mistakes in the oracle are caught by the pins above.
"""
import json
import os
import random

import pytest

from oracle import o2, ref
from paper_2203_12878_amd import workloads as w

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NONE = None


def o2_check(text, n):
    return o2.check(text, n)


ORACLES = {"O1": ref.check_literal, "O3": ref.check_split, "O2": o2_check}


def _expect_ok(res, racy, witness, counts):
    return res.status == 0 and res.racy == racy and res.witness == witness and \
        list(res.phase_counts) == list(counts) and res.num_records == sum(counts)


# ------------------------------------------------------------ paper examples
def load_golden():
    with open(os.path.join(GOLDEN, "paper_examples.json")) as f:
        return json.load(f)["cases"]


def golden_failures(check):
    bad = []
    for c in load_golden():
        r = check(c["text"], c["n"])
        e = c["expect"]
        if r.status != e["status"]:
            bad.append(c["name"])
            continue
        if e["status"] != 0:
            continue
        wit = tuple(e["witness"]) if e["witness"] is not None else None
        if not _expect_ok(r, e["racy"], wit, e["phase_counts"]):
            bad.append(c["name"])
    return bad


@pytest.mark.parametrize("name", list(ORACLES))
def test_paper_examples(name):
    assert golden_failures(ORACLES[name]) == []


# -------------------------------------------------------------- closed forms
def tree_expect(k, removed):
    """Tree reduction over N = 2^k threads (level l: s = N >> (l+1); threads
    tid < s read tid and tid+s and write tid; sync after each level).
    All syncs: race free, counts 3s per level plus a trailing empty phase.
    Sync after level l* < k-1 removed: levels l* and l*+1 share a phase;
    thread 0 reads s2 = N >> (l*+2) at level l*+1 while thread s2 writes it
    at level l*; every smaller index is touched by one thread only.
    Sync after the last level removed: race free, no trailing phase."""
    N = 1 << k
    per = [3 * (N >> (l + 1)) for l in range(k)]
    if removed is None:
        return 0, None, per + [0]
    if removed == k - 1:
        return 0, None, per
    counts = per[:removed] + [per[removed] + per[removed + 1]] + per[removed + 2:] + [0]
    s2 = N >> (removed + 2)
    return 1, (removed, s2, 0, s2), counts


def closed_form_cases():
    cases = []
    for k in range(1, 7):
        for removed in [None] + list(range(k)):
            t, n = w.tree_protocol(k, removed)
            racy, wit, counts = tree_expect(k, removed)
            cases.append(("tree k=%d rm=%s" % (k, removed), t, n, racy, wit, counts))
    for n in (0, 1, 2, 5):
        c = 7
        # one constant cell written by every thread: racy iff two threads exist
        cases.append(("const n=%d" % n, "(wr %d)" % c, n, int(n >= 2),
                      (0, c, 0, 1) if n >= 2 else None, [n]))
        # every thread writes its own cell
        cases.append(("own n=%d" % n, "(wr tid)", n, 0, None, [n]))
        # read-only sharing never races (a race needs a write)
        cases.append(("readonly n=%d" % n, "(seq (rd 0) (rd tid))", n, 0, None, [2 * n]))
        for K in (0, 1, 2, 3):
            # ring: write own cell, barrier, read the next thread's cell, barrier
            ring = "(fors x 0 %d (seq (wr tid) (sync) (rd (mod (+ tid 1) %d)) (sync)))" % (K, max(n, 1))
            cases.append(("ring n=%d K=%d" % (n, K), ring, n, 0, None, [n] * (2 * K) + [0]))
            # without the second barrier the reads of iteration x share a
            # phase with the writes of iteration x+1: thread n-1 reads cell 0,
            # which thread 0 writes
            ring2 = "(fors x 0 %d (seq (wr tid) (sync) (rd (mod (+ tid 1) %d))))" % (K, max(n, 1))
            racy = int(K >= 2 and n >= 2)
            counts = [n] + [2 * n] * (K - 1) + [n] if K >= 1 else [0]
            cases.append(("ring-nosync n=%d K=%d" % (n, K), ring2, n, racy,
                          (1, 0, 0, n - 1) if racy else None, counts))
    for M in (0, 1, 2, 3):
        for n in (1, 2, 3):
            racy = int(M >= 1 and n >= 2)
            cases.append(("rdwr-loop M=%d n=%d" % (M, n), "(foru x 0 %d (seq (rd x) (wr x)))" % M, n,
                          racy, (0, 0, 0, 1) if racy else None, [2 * M * n]))
    # natural-number conventions, observed through verdicts
    cases += [
        ("monus", "(wr (- tid 1))", 2, 1, (0, 0, 0, 1), [2]),             # 0-1 = 0
        ("monus2", "(wr (- 1 tid))", 3, 1, (0, 0, 1, 2), [3]),            # 1,0,0
        ("div0-drf", "(wr (/ 5 tid))", 3, 0, None, [3]),                  # 0,5,2
        ("div0-racy", "(wr (/ 5 tid))", 6, 1, (0, 1, 3, 4), [6]),         # 0,5,2,1,1,1
        ("mod0-drf", "(wr (mod 7 tid))", 3, 0, None, [3]),                # 7,0,1
        ("mod0-racy", "(wr (mod 7 tid))", 8, 1, (0, 0, 1, 7), [8]),       # 7,0,1,1,3,2,1,0
        ("shr-drf", "(wr (>> 8 tid))", 5, 0, None, [5]),                  # 8,4,2,1,0
        ("shr-racy", "(wr (>> 8 tid))", 6, 1, (0, 0, 4, 5), [6]),
        ("shl", "(wr (<< 1 tid))", 32, 0, None, [32]),
        ("min", "(wr (min tid 2))", 4, 1, (0, 2, 2, 3), [4]),
        ("max", "(rd (max tid 2))", 4, 0, None, [4]),
        ("halfopen", "(foru x 2 4 (wr (+ (* tid 10) x)))", 3, 0, None, [6]),
        ("guard-and", "(if (and (< tid 3) (>= tid 1)) (wr 0) (skip))", 5, 1, (0, 0, 1, 2), [2]),
        ("guard-or-not", "(if (or (= tid 0) (not (< tid 4))) (wr 9) (rd 9))", 5, 1, (0, 9, 0, 1), [5]),
        ("sync-free-fors", "(fors x 0 3 (wr (+ tid x)))", 2, 1, (0, 1, 0, 1), [6]),
        ("empty-phases", "(seq (sync) (sync) (wr tid))", 2, 0, None, [0, 0, 2]),
        ("seq-reuse", "(seq (fors x 0 2 (wr (+ (* 2 tid) x))) (fors x 0 2 (rd (+ (* 2 tid) x))))", 2, 0, None, [8]),
        # relations at their boundary values: the guarded threads are the
        # writers, so the verdict and the count name exactly which tids pass
        ("le-two", "(if (<= tid 1) (wr 0) (skip))", 3, 1, (0, 0, 0, 1), [2]),        # tids 0, 1
        ("le-one", "(if (<= tid 0) (wr 0) (skip))", 3, 0, None, [1]),                # tid 0 only
        ("le-rev", "(if (<= 2 tid) (wr 6) (rd tid))", 4, 1, (0, 6, 2, 3), [4]),      # tids 2, 3 write
        ("ne", "(if (!= tid 1) (wr 5) (skip))", 3, 1, (0, 5, 0, 2), [2]),            # tids 0, 2
        ("ne-none", "(if (!= tid tid) (wr 5) (rd 5))", 3, 0, None, [3]),             # never true
        ("gt", "(if (> tid 1) (wr 3) (skip))", 4, 1, (0, 3, 2, 3), [2]),             # tids 2, 3
        ("gt-one", "(if (> tid 2) (wr 3) (rd 4))", 4, 0, None, [4]),                 # tid 3 alone writes
        ("gt-rev", "(if (> 1 tid) (wr 3) (rd 3))", 3, 1, (0, 3, 0, 1), [3]),         # tid 0 writes, 1, 2 read
        # the literal false
        ("false", "(if false (wr 0) (rd 0))", 3, 0, None, [3]),
        ("not-false", "(if (not false) (wr 0) (skip))", 2, 1, (0, 0, 0, 1), [2]),
        ("or-false", "(if (or false (= tid 1)) (wr 4) (rd 4))", 3, 1, (0, 4, 0, 1), [3]),
        ("and-false", "(if (and false true) (wr 4) (rd 4))", 3, 0, None, [3]),
        # values just below the 2^63 limit through * and +: 2^62 mod 7 = 4,
        # (2^63 - 8 + i) mod 5 = i mod 5
        ("mul-below-limit", "(wr (mod (* tid 4611686018427387904) 7))", 2, 0, None, [2]),
        ("add-below-limit", "(wr (mod (+ 9223372036854775800 tid) 5))", 8, 1, (0, 0, 0, 5), [8]),
    ]
    return cases


ERROR_CASES = [
    ("(rd y)", 1, ref.E_UNBOUND),
    ("(fors x 0 y (sync))", 1, ref.E_UNBOUND),
    ("(if (< z 1) (skip) (skip))", 1, ref.E_UNBOUND),
    ("(fors x 0 2 (fors x 0 2 (wr x)))", 1, ref.E_SHADOW),
    ("(foru tid 0 1 (skip))", 1, ref.E_SHADOW),
    ("(foru x 0 2 (foru x 0 1 (skip)))", 1, ref.E_SHADOW),
    ("(if true (sync) (skip))", 1, ref.E_SYNC_IN_U),
    ("(foru x 0 2 (fors y 0 1 (skip)))", 1, ref.E_SYNC_IN_U),
    ("(fors x 0 tid (sync))", 1, ref.E_DIVERGENT),
    ("(fors x (+ tid 1) 3 (skip))", 0, ref.E_DIVERGENT),
    ("(seq (rd y) (if true (sync) (skip)))", 1, ref.E_UNBOUND),    # first violation wins
    ("(seq (if true (sync) (skip)) (rd y))", 1, ref.E_SYNC_IN_U),
    ("(wr 4294967296)", 1, ref.E_RANGE),                            # index limit 2^32
    ("(wr (<< 1 tid))", 33, ref.E_RANGE),
    ("(wr (- 9223372036854775808 9223372036854775800))", 1, ref.E_RANGE),  # value limit 2^63
    ("(fors x 0 9223372036854775808 (sync))", 0, ref.E_RANGE),     # for^S bounds checked once, even with no thread
    ("(if (or true (< (<< 1 100) 1)) (wr 0) (skip))", 1, ref.E_RANGE),  # both operands evaluated
    ("(if (< tid 1) (wr 0) (wr (* tid 4294967296)))", 1, 0),          # untaken branch is not evaluated
    ("(wr (mod (* tid 4611686018427387904) 7))", 3, ref.E_RANGE),    # 2 * 2^62 reaches 2^63
    ("(wr (mod (+ 9223372036854775800 tid) 5))", 9, ref.E_RANGE),    # 2^63 - 8 + 8
    ("(if (< tid 2) (wr (mod (* tid 4611686018427387904) 7)) (skip))", 3, 0),   # guarded below the limit
    ("(wr 4294967295)", 1, 0),
    ("(wr (- 9223372036854775807 9223372036854775800))", 1, 0),
]


def closed_form_failures(check):
    bad = []
    for name, t, n, racy, wit, counts in closed_form_cases():
        r = check(t, n)
        if not _expect_ok(r, racy, wit, counts):
            bad.append(name)
    for t, n, st in ERROR_CASES:
        if check(t, n).status != st:
            bad.append("status " + t)
    return bad


@pytest.mark.parametrize("name", list(ORACLES))
def test_closed_forms(name):
    assert closed_form_failures(ORACLES[name]) == []


def test_closed_forms_o2_batch():
    items = [(t, n) for _, t, n, *_ in closed_form_cases()]
    res = o2.check_many(items, jobs=4)
    for (name, t, n, racy, wit, counts), r in zip(closed_form_cases(), res):
        assert _expect_ok(r, racy, wit, counts), name


# ---------------------------------------------------------------- tiny space
def test_tiny_enumeration_three_formulations_agree():
    items = list(w.enumerate_tiny())
    assert len(items) > 50000
    r2 = o2.check_many(items, jobs=8)
    racy = 0
    for (t, n), b in zip(items, r2):
        a = ref.check_literal(t, n)
        assert a.key() == b.key(), (t, n, a, b)
        racy += a.racy
    assert racy > 5000
    # O3 (split) on a seeded subset to bound the time
    rnd = random.Random(0)
    for t, n in rnd.sample(items, 15000):
        assert ref.check_split(t, n).key() == ref.check_literal(t, n).key(), (t, n)


# ---------------------------------------------------------------- invariants
def _random_protocols(count, seed):
    r = random.Random(seed)
    items = list(w.enumerate_tiny(limit_random=3000, seed=seed))
    return [items[r.randrange(len(items))] for _ in range(count)]


def _accesses(stmt, path=()):
    h = stmt[0]
    if h in ("rd", "wr"):
        yield path
    elif h == "seq":
        for i, c in enumerate(stmt[1:]):
            yield from _accesses(c, path + (i + 1,))
    elif h == "if":
        yield from _accesses(stmt[2], path + (2,))
        yield from _accesses(stmt[3], path + (3,))
    elif h in ("foru", "fors"):
        yield from _accesses(stmt[4], path + (4,))


def _replace(stmt, path, new):
    if not path:
        return new
    i = path[0]
    return stmt[:i] + (_replace(stmt[i], path[1:], new),) + stmt[i + 1:]


def _get(stmt, path):
    for i in path:
        stmt = stmt[i]
    return stmt


def _text(stmt):
    return w.to_text(stmt)


def test_invariants():
    for t, n in _random_protocols(1500, 1):
        p = ref.parse(t)
        base = ref.check_literal(p, n)
        if base.status:
            continue
        accs = list(_accesses(p))
        # I3: more threads never remove a race, and the witness only decreases
        big = ref.check_literal(p, n + 1)
        if base.racy:
            assert big.racy and big.witness <= base.witness
        for path in accs:
            a = _get(p, path)
            # I4: deleting an access never creates a race
            r = ref.check_literal(_replace(p, path, ("skip",)), n)
            assert base.racy or not r.racy
            # I5: duplicating an access changes only the counts
            r = ref.check_literal(_replace(p, path, ("seq", a, a)), n)
            assert (r.racy, r.witness) == (base.racy, base.witness)
            # I6: turning a read into a write never removes a race
            if a[0] == "rd":
                r = ref.check_literal(_replace(p, path, ("wr", a[1])), n)
                assert r.racy or not base.racy
        # I2: inserting a sync at the top level never turns DRF into racy
        if p[0] == "seq":
            for i in range(1, len(p) + 1):
                q = p[:i] + (("sync",),) + p[i:]
                r = ref.check_literal(q, n)
                assert base.racy or not r.racy
                assert r.num_records == base.num_records
        # I7: permuting the statements of a sync-free sequence changes nothing
        if p[0] == "seq" and not ref._has_s(p):
            q = ("seq",) + tuple(reversed(p[1:]))
            assert ref.check_literal(q, n).key() == base.key()


def test_batch_result_equals_single():
    # I8 on the C oracle: a protocol's result does not depend on its batch
    items = _random_protocols(400, 2)
    together = o2.check_many(items, jobs=4)
    alone = [o2.check(t, n) for t, n in items[:40]]
    assert [r.key() for r in together[:40]] == [r.key() for r in alone]


# ------------------------------------------------------------ generators
def test_small_config_three_formulations():
    for seed in range(3):
        t, n = w.gen_small(seed)
        a = ref.check_literal(t, n)
        assert a.phase_counts == [4096] * 16 + [0]
        assert o2.check(t, n).key() == a.key()
        if seed == 0:
            assert ref.check_split(t, n).key() == a.key()


def test_large_config_shrunk():
    # the large generator with few threads and small loops: O1 == O2
    for seed in range(4):
        t, _ = w.gen_large(seed, n=24, lo_prod=1, hi_prod=12)
        assert o2.check(t, 24).key() == ref.check_literal(t, 24).key()


def test_tree_batch_matches_closed_form():
    batch = w.gen_tree_batch(0, count=24, kmax=11)
    res = o2.check_many([(t, n) for t, n, _ in batch], jobs=4)
    for (t, n, lab), r in zip(batch, res):
        k = n.bit_length() - 1
        removed = None if lab == "drf" else int(lab.split("@")[1])
        racy, wit, counts = tree_expect(k, removed)
        assert _expect_ok(r, racy, wit, counts), lab


def test_mixed_batch_labels():
    # race free by construction, or racy by construction
    batch = w.gen_mixed_batch(0, count=64)
    small = [(t, n, lab) for t, n, lab in batch if len(t) < 2000]
    res, _ = o2.check_many([(t, n) for t, n, _ in small], jobs=8, timing=True)
    for (t, n, lab), r in zip(small, res):
        assert r.status == 0
        assert r.racy == (lab != "drf"), (lab, t)


# ------------------------------------------------------ planted mistakes
def _all_failures():
    return golden_failures(ref.check_literal) + closed_form_failures(ref.check_literal)


def test_pins_pass_unmodified():
    assert _all_failures() == []


def _mut_same_thread(k, events, n):
    R = [set() for _ in range(n)]
    W = [set() for _ in range(n)]
    for (i, o, j) in events:
        (W if o == "wr" else R)[i].add(j)
    best = None
    for a in range(n):
        for b in range(a, n):            # mistake: allows a == b
            conf = (W[a] & (R[b] | W[b])) | (W[b] & (R[a] | W[a]))
            if conf:
                cand = (k, min(conf), a, b)
                best = cand if best is None or cand < best else best
    return best


def _mut_read_read(k, events, n):
    R = [set() for _ in range(n)]
    W = [set() for _ in range(n)]
    for (i, o, j) in events:
        (W if o == "wr" else R)[i].add(j)
    best = None
    for a in range(n):
        for b in range(a + 1, n):
            conf = (R[a] | W[a]) & (R[b] | W[b])   # mistake: no write needed
            if conf:
                cand = (k, min(conf), a, b)
                best = cand if best is None or cand < best else best
    return best


def _mut_one_sided(k, events, n):
    R = [set() for _ in range(n)]
    W = [set() for _ in range(n)]
    for (i, o, j) in events:
        (W if o == "wr" else R)[i].add(j)
    best = None
    for a in range(n):
        for b in range(a + 1, n):
            conf = W[a] & (R[b] | W[b])          # mistake: only the lower tid as writer
            if conf:
                cand = (k, min(conf), a, b)
                best = cand if best is None or cand < best else best
    return best


_orig_apply_op = ref.apply_op


def _mut_wrapping_monus(op, a, b):
    if op == "-":
        return ref._chk((a - b) % (1 << 64))
    return _orig_apply_op(op, a, b)


def _mut_div0(op, a, b):
    if op in ("/", "mod") and b == 0:
        return 0 if op == "mod" else a
    return _orig_apply_op(op, a, b)


_orig_run_u = ref._run_u


def _mut_inclusive_loop(u, env, tid, out):
    if u[0] == "foru":
        _, x, lo, hi, body = u
        for v in range(ref.eval_n(lo, env), ref.eval_n(hi, env) + 1):
            e = dict(env)
            e[x] = v
            _mut_inclusive_loop(body, e, tid, out)
        return
    if u[0] in ("seq", "if"):
        if u[0] == "seq":
            for c in u[1:]:
                _mut_inclusive_loop(c, env, tid, out)
        else:
            _mut_inclusive_loop(u[2] if ref.eval_b(u[1], env) else u[3], env, tid, out)
        return
    _orig_run_u(u, env, tid, out)


_orig_expand = ref.expand


def _mut_no_barrier(stmt, n):
    phases = _orig_expand(stmt, n)
    merged = [e for p in phases for e in p]
    return [merged]


def _mut_reversed_phases(stmt, n):
    return list(reversed(_orig_expand(stmt, n)))


_orig_apply_rel = ref.apply_rel


def _mut_le_strict(op, a, b):
    return a < b if op == "<=" else _orig_apply_rel(op, a, b)


def _mut_ne_as_eq(op, a, b):
    return a == b if op == "!=" else _orig_apply_rel(op, a, b)


def _mut_gt_as_ge(op, a, b):
    return a >= b if op == ">" else _orig_apply_rel(op, a, b)


def _mut_swapped_operands(op, a, b):
    return _orig_apply_rel(op, b, a) if op in ("<=", ">") else _orig_apply_rel(op, a, b)


_orig_eval_b = ref.eval_b


def _mut_false_true(c, env):
    if c == "false":
        return True
    if isinstance(c, tuple) and c[0] in ("and", "or", "not"):
        args = [_mut_false_true(x, env) for x in c[1:]]
        return (not args[0]) if c[0] == "not" else (all(args) if c[0] == "and" else any(args))
    return _orig_eval_b(c, env)


def _mut_mul_wraps(op, a, b):
    if op == "*":
        return (a * b) % (1 << 64)            # no value-limit check
    return _orig_apply_op(op, a, b)


def _mut_add_unchecked(op, a, b):
    if op == "+":
        return a + b                          # no value-limit check
    return _orig_apply_op(op, a, b)


@pytest.mark.parametrize("target,mutant", [
    ("_pairwise_witness", _mut_same_thread),
    ("_pairwise_witness", _mut_read_read),
    ("_pairwise_witness", _mut_one_sided),
    ("apply_op", _mut_wrapping_monus),
    ("apply_op", _mut_div0),
    ("_run_u", _mut_inclusive_loop),
    ("expand", _mut_no_barrier),
    ("expand", _mut_reversed_phases),
    ("apply_rel", _mut_le_strict),
    ("apply_rel", _mut_ne_as_eq),
    ("apply_rel", _mut_gt_as_ge),
    ("apply_rel", _mut_swapped_operands),
    ("eval_b", _mut_false_true),
    ("apply_op", _mut_mul_wraps),
    ("apply_op", _mut_add_unchecked),
])
def test_planted_mistake_is_caught(monkeypatch, target, mutant):
    monkeypatch.setattr(ref, target, mutant)
    assert _all_failures() != []
