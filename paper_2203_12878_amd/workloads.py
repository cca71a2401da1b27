"""Seeded synthetic memory-access-protocol workloads (text form only).

This module builds protocol ASTs and prints them in the s-expression text
form that both the CPU oracle and the HIP path parse with their own parsers.
It evaluates nothing: no index arithmetic, no phases, no race logic.

Protocol language (the paper's syntax of memory access protocols, with a
``u`` leaf allowed inside synchronized protocols):

  stmt ::= (skip) | (rd E) | (wr E) | (seq S ...) | (if C S S)
         | (foru X E E S) | (sync) | (fors X E E S)
  E    ::= <natural> | tid | X | (OP E E)
           OP in + - * / mod << >> min max   ('-' is truncated subtraction)
  C    ::= true | false | (REL E E) | (and C C) | (or C C) | (not C)
           REL in < <= = != > >=

Loops run over the half-open range lo..hi with stride 1.

Random streams: numpy ``Generator(PCG64(SeedSequence([config_id, ...])))``.
"""
from __future__ import annotations

import itertools
import math
import re
from typing import Iterator, List, Sequence, Tuple

import numpy as np

# ---------------------------------------------------------------- AST helpers
# Statements and expressions are plain nested tuples; ints are naturals,
# 'tid' is the thread id and any other str is a loop variable.


def skip():
    return ("skip",)


def rd(e):
    return ("rd", e)


def wr(e):
    return ("wr", e)


def acc(mode: str, e):
    assert mode in ("rd", "wr")
    return (mode, e)


def seq(*stmts):
    return ("seq",) + tuple(stmts)


def if_(c, then, els=None):
    return ("if", c, then, skip() if els is None else els)


def foru(x: str, lo, hi, body):
    return ("foru", x, lo, hi, body)


def fors(x: str, lo, hi, body):
    return ("fors", x, lo, hi, body)


def sync():
    return ("sync",)


def to_text(node) -> str:
    """Print a statement, expression or condition as an s-expression."""
    if isinstance(node, bool):
        raise TypeError("use 'true'/'false' strings for boolean literals")
    if isinstance(node, (int, np.integer)):
        if node < 0:
            raise ValueError("naturals only")
        return str(int(node))
    if isinstance(node, str):
        return node
    return "(" + " ".join(to_text(c) for c in node) + ")"


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def _sum(terms):
    out = terms[0]
    for t in terms[1:]:
        out = ("+", out, t)
    return out


# ------------------------------------------------------ plain single, small
def gen_small(seed: int = 0) -> Tuple[str, int]:
    """256 threads; fors x in 0..16 { fors y in 0..4 { 4 accesses } ; sync }.

    Each access: index (a*tid + b*x + c*y + d) mod 4096 with a,b,c uniform in
    {0..4}, d uniform in {0..63}; write with probability 0.5.
    """
    r = _rng(0, seed)
    accs = []
    for _ in range(4):
        a, b, c = (int(v) for v in r.integers(0, 5, size=3))
        d = int(r.integers(0, 64))
        mode = "wr" if r.random() < 0.5 else "rd"
        idx = ("mod", _sum([("*", a, "tid"), ("*", b, "x"), ("*", c, "y"), d]), 4096)
        accs.append(acc(mode, idx))
    p = fors("x", 0, 16, seq(fors("y", 0, 4, seq(*accs)), sync()))
    return to_text(p), 256


# ------------------------------------------------------ plain single, large
def gen_large(seed: int = 0, n: int = 65536, lo_prod: int = 128, hi_prod: int = 508):
    """65,536 threads, three nested fors loops with bounds in 1..32 and six
    accesses in the innermost body; each loop body ends with a sync with
    probability 0.7; writes with probability 0.3; index
    (a*tid + b1*x1 + b2*x2 + b3*x3 + d) mod 2^24 with a in {0..255},
    b_i in {0..4095}, d in {0..2^24-1}.  The bounds are redrawn from the
    same stream until their product lies in [lo_prod, hi_prod], which keeps
    the record count near 10^8.
    """
    r = _rng(1, seed)
    while True:
        bounds = [int(v) for v in r.integers(1, 33, size=3)]
        if lo_prod <= bounds[0] * bounds[1] * bounds[2] <= hi_prod:
            break
    syncs = [bool(r.random() < 0.7) for _ in range(3)]
    accs = []
    for _ in range(6):
        mode = "wr" if r.random() < 0.3 else "rd"
        a = int(r.integers(0, 256))
        b = [int(v) for v in r.integers(0, 4096, size=3)]
        d = int(r.integers(0, 1 << 24))
        idx = ("mod", _sum([("*", a, "tid"), ("*", b[0], "x1"), ("*", b[1], "x2"),
                            ("*", b[2], "x3"), d]), 1 << 24)
        accs.append(acc(mode, idx))
    body3 = seq(*accs, sync()) if syncs[2] else seq(*accs)
    l3 = fors("x3", 0, bounds[2], body3)
    body2 = seq(l3, sync()) if syncs[1] else l3
    l2 = fors("x2", 0, bounds[1], body2)
    body1 = seq(l2, sync()) if syncs[0] else l2
    p = fors("x1", 0, bounds[0], body1)
    return to_text(p), n


# ----------------------------------------------------------- batched, mixed
def _mixed_protocol(r: np.random.Generator):
    """One protocol of the mixed batch: returns (text, n, intended_label)."""
    n = int(math.floor(math.exp(r.uniform(math.log(32), math.log(4097)))))
    depth = int(r.integers(1, 4))
    bounds = [int(math.floor(math.exp(r.uniform(0.0, math.log(65))))) for _ in range(depth)]
    A = int(r.integers(2, 9))
    cells = 1 << int(r.integers(12, 21))
    S = cells // n
    xs = [f"x{i + 1}" for i in range(depth)]

    def offset():
        b = [int(v) for v in r.integers(0, 8, size=depth)]
        d = int(r.integers(0, S))
        return ("mod", _sum([("*", bi, x) for bi, x in zip(b, xs)] + [d]), S)

    u = r.random()
    kind = "drf" if u >= 0.2 else ("sync_removed" if u < 0.1 else "stride_collision")
    n_own = (A + 1) // 2
    n_nb = A // 2
    own_offs = [offset() for _ in range(n_own)]
    own_modes = ["wr"] + ["wr" if r.random() < 0.5 else "rd" for _ in range(n_own - 1)]
    own = [acc(m, ("+", ("*", "tid", S), o)) for m, o in zip(own_modes, own_offs)]
    nb_offs = [offset() for _ in range(n_nb)]
    if kind == "sync_removed":
        # one neighbour read lands on an offset the neighbour thread writes
        if n_nb == 0:
            nb_offs = [own_offs[0]]
        else:
            nb_offs[int(r.integers(0, n_nb))] = own_offs[0]
    nb = [rd(("+", ("*", ("mod", ("+", "tid", 1), n), S), o)) for o in nb_offs]
    if kind == "stride_collision":
        # a write one slot past the own slot, beside an own access at offset 0
        pos = int(r.integers(0, len(own)))
        mode0 = "wr" if r.random() < 0.5 else "rd"
        own = own[:pos] + [wr(("+", ("*", "tid", S), S)), acc(mode0, ("*", "tid", S))] + own[pos:]
    if kind == "sync_removed":
        body = seq(*own, *nb, sync())
    else:
        body = seq(*own, sync(), *nb, sync())
    for x, b in reversed(list(zip(xs, bounds))):
        body = fors(x, 0, b, body)
    return to_text(body), n, kind


def gen_mixed_batch(batch_seed: int = 0, count: int = 4096):
    """Mixed batch: thread counts log-uniform in 32..4096, fors depth 1..3
    with bounds log-uniform in 1..64, 2..8 accesses per body into per-protocol
    arrays of 2^12..2^20 cells.  80% are race free by construction (own slot
    of size cells//n per thread, a sync, reads of the neighbour's slot, a
    sync); 10% drop the first sync and read a cell the neighbour writes; 10%
    write one slot past their own.  Returns a list of (text, n, label).
    """
    return [_mixed_protocol(_rng(2, batch_seed, i)) for i in range(count)]


# ------------------------------------------------------ batched, tree shape
def _tree_level(l, N):
    s = (">>", N, ("+", l, 1))
    return if_(("<", "tid", s), seq(rd("tid"), rd(("+", "tid", s)), wr("tid")), skip())


def tree_protocol(k: int, removed_level: int | None = None) -> Tuple[str, int]:
    """Tree reduction over N = 2^k threads: at level l with s = N >> (l+1),
    threads tid < s read A[tid] and A[tid+s] and write A[tid], then sync.
    With removed_level set, the sync after that level is dropped."""
    N = 1 << k
    if removed_level is None:
        p = fors("l", 0, k, seq(_tree_level("l", N), sync()))
    else:
        ls = removed_level
        parts = []
        if ls > 0:
            parts.append(fors("l", 0, ls, seq(_tree_level("l", N), sync())))
        parts.append(_tree_level(ls, N))
        if ls + 1 < k:
            parts.append(fors("l", ls + 1, k, seq(_tree_level("l", N), sync())))
        p = seq(*parts) if len(parts) > 1 else parts[0]
    return to_text(p), N


def _tree_instance(r: np.random.Generator, kmax: int = 20):
    k = int(r.integers(8, kmax + 1))
    removed = bool(r.random() < 0.5)
    ls = int(r.integers(0, k))
    text, n = tree_protocol(k, ls if removed else None)
    return text, n, ("removed@%d" % ls) if removed else "drf"


def gen_tree_batch(batch_seed: int = 0, count: int = 2048, kmax: int = 20):
    """Tree-reduction batch: k uniform in 8..kmax, N = 2^k threads; in half
    of the instances the sync of one uniformly chosen level is removed."""
    return [_tree_instance(_rng(3, batch_seed, i), kmax) for i in range(count)]


# ------------------------------------------------- several arrays, sweeps
def gen_multi_array(seed: int = 0, count: int = 16, arrays: int = 3, max_threads: int = 512):
    """Protocols over several shared arrays: mixed-batch shapes (thread
    counts capped at max_threads) whose accesses are spread uniformly over
    `arrays` named arrays A0.. (text form rd:Ak / wr:Ak).  Returns a list of
    (text, n)."""
    out = []
    for i in range(count):
        r = _rng(5, seed, i)
        while True:
            text, n, _ = _mixed_protocol(r)
            if n <= max_threads:
                break
        parts = re.split(r"\((rd|wr) ", text)
        acc_text = parts[0]
        for j in range(1, len(parts), 2):
            acc_text += "(%s:A%d %s" % (parts[j], int(r.integers(0, arrays)), parts[j + 1])
        out.append((acc_text, n))
    return out


def gen_sweep_protocols():
    """Parametric protocols (free parameter M) and the thread counts they
    run with: the racy loop of the paper's Section 2, own / overlapping
    slots of width M, M synchronized iterations (phases depend on M), and a
    tree-like halving whose stride is M."""
    return [
        ("(foru x 0 M (seq (rd x) (wr x)))", 4),
        ("(foru x 0 M (wr (+ (* tid M) x)))", 64),
        ("(foru x 0 (+ M 1) (wr (+ (* tid M) x)))", 64),
        ("(fors y 0 M (seq (wr (+ tid y)) (sync) (rd (mod (+ tid 1) 32))))", 32),
        ("(if (< tid M) (seq (rd tid) (rd (+ tid M)) (wr tid)) (skip))", 256),
        ("(seq (wr (* tid 3)) (if (< tid (- 64 M)) (rd (+ (* tid 3) (* 3 M))) (skip)))", 64),
    ]


# ------------------------------------------------------- BabyCUDA programs
def gen_babycuda(seed: int, ill_typed: bool = False):
    """A random BabyCUDA program (text form (skip) (sync) (wr n n')
    (rd y n b) (seq ..) (if c b b) (for x n n b), rd:A / wr:A for a second
    array), its thread count and parameter values.  Well typed unless
    ill_typed: then one read-bound variable is used in an index, a guard or
    a loop bound (a data-dependent access).  Returns (text, n, params)."""
    r = _rng(6, seed, int(ill_typed))
    n = int(r.integers(2, 7))
    params = {"M": int(r.integers(0, 4))} if r.random() < 0.5 else {}
    arrays = ["", "B"] if r.random() < 0.3 else [""]
    fresh = itertools.count()
    state = {"planted": False}

    def pick(xs):
        return xs[int(r.integers(0, len(xs)))]

    def small(V):
        terms = [int(r.integers(0, 4))]
        for v in V:
            if r.random() < 0.5:
                terms.append(("*", int(r.integers(0, 3)), v))
        return _sum(terms)

    def index(V, D):
        e = ("mod", small(V), int(r.integers(2, 7)))
        if ill_typed and D and not state["planted"] and r.random() < 0.5:
            state["planted"] = True
            e = ("+", e, pick(D))
        return e

    def payload(V, D):
        return _sum([int(r.integers(0, 9))] + [v for v in V + D if r.random() < 0.3])

    def access(mode, arr):
        return mode + (":" + arr if arr else "")

    def block(V, D, depth):
        k = r.random()
        if depth >= 3 or k < 0.35:
            if r.random() < 0.5 or not V:
                return ("wr_", access("wr", pick(arrays)), index(V, D), payload(V, D))
            y = "y%d" % next(fresh)
            return ("rd_", access("rd", pick(arrays)), y, index(V, D), block(V, D + [y], depth + 1))
        if k < 0.55:
            y = "y%d" % next(fresh)
            return ("rd_", access("rd", pick(arrays)), y, index(V, D), block(V, D + [y], depth + 1))
        if k < 0.75:
            c = (pick(["<", "<=", "=", "!=", ">", ">="]), small(V), small(V))
            if ill_typed and D and not state["planted"] and r.random() < 0.5:
                state["planted"] = True
                c = ("<", pick(D), small(V))
            return ("if", c, block(V, D, depth + 1), block(V, D, depth + 1))
        if k < 0.9:
            x = "x%d" % next(fresh)
            hi = int(r.integers(0, 4))
            hi_e = ("+", hi, pick(D)) if ill_typed and D and not state["planted"] and r.random() < 0.3 else hi
            if hi_e is not hi:
                state["planted"] = True
            return ("for", x, 0, hi_e, block(V + [x], D, depth + 1))
        return ("seq", block(V, D, depth + 1), block(V, D, depth + 1))

    V0 = ["tid"] + list(params)
    parts = []
    for i in range(int(r.integers(1, 4))):
        if r.random() < 0.3:
            # a synchronized loop: its bounds are tid-free
            x = "s%d" % next(fresh)
            body = ("seq", block(V0[1:] + [x] + ["tid"], [], 1), ("sync",))
            parts.append(("for", x, 0, int(r.integers(1, 3)), body))
        else:
            parts.append(block(V0, [], 0))
        if r.random() < 0.6:
            parts.append(("sync",))
    if ill_typed and not state["planted"]:
        parts.append(("rd_", "rd", "yz", 0, ("wr_", "wr", ("+", "yz", 1), 0)))

    def text(b):
        if isinstance(b, tuple) and b and b[0] == "wr_":
            return "(%s %s %s)" % (b[1], to_text(b[2]), to_text(b[3]))
        if isinstance(b, tuple) and b and b[0] == "rd_":
            return "(%s %s %s %s)" % (b[1], b[2], to_text(b[3]), text(b[4]))
        if isinstance(b, tuple) and b and b[0] == "if":
            return "(if %s %s %s)" % (to_text(b[1]), text(b[2]), text(b[3]))
        if isinstance(b, tuple) and b and b[0] == "for":
            return "(for %s %s %s %s)" % (b[1], to_text(b[2]), to_text(b[3]), text(b[4]))
        if isinstance(b, tuple) and b and b[0] == "seq":
            return "(seq %s)" % " ".join(text(c) for c in b[1:])
        if b == ("sync",):
            return "(sync)"
        raise AssertionError(b)

    return "(seq %s)" % " ".join(text(p) for p in parts), n, params


# ------------------------------------------------------------------ serving
def gen_requests(rate: float, max_requests: int = 20000, horizon_s: float = 10.0):
    """Poisson request stream at `rate` req/s: (arrival_s, text, n, source).
    Each request is a mixed-batch protocol with probability 0.7, else a
    tree-reduction instance."""
    r = _rng(4, int(rate))
    out = []
    t = 0.0
    i = 0
    while i < max_requests:
        t += float(r.exponential(1.0 / rate))
        if t > horizon_s:
            break
        rr = _rng(4, int(rate), i)
        if rr.random() < 0.7:
            text, n, lab = _mixed_protocol(rr)
            src = "mixed"
        else:
            text, n, lab = _tree_instance(rr)
            src = "tree"
        out.append((t, text, n, src + ":" + lab))
        i += 1
    return out


# ------------------------------------------------------- tiny enumeration
_TINY_IDX_NOVAR = ["0", "1", "tid", "(+ tid 1)"]
_TINY_IDX_VAR = ["x", "(+ tid x)", "(mod (+ tid x) 2)"]
_TINY_GUARDS = ["true", "(= tid 0)", "(< tid 1)", "(<= tid 1)", "(!= tid 1)", "(> tid 1)", "false"]


def _tiny_access(mode, idx, guard):
    a = f"({mode} {idx})"
    if guard == "true":
        return a
    return f"(if {guard} {a} (skip))"


def enumerate_tiny(limit_random: int = 12000, seed: int = 0) -> Iterator[Tuple[str, int]]:
    """Small protocols for exhaustive cross-checks.

    Exhaustive part: every sequence of up to two accesses and up to two
    syncs (any interleaving), each access drawn from modes {rd, wr}, indices
    {0, 1, tid, tid+1} and guards {true, tid=0, tid<1, tid<=1, tid!=1,
    tid>1, false}, optionally wrapped
    whole in a fors or foru (when sync free) loop x in 0..b, b in {0,1,2}, in
    which case indices may also be x, tid+x, (tid+x) mod 2; thread counts
    n in {0,1,2,3}.  Random part: `limit_random` seeded draws with up to
    three accesses and a loop around any contiguous run of items.
    """
    modes = ["rd", "wr"]
    seen = set()

    def emit(text, n):
        key = (text, n)
        if key not in seen:
            seen.add(key)
            return True
        return False

    # exhaustive part
    for k in (1, 2):
        for s in (0, 1, 2):
            for shape in set(itertools.permutations(["A"] * k + ["S"] * s)):
                for loop in ("none", "fors", "foru"):
                    if loop == "foru" and s > 0:
                        continue
                    idxs = _TINY_IDX_NOVAR + (_TINY_IDX_VAR if loop != "none" else [])
                    bounds = (0, 1, 2) if loop != "none" else (None,)
                    for accs in itertools.product(itertools.product(modes, idxs, _TINY_GUARDS), repeat=k):
                        # keep the cross product bounded: guards only on the first access
                        if k == 2 and accs[1][2] != "true":
                            continue
                        items = []
                        ai = 0
                        for tok in shape:
                            if tok == "A":
                                items.append(_tiny_access(*accs[ai]))
                                ai += 1
                            else:
                                items.append("(sync)")
                        body = items[0] if len(items) == 1 else "(seq " + " ".join(items) + ")"
                        for b in bounds:
                            if loop == "none":
                                text = body
                            else:
                                text = f"({loop} x 0 {b} {body})"
                            for n in (0, 1, 2, 3):
                                if emit(text, n):
                                    yield text, n
    # random part
    r = _rng(5, seed)
    made = 0
    while made < limit_random:
        k = int(r.integers(1, 4))
        s = int(r.integers(0, 3))
        toks = ["A"] * k + ["S"] * s
        r.shuffle(toks)
        nitems = len(toks)
        loop = ["none", "fors", "foru"][int(r.integers(0, 3))]
        lo_i = int(r.integers(0, nitems))
        hi_i = int(r.integers(lo_i + 1, nitems + 1))
        if loop == "foru" and "S" in toks[lo_i:hi_i]:
            loop = "fors"
        items = []
        for j, tok in enumerate(toks):
            inside = loop != "none" and lo_i <= j < hi_i
            if tok == "S":
                items.append("(sync)")
            else:
                pool = _TINY_IDX_NOVAR + (_TINY_IDX_VAR if inside else [])
                items.append(_tiny_access(modes[int(r.integers(0, 2))], pool[int(r.integers(0, len(pool)))],
                                          _TINY_GUARDS[int(r.integers(0, len(_TINY_GUARDS)))]))
        if loop != "none":
            inner = items[lo_i:hi_i]
            inner_t = inner[0] if len(inner) == 1 else "(seq " + " ".join(inner) + ")"
            b = int(r.integers(0, 3))
            items = items[:lo_i] + [f"({loop} x 0 {b} {inner_t})"] + items[hi_i:]
        text = items[0] if len(items) == 1 else "(seq " + " ".join(items) + ")"
        n = int(r.integers(0, 4))
        if emit(text, n):
            made += 1
            yield text, n
