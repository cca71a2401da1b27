"""CPU oracle for data-race freedom of memory access protocols (test
infrastructure only: the product path never imports or runs this).

Plain, slow, obviously correct.  Everything is exact Python integers.

What is computed (paper: "Provable GPU Data-Races in Static Race Detection",
Liew, Cogumbreiro, Lange, PLACES 2022):

* Protocol syntax: Fig. "Syntax of MAPs" (arithmetic n, modes rd/wr,
  booleans c, unsynchronized U: skip, o[n], u;u, if, for^U; synchronized S:
  sync, p;p, for^S), with a U leaf allowed inside S (the figure's S grammar
  has no production that embeds an access; without it a synchronized
  protocol could not access memory).
* Thread-level control flow: Fig. "Syntax and semantics of BabyCUDA", rules
  seq, if-t, if-f, for-1, for-2 (half-open lo..hi, stride 1), skip; every
  thread runs independently (rule par) on T = {0..n-1}.
* Synchronized fragment (left out of the paper's presentation): sync is a
  barrier over all of T that closes the current phase and opens an empty one
  (histories are lists of phases, H ::= [] | P::H); phase k = the accesses
  performed after exactly k syncs.  for^S bounds are evaluated once and may
  not mention tid.
* Race predicate: Definition 1 (DRF program): a phase is racy iff there are
  threads i1 != i2 and an index j with j written by i1 and read or written
  by i2; a history is DRF iff every phase is.  Access values i:o[j] and the
  transport of a phase to a set of access values (Section 4, before
  Theorem 1) make a phase of a protocol the set of its access values.

Outputs per protocol (all exact integers):
  status          0, or a negative code (static checks, range overflow)
  racy            0/1
  witness         lexicographic minimum of (phase, index, i1, i2) over
                  i1 < i2 both accessing index in phase, at least one writing
  phase_counts    number of executed access events per phase (syncs + 1)
  num_records     sum of phase_counts

Three formulations live here and in o2.c:
  O1 (check_literal) - direct interpreter + all thread pairs per phase.
  O3 (check_split)   - split into closed unsynchronized protocols by
                       unrolling for^S with substitution, cut at sync, each
                       fragment run with the thread-level rules and checked
                       on its own.
  O2 (o2.c)          - the same expansion in plain C with a per-(phase,
                       index) aggregate (min tid, second tid, min writer).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Set, Tuple

# status codes (shared meaning with the C ABI; values written out here)
OK = 0
E_UNBOUND = -3
E_SHADOW = -4
E_SYNC_IN_U = -5
E_DIVERGENT = -6
E_RANGE = -7

VALUE_LIMIT = 1 << 63   # every evaluated value must stay below this
INDEX_LIMIT = 1 << 32   # every accessed index must stay below this

ARITH = ("+", "-", "*", "/", "mod", "<<", ">>", "min", "max")
RELS = ("<", "<=", "=", "!=", ">", ">=")


class ParseError(ValueError):
    pass


class RangeOverflow(Exception):
    pass


@dataclass
class Result:
    status: int
    racy: int = 0
    witness: Optional[Tuple[int, int, int, int]] = None
    phase_counts: List[int] = field(default_factory=list)
    num_records: int = 0

    def key(self):
        return (self.status, self.racy, self.witness, tuple(self.phase_counts), self.num_records)


def error_result(status: int) -> Result:
    return Result(status=status)


# ------------------------------------------------------------------ parsing
def _tokens(text: str):
    out = []
    i = 0
    while i < len(text):
        c = text[i]
        if c.isspace():
            i += 1
        elif c in "()":
            out.append(c)
            i += 1
        else:
            j = i
            while j < len(text) and not text[j].isspace() and text[j] not in "()":
                j += 1
            out.append(text[i:j])
            i = j
    return out


def _sexpr(toks, pos):
    if pos >= len(toks):
        raise ParseError("unexpected end")
    t = toks[pos]
    if t == "(":
        items = []
        pos += 1
        while True:
            if pos >= len(toks):
                raise ParseError("missing )")
            if toks[pos] == ")":
                return items, pos + 1
            item, pos = _sexpr(toks, pos)
            items.append(item)
    if t == ")":
        raise ParseError("unexpected )")
    return t, pos + 1


_KEYWORDS = set(ARITH) | set(RELS) | {"and", "or", "not", "true", "false", "skip", "rd", "wr",
                                      "seq", "if", "foru", "fors", "sync"}


def _is_ident(t):
    return isinstance(t, str) and (t[0].isalpha() or t[0] == "_") and \
        all(ch.isalnum() or ch == "_" for ch in t) and t not in _KEYWORDS


def _nexp(s):
    if isinstance(s, str):
        if s.isdigit():
            v = int(s)
            if v >= 1 << 64:
                raise ParseError("literal too large")
            return v
        if s == "tid" or _is_ident(s):
            return s
        raise ParseError("bad arithmetic atom %r" % s)
    if len(s) == 3 and s[0] in ARITH:
        return (s[0], _nexp(s[1]), _nexp(s[2]))
    raise ParseError("bad arithmetic expression %r" % (s,))


def _bexp(s):
    if s in ("true", "false"):
        return s
    if isinstance(s, list):
        if len(s) == 3 and s[0] in RELS:
            return (s[0], _nexp(s[1]), _nexp(s[2]))
        if len(s) == 3 and s[0] in ("and", "or"):
            return (s[0], _bexp(s[1]), _bexp(s[2]))
        if len(s) == 2 and s[0] == "not":
            return ("not", _bexp(s[1]))
    raise ParseError("bad boolean expression %r" % (s,))


def _stmt(s):
    if not isinstance(s, list) or not s:
        raise ParseError("statement expected, got %r" % (s,))
    h = s[0]
    if h == "skip" and len(s) == 1:
        return ("skip",)
    if h == "sync" and len(s) == 1:
        return ("sync",)
    if h in ("rd", "wr") and len(s) == 2:
        return (h, _nexp(s[1]))
    if h == "seq":
        return ("seq",) + tuple(_stmt(c) for c in s[1:])
    if h == "if" and len(s) == 4:
        return ("if", _bexp(s[1]), _stmt(s[2]), _stmt(s[3]))
    if h in ("foru", "fors") and len(s) == 5:
        if not (isinstance(s[1], str) and (s[1] == "tid" or _is_ident(s[1]))):
            raise ParseError("bad loop variable %r" % (s[1],))
        return (h, s[1], _nexp(s[2]), _nexp(s[3]), _stmt(s[4]))
    raise ParseError("bad statement %r" % (s,))


def parse(text: str):
    toks = _tokens(text)
    tree, pos = _sexpr(toks, 0)
    if pos != len(toks):
        raise ParseError("trailing tokens")
    return _stmt(tree)


# ----------------------------------------------------------- static checks
def free_vars(e) -> Set[str]:
    if isinstance(e, int) or e in ("true", "false"):
        return set()
    if isinstance(e, str):
        return {e}
    out = set()
    for c in e[1:]:
        out |= free_vars(c)
    return out


def static_status(stmt) -> int:
    """First violation in a left-to-right pre-order walk, or OK.

    Index and guard expressions may only mention tid and enclosing loop
    variables (typing rules t-n, t-b); nested binders are distinct (side
    condition x not in V of t-for / t-read); sync and for^S never occur under
    if or for^U (U has no synchronization); for^S bounds are tid-free, which
    makes every thread execute the same barriers.
    """
    def unbound(e, scope):
        return any(v != "tid" and v not in scope for v in free_vars(e))

    def walk(s, scope, in_u):
        h = s[0]
        if h == "skip":
            return OK
        if h in ("rd", "wr"):
            return E_UNBOUND if unbound(s[1], scope) else OK
        if h == "seq":
            for c in s[1:]:
                st = walk(c, scope, in_u)
                if st:
                    return st
            return OK
        if h == "if":
            if unbound(s[1], scope):
                return E_UNBOUND
            return walk(s[2], scope, True) or walk(s[3], scope, True)
        if h == "sync":
            return E_SYNC_IN_U if in_u else OK
        if h in ("foru", "fors"):
            if h == "fors" and in_u:
                return E_SYNC_IN_U
            _, x, lo, hi, body = s
            if unbound(lo, scope) or unbound(hi, scope):
                return E_UNBOUND
            if h == "fors" and "tid" in (free_vars(lo) | free_vars(hi)):
                return E_DIVERGENT
            if x == "tid" or x in scope:
                return E_SHADOW
            return walk(body, scope | {x}, in_u or h == "foru")
        raise AssertionError(h)

    return walk(stmt, frozenset(), False)


# ------------------------------------------------------------- arithmetic
def _chk(v: int) -> int:
    if v >= VALUE_LIMIT:
        raise RangeOverflow()
    return v


def apply_op(op: str, a: int, b: int) -> int:
    """Binary operators on naturals.  Truncated subtraction, and division and
    modulus by zero follow the usual natural-number conventions: a - b = 0
    when b > a, a / 0 = 0, a mod 0 = a.  Shifts are a * 2^b and floor(a/2^b).
    """
    if op == "+":
        r = a + b
    elif op == "-":
        r = a - b if a > b else 0
    elif op == "*":
        r = a * b
    elif op == "/":
        r = a // b if b else 0
    elif op == "mod":
        r = a % b if b else a
    elif op == "<<":
        if a == 0:
            r = 0
        elif b >= 64:
            raise RangeOverflow()
        else:
            r = a << b
    elif op == ">>":
        r = a >> b if b < 64 else 0
    elif op == "min":
        r = min(a, b)
    elif op == "max":
        r = max(a, b)
    else:
        raise AssertionError(op)
    return _chk(r)


def apply_rel(op: str, a: int, b: int) -> bool:
    return {"<": a < b, "<=": a <= b, "=": a == b, "!=": a != b, ">": a > b, ">=": a >= b}[op]


def eval_n(e, env: Dict[str, int]) -> int:
    """Evaluate an arithmetic expression; every sub-expression is evaluated
    and checked against the value limit."""
    if isinstance(e, int):
        return _chk(e)
    if isinstance(e, str):
        return env[e]
    return apply_op(e[0], eval_n(e[1], env), eval_n(e[2], env))


def eval_b(c, env: Dict[str, int]) -> bool:
    """Evaluate a guard.  Both operands of and/or are always evaluated."""
    if c == "true":
        return True
    if c == "false":
        return False
    if c[0] in RELS:
        return apply_rel(c[0], eval_n(c[1], env), eval_n(c[2], env))
    if c[0] == "not":
        return not eval_b(c[1], env)
    a = eval_b(c[1], env)
    b = eval_b(c[2], env)
    return (a and b) if c[0] == "and" else (a or b)


# ------------------------------------------------- direct interpreter (O1)
def _run_u(u, env, tid, out: list):
    """Thread-level evaluation of an unsynchronized protocol for one thread:
    appends (tid, mode, index) per executed access, in program order."""
    h = u[0]
    if h == "skip":
        return
    if h in ("rd", "wr"):
        j = eval_n(u[1], env)
        if j >= INDEX_LIMIT:
            raise RangeOverflow()
        out.append((tid, h, j))
        return
    if h == "seq":
        for c in u[1:]:
            _run_u(c, env, tid, out)
        return
    if h == "if":
        _run_u(u[2] if eval_b(u[1], env) else u[3], env, tid, out)
        return
    if h == "foru":
        _, x, lo, hi, body = u
        a = eval_n(lo, env)
        b = eval_n(hi, env)
        for v in range(a, b):
            env2 = dict(env)
            env2[x] = v
            _run_u(body, env2, tid, out)
        return
    raise AssertionError(h)


def _has_s(s) -> bool:
    """True when s contains a synchronized construct (sync or for^S)."""
    if s[0] in ("sync", "fors"):
        return True
    if s[0] == "seq":
        return any(_has_s(c) for c in s[1:])
    return False


def expand(stmt, n: int) -> List[List[Tuple[int, str, int]]]:
    """Walk the synchronized structure with the phase counter; run each
    unsynchronized leaf for every thread of T = {0..n-1} (rule par).
    for^S bounds are evaluated once per loop entry, whether or not the body
    holds a sync.  Returns phases, each a list of access events
    (tid, mode, index)."""
    phases: List[list] = [[]]

    def walk(s, env):
        h = s[0]
        if h == "sync":
            phases.append([])
        elif h == "seq" and _has_s(s):
            for c in s[1:]:
                walk(c, env)
        elif h == "fors":
            _, x, lo, hi, body = s
            a = eval_n(lo, env)
            b = eval_n(hi, env)
            for v in range(a, b):
                env2 = dict(env)
                env2[x] = v
                walk(body, env2)
        else:
            for i in range(n):
                env_i = dict(env)
                env_i["tid"] = i
                _run_u(s, env_i, i, phases[-1])

    walk(stmt, {})
    return phases


def _pairwise_witness(k: int, events, n: int):
    """Definition 1 on one phase, literally: every pair of distinct threads
    of T, per-thread read set R and write set W.  Returns the least
    (k, j, i1, i2) with i1 < i2 or None."""
    R = [set() for _ in range(n)]
    W = [set() for _ in range(n)]
    for (i, o, j) in events:
        (W if o == "wr" else R)[i].add(j)
    best = None
    for a in range(n):
        for b in range(a + 1, n):
            conf = (W[a] & (R[b] | W[b])) | (W[b] & (R[a] | W[a]))
            if conf:
                cand = (k, min(conf), a, b)
                if best is None or cand < best:
                    best = cand
    return best


def check_literal(text_or_ast, n: int) -> Result:
    """O1: direct interpreter + all thread pairs per phase."""
    stmt = parse(text_or_ast) if isinstance(text_or_ast, str) else text_or_ast
    st = static_status(stmt)
    if st:
        return error_result(st)
    try:
        phases = expand(stmt, n)
    except RangeOverflow:
        return error_result(E_RANGE)
    counts = [len(p) for p in phases]
    wit = None
    for k, ev in enumerate(phases):
        wit = _pairwise_witness(k, ev, n)
        if wit is not None:
            break
    return Result(OK, int(wit is not None), wit, counts, sum(counts))


# -------------------------------------------------------------- split (O3)
def subst(node, x: str, v: int):
    """node[v/x]: replace free occurrences of variable x by the natural v."""
    if isinstance(node, int):
        return node
    if isinstance(node, str):
        return v if node == x else node
    h = node[0]
    if h in ("foru", "fors"):
        _, y, lo, hi, body = node
        lo2, hi2 = subst(lo, x, v), subst(hi, x, v)
        return (h, y, lo2, hi2, body if y == x else subst(body, x, v))
    return (h,) + tuple(subst(c, x, v) if not (isinstance(c, str) and c in _KEYWORDS) else c
                        for c in node[1:])


def _closed_n(e) -> int:
    if isinstance(e, int):
        return _chk(e)
    if isinstance(e, str):
        raise AssertionError("open expression: %r" % e)
    return apply_op(e[0], _closed_n(e[1]), _closed_n(e[2]))


def _closed_b(c) -> bool:
    if c == "true":
        return True
    if c == "false":
        return False
    if c[0] in RELS:
        return apply_rel(c[0], _closed_n(c[1]), _closed_n(c[2]))
    if c[0] == "not":
        return not _closed_b(c[1])
    a = _closed_b(c[1])
    b = _closed_b(c[2])
    return (a and b) if c[0] == "and" else (a or b)


def split(stmt) -> list:
    """Split a validated synchronized protocol into its list of closed
    unsynchronized protocols [u_0, ..., u_K], one per phase: for^S loops are
    unrolled with their variable substituted (the for-2 rule's b[n/x]), and
    the sequence is cut at every sync.  The fragment after the last sync of
    one iteration and the one before the first sync of the next iteration
    fall in the same phase, so they are joined."""
    h = stmt[0]
    if h == "sync":
        return [("skip",), ("skip",)]
    if h == "seq":
        frags = [("skip",)]
        for c in stmt[1:]:
            f = split(c)
            frags[-1] = ("seq", frags[-1], f[0])
            frags.extend(f[1:])
        return frags
    if h == "fors":
        _, x, lo, hi, body = stmt
        a = _closed_n(lo)
        b = _closed_n(hi)
        frags = [("skip",)]
        for v in range(a, b):
            f = split(subst(body, x, v))
            frags[-1] = ("seq", frags[-1], f[0])
            frags.extend(f[1:])
        return frags
    return [stmt]


def _thread_eval(u, out: list, tid: int):
    """Thread-level rules on a closed unsynchronized protocol (tid already
    substituted): skip, seq, if-t/if-f, for-1/for-2 by substitution."""
    h = u[0]
    if h == "skip":
        return
    if h in ("rd", "wr"):
        j = _closed_n(u[1])
        if j >= INDEX_LIMIT:
            raise RangeOverflow()
        out.append((tid, h, j))
    elif h == "seq":
        for c in u[1:]:
            _thread_eval(c, out, tid)
    elif h == "if":
        _thread_eval(u[2] if _closed_b(u[1]) else u[3], out, tid)
    elif h == "foru":
        _, x, lo, hi, body = u
        a = _closed_n(lo)
        b = _closed_n(hi)
        # for-2 unfolded: body[a/x]; then the loop from a+1 (for-1 ends it)
        while a < b:
            _thread_eval(subst(body, x, a), out, tid)
            a += 1
    else:
        raise AssertionError(h)


def check_split(text_or_ast, n: int) -> Result:
    """O3: DRF(p) iff every closed unsynchronized fragment u_k is DRF; the
    witness is that of the first racy fragment, with its phase number."""
    stmt = parse(text_or_ast) if isinstance(text_or_ast, str) else text_or_ast
    st = static_status(stmt)
    if st:
        return error_result(st)
    try:
        frags = split(stmt)
        phases = []
        for u in frags:
            ev = []
            for i in range(n):
                _thread_eval(subst(u, "tid", i), ev, i)
            phases.append(ev)
    except RangeOverflow:
        return error_result(E_RANGE)
    counts = [len(p) for p in phases]
    wit = None
    for k, ev in enumerate(phases):
        wit = _pairwise_witness(k, ev, n)
        if wit is not None:
            break
    return Result(OK, int(wit is not None), wit, counts, sum(counts))
