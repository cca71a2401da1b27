"""CPU oracle: BabyCUDA programs run with data (test infrastructure only: the
product path never imports or runs this).

Follows Section 3 (Fig. "Syntax and semantics of BabyCUDA"), with its own
parser of the text form
    b ::= (skip) | (sync) | (wr n n') | (rd y n b) | (seq b ...)
        | (if c b b) | (for x n n b)        (wr:A / rd:A: array A)
* A history is a list of phases, earliest first here; a phase maps each
  thread to its reads R (a set of indices) and writes W (index -> value).
* Rule read: evaluate the index j, add j to R, continue with y replaced by
  lastwrite(j) over {tid: (R, W)} :: H -- the thread's own current phase
  first, then earlier phases from the most recent; undefined (None) when no
  phase wrote j.  lastwrite-curr takes the value of some writer of the
  phase; with several writers (only in a racy phase) the least thread id's.
* Rule write: evaluate index j and payload z, set W[j] = z.
* seq, if-t/if-f, for-1/for-2 (half-open range, stride 1, bounds evaluated
  at entry), skip: standard.  Arithmetic and relations as in oracle.ref
  (natural numbers; an undefined payload stays undefined).
* Rule par: every thread runs the program on its own, seeing only its own
  part of the current phase and the whole earlier history; the phase is the
  union of the threads' results.
* The synchronized fragment (left out of the paper's presentation): sync is
  a barrier of all threads; each thread runs to its next sync, the phase
  closes, and the next one starts with the closed phase appended to the
  history.  A program whose threads reach different numbers of syncs is
  rejected (barrier divergence).
* Definition 1 on a phase: threads i1 != i2 and an index j written by i1 and
  read or written by i2.

Arrays: several named arrays keep separate (R, W) per array; accesses to
different arrays never conflict (one behavioural type per array).
"""
from __future__ import annotations

from typing import Dict, List, Optional, Tuple

from . import ref

Phase = Dict[int, Dict[str, Tuple[set, dict]]]   # tid -> array -> (R, W)


class Diverged(Exception):
    """Threads reached different numbers of barriers."""


class DataDependent(Exception):
    """An undefined value (a read of an index nobody wrote) reached control
    flow or an index; cannot happen in a well-typed program."""


# ------------------------------------------------------------------ parsing
def _access(h: str, mode: str):
    if h == mode:
        return ""
    if h.startswith(mode + ":") and ref._is_ident(h[len(mode) + 1:]):
        return h[len(mode) + 1:]
    return None


def _stmt(s):
    if not isinstance(s, list) or not s or not isinstance(s[0], str):
        raise ref.ParseError("statement expected: %r" % (s,))
    h = s[0]
    if h == "skip" and len(s) == 1:
        return ("skip",)
    if h == "sync" and len(s) == 1:
        return ("sync",)
    a = _access(h, "wr")
    if a is not None and len(s) == 3:
        return ("wr", a, ref._nexp(s[1]), ref._nexp(s[2]))
    a = _access(h, "rd")
    if a is not None and len(s) == 4 and isinstance(s[1], str):
        return ("rd", a, s[1], ref._nexp(s[2]), _stmt(s[3]))
    if h == "seq":
        return ("seq",) + tuple(_stmt(c) for c in s[1:])
    if h == "if" and len(s) == 4:
        return ("if", ref._bexp(s[1]), _stmt(s[2]), _stmt(s[3]))
    if h == "for" and len(s) == 5 and isinstance(s[1], str):
        return ("for", s[1], ref._nexp(s[2]), ref._nexp(s[3]), _stmt(s[4]))
    raise ref.ParseError("bad statement %r" % (s,))


def parse(text: str):
    toks = ref._tokens(text)
    tree, pos = ref._sexpr(toks, 0)
    if pos != len(toks):
        raise ref.ParseError("trailing tokens")
    return _stmt(tree)


# --------------------------------------------------------------- evaluation
def _val(e, env):
    """Arithmetic with undefined values: an operand that is undefined makes
    the result undefined (payloads only)."""
    if isinstance(e, int):
        return e
    if isinstance(e, str):
        return env[e]
    a, b = _val(e[1], env), _val(e[2], env)
    if a is None or b is None:
        return None
    return ref.apply_op(e[0], a, b)


def _defined(e, env) -> int:
    v = _val(e, env)
    if v is None:
        raise DataDependent()
    return v


def _cond(c, env) -> bool:
    if c == "true":
        return True
    if c == "false":
        return False
    if c[0] in ref.RELS:
        return ref.apply_rel(c[0], _defined(c[1], env), _defined(c[2], env))
    if c[0] == "not":
        return not _cond(c[1], env)
    a, b = _cond(c[1], env), _cond(c[2], env)
    return (a and b) if c[0] == "and" else (a or b)


class _State:
    """The current phase (being built) and the closed phases before it."""

    def __init__(self, history: List[Phase]):
        self.current: Phase = {}
        self.history = history


def lastwrite(j: int, array: str, tid: int, current: Phase, history: List[Phase]):
    """Value last written to index j of `array`: the thread's own part of
    the current phase, then earlier phases from the most recent; None when
    undefined."""
    own = current.get(tid, {}).get(array)
    if own is not None and j in own[1]:
        return own[1][j]
    for ph in reversed(history):
        for t in sorted(ph):
            rw = ph[t].get(array)
            if rw is not None and j in rw[1]:
                return rw[1][j]
    return None


def _thread(stmt, tid: int, env: dict, st: _State):
    """One thread's run; a generator that yields at every barrier (the
    caller then closes the phase) and records its accesses into its own
    part of the current phase."""
    h = stmt[0]
    if h == "skip":
        return
    if h == "sync":
        yield
        return
    if h == "wr":
        _, arr, n, payload = stmt
        j = _defined(n, env)
        z = _val(payload, env)
        st.current.setdefault(tid, {}).setdefault(arr, (set(), {}))[1][j] = z
        return
    if h == "rd":
        _, arr, y, n, body = stmt
        j = _defined(n, env)
        st.current.setdefault(tid, {}).setdefault(arr, (set(), {}))[0].add(j)
        env2 = dict(env)
        env2[y] = lastwrite(j, arr, tid, st.current, st.history)
        yield from _thread(body, tid, env2, st)
        return
    if h == "seq":
        for c in stmt[1:]:
            yield from _thread(c, tid, env, st)
        return
    if h == "if":
        yield from _thread(stmt[2] if _cond(stmt[1], env) else stmt[3], tid, env, st)
        return
    if h == "for":
        _, x, lo, hi, body = stmt
        v, end = _defined(lo, env), _defined(hi, env)
        while v < end:                      # for-2, then for-1 ends the loop
            env2 = dict(env)
            env2[x] = v
            yield from _thread(body, tid, env2, st)
            v += 1
        return
    raise AssertionError(h)


def run(text_or_ast, n: int, params: Optional[dict] = None, initial: Optional[List[Phase]] = None) -> List[Phase]:
    """Rule par phase by phase: the phases the program produces (earliest
    first), starting from the history `initial` (earliest first)."""
    stmt = parse(text_or_ast) if isinstance(text_or_ast, str) else text_or_ast
    st = _State(list(initial or []))
    produced: List[Phase] = []
    runs = []
    for t in range(n):
        env = dict(params or {})
        env["tid"] = t
        runs.append(_thread(stmt, t, env, st))
    while True:
        # every thread runs to its next barrier or to its end, seeing only
        # its own part of the current phase and the closed phases
        stopped, ended = [], []
        for t in range(n):
            try:
                next(runs[t])
                stopped.append(t)
            except StopIteration:
                ended.append(t)
        if stopped and ended:
            raise Diverged()
        produced.append(st.current)
        if not stopped:
            return produced
        st.history.append(st.current)
        st.current = {}


def access_values(phase: Phase):
    """The access values i:o[j] of a phase (Section 4, before Theorem 1):
    (tid, mode, array, index) for j in R (rd) and j in dom(W) (wr)."""
    out = set()
    for t, arrs in phase.items():
        for a, (R, W) in arrs.items():
            out |= {(t, "rd", a, j) for j in R}
            out |= {(t, "wr", a, j) for j in W}
    return out


def racy_witness(phases: List[Phase], array: str = ""):
    """Definition 1 on every phase of one array: the least (phase, index,
    i1, i2) with i1 < i2, j written by one of them and accessed by the
    other; None when the history is DRF."""
    for k, ph in enumerate(phases):
        events = [(t, o, j) for (t, o, a, j) in access_values(ph) if a == array]
        w = ref._pairwise_witness(k, events, max([t for t, _, _ in events], default=-1) + 1)
        if w is not None:
            return w
    return None
