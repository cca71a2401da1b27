"""CPU oracle for protocols over several shared arrays (test infrastructure
only: the product path never imports or runs this).

The analysis assigns one behavioural type per shared array (Section 3,
Syntax): a kernel that uses several arrays has one memory access protocol
per array, and Definition 1 is applied to each of them on its own.  Array
a's protocol is the written protocol with every access to another array
replaced by skip (its own accesses keep their mode and index).  Each such
protocol is then decided by the literal oracle (ref.check_literal: direct
interpreter, all pairs of threads per phase), so static statuses and value
overflow count against the arrays whose protocol contains them.

Text form: rd:A e / wr:A e name array A; plain rd / wr name the unnamed
array.  Arrays are numbered in order of first appearance in the text (the
unnamed one too).
"""
from __future__ import annotations

from typing import Dict, List

from . import ref


def _is_access(h) -> bool:
    return isinstance(h, str) and (h in ("rd", "wr") or h.startswith("rd:") or h.startswith("wr:"))


def _stmt(s, arrays: Dict[str, int]):
    """Parse one statement; accesses become ("acc", mode, array_id, index)."""
    if isinstance(s, list) and s and _is_access(s[0]) and len(s) == 2:
        h = s[0]
        name = h[3:] if len(h) > 2 else ""
        if len(h) > 2 and not ref._is_ident(name):
            raise ref.ParseError("bad array name %r" % h)
        if name not in arrays:
            arrays[name] = len(arrays)
        return ("acc", h[:2], arrays[name], ref._nexp(s[1]))
    if isinstance(s, list) and s and s[0] == "seq":
        return ("seq",) + tuple(_stmt(c, arrays) for c in s[1:])
    if isinstance(s, list) and s and s[0] == "if" and len(s) == 4:
        return ("if", ref._bexp(s[1]), _stmt(s[2], arrays), _stmt(s[3], arrays))
    if isinstance(s, list) and s and s[0] in ("foru", "fors") and len(s) == 5:
        if not (isinstance(s[1], str) and (s[1] == "tid" or ref._is_ident(s[1]))):
            raise ref.ParseError("bad loop variable %r" % (s[1],))
        return (s[0], s[1], ref._nexp(s[2]), ref._nexp(s[3]), _stmt(s[4], arrays))
    return ref._stmt(s)


def parse(text: str):
    """(statement, number of arrays)."""
    toks = ref._tokens(text)
    tree, pos = ref._sexpr(toks, 0)
    if pos != len(toks):
        raise ref.ParseError("trailing tokens")
    arrays: Dict[str, int] = {}
    st = _stmt(tree, arrays)
    return st, max(1, len(arrays))


def array_protocol(s, a: int):
    """The protocol of array a: its own accesses, skip for the others."""
    h = s[0]
    if h == "acc":
        return (s[1], s[3]) if s[2] == a else ("skip",)
    if h == "seq":
        return ("seq",) + tuple(array_protocol(c, a) for c in s[1:])
    if h == "if":
        return ("if", s[1], array_protocol(s[2], a), array_protocol(s[3], a))
    if h in ("foru", "fors"):
        return (h, s[1], s[2], s[3], array_protocol(s[4], a))
    return s


def check_arrays(text: str, n: int) -> List[ref.Result]:
    """One Result per array: Definition 1 on that array's protocol."""
    stmt, na = parse(text)
    return [ref.check_literal(array_protocol(stmt, a), n) for a in range(na)]
