"""Build and run the plain C oracle (o2.c).  Test infrastructure only."""
from __future__ import annotations

import os
import subprocess
import time
from typing import List, Sequence, Tuple

from .ref import Result

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "o2.c")
BIN = os.path.join(HERE, "o2.bin")


def build(force: bool = False) -> str:
    """Compile o2.c with gcc (plain C11, pthreads)."""
    if force or not os.path.exists(BIN) or os.path.getmtime(BIN) < os.path.getmtime(SRC):
        tmp = BIN + ".tmp"
        subprocess.check_call(["gcc", "-std=gnu11", "-O2", "-Wall", "-pthread", "-o", tmp, SRC])
        os.replace(tmp, BIN)
    return BIN


def _parse_line(line: str) -> Result:
    f = line.split()
    st, racy, k, j, i1, i2, nrec, nph = (int(x) for x in f[:8])
    if st == -100:
        raise ValueError("o2: parse error")
    counts = [int(x) for x in f[8:8 + nph]]
    wit = (k, j, i1, i2) if racy else None
    return Result(st, racy, wit, counts, nrec)


def check_many(items: Sequence[Tuple[str, int]], jobs: int = 1, timeout: float | None = None,
               timing: bool = False):
    """Run O2 over (text, n) pairs; returns list of Result (and the wall
    seconds of the whole run when timing=True)."""
    build()
    data = "".join("%d %s\n" % (n, " ".join(t.split())) for t, n in items)
    t0 = time.perf_counter()
    p = subprocess.run([BIN, "-j", str(jobs)], input=data, capture_output=True, text=True,
                       timeout=timeout, check=True)
    secs = time.perf_counter() - t0
    out = [_parse_line(l) for l in p.stdout.splitlines()]
    assert len(out) == len(items)
    return (out, secs) if timing else out


def check(text: str, n: int) -> Result:
    return check_many([(text, n)])[0]
