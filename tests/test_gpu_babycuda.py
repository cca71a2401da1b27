"""BabyCUDA programs checked on the GPU through their inferred protocols
(drf_babycuda_infer, then drf_check_arrays), against the oracle's run of
the programs with data: by Theorem 1 a well-typed program's history is DRF
exactly when its protocol is, so the GPU's verdict and least witness per
array must equal Definition 1 applied to the program's own history."""
import re

import pytest

from oracle import baby
from paper_2203_12878_amd import workloads as w

pytestmark = pytest.mark.gpu

INIT = [{0: {"": (set(), {i: 100 + i for i in range(8)}), "B": (set(), {i: 200 + i for i in range(8)})}}]


def bind(text, params):
    for k, v in params.items():
        text = re.sub(r"(?<![\w:])%s(?![\w])" % re.escape(k), str(v), text)
    return text


def test_programs_checked_through_their_protocols():
    from paper_2203_12878_amd import drf
    chk = drf.Checker(0)
    racy = 0
    for seed in range(200):
        prog, n, params = w.gen_babycuda(seed)
        st, proto = drf.infer(prog, list(params))
        assert st == 0
        hist = baby.run(prog, n, params, initial=INIT)
        names = []
        for _, nm in re.findall(r"\((rd|wr)(?::(\w+))? ", proto):
            if nm not in names:
                names.append(nm)
        got = chk.check_arrays(bind(proto, params), n)
        assert len(got) == max(1, len(names))
        for r, name in zip(got, names or [""]):
            assert r.status == 0
            assert r.witness == baby.racy_witness(hist, name), (prog, name)
            assert len(r.phase_counts) == len(hist)
            racy += r.racy
    chk.close()
    assert 0 < racy
