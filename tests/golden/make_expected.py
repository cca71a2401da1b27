#!/usr/bin/env python3
"""Write the stored oracle results for the full-size synthetic configs.

Calls only the CPU oracle (oracle/o2.c) on the seeded generators; the GPU
tests and bench compare the HIP path against these files.  Usage:
    python tests/golden/make_expected.py [small large large1 large2 tree mixed serve<R>k ...] [-j N]
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import o2  # noqa: E402
from paper_2203_12878_amd import workloads as w  # noqa: E402


def counts_digest(counts):
    return hashlib.sha256(" ".join(str(c) for c in counts).encode()).hexdigest()


def items_of(name):
    if name == "small":
        return [w.gen_small(0)], "gen_small(0)"
    if name == "large":
        return [w.gen_large(0)], "gen_large(0)"
    if name.startswith("large") and name[5:].isdigit():
        # seeds whose protocol writes (seed 0 only reads)
        return [w.gen_large(int(name[5:]))], "gen_large(%d)" % int(name[5:])
    if name == "tree":
        return [(t, n) for t, n, _ in w.gen_tree_batch(0, 2048)], "gen_tree_batch(0, 2048)"
    if name.startswith("serve") and name.endswith("k") and name[5:-1].isdigit():
        # 1000-request Poisson streams (the serving rows of the bench)
        rate = 1000 * int(name[5:-1])
        reqs = w.gen_requests(rate=float(rate), max_requests=1000, horizon_s=1.0)
        return [(t, n) for _, t, n, _ in reqs], "gen_requests(rate=%d, max_requests=1000, horizon_s=1)" % rate
    if name == "mixed":
        return [(t, n) for t, n, _ in w.gen_mixed_batch(0, 4096)], "gen_mixed_batch(0, 4096)"
    raise SystemExit(name)


def main():
    args = [a for a in sys.argv[1:] if not a.startswith("-")]
    jobs = 8
    if "-j" in sys.argv:
        jobs = int(sys.argv[sys.argv.index("-j") + 1])
        args = [a for a in args if a != str(jobs)]
    for name in args or ["small", "large", "tree", "mixed"]:
        items, gen = items_of(name)
        # biggest first keeps the worker threads busy to the end
        t0 = time.time()
        res = o2.check_many(items, jobs=jobs)
        secs = time.time() - t0
        out = {
            "about": "CPU oracle (oracle/o2.c) results for %s, written by tests/golden/make_expected.py" % gen,
            "oracle_seconds": round(secs, 1),
            "results": [{"status": r.status, "racy": r.racy, "witness": list(r.witness) if r.witness else None,
                         "num_records": r.num_records, "num_phases": len(r.phase_counts),
                         "phase_counts": r.phase_counts if len(r.phase_counts) <= 1024 else None,
                         "phase_counts_sha256": counts_digest(r.phase_counts)} for r in res],
        }
        with open(os.path.join(HERE, "expected_%s.json" % name), "w") as f:
            json.dump(out, f, separators=(",", ":"))
        print(name, len(items), "protocols", sum(r.num_records for r in res), "records", round(secs, 1), "s",
              flush=True)


if __name__ == "__main__":
    main()
