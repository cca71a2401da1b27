#!/usr/bin/env python3
"""Throughput of data-race-freedom checking on one MI355X.

One step = one full check (count, fused / partition / sort / scan passes,
witness) of the workload's protocols through the C ABI, inputs already in
host memory as compiled bytecode and outputs in device memory.  The default
workload is the plain single large protocol: 65,536 threads, three nested
for^S loops (bounds 1..32, product redrawn into [128, 508]), six affine-mod
accesses into 2^24 cells (seed 0: 121,896,960 access events in 373 phases).

Prints one JSON line.  Per-kernel times come from HIP events the library
records around its own launches on its own stream while the timed steps
run; the roofline entry is for the kernel class with the largest total
time.  The CPU baseline is the C oracle run on the same protocol on the
host (single thread: it checks one protocol at a time).
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# bytes per record the method must move with records materialized in HBM
# (one 8-byte record write, its read-back by the conflict pass, and the
# 8-byte histogram read of one partition level)
EFFECTIVE_BYTES_PER_RECORD = 24
# integer VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one 32-bit op per lane per clock)
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def workload(name: str):
    from paper_2203_12878_amd import workloads as w
    if name == "large":
        t, n = w.gen_large(0)
        return [(t, n)], "plain single large protocol, seed 0: 65536 threads, 3 nested for^S, 6 accesses, 2^24 cells"
    if name == "small":
        t, n = w.gen_small(0)
        return [(t, n)], "plain single small protocol, seed 0: 256 threads, for^S 16 x 4, 4 accesses, 4096 cells"
    if name == "mixed":
        b = w.gen_mixed_batch(0, 4096)
        return [(t, n) for t, n, _ in b], "mixed batch, seed 0: 4096 protocols, 32..4096 threads, depth 1..3"
    if name == "tree":
        b = w.gen_tree_batch(0, 2048)
        return [(t, n) for t, n, _ in b], "tree-reduction batch, seed 0: 2048 instances, 2^8..2^20 threads"
    raise SystemExit("unknown workload " + name)


def expr_ops(text: str) -> int:
    """Arithmetic operators in the access index expressions (per event)."""
    ops = 0
    accs = 0
    for m in re.finditer(r"\((rd|wr) ", text):
        depth, i = 0, m.end()
        j = i
        while j < len(text):
            c = text[j]
            if c == "(":
                depth += 1
            elif c == ")":
                if depth == 0:
                    break
                depth -= 1
            j += 1
        ops += len(re.findall(r"\((?:\+|-|\*|/|mod|<<|>>|min|max) ", text[i:j]))
        accs += 1
    return max(1, round(ops / max(1, accs)))


class KStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 16), ("launches", ctypes.c_uint64), ("ms", ctypes.c_double),
                ("records", ctypes.c_uint64), ("bytes", ctypes.c_uint64)]


def kernel_stats(lib, ctx, reset=True):
    arr = (KStat * 16)()
    n = ctypes.c_uint32(0)
    lib.drf_ctx_kernel_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(KStat), ctypes.c_uint32,
                                         ctypes.POINTER(ctypes.c_uint32), ctypes.c_int]
    lib.drf_ctx_kernel_stats(ctx, arr, 16, ctypes.byref(n), 1 if reset else 0)
    return {a.name.decode(): {"launches": a.launches, "ms": a.ms, "records": a.records, "bytes": a.bytes}
            for a in arr[:n.value]}


def kernels_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp", "drf_layout.hpp"):
        with open(os.path.join(ROOT, "paper_2203_12878_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary, or None when none exists or the kernels have
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "%s_%s_counters.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            m = re.match(r"^- (\w+): `?([^`\s]+)`?", line.strip())
            if m:
                vals[m.group(1)] = m.group(2)
    if vals.get("kernels_sha256") != kernels_sha256():
        return None
    try:
        return int(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def compare_paths(drf, chk):
    """Batched (one check over the whole set) against plain (one protocol
    per call) on a sample of the batched workloads."""
    import torch
    from paper_2203_12878_amd import workloads as w
    items = [(t, n) for t, n, _ in w.gen_mixed_batch(0, 512)] + [(t, n) for t, n, _ in w.gen_tree_batch(0, 128)]
    batch = drf.Batch(items, 0)
    out = {}
    for name, run in (("batched", chk.run_batch), ("plain", chk.run_plain)):
        run(batch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 2
        for _ in range(reps):
            run(batch)
        torch.cuda.synchronize()
        out[name] = (time.perf_counter() - t0) / reps
    recs = sum(r.num_records for r in batch.collect())
    return {"sample": "first 512 protocols of the mixed batch and first 128 tree instances (seed 0), %d records" % recs,
            "batched_records_per_s": round(recs / out["batched"], 1), "plain_records_per_s": round(recs / out["plain"], 1),
            "batched_ms": round(out["batched"] * 1e3, 3), "plain_ms": round(out["plain"] * 1e3, 3),
            "speedup": round(out["plain"] / out["batched"], 3)}


def serving(rates, requests_per_rate=5000):
    """Poisson streams of check requests through the continuous-batching
    server: latency percentiles and throughput per offered rate.  Each
    stream lasts about requests_per_rate / rate seconds (one second at
    most)."""
    from paper_2203_12878_amd import workloads as w
    from paper_2203_12878_amd.server import Server, run_stream
    rows = []
    for rate in rates:
        horizon_s = min(1.0, requests_per_rate / rate)
        reqs = w.gen_requests(rate=float(rate), max_requests=int(rate * horizon_s * 2), horizon_s=horizon_s)
        with Server(device=0, workers=4, budget_bytes=8 << 30) as srv:
            # warm both workers (first launches, pinned staging) outside the figures
            run_stream(srv, [(0.0,) + tuple(q[1:]) for q in reqs[:16]])
            srv.reset_stats()
            res, wall = run_stream(srv, reqs)
            st = srv.stats
        recs = sum(r.num_records for r in res)
        rows.append({"offered_req_per_s": rate, "requests": len(reqs), "p50_ms": round(st.percentile(50) * 1e3, 3),
                     "p99_ms": round(st.percentile(99) * 1e3, 3), "records_per_s": round(recs / wall, 1),
                     "req_per_s": round(len(reqs) / wall, 1), "batches": st.batches})
    return rows


def cpu_baseline(items, records_per_step):
    """The C oracle on the same protocols, on host cores."""
    from oracle import o2
    t0 = time.perf_counter()
    res, secs = o2.check_many(items, jobs=1, timing=True)
    recs = sum(r.num_records for r in res)
    return {"value": recs / secs, "unit": "records/s", "cores": 1, "kind": "oracle",
            "sample": "the whole workload (%d protocol(s), %d access events) through the C oracle, one thread, %.1f s"
                      % (len(items), recs, secs)}, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=["large", "small", "mixed", "tree"])
    ap.add_argument("--path", default="auto", choices=["auto", "plain", "batch"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile-events", type=int, default=0, help="tuning override (0: library default)")
    ap.add_argument("--digit-bits", type=int, default=0)
    ap.add_argument("--unit-events", type=int, default=0)
    ap.add_argument("--item-events", type=int, default=0)
    ap.add_argument("--no-extras", action="store_true", help="skip the batched-vs-plain and serving sections")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the checker runs on one GPU; --gpus %d is not supported (there is no "
              "multi-GPU path)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2203_12878_amd import drf

    items, desc = workload(args.workload)
    path = args.path if args.path != "auto" else ("plain" if len(items) == 1 else "batch")
    chk = drf.Checker(0)
    chk.set_tuning(tile_events=args.tile_events, digit_bits=args.digit_bits, unit_events=args.unit_events,
                   item_events=args.item_events)
    lib = drf.lib()
    lib.drf_ctx_set_profiling.argtypes = [ctypes.c_void_p, ctypes.c_int]
    batch = drf.Batch(items, 0)
    run = chk.run_plain if path == "plain" else chk.run_batch
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        run(batch)
    stream.synchronize()
    lib.drf_ctx_set_profiling(chk._ctx, 1)
    kernel_stats(lib, chk._ctx, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run(batch)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.drf_ctx_set_profiling(chk._ctx, 0)
    stats = kernel_stats(lib, chk._ctx, reset=True)
    results = batch.collect()
    records = sum(r.num_records for r in results)
    racy = sum(r.racy for r in results)
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    value = records / ((t1 - t0) / args.steps)

    # parity of this run against stored oracle results (when present)
    parity = None
    gold = os.path.join(ROOT, "tests", "golden", "expected_%s.json" % args.workload)
    if os.path.exists(gold):
        with open(gold) as f:
            exp = json.load(f)["results"]
        def counts_sha(c):   # the stored digest: sha256 of the counts in decimal, space separated
            c = c.tolist() if hasattr(c, "tolist") else list(c)
            return hashlib.sha256(" ".join(str(x) for x in c).encode()).hexdigest()
        parity = len(exp) == len(results) and all(
            [r.status, r.racy, list(r.witness) if r.witness else None, r.num_records] ==
            [e["status"], e["racy"], e["witness"], e["num_records"]] and
            (r.status != 0 or counts_sha(r.phase_counts) == e["phase_counts_sha256"]) for r, e in zip(results, exp))

    dom = max(stats.items(), key=lambda kv: kv[1]["ms"])
    dname, d = dom
    launches = max(1, d["launches"])
    avg_ms = d["ms"] / launches
    if d["bytes"] > 0:
        achieved = d["bytes"] / (d["ms"] / 1e3) / 1e9
        roof = {"kernel": dname, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": committed_traffic(dname, args.workload),
                "bytes_per_launch": d["bytes"] // launches, "avg_launch_ms": round(avg_ms, 4)}
    else:
        ops = expr_ops(items[0][0]) if len(items) == 1 else 1
        achieved = d["records"] * ops / (d["ms"] / 1e3) / 1e12
        roof = {"kernel": dname, "bound": "alu", "achieved": round(achieved, 3), "peak": ALU_PEAK_TOPS,
                "unit": "Tops/s", "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": None,
                "ops_per_record": ops, "avg_launch_ms": round(avg_ms, 4)}

    line = {
        "metric": "access records checked/s",
        "value": round(value, 1),
        "unit": "records/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "path": path, "protocols": len(items),
                   "records_per_step": records, "racy_protocols": racy, "tuning": chk.tuning()},
        "parity_vs_stored_oracle": parity,
        "roofline": roof,
        "effective_hbm_frac": round(value * EFFECTIVE_BYTES_PER_RECORD / (HBM_PEAK_GBS * 1e9), 4),
        "kernels": {k: {"ms_per_step": round(v["ms"] / args.steps, 4), "launches_per_step": v["launches"] // args.steps,
                        "records_per_step": v["records"] // args.steps, "bytes_per_step": v["bytes"] // args.steps}
                    for k, v in stats.items() if v["launches"]},
    }
    if not args.no_cpu_baseline:
        cb, _ = cpu_baseline(items if len(items) == 1 else items[:64], records)
        line["cpu_baseline"] = cb
    if not args.no_extras:
        line["batched_vs_plain"] = compare_paths(drf, chk)
        line["serving"] = serving([1000, 5000, 20000, 50000])
    print(json.dumps(line), flush=True)
    chk.close()


if __name__ == "__main__":
    main()
