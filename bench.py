#!/usr/bin/env python3
"""Throughput of data-race-freedom checking on one MI355X.

One step = one full check (count, fused / partition / tile passes, witness)
of the workload's protocols through the C ABI, inputs already in host
memory as compiled bytecode and outputs in device memory.  The default
workload is the batched configuration: 4096 seeded protocols (32..4096
threads, loop depth 1..3, bounds 1..64, 2..8 accesses, 2^12..2^20 cells,
about 20% racy by construction), 22.1 G access events, checked in one
drf_check_batch call.

Prints one JSON line:
* the headline: records checked per second on the workload's path, with
  parity against the stored oracle results;
* `roofline`: the kernel class with the largest time, from HIP events the
  library records around its own launches on its own stream;
* `paths` and `large` run with their own workloads' cached tunings (size
  classes of the autotuner), the headline with its own;
* `paths`: the batched path against the plain path (one drf_check_protocol
  per protocol) on the whole mixed and tree-reduction batches, both with
  parity;
* `large`: the plain single large protocol (65,536 threads, 2^24 cells; a
  seed whose protocol writes) with its tile-kernel roofline;
* `serving`: Poisson streams of 1000 requests through the continuous-
  batching server at 1k..50k req/s, p50/p99 latency, parity against the
  stored oracle results and against each request checked alone;
* `cpu_baseline`: the C oracle on a bounded sample of the workload, on one
  host core and on all of them.

`--calibrate-copy MiB` instead runs one plain device copy of that size (the
reference for the HBM byte counters) and exits.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import platform
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# 32-bit VALU lane operations: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_GOPS = 256 * 4 * 16 * 2.4
# bytes per record the method must move with records materialized in HBM
# (one 8-byte record write, its read-back by the conflict pass, and the
# 8-byte histogram read of one partition level)
EFFECTIVE_BYTES_PER_RECORD = 24
GOLDEN = os.path.join(ROOT, "tests", "golden")


def workload(name: str, seed: int):
    from paper_2203_12878_amd import workloads as w
    if name == "large":
        t, n = w.gen_large(seed)
        return [(t, n)], "large", ("plain single large protocol, seed %d: 65536 threads, 3 nested for^S "
                                   "(bounds 1..32), 6 accesses, 2^24 cells" % seed)
    if name == "small":
        t, n = w.gen_small(0)
        return [(t, n)], "small", "plain single small protocol, seed 0: 256 threads, for^S 16 x 4, 4 accesses"
    if name == "mixed":
        b = w.gen_mixed_batch(0, 4096)
        return [(t, n) for t, n, _ in b], "mixed", ("batched: 4096 seeded protocols (seed 0), 32..4096 threads, "
                                                    "depth 1..3, bounds 1..64, 2..8 accesses, 2^12..2^20 cells")
    if name == "tree":
        b = w.gen_tree_batch(0, 2048)
        return [(t, n) for t, n, _ in b], "tree", ("batched tree reductions: 2048 instances (seed 0), "
                                                   "2^8..2^20 threads, one level's sync removed in half")
    raise SystemExit("unknown workload " + name)


def golden_name(name: str, seed: int) -> str:
    return "large%d" % seed if name == "large" and seed else name


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
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp", "drf_layout.hpp"):
        with open(os.path.join(ROOT, "paper_2203_12878_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_value(kernel: str, wl: str, key: str = "traffic_bytes_per_launch"):
    """A per-launch value of `kernel` on workload `wl` from the committed
    rocprofv3 counter summary (HBM bytes, VALU lane operations), or None when
    none exists or the kernels have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "%s_%s_counters.md" % (kernel, wl))
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
        return int(vals[key])
    except (KeyError, ValueError):
        return None


def counts_sha(c) -> str:
    """The stored digest: sha256 of the per-phase counts in decimal, space separated."""
    c = c.tolist() if hasattr(c, "tolist") else list(c)
    return hashlib.sha256(" ".join(str(int(x)) for x in c).encode()).hexdigest()


def parity(results, gname: str):
    """Every field of every result against the stored oracle results (None
    when none are stored for this workload)."""
    path = os.path.join(GOLDEN, "expected_%s.json" % gname)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        exp = json.load(f)["results"]
    return len(exp) == len(results) and all(
        [r.status, r.racy, list(r.witness) if r.witness else None, r.num_records] ==
        [e["status"], e["racy"], e["witness"], e["num_records"]] and
        (r.status != 0 or (len(r.phase_counts) == e["num_phases"] and counts_sha(r.phase_counts) ==
                           e["phase_counts_sha256"])) for r, e in zip(results, exp))


def parity_subset(results, gname: str, idx):
    """Results of the protocols idx of a stored workload against its stored
    oracle results."""
    path = os.path.join(GOLDEN, "expected_%s.json" % gname)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        exp = json.load(f)["results"]
    sub = [exp[i] for i in idx]
    return len(sub) == len(results) and all(
        [r.status, r.racy, list(r.witness) if r.witness else None, r.num_records] ==
        [e["status"], e["racy"], e["witness"], e["num_records"]] and
        (r.status != 0 or (len(r.phase_counts) == e["num_phases"] and counts_sha(r.phase_counts) ==
                           e["phase_counts_sha256"])) for r, e in zip(results, sub))


def table_ab(drf, chk, steps, lib):
    """The sort-free table path for dense big phases against the partition
    path on the whole mixed and tree batches (same tuning otherwise), both
    with parity against the stored oracle results."""
    out = {}
    for name, bits in (("mixed", 20), ("tree", 24)):
        items, wl, _ = workload(name, 0)
        b = drf.Batch(items, 0)
        row = {"table_bits": bits}
        for leg, tb in (("partition", drf.TABLE_OFF), ("table", bits)):
            chk.set_tuning(table_bits=tb)
            secs, st = timed(chk.run_batch, b, steps, 1, lib, chk._ctx)
            res = b.collect()
            row[leg + "_ms"] = round(secs * 1e3, 3)
            row[leg + "_records_per_s"] = round(sum(r.num_records for r in res) / secs, 1)
            row[leg + "_parity"] = parity(res, wl)
            row[leg + "_kernels"] = {k: [round(v["ms_per_step"], 3), v["records_per_step"]]
                                     for k, v in per_kernel(st, steps).items()}
        chk.set_tuning(table_bits=drf.TABLE_OFF)
        out[name] = row
    return out


def graph_leg(drf, chk, steps):
    """Shape-class graph against the direct batched call on the statically
    small protocols of the mixed batch: the whole subset as one batch, and
    batches of 8 (where launch overhead matters), both with parity."""
    import torch
    items, _, _ = workload("mixed", 0)
    tile = chk.tuning()["tile_events"]
    all_plans, _ = drf.plan_batch(items, chk)
    idx = [i for i, p in enumerate(all_plans) if p.status == 0 and p.max_phase_records <= tile]
    sub = [items[i] for i in idx]
    plans = [all_plans[i] for i in idx]
    phases = sum(p.num_phases for p in plans)
    gc = chk.graph_class(max_protocols=len(sub), max_nests=1 << 20, max_code_words=1 << 22, max_fixed=1 << 20,
                         max_phases=phases, max_units=1 << 20)
    out = {"protocols": len(sub)}
    b = drf.Batch(sub, 0, plans=plans)
    for name, run in (("direct", lambda bb: chk.run_batch(bb)), ("graph", lambda bb: gc.check(bb))):
        secs, _ = timed(run, b, steps, 1)
        res = b.collect()
        out[name + "_records_per_s"] = round(sum(r.num_records for r in res) / secs, 1)
        out[name + "_ms"] = round(secs * 1e3, 3)
        out["parity_" + name] = parity_subset(res, "mixed", idx)
    small = [drf.Batch(sub[j:j + 8], 0, plans=plans[j:j + 8]) for j in range(0, 64, 8)]
    for name, run in (("direct", lambda bb: chk.run_batch(bb)), ("graph", lambda bb: gc.check(bb))):
        for bb in small:
            run(bb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            for bb in small:
                run(bb)
                torch.cuda.synchronize()
        out["batch8_" + name + "_ms"] = round((time.perf_counter() - t0) / (5 * len(small)) * 1e3, 4)
        res = [r for bb in small for r in bb.collect()]
        out["batch8_parity_" + name] = parity_subset(res, "mixed", idx[:64])
    gc.close()
    return out


def timed(run, batch, steps, warmup, lib=None, ctx=None):
    """Warm-up runs, then `steps` timed runs bracketed by device syncs.
    Returns (seconds per step, per-kernel stats of the timed runs)."""
    import torch
    for _ in range(warmup):
        run(batch)
    torch.cuda.synchronize()
    if lib is not None:
        lib.drf_ctx_set_profiling(ctx, 1)
        kernel_stats(lib, ctx, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run(batch)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = None
    if lib is not None:
        lib.drf_ctx_set_profiling(ctx, 0)
        stats = kernel_stats(lib, ctx, reset=True)
    return (t1 - t0) / steps, stats


def roofline(stats, steps, records, wl):
    """Roofline entry of the kernel class with the largest time."""
    dname, d = max(stats.items(), key=lambda kv: kv[1]["ms"])
    launches = max(1, d["launches"])
    avg_ms = d["ms"] / launches
    if dname == "fused":
        # the fused path keeps its records in LDS and moves almost nothing
        # through HBM: it is bounded by instruction issue.  achieved = VALU
        # lane operations per launch (the committed rocprofv3 SQ_INSTS_VALU
        # x 64 of this workload, null once the kernels change) over the
        # launch time measured now, against the chip's 32-bit VALU peak
        ops = committed_value(dname, wl, "valu_lane_ops_per_launch")
        achieved = ops / (avg_ms / 1e3) / 1e9 if ops else None
        return {"kernel": dname, "bound": "alu", "achieved": round(achieved, 1) if achieved else None,
                "peak": round(VALU_PEAK_GOPS, 1), "unit": "Gops/s",
                "frac": round(achieved / VALU_PEAK_GOPS, 4) if achieved else None,
                "traffic": committed_value(dname, wl), "valu_lane_ops_per_launch": ops,
                "avg_launch_ms": round(avg_ms, 4)}
    achieved = d["bytes"] / (d["ms"] / 1e3) / 1e9
    return {"kernel": dname, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": committed_value(dname, wl),
            "bytes_per_launch": d["bytes"] // launches, "avg_launch_ms": round(avg_ms, 4)}


def per_kernel(stats, steps):
    return {k: {"ms_per_step": round(v["ms"] / steps, 4), "launches_per_step": v["launches"] // steps,
                "records_per_step": v["records"] // steps, "bytes_per_step": v["bytes"] // steps}
            for k, v in stats.items() if v["launches"]}


def leg_tuning(chk, batch, cache, base):
    """The headline's tuning, then the cached tuning of the batch's size
    class when there is one (cache None: the headline's)."""
    from paper_2203_12878_amd import autotune
    chk.set_tuning(**base)
    ent = autotune.apply_cached(chk, batch, cache_path=cache) if cache else None
    return dict(chk.tuning(), source="autotuner cache (%s)" % autotune.size_class(batch) if ent else "headline's")


def compare_paths(drf, chk, name, steps, cache=None, base=None):
    """Batched (one check over the whole set) against plain (one protocol
    per call) on a whole batched workload, both compared with the oracle:
    the batched check with the workload's own cached tuning (chosen for the
    whole batch), the plain calls with the library's default (tuning every
    call by its own protocol's size class is not part of the plain path)."""
    from paper_2203_12878_amd import autotune
    items, wl, _ = workload(name, 0)
    batch = drf.Batch(items, 0)
    tuning = leg_tuning(chk, batch, cache, base) if base else None
    out = {}
    for path, run, k in (("batched", chk.run_batch, steps), ("plain", chk.run_plain, 1)):
        if path == "plain" and base:
            chk.set_tuning(**autotune.DEFAULT)
        secs, _ = timed(run, batch, k, 1)
        res = batch.collect()
        out[path] = (secs, parity(res, wl))
    recs = sum(r.num_records for r in batch.collect())
    return {"protocols": len(items), "records": recs,
            "batched_records_per_s": round(recs / out["batched"][0], 1),
            "plain_records_per_s": round(recs / out["plain"][0], 1),
            "batched_ms": round(out["batched"][0] * 1e3, 3), "plain_ms": round(out["plain"][0] * 1e3, 3),
            "speedup": round(out["plain"][0] / out["batched"][0], 3),
            "parity_batched": out["batched"][1], "parity_plain": out["plain"][1], "tuning": tuning,
            "plain_tuning": "library default" if base else None}


def serving(drf, rates):
    """Poisson streams of 1000 requests (70/30 mixed / tree generators)
    through the server: latency percentiles, throughput, and parity of every
    result against the stored oracle results and against the request
    checked alone."""
    from paper_2203_12878_amd import workloads as w
    from paper_2203_12878_amd.server import Server, run_stream
    rows = []
    alone_chk = drf.Checker(0)
    for rate in rates:
        reqs = w.gen_requests(rate=float(rate), max_requests=1000, horizon_s=1.0)
        with Server(device=0, workers=4, budget_bytes=8 << 30) as srv:
            # warm the workers (first launches, pinned staging) outside the figures
            run_stream(srv, [(0.0,) + tuple(q[1:]) for q in reqs[:16]])
            srv.reset_stats()
            res, wall = run_stream(srv, reqs)
            st = srv.stats
        b = drf.Batch([(t, n) for _, t, n, _ in reqs], 0)
        alone_chk.run_plain(b)
        import torch
        torch.cuda.synchronize()
        alone = b.collect()
        recs = sum(r.num_records for r in res)
        rows.append({"offered_req_per_s": rate, "requests": len(reqs), "p50_ms": round(st.percentile(50) * 1e3, 3),
                     "p99_ms": round(st.percentile(99) * 1e3, 3), "records_per_s": round(recs / wall, 1),
                     "req_per_s": round(len(reqs) / wall, 1), "batches": st.batches,
                     "max_in_flight_bytes": st.max_in_flight_bytes, "graph_batches": st.graph_batches,
                     "parity_vs_oracle": parity(res, "serve%dk" % (rate // 1000)),
                     "parity_vs_alone": all(a.key() == m.key() for a, m in zip(alone, res))})
    alone_chk.close()
    return rows


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(items, records_target=2.0e8):
    """The C oracle on a bounded sample of the workload: the protocols in
    order until their planned events reach records_target, on one host
    thread and on all of the host's threads (up to 16)."""
    from oracle import o2
    from paper_2203_12878_amd import drf
    sample, est = [], 0
    for t, n in items:
        p = drf.plan(t, n)
        if sample and est + p.max_records > records_target:
            continue
        sample.append((t, n))
        est += p.max_records
        if est >= records_target:
            break
    nproc = os.cpu_count() or 1
    jobs = max(1, min(16, nproc, len(sample)))
    res1, s1 = o2.check_many(sample, jobs=1, timing=True)
    resn, sn = o2.check_many(sample, jobs=jobs, timing=True)
    recs = sum(r.num_records for r in res1)
    assert [r.key() for r in res1] == [r.key() for r in resn]
    what = "%d protocol(s) of the workload in generator order, %d access events" % (len(sample), recs)
    return {"value": round(recs / sn, 1), "unit": "records/s", "cores": jobs, "kind": "oracle",
            "sample": what + "; %d threads %.1f s" % (jobs, sn),
            "single_core": {"value": round(recs / s1, 1), "cores": 1, "seconds": round(s1, 2)},
            "nproc": nproc, "cpu_model": cpu_model()}


def calibrate_copy(mib: int):
    import torch
    n = mib << 20
    src = torch.ones(n // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": n, "read": n, "write": n}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mixed", choices=["mixed", "tree", "large", "small"])
    ap.add_argument("--seed", type=int, default=1, help="seed of the large protocol (1: one that writes)")
    ap.add_argument("--path", default="auto", choices=["auto", "plain", "batch"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline only (no paths / large / serving)")
    ap.add_argument("--tune", action="store_true", help="run the autotuner for this workload first (cached)")
    ap.add_argument("--no-tuning-cache", action="store_true", help="library default tuning")
    ap.add_argument("--tuning-cache", default=None, help="tuning cache file (default: the package's)")
    ap.add_argument("--tile-events", type=int, default=0, help="tuning override (0: cached or default)")
    ap.add_argument("--digit-bits", type=int, default=0)
    ap.add_argument("--unit-events", type=int, default=0)
    ap.add_argument("--item-events", type=int, default=0)
    ap.add_argument("--table-bits", type=int, default=0, help="table path for big phases (255: off)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the checker runs on one GPU; --gpus %d is not supported (there is no "
              "multi-GPU path)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return

    from paper_2203_12878_amd import autotune, drf

    items, wl, desc = workload(args.workload, args.seed)
    gname = golden_name(args.workload, args.seed)
    path = args.path if args.path != "auto" else ("plain" if len(items) == 1 else "batch")
    chk = drf.Checker(0)
    lib = drf.lib()
    batch = drf.Batch(items, 0)
    tuning_source = "library default"
    cache = args.tuning_cache or autotune.CACHE
    if args.tune:
        autotune.tune(chk, batch, cache_path=cache, verbose=True)
        tuning_source = "autotuned now"
    elif not args.no_tuning_cache and autotune.apply_cached(chk, batch, cache_path=cache):
        tuning_source = "autotuner cache (%s)" % autotune.size_class(batch)
    chk.set_tuning(tile_events=args.tile_events, digit_bits=args.digit_bits, unit_events=args.unit_events,
                   item_events=args.item_events, table_bits=args.table_bits)
    run = chk.run_plain if path == "plain" else chk.run_batch
    secs, stats = timed(run, batch, args.steps, args.warmup, lib, chk._ctx)
    results = batch.collect()
    records = sum(r.num_records for r in results)
    value = records / secs

    line = {
        "metric": "access records checked/s",
        "value": round(value, 1),
        "unit": "records/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(secs * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": desc, "name": wl, "path": "batched" if path == "batch" else "plain",
                   "protocols": len(items), "records_per_step": records,
                   "racy_protocols": sum(r.racy for r in results),
                   "tuning": dict(chk.tuning(), source=tuning_source)},
        "parity_vs_stored_oracle": parity(results, gname),
        "roofline": roofline(stats, args.steps, records, wl),
        "effective_hbm_frac": round(value * EFFECTIVE_BYTES_PER_RECORD / (HBM_PEAK_GBS * 1e9), 4),
        "kernels": per_kernel(stats, args.steps),
    }
    if not args.no_extras:
        base = chk.tuning()
        leg_cache = None if args.no_tuning_cache else cache
        line["paths"] = {n: compare_paths(drf, chk, n, args.steps, leg_cache, base) for n in ("mixed", "tree")}
        litems, _, ldesc = workload("large", args.seed)
        lb = drf.Batch(litems, 0)
        ltuning = leg_tuning(chk, lb, leg_cache, base)
        lsecs, lstats = timed(chk.run_plain, lb, max(3, args.steps), 1, lib, chk._ctx)
        lres = lb.collect()
        lrec = sum(r.num_records for r in lres)
        line["large"] = {"workload": ldesc, "path": "plain", "records_per_s": round(lrec / lsecs, 1),
                         "ms_per_step": round(lsecs * 1e3, 3), "records_per_step": lrec,
                         "racy": lres[0].racy, "parity_vs_stored_oracle": parity(lres, golden_name("large", args.seed)),
                         "roofline": roofline(lstats, max(3, args.steps), lrec, "large"),
                         "effective_hbm_frac": round(lrec / lsecs * EFFECTIVE_BYTES_PER_RECORD /
                                                     (HBM_PEAK_GBS * 1e9), 4),
                         "kernels": per_kernel(lstats, max(3, args.steps)), "tuning": ltuning}
        chk.set_tuning(**base)
        line["graph"] = graph_leg(drf, chk, args.steps)
        line["table_vs_partition"] = table_ab(drf, chk, min(args.steps, 5), lib)
        line["serving"] = serving(drf, [1000, 5000, 20000, 50000])
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(items)
    chk.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
