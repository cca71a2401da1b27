"""Autotuner for libdrf tile and radix-digit sizes.

For a workload (a prepared Batch) it measures full checks under candidate
tunings by coordinate descent over
    tile_events  (events sorted in one LDS tile / fused-path threshold)
    digit_bits   (most index bits of one MSD partition level)
    unit_events  (events per fused unit)
    item_events  (events per count / emit work item)
and keeps the fastest (a candidate replaces the best so far when it is at
least 1% faster: the check-to-check spread of the large workloads is about
0.5%).  Results are cached per size class of the workload
(log2 of its planned access events, log2 of its protocol count, whether it
has phases above one tile) in a JSON file; apply_cached() sets the cached
tuning of a batch's size class on a Checker.  The package ships the cache
of the tunings measured on an MI355X (tuning.json next to this file);
DRF_TUNING_CACHE points elsewhere.  Tunings never change results, only
speed.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Optional

from . import drf

SPACE = {
    "tile_events": [2048, 4096, 8192],
    "digit_bits": [6, 8, 10],
    "unit_events": [4096, 16384, 32768, 49152, 65536, 262144],
    "item_events": [1 << 14, 1 << 16, 1 << 18],
}
DEFAULT = {"tile_events": 8192, "digit_bits": 10, "unit_events": 1 << 15, "item_events": 1 << 16}
CACHE = os.environ.get("DRF_TUNING_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json"))


def size_class(batch: "drf.Batch") -> str:
    ev = sum(int(p.max_records) for p in batch.plans if p.status == 0)
    big = any(p.status == 0 and p.max_phase_records > 8192 for p in batch.plans)
    return "e%d-p%d-%s" % (int(math.log2(ev + 1)), int(math.log2(batch.count + 1)), "big" if big else "small")


def load_cache(path: str = CACHE) -> Dict[str, dict]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: Dict[str, dict], path: str = CACHE) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_config(chk: "drf.Checker", batch: "drf.Batch", cfg: dict, reps: int = 2) -> float:
    import torch
    chk.set_tuning(**cfg)
    chk.run_batch(batch)                      # warm (pools grow here)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        chk.run_batch(batch)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def tune(chk: "drf.Checker", batch: "drf.Batch", rounds: int = 2, reps: int = 2,
         cache_path: Optional[str] = CACHE, verbose: bool = False) -> dict:
    """Coordinate descent from the default tuning; returns the best config
    and stores it in the cache under the batch's size class."""
    best = dict(DEFAULT)
    best_t = time_config(chk, batch, best, reps)
    trials = [(dict(best), best_t)]
    for _ in range(rounds):
        improved = False
        for key, values in SPACE.items():
            for v in values:
                if v == best[key]:
                    continue
                cfg = dict(best)
                cfg[key] = v
                t = time_config(chk, batch, cfg, reps)
                trials.append((cfg, t))
                if verbose:
                    print("tune", cfg, "%.3f ms" % (t * 1e3), flush=True)
                if t < best_t * 0.99:
                    best, best_t, improved = cfg, t, True
        if not improved:
            break
    chk.set_tuning(**best)
    if cache_path:
        cache = load_cache(cache_path)
        cache[size_class(batch)] = {"config": best, "seconds": best_t, "trials": len(trials)}
        save_cache(cache, cache_path)
    return {"config": best, "seconds": best_t, "default_seconds": trials[0][1], "trials": trials}


def apply_cached(chk: "drf.Checker", batch: "drf.Batch", cache_path: str = CACHE) -> Optional[dict]:
    """Set the cached tuning of the batch's size class (if any)."""
    ent = load_cache(cache_path).get(size_class(batch))
    if ent:
        chk.set_tuning(**ent["config"])
        return ent["config"]
    return None
