"""Autotuner of the batched path: picks the constructor schedule, its lanes
per wave and the search-grid bin occupancy that track a sample batch
fastest, then the neighbours finder's LDS stage for that setting, and caches
the choice per GPU and multiplicity bucket.  Every candidate gives bitwise
the same tracks, so tuning only ever changes speed.
"""
from __future__ import annotations

import json
import math
import os
import time

CANDIDATES = ([dict(construct_schedule=0, construct_blocks=0, construct_lanes=a, bin_occupancy=o)
               for a in (0, 16, 32, 64) for o in (1.0, 2.0)] +
              [dict(construct_schedule=1, construct_blocks=0, bin_occupancy=1.0)])
NF_STAGES = (1, 2, 3)   # tried with the best of CANDIDATES (0, automatic, is part of it)


def bucket(evs) -> int:
    """Multiplicity bucket of a batch: log2 of the mean clusters per event."""
    n = sum(e.n_clusters for e in evs) / max(1, len(evs))
    return int(math.log2(max(n, 1.0)))


def cache_path() -> str:
    return os.environ.get("TPC_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "tpctrack", "tune.json"))


def _key(device_name: str, evs) -> str:
    return f"{device_name}|events={len(evs)}|bucket={bucket(evs)}"


def load(device_name: str, evs):
    try:
        return json.load(open(cache_path())).get(_key(device_name, evs))
    except (OSError, ValueError):
        return None


def autotune(tracker, evs, geo, bz, params=None, reps: int = 2, candidates=None,
             device_name: str = "gpu", use_cache: bool = True, log=None):
    """Time each candidate on the batch `evs` (device events) and return the
    best setting with the measurements.  The winner is applied to `tracker`."""
    import torch
    if use_cache:
        hit = load(device_name, evs)
        if hit:
            tracker.set_tuning(use_graph=1, **hit["best"])
            return hit
    results = []

    def timed(cand):
        tracker.set_tuning(use_graph=1, **cand)
        tracker.track_batch(evs, geo, bz, params)          # capture + warm
        torch.cuda.synchronize()
        best = math.inf
        for _ in range(reps):
            t0 = time.perf_counter()
            tracker.track_batch(evs, geo, bz, params)
            best = min(best, time.perf_counter() - t0)
        results.append(dict(setting=cand, seconds=best))
        if log:
            log(f"tune {cand}: {best * 1e3:.2f} ms")

    for cand in (candidates or CANDIDATES):
        timed(cand)
    if candidates is None:   # then the neighbours finder's stage for the best setting
        base = min(results, key=lambda r: r["seconds"])["setting"]
        for stage in NF_STAGES:
            timed(dict(base, nf_stage=stage))
    win = min(results, key=lambda r: r["seconds"])
    tracker.set_tuning(use_graph=1, **win["setting"])
    rec = dict(best=win["setting"], seconds=win["seconds"], tried=results,
               key=_key(device_name, evs))
    if use_cache:
        p = cache_path()
        try:
            os.makedirs(os.path.dirname(p), exist_ok=True)
            data = json.load(open(p)) if os.path.exists(p) else {}
            data[rec["key"]] = rec
            json.dump(data, open(p, "w"), indent=1)
        except OSError:
            pass
    return rec
