"""Autotuner for the batched forest: leaf size per cloud-size bucket and the
query launch shape.

The leaf size L of a zd-tree (the paper's sizeCutoff - 1, which it leaves
open) changes only the tree's shape, never the rows: a larger L scores more
points per leaf and visits fewer nodes.  Its best value depends on the cloud
size and on k, so the tuner picks one L per cloud-size bucket (clouds with
floor(log2(size)) == b share bucket b).  The query launch packs 1, 2 or 4
wavefronts (each answering 64 queries) into a workgroup; that changes the
scheduling, never the rows.  The search: the best single L for the whole
forest, then the best wavefronts-per-workgroup with that L, then, bucket by
bucket, the best L for that bucket with everything else held.  Every
candidate is timed as one full forest pass (build + all-points query)
through the library on the current GPU.  Choices are cached in a JSON file
keyed by "d{dim}:k{k}:b{bucket}" and "d{dim}:k{k}:waves".
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from ._lib import ZdForest

CANDIDATES = (4, 8, 12, 16, 24, 32)
WAVES = (1, 2, 4)


def size_buckets(offsets) -> np.ndarray:
    sizes = np.diff(np.asarray(offsets, dtype=np.int64))
    return np.floor(np.log2(np.maximum(sizes, 1))).astype(np.int64)


def _time_pass(xyz, offsets, k, leaf_sizes, reps, waves=1):
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        f = ZdForest(xyz, offsets, leaf_sizes=leaf_sizes, query_waves=waves)
        f.knn(k)
        e1.record()
        torch.cuda.synchronize()
        f.close()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune_forest(xyz, offsets, k, candidates=CANDIDATES, reps=2, cache_path=None,
                per_bucket=True, log=None, waves=WAVES):
    """Return (leaf_sizes int32 [C], query_waves, report dict).  xyz is the
    forest's SoA device tensor, offsets its host cloud bounds."""
    dim = int(xyz.shape[0])
    buckets = size_buckets(offsets)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    key = lambda b: f"d{dim}:k{k}:b{int(b)}"  # noqa: E731
    wkey = f"d{dim}:k{k}:waves"
    ub = sorted(set(int(b) for b in buckets))
    if wkey in cache and all(key(b) in cache for b in ub):
        ls = np.array([cache[key(b)] for b in buckets], dtype=np.int32)
        return ls, int(cache[wkey]), {"cached": True}

    def leaf_table(choice):
        return np.array([choice[int(x)] for x in buckets], dtype=np.int32)

    report = {"uniform": {}, "waves": {}, "per_bucket": {}}
    for L in candidates:
        ms = _time_pass(xyz, offsets, k, np.full(len(buckets), L, dtype=np.int32), reps)
        report["uniform"][L] = ms
        if log:
            log(f"autotune: L={L} all clouds: {ms:.3f} ms")
    best_l = min(report["uniform"], key=report["uniform"].get)
    choice = {b: best_l for b in ub}
    best_w, best_ms = 1, report["uniform"][best_l]
    for w in waves:
        ms = best_ms if w == 1 else _time_pass(xyz, offsets, k, leaf_table(choice), reps, w)
        report["waves"][w] = ms
        if log:
            log(f"autotune: {w} wavefronts per workgroup: {ms:.3f} ms")
        if ms < best_ms:
            best_w, best_ms = w, ms
    if per_bucket and len(ub) > 1:
        for b in ub:
            for L in candidates:
                if L == choice[b]:
                    continue
                trial = dict(choice)
                trial[b] = L
                ms = _time_pass(xyz, offsets, k, leaf_table(trial), reps, best_w)
                report["per_bucket"][f"{b}:{L}"] = ms
                if ms < best_ms:
                    best_ms, choice = ms, trial
            if log:
                log(f"autotune: bucket {b} -> L={choice[b]}")
    report["best_ms"] = best_ms
    report["choice"] = {int(b): int(v) for b, v in choice.items()}
    report["query_waves"] = best_w
    if cache_path:
        cache.update({key(b): int(v) for b, v in choice.items()})
        cache[wkey] = best_w
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return leaf_table(choice), best_w, report
