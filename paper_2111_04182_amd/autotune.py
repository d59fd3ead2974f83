"""Leaf-size autotuner for the batched forest.

The leaf size L of a zd-tree (the paper's sizeCutoff - 1, which it leaves
open) changes only the tree's shape, never the rows: a larger L scores more
points per leaf and visits fewer nodes.  Its best value depends on the cloud
size and on k, so the tuner picks one L per cloud-size bucket (clouds with
floor(log2(size)) == b share bucket b): first the best single L for the whole
forest, then, bucket by bucket, the best L for that bucket with the others
held.  Every candidate is timed as one full forest pass (build + all-points
query) through the library on the current GPU.  Choices are cached in a JSON
file keyed by "d{dim}:k{k}:b{bucket}".
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from ._lib import ZdForest

CANDIDATES = (4, 8, 12, 16, 24, 32)


def size_buckets(offsets) -> np.ndarray:
    sizes = np.diff(np.asarray(offsets, dtype=np.int64))
    return np.floor(np.log2(np.maximum(sizes, 1))).astype(np.int64)


def _time_pass(xyz, offsets, k, leaf_sizes, reps):
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        f = ZdForest(xyz, offsets, leaf_sizes=leaf_sizes)
        f.knn(k)
        e1.record()
        torch.cuda.synchronize()
        f.close()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune_forest(xyz, offsets, k, candidates=CANDIDATES, reps=2, cache_path=None,
                per_bucket=True, log=None):
    """Return (leaf_sizes int32 [C], report dict).  xyz is the forest's SoA
    device tensor, offsets its host cloud bounds."""
    dim = int(xyz.shape[0])
    buckets = size_buckets(offsets)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    key = lambda b: f"d{dim}:k{k}:b{int(b)}"  # noqa: E731
    ub = sorted(set(int(b) for b in buckets))
    if all(key(b) in cache for b in ub):
        ls = np.array([cache[key(b)] for b in buckets], dtype=np.int32)
        return ls, {"cached": True}
    report = {"uniform": {}, "per_bucket": {}}
    for L in candidates:
        ms = _time_pass(xyz, offsets, k, np.full(len(buckets), L, dtype=np.int32), reps)
        report["uniform"][L] = ms
        if log:
            log(f"autotune: L={L} all clouds: {ms:.3f} ms")
    best_l = min(report["uniform"], key=report["uniform"].get)
    choice = {b: best_l for b in ub}
    best_ms = report["uniform"][best_l]
    if per_bucket and len(ub) > 1:
        for b in ub:
            for L in candidates:
                if L == choice[b]:
                    continue
                trial = dict(choice)
                trial[b] = L
                ls = np.array([trial[int(x)] for x in buckets], dtype=np.int32)
                ms = _time_pass(xyz, offsets, k, ls, reps)
                report["per_bucket"][f"{b}:{L}"] = ms
                if ms < best_ms:
                    best_ms, choice = ms, trial
            if log:
                log(f"autotune: bucket {b} -> L={choice[b]}")
    report["best_ms"] = best_ms
    report["choice"] = {int(b): int(v) for b, v in choice.items()}
    if cache_path:
        cache.update({key(b): int(v) for b, v in choice.items()})
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    ls = np.array([choice[int(b)] for b in buckets], dtype=np.int32)
    return ls, report
