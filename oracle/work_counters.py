"""Algorithmic work per all-points query, from the oracle's counters.

The roofline of the query kernel prices the work the method itself needs:
per query, C candidate distances (8 FP64 operations each: 3 subtractions,
3 multiplications, 2 additions) and V box tests (17 operations each) of the
paper's leaf-based search (Algorithms 2 and 3), as the serial oracle performs
them on the same tree.  This script builds the oracle tree of a workload,
runs the leaf-based search for an evenly spaced sample of ids and prints the
mean and 99th-percentile counts per query, the tree's node counts and depth
and its leaf-size histogram as one JSON line.

    python oracle/work_counters.py --n 10000000 --leaf 16 --k 10 --sample 200000

Test and measurement infrastructure only (it runs the oracle).
"""
import argparse
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--leaf", type=int, default=16)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--sample", type=int, default=200_000)
    a = ap.parse_args()
    P = W.uniform(a.n, 3, 0)
    t = oracle.Tree(P, a.leaf, box=(np.zeros(3), np.ones(3)), seed=0)
    qids = np.arange(0, a.n, max(1, a.n // a.sample))[: a.sample]
    _, _, cand, box = t.knn_all(a.k, qids=qids, work=True)
    info = t.info()
    sizes = t.export()["leaf_count"]
    hist = np.bincount(sizes)
    print(json.dumps({"workload": f"3D uniform n={a.n}, seed 0, box [0,1]^3", "leaf": a.leaf,
                      "k": a.k, "queries": int(len(qids)),
                      "candidates_per_query": round(float(cand.mean()), 2),
                      "candidates_p99": int(np.percentile(cand, 99)),
                      "box_tests_per_query": round(float(box.mean()), 2),
                      "box_tests_p99": int(np.percentile(box, 99)),
                      "fp64_ops_per_query": round(8 * float(cand.mean()) + 17 * float(box.mean()), 1),
                      "n_leaves": info["n_leaves"], "n_internal": info["n_internal"],
                      "depth": info["depth"], "mean_leaf_size": round(float(sizes.mean()), 2),
                      "leaf_size_hist": {int(s_): int(c) for s_, c in enumerate(hist) if c}}))
    t.close()


if __name__ == "__main__":
    main()
