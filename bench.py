"""Benchmark of the zd-tree k-NN hot path on one MI355X.

Default workload (3D uniform, the headline configuration): n = 10,000,000
points uniform in [0,1)^3, leaf size 24 (the fastest whole step in a sweep
of leaf sizes 12-64), k = 10.  One step is one pass of the
whole path over resident inputs:

    build(10M) -> all-points k-NN -> insert 1M -> delete 1M -> all-points k-NN

`value` is whole-step throughput: the 20M all-points rows answered per step
divided by the step time.  Per-phase rates (build Mpts/s, query queries/s,
insert / delete Mpts/s) are reported beside it, each from HIP events on the
stream the library launches on.  The dominant kernel is the all-points query;
its roofline entry compares the algorithmic FP64 work it must do (from the
oracle's work counters on this workload) with the chip's FP64 vector issue
rate.  The CPU oracle is timed on a bounded sample for the cpu_baseline
entry (serial build; queries on one core and on a thread pool), and sampled
GPU rows are checked against it after the timed region.

After the headline step, the same line carries the other workloads under
"extra" (skip them with --no-extra), each timed on its own with HIP events
around library calls only: 1M external queries against the 10M tree, the
spheres set (build, k=10, k=50), the 4096-cloud forest (autotuned, one graph
replay against per-cloud calls) and the gradient workload.

Each workload also runs alone (one JSON line each, not the headline):
  --workload skewed    Plummer sphere and Kuzmin disk, 10M points each:
                       leaf-, bit- and root-based searches, k=10.
  --workload spheres   10M points on 64 noisy spheres + 1% background:
                       build, all-points k=10 and k=50.
  --workload forest    4096 Gaussian-mixture clouds (1,000-65,536 points):
                       autotuned leaf sizes, build + all-points k=16 as one
                       replayed HIP graph, against one build + query call
                       pair per cloud on the same GPU.
  --workload grad      1M uniform points, k=8: forward rows, backward kernel,
                       10 rounds of 1% insert + 1% delete; central finite
                       differences checked on 1,000 sampled coordinates.

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--no-cpu] [--no-extra]
                       [--workload W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 vector issue rate of MI355X: 256 CUs x 64 FP64 lanes per clock x 2.4 GHz
# (78.6 TFLOP/s counts a fused multiply-add as two operations; the distance
# code is built without fused operations, so each lane retires one op/clock).
FP64_VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0

# HBM bytes per point that this implementation's build moves (3D, 8 sort
# passes): Morton keys (24 B read, 8 B key + 4 B id written), 8 radix passes
# (8 B counted + 12 B read + 12 B written each), the gather into sorted order
# (4 B id + 24 B read, 24 B + 4 B id map written), and the tree pass (8 B
# keys read, 1 B split bit written and read, 4 + 4 B flag scan, 24 B
# coordinates read for the leaf boxes, 4 B leaf map, about 12 B of node
# records).  Reported beside the algorithmic fraction, not as it.
BUILD_BYTES_PER_POINT_IMPL = (24 + 12) + 8 * (8 + 12 + 12) + (4 + 24 + 24 + 4) + (8 + 2 + 8 + 24 + 4 + 12)


def build_bytes(n, n_nodes, dim=3):
    """Compulsory HBM bytes of one build: per point the coordinates read, the
    key written, one sort pass (key read and written, permutation written),
    the gather (coordinates read and written), the sorted keys read and the
    id map; per node one record of its split and tight box."""
    return n * 112 + 64 * n_nodes if dim == 3 else n * 88 + 48 * n_nodes


# Algorithmic FP64 work per all-points query on this workload (3D uniform,
# 10M points, k = 10), by leaf size: mean candidate distances (8 ops each:
# 3 sub, 3 mul, 2 add) and box tests (17 ops each) of the serial oracle's
# leaf-based search over 200,000 evenly spaced ids, printed by
# `python oracle/work_counters.py --leaf L`.
WORK_PER_QUERY = {8: (59.59, 64.24), 16: (92.0, 49.21), 24: (120.42, 41.3), 32: (134.92, 38.39),
                  40: (161.18, 34.25), 48: (180.7, 31.62)}


def ops_per_query(leaf):
    if leaf not in WORK_PER_QUERY:
        return None
    cand, box = WORK_PER_QUERY[leaf]
    return 8 * cand + 17 * box


PAPER_BUILD_QUERY_K10_QPS = 10_000_000 / 0.453  # CPU context only (144 threads)

# HBM bytes per launch of the all-points query kernel on this workload, from
# rocprofv3 FETCH_SIZE and WRITE_SIZE runs scaled by the same counters on a
# 1 GiB elementwise pass (profiles/knn_all_uniform3d_10M_k10_hbm_bytes.md).
# They describe the kernel sources whose code (comments stripped) has this
# sha1 only; after any change to that code the figure is reported as null
# until the counters are taken again.
KNN_TRAFFIC = {"sources_sha1": "bd39e10eeacda31631dec4386fd41d14d50a559d",
               "fetch_bytes": 2.015e+09, "write_bytes": 2.291e+09}
TRAFFIC_LEAF = 24  # leaf size of the profiled run
KNN_SOURCES = ("paper_2111_04182_amd/csrc/zd_knn_impl.h", "paper_2111_04182_amd/csrc/zd_internal.h",
               "paper_2111_04182_amd/csrc/zd_sortnet.h", "paper_2111_04182_amd/csrc/zd_knn_all_d3.hip")


def sources_sha1(paths):
    """sha1 of the code of C++/HIP sources: comments removed and whitespace
    collapsed, so that a comment-only edit does not count as a change."""
    import hashlib
    import re
    h = hashlib.sha1()
    for s in paths:
        with open(os.path.join(ROOT, s)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def knn_traffic():
    if KNN_TRAFFIC["sources_sha1"] != sources_sha1(KNN_SOURCES) or KNN_TRAFFIC["fetch_bytes"] is None:
        return None
    return KNN_TRAFFIC["fetch_bytes"] + KNN_TRAFFIC["write_bytes"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_info():
    """nproc, the threads this process may use (capped at 16, the host share
    of one GPU), and the CPU model name."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable": usable, "threads": max(1, min(usable, 16)),
            "model": model}


def cpu_baseline(P, n_sample: int, leaf: int):
    """The oracle as it stands (serial C), on a bounded sample of the same
    workload: a full serial build of all n points, then the leaf-based search
    for n_sample of them (every (n / n_sample)-th id), once on one core and
    once split over a pool of T threads (independent queries on the shared,
    read-only tree; the build stays serial)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    ci = cpu_info()
    t0 = time.perf_counter()
    tr = oracle.Tree(P, leaf, box=(np.zeros(3), np.ones(3)), seed=0)
    t_build = time.perf_counter() - t0
    qids = np.arange(0, P.shape[0], P.shape[0] // n_sample)[:n_sample]
    t0 = time.perf_counter()
    ids, d2 = tr.knn_all(10, qids=qids)
    t_query1 = time.perf_counter() - t0
    T = ci["threads"]
    chunks = np.array_split(qids, T * 4)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=T) as ex:
        parts = list(ex.map(lambda c: tr.knn_all(10, qids=c), chunks))
    t_queryT = time.perf_counter() - t0
    same = (np.array_equal(np.concatenate([x[0] for x in parts]), ids)
            and np.array_equal(np.concatenate([x[1] for x in parts]), d2))
    n = P.shape[0]
    per_q1, per_qT = t_query1 / len(qids), t_queryT / len(qids)
    return tr, qids, (ids, d2), {
        "value": n / (t_build + per_qT * n),
        "unit": "queries/s",
        "cores": T,
        "kind": "oracle",
        "sample": (f"serial oracle build of all {n} points ({t_build:.2f} s, 1 core) + "
                   f"leaf-based search of {len(qids)} of them on {T} threads "
                   f"({t_queryT:.2f} s; on 1 core {t_query1:.2f} s); value = n / (build + n x "
                   f"per-query time), i.e. build + one all-points pass"),
        "nproc": ci["nproc"], "cpu_model": ci["model"],
        "build_mpts_s_1core": n / t_build / 1e6,
        "query_qps_1core": len(qids) / t_query1,
        "query_qps_threads": len(qids) / t_queryT,
        "value_1core": n / (t_build + per_q1 * n),
        "threaded_rows_equal_serial": bool(same),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--m", type=int, default=1_000_000)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--leaf", type=int, default=24)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sample", type=int, default=500_000)
    ap.add_argument("--workload", default="uniform3d",
                    choices=["uniform3d", "spheres", "forest", "grad", "skewed"])
    ap.add_argument("--no-extra", action="store_true",
                    help="default workload only: skip the other workloads' keys (external "
                         "queries, spheres, forest, gradient)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one elementwise pass over a 1 GiB tensor (reads and writes "
                         "1 GiB: the reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2111_04182_amd as zd
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.add(src, 1.0, out=dst)  # one elementwise pass: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
    if args.workload != "uniform3d":
        {"spheres": bench_spheres, "forest": bench_forest, "grad": bench_grad,
         "skewed": bench_skewed}[args.workload](args)
        return
    n, m, k, L = args.n, args.m, args.k, args.leaf
    log(f"bench: generating inputs n={n} m={m}")
    P = W.uniform(n, 3, 0)
    Q = W.uniform(m, 3, 1)
    D = np.random.default_rng(2).choice(n + m, m, replace=False).astype(np.int32)
    xyz = zd.soa(torch.from_numpy(P))
    qxyz = zd.soa(torch.from_numpy(Q))
    dids = torch.from_numpy(D).cuda()
    box = (np.zeros(3), np.ones(3))
    torch.cuda.synchronize()

    phases = ["build", "query", "insert", "delete", "requery"]

    def step(record):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(phases) + 1)]
        ev[0].record()
        tree = zd.ZdTree(xyz, L, box=box, shift_seed=0)
        ev[1].record()
        out = tree.knn(k)
        ev[2].record()
        tree.insert(qxyz)
        ev[3].record()
        tree.delete(dids)
        ev[4].record()
        out2 = tree.knn(k)
        ev[5].record()
        record.append(ev)
        return tree, out, out2

    for i in range(args.warmup):
        log(f"bench: warmup {i}")
        t, _, _ = step([])
        t.close()
    torch.cuda.synchronize()
    recs = []
    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    for i in range(args.steps):
        tree, out, out2 = step(recs)
        if i < args.steps - 1:
            tree.close()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    ph = {p: float(np.mean([r[j].elapsed_time(r[j + 1]) for r in recs]))
          for j, p in enumerate(phases)}
    log("bench: phases (ms) " + json.dumps({p: round(v, 3) for p, v in ph.items()}))
    rows = 2 * n  # live rows answered per step (n before and n after the updates)
    value = rows / (ms_step / 1e3)
    # the query kernel runs twice per step (before and after the updates, 10M
    # live rows each); its launch time is the mean of the two
    q_launch_s = (ph["query"] + ph["requery"]) / 2 / 1e3
    opq = ops_per_query(L) if (n, k) == (10_000_000, 10) else None
    achieved_tops = n * opq / q_launch_s / 1e12 if opq else None
    # node count of the build (deterministic for these inputs), for the
    # build's compulsory bytes; taken outside the timed region
    probe = zd.ZdTree(xyz, L, box=box, shift_seed=0)
    pinfo = probe.info(depth=True)
    probe.close()
    n_nodes = pinfo["n_leaves"] + pinfo["n_internal"]
    b_bytes = build_bytes(n, n_nodes)
    result = {
        "metric": "all-points kNN queries/s and build Mpts/s (3D, 10M, k=10) at 1 MI355X",
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3D uniform [0,1)^3 n=10M, leaf {L}, k=10: build, all-points "
                               "k-NN, insert 1M, delete 1M, all-points k-NN",
                   "n": n, "k": k, "leaf_size": L, "insert": m, "delete": m},
        "build_mpts_s": n / (ph["build"] / 1e3) / 1e6,
        # compulsory bytes n*112 + 64*N_nodes against the time of the build
        "build_hbm_frac": b_bytes / (ph["build"] / 1e3) / (HBM_PEAK_GBS * 1e9),
        "build_bytes": b_bytes, "n_nodes": n_nodes, "depth": pinfo["depth"],
        # the bytes this implementation's build moves (8 sort passes) instead
        "build_hbm_frac_impl_bytes": n * BUILD_BYTES_PER_POINT_IMPL / (ph["build"] / 1e3)
        / (HBM_PEAK_GBS * 1e9),
        "query_qps": n / q_launch_s,
        "insert_mpts_s": m / (ph["insert"] / 1e3) / 1e6,
        "delete_mpts_s": m / (ph["delete"] / 1e3) / 1e6,
        "build_plus_query_qps": n / ((ph["build"] + ph["query"]) / 1e3),
        "phase_ms": ph,
        "paper_cpu_context": {"build_plus_query_k10_qps": PAPER_BUILD_QUERY_K10_QPS,
                              "hw": "4x Xeon E7-8867 v4, 144 threads"},
        "roofline": {"bound": "alu", "kernel": f"k_knn_all<3, {k}>",
                     "achieved": achieved_tops, "peak": FP64_VALU_PEAK_TOPS,
                     "unit": "TFLOP/s",
                     "frac": achieved_tops / FP64_VALU_PEAK_TOPS if achieved_tops else None,
                     "traffic": knn_traffic() if (n, k, L) == (10_000_000, 10, TRAFFIC_LEAF) else None,
                     "ops_per_query": opq, "launch_ms": q_launch_s * 1e3,
                     # the same launches against the HBM roofline: compulsory bytes
                     # per query = 24 B coordinates + 4 B id map + 12 B per
                     # neighbour written (the tree's nodes add < 2%)
                     "hbm_frac": n * (28 + 12 * k) / q_launch_s / (HBM_PEAK_GBS * 1e9)},
    }
    if not args.no_cpu:
        log("bench: CPU oracle baseline")
        tr, qids, want, cb = cpu_baseline(P, args.cpu_sample, L)
        result["cpu_baseline"] = cb
        # verification outside the timed region: sampled rows of the first query
        chk = qids[:: max(1, len(qids) // 2000)]
        sel = torch.from_numpy(chk).cuda()
        gi = out[0][sel].cpu().numpy()
        gd = out[1][sel].cpu().numpy()
        wi = want[0][:: max(1, len(qids) // 2000)]
        wd = want[1][:: max(1, len(qids) // 2000)]
        result["verified_rows"] = int(len(chk))
        result["verified"] = bool(np.array_equal(gi, wi) and np.array_equal(gd, wd))
    del out, out2
    if not args.no_extra:
        # the other workloads, each timed on its own (library work only,
        # HIP events on the stream the library launches on)
        extra = {}
        tree.close()
        legs = [("external_1M_k10",
                 lambda: leg_external(xyz, L, args.steps, tr if not args.no_cpu else None)),
                ("small_updates", lambda: leg_small_updates(P, L)),
                ("spheres_10M", lambda: leg_spheres(args.leaf, args.steps)),
                ("skewed_10M", lambda: leg_skewed(args.leaf, args.steps)),
                ("forest_4096", lambda: leg_forest(args.steps)),
                ("grad_1M_k8", lambda: leg_grad(fd_coords=100))]
        for name, fn in legs:
            log(f"bench: extra leg {name}")
            try:
                extra[name] = fn()
            except Exception as e:  # noqa: BLE001  (a failed leg must not hide the headline)
                extra[name] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
        result["extra"] = extra
    else:
        tree.close()
    print(json.dumps(result), flush=True)


def _events(fn, reps):
    """min and median over reps of fn's time between HIP events on the
    current stream (the library launches on it)."""
    import torch
    times = []
    out = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        out = fn()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times)), out


def _rows_equal(got, want, sel):
    gi = got[0][sel].cpu().numpy()
    gd = got[1][sel].cpu().numpy()
    return bool(np.array_equal(gi, want[0]) and np.array_equal(gd, want[1]))


def leg_external(xyz, L, steps, oracle_tree=None, m=1_000_000, k=10):
    """1M external queries (uniform in [0,1)^3, seed 3) against the 10M tree:
    the bit-based search of Section 2 after a Morton presort of the queries."""
    import torch
    import paper_2111_04182_amd as zd
    import workloads as W
    Q = W.uniform(m, 3, 3)
    qx = zd.soa(torch.from_numpy(Q))
    tree = zd.ZdTree(xyz, L, box=W.UNIT3, shift_seed=0)
    tree.knn(k, qx)
    ms, out = _events(lambda: tree.knn(k, qx), max(3, steps))
    res = {"queries": m, "k": k, "leaf_size": L, "query_ms": ms, "queries_per_s": m / ms * 1e3}
    if oracle_tree is not None:
        sel = np.arange(0, m, m // 500)
        res["verified_rows"] = int(len(sel))
        res["verified"] = _rows_equal(out, oracle_tree.knn(Q[sel], k), torch.from_numpy(sel).cuda())
    tree.close()
    return res


def leg_small_updates(P, leaf, batches=(1, 10, 100, 1000, 10000), reps=6, verify=200):
    """Latency of one insert and one delete call for small batches into
    trees of 1M (the first 1M points) and 10M points (Algorithm 4 applied in
    place: Fig. 4's small-batch end).  Each rep inserts m new uniform points
    and then deletes m random live ids (so n stays put); the median over
    reps 2..reps is reported, with the in-place state left pending.  Rows
    of sampled live points are checked against brute force at the end."""
    import torch
    import oracle
    import paper_2111_04182_amd as zd
    import workloads as W
    out = {}
    for n in (1_000_000, P.shape[0]):
        base = P[:n]
        t = zd.ZdTree(zd.soa(torch.from_numpy(base)), leaf, box=W.UNIT3, shift_seed=0)
        allp = [base]
        live = np.ones(n, dtype=bool)
        rng = np.random.default_rng(7)
        res = {}
        for m in batches:
            ti, td = [], []
            for rep in range(reps):
                B = rng.random((m, 3))
                Bx = zd.soa(torch.from_numpy(B))
                live = np.concatenate([live, np.ones(m, dtype=bool)])
                D = rng.choice(np.flatnonzero(live), m, replace=False).astype(np.int32)
                Dt = torch.from_numpy(D).cuda()
                torch.cuda.synchronize()
                e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                e[0].record()
                t.insert(Bx)
                e[1].record()
                t.delete(Dt)
                e[2].record()
                torch.cuda.synchronize()
                allp.append(B)
                live[D] = False
                if rep:
                    ti.append(e[0].elapsed_time(e[1]))
                    td.append(e[1].elapsed_time(e[2]))
            res[str(m)] = {"insert_us": float(np.median(ti)) * 1e3,
                           "delete_us": float(np.median(td)) * 1e3,
                           "pending_after": list(t.pending())}
        if verify:
            pts = np.concatenate(allp)
            sel = rng.choice(np.flatnonzero(live), verify, replace=False)
            got = t.knn(10)
            want = oracle.brute_knn(pts, 10, live=live, qids=sel)
            res["verified_rows"] = int(verify)
            res["verified"] = _rows_equal(got, want, torch.from_numpy(sel).cuda())
        t.check()
        t.close()
        out[f"n={n}"] = res
    return out


def leg_spheres(leaf, steps, verify=50):
    """10M points on 64 noisy spheres + 1% background: build, all-points
    k=10 and k=50."""
    import torch
    import oracle
    import paper_2111_04182_amd as zd
    import workloads as W
    log("bench spheres: generating 10M sphere-surface points")
    P = W.spheres_10m()
    xyz = zd.soa(torch.from_numpy(P))
    n = P.shape[0]
    res = {"n": n, "leaf_size": leaf}
    trees = []

    def build():
        t = zd.ZdTree(xyz, leaf, shift_seed=0)
        trees.append(t)
        return t

    res["build_ms"], tree = _events(build, max(3, steps))
    for t in trees[:-1]:
        t.close()
    outs = {}
    for k in (10, 50):
        res[f"query_k{k}_ms"], outs[k] = _events(lambda: tree.knn(k), max(3, steps))
        res[f"query_k{k}_qps"] = n / res[f"query_k{k}_ms"] * 1e3
    res["root_based_k10_ms"], _ = _events(lambda: tree.knn(10, root=True), max(3, steps))
    res["build_mpts_s"] = n / res["build_ms"] / 1e3
    if verify:
        sel = np.random.default_rng(5).choice(n, verify, replace=False)
        st = torch.from_numpy(sel).cuda()
        res["verified_rows"] = int(verify)
        res["verified"] = all(_rows_equal(outs[k], oracle.brute_knn(P, k, qids=sel), st)
                              for k in (10, 50))
    tree.close()
    return res


def leg_skewed(leaf, steps, n=10_000_000, k=10, verify=50):
    """The paper's skewed sets as synthetic stand-ins (Plummer sphere and
    Kuzmin disk, 10M points each, drawn from their published densities):
    build, then the three search starts of Section 2 -- leaf-based
    all-points rows, root-based all-points rows, and bit-based queries (the
    same points submitted as external queries, so rows include the point
    itself; the work has the same shape)."""
    import torch
    import oracle
    import paper_2111_04182_amd as zd
    import workloads as W
    out = {}
    for name, gen in (("plummer", W.plummer), ("kuzmin", W.kuzmin)):
        log(f"bench skewed: generating {name}")
        P = gen(n, seed=0)
        xyz = zd.soa(torch.from_numpy(P))
        trees = []

        def build():
            t = zd.ZdTree(xyz, leaf, shift_seed=0)
            trees.append(t)
            return t

        res = {"n": n, "k": k, "leaf_size": leaf}
        res["build_ms"], tree = _events(build, max(3, steps))
        for t in trees[:-1]:
            t.close()
        res["leaf_based_ms"], leaf_rows = _events(lambda: tree.knn(k), max(3, steps))
        res["root_based_ms"], root_rows = _events(lambda: tree.knn(k, root=True), max(3, steps))
        res["bit_based_ms"], _ = _events(lambda: tree.knn(k, xyz), max(3, steps))
        res["root_over_leaf"] = res["root_based_ms"] / res["leaf_based_ms"]
        res["bit_over_leaf"] = res["bit_based_ms"] / res["leaf_based_ms"]
        if verify:
            sel = np.random.default_rng(5).choice(n, verify, replace=False)
            st = torch.from_numpy(sel).cuda()
            want = oracle.brute_knn(P, k, qids=sel)
            res["verified_rows"] = int(verify)
            res["verified"] = _rows_equal(leaf_rows, want, st) and _rows_equal(root_rows, want, st)
        tree.check()
        tree.close()
        del xyz
        out[name] = res
    return out


def leg_forest(steps, k=16):
    """4096 Gaussian-mixture clouds: the tuner (3 timings per candidate),
    then build + all-points k=16 of every cloud as one captured-graph
    replay, the same as one persistent kernel launch, and one zd_build +
    zd_knn pair per cloud on the same GPU."""
    import torch
    import paper_2111_04182_amd as zd
    import workloads as W
    from paper_2111_04182_amd.autotune import tune_forest
    log("bench forest: generating 4096 clouds")
    P, off = W.forest_4096_clouds()
    N = P.shape[0]
    xyz = zd.soa(torch.from_numpy(P))
    log(f"bench forest: N={N}, autotuning leaf sizes and launch shape")
    ls, waves, rep = tune_forest(xyz, off, k, reps=3, log=log)
    plan = zd.ZdForestPlan(xyz, off, k, leaf_sizes=ls, query_waves=waves)
    plan.run()
    torch.cuda.synchronize()
    ms_forest, _ = _events(plan.run, max(5, steps))
    plan.check()
    # the same build + query as one persistent kernel launch (same leaf sizes)
    log("bench forest: persistent launch")
    pplan = zd.ZdForestPlan(xyz, off, k, leaf_sizes=ls, persistent=True)
    pplan.run()
    torch.cuda.synchronize()
    ms_persistent, _ = _events(pplan.run, max(5, steps))
    pplan.check()
    persistent_same = bool(torch.equal(pplan.ids, plan.ids) and torch.equal(pplan.d2, plan.d2))
    pplan.close()
    # the same work as one zd_build + zd_knn pair per cloud (boxes precomputed
    # on the host so no call synchronises)
    clouds = []
    for c in range(len(off) - 1):
        a, b = int(off[c]), int(off[c + 1])
        sub = P[a:b]
        lo = sub.min(axis=0)
        side = float((sub.max(axis=0) - lo).max()) or 1.0
        clouds.append((a, b, zd.soa(torch.from_numpy(sub)), (lo, lo + side), int(ls[c])))
    ids_pc = torch.empty((N, k), dtype=torch.int32, device="cuda")
    d2_pc = torch.empty((N, k), dtype=torch.float64, device="cuda")

    def per_cloud():
        for a, b, cx, box, L in clouds:
            t = zd.ZdTree(cx, L, box=box, query_waves=waves)
            zd.zd_knn(t.handle, None, b - a, k, ids_pc[a:b], d2_pc[a:b])
            t.close()

    per_cloud()
    torch.cuda.synchronize()
    ms_pc, _ = _events(per_cloud, 1)
    # same rows (ids of the per-cloud calls are local to the cloud)
    ok = True
    for a, b, _, _, _ in clouds[::64]:
        li = ids_pc[a:b]
        gi = torch.where(li >= 0, li + a, li)
        ok &= bool(torch.equal(gi, plan.ids[a:b]) and torch.equal(d2_pc[a:b], plan.d2[a:b]))
    plan.close()
    return {"N": N, "clouds": len(off) - 1, "k": k, "forest_graph_ms": ms_forest,
            "queries_per_s": N / ms_forest * 1e3, "per_cloud_calls_ms": ms_pc,
            "speedup_vs_per_cloud": ms_pc / ms_forest, "rows_match_per_cloud": ok,
            "persistent_launch_ms": ms_persistent,
            "persistent_rows_match_graph": persistent_same,
            "leaf_size_by_bucket": rep.get("choice"), "query_waves": waves,
            "autotune_best_ms": rep.get("best_ms"), "autotune_reps": 3}


def leg_grad(fd_coords=1000):
    """1M uniform points, k=8: forward rows, the backward kernel on its own,
    10 rounds of 1% insert + 1% delete (library calls only inside the
    events); central finite differences of the local loss on sampled
    coordinates, outside the timed regions."""
    import torch
    import paper_2111_04182_amd as zd
    import workloads as W
    k = 8
    P, fd, inserts, delete_rngs, m = W.uniform3d_1m_rounds()
    n0 = P.shape[0]
    pts = P.copy()
    live = np.ones(n0, dtype=bool)
    tree = zd.ZdTree(zd.soa(torch.from_numpy(P)), 16, box=W.UNIT3)
    times = {"forward": [], "backward": [], "backward_tree_order": [], "autograd_backward": [],
             "insert": [], "delete": []}
    tree_vs_id_order = 0.0
    worst = 0.0
    checked = 0
    for r in range(len(inserts)):
        xyz = zd.soa(torch.from_numpy(pts))
        live_t = torch.from_numpy(live).cuda()
        # forward: the library's k-NN rows
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        ids, d2 = tree.knn(k)
        e[1].record()
        torch.cuda.synchronize()
        times["forward"].append(e[0].elapsed_time(e[1]))
        # the backward kernel alone on dL/dd2 = 1 for live rows (prepared
        # before the events)
        g = live_t[:, None].to(torch.float64).expand(-1, k).contiguous()
        gx = torch.empty_like(xyz)
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        zd.zd_knn_backward(xyz, ids, g, gx)
        e[1].record()
        torch.cuda.synchronize()
        times["backward"].append(e[0].elapsed_time(e[1]))
        # the same in the tree's Morton order (three calls: the first one may
        # also take its scratch buffer from the library's caching allocator)
        for _ in range(3):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            e[0].record()
            gt = tree.knn_backward(ids, g)
            e[1].record()
            torch.cuda.synchronize()
            times["backward_tree_order"].append(e[0].elapsed_time(e[1]))
        tree_vs_id_order = max(tree_vs_id_order, float((gt - gx).abs().max() /
                                                       gx.abs().max().clamp(min=1.0)))
        # the autograd function end to end (torch's masking and sum included)
        xg = xyz.clone().requires_grad_(True)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        dd, _ = zd.knn_sq_dist(xg, tree, k)
        dd[live_t].sum().backward()
        e[1].record()
        torch.cuda.synchronize()
        times["autograd_backward"].append(e[0].elapsed_time(e[1]))
        grad = gx.cpu().numpy().T
        # central finite differences of the local loss (the terms touching
        # the perturbed point) on the sampled coordinates, untimed
        nb = ids.cpu().numpy()
        rows = np.arange(len(pts))
        for i, c in fd[: fd_coords if r == 0 else max(1, fd_coords // 10)]:
            if not live[i]:
                continue
            touch = (((rows == i)[:, None] | (nb == i)) & live[:, None]) & (nb >= 0)
            rr, jj = np.nonzero(touch)

            def local(Qp):
                diff = Qp[rr] - Qp[nb[rr, jj]]
                return float(np.sum(diff * diff))

            h = 1e-6
            Pp, Pm = pts.copy(), pts.copy()
            Pp[i, c] += h
            Pm[i, c] -= h
            fdv = (local(Pp) - local(Pm)) / (Pp[i, c] - Pm[i, c])
            worst = max(worst, abs(fdv - grad[i, c]) / max(1e-30, abs(grad[i, c])))
            checked += 1
        # 1% insert, 1% delete: batches and ids prepared before the events
        ins = zd.soa(torch.from_numpy(inserts[r]))
        new_live = np.concatenate([live, np.ones(m, dtype=bool)])
        D = delete_rngs[r].choice(np.flatnonzero(new_live), m, replace=False).astype(np.int32)
        Dt = torch.from_numpy(D).cuda()
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        tree.insert(ins)
        e[1].record()
        tree.delete(Dt)
        e[2].record()
        torch.cuda.synchronize()
        times["insert"].append(e[0].elapsed_time(e[1]))
        times["delete"].append(e[1].elapsed_time(e[2]))
        pts = np.concatenate([pts, inserts[r]])
        live = new_live
        live[D] = False
    tree.check()
    tree.close()
    med = {kk: float(np.median(v)) if v else None for kk, v in times.items()}
    return {"n": n0, "k": k, "median_ms": med, "fwd_bwd_points_per_s":
            n0 / (med["forward"] + med["backward"]) * 1e3, "fd_checked": checked,
            "fd_max_rel_err": worst, "backward_tree_order_calls": len(times["backward_tree_order"]),
            "backward_tree_vs_id_order_max_rel_diff": tree_vs_id_order}


def bench_spheres(args):
    res = leg_spheres(args.leaf, args.steps)
    total = res["build_ms"] + res["query_k10_ms"] + res["query_k50_ms"]
    print(json.dumps({
        "metric": "all-points kNN queries/s, 3D clustered spheres 10M (k=10 and k=50)",
        "value": 2 * res["n"] / (total / 1e3), "unit": "queries/s", "n_gpus": 1, "dtype": "f64",
        "data": "synthetic", "config": {"workload": "64 noisy spheres + 1% background, n=10M, "
                                                    f"leaf {args.leaf}: build, k=10, k=50"},
        **res}), flush=True)


def bench_skewed(args):
    res = leg_skewed(args.leaf, args.steps)
    print(json.dumps({
        "metric": "all-points kNN, leaf- vs bit- vs root-based search, skewed 10M sets (k=10)",
        "value": None, "unit": "ms", "n_gpus": 1, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "Plummer sphere and Kuzmin disk, 10M points each, "
                               f"leaf {args.leaf}, k=10"}, **res}), flush=True)


def bench_forest(args):
    res = leg_forest(args.steps)
    print(json.dumps({
        "metric": "batched forest all-points kNN queries/s (4096 clouds, k=16)",
        "value": res["queries_per_s"], "unit": "queries/s", "n_gpus": 1, "dtype": "f64",
        "data": "synthetic", "config": {"workload": "4096 Gaussian-mixture clouds, sizes "
                                                    "log-uniform 1000-65536, k=16"},
        **res}), flush=True)


def bench_grad(args):
    res = leg_grad()
    print(json.dumps({
        "metric": "differentiable k=8 squared-distance loss, 1M points, 10 update rounds",
        "value": res["fwd_bwd_points_per_s"], "unit": "points/s (fwd+bwd)",
        "n_gpus": 1, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "3D uniform n=1M, k=8, 1% insert + 1% delete per round"},
        **res}), flush=True)


if __name__ == "__main__":
    main()
