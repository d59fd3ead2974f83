"""GPU parity of the batched forest: every cloud's rows equal the oracle's
brute force over that cloud alone (ids global), for the eager calls and for
the captured graph, whatever leaf size each cloud uses."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2111_04182_amd as zd  # noqa: E402


def dev(P):
    return zd.soa(torch.from_numpy(np.asarray(P, dtype=np.float64)))


def mixed_clouds(seed=0, dim=3):
    """Clouds of very different sizes and shapes, including 0-, 1- and 2-point
    clouds, duplicated points and an exact grid (ties)."""
    rng = np.random.default_rng(seed)
    parts = [W.uniform(1, dim, seed + 1), W.uniform(2, dim, seed + 2), np.zeros((0, dim)),
             W.with_duplicates(40, dim, 5, seed + 3), W.grid_points((7,) * dim, 2, seed + 4)[:300],
             W.clustered_small(2500, dim, seed + 5), np.full((20, dim), 0.5)]
    for c in range(40):
        m = int(rng.integers(3, 1500))
        parts.append(rng.normal(rng.random(dim), rng.uniform(0.01, 0.2), (m, dim)))
    order = rng.permutation(len(parts))
    parts = [parts[i] for i in order]
    offsets = np.zeros(len(parts) + 1, dtype=np.int64)
    np.cumsum([len(p) for p in parts], out=offsets[1:])
    return np.concatenate(parts), offsets


def oracle_rows(P, offsets, k):
    ids = np.full((len(P), k), -1, dtype=np.int32)
    d2 = np.full((len(P), k), np.inf)
    for c in range(len(offsets) - 1):
        a, b = offsets[c], offsets[c + 1]
        if b == a:
            continue
        ci, cd = oracle.brute_knn(P[a:b], k)
        ids[a:b] = np.where(ci >= 0, ci + a, -1)
        d2[a:b] = cd
    return ids, d2


def same(got, want, what):
    gi, gd = (x.cpu().numpy() for x in got)
    bad = np.argwhere(gi != want[0])
    assert bad.size == 0, f"{what}: ids differ at {bad[:5].tolist()}"
    assert np.array_equal(gd, want[1]), f"{what}: d2 differ"


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("k", [1, 8, 16, 33, 90])
def test_forest_rows_match_per_cloud_oracle(dim, k):
    P, off = mixed_clouds(10 + dim, dim)
    f = zd.ZdForest(dev(P), off, leaf_size=16, shift_seed=3)
    same(f.knn(k), oracle_rows(P, off, k), f"forest d={dim} k={k}")
    f.check()
    f.close()


def test_forest_per_cloud_leaf_sizes_do_not_change_rows():
    P, off = mixed_clouds(21)
    want = oracle_rows(P, off, 10)
    rng = np.random.default_rng(5)
    for trial in range(3):
        ls = rng.integers(1, 40, len(off) - 1).astype(np.int32)
        f = zd.ZdForest(dev(P), off, leaf_sizes=ls, shift_seed=trial)
        same(f.knn(10), want, f"leaf sizes trial {trial}")
        f.close()


@pytest.mark.parametrize("waves", [2, 4])
def test_forest_query_waves_do_not_change_rows(waves):
    P, off = mixed_clouds(25)
    want = oracle_rows(P, off, 16)
    f = zd.ZdForest(dev(P), off, leaf_size=12, query_waves=waves)
    same(f.knn(16), want, f"forest waves={waves}")
    f.close()
    plan = zd.ZdForestPlan(dev(P), off, 16, leaf_size=12, query_waves=waves)
    ids, d2 = plan.run()
    torch.cuda.synchronize()
    same((ids, d2), want, f"forest plan waves={waves}")
    plan.close()


def test_forest_with_declared_box():
    P, off = mixed_clouds(22)
    P = (P - P.min(axis=0)) / (P.max(axis=0) - P.min(axis=0) + 1e-9)
    f = zd.ZdForest(dev(P), off, leaf_size=8, box=W.UNIT3)
    same(f.knn(6), oracle_rows(P, off, 6), "declared box")
    f.close()


def test_forest_graph_replays():
    P, off = mixed_clouds(23)
    xyz = dev(P)
    plan = zd.ZdForestPlan(xyz, off, 12, leaf_size=16, shift_seed=1)
    want = oracle_rows(P, off, 12)
    for rep in range(3):
        ids, d2 = plan.run()
        torch.cuda.synchronize()
        same((ids.clone(), d2.clone()), want, f"replay {rep}")
        # eager work between replays
        f = zd.ZdForest(xyz, off, leaf_size=4)
        same(f.knn(12), want, f"eager between replays {rep}")
        f.close()
    # new point coordinates in the same buffer: the replay rebuilds from them
    P2 = P.copy()
    P2[:, 0] = P2[:, 0] * 0.5 + 0.25
    xyz.copy_(dev(P2))
    ids, d2 = plan.run()
    torch.cuda.synchronize()
    same((ids, d2), oracle_rows(P2, off, 12), "replay on new coordinates")
    plan.check()
    plan.close()


def test_forest_scaled_matches_single_trees():
    P, off = W.forest_4096_clouds(n_clouds=48, seed=7)
    xyz = dev(P)
    k = 16
    f = zd.ZdForest(xyz, off, leaf_size=16)
    gi, gd = f.knn(k)
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    rng = np.random.default_rng(8)
    for c in range(len(off) - 1):
        a, b = int(off[c]), int(off[c + 1])
        t = zd.ZdTree(dev(P[a:b]), 16)
        ti, td = t.knn(k)
        ti, td = ti.cpu().numpy(), td.cpu().numpy()
        assert np.array_equal(gi[a:b], np.where(ti >= 0, ti + a, -1)), f"cloud {c} ids"
        assert np.array_equal(gd[a:b], td), f"cloud {c} d2"
        t.close()
        if c % 8 == 0:
            rows = rng.choice(b - a, 25, replace=False)
            wi, wd = oracle.brute_knn(P[a:b], k, qids=rows)
            assert np.array_equal(gi[a + rows], np.where(wi >= 0, wi + a, -1))
            assert np.array_equal(gd[a + rows], wd)
    f.close()


def test_forest_argument_errors():
    P, off = mixed_clouds(24)
    xyz = dev(P)
    bad = off.copy()
    bad[-1] += 1
    with pytest.raises(zd.ZdError):
        zd.ZdForest(xyz, bad)
    bad = off.copy()
    bad[3], bad[4] = bad[4], bad[3]
    if bad[3] > bad[4]:
        with pytest.raises(zd.ZdError):
            zd.ZdForest(xyz, bad)
    with pytest.raises(zd.ZdError):
        zd.ZdForest(xyz, off, leaf_sizes=np.zeros(len(off) - 1, dtype=np.int32))


@pytest.mark.timeout(900)
def test_forest_4096_clouds_full_size_sampled():
    """The full batched workload (4096 clouds, 62M points, k=16) as the bench
    runs it (captured plan, per-bucket leaf sizes): sampled rows of sampled
    clouds against the oracle's brute force over that cloud."""
    P, off = W.forest_4096_clouds()
    xyz = dev(P)
    k = 16
    sizes = np.diff(off)
    buckets = np.floor(np.log2(np.maximum(sizes, 1))).astype(np.int64)
    ls = np.where(buckets < 10, 24, 32).astype(np.int32)
    plan = zd.ZdForestPlan(xyz, off, k, leaf_sizes=ls)
    ids, d2 = plan.run()
    torch.cuda.synchronize()
    gi_all, gd_all = ids, d2
    rng = np.random.default_rng(11)
    for c in rng.choice(len(off) - 1, 12, replace=False):
        a, b = int(off[c]), int(off[c + 1])
        rows = rng.choice(b - a, min(40, b - a), replace=False)
        wi, wd = oracle.brute_knn(P[a:b], k, qids=rows)
        sel = torch.from_numpy(a + rows).cuda()
        gi = gi_all[sel].cpu().numpy()
        gd = gd_all[sel].cpu().numpy()
        assert np.array_equal(gi, np.where(wi >= 0, wi + a, -1)), f"cloud {c} ids"
        assert np.array_equal(gd, wd), f"cloud {c} d2"
    plan.close()
