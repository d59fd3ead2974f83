"""GPU parity of the forest's single persistent launch
(zd_forest_plan_persistent): every cloud's rows equal the oracle's brute
force over that cloud alone (ids global) and the pass-by-pass plan's rows,
bit for bit, across dimensions, k buckets, per-cloud leaf sizes, a declared
box, degenerate clouds (empty, one and two points, duplicates, an exact
grid) and repeated replays on changing coordinates."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.test_gpu_forest import dev, mixed_clouds, oracle_rows, same

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2111_04182_amd as zd  # noqa: E402


def run(plan):
    ids, d2 = plan.run()
    torch.cuda.synchronize()
    return ids, d2


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("k", [1, 8, 16, 33, 90])
def test_persistent_rows_match_per_cloud_oracle(dim, k):
    P, off = mixed_clouds(30 + dim, dim)
    plan = zd.ZdForestPlan(dev(P), off, k, leaf_size=16, shift_seed=3, persistent=True)
    same(run(plan), oracle_rows(P, off, k), f"persistent d={dim} k={k}")
    plan.check()
    plan.close()


def test_persistent_leaf_sizes_and_box():
    P, off = mixed_clouds(31)
    P = (P - P.min(axis=0)) / (P.max(axis=0) - P.min(axis=0) + 1e-9)
    want = oracle_rows(P, off, 10)
    rng = np.random.default_rng(6)
    for trial in range(3):
        ls = rng.integers(1, 40, len(off) - 1).astype(np.int32)
        box = W.UNIT3 if trial == 1 else None
        plan = zd.ZdForestPlan(dev(P), off, 10, leaf_sizes=ls, box=box, shift_seed=trial,
                               persistent=True)
        same(run(plan), want, f"leaf sizes trial {trial}")
        plan.check()
        plan.close()


def test_plan_queries_need_a_run():
    """A plan's trees exist only after its first run: an eager query before
    it is refused instead of walking unbuilt arrays."""
    P, off = mixed_clouds(34)
    for persistent in (False, True):
        plan = zd.ZdForestPlan(dev(P), off, 8, leaf_size=16, persistent=persistent)
        ids = torch.empty_like(plan.ids)
        d2 = torch.empty_like(plan.d2)
        with pytest.raises(zd.ZdError):
            zd.zd_forest_knn(plan._h, 8, ids, d2)
        run(plan)
        zd.zd_forest_knn(plan._h, 8, ids, d2)
        torch.cuda.synchronize()
        same((ids, d2), oracle_rows(P, off, 8), f"after the first run ({persistent})")
        plan.close()


def test_persistent_replays_and_eager_queries():
    P, off = mixed_clouds(32)
    xyz = dev(P)
    plan = zd.ZdForestPlan(xyz, off, 12, leaf_size=16, shift_seed=1, persistent=True)
    want = oracle_rows(P, off, 12)
    for rep in range(3):
        ids, d2 = run(plan)
        same((ids.clone(), d2.clone()), want, f"replay {rep}")
        # eager work between replays, and an eager query of the trees the
        # launch built (the same rows through the all-points kernel)
        ids2 = torch.empty_like(ids)
        d22 = torch.empty_like(d2)
        zd.zd_forest_knn(plan._h, 12, ids2, d22)
        torch.cuda.synchronize()
        same((ids2, d22), want, f"eager query of the launch's trees {rep}")
        f = zd.ZdForest(xyz, off, leaf_size=4)
        same(f.knn(12), want, f"eager forest between replays {rep}")
        f.close()
    P2 = P.copy()
    P2[:, 0] = P2[:, 0] * 0.5 + 0.25
    xyz.copy_(dev(P2))
    same(run(plan), oracle_rows(P2, off, 12), "replay on new coordinates")
    plan.check()
    plan.close()


def test_persistent_matches_pass_by_pass_plan():
    """48 clouds of the batched workload's shape (Gaussian mixtures, sizes
    log-uniform in [1000, 65536]): the two plans' rows are identical."""
    P, off = W.forest_4096_clouds(n_clouds=48, seed=9)
    xyz = dev(P)
    sizes = np.diff(off)
    ls = np.where(np.log2(np.maximum(sizes, 1)) < 10, 24, 32).astype(np.int32)
    a = zd.ZdForestPlan(xyz, off, 16, leaf_sizes=ls)
    b = zd.ZdForestPlan(xyz, off, 16, leaf_sizes=ls, persistent=True)
    ai, ad = run(a)
    bi, bd = run(b)
    assert torch.equal(ai, bi) and torch.equal(ad, bd)
    rng = np.random.default_rng(10)
    for c in rng.choice(len(off) - 1, 6, replace=False):
        lo, hi = int(off[c]), int(off[c + 1])
        rows = rng.choice(hi - lo, 30, replace=False)
        wi, wd = oracle.brute_knn(P[lo:hi], 16, qids=rows)
        sel = torch.from_numpy(lo + rows).cuda()
        assert np.array_equal(bi[sel].cpu().numpy(), np.where(wi >= 0, wi + lo, -1))
        assert np.array_equal(bd[sel].cpu().numpy(), wd)
    b.check()
    a.close()
    b.close()


@pytest.mark.timeout(900)
def test_persistent_4096_clouds_full_size():
    """The full batched workload (4096 clouds, 62M points, k=16) in the
    bench's launch configuration: all rows equal the pass-by-pass plan's,
    and sampled rows of sampled clouds the oracle's brute force."""
    P, off = W.forest_4096_clouds()
    xyz = dev(P)
    k = 16
    sizes = np.diff(off)
    ls = np.where(np.log2(np.maximum(sizes, 1)) < 10, 24, 32).astype(np.int32)
    b = zd.ZdForestPlan(xyz, off, k, leaf_sizes=ls, persistent=True)
    bi, bd = run(b)
    b.check()
    a = zd.ZdForestPlan(xyz, off, k, leaf_sizes=ls)
    ai, ad = run(a)
    assert torch.equal(ai, bi) and torch.equal(ad, bd)
    a.close()
    rng = np.random.default_rng(12)
    for c in rng.choice(len(off) - 1, 8, replace=False):
        lo, hi = int(off[c]), int(off[c + 1])
        rows = rng.choice(hi - lo, min(40, hi - lo), replace=False)
        wi, wd = oracle.brute_knn(P[lo:hi], k, qids=rows)
        sel = torch.from_numpy(lo + rows).cuda()
        assert np.array_equal(bi[sel].cpu().numpy(), np.where(wi >= 0, wi + lo, -1))
        assert np.array_equal(bd[sel].cpu().numpy(), wd)
    b.close()
