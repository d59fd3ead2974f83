"""Every query kernel instantiation against the oracle's brute force.

The search kernels are instantiated once per (dimension, k bucket, search:
leaf-based all-points, bit-based external, root-based all-points and
external); each runs here at the bucket's top k and at
top - 1 (one padding slot), on an exact grid (every distance exactly
representable, so ties in d2 are everywhere and the (d2, id) order decides)
and on tight clusters with a sparse background.  Rows must equal brute force
bit for bit.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.kbuckets import bucket_cases

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2111_04182_amd as zd  # noqa: E402


def dev(P):
    return zd.soa(torch.from_numpy(np.asarray(P, dtype=np.float64)))


SETS = {
    ("grid", 2): lambda: W.grid_points((48, 40), 4, 21),
    ("grid", 3): lambda: W.grid_points((13, 12, 11), 3, 22),
    ("clustered", 2): lambda: W.clustered_small(2100, 2, 23),
    ("clustered", 3): lambda: W.clustered_small(2300, 3, 24),
}
_cache = {}


def case(name, dim):
    key = (name, dim)
    if key not in _cache:
        P = SETS[key]()
        rng = np.random.default_rng(30 + dim)
        lo, hi = P.min(axis=0), P.max(axis=0)
        # external queries: inside and around the data, plus copies of points
        Q = np.concatenate([lo + (hi - lo) * (rng.random((500, dim)) * 1.2 - 0.1), P[::17]])
        _cache[key] = (P, Q)
    return _cache[key]


def assert_rows(got, want, what):
    gi, gd = got[0].cpu().numpy(), got[1].cpu().numpy()
    if not np.array_equal(gi, want[0]):
        bad = np.argwhere(gi != want[0])[:5]
        raise AssertionError(f"{what}: ids differ at {bad.tolist()}")
    assert np.array_equal(gd, want[1]), f"{what}: d2 differ"


@pytest.mark.parametrize("mode", ["all", "ext", "root_all", "root_ext"])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("data", ["grid", "clustered"])
@pytest.mark.parametrize("k,bucket", bucket_cases(), ids=[f"k{k}-b{b}" for k, b in bucket_cases()])
def test_every_bucket_matches_brute_force(k, bucket, data, dim, mode):
    P, Q = case(data, dim)
    print(f"bucket {bucket} k={k} {data} {dim}D {mode} n={len(P)}", flush=True)
    t = zd.ZdTree(dev(P), leaf_size=8, shift_seed=bucket)
    root = mode.startswith("root")
    if mode.endswith("all"):
        assert_rows(t.knn(k, root=root), oracle.brute_knn(P, k), f"{data}{dim} {mode} k={k}")
    else:
        assert_rows(t.knn(k, dev(Q), root=root), oracle.brute_knn(P, k, queries=Q),
                    f"{data}{dim} {mode} k={k}")
    t.check()
    t.close()


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("data", ["grid", "clustered"])
@pytest.mark.parametrize("k,bucket", [(k, b) for k, b in bucket_cases() if 8 <= b <= 16],
                         ids=[f"k{k}-b{b}" for k, b in bucket_cases() if 8 <= b <= 16])
def test_sparse_external_queries(k, bucket, data, dim):
    """External queries at most a quarter as many as the tree's points run
    in lane teams at k = 8-16 (denser ones, as in the test above, one lane
    per query): the same rows as brute force."""
    P, Q = case(data, dim)
    Qs = Q[: len(P) // 5]
    assert 4 * len(Qs) <= len(P)
    print(f"bucket {bucket} k={k} {data} {dim}D sparse ext m={len(Qs)} n={len(P)}", flush=True)
    t = zd.ZdTree(dev(P), leaf_size=8, shift_seed=bucket)
    assert_rows(t.knn(k, dev(Qs)), oracle.brute_knn(P, k, queries=Qs),
                f"{data}{dim} sparse ext k={k}")
    t.check()
    t.close()
