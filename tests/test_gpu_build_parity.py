"""GPU parity of fresh builds on larger and degenerate inputs, against the
oracle's tree field by field:

* uniform sets of 300,000 points (2-D and 3-D: many sort tiles, deep trees);
* points in a ball far smaller than the declared box (keys that share their
  top 40 bits and more);
* repeated locations (equal keys, which order by id), up to one location
  repeated 20,000 times;
* sizes around one and two sort tiles.

All-points rows check the coordinates and the id -> slot map the build
writes beside the keys."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.treecheck import check_tree

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2111_04182_amd as zd  # noqa: E402
from tests.test_gpu_parity import assert_same_rows, assert_same_tree, dev  # noqa: E402

TILE = 4096  # keys per radix-sort workgroup


def ball(n, dim, seed, centre=0.5, side=1e-4):
    return centre + side * np.random.default_rng(seed).random((n, dim))


def cases():
    unit3 = (np.zeros(3), np.ones(3))
    unit2 = (np.zeros(2), np.ones(2))
    rng = np.random.default_rng(40)
    many = np.concatenate([np.repeat(rng.random((3, 3)), 10_000, axis=0),
                           rng.random((10_000, 3))])
    rng.shuffle(many)
    return [
        ("uniform3d_300k", W.uniform(300_000, 3, 41), unit3),
        ("uniform2d_300k", W.uniform(300_000, 2, 42), unit2),
        ("ball3d_60k", ball(60_000, 3, 43), unit3),
        ("ball2d_40k", ball(40_000, 2, 44, side=1e-6), unit2),
        ("ball3d_tile_plus_1", ball(TILE + 1, 3, 45), unit3),
        ("ball3d_two_tiles", ball(2 * TILE, 3, 46), unit3),
        ("dups2d_50k", W.with_duplicates(50_000, 2, 500, 47), None),
        ("dups3d_40k_heavy", many, None),
        ("equal3d_20k", np.full((20_000, 3), 0.375), unit3),
        ("equal2d_7k", np.full((7_000, 2), 0.625), unit2),
    ]


CASES = cases()


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_build_matches_oracle(case):
    name, P, box = CASES[case]
    dim = P.shape[1]
    g = zd.ZdTree(dev(P), leaf_size=16, box=box, shift_seed=5)
    g.check()
    gex = g.export()
    o = oracle.Tree(P, 16, box=box, seed=5)
    assert_same_tree(gex, o.export(), dim, name)
    check_tree(gex, P, 16)
    # rows of a sample of ids: coordinates and slot map in the sorted order
    ids = np.random.default_rng(case).choice(P.shape[0], min(2000, P.shape[0]), replace=False)
    gi, gd = (x.cpu().numpy() for x in g.knn(6))
    assert_same_rows((gi[ids], gd[ids]), o.knn_all(6, qids=ids), name)
    g.close()


def test_build_repeats_exactly():
    """Two builds of the same set give the same tree (the climb's arrival
    order varies from run to run; the links and boxes it writes do not)."""
    P = ball(80_000, 3, 48)
    box = (np.zeros(3), np.ones(3))
    a = zd.ZdTree(dev(P), leaf_size=8, box=box, shift_seed=2).export()
    b = zd.ZdTree(dev(P), leaf_size=8, box=box, shift_seed=2).export()
    for k in ("keys", "ids", "leaf_count", "int_bit", "leaf_lo", "leaf_hi"):
        assert np.array_equal(a[k], b[k]), k
