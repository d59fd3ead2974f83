"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Ids and squared distances must be bit-identical (neighbours are exact; d2 is
evaluated in the same order with no fused operations on both sides).  Trees
are compared in their canonical in-order form.  Structure tests come first:
a tree that fails them stops the run before any query walks it.
"""
import os

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


def dev(P):
    return zd.soa(torch.from_numpy(np.asarray(P, dtype=np.float64)))


def canon(ex, dim):
    return dict(keys=ex["keys"], ids=ex["ids"], leaf_count=ex["leaf_count"],
                leaf_lo=ex["leaf_lo"][:, :dim], leaf_hi=ex["leaf_hi"][:, :dim],
                int_bit=ex["int_bit"], int_lo=ex["int_lo"][:, :dim], int_hi=ex["int_hi"][:, :dim])


def assert_same_tree(gex, oex, dim, what=""):
    a, b = canon(gex, dim), canon(oex, dim)
    for key in a:
        assert np.array_equal(a[key], b[key]), f"{what}: tree field {key} differs"


def assert_same_rows(got, want, what=""):
    gi, gd = (x.cpu().numpy() if hasattr(x, "cpu") else x for x in got)
    wi, wd = want
    if not np.array_equal(gi, wi):
        bad = np.argwhere(gi != wi)[:5]
        raise AssertionError(f"{what}: ids differ at {bad.tolist()}: "
                             f"{[(gi[r, c], wi[r, c]) for r, c in bad]}")
    assert np.array_equal(gd, wd), f"{what}: d2 differ"


def datasets():
    return [
        ("uniform2d", W.uniform(4000, 2, 1), (np.zeros(2), np.ones(2))),
        ("uniform3d", W.uniform(6000, 3, 2), (np.zeros(3), np.ones(3))),
        ("grid2d", W.grid_points((50, 50), 4, 3), None),
        ("grid3d", W.grid_points((14, 14, 14), 3, 4), None),
        ("dups3d", W.with_duplicates(3000, 3, 300, 5), None),
        ("dups2d", W.with_duplicates(2000, 2, 40, 6), None),
        ("collinear3d", W.collinear(2500, 3, 7), None),
        ("clustered3d", W.clustered_small(5000, 3, 8), None),
        ("allequal3d", np.full((50, 3), 0.25), None),
        ("single3d", W.uniform(1, 3, 9), None),
        ("pair2d", W.uniform(2, 2, 10), None),
    ]


DATA = datasets()
IDS = [d[0] for d in DATA]


# ------------------------------------------------------------ structure ----

@pytest.mark.parametrize("L", [1, 5, 16])
@pytest.mark.parametrize("case", range(len(DATA)), ids=IDS)
def test_tree_matches_oracle(case, L):
    name, P, box = DATA[case]
    dim = P.shape[1]
    g = zd.ZdTree(dev(P), leaf_size=L, box=box, shift_seed=17)
    gex = g.export()
    o = oracle.Tree(P, L, box=box, seed=17)
    oex = o.export()
    lo, hi, S, sh = o.params()
    assert np.array_equal(gex["params"], np.concatenate([lo, hi, S])), name
    assert np.array_equal(gex["shift"], sh), name
    check_tree(gex, P, L)
    assert_same_tree(gex, oex, dim, name)
    g.close()


# ------------------------------------------------------- all-points rows ----

@pytest.mark.parametrize("k", [1, 3, 10, 16, 18, 24, 29, 37, 50, 64])
@pytest.mark.parametrize("case", range(len(DATA)), ids=IDS)
def test_all_points_match_oracle(case, k):
    name, P, box = DATA[case]
    g = zd.ZdTree(dev(P), leaf_size=16, box=box, shift_seed=3)
    assert_same_rows(g.knn(k), oracle.brute_knn(P, k), f"{name} k={k}")
    g.close()


@pytest.mark.parametrize("L", [1, 2, 7, 32])
def test_leaf_size_does_not_change_rows(L):
    P = W.clustered_small(4000, 3, 11)
    want = oracle.brute_knn(P, 12)
    g = zd.ZdTree(dev(P), leaf_size=L, shift_seed=L)
    assert_same_rows(g.knn(12), want, f"L={L}")
    g.close()


@pytest.mark.parametrize("waves", [2, 4])
@pytest.mark.parametrize("k", [10, 20, 50, 64])
def test_query_waves_do_not_change_rows(waves, k):
    # 6,037 points = 95 wavefronts and 1,013 queries = 16 wavefronts: the last
    # workgroup of each launch is partly empty
    P = W.clustered_small(6037, 3, 12)
    Q = W.uniform(1013, 3, 13)
    g = zd.ZdTree(dev(P), leaf_size=16, shift_seed=4, query_waves=waves)
    assert_same_rows(g.knn(k), oracle.brute_knn(P, k), f"waves={waves} k={k}")
    assert_same_rows(g.knn(k, dev(Q)), oracle.brute_knn(P, k, queries=Q),
                     f"waves={waves} ext k={k}")
    g.close()


def test_uniform2d_10k_full():
    P = W.uniform2d_10k()
    g = zd.ZdTree(dev(P), leaf_size=16, box=W.UNIT2, shift_seed=0)
    o = oracle.Tree(P, 16, box=W.UNIT2, seed=0)
    assert_same_tree(g.export(), o.export(), 2, "uniform2d 10k")
    assert_same_rows(g.knn(10), oracle.brute_knn(P, 10), "uniform2d 10k")
    g.close()


# -------------------------------------------------------- external rows ----

@pytest.mark.parametrize("k", [1, 8, 16, 20, 30, 40, 45])
@pytest.mark.parametrize("case", [0, 1, 3, 4, 7], ids=[IDS[i] for i in (0, 1, 3, 4, 7)])
def test_external_queries_match_oracle(case, k):
    name, P, box = DATA[case]
    dim = P.shape[1]
    # queries inside and outside the data (outside the box is legal), plus copies of points
    Q = np.concatenate([W.uniform(700, dim, 40 + case) * 1.2 - 0.1, P[:100]])
    g = zd.ZdTree(dev(P), leaf_size=16, box=box, shift_seed=5)
    assert_same_rows(g.knn(k, dev(Q)), oracle.brute_knn(P, k, queries=Q), f"{name} ext k={k}")
    g.close()


# --------------------------------------------------------------- updates ----

@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("L", [1, 16])
def test_update_sequence_matches_oracle(dim, L):
    rng = np.random.default_rng(100 + dim + L)
    box = (np.zeros(dim), np.ones(dim))
    P = W.clustered_small(3000, dim, 101).clip(0, 1)
    g = zd.ZdTree(dev(P), leaf_size=L, box=box, shift_seed=9)
    o = oracle.Tree(P, L, box=box, seed=9)
    allp = P.copy()
    live = np.ones(len(P), dtype=bool)
    for rnd in range(5):
        Q = np.concatenate([rng.random((400, dim)),
                            W.with_duplicates(50, dim, 4, 200 + rnd).clip(0, 1)])
        new_g = g.insert(dev(Q)).cpu().numpy()
        new_o = o.insert(Q)
        assert np.array_equal(new_g, new_o)
        allp = np.concatenate([allp, Q])
        live = np.concatenate([live, np.ones(len(Q), dtype=bool)])
        assert_same_tree(g.export(), o.export(), dim, f"after insert {rnd}")
        D = rng.choice(np.flatnonzero(live), 450, replace=False).astype(np.int32)
        g.delete(torch.from_numpy(D).cuda())
        o.delete(D)
        live[D] = False
        gex = g.export()
        check_tree(gex, allp, L, np.flatnonzero(live))
        assert_same_tree(gex, o.export(), dim, f"after delete {rnd}")
        assert_same_rows(g.knn(9), oracle.brute_knn(allp, 9, live=live), f"round {rnd}")
    g.close()


def test_empty_tree_then_insert():
    box = W.UNIT3
    g = zd.ZdTree(torch.zeros((3, 0), dtype=torch.float64, device="cuda"), 8, box=box)
    assert g.info()["n_live"] == 0
    ids, d2 = g.knn(4, dev(W.uniform(10, 3, 1)))
    assert (ids.cpu().numpy() == -1).all() and np.isinf(d2.cpu().numpy()).all()
    P = W.uniform(300, 3, 2)
    g.insert(dev(P))
    assert_same_rows(g.knn(4), oracle.brute_knn(P, 4), "after first insert")
    g.delete(torch.arange(300, dtype=torch.int32, device="cuda"))
    assert g.info()["n_live"] == 0
    ids, _ = g.knn(4)
    assert (ids.cpu().numpy() == -1).all()
    g.close()


def test_update_errors_leave_tree_unchanged():
    P = W.uniform(2000, 3, 300)
    g = zd.ZdTree(dev(P), 8, box=W.UNIT3, shift_seed=1)
    before = g.export()
    bad = W.uniform(100, 3, 301)
    bad[42, 2] = 1.5
    with pytest.raises(zd.ZdError) as e:
        g.insert(dev(bad))
    assert e.value.code == 2
    for ids in ([1, 2, 2], [5, 2000], [-3], [7, 8, 10**7]):
        with pytest.raises(zd.ZdError) as e:
            g.delete(torch.tensor(ids, dtype=torch.int32))
        assert e.value.code == 3
    assert_same_tree(g.export(), before, 3, "after rejected updates")
    g.delete(torch.tensor([11], dtype=torch.int32))
    with pytest.raises(zd.ZdError) as e:
        g.delete(torch.tensor([11], dtype=torch.int32))
    assert e.value.code == 3
    live = np.ones(2000, dtype=bool)
    live[11] = False
    assert_same_rows(g.knn(5), oracle.brute_knn(P, 5, live=live), "after delete")
    g.close()


def test_invalid_arguments():
    P = dev(W.uniform(100, 3, 5))
    with pytest.raises(zd.ZdError):
        zd.ZdTree(P, leaf_size=0)
    with pytest.raises(zd.ZdError):
        zd.ZdTree(P, box=(np.zeros(3), np.array([1.0, 0.0, 1.0])))
    for w in (-1, 3, 8):
        with pytest.raises(zd.ZdError):
            zd.ZdTree(P, query_waves=w)
    g = zd.ZdTree(P, 4)
    with pytest.raises(zd.ZdError) as e:
        g.knn(zd.ZD_KMAX + 1)
    assert e.value.code == 6
    g.close()


@pytest.mark.parametrize("k", [65, 80, 100])
def test_large_k_matches_oracle(k):
    # the paper sweeps k up to 100 (Fig. 3(e)); 65-100 run in the LDS heap
    P = W.clustered_small(9000, 3, 31)
    Q = W.uniform(1500, 3, 32)
    g = zd.ZdTree(dev(P), leaf_size=24, shift_seed=8)
    assert_same_rows(g.knn(k), oracle.brute_knn(P, k), f"all k={k}")
    assert_same_rows(g.knn(k, dev(Q)), oracle.brute_knn(P, k, queries=Q), f"ext k={k}")
    assert_same_rows(g.knn(k, root=True), oracle.brute_knn(P, k), f"root k={k}")
    g.check()
    g.close()


# -------------------------------------------------------------- backward ----

@pytest.mark.parametrize("deterministic", [False, True])
def test_backward_matches_closed_form_and_fd(deterministic):
    P = W.uniform(3000, 3, 400)
    g = zd.ZdTree(dev(P), 16, box=W.UNIT3)
    xyz = dev(P)
    ids, d2 = g.knn(8)
    wn = np.random.default_rng(401).uniform(0.5, 2, (3000, 8))
    w = torch.from_numpy(wn).cuda()
    grad = zd.zd_knn_backward(xyz, ids, w, deterministic=deterministic).cpu().numpy().T
    ref = oracle.knn_grad(P, ids.cpu().numpy(), wn)
    scale = np.abs(ref).max()
    assert np.abs(grad - ref).max() <= 1e-13 * max(scale, 1.0)
    assert np.abs(grad.sum(axis=0)).max() < 1e-10
    # central finite differences of L = sum w * d2 over the fixed neighbour
    # table: L is quadratic in each coordinate, so the difference is exact up
    # to rounding (h_eff = fl(x + h) - fl(x - h))
    nb = ids.cpu().numpy()
    rows = np.repeat(np.arange(3000), 8)
    cols = nb.ravel()
    wf = wn.ravel()

    def loss(Q):
        diff = Q[rows] - Q[cols]
        return float(np.sum(wf * np.sum(diff * diff, axis=1)))

    rng = np.random.default_rng(402)
    for i, c in zip(rng.integers(0, 3000, 25), rng.integers(0, 3, 25)):
        Pp, Pm = P.copy(), P.copy()
        Pp[i, c] += 1e-6
        Pm[i, c] -= 1e-6
        fd = (loss(Pp) - loss(Pm)) / (Pp[i, c] - Pm[i, c])
        assert abs(fd - grad[i, c]) <= 1e-6 * max(abs(grad[i, c]), 1e-3), (i, c)
    if deterministic:
        again = zd.zd_knn_backward(xyz, ids, w, deterministic=True).cpu().numpy().T
        assert np.array_equal(grad, again)
    g.close()


def test_backward_modes_after_deletes():
    # dead rows (-1 neighbours) and rows beyond the table: both modes agree
    # with the closed form
    P = W.uniform(4000, 2, 403)
    g = zd.ZdTree(dev(P), 8, box=W.UNIT2)
    g.delete(torch.arange(0, 4000, 9, dtype=torch.int32, device="cuda"))
    ids, d2 = g.knn(6)
    wn = np.where(ids.cpu().numpy() >= 0, 1.0, 0.0)
    w = torch.from_numpy(wn).cuda()
    ref = oracle.knn_grad(P, ids.cpu().numpy(), wn)
    for det in (False, True):
        got = zd.zd_knn_backward(dev(P), ids, w, deterministic=det).cpu().numpy().T
        assert np.abs(got - ref).max() <= 1e-13 * max(np.abs(ref).max(), 1.0), det
    g.close()


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("dead", [False, True])
def test_backward_in_tree_order(dim, dead):
    """zd_knn_backward_tree (rows in the tree's Morton order, in-tile sums in
    LDS) against the closed form and the id-order kernel, over several
    1,024-point tiles: k = 8 and 12 (vector row loads; 12 with a half batch),
    k = 13 (one scalar batch and a ragged one), rows read through an
    unaligned view (scalar loads), with every id live or with dead rows
    after a streaming delete, then with small batches pending in place."""
    n = 5000 if dim == 3 else 4000
    P = W.uniform(n, dim, 412 + dim)
    box = (np.zeros(dim), np.ones(dim))
    g = zd.ZdTree(dev(P), 12, box=box)
    if dead:
        g.delete(torch.arange(0, n, 7, dtype=torch.int32, device="cuda"))
    assert g.pending() == (0, 0)
    rng = np.random.default_rng(414)
    for k in (8, 12, 13):
        ids, d2 = g.knn(k)
        idn = ids.cpu().numpy()
        wn = np.where(idn >= 0, rng.uniform(0.5, 2, idn.shape), 0.0)
        ref = oracle.knn_grad(P, idn, wn)
        tol = 1e-13 * max(np.abs(ref).max(), 1.0)
        w = torch.from_numpy(wn).cuda()
        # the same rows one element into a larger buffer: 8-byte aligned only
        wbuf = torch.zeros(wn.size + 1, dtype=torch.float64, device="cuda")
        wbuf[1:] = w.reshape(-1)
        for ww in (w, wbuf[1:].view(n, k)):
            got = g.knn_backward(ids, ww).cpu().numpy().T
            assert np.abs(got - ref).max() <= tol, (k, ww.data_ptr() % 16)
        plain = zd.zd_knn_backward(dev(P), ids, w).cpu().numpy().T
        assert np.abs(got - plain).max() <= tol
        if dead:
            assert np.all(got[np.arange(0, n, 7)] == 0.0)
    # in-place batches pending: points in the side pool (their rows in the
    # pool pass) and dead slots
    P2 = W.uniform(3, dim, 415) * 0.5 + 0.25
    g.insert(dev(P2))
    g.delete(torch.tensor([1, 2, 3], dtype=torch.int32, device="cuda"))
    assert g.pending()[0] > 0 and g.pending()[1] > 0
    allp = np.concatenate([P, P2])
    for k in (8, 13):
        ids, d2 = g.knn(k)
        idn = ids.cpu().numpy()
        assert np.all(idn[[1, 2, 3]] == -1)
        wn = np.where(idn >= 0, rng.uniform(0.5, 2, idn.shape), 0.0)
        ref = oracle.knn_grad(allp, idn, wn)
        tol = 1e-13 * max(np.abs(ref).max(), 1.0)
        w = torch.from_numpy(wn).cuda()
        got = g.knn_backward(ids, w).cpu().numpy().T
        assert np.abs(got - ref).max() <= tol, ("pending", k)
        assert np.all(got[[1, 2, 3]] == 0.0)
        plain = zd.zd_knn_backward(dev(allp), ids, w).cpu().numpy().T
        assert np.abs(got - plain).max() <= tol
    g.close()


@pytest.mark.parametrize("deterministic", [False, True])
def test_autograd_function(deterministic):
    P = W.uniform(2000, 3, 410)
    g = zd.ZdTree(dev(P), 16, box=W.UNIT3)
    xyz = dev(P).requires_grad_(True)
    d2, ids = zd.knn_sq_dist(xyz, g, 6, deterministic)
    loss = d2.sum()
    loss.backward()
    ref = oracle.knn_grad(P, ids.cpu().numpy(), np.ones((2000, 6)))
    assert np.allclose(xyz.grad.cpu().numpy().T, ref, rtol=1e-12, atol=1e-13)
    # with an in-place batch pending (the tree kernel takes the side pool's rows
    # in its second pass)
    Q = W.uniform(5, 3, 411) * 0.5 + 0.25
    g.insert(dev(Q))
    P2 = np.concatenate([P, Q])
    xyz2 = dev(P2).requires_grad_(True)
    d2, ids = zd.knn_sq_dist(xyz2, g, 6, deterministic)
    d2.sum().backward()
    ref = oracle.knn_grad(P2, ids.cpu().numpy(), np.ones((2005, 6)))
    assert np.allclose(xyz2.grad.cpu().numpy().T, ref, rtol=1e-12, atol=1e-13)
    g.close()


# ---------------------------------------------------- full-size sampled ----

@pytest.mark.timeout(600)
@pytest.mark.parametrize("L", [16, 24])
def test_uniform3d_10m_full_size_sampled(L):
    """3D uniform, n = 10M (leaf 24 is the bench's): tree equals the oracle's;
    sampled rows equal the oracle's; then insert 1M, delete 1M, re-query
    (sampled)."""
    P, Q, D = W.uniform3d_10m_updates()
    print(f"uniform3d 10M L={L}: building", flush=True)
    g = zd.ZdTree(dev(P), L, box=W.UNIT3, shift_seed=0)
    o = oracle.Tree(P, L, box=W.UNIT3, seed=0)
    gex, oex = g.export(), o.export()
    for key in ("keys", "ids", "leaf_count", "int_bit"):
        assert np.array_equal(gex[key], oex[key]), key
    ids, d2 = g.knn(10)
    rows = np.random.default_rng(5).choice(len(P), 20000, replace=False)
    want = o.knn_all(10, qids=rows)
    assert_same_rows((ids[torch.from_numpy(rows).cuda()], d2[torch.from_numpy(rows).cuda()]), want,
                     "uniform3d 10M rows")
    few = rows[:25]
    assert_same_rows((ids[torch.from_numpy(few).cuda()], d2[torch.from_numpy(few).cuda()]),
                     oracle.brute_knn(P, 10, qids=few), "uniform3d 10M brute rows")
    print(f"uniform3d 10M L={L}: updates", flush=True)
    g.insert(dev(Q))
    o.insert(Q)
    g.delete(torch.from_numpy(D).cuda())
    o.delete(D)
    gex, oex = g.export(), o.export()
    for key in ("keys", "ids", "leaf_count", "int_bit"):
        assert np.array_equal(gex[key], oex[key]), key
    ids, d2 = g.knn(10)
    live = np.flatnonzero(~np.isin(np.arange(len(P) + len(Q)), D))
    rows = np.random.default_rng(6).choice(live, 20000, replace=False)
    want = o.knn_all(10, qids=rows)
    assert_same_rows((ids[torch.from_numpy(rows).cuda()], d2[torch.from_numpy(rows).cuda()]), want,
                     "uniform3d 10M rows after updates")
    dead = D[:100]
    assert (ids[torch.from_numpy(dead).cuda()].cpu().numpy() == -1).all()
    g.close()


@pytest.mark.timeout(600)
def test_uniform3d_10m_external_sampled():
    """1M external queries (inside and slightly outside the box) against a
    10M-point tree at the bench's leaf size: sampled rows against the
    oracle's bit-based search and a few against brute force."""
    P = W.uniform(10_000_000, 3, 0)
    Q = W.uniform(1_000_000, 3, 7) * 1.02 - 0.01
    g = zd.ZdTree(dev(P), 24, box=W.UNIT3, shift_seed=0)
    o = oracle.Tree(P, 24, box=W.UNIT3, seed=0)
    ids, d2 = g.knn(10, dev(Q))
    rows = np.random.default_rng(8).choice(len(Q), 2000, replace=False)
    sel = torch.from_numpy(rows).cuda()
    assert_same_rows((ids[sel], d2[sel]), o.knn(Q[rows], 10), "external 1M rows")
    few = rows[:20]
    assert_same_rows((ids[torch.from_numpy(few).cuda()], d2[torch.from_numpy(few).cuda()]),
                     oracle.brute_knn(P, 10, queries=Q[few]), "external 1M brute rows")
    g.close()


@pytest.mark.parametrize("k", [10, 50])
def test_spheres_scaled(k):
    """Points on 64 noisy sphere surfaces plus uniform background (the
    sphere-surface workload at 1/25 scale): full rows against brute force on a
    sample, and against the oracle's own tree search on a larger sample."""
    P = W.spheres_10m(n=400_000)
    g = zd.ZdTree(dev(P), 16, shift_seed=2)
    ids, d2 = g.knn(k)
    rows = np.random.default_rng(k).choice(len(P), 4000, replace=False)
    sel = torch.from_numpy(rows).cuda()
    o = oracle.Tree(P, 16, seed=2)
    assert_same_tree(g.export(), o.export(), 3, "spheres tree")
    assert_same_rows((ids[sel], d2[sel]), o.knn_all(k, qids=rows), f"spheres k={k}")
    few = rows[:40]
    sel = torch.from_numpy(few).cuda()
    assert_same_rows((ids[sel], d2[sel]), oracle.brute_knn(P, k, qids=few), f"spheres brute k={k}")
    g.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("L", [16, 24])
def test_spheres_10m_full_size_sampled(L):
    """10M sphere-surface points, k = 10 and k = 50, sampled rows (leaf 24 is
    the bench's)."""
    P = W.spheres_10m()
    print(f"spheres 10M L={L}: building", flush=True)
    g = zd.ZdTree(dev(P), L, shift_seed=0)
    o = oracle.Tree(P, L, seed=0)
    gex, oex = g.export(), o.export()
    for key in ("keys", "ids", "leaf_count", "int_bit"):
        assert np.array_equal(gex[key], oex[key]), key
    rows = np.random.default_rng(9).choice(len(P), 5000, replace=False)
    sel = torch.from_numpy(rows).cuda()
    for k in (10, 50):
        ids, d2 = g.knn(k)
        assert_same_rows((ids[sel], d2[sel]), o.knn_all(k, qids=rows), f"spheres 10M k={k}")
        del ids, d2
    g.close()


def test_streams_and_block_reuse():
    """Trees built, queried, updated and freed on two streams in turn: the
    library's cached device blocks are reused only on the stream that
    released them, and a tree used on a second stream waits for its first."""
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    sets = [W.uniform(2000 + 700 * i, 3, 60 + i) for i in range(5)]
    wants = [oracle.brute_knn(P, 8) for P in sets]
    for rep in range(2):
        for i, P in enumerate(sets):
            s = sa if (i + rep) % 2 == 0 else sb
            other = sb if s is sa else sa
            with torch.cuda.stream(s):
                xyz = dev(P)
                t = zd.ZdTree(xyz, 16, stream=s)
            # query on the other stream, then on the tree's own
            with torch.cuda.stream(other):
                got = t.knn(8, stream=other)
            other.synchronize()
            assert_same_rows(got, wants[i], f"set {i} rep {rep} other stream")
            with torch.cuda.stream(s):
                got = t.knn(8, stream=s)
            s.synchronize()
            assert_same_rows(got, wants[i], f"set {i} rep {rep} own stream")
            t.close()
    torch.cuda.synchronize()
