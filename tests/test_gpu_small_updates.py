"""Small batches applied in place (Algorithm 4 without rewriting the sorted
arrays): inserted points join their leaves' side blocks, deleted points
keep their slots marked dead.  After every batch the rows -- all-points
(leaf-based and root-based), external and allocation-free -- must equal
brute force over the live points; the canonical tree that zd_export then
restores must equal the oracle's build of the live set."""
import ctypes as C

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2111_04182_amd as zd  # noqa: E402
from paper_2111_04182_amd._lib import ZD_OK  # noqa: E402


def dev(P):
    return zd.soa(torch.from_numpy(np.asarray(P, dtype=np.float64)))


def rows(got):
    return got[0].cpu().numpy(), got[1].cpu().numpy()


def check_rows(t, allp, live, k, Q, what):
    want = oracle.brute_knn(allp, k, live=live)
    got = rows(t.knn(k))
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), what + " all"
    got = rows(t.knn(k, root=True))
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), what + " root"
    wq = oracle.brute_knn(allp, k, queries=Q, live=live)
    got = rows(t.knn(k, dev(Q)))
    assert np.array_equal(got[0], wq[0]) and np.array_equal(got[1], wq[1]), what + " ext"
    got = rows(t.knn(k, dev(Q), root=True))
    assert np.array_equal(got[0], wq[0]) and np.array_equal(got[1], wq[1]), what + " ext root"
    # the allocation-free call gives the same all-points rows
    m = t.cap
    o_ids = torch.empty((m, k), dtype=torch.int32, device="cuda")
    o_d2 = torch.empty((m, k), dtype=torch.float64, device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert zd.lib().zd_knn_noalloc(t.handle, None, m, k, C.c_void_p(o_ids.data_ptr()),
                                   C.c_void_p(o_d2.data_ptr()), s) == ZD_OK
    torch.cuda.synchronize()
    want = oracle.brute_knn(allp, k, live=live)
    assert np.array_equal(o_ids.cpu().numpy(), want[0]), what + " noalloc"


@pytest.mark.parametrize("dim,L,k", [(3, 16, 10), (2, 8, 5), (3, 24, 70), (2, 12, 33)])
def test_small_batches_in_place(dim, L, k):
    rng = np.random.default_rng(200 + dim + L)
    box = (np.zeros(dim), np.ones(dim))
    P = W.uniform(8000, dim, 201)
    t = zd.ZdTree(dev(P), leaf_size=L, box=box, shift_seed=4)
    allp = P.copy()
    live = np.ones(len(P), dtype=bool)
    Q = W.uniform(400, dim, 202)
    placed = 0
    for rnd in range(6):
        m = int(rng.integers(1, 60))
        B = rng.random((m, dim))
        new = t.insert(dev(B)).cpu().numpy()
        assert new.tolist() == list(range(len(allp), len(allp) + m))
        allp = np.concatenate([allp, B])
        live = np.concatenate([live, np.ones(m, dtype=bool)])
        pend = t.pending()
        placed = max(placed, pend[0])
        # delete a few: old points and some just inserted
        D = np.concatenate([rng.choice(np.flatnonzero(live[:8000]), 7, replace=False),
                            rng.choice(np.arange(len(allp) - m, len(allp)), min(3, m),
                                       replace=False)]).astype(np.int32)
        t.delete(torch.from_numpy(D).cuda())
        live[D] = False
        assert t.pending()[1] > 0
        check_rows(t, allp, live, k, Q, f"round {rnd}")
    assert placed > 0, "no batch was placed in place"
    t.check()
    # canonical again: the same tree as the oracle's build of the live set
    ex = t.export()
    assert t.pending() == (0, 0)
    ids = np.flatnonzero(live)
    o = oracle.Tree(allp[ids], L, box=box, shift=ex["shift"])
    oex = o.export()
    assert np.array_equal(ex["keys"], oex["keys"])
    assert np.array_equal(ex["ids"], ids[oex["ids"]])
    assert np.array_equal(ex["leaf_count"], oex["leaf_count"])
    assert np.array_equal(ex["int_bit"], oex["int_bit"])
    for f in ("leaf_lo", "leaf_hi", "int_lo", "int_hi"):
        assert np.array_equal(ex[f], oex[f]), f
    check_rows(t, allp, live, k, Q, "after export")
    t.close()


def test_same_leaf_overflow_falls_back():
    # many points into one spot: the leaf's block overflows, the batch takes
    # the rebuilding path; rows stay exact either way
    P = W.uniform(5000, 3, 210)
    t = zd.ZdTree(dev(P), leaf_size=16, box=W.UNIT3, shift_seed=5)
    allp, live = P.copy(), np.ones(len(P), dtype=bool)
    for rnd in range(4):
        B = 0.5 + 1e-4 * W.uniform(6, 3, 211 + rnd)
        t.insert(dev(B))
        allp = np.concatenate([allp, B])
        live = np.concatenate([live, np.ones(6, dtype=bool)])
        want = oracle.brute_knn(allp, 8, live=live)
        got = rows(t.knn(8))
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), rnd
    t.check()
    t.close()


def test_delete_everything_in_place_then_insert():
    P = W.uniform(300, 2, 220)
    t = zd.ZdTree(dev(P), leaf_size=4, box=W.UNIT2, shift_seed=6)
    allp, live = P.copy(), np.ones(300, dtype=bool)
    for a in range(0, 300, 15):
        t.delete(torch.arange(a, a + 15, dtype=torch.int32, device="cuda"))
        live[a:a + 15] = False
    want = oracle.brute_knn(allp, 3, live=live)
    got = rows(t.knn(3))
    assert np.array_equal(got[0], want[0])
    B = W.uniform(5, 2, 221)
    t.insert(dev(B))
    allp = np.concatenate([allp, B])
    live = np.concatenate([live, np.ones(5, dtype=bool)])
    want = oracle.brute_knn(allp, 3, live=live)
    got = rows(t.knn(3))
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    assert t.info()["n_live"] == 5
    t.close()


def test_small_update_rounds_1m_sampled():
    # config-5 sized rounds (1% of 1M) at a smaller rate: 2,000 in, 2,000 out
    rng = np.random.default_rng(230)
    P = W.uniform(1_000_000, 3, 231)
    t = zd.ZdTree(dev(P), leaf_size=16, box=W.UNIT3, shift_seed=7)
    allp, live = P.copy(), np.ones(len(P), dtype=bool)
    in_place = 0
    for rnd in range(3):
        B = rng.random((2000, 3))
        t.insert(dev(B))
        in_place = max(in_place, t.pending()[0])
        allp = np.concatenate([allp, B])
        live = np.concatenate([live, np.ones(2000, dtype=bool)])
        D = rng.choice(np.flatnonzero(live), 2000, replace=False).astype(np.int32)
        t.delete(torch.from_numpy(D).cuda())
        live[D] = False
        sel = np.concatenate([rng.choice(np.flatnonzero(live), 300, replace=False),
                              np.arange(len(allp) - 2000, len(allp), 50)])
        sel = sel[live[sel]]
        ids, d2 = t.knn(10)
        want = oracle.brute_knn(allp, 10, live=live, qids=sel)
        st = torch.from_numpy(sel).cuda()
        assert np.array_equal(ids[st].cpu().numpy(), want[0]), rnd
        assert np.array_equal(d2[st].cpu().numpy(), want[1]), rnd
    assert in_place > 0
    t.check()
    t.close()


def test_fold_large_batch_with_duplicates():
    # duplicate points give equal keys: folding pending small batches with
    # a large batch (past one workgroup's sort) must keep (key, id) order
    rng = np.random.default_rng(240)
    P = W.with_duplicates(20000, 3, 700, 241)
    box = (np.zeros(3), np.ones(3))
    t = zd.ZdTree(dev(P), leaf_size=8, box=box, shift_seed=9)
    allp, live = P.copy(), np.ones(len(P), dtype=bool)
    for rnd in range(3):
        B = P[rng.choice(len(P), 40, replace=False)]  # copies of existing points
        t.insert(dev(B))
        allp = np.concatenate([allp, B])
        live = np.concatenate([live, np.ones(40, dtype=bool)])
        D = rng.choice(np.flatnonzero(live), 30, replace=False).astype(np.int32)
        t.delete(torch.from_numpy(D).cuda())
        live[D] = False
    assert t.pending() != (0, 0)
    B = np.concatenate([P[rng.choice(len(P), 3000)], rng.random((2500, 3))])
    t.insert(dev(B))  # too large for the pool: folds everything in
    allp = np.concatenate([allp, B])
    live = np.concatenate([live, np.ones(len(B), dtype=bool)])
    assert t.pending() == (0, 0)
    want = oracle.brute_knn(allp, 6, live=live)
    got = rows(t.knn(6))
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    ex = t.export()
    ids = np.flatnonzero(live)
    oex = oracle.Tree(allp[ids], 8, box=box, shift=ex["shift"]).export()
    assert np.array_equal(ex["keys"], oex["keys"])
    assert np.array_equal(ex["ids"], ids[oex["ids"]])
    assert np.array_equal(ex["int_bit"], oex["int_bit"])
    t.check()
    t.close()
