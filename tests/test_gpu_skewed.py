"""Skewed data (Plummer sphere, Kuzmin disk): the three search starts of
Section 2 (leaf-based all-points rows, bit-based external queries, root-based
both ways) against brute force and against the oracle's own searches."""
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


def rows(got):
    return got[0].cpu().numpy(), got[1].cpu().numpy()


def eq(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


GEN = {"plummer": W.plummer, "kuzmin": W.kuzmin}


@pytest.mark.parametrize("k", [1, 10, 24, 50])
@pytest.mark.parametrize("name", ["plummer", "kuzmin"])
def test_skewed_small_all_searches(name, k):
    P = GEN[name](20000, seed=3)
    Q = GEN[name](3000, seed=4)
    t = zd.ZdTree(dev(P), leaf_size=16, shift_seed=7)
    o = oracle.Tree(P, 16, seed=7)
    want_all = oracle.brute_knn(P, k)
    want_ext = oracle.brute_knn(P, k, queries=Q)
    assert eq(rows(t.knn(k)), want_all), "leaf-based"
    assert eq(rows(t.knn(k, root=True)), want_all), "root-based"
    assert eq(rows(t.knn(k, dev(Q))), want_ext), "bit-based"
    assert eq(rows(t.knn(k, dev(Q), root=True)), want_ext), "root-based external"
    # the oracle's own root- and bit-based searches give the same rows
    assert eq(o.knn_root(k), want_all)
    assert eq(o.knn(Q, k), want_ext)
    t.check()
    t.close()


@pytest.mark.parametrize("name", ["plummer", "kuzmin"])
def test_skewed_1m_sampled(name):
    P = GEN[name](1_000_000, seed=0)
    t = zd.ZdTree(dev(P), leaf_size=24, shift_seed=0)
    sel = np.random.default_rng(9).choice(len(P), 300, replace=False)
    st = torch.from_numpy(sel).cuda()
    want = oracle.brute_knn(P, 10, qids=sel)
    for root in (False, True):
        ids, d2 = t.knn(10, root=root)
        assert eq((ids[st].cpu().numpy(), d2[st].cpu().numpy()), want), (name, root)
    Q = P[sel] * (1 + 1e-9)
    want_q = oracle.brute_knn(P, 10, queries=Q)
    for root in (False, True):
        assert eq(rows(t.knn(10, dev(Q), root=root)), want_q), (name, "external", root)
    t.check()
    t.close()
