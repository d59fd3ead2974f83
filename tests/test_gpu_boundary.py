"""The C ABI's contract beyond the rows: self-checks that turn an unfinished
search into ZD_EDEVICE, the depth reported by zd_info, and queries from
several host threads on several streams."""
import threading

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2111_04182_amd as zd  # noqa: E402
from paper_2111_04182_amd._lib import ZD_EDEVICE, ZdError  # noqa: E402


def dev(P):
    return zd.soa(torch.from_numpy(np.asarray(P, dtype=np.float64)))


@pytest.mark.parametrize("external", [False, True])
def test_unfinished_search_is_reported(external):
    # a step limit far below what the walk needs: every search stops early
    # (and exits normally); the next synchronising call must say so
    P = W.uniform(5000, 3, 61)
    Q = W.uniform(700, 3, 62)
    t = zd.ZdTree(dev(P), leaf_size=8, box=W.UNIT3, shift_seed=1)
    t.knn(10, dev(Q) if external else None)
    t.check()  # the default limit is never reached
    zd.zd_set_walk_limit(t.handle, 3)
    t.knn(10, dev(Q) if external else None)
    with pytest.raises(ZdError) as e:
        t.check()
    assert e.value.code == ZD_EDEVICE
    # the tree is broken from now on: queries, info and updates refuse
    with pytest.raises(ZdError) as e:
        t.knn(10)
    assert e.value.code == ZD_EDEVICE
    with pytest.raises(ZdError):
        t.info()
    t.close()


def test_walk_limit_zero_restores_the_default():
    P = W.uniform(3000, 2, 63)
    t = zd.ZdTree(dev(P), leaf_size=8, box=W.UNIT2, shift_seed=2)
    zd.zd_set_walk_limit(t.handle, 0)
    ids, d2 = t.knn(5)
    t.check()
    want = oracle.brute_knn(P, 5)
    assert np.array_equal(ids.cpu().numpy(), want[0]) and np.array_equal(d2.cpu().numpy(), want[1])
    t.close()


@pytest.mark.parametrize("L", [1, 8, 24])
def test_depth_matches_oracle(L):
    for P, box in ((W.uniform(20000, 3, 64), W.UNIT3), (W.clustered_small(6000, 2, 65), None),
                   (W.with_duplicates(3000, 3, 50, 66), None)):
        t = zd.ZdTree(dev(P), leaf_size=L, box=box, shift_seed=3)
        o = oracle.Tree(P, L, box=box, seed=3)
        gi, oi = t.info(depth=True), o.info()
        assert gi["depth"] == oi["depth"]
        assert (gi["n_leaves"], gi["n_internal"]) == (oi["n_leaves"], oi["n_internal"])
        t.close()


def test_concurrent_queries_from_two_threads():
    P = W.uniform(40000, 3, 67)
    Q = W.uniform(5000, 3, 68)
    t = zd.ZdTree(dev(P), leaf_size=16, box=W.UNIT3, shift_seed=4)
    qd = dev(Q)
    want_all = oracle.brute_knn(P, 8)
    want_ext = oracle.brute_knn(P, 8, queries=Q)
    torch.cuda.synchronize()
    errors = []

    def worker(tag):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for _ in range(4):
                    a = t.knn(8, stream=s)
                    b = t.knn(8, qd, stream=s)
                    s.synchronize()
                    if not (np.array_equal(a[0].cpu().numpy(), want_all[0])
                            and np.array_equal(b[0].cpu().numpy(), want_ext[0])
                            and np.array_equal(b[1].cpu().numpy(), want_ext[1])):
                        errors.append(tag)
        except Exception as e:  # noqa: BLE001
            errors.append(f"{tag}: {e}")

    th = [threading.Thread(target=worker, args=(i,)) for i in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert not errors, errors
    t.check()
    t.close()


def test_update_waits_for_query_on_another_stream():
    # a query enqueued on a side stream reads the tree before the insert that
    # follows on the tree's own stream rewrites it
    P = W.uniform(200000, 3, 69)
    Q = W.uniform(50000, 3, 70)
    t = zd.ZdTree(dev(P), leaf_size=16, box=W.UNIT3, shift_seed=5)
    want = oracle.brute_knn(P, 10, qids=np.arange(0, len(P), 997))
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ids, d2 = t.knn(10, stream=s)
    t.insert(dev(Q))  # on the tree's stream, ordered after the query by the library
    torch.cuda.synchronize()
    sel = np.arange(0, len(P), 997)
    assert np.array_equal(ids.cpu().numpy()[sel], want[0])
    assert np.array_equal(d2.cpu().numpy()[sel], want[1])
    t.check()
    t.close()
