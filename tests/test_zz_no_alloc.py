"""zd_knn_noalloc (the allocation-free query call) against zd_knn, through
the C ABI: two calls in a row, the second smaller, each bit-identical to
zd_knn's rows; the size limit is refused before anything runs."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2111_04182_amd as zd  # noqa: E402
from paper_2111_04182_amd._lib import ZD_ELIMIT, ZD_OK  # noqa: E402


def dev(P):
    return zd.soa(torch.from_numpy(np.asarray(P, dtype=np.float64)))


def p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def call(fn, tree, q, m, k):
    ids = torch.full((m, k), -7, dtype=torch.int32, device="cuda")
    d2 = torch.full((m, k), -7.0, dtype=torch.float64, device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert fn(tree.handle, p(q), m, k, p(ids), p(d2), s) == ZD_OK
    torch.cuda.synchronize()
    return ids.cpu().numpy(), d2.cpu().numpy()


@pytest.mark.parametrize("dim,k", [(3, 10), (2, 16), (3, 40)])
def test_noalloc_matches_zd_knn(dim, k):
    L = zd.lib()
    P = W.clustered_small(30000, dim, 80 + dim)
    t = zd.ZdTree(dev(P), leaf_size=16, shift_seed=6)
    # two external batches in a row, the second smaller: the scratch keeps
    # the first call's contents, which must not leak into the second
    for m, seed in ((70001, 81), (4099, 82)):
        Q = dev(W.uniform(m, dim, seed) * 1.1 - 0.05)
        a = call(L.zd_knn_noalloc, t, Q, m, k)
        b = call(L.zd_knn, t, Q, m, k)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), (dim, k, m)
    # all-points rows (no scratch needed), after a delete so dead rows exist
    t.delete(torch.arange(0, 30000, 11, dtype=torch.int32, device="cuda"))
    a = call(L.zd_knn_noalloc, t, None, t.cap, k)
    b = call(L.zd_knn, t, None, t.cap, k)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    t.check()
    t.close()


def test_noalloc_refuses_batches_beyond_its_scratch():
    L = zd.lib()
    P = W.uniform(1000, 3, 83)
    t = zd.ZdTree(dev(P), leaf_size=16, box=W.UNIT3)
    m = (1 << 20) + 1
    Q = torch.zeros((3, m), dtype=torch.float64, device="cuda")
    ids = torch.full((m, 1), -7, dtype=torch.int32, device="cuda")
    d2 = torch.full((m, 1), -7.0, dtype=torch.float64, device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.zd_knn_noalloc(t.handle, p(Q), m, 1, p(ids), p(d2), s) == ZD_ELIMIT
    torch.cuda.synchronize()
    assert int((ids != -7).sum()) == 0  # nothing ran
    # the largest allowed batch runs
    m = 1 << 20
    a = call(L.zd_knn_noalloc, t, Q[:, :m].contiguous(), m, 1)
    assert np.all(a[0] >= 0)
    t.close()
