"""Serial CPU oracle for the zd-tree k-NN hot path (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU product library never imports,
links or calls it, and the two share no code.

The arithmetic lives in ``zd_oracle.c`` (plain C, ``-O2 -ffp-contract=off``):

* ``brute_knn`` -- the definition of the result (Section 1.1 of Blelloch &
  Dobson: the k-nearest-neighbor graph of P and dynamic queries), k smallest
  (d2, id) pairs per query, ties to the lower id;
* ``Tree`` -- the zd-tree step by step: random shift and Morton sort
  (Section 2, "Construction"), integer rounding (Section 3.1), buildTree
  (Algorithm 1, empty cuts pruned as in Section 2.1), searchDown / searchUp
  (Algorithms 2 and 3), bit-based queries (Section 2), batchInsert
  (Algorithm 4) and deletion (Section 2, "Batch-dynamic updates");
* ``knn_grad`` -- the closed-form gradient of a weighted sum of k-NN squared
  distances for a fixed neighbour table.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "zd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-fvisibility=hidden", "-Wall", "-Wextra", "-Wno-unused-parameter"]

OK, EINVAL, EBOUNDS, EID, ENOMEM = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile zd_oracle.c into oracle/liboracle.so with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
        vp, i64, i32, u64, dp = C.c_void_p, C.c_int64, C.c_int, C.c_uint64, C.c_void_p
        lib.zo_build.restype = vp
        lib.zo_build.argtypes = [i32, i32, dp, dp, u64, dp, dp, i64, C.POINTER(C.c_int)]
        lib.zo_free.argtypes = [vp]
        lib.zo_brute_knn.restype = i32
        lib.zo_brute_knn.argtypes = [i32, dp, i64, dp, i64, dp, dp, i64, i32, dp, dp]
        for fn in ("zo_knn_rows_work", "zo_knn_root_work", "zo_knn_ext_work"):
            getattr(lib, fn).restype = i32
            getattr(lib, fn).argtypes = [vp, dp, i64, i32, dp, dp, dp, dp]
        lib.zo_insert.restype = i32
        lib.zo_insert.argtypes = [vp, dp, i64, dp]
        lib.zo_delete.restype = i32
        lib.zo_delete.argtypes = [vp, dp, i64]
        lib.zo_info.argtypes = [vp, dp, dp, dp, dp, dp]
        lib.zo_export.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, dp]
        lib.zo_params.argtypes = [vp, dp, dp, dp, dp]
        lib.zo_counters.argtypes = [vp, dp, dp, dp]
        lib.zo_keys.argtypes = [i32, dp, dp, dp, dp, i64, dp]
        lib.zo_shift.argtypes = [i32, u64, dp]
        lib.zo_splitmix64.restype = u64
        lib.zo_splitmix64.argtypes = [u64, u64]
        lib.zo_knn_grad.argtypes = [i32, dp, i64, i64, i32, dp, dp, dp]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _soa(xyz) -> np.ndarray:
    """Row-major (n, d) float64 points -> contiguous SoA (d, n)."""
    a = np.asarray(xyz, dtype=np.float64)
    if a.ndim != 2 or a.shape[1] not in (2, 3):
        raise ValueError("points must have shape (n, 2) or (n, 3)")
    return np.ascontiguousarray(a.T)


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


def _check(code):
    if code != OK:
        raise OracleError(code)


def splitmix64(seed: int, i: int) -> int:
    return int(_load().zo_splitmix64(seed, i))


def shift(dim: int, seed: int) -> np.ndarray:
    out = np.zeros(3, dtype=np.uint64)
    _load().zo_shift(dim, seed, _p(out))
    return out[:dim].copy()


def keys(dim, lo, scale, shift_, xyz) -> np.ndarray:
    """Morton keys of the points (SoA or row-major) for a given box, scale and shift."""
    s = _soa(xyz)
    n = s.shape[1]
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    scale = np.ascontiguousarray(scale, dtype=np.float64)
    sh = np.ascontiguousarray(shift_, dtype=np.uint64)
    out = np.zeros(n, dtype=np.uint64)
    _load().zo_keys(dim, _p(lo), _p(scale), _p(sh), _p(s), n, _p(out))
    return out


def brute_knn(pts, k: int, queries=None, live=None, qids=None):
    """Brute-force k-NN (the definition).

    pts: points by id, (n, d).  queries: external query points or
    None for all-points rows (self excluded).  live: optional bool mask over
    ids.  qids: for all-points, the ids whose rows to compute.
    Returns (ids int32 [m, k], d2 float64 [m, k])."""
    s = _soa(pts)
    dim, cap = s.shape
    lv = None if live is None else np.ascontiguousarray(live, dtype=np.uint8)
    q = None
    qi = None
    if queries is not None:
        q = _soa(queries)
        m = q.shape[1]
    elif qids is not None:
        qi = np.ascontiguousarray(qids, dtype=np.int64)
        m = qi.shape[0]
    else:
        m = cap
    ids = np.empty((m, k), dtype=np.int32)
    d2 = np.empty((m, k), dtype=np.float64)
    _check(_load().zo_brute_knn(dim, _p(s), cap, _p(lv), cap, _p(q), _p(qi), m, k,
                                _p(ids), _p(d2)))
    return ids, d2


def knn_grad(pts, ids, g):
    """Closed-form gradient of sum g[r, j] * d2(p_r, p_ids[r, j]) w.r.t. points.

    pts (n, d) by id; ids, g: [rows, k] with rows <= n.
    Returns the gradient as (n, d)."""
    s = _soa(pts)
    dim, n = s.shape
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    g = np.ascontiguousarray(g, dtype=np.float64)
    rows, k = ids.shape
    out = np.zeros((dim, n), dtype=np.float64)
    _load().zo_knn_grad(dim, _p(s), n, rows, k, _p(ids), _p(g), _p(out))
    return out.T.copy()


class Tree:
    """The serial zd-tree (Algorithms 1-4)."""

    def __init__(self, pts, leaf_size=16, box=None, seed=0, shift=None):
        s = _soa(pts)
        self.dim, n = s.shape
        lo = hi = None
        if box is not None:
            lo = np.ascontiguousarray(box[0], dtype=np.float64)
            hi = np.ascontiguousarray(box[1], dtype=np.float64)
        sh = None if shift is None else np.ascontiguousarray(shift, dtype=np.uint64)
        st = C.c_int(-1)
        self._h = _load().zo_build(self.dim, leaf_size, _p(lo), _p(hi), seed, _p(sh),
                                   _p(s), n, C.byref(st))
        if not self._h:
            raise OracleError(st.value)
        self.leaf_size = leaf_size

    def close(self):
        if self._h:
            _load().zo_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        lo = np.zeros(3); hi = np.zeros(3); S = np.zeros(3)
        sh = np.zeros(3, dtype=np.uint64)
        _load().zo_params(self._h, _p(lo), _p(hi), _p(S), _p(sh))
        d = self.dim
        return lo[:d].copy(), hi[:d].copy(), S[:d].copy(), sh[:d].copy()

    def info(self):
        v = [np.zeros(1, dtype=np.int64) for _ in range(4)]
        dep = np.zeros(1, dtype=np.int32)
        _load().zo_info(self._h, *[_p(a) for a in v], _p(dep))
        return dict(n_live=int(v[0][0]), cap=int(v[1][0]), n_leaves=int(v[2][0]),
                    n_internal=int(v[3][0]), depth=int(dep[0]))

    def _rows(self, fn, k, qids, work):
        cap = self.info()["cap"]
        qi = None if qids is None else np.ascontiguousarray(qids, dtype=np.int64)
        m = cap if qi is None else qi.shape[0]
        return self._run(fn, _p(qi), m, k, work)

    def _run(self, fn, src, m, k, work):
        ids = np.empty((m, k), dtype=np.int32)
        d2 = np.empty((m, k), dtype=np.float64)
        wc = np.zeros(m, dtype=np.int64) if work else None
        wb = np.zeros(m, dtype=np.int64) if work else None
        _check(getattr(_load(), fn)(self._h, src, m, k, _p(ids), _p(d2), _p(wc), _p(wb)))
        return (ids, d2, wc, wb) if work else (ids, d2)

    def knn_all(self, k, qids=None, work=False):
        """Leaf-based rows (searchUp from each point's own leaf).  With
        work=True also the candidates scored and boxes tested per row."""
        return self._rows("zo_knn_rows_work", k, qids, work)

    def knn_root(self, k, qids=None, work=False):
        """Root-based rows (searchDown from the root)."""
        return self._rows("zo_knn_root_work", k, qids, work)

    def knn(self, queries, k, work=False):
        """Bit-based dynamic queries."""
        q = _soa(queries)
        return self._run("zo_knn_ext_work", _p(q), q.shape[1], k, work)

    def counters(self):
        v = [np.zeros(1, dtype=np.int64) for _ in range(3)]
        _load().zo_counters(self._h, *[_p(a) for a in v])
        return dict(candidates=int(v[0][0]), box_tests=int(v[1][0]), rows=int(v[2][0]))

    def insert(self, pts):
        q = _soa(pts)
        m = q.shape[1]
        out = np.empty(m, dtype=np.int32)
        _check(_load().zo_insert(self._h, _p(q), m, _p(out)))
        return out

    def delete(self, ids):
        a = np.ascontiguousarray(ids, dtype=np.int32)
        _check(_load().zo_delete(self._h, _p(a), a.shape[0]))

    def export(self):
        """In-order canonical form: dict of numpy arrays."""
        inf = self.info()
        n, nl, ni, d = inf["n_live"], inf["n_leaves"], inf["n_internal"], self.dim
        out = dict(keys=np.zeros(n, dtype=np.uint64), ids=np.zeros(n, dtype=np.int32),
                   leaf_count=np.zeros(nl, dtype=np.int64),
                   leaf_lo=np.zeros((nl, d)), leaf_hi=np.zeros((nl, d)),
                   int_bit=np.zeros(ni, dtype=np.int32),
                   int_lo=np.zeros((ni, d)), int_hi=np.zeros((ni, d)))
        _load().zo_export(self._h, *[_p(out[x]) for x in
                                     ("keys", "ids", "leaf_count", "leaf_lo", "leaf_hi",
                                      "int_bit", "int_lo", "int_hi")])
        out.update(inf)
        return out
