"""ctypes binding of libzd (include/zd.h): argument marshalling only.

Every step of the k-NN path runs in the library's HIP kernels; PyTorch only
provides device memory (tensors) and the current HIP stream.  torch is
imported before the library is loaded so that both share one HIP runtime.
There is no fallback: if libzd.so is missing or fails to load, every call
raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libzd.so")

ZD_OK, ZD_EINVAL, ZD_EBOUNDS, ZD_EID, ZD_ENOMEM, ZD_EDEVICE, ZD_EKMAX, ZD_ELIMIT = range(8)
ZD_KMAX = 100

EXPORTED = ("zd_build", "zd_knn", "zd_knn_root", "zd_knn_noalloc", "zd_insert_batch", "zd_delete_batch", "zd_free", "zd_info",
            "zd_check", "zd_pending", "zd_set_walk_limit", "zd_export", "zd_knn_backward", "zd_knn_backward_det", "zd_knn_backward_tree", "zd_forest_build", "zd_forest_knn", "zd_forest_plan",
            "zd_forest_plan_persistent",
            "zd_forest_run", "zd_forest_check", "zd_forest_free", "zd_status_str")


class ZdError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().zd_status_str(code).decode() if code >= 0 else "error"
        super().__init__(f"{where}: {msg} (status {code})")
        self.code = code


class _Params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("leaf_size", C.c_int32), ("shift_seed", C.c_uint64),
                ("shift", C.c_void_p), ("box_lo", C.c_void_p), ("box_hi", C.c_void_p),
                ("query_waves", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    """Load libzd.so (built by paper_2111_04182_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2111_04182_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.zd_status_str.restype = C.c_char_p
        L.zd_status_str.argtypes = [C.c_int]
        L.zd_build.restype = C.c_int
        L.zd_build.argtypes = [C.POINTER(_Params), vp, i64, vp, C.POINTER(vp)]
        L.zd_knn.restype = C.c_int
        L.zd_knn.argtypes = [vp, vp, i64, i32, vp, vp, vp]
        L.zd_knn_root.restype = C.c_int
        L.zd_knn_root.argtypes = [vp, vp, i64, i32, vp, vp, vp]
        L.zd_knn_noalloc.restype = C.c_int
        L.zd_knn_noalloc.argtypes = [vp, vp, i64, i32, vp, vp, vp]
        L.zd_insert_batch.restype = C.c_int
        L.zd_insert_batch.argtypes = [vp, vp, i64, vp, vp]
        L.zd_delete_batch.restype = C.c_int
        L.zd_delete_batch.argtypes = [vp, vp, i64, vp]
        L.zd_free.restype = C.c_int
        L.zd_free.argtypes = [vp]
        L.zd_info.restype = C.c_int
        L.zd_info.argtypes = [vp, vp, vp, vp, vp, vp]
        L.zd_pending.restype = C.c_int
        L.zd_pending.argtypes = [vp, vp, vp]
        L.zd_check.restype = C.c_int
        L.zd_check.argtypes = [vp]
        L.zd_set_walk_limit.restype = C.c_int
        L.zd_set_walk_limit.argtypes = [vp, i64]
        L.zd_export.restype = C.c_int
        L.zd_export.argtypes = [vp] * 11
        L.zd_knn_backward_det.restype = C.c_int
        L.zd_knn_backward_det.argtypes = [i32, vp, i64, i64, i32, vp, vp, vp, vp]
        L.zd_knn_backward_tree.restype = C.c_int
        L.zd_knn_backward_tree.argtypes = [vp, i32, vp, vp, vp, vp]
        L.zd_knn_backward.restype = C.c_int
        L.zd_knn_backward.argtypes = [i32, vp, i64, i64, i32, vp, vp, vp, vp]
        L.zd_forest_build.restype = C.c_int
        L.zd_forest_build.argtypes = [C.POINTER(_Params), vp, i64, vp, i32, vp, vp, C.POINTER(vp)]
        L.zd_forest_knn.restype = C.c_int
        L.zd_forest_knn.argtypes = [vp, i32, vp, vp, vp]
        L.zd_forest_plan.restype = C.c_int
        L.zd_forest_plan.argtypes = [C.POINTER(_Params), vp, i64, vp, i32, vp, i32, vp, vp, vp,
                                     C.POINTER(vp)]
        L.zd_forest_plan_persistent.restype = C.c_int
        L.zd_forest_plan_persistent.argtypes = L.zd_forest_plan.argtypes
        L.zd_forest_run.restype = C.c_int
        L.zd_forest_run.argtypes = [vp, vp]
        L.zd_forest_check.restype = C.c_int
        L.zd_forest_check.argtypes = [vp]
        L.zd_forest_free.restype = C.c_int
        L.zd_forest_free.argtypes = [vp]
        _lib = L
    return _lib


def _check(code: int, where: str):
    if code != ZD_OK:
        raise ZdError(code, where)


def _stream(stream=None) -> C.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dptr(t: torch.Tensor | None) -> C.c_void_p | None:
    return None if t is None else C.c_void_p(t.data_ptr())


def _hptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def soa(points: torch.Tensor) -> torch.Tensor:
    """(n, d) points -> contiguous float64 SoA (d, n) on the current device."""
    if points.dim() != 2 or points.shape[1] not in (2, 3):
        raise ValueError("points must have shape (n, 2) or (n, 3)")
    return points.to(device="cuda", dtype=torch.float64).t().contiguous()


def _check_soa(xyz: torch.Tensor, dim: int | None = None):
    if not (xyz.is_cuda and xyz.dtype == torch.float64 and xyz.dim() == 2 and xyz.is_contiguous()):
        raise ValueError("coordinates must be a contiguous float64 CUDA tensor of shape (d, n)")
    if xyz.shape[0] not in (2, 3) or (dim is not None and xyz.shape[0] != dim):
        raise ValueError("coordinates must have shape (d, n) with d = 2 or 3 (the tree's d)")


# --------------------------------------------------------------------------
# one Python function per C entry point
# --------------------------------------------------------------------------

def zd_build(xyz: torch.Tensor, leaf_size: int = 16, box=None, shift_seed: int = 0,
             shift=None, stream=None, query_waves: int = 0) -> C.c_void_p:
    """Build a tree over SoA points xyz (d, n); returns the handle."""
    _check_soa(xyz)
    dim, n = xyz.shape
    lo = hi = sh = None
    if box is not None:
        lo = np.ascontiguousarray(box[0], dtype=np.float64)
        hi = np.ascontiguousarray(box[1], dtype=np.float64)
        if lo.shape != (dim,) or hi.shape != (dim,):
            raise ValueError("box corners must have d entries")
    if shift is not None:
        sh = np.ascontiguousarray(shift, dtype=np.uint64)
        if sh.shape != (dim,):
            raise ValueError("shift must have d entries")
    p = _Params(dim, leaf_size, shift_seed & 0xFFFFFFFFFFFFFFFF, _hptr(sh), _hptr(lo), _hptr(hi),
                query_waves)
    out = C.c_void_p()
    _check(lib().zd_build(C.byref(p), _dptr(xyz), n, _stream(stream), C.byref(out)), "zd_build")
    return out


def _knn_args(q_xyz, m, k, out_ids, out_d2):
    if q_xyz is not None:
        _check_soa(q_xyz)
    for t, dt in ((out_ids, torch.int32), (out_d2, torch.float64)):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous() and t.numel() >= m * k):
            raise ValueError("outputs must be contiguous CUDA tensors of m*k entries")


def zd_knn(tree, q_xyz: torch.Tensor | None, m: int, k: int, out_ids: torch.Tensor,
           out_d2: torch.Tensor, stream=None):
    _knn_args(q_xyz, m, k, out_ids, out_d2)
    _check(lib().zd_knn(tree, _dptr(q_xyz), m, k, _dptr(out_ids), _dptr(out_d2),
                        _stream(stream)), "zd_knn")


def zd_knn_root(tree, q_xyz: torch.Tensor | None, m: int, k: int, out_ids: torch.Tensor,
                out_d2: torch.Tensor, stream=None):
    _knn_args(q_xyz, m, k, out_ids, out_d2)
    _check(lib().zd_knn_root(tree, _dptr(q_xyz), m, k, _dptr(out_ids), _dptr(out_d2),
                             _stream(stream)), "zd_knn_root")


def zd_insert_batch(tree, xyz: torch.Tensor, out_new_ids: torch.Tensor | None = None,
                    stream=None):
    _check_soa(xyz)
    m = xyz.shape[1]
    _check(lib().zd_insert_batch(tree, _dptr(xyz), m, _dptr(out_new_ids), _stream(stream)),
           "zd_insert_batch")


def zd_delete_batch(tree, ids: torch.Tensor, stream=None):
    if not (ids.is_cuda and ids.dtype == torch.int32 and ids.is_contiguous() and ids.dim() == 1):
        raise ValueError("ids must be a contiguous 1-D int32 CUDA tensor")
    _check(lib().zd_delete_batch(tree, _dptr(ids), ids.numel(), _stream(stream)),
           "zd_delete_batch")


def zd_free(tree):
    if tree:
        _check(lib().zd_free(tree), "zd_free")


def zd_info(tree, depth: bool = False) -> dict:
    v = [C.c_int64() for _ in range(4)]
    d = C.c_int32()
    _check(lib().zd_info(tree, *[C.byref(x) for x in v], C.byref(d) if depth else None),
           "zd_info")
    out = dict(n_live=v[0].value, cap=v[1].value, n_leaves=v[2].value, n_internal=v[3].value)
    if depth:
        out["depth"] = d.value
    return out


def zd_pending(tree) -> tuple:
    a, b = C.c_int64(), C.c_int64()
    _check(lib().zd_pending(tree, C.byref(a), C.byref(b)), "zd_pending")
    return a.value, b.value


def zd_check(tree):
    _check(lib().zd_check(tree), "zd_check")


def zd_set_walk_limit(tree, steps: int):
    _check(lib().zd_set_walk_limit(tree, steps), "zd_set_walk_limit")


def zd_export(tree, dim: int) -> dict:
    inf = zd_info(tree)
    n, nl, ni = inf["n_live"], inf["n_leaves"], inf["n_internal"]
    out = dict(keys=np.zeros(n, dtype=np.uint64), ids=np.zeros(n, dtype=np.int32),
               leaf_count=np.zeros(nl, dtype=np.int64), leaf_lo=np.zeros((nl, dim)),
               leaf_hi=np.zeros((nl, dim)), int_bit=np.zeros(ni, dtype=np.int32),
               int_lo=np.zeros((ni, dim)), int_hi=np.zeros((ni, dim)),
               params=np.zeros(3 * dim), shift=np.zeros(dim, dtype=np.uint64))
    _check(lib().zd_export(tree, *[_hptr(out[x]) for x in
                                   ("keys", "ids", "leaf_count", "leaf_lo", "leaf_hi", "int_bit",
                                    "int_lo", "int_hi", "params", "shift")]), "zd_export")
    out.update(inf)
    return out


def zd_knn_backward(xyz: torch.Tensor, ids: torch.Tensor, grad_d2: torch.Tensor,
                    grad_xyz: torch.Tensor | None = None, stream=None,
                    deterministic: bool = False) -> torch.Tensor:
    """Gradient of sum(grad_d2 * d2) w.r.t. SoA points xyz (d, n) for the fixed
    neighbour table ids [rows, k] (row r = point r).  deterministic=True
    sums in a fixed order without atomics (the same bits on every run)."""
    _check_soa(xyz)
    dim, n = xyz.shape
    rows, k = ids.shape
    if grad_xyz is None:
        grad_xyz = torch.empty_like(xyz)
    ids = ids.contiguous()
    grad_d2 = grad_d2.to(torch.float64).contiguous()
    fn = lib().zd_knn_backward_det if deterministic else lib().zd_knn_backward
    _check(fn(dim, _dptr(xyz), n, rows, k, _dptr(ids), _dptr(grad_d2), _dptr(grad_xyz),
              _stream(stream)), "zd_knn_backward")
    return grad_xyz


def zd_knn_backward_tree(tree, dim: int, cap: int, ids: torch.Tensor, grad_d2: torch.Tensor,
                         grad_xyz: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """zd_knn_backward for the tree's own all-points rows ids [cap, k], in the
    tree's Morton order (tree: a zd_tree handle, unchanged since the rows
    were computed; points pending in place take a second pass).  Returns
    the gradient as SoA (dim, cap)."""
    rows, k = ids.shape
    if rows != cap:
        raise ValueError("ids must hold one row per id of the tree")
    if grad_xyz is None:
        grad_xyz = torch.empty((dim, cap), dtype=torch.float64, device="cuda")
    ids = ids.contiguous()
    grad_d2 = grad_d2.to(torch.float64).contiguous()
    _check(lib().zd_knn_backward_tree(tree, k, _dptr(ids), _dptr(grad_d2), _dptr(grad_xyz),
                                      _stream(stream)), "zd_knn_backward_tree")
    return grad_xyz


# --------------------------------------------------------------------------
# convenience object
# --------------------------------------------------------------------------

class ZdTree:
    """A zd-tree on the current GPU (owns one libzd handle)."""

    def __init__(self, xyz: torch.Tensor, leaf_size: int = 16, box=None, shift_seed: int = 0,
                 shift=None, stream=None, query_waves: int = 0):
        self.dim = xyz.shape[0]
        self.leaf_size = leaf_size
        self._h = zd_build(xyz, leaf_size, box, shift_seed, shift, stream, query_waves)
        self.cap = xyz.shape[1]  # id capacity, tracked here to avoid a sync
        self.version = 0  # counts the updates (a backward checks its rows are current)

    @property
    def handle(self):
        return self._h

    def info(self, depth: bool = False) -> dict:
        return zd_info(self._h, depth)

    def check(self):
        zd_check(self._h)

    def pending(self) -> tuple:
        """(points placed in place by small inserts, deleted points holding
        their slot) since the last rebuild."""
        return zd_pending(self._h)

    def knn(self, k: int, queries: torch.Tensor | None = None, stream=None, root=False):
        """All-points rows (queries None, one row per id) or external queries
        (SoA (d, m)); root=True runs the root-based search instead.  Returns
        (ids int32 [rows, k], d2 float64 [rows, k])."""
        m = self.cap if queries is None else queries.shape[1]
        ids = torch.empty((m, k), dtype=torch.int32, device="cuda")
        d2 = torch.empty((m, k), dtype=torch.float64, device="cuda")
        (zd_knn_root if root else zd_knn)(self._h, queries, m, k, ids, d2, stream)
        return ids, d2

    def insert(self, xyz: torch.Tensor, stream=None) -> torch.Tensor:
        out = torch.empty(xyz.shape[1], dtype=torch.int32, device="cuda")
        zd_insert_batch(self._h, xyz, out, stream)
        self.cap += xyz.shape[1]
        self.version += 1
        return out

    def delete(self, ids: torch.Tensor, stream=None):
        zd_delete_batch(self._h, ids.to(device="cuda", dtype=torch.int32).contiguous(), stream)
        self.version += 1

    def knn_backward(self, ids: torch.Tensor, grad_d2: torch.Tensor, stream=None) -> torch.Tensor:
        """Gradient of sum(grad_d2 * d2) over this tree's all-points rows ids
        (unchanged since knn), w.r.t. its points by id, in its Morton order."""
        return zd_knn_backward_tree(self._h, self.dim, self.cap, ids, grad_d2, None, stream)

    def export(self) -> dict:
        return zd_export(self._h, self.dim)

    def close(self):
        if getattr(self, "_h", None):
            zd_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# batched forest
# --------------------------------------------------------------------------

def _forest_args(xyz, offsets, leaf_size, leaf_sizes, box, shift_seed, shift, query_waves):
    _check_soa(xyz)
    dim, n = xyz.shape
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    ls = None if leaf_sizes is None else np.ascontiguousarray(leaf_sizes, dtype=np.int32)
    lo = hi = sh = None
    if box is not None:
        lo = np.ascontiguousarray(box[0], dtype=np.float64)
        hi = np.ascontiguousarray(box[1], dtype=np.float64)
    if shift is not None:
        sh = np.ascontiguousarray(shift, dtype=np.uint64)
    p = _Params(dim, leaf_size, shift_seed & 0xFFFFFFFFFFFFFFFF, _hptr(sh), _hptr(lo), _hptr(hi),
                query_waves)
    return p, dim, n, off, ls, (lo, hi, sh)


def zd_forest_build(xyz, offsets, leaf_size=16, leaf_sizes=None, box=None, shift_seed=0,
                    shift=None, stream=None, query_waves=0):
    p, dim, n, off, ls, keep = _forest_args(xyz, offsets, leaf_size, leaf_sizes, box,
                                            shift_seed, shift, query_waves)
    out = C.c_void_p()
    _check(lib().zd_forest_build(C.byref(p), _dptr(xyz), n, _hptr(off), len(off) - 1, _hptr(ls),
                                 _stream(stream), C.byref(out)), "zd_forest_build")
    return out


def zd_forest_knn(forest, k, out_ids, out_d2, stream=None):
    _check(lib().zd_forest_knn(forest, k, _dptr(out_ids), _dptr(out_d2), _stream(stream)),
           "zd_forest_knn")


def zd_forest_plan(xyz, offsets, k, out_ids, out_d2, leaf_size=16, leaf_sizes=None, box=None,
                   shift_seed=0, shift=None, stream=None, query_waves=0):
    p, dim, n, off, ls, keep = _forest_args(xyz, offsets, leaf_size, leaf_sizes, box,
                                            shift_seed, shift, query_waves)
    out = C.c_void_p()
    _check(lib().zd_forest_plan(C.byref(p), _dptr(xyz), n, _hptr(off), len(off) - 1, _hptr(ls),
                                k, _dptr(out_ids), _dptr(out_d2), _stream(stream), C.byref(out)),
           "zd_forest_plan")
    return out


def zd_forest_plan_persistent(xyz, offsets, k, out_ids, out_d2, leaf_size=16, leaf_sizes=None,
                              box=None, shift_seed=0, shift=None, stream=None):
    p, dim, n, off, ls, keep = _forest_args(xyz, offsets, leaf_size, leaf_sizes, box,
                                            shift_seed, shift, 0)
    out = C.c_void_p()
    _check(lib().zd_forest_plan_persistent(C.byref(p), _dptr(xyz), n, _hptr(off), len(off) - 1,
                                           _hptr(ls), k, _dptr(out_ids), _dptr(out_d2),
                                           _stream(stream), C.byref(out)),
           "zd_forest_plan_persistent")
    return out


def zd_forest_run(forest, stream=None):
    _check(lib().zd_forest_run(forest, _stream(stream)), "zd_forest_run")


def zd_forest_check(forest):
    _check(lib().zd_forest_check(forest), "zd_forest_check")


def zd_forest_free(forest):
    if forest:
        _check(lib().zd_forest_free(forest), "zd_forest_free")


class ZdForest:
    """Many independent clouds in one device structure (cloud c = points
    offsets[c]..offsets[c+1] of the SoA tensor xyz)."""

    def __init__(self, xyz, offsets, leaf_size=16, leaf_sizes=None, box=None, shift_seed=0,
                 shift=None, stream=None, query_waves=0):
        self.n = xyz.shape[1]
        self._xyz = xyz
        self._h = zd_forest_build(xyz, offsets, leaf_size, leaf_sizes, box, shift_seed, shift,
                                  stream, query_waves)

    def knn(self, k, stream=None):
        ids = torch.empty((self.n, k), dtype=torch.int32, device="cuda")
        d2 = torch.empty((self.n, k), dtype=torch.float64, device="cuda")
        zd_forest_knn(self._h, k, ids, d2, stream)
        return ids, d2

    def check(self):
        zd_forest_check(self._h)

    def close(self):
        if getattr(self, "_h", None):
            zd_forest_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ZdForestPlan:
    """Build + all-points query of a forest captured as one HIP graph; run()
    replays it on the current contents of xyz, filling self.ids / self.d2.
    persistent=True captures the single persistent launch
    (zd_forest_plan_persistent) instead of the pass-by-pass sequence."""

    def __init__(self, xyz, offsets, k, leaf_size=16, leaf_sizes=None, box=None, shift_seed=0,
                 shift=None, stream=None, query_waves=0, persistent=False):
        n = xyz.shape[1]
        self._xyz = xyz
        self.ids = torch.empty((n, k), dtype=torch.int32, device="cuda")
        self.d2 = torch.empty((n, k), dtype=torch.float64, device="cuda")
        if persistent:
            self._h = zd_forest_plan_persistent(xyz, offsets, k, self.ids, self.d2, leaf_size,
                                                leaf_sizes, box, shift_seed, shift, stream)
        else:
            self._h = zd_forest_plan(xyz, offsets, k, self.ids, self.d2, leaf_size, leaf_sizes,
                                     box, shift_seed, shift, stream, query_waves)

    def run(self, stream=None):
        zd_forest_run(self._h, stream)
        return self.ids, self.d2

    def check(self):
        zd_forest_check(self._h)

    def close(self):
        if getattr(self, "_h", None):
            zd_forest_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
