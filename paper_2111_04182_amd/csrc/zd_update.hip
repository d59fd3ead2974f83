// zd_update.hip -- kernels behind batch insertion and deletion.
//
// Algorithm 4 inserts a Morton-sorted batch by descending the tree, appending
// to leaves with room and splitting leaves that overflow; deletion is the
// mirror image (Section 2, "Batch-dynamic updates").  Done as the paper
// states, the tree after an update equals a fresh build of the live points
// (inserted points join the leaves their keys select, overflowing leaves are
// rebuilt with Algorithm 1, emptied nodes disappear).  Here the points live
// contiguously in Morton order, so an update is a streaming pass: merge the
// sorted batch into the sorted point array (insert) or compact the survivors
// (delete), then relink the tree with the bottom-up pass of zd_build.hip.
// Every step is a coalesced O(n + m) sweep at HBM bandwidth.
#include "zd_internal.h"

namespace zd {

// --------------------------------------------------------- bounds / boxes --

template <int D>
__global__ void k_count_outside(const double *__restrict__ xyz, int64_t m, Box3 box,
                                int32_t *counter) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  if (i < m) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double v = xyz[c * m + i];
      if (!(v >= box.lo[c] && v <= box.hi[c])) bad = true;
    }
  }
  uint64_t b = __ballot(bad);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(counter, (int32_t)__popcll(b));
}

hipError_t count_outside_box(int dim, const double *xyz, int64_t m, const double *lo,
                             const double *hi, int32_t *counter, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  Box3 box{};
  for (int c = 0; c < dim; ++c) {
    box.lo[c] = lo[c];
    box.hi[c] = hi[c];
  }
  unsigned grid = (unsigned)((m + 255) / 256);
  if (dim == 3) k_count_outside<3><<<grid, 256, 0, s>>>(xyz, m, box, counter);
  else k_count_outside<2><<<grid, 256, 0, s>>>(xyz, m, box, counter);
  return hipGetLastError();
}

// per-block min/max of each coordinate -> partial[blk][6]
__global__ void k_box_partial(const double *__restrict__ xyz, int64_t n, int dim,
                              double *__restrict__ partial) {
  __shared__ double red[6][256];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    for (int c = 0; c < dim; ++c) {
      double v = xyz[c * n + i];
      lo[c] = fmin(lo[c], v);
      hi[c] = fmax(hi[c], v);
    }
  }
  for (int c = 0; c < 3; ++c) {
    red[c][threadIdx.x] = lo[c];
    red[3 + c][threadIdx.x] = hi[c];
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 3; ++c) {
        red[c][threadIdx.x] = fmin(red[c][threadIdx.x], red[c][threadIdx.x + w]);
        red[3 + c][threadIdx.x] = fmax(red[3 + c][threadIdx.x], red[3 + c][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) partial[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_box_final(const double *__restrict__ partial, int nblk, double *out) {
  if (threadIdx.x >= 6) return;
  const int c = threadIdx.x;
  double v = c < 3 ? INFINITY : -INFINITY;
  for (int b = 0; b < nblk; ++b) {
    double x = partial[b * 6 + c];
    v = c < 3 ? fmin(v, x) : fmax(v, x);
  }
  out[c] = v;
}

hipError_t box_reduce(int dim, const double *xyz, int64_t n, double *out_lo_hi, hipStream_t s) {
  const int nblk = 512;
  double *partial = nullptr;
  hipError_t e = dev_alloc_n(&partial, (int64_t)nblk * 6, s);
  if (e != hipSuccess) return e;
  k_box_partial<<<nblk, 256, 0, s>>>(xyz, n, dim, partial);
  e = hipGetLastError();
  if (e == hipSuccess) {
    k_box_final<<<1, 64, 0, s>>>(partial, nblk, out_lo_hi);
    e = hipGetLastError();
  }
  dev_release(partial, s);
  return e;
}

// ------------------------------------------------------------------ merge --

// number of entries of the sorted (key, id) list a[0..na) that precede (k, i)
__device__ __forceinline__ int64_t rank_in(const uint64_t *ka, const int32_t *ia, int64_t na,
                                           uint64_t k, int32_t i) {
  int64_t lo = 0, hi = na;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    uint64_t km = ka[mid];
    bool before = km < k || (km == k && ia[mid] < i);
    if (before) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ void k_mark_b(const uint64_t *__restrict__ ka, const int32_t *__restrict__ ia,
                         int64_t na, const uint64_t *__restrict__ kb,
                         const int32_t *__restrict__ ib, int64_t nb, int32_t *__restrict__ isb) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nb) return;
  isb[j + rank_in(ka, ia, na, kb[j], ib[j])] = 1;
}

__global__ void k_merge_gather(const uint64_t *__restrict__ ka, const int32_t *__restrict__ ia,
                               int64_t na, const uint64_t *__restrict__ kb,
                               const int32_t *__restrict__ ib, const int32_t *__restrict__ isb,
                               const int32_t *__restrict__ nbefore, int64_t ntot,
                               uint64_t *__restrict__ kout, int32_t *__restrict__ iout,
                               int32_t *__restrict__ src) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ntot) return;
  int32_t nb = nbefore[p];
  if (isb[p]) {
    kout[p] = kb[nb];
    iout[p] = ib[nb];
    src[p] = (int32_t)(na + nb);
  } else {
    int64_t i = p - nb;
    kout[p] = ka[i];
    iout[p] = ia[i];
    src[p] = (int32_t)i;
  }
}

hipError_t merge_sorted(const uint64_t *ka, const int32_t *ia, int64_t na, const uint64_t *kb,
                        const int32_t *ib, int64_t nb, int32_t *mark_scratch, uint64_t *kout,
                        int32_t *iout, int32_t *src, hipStream_t s) {
  const int64_t ntot = na + nb;
  if (ntot <= 0) return hipSuccess;
  // mark_scratch needs 2 * ntot entries: isb flags, then their exclusive scan
  int32_t *isb = mark_scratch, *nbefore = mark_scratch + ntot;
  hipError_t e = fill_i32(isb, 0, ntot, s);
  if (e != hipSuccess) return e;
  if (nb > 0) {
    k_mark_b<<<(unsigned)((nb + 255) / 256), 256, 0, s>>>(ka, ia, na, kb, ib, nb, isb);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = exclusive_scan_i32(isb, nbefore, ntot, nullptr, s);
  if (e == hipSuccess) {
    k_merge_gather<<<(unsigned)((ntot + 255) / 256), 256, 0, s>>>(ka, ia, na, kb, ib, isb,
                                                                  nbefore, ntot, kout, iout, src);
    e = hipGetLastError();
  }
  return e;
}

// Coordinates of the merged order.  A point from the tree is read at its old
// sorted position; a batch point at its input position, which is its id
// minus the first new id (the batch was sorted, its ids were not).
template <int D>
__global__ void k_gather_merged(const int32_t *__restrict__ src, int64_t n,
                                const double *__restrict__ X, const double *__restrict__ Y,
                                const double *__restrict__ Z, int64_t na,
                                const double *__restrict__ bxyz, int64_t nb, int32_t id_base,
                                const int32_t *__restrict__ iout, double *__restrict__ X2,
                                double *__restrict__ Y2, double *__restrict__ Z2,
                                int32_t *__restrict__ slot_of) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int64_t sidx = src[p];
  if (sidx < na) {
    X2[p] = X[sidx];
    Y2[p] = Y[sidx];
    if (D == 3) Z2[p] = Z[sidx];
  } else {
    int64_t j = (int64_t)iout[p] - id_base;
    X2[p] = bxyz[j];
    Y2[p] = bxyz[nb + j];
    if (D == 3) Z2[p] = bxyz[2 * nb + j];
  }
  slot_of[iout[p]] = (int32_t)p;
}

hipError_t gather_merged(int dim, const int32_t *src, int64_t n, const double *X, const double *Y,
                         const double *Z, const double *bxyz, int64_t nb, int32_t id_base,
                         const int32_t *iout, double *X2, double *Y2, double *Z2,
                         int32_t *slot_of, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t na = n - nb;
  unsigned grid = (unsigned)((n + 255) / 256);
  if (dim == 3)
    k_gather_merged<3><<<grid, 256, 0, s>>>(src, n, X, Y, Z, na, bxyz, nb, id_base, iout, X2,
                                           Y2, Z2, slot_of);
  else
    k_gather_merged<2><<<grid, 256, 0, s>>>(src, n, X, Y, Z, na, bxyz, nb, id_base, iout, X2,
                                           Y2, Z2, slot_of);
  return hipGetLastError();
}

// ----------------------------------------------------------------- delete --

__global__ void k_validate_delete(const int32_t *__restrict__ ids, int64_t m, int64_t cap,
                                  const int32_t *__restrict__ slot_of, int32_t *mark,
                                  int32_t *err) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  if (j < m) {
    int32_t id = ids[j];
    if (id < 0 || id >= cap) bad = true;
    else if (slot_of[id] < 0) bad = true;
    else if (atomicExch(&mark[id], 1) != 0) bad = true;  // repeated in the batch
  }
  uint64_t b = __ballot(bad);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(err, (int32_t)__popcll(b));
}

hipError_t validate_delete(const int32_t *ids, int64_t m, int64_t cap, const int32_t *slot_of,
                           int32_t *mark, int32_t *err, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  k_validate_delete<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(ids, m, cap, slot_of, mark, err);
  return hipGetLastError();
}

__global__ void k_unmark(const int32_t *__restrict__ ids, int64_t m, int64_t cap, int32_t *mark) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  int32_t id = ids[j];
  if (id >= 0 && id < cap) mark[id] = 0;
}

hipError_t unmark_ids(const int32_t *ids, int64_t m, int64_t cap, int32_t *mark, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  k_unmark<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(ids, m, cap, mark);
  return hipGetLastError();
}

__global__ void k_kill(const int32_t *__restrict__ ids, int64_t m, int32_t *slot_of, int32_t *mark,
                       int32_t *dead_slot) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  int32_t id = ids[j];
  dead_slot[slot_of[id]] = 1;
  slot_of[id] = -1;
  mark[id] = 0;
}

hipError_t kill_ids(const int32_t *ids, int64_t m, int32_t *slot_of, int32_t *mark,
                    int32_t *dead_slot, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  k_kill<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(ids, m, slot_of, mark, dead_slot);
  return hipGetLastError();
}

__global__ void k_keep_flags(const int32_t *__restrict__ dead, int64_t n, int32_t *__restrict__ keep) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) keep[i] = dead[i] ? 0 : 1;
}

template <int D>
__global__ void k_compact_live(const int32_t *__restrict__ dead, const int32_t *__restrict__ pos,
                               int64_t n, const uint64_t *__restrict__ key,
                               const int32_t *__restrict__ id, const double *__restrict__ X,
                               const double *__restrict__ Y, const double *__restrict__ Z,
                               uint64_t *__restrict__ key2, int32_t *__restrict__ id2,
                               double *__restrict__ X2, double *__restrict__ Y2,
                               double *__restrict__ Z2, int32_t *__restrict__ slot_of) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || dead[i]) return;
  int32_t p = pos[i];
  key2[p] = key[i];
  id2[p] = id[i];
  X2[p] = X[i];
  Y2[p] = Y[i];
  if (D == 3) Z2[p] = Z[i];
  slot_of[id[i]] = p;
}

hipError_t compact_live(int dim, const int32_t *dead_slot, int64_t n, int32_t *scan_scratch,
                        const uint64_t *key, const int32_t *id, const double *X,
                        const double *Y, const double *Z, uint64_t *key2, int32_t *id2,
                        double *X2, double *Y2, double *Z2, int32_t *slot_of, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  unsigned grid = (unsigned)((n + 255) / 256);
  k_keep_flags<<<grid, 256, 0, s>>>(dead_slot, n, scan_scratch);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = exclusive_scan_i32(scan_scratch, scan_scratch, n, nullptr, s);
  if (e != hipSuccess) return e;
  if (dim == 3)
    k_compact_live<3><<<grid, 256, 0, s>>>(dead_slot, scan_scratch, n, key, id, X, Y, Z, key2,
                                          id2, X2, Y2, Z2, slot_of);
  else
    k_compact_live<2><<<grid, 256, 0, s>>>(dead_slot, scan_scratch, n, key, id, X, Y, Z, key2,
                                          id2, X2, Y2, Z2, slot_of);
  return hipGetLastError();
}

}  // namespace zd
