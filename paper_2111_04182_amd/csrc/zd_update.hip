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

#include <algorithm>

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

namespace zd {

// ------------------------------------------------------- small batches --
//
// A small batch is applied in place, as Algorithm 4 does it: each inserted
// point descends by its key bits to the leaf whose cell holds it and is
// appended there, and the boxes on its path are expanded; a deleted point
// is removed from its leaf.  With the points stored contiguously in Morton
// order, "appended" means written to the leaf's block of a side pool
// (kOvfBlock entries), and "removed" means its x coordinate becomes NaN:
// a NaN distance never enters a candidate set.  Boxes only ever grow here,
// so they stay supersets of their points, and every point stays inside the
// key cell of each node above it, which is what the pruning and the
// stopping rule of Algorithms 2 and 3 rely on: the rows stay exact.  What
// this defers is only the canonical shape (leaves past L points, Patricia
// edge splits, tight boxes, spliced nodes); the library restores it, with
// a rebuild from the live points, when the side pool or the deleted
// points pass their bounds, and before the tree is exported.

// Descend by key bits to the leaf (Algorithm 4's descent), recording the
// path: path[j * kMaxPath + d] = (node << 1) | side taken at depth d.  The
// pruned tree skips bits where all of a node's points agree, so the key
// must also agree with them there, or Algorithm 4 would split that edge:
// it suffices to compare the key with one point of the leaf above the
// split bit of the leaf's parent (every point of an ancestor shares that
// leaf point's bits above the ancestor's higher split bit).
__device__ __forceinline__ bool ins_locate_one(const INode *__restrict__ inode,
                                               const uint64_t *__restrict__ tkey,
                                               const int32_t *__restrict__ leaf_begin,
                                               int32_t root, uint64_t key, int64_t j,
                                               int32_t *__restrict__ leaf_out,
                                               int32_t *__restrict__ path,
                                               int32_t *__restrict__ depth_out) {
  int32_t x = root;
  bool ok = x != kNoRoot;
  int d = 0, last_bit = 64;
  for (; ok && x >= 0; ++d) {
    if (d == kMaxPath) {
      ok = false;
      break;
    }
    const int bit = inode[x].bit;
    const int side = (int)((key >> bit) & 1);
    path[j * kMaxPath + d] = (x << 1) | side;
    last_bit = bit;
    x = inode[x].child[side];
  }
  if (ok && last_bit < 63 && ((key ^ tkey[leaf_begin[~x]]) >> (last_bit + 1)) != 0) ok = false;
  leaf_out[j] = ok ? ~x : -1;
  depth_out[j] = ok ? d : 0;
  return ok;
}

__global__ void k_ins_locate(const INode *__restrict__ inode, const uint64_t *__restrict__ tkey,
                             const int32_t *__restrict__ leaf_begin, const int32_t *meta,
                             const uint64_t *__restrict__ bk, int64_t m,
                             int32_t *__restrict__ leaf_out, int32_t *__restrict__ path,
                             int32_t *__restrict__ depth_out, int32_t *local_fail) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  if (!ins_locate_one(inode, tkey, leaf_begin, meta[kMetaRoot], bk[j], j, leaf_out, path,
                      depth_out))
    atomicAdd(local_fail, 1);
}

// One thread per run of batch points bound for one leaf (the batch is
// sorted by key, and leaves hold consecutive key ranges): the run must fit
// in the leaf's block; count the leaves that need a new block.
__device__ __forceinline__ void ins_run_check(const int32_t *leaf, int64_t m, int64_t j,
                                              const int32_t *__restrict__ ovf_blk,
                                              const int32_t *__restrict__ ovf_cnt,
                                              int32_t *local_fail, int32_t *blocks_needed) {
  const int32_t l = leaf[j];
  if (l < 0 || (j > 0 && leaf[j - 1] == l)) return;
  int64_t r = 1;
  while (j + r < m && leaf[j + r] == l) ++r;
  if (ovf_cnt[l] + r > kOvfBlock) atomicAdd(local_fail, 1);
  if (ovf_blk[l] < 0) atomicAdd(blocks_needed, 1);
}

__global__ void k_ins_runs(const int32_t *__restrict__ leaf, int64_t m,
                           const int32_t *__restrict__ ovf_blk, const int32_t *__restrict__ ovf_cnt,
                           int32_t *local_fail, int32_t *blocks_needed) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  ins_run_check(leaf, m, j, ovf_blk, ovf_cnt, local_fail, blocks_needed);
}

// A batch of at most kSmallSortKeys points in one workgroup and one launch:
// the declared-box check, keys (ids id_base, id_base + 1, ...), the sort by
// (key, id) in LDS (a bitonic network), the descent of every point with its
// path, and the per-leaf room check.  The three counts go to
// meta[kMetaCheck], meta[kMetaLocal] and meta[kMetaBlocks].
template <int D>
__global__ void __launch_bounds__(1024)
    k_ins_prepare(Geometry g, Box3 box, const double *__restrict__ xyz, int m, int np2,
                  int32_t id_base, const INode *__restrict__ inode,
                  const uint64_t *__restrict__ tkey, const int32_t *__restrict__ leaf_begin,
                  int32_t *meta, const int32_t *__restrict__ ovf_blk,
                  const int32_t *__restrict__ ovf_cnt, uint64_t *__restrict__ bk,
                  int32_t *__restrict__ bi, int32_t *__restrict__ leaf,
                  int32_t *__restrict__ path, int32_t *__restrict__ depth) {
  __shared__ uint64_t sk[kSmallSortKeys];
  __shared__ int32_t sv[kSmallSortKeys];
  __shared__ int32_t sl[kSmallSortKeys];
  __shared__ int32_t cnt[3];  // outside the box, no room in place, new blocks
  const int t = threadIdx.x;
  if (t < 3) cnt[t] = 0;
  __syncthreads();
  for (int i = t; i < np2; i += blockDim.x) {
    if (i < m) {
      const double x = xyz[i], y = xyz[m + i], z = D == 3 ? xyz[2 * m + i] : 0.0;
      bool bad = !(x >= box.lo[0] && x <= box.hi[0]) || !(y >= box.lo[1] && y <= box.hi[1]);
      if (D == 3) bad = bad || !(z >= box.lo[2] && z <= box.hi[2]);
      if (bad) atomicAdd(&cnt[0], 1);
      sk[i] = morton_key<D>(g, x, y, z);
      sv[i] = id_base + i;
    } else {
      sk[i] = ~uint64_t(0);
      sv[i] = INT_MAX;
    }
  }
  __syncthreads();
  for (int size = 2; size <= np2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = t; i < np2 / 2; i += blockDim.x) {
        const int a = 2 * stride * (i / stride) + (i % stride);
        const int b = a + stride;
        const bool up = (a & size) == 0;
        const uint64_t ka = sk[a], kb = sk[b];
        const int32_t va = sv[a], vb = sv[b];
        const bool b_first = kb < ka || (kb == ka && vb < va);
        if (b_first == up) {
          sk[a] = kb;
          sk[b] = ka;
          sv[a] = vb;
          sv[b] = va;
        }
      }
      __syncthreads();
    }
  }
  const int32_t root = meta[kMetaRoot];
  for (int j = t; j < m; j += blockDim.x) {
    bk[j] = sk[j];
    bi[j] = sv[j];
    if (!ins_locate_one(inode, tkey, leaf_begin, root, sk[j], j, leaf, path, depth))
      atomicAdd(&cnt[1], 1);
    sl[j] = leaf[j];
  }
  __syncthreads();
  for (int j = t; j < m; j += blockDim.x) ins_run_check(sl, m, j, ovf_blk, ovf_cnt, &cnt[1], &cnt[2]);
  __syncthreads();
  if (t == 0) {
    meta[kMetaCheck] = cnt[0];
    meta[kMetaLocal] = cnt[1];
    meta[kMetaBlocks] = cnt[2];
  }
}

hipError_t insert_in_place_prepare(const Geometry &g, const double *lo, const double *hi,
                                   const double *xyz, int64_t m, int32_t id_base,
                                   const INode *inode, const uint64_t *tkey,
                                   const int32_t *leaf_begin, int32_t *meta,
                                   const int32_t *ovf_blk, const int32_t *ovf_cnt, uint64_t *bk,
                                   int32_t *bi, int32_t *leaf, int32_t *path, int32_t *depth,
                                   hipStream_t s) {
  if (m <= 0 || m > kSmallSortKeys) return hipErrorInvalidValue;
  int np2 = 2;
  while (np2 < m) np2 <<= 1;
  Box3 box{};
  for (int c = 0; c < g.dim; ++c) {
    box.lo[c] = lo[c];
    box.hi[c] = hi[c];
  }
  // a thread per point for the descents (up to 1,024), at least one per
  // compare-exchange pair of the network
  const int want = (int)std::max<int64_t>(m, np2 / 2);
  const int threads = want < 1024 ? (want + 63) / 64 * 64 : 1024;
  if (g.dim == 3)
    k_ins_prepare<3><<<1, threads, 0, s>>>(g, box, xyz, (int)m, np2, id_base, inode, tkey,
                                           leaf_begin, meta, ovf_blk, ovf_cnt, bk, bi, leaf,
                                           path, depth);
  else
    k_ins_prepare<2><<<1, threads, 0, s>>>(g, box, xyz, (int)m, np2, id_base, inode, tkey,
                                           leaf_begin, meta, ovf_blk, ovf_cnt, bk, bi, leaf,
                                           path, depth);
  return hipGetLastError();
}

// FP64 atomic min / max in L2 (global_atomic_min_f64 / max_f64 on gfx950;
// the result is unused, so the climb does not wait for them)
__device__ __forceinline__ void atomic_min_f64(double *a, double v) {
  __hip_atomic_fetch_min(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_max_f64(double *a, double v) {
  __hip_atomic_fetch_max(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One wavefront per batch point; the wavefronts of run starts place their
// run: lane 0 takes a block for the leaf if it has none and writes the
// points (coordinates from the caller's batch, read at id - id_base), ids
// and slot map; then lane d merges the run's box into the box at depth d
// of the recorded path (each parent stores its children's boxes; an atomic
// is issued only where the box grows), all levels at once, and lane 0 into
// the root box.
template <int D>
__global__ void __launch_bounds__(64)
    k_ins_commit(const int32_t *__restrict__ leaf, int64_t m, const int32_t *__restrict__ path,
                 const int32_t *__restrict__ depth, const int32_t *__restrict__ bi,
                 const double *__restrict__ bxyz, int64_t nb, int32_t id_base, int32_t *ovf_blk,
                 int32_t *ovf_cnt, int32_t *blocks_used, double *pxyz, int64_t pcap,
                 int32_t *pid, int32_t *slot_of, INode *inode, double *root_box,
                 int32_t *new_ids) {
  const int64_t j = blockIdx.x;
  const int lane = threadIdx.x;
  const int32_t l = leaf[j];
  if (j > 0 && leaf[j - 1] == l) return;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (lane == 0) {
    int32_t blk = ovf_blk[l];
    if (blk < 0) {
      blk = atomicAdd(blocks_used, 1);
      ovf_blk[l] = blk;
    }
    const int32_t c0 = ovf_cnt[l];
    int64_t r = 0;
    for (; j + r < m && leaf[j + r] == l; ++r) {
      const int64_t e = (int64_t)blk * kOvfBlock + c0 + r;
      const int32_t id = bi[j + r];
      const int64_t src = (int64_t)id - id_base;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const double v = bxyz[c * nb + src];
        pxyz[c * pcap + e] = v;
        lo[c] = fmin(lo[c], v);
        hi[c] = fmax(hi[c], v);
      }
      pid[e] = id;
      slot_of[id] = kPoolSlot + (int32_t)e;
      if (new_ids) new_ids[src] = id;
    }
    ovf_cnt[l] = c0 + (int32_t)r;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      atomic_min_f64(&root_box[c], lo[c]);
      atomic_max_f64(&root_box[3 + c], hi[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < D; ++c) {
    lo[c] = __shfl(lo[c], 0, 64);
    hi[c] = __shfl(hi[c], 0, 64);
  }
  if (lane < depth[j]) {
    const int32_t link = path[j * kMaxPath + lane];
    INode *P = &inode[link >> 1];
    const int side = link & 1;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      if (lo[c] < P->lo[side][c]) atomic_min_f64(&P->lo[side][c], lo[c]);
      if (hi[c] > P->hi[side][c]) atomic_max_f64(&P->hi[side][c], hi[c]);
    }
  }
}

hipError_t insert_in_place_locate(const INode *inode, const uint64_t *tkey,
                                  const int32_t *leaf_begin, const int32_t *meta,
                                  const uint64_t *bk, int64_t m, const int32_t *ovf_blk,
                                  const int32_t *ovf_cnt, int32_t *leaf, int32_t *path,
                                  int32_t *depth, int32_t *local_fail, int32_t *blocks_needed,
                                  hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((m + 255) / 256);
  k_ins_locate<<<grid, 256, 0, s>>>(inode, tkey, leaf_begin, meta, bk, m, leaf, path, depth,
                                    local_fail);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_ins_runs<<<grid, 256, 0, s>>>(leaf, m, ovf_blk, ovf_cnt, local_fail, blocks_needed);
  return hipGetLastError();
}

hipError_t insert_in_place_commit(int dim, const int32_t *leaf, int64_t m, const int32_t *path,
                                  const int32_t *depth, const int32_t *bi, const double *bxyz,
                                  int32_t id_base, int32_t *ovf_blk, int32_t *ovf_cnt,
                                  int32_t *blocks_used, double *pxyz, int64_t pcap, int32_t *pid,
                                  int32_t *slot_of, INode *inode, double *root_box,
                                  int32_t *new_ids, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  static_assert(kMaxPath <= 64, "one lane per path level");
  const unsigned grid = (unsigned)m;
  if (dim == 3)
    k_ins_commit<3><<<grid, 64, 0, s>>>(leaf, m, path, depth, bi, bxyz, m, id_base, ovf_blk,
                                        ovf_cnt, blocks_used, pxyz, pcap, pid, slot_of, inode,
                                        root_box, new_ids);
  else
    k_ins_commit<2><<<grid, 64, 0, s>>>(leaf, m, path, depth, bi, bxyz, m, id_base, ovf_blk,
                                        ovf_cnt, blocks_used, pxyz, pcap, pid, slot_of, inode,
                                        root_box, new_ids);
  return hipGetLastError();
}

// Small deletes: the point keeps its slot (sorted position or pool entry)
// with a NaN x; its id becomes dead.
__global__ void k_tombstone(const int32_t *__restrict__ ids, int64_t m, int32_t *slot_of,
                            int32_t *mark, double *X, double *pX) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int32_t id = ids[j];
  const int32_t sl = slot_of[id];
  if (sl >= kPoolSlot) pX[sl - kPoolSlot] = NAN;
  else X[sl] = NAN;
  slot_of[id] = -1;
  mark[id] = 0;
}

hipError_t tombstone_ids(const int32_t *ids, int64_t m, int32_t *slot_of, int32_t *mark,
                         double *X, double *pX, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  k_tombstone<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(ids, m, slot_of, mark, X, pX);
  return hipGetLastError();
}

// Live flags of the sorted slots and the pool entries (x not NaN).
__global__ void k_live_flags(const double *__restrict__ X, int64_t n, const double *__restrict__ pX,
                             int64_t np, int32_t *__restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n + np) return;
  const double x = i < n ? X[i] : pX[i - n];
  flag[i] = isnan(x) ? 0 : 1;
}



}  // namespace zd

namespace zd {

// ------------------------------------------------------ folding a pool --
//
// The canonical shape back after small batches, in streaming passes: the
// live sorted points compact in place of order (their keys stay sorted),
// the live pool points and a new batch are keyed and sorted by (key, id),
// and the two sorted lists merge as in an insert.

// live sorted points to their compacted positions (pos from count_live)
template <int D>
__global__ void k_fold_main(const int32_t *__restrict__ pos, int64_t n,
                            const uint64_t *__restrict__ key, const int32_t *__restrict__ id,
                            const double *__restrict__ X, const double *__restrict__ Y,
                            const double *__restrict__ Z, uint64_t *__restrict__ key2,
                            int32_t *__restrict__ id2, double *__restrict__ X2,
                            double *__restrict__ Y2, double *__restrict__ Z2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || isnan(X[i])) return;
  const int32_t p = pos[i];
  key2[p] = key[i];
  id2[p] = id[i];
  X2[p] = X[i];
  Y2[p] = Y[i];
  if (D == 3) Z2[p] = Z[i];
}

// live pool entries (at pos - na) and the batch (after them): their
// coordinates, for the keys, and their ids
template <int D>
__global__ void k_fold_extra(const int32_t *__restrict__ pos, int64_t n, int64_t np, int64_t na,
                             const double *__restrict__ pxyz, int64_t pcap,
                             const int32_t *__restrict__ pid, const double *__restrict__ bxyz,
                             int64_t nb, int32_t id_base, int64_t ne, double *__restrict__ out,
                             int32_t *__restrict__ out_id) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) {
    if (isnan(pxyz[i])) return;
    const int64_t p = pos[n + i] - na;
#pragma unroll
    for (int c = 0; c < D; ++c) out[c * ne + p] = pxyz[c * pcap + i];
    out_id[p] = pid[i];
  } else if (i < np + nb) {
    const int64_t b = i - np;
    const int64_t p = ne - nb + b;
#pragma unroll
    for (int c = 0; c < D; ++c) out[c * ne + p] = bxyz[c * nb + b];
    out_id[p] = id_base + (int32_t)b;
  }
}

// coordinates of the merged order: from the compacted sorted points, or
// for an extra point from the batch (id >= id_base) or its pool entry
// (found through the slot map before this thread overwrites it)
template <int D>
__global__ void k_fold_gather(const int32_t *__restrict__ src, int64_t n2, int64_t na,
                              const double *__restrict__ X, const double *__restrict__ Y,
                              const double *__restrict__ Z, const double *__restrict__ pxyz,
                              int64_t pcap, const double *__restrict__ bxyz, int64_t nb,
                              int32_t id_base, const int32_t *__restrict__ iout,
                              double *__restrict__ X2, double *__restrict__ Y2,
                              double *__restrict__ Z2, int32_t *__restrict__ slot_of) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n2) return;
  const int64_t sidx = src[p];
  const int32_t v = iout[p];
  if (sidx < na) {
    X2[p] = X[sidx];
    Y2[p] = Y[sidx];
    if (D == 3) Z2[p] = Z[sidx];
  } else if (nb > 0 && v >= id_base) {
    const int64_t b = (int64_t)v - id_base;
    X2[p] = bxyz[b];
    Y2[p] = bxyz[nb + b];
    if (D == 3) Z2[p] = bxyz[2 * nb + b];
  } else {
    const int64_t e = (int64_t)slot_of[v] - kPoolSlot;
    X2[p] = pxyz[e];
    Y2[p] = pxyz[pcap + e];
    if (D == 3) Z2[p] = pxyz[2 * pcap + e];
  }
  slot_of[v] = (int32_t)p;
}

hipError_t count_live(const double *X, int64_t n, const double *pX, int64_t np,
                      int32_t *scan_scratch, int32_t *nlive_dev, hipStream_t s) {
  if (n + np <= 0) return fill_i32(nlive_dev, 0, 1, s);
  k_live_flags<<<(unsigned)((n + np + 255) / 256), 256, 0, s>>>(X, n, pX, np, scan_scratch);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = exclusive_scan_i32(scan_scratch, scan_scratch, n + np, nlive_dev, s);
  return e;
}

__global__ void k_id_as_key(const int32_t *__restrict__ id, int64_t n, uint64_t *__restrict__ k) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) k[i] = (uint64_t)(uint32_t)id[i];
}

__global__ void k_permute_pairs(const int32_t *__restrict__ order, int64_t n,
                                const uint64_t *__restrict__ key, const int32_t *__restrict__ id,
                                uint64_t *__restrict__ key2, int32_t *__restrict__ id2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key2[i] = key[order[i]];
  id2[i] = id[order[i]];
}

// (key, id) pairs, ids distinct, into (key, id) order: by id first, then a
// stable sort by key (one workgroup when they are few)
hipError_t sort_key_id(uint64_t *key, int32_t *id, int64_t n, int key_bits, uint64_t *ktmp,
                       int32_t *itmp, uint64_t *k2, int32_t *i2, hipStream_t s) {
  if (n <= 1) return hipSuccess;
  if (n <= kSmallSortKeys) return sort_pairs_small(key, id, n, s);
  // ids as keys (31 bits), the positions as values
  hipError_t e = hipMemcpyAsync(itmp, id, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = iota_i32(i2, 0, n, s);
  if (e != hipSuccess) return e;
  k_id_as_key<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(itmp, n, k2);
  e = hipGetLastError();
  if (e == hipSuccess) e = radix_sort_pairs(k2, i2, ktmp, itmp, n, 32, s);
  if (e != hipSuccess) return e;
  k_permute_pairs<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(i2, n, key, id, k2, itmp);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(key, k2, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(id, itmp, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = radix_sort_pairs(key, id, ktmp, itmp, n, key_bits, s);
  return e;
}

hipError_t fold_main(int dim, const int32_t *pos, int64_t n, const uint64_t *key,
                     const int32_t *id, const double *X, const double *Y, const double *Z,
                     uint64_t *key2, int32_t *id2, double *X2, double *Y2, double *Z2,
                     hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (dim == 3)
    k_fold_main<3><<<grid, 256, 0, s>>>(pos, n, key, id, X, Y, Z, key2, id2, X2, Y2, Z2);
  else
    k_fold_main<2><<<grid, 256, 0, s>>>(pos, n, key, id, X, Y, Z, key2, id2, X2, Y2, Z2);
  return hipGetLastError();
}

hipError_t fold_extra(int dim, const int32_t *pos, int64_t n, int64_t np, int64_t na,
                      const double *pxyz, int64_t pcap, const int32_t *pid, const double *bxyz,
                      int64_t nb, int32_t id_base, int64_t ne, double *out, int32_t *out_id,
                      hipStream_t s) {
  if (np + nb <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((np + nb + 255) / 256);
  if (dim == 3)
    k_fold_extra<3><<<grid, 256, 0, s>>>(pos, n, np, na, pxyz, pcap, pid, bxyz, nb, id_base, ne,
                                         out, out_id);
  else
    k_fold_extra<2><<<grid, 256, 0, s>>>(pos, n, np, na, pxyz, pcap, pid, bxyz, nb, id_base, ne,
                                         out, out_id);
  return hipGetLastError();
}

hipError_t fold_gather(int dim, const int32_t *src, int64_t n2, int64_t na, const double *X,
                       const double *Y, const double *Z, const double *pxyz, int64_t pcap,
                       const double *bxyz, int64_t nb, int32_t id_base, const int32_t *iout,
                       double *X2, double *Y2, double *Z2, int32_t *slot_of, hipStream_t s) {
  if (n2 <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n2 + 255) / 256);
  if (dim == 3)
    k_fold_gather<3><<<grid, 256, 0, s>>>(src, n2, na, X, Y, Z, pxyz, pcap, bxyz, nb, id_base,
                                          iout, X2, Y2, Z2, slot_of);
  else
    k_fold_gather<2><<<grid, 256, 0, s>>>(src, n2, na, X, Y, Z, pxyz, pcap, bxyz, nb, id_base,
                                          iout, X2, Y2, Z2, slot_of);
  return hipGetLastError();
}

}  // namespace zd
