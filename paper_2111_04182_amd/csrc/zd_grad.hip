// zd_grad.hip -- backward of the k-NN squared distances.
//
// For a fixed neighbour table the loss L = sum_{r,j} g[r][j] * d2(p_r, p_q),
// q = ids[r][j], is quadratic in the coordinates:
//   dL/dp_r += 2 (p_r - p_q) g,   dL/dp_q -= 2 (p_r - p_q) g.
// One thread per row forms each term once: the row's own terms are summed in
// registers and added to its gradient once, the neighbours' terms are
// scatter-added with hardware FP64 atomics (a neighbour can be in many
// rows).  Neighbour selection is untouched.
#include "zd_internal.h"

namespace zd {

template <int D>
__global__ void k_knn_backward(const double *__restrict__ xyz, int64_t stride, int64_t rows,
                               int k, const int32_t *__restrict__ ids,
                               const double *__restrict__ g, double *grad) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  double p[D], acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    p[c] = xyz[c * stride + r];
    acc[c] = 0.0;
  }
  for (int j = 0; j < k; ++j) {
    const int32_t q = ids[r * k + j];
    if (q < 0 || q >= stride) continue;
    const double w = g[r * k + j];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double t = 2.0 * (p[c] - xyz[c * stride + q]) * w;
      acc[c] += t;
      unsafeAtomicAdd(&grad[c * stride + q], -t);
    }
  }
#pragma unroll
  for (int c = 0; c < D; ++c) unsafeAtomicAdd(&grad[c * stride + r], acc[c]);
}

hipError_t knn_backward(int dim, const double *xyz, int64_t stride, int64_t rows, int k,
                        const int32_t *ids, const double *g, double *grad, hipStream_t s) {
  hipError_t e = fill_f64(grad, 0.0, (int64_t)dim * stride, s);
  if (e != hipSuccess || rows <= 0) return e;
  unsigned grid = (unsigned)((rows + 255) / 256);
  if (dim == 3) k_knn_backward<3><<<grid, 256, 0, s>>>(xyz, stride, rows, k, ids, g, grad);
  else k_knn_backward<2><<<grid, 256, 0, s>>>(xyz, stride, rows, k, ids, g, grad);
  return hipGetLastError();
}

}  // namespace zd

namespace zd {

// ---------------------------------------------------------------------------
// The same gradient without atomics, in a fixed order: the edges (r, j) are
// sorted by their neighbour q (stable, so by r * k + j within one q), which
// gives every point the list of rows that chose it; one thread per point
// then sums its own terms (j ascending) and the terms of the rows that chose
// it (in that list's order):
//   dL/dp = sum_j 2 (p - p_{ids[p][j]}) g[p][j] + sum_{(r,j): ids[r][j] = p} 2 (p - p_r) g[r][j].
// The result does not depend on scheduling: every run gives the same bits.
// ---------------------------------------------------------------------------

__global__ void k_edge_keys(const int32_t *__restrict__ ids, int64_t ne, int64_t stride,
                            uint64_t *__restrict__ key, int32_t *__restrict__ edge) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int32_t q = ids[e];
  // an absent neighbour (-1) sorts after every point
  key[e] = (q < 0 || q >= stride) ? (uint64_t)stride : (uint64_t)q;
  edge[e] = (int32_t)e;
}

// first[p] = first sorted edge whose neighbour is >= p (a lower bound)
__global__ void k_edge_starts(const uint64_t *__restrict__ key, int64_t ne, int64_t npts,
                              int32_t *__restrict__ first) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p > npts) return;
  int64_t lo = 0, hi = ne;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key[mid] < (uint64_t)p) lo = mid + 1;
    else hi = mid;
  }
  first[p] = (int32_t)lo;
}

template <int D>
__global__ void k_grad_gather(const double *__restrict__ xyz, int64_t stride, int64_t rows,
                              int k, const int32_t *__restrict__ ids,
                              const double *__restrict__ g, const int32_t *__restrict__ edge,
                              const int32_t *__restrict__ first, double *__restrict__ grad) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= stride) return;
  double pc[D], acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    pc[c] = xyz[c * stride + p];
    acc[c] = 0.0;
  }
  if (p < rows) {
    for (int j = 0; j < k; ++j) {
      const int32_t q = ids[p * k + j];
      if (q < 0 || q >= stride) continue;
      const double w = g[p * k + j];
#pragma unroll
      for (int c = 0; c < D; ++c) acc[c] += 2.0 * (pc[c] - xyz[c * stride + q]) * w;
    }
  }
  const int32_t b = first[p], e = first[p + 1];
  for (int32_t x = b; x < e; ++x) {
    const int32_t ed = edge[x];
    const int64_t r = ed / k;
    const double w = g[ed];
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] += 2.0 * (pc[c] - xyz[c * stride + r]) * w;
  }
#pragma unroll
  for (int c = 0; c < D; ++c) grad[c * stride + p] = acc[c];
}

hipError_t knn_backward_det(int dim, const double *xyz, int64_t stride, int64_t rows, int k,
                            const int32_t *ids, const double *g, double *grad, hipStream_t s) {
  if (stride <= 0) return hipSuccess;
  const int64_t ne = rows * (int64_t)k;
  if (ne == 0) return fill_f64(grad, 0.0, (int64_t)dim * stride, s);
  uint64_t *key = nullptr, *ktmp = nullptr;
  int32_t *edge = nullptr, *etmp = nullptr, *first = nullptr;
  hipError_t e = dev_alloc_n(&key, ne, s);
  if (e == hipSuccess) e = dev_alloc_n(&ktmp, ne, s);
  if (e == hipSuccess) e = dev_alloc_n(&edge, ne, s);
  if (e == hipSuccess) e = dev_alloc_n(&etmp, ne, s);
  if (e == hipSuccess) e = dev_alloc_n(&first, stride + 1, s);
  if (e == hipSuccess) {
    k_edge_keys<<<(unsigned)((ne + 255) / 256), 256, 0, s>>>(ids, ne, stride, key, edge);
    e = hipGetLastError();
  }
  int bits = 1;
  while (bits < 63 && (uint64_t(1) << bits) <= (uint64_t)stride) ++bits;
  if (e == hipSuccess) e = radix_sort_pairs(key, edge, ktmp, etmp, ne, bits, s);
  if (e == hipSuccess) {
    k_edge_starts<<<(unsigned)((stride + 1 + 255) / 256), 256, 0, s>>>(key, ne, stride, first);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const unsigned grid = (unsigned)((stride + 255) / 256);
    if (dim == 3)
      k_grad_gather<3><<<grid, 256, 0, s>>>(xyz, stride, rows, k, ids, g, edge, first, grad);
    else
      k_grad_gather<2><<<grid, 256, 0, s>>>(xyz, stride, rows, k, ids, g, edge, first, grad);
    e = hipGetLastError();
  }
  dev_release(key, s);
  dev_release(ktmp, s);
  dev_release(edge, s);
  dev_release(etmp, s);
  dev_release(first, s);
  return e;
}

}  // namespace zd

namespace zd {

// ---------------------------------------------------------------------------
// The same gradient for the all-points rows of a tree, taken in the tree's
// Morton order: workgroup w takes sorted positions [kBwdTile w,
// kBwdTile (w + 1)).  A row's neighbours are mostly Morton neighbours (on
// uniform points, 84% of the k = 8 neighbours fall in the row's own tile), so
// most neighbour terms are summed in LDS; the others are added with FP64
// atomics into a buffer in sorted order (near the row's own position, not
// at a random id).  The tile's sums are stored to a second sorted-order
// buffer, and a last pass writes the sum of the two at each position's id.
// Points that small inserts placed in the side pool (pending in-place
// batches) have their rows taken by a second kernel, one thread per pool
// entry, and their terms summed in a pool-order buffer; a deleted point's
// row is empty (its slot's coordinate is NaN, its row all -1).
// ---------------------------------------------------------------------------
constexpr int kBwdTile = 1024;
constexpr int kBwdBatch = 8;  // neighbours whose loads a thread issues together
static_assert(kBwdBatch == 8, "the vector row loads below take eight entries");

// The terms of row r (point p): each neighbour's share is added to the LDS
// tile sums (a sorted position inside [t0, t0 + kBwdTile), kTile only), to
// gs (another sorted position) or to gp (a pool entry); the row's own terms
// are summed in own.
template <int D, bool kVec, bool kTile>
__device__ __forceinline__ void bwd_row(const TreeView &t, const int32_t *__restrict__ slot_of,
                                        int64_t cap, int k, const int32_t *__restrict__ ids,
                                        const double *__restrict__ g, int64_t r, const double *p,
                                        double *own, int64_t t0, double *acc, double *gs,
                                        double *gp, int64_t pcap) {
  // kBwdBatch neighbours at a time, each step's loads issued together (the
  // row, then the positions, then their coordinates): every load reads a
  // clamped, valid address and the invalid ones are dropped after it, so no
  // branch splits the batch
  const int32_t nmax = (int32_t)t.n - 1;
  for (int j0 = 0; j0 < k; j0 += kBwdBatch) {
    int32_t q[kBwdBatch], sq[kBwdBatch];
    double w[kBwdBatch];
    if constexpr (kVec) {
      // k a multiple of 4 and both tables 16-byte aligned: the row's eight
      // entries in two int4 and four double2 loads (a short row reads its
      // first four twice and drops the copy)
      const bool hi = j0 + 4 < k;
      const int64_t e0 = r * k + j0, e1 = hi ? e0 + 4 : e0;
      const int4 a = *reinterpret_cast<const int4 *>(ids + e0);
      const int4 b = *reinterpret_cast<const int4 *>(ids + e1);
      const double2 w0 = *reinterpret_cast<const double2 *>(g + e0);
      const double2 w1 = *reinterpret_cast<const double2 *>(g + e0 + 2);
      const double2 w2 = *reinterpret_cast<const double2 *>(g + e1);
      const double2 w3 = *reinterpret_cast<const double2 *>(g + e1 + 2);
      q[0] = a.x, q[1] = a.y, q[2] = a.z, q[3] = a.w;
      q[4] = hi ? b.x : -1, q[5] = hi ? b.y : -1, q[6] = hi ? b.z : -1, q[7] = hi ? b.w : -1;
      w[0] = w0.x, w[1] = w0.y, w[2] = w1.x, w[3] = w1.y;
      w[4] = w2.x, w[5] = w2.y, w[6] = w3.x, w[7] = w3.y;
    } else {
#pragma unroll
      for (int u = 0; u < kBwdBatch; ++u) {
        const int64_t e = r * k + min(j0 + u, k - 1);
        q[u] = j0 + u < k ? ids[e] : -1;
        w[u] = g[e];
      }
    }
    // sq: a sorted position (>= 0), a pool entry e as -2 - e, or -1 for
    // padding and dead ids
#pragma unroll
    for (int u = 0; u < kBwdBatch; ++u) {
      const bool in = q[u] >= 0 && q[u] < cap;
      const int32_t v = slot_of[in ? q[u] : 0];
      const bool pool = in && v >= kPoolSlot && (int64_t)(v - kPoolSlot) < pcap;
      sq[u] = in && v >= 0 && v <= nmax ? v : (pool ? -2 - (v - kPoolSlot) : -1);
    }
    double pq[kBwdBatch][3];
#pragma unroll
    for (int u = 0; u < kBwdBatch; ++u) {
      const bool pool = sq[u] <= -2;
      const int32_t v = pool ? -2 - sq[u] : (sq[u] < 0 ? 0 : sq[u]);
      pq[u][0] = (pool ? t.pX : t.X)[v];
      pq[u][1] = (pool ? t.pY : t.Y)[v];
      pq[u][2] = D == 3 ? (pool ? t.pZ : t.Z)[v] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kBwdBatch; ++u) {
      if (sq[u] == -1) continue;
      const int64_t ls = sq[u] - t0;
      const bool local = kTile && sq[u] >= 0 && ls >= 0 && ls < kBwdTile;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const double term = 2.0 * (p[c] - pq[u][c]) * w[u];
        own[c] += term;
        if (local) atomicAdd(&acc[c * kBwdTile + ls], -term);
        else if (sq[u] >= 0) unsafeAtomicAdd(&gs[c * t.n + sq[u]], -term);
        else unsafeAtomicAdd(&gp[c * pcap + (-2 - sq[u])], -term);
      }
    }
  }
}

template <int D, bool kVec>
__global__ void __launch_bounds__(kBwdTile)
    k_knn_backward_tree(TreeView t, const int32_t *__restrict__ slot_of, int64_t cap, int k,
                        const int32_t *__restrict__ ids, const double *__restrict__ g,
                        double *gs, double *__restrict__ gt, double *gp, int64_t pcap) {
  __shared__ double acc[D * kBwdTile];
  const int tid = threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.x * kBwdTile;
  const int64_t i = t0 + tid;
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c * kBwdTile + tid] = 0.0;
  __syncthreads();
  if (i < t.n) {
    const int64_t r = t.id[i];
    const double p[3] = {t.X[i], t.Y[i], D == 3 ? t.Z[i] : 0.0};
    double own[3] = {0.0, 0.0, 0.0};
    bwd_row<D, kVec, true>(t, slot_of, cap, k, ids, g, r, p, own, t0, acc, gs, gp, pcap);
#pragma unroll
    for (int c = 0; c < D; ++c) atomicAdd(&acc[c * kBwdTile + tid], own[c]);
  }
  __syncthreads();
  if (i < t.n) {
#pragma unroll
    for (int c = 0; c < D; ++c) gt[c * t.n + i] = acc[c * kBwdTile + tid];
  }
}

// rows of the live pool entries (a NaN coordinate marks an unused or
// deleted entry)
template <int D, bool kVec>
__global__ void k_knn_backward_pool(TreeView t, const int32_t *__restrict__ slot_of, int64_t cap,
                                    int k, const int32_t *__restrict__ ids,
                                    const double *__restrict__ g, double *gs, double *gp,
                                    int64_t pcap) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= pcap) return;
  const double p[3] = {t.pX[e], t.pY[e], D == 3 ? t.pZ[e] : 0.0};
  if (isnan(p[0])) return;
  const int64_t r = t.pid[e];
  double own[3] = {0.0, 0.0, 0.0};
  bwd_row<D, kVec, false>(t, slot_of, cap, k, ids, g, r, p, own, 0, nullptr, gs, gp, pcap);
#pragma unroll
  for (int c = 0; c < D; ++c) unsafeAtomicAdd(&gp[c * pcap + e], own[c]);
}

template <int D>
__global__ void k_unsort_grad(const int32_t *__restrict__ id, int64_t n,
                              const double *__restrict__ gs, const double *__restrict__ gt,
                              int64_t stride, double *grad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t r = id[i];
#pragma unroll
  for (int c = 0; c < D; ++c) grad[c * stride + r] = gt[c * n + i] + gs[c * n + i];
}

template <int D>
__global__ void k_unsort_pool(TreeView t, int64_t pcap, const double *__restrict__ gp,
                              int64_t stride, double *grad) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= pcap || isnan(t.pX[e])) return;
  const int64_t r = t.pid[e];
#pragma unroll
  for (int c = 0; c < D; ++c) grad[c * stride + r] = gp[c * pcap + e];
}

template <int D, bool kVec>
void launch_backward_tree(const TreeView &t, const int32_t *slot_of, int64_t cap, int k,
                          const int32_t *ids, const double *g, double *gs, double *gt, double *gp,
                          int64_t pcap, double *grad, hipStream_t s) {
  const unsigned tiles = (unsigned)((t.n + kBwdTile - 1) / kBwdTile);
  const unsigned grid = (unsigned)((t.n + 255) / 256);
  k_knn_backward_tree<D, kVec><<<tiles, kBwdTile, 0, s>>>(t, slot_of, cap, k, ids, g, gs, gt, gp,
                                                          pcap);
  if (pcap > 0) {
    const unsigned pgrid = (unsigned)((pcap + 255) / 256);
    k_knn_backward_pool<D, kVec><<<pgrid, 256, 0, s>>>(t, slot_of, cap, k, ids, g, gs, gp, pcap);
    k_unsort_pool<D><<<pgrid, 256, 0, s>>>(t, pcap, gp, cap, grad);
  }
  k_unsort_grad<D><<<grid, 256, 0, s>>>(t.id, t.n, gs, gt, cap, grad);
}

hipError_t knn_backward_tree(int dim, const TreeView &t, const int32_t *slot_of, int64_t cap,
                             int64_t pcap, int k, const int32_t *ids, const double *g,
                             double *grad, hipStream_t s) {
  // every id of the sorted arrays and of the live pool entries is written by
  // the last passes; only dead or unplaced ids need the zero
  hipError_t e = t.n + pcap < cap || pcap > 0 ? fill_f64(grad, 0.0, (int64_t)dim * cap, s)
                                              : hipSuccess;
  if (e != hipSuccess || t.n <= 0) return e;
  const int64_t ns = (int64_t)dim * t.n, np = (int64_t)dim * pcap;
  double *gs = nullptr;
  e = dev_alloc_n(&gs, 2 * ns + np, s);
  if (e == hipSuccess) e = fill_f64(gs, 0.0, ns, s);
  if (e == hipSuccess && np > 0) e = fill_f64(gs + 2 * ns, 0.0, np, s);
  if (e == hipSuccess) {
    double *gt = gs + ns, *gp = pcap > 0 ? gs + 2 * ns : nullptr;
    const bool vec = k % 4 == 0 && (uintptr_t)ids % 16 == 0 && (uintptr_t)g % 16 == 0;
    if (dim == 3) {
      if (vec) launch_backward_tree<3, true>(t, slot_of, cap, k, ids, g, gs, gt, gp, pcap, grad, s);
      else launch_backward_tree<3, false>(t, slot_of, cap, k, ids, g, gs, gt, gp, pcap, grad, s);
    } else {
      if (vec) launch_backward_tree<2, true>(t, slot_of, cap, k, ids, g, gs, gt, gp, pcap, grad, s);
      else launch_backward_tree<2, false>(t, slot_of, cap, k, ids, g, gs, gt, gp, pcap, grad, s);
    }
    e = hipGetLastError();
  }
  dev_release(gs, s);
  return e;
}

}  // namespace zd

