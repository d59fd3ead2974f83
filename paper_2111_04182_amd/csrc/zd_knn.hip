// zd_knn.hip -- exact k-NN queries on the zd-tree (gfx950).
//
// One thread answers one query, walking the tree as Algorithm 3 (searchUp)
// prescribes: scan the query's own leaf, then while the ball of the current
// k-th distance is not inside the current node's box, search the sibling
// subtree with Algorithm 2 (searchDown) and move to the parent.  searchDown
// visits a child iff its box distance is <= the current k-th squared
// distance, nearer box centre first (on a tie the right child, Algorithm 2's
// else branch).  It runs without a stack: every node records its parent and
// side, and the child order is recomputed when the walk returns to a node.
//
// All-points queries run in Morton order (thread i = sorted position i), so
// a wavefront's 64 queries share leaves and paths (the query presort of
// Section 3.1); external queries descend from the root by their Morton bits
// (the bit-based search of Section 2).
//
// The candidate set N is a sorted array of K (d2, id) pairs in registers
// (the paper keeps a vector for small k, Section 3.1); k <= K is a runtime
// value and K a compile-time bucket, so every array index is static.
#include "zd_internal.h"

#include <climits>

namespace zd {

template <int K>
struct Heap {
  double d[K];
  int32_t id[K];
  double kth_d;    // d2 of the k-th entry (+inf while fewer than k)
  int32_t kth_id;  // id of the k-th entry (INT_MAX while fewer than k)
  int k;

  __device__ __forceinline__ void init(int k_) {
    k = k_;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      d[j] = INFINITY;
      id[j] = INT_MAX;
    }
    kth_d = INFINITY;
    kth_id = INT_MAX;
  }

  // candidate enters iff it precedes the current k-th entry
  __device__ __forceinline__ void offer(double dd, int32_t q) {
    if (!cand_lt(dd, q, kth_d, kth_id)) return;
#pragma unroll
    for (int j = K - 1; j >= 0; --j) {
      if (j < k) {
        bool lt_prev = (j > 0) && cand_lt(dd, q, d[j > 0 ? j - 1 : 0], id[j > 0 ? j - 1 : 0]);
        bool lt_here = cand_lt(dd, q, d[j], id[j]);
        double nd = lt_prev ? d[j > 0 ? j - 1 : 0] : (lt_here ? dd : d[j]);
        int32_t ni = lt_prev ? id[j > 0 ? j - 1 : 0] : (lt_here ? q : id[j]);
        d[j] = nd;
        id[j] = ni;
      }
    }
    kth_d = d[0];
    kth_id = id[0];
#pragma unroll
    for (int j = 1; j < K; ++j)
      if (j == k - 1) {
        kth_d = d[j];
        kth_id = id[j];
      }
  }
};

template <int D>
__device__ __forceinline__ double centre_dist2(double px, double py, double pz, const double *lo,
                                               const double *hi) {
  double cx = (lo[0] + hi[0]) * 0.5;
  double cy = (lo[1] + hi[1]) * 0.5;
  double cz = D == 3 ? (lo[2] + hi[2]) * 0.5 : 0.0;
  return dist2<D>(px, py, pz, cx, cy, cz);
}

// withinBox(C, p, -r) of Algorithm 3, squared: p in the box and every face
// strictly farther than the k-th d2 (never true while N holds fewer than k,
// because the k-th d2 is then +inf).
template <int D>
__device__ __forceinline__ bool ball_inside(double px, double py, double pz, const double *lo,
                                            const double *hi, double kth) {
  double p[3] = {px, py, pz};
#pragma unroll
  for (int c = 0; c < D; ++c) {
    if (p[c] < lo[c] || p[c] > hi[c]) return false;
    double a = p[c] - lo[c], b = hi[c] - p[c];
    if (!(a * a > kth) || !(b * b > kth)) return false;
  }
  return true;
}

template <int D, int K>
__device__ __forceinline__ void scan_leaf(const TreeView &t, int32_t leaf, double px, double py,
                                          double pz, int32_t self, Heap<K> &h) {
  const int32_t b = t.leaf_begin[leaf], e = t.leaf_begin[leaf + 1];
  for (int32_t s = b; s < e; ++s) {
    const int32_t q = t.id[s];
    const double dd = dist2<D>(px, py, pz, t.X[s], t.Y[s], D == 3 ? t.Z[s] : 0.0);
    if (q != self) h.offer(dd, q);
  }
}

// searchDown (Algorithm 2) of the subtree under internal node `top`, whose
// own box already passed the test.  Stackless: the walk state is the current
// node, whether it is being entered, and from which side it was re-entered.
// `budget` bounds the walk: a valid tree enters each internal node at most
// three times, so the bound is never reached; it only turns a corrupted tree
// into wrong rows instead of a wave that never retires.
template <int D, int K>
__device__ __forceinline__ void search_down(const TreeView &t, int32_t top, double px, double py,
                                            double pz, int32_t self, Heap<K> &h,
                                            int64_t &budget) {
  int32_t n = top;
  bool entering = true;
  int from_side = 0;
  while (--budget > 0) {
    const INode *N = &t.inode[n];
    const double c0 = centre_dist2<D>(px, py, pz, N->lo[0], N->hi[0]);
    const double c1 = centre_dist2<D>(px, py, pz, N->lo[1], N->hi[1]);
    const int first = c0 < c1 ? 0 : 1;
    int s = entering ? first : (from_side == first ? 1 - first : 2);
    bool descended = false;
    while (s != 2) {
      if (box_dist2<D>(px, py, pz, N->lo[s], N->hi[s]) <= h.kth_d) {
        const int32_t ch = N->child[s];
        if (ch < 0) {
          scan_leaf<D, K>(t, ~ch, px, py, pz, self, h);
        } else {
          n = ch;
          entering = true;
          descended = true;
          break;
        }
      }
      s = (s == first) ? 1 - first : 2;
    }
    if (descended) continue;
    if (n == top) return;
    const int32_t par = N->parent;
    if (par < 0) return;
    from_side = par & 1;
    n = par >> 1;
    entering = false;
  }
}

// searchUp (Algorithm 3) after the start leaf has been scanned
template <int D, int K>
__device__ __forceinline__ void search_up(const TreeView &t, int32_t leaf, double px, double py,
                                          double pz, int32_t self, Heap<K> &h) {
  int64_t budget = 4 * t.n + 256;
  int32_t link = t.leaf_parent[leaf];
  while (link >= 0 && --budget > 0) {
    const int32_t p = link >> 1;
    const int side = link & 1;
    const INode *P = &t.inode[p];
    if (ball_inside<D>(px, py, pz, P->lo[side], P->hi[side], h.kth_d)) break;
    const int os = 1 - side;
    if (box_dist2<D>(px, py, pz, P->lo[os], P->hi[os]) <= h.kth_d) {
      const int32_t ch = P->child[os];
      if (ch < 0) scan_leaf<D, K>(t, ~ch, px, py, pz, self, h);
      else search_down<D, K>(t, ch, px, py, pz, self, h, budget);
    }
    link = P->parent;
  }
}

template <int K>
__device__ __forceinline__ void write_row(const Heap<K> &h, int k, int32_t *out_ids,
                                          double *out_d2) {
#pragma unroll
  for (int j = 0; j < K; ++j)
    if (j < k) {
      out_ids[j] = h.id[j] == INT_MAX ? -1 : h.id[j];
      out_d2[j] = h.d[j];
    }
}

template <int D, int K>
__global__ void __launch_bounds__(256) k_knn_all(TreeView t, int k, int32_t *__restrict__ out_ids,
                                                 double *__restrict__ out_d2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= t.n) return;
  const double px = t.X[i], py = t.Y[i], pz = D == 3 ? t.Z[i] : 0.0;
  const int32_t self = t.id[i];
  const int32_t leaf = t.leaf_of[i];
  Heap<K> h;
  h.init(k);
  scan_leaf<D, K>(t, leaf, px, py, pz, self, h);
  search_up<D, K>(t, leaf, px, py, pz, self, h);
  write_row<K>(h, k, out_ids + (int64_t)self * k, out_d2 + (int64_t)self * k);
}

template <int D, int K>
__global__ void __launch_bounds__(256) k_knn_ext(TreeView t, Geometry g,
                                                 const double *__restrict__ q, int64_t m, int k,
                                                 int32_t *__restrict__ out_ids,
                                                 double *__restrict__ out_d2) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  const double px = q[r], py = q[m + r], pz = D == 3 ? q[2 * m + r] : 0.0;
  Heap<K> h;
  h.init(k);
  int32_t node = t.meta[kMetaRoot];
  if (node != kNoRoot) {
    const uint64_t key = morton_key<D>(g, px, py, pz);
    // a path has at most 64 internal nodes: each splits on a lower bit
    for (int guard = 0; node >= 0 && guard < 66; ++guard) {
      const INode *N = &t.inode[node];
      node = N->child[(key >> N->bit) & 1];
    }
    if (node < 0) {
      const int32_t leaf = ~node;
      scan_leaf<D, K>(t, leaf, px, py, pz, -1, h);
      search_up<D, K>(t, leaf, px, py, pz, -1, h);
    }
  }
  write_row<K>(h, k, out_ids + r * k, out_d2 + r * k);
}

__global__ void k_dead_rows(const int32_t *__restrict__ slot_of, int64_t cap, int k,
                            int32_t *__restrict__ out_ids, double *__restrict__ out_d2) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= cap || slot_of[r] >= 0) return;
  for (int j = 0; j < k; ++j) {
    out_ids[r * k + j] = -1;
    out_d2[r * k + j] = INFINITY;
  }
}

hipError_t fill_dead_rows(const int32_t *slot_of, int64_t cap, int k, int32_t *out_ids,
                          double *out_d2, hipStream_t s) {
  if (cap <= 0) return hipSuccess;
  k_dead_rows<<<(unsigned)((cap + 255) / 256), 256, 0, s>>>(slot_of, cap, k, out_ids, out_d2);
  return hipGetLastError();
}

template <int D, int K>
static hipError_t launch_all(const TreeView &t, int k, int32_t *ids, double *d2, hipStream_t s) {
  k_knn_all<D, K><<<(unsigned)((t.n + 255) / 256), 256, 0, s>>>(t, k, ids, d2);
  return hipGetLastError();
}

template <int D>
static hipError_t dispatch_all(const TreeView &t, int k, int32_t *ids, double *d2,
                               hipStream_t s) {
  if (k <= 1) return launch_all<D, 1>(t, k, ids, d2, s);
  if (k <= 4) return launch_all<D, 4>(t, k, ids, d2, s);
  if (k <= 8) return launch_all<D, 8>(t, k, ids, d2, s);
  if (k <= 16) return launch_all<D, 16>(t, k, ids, d2, s);
  if (k <= 32) return launch_all<D, 32>(t, k, ids, d2, s);
  return launch_all<D, 64>(t, k, ids, d2, s);
}

hipError_t knn_all_points(int dim, const TreeView &t, int k, int32_t *out_ids, double *out_d2,
                          hipStream_t s) {
  if (t.n <= 0) return hipSuccess;
  return dim == 3 ? dispatch_all<3>(t, k, out_ids, out_d2, s)
                  : dispatch_all<2>(t, k, out_ids, out_d2, s);
}

template <int D, int K>
static hipError_t launch_ext(const TreeView &t, const Geometry &g, const double *q, int64_t m,
                             int k, int32_t *ids, double *d2, hipStream_t s) {
  k_knn_ext<D, K><<<(unsigned)((m + 255) / 256), 256, 0, s>>>(t, g, q, m, k, ids, d2);
  return hipGetLastError();
}

template <int D>
static hipError_t dispatch_ext(const TreeView &t, const Geometry &g, const double *q, int64_t m,
                               int k, int32_t *ids, double *d2, hipStream_t s) {
  if (k <= 1) return launch_ext<D, 1>(t, g, q, m, k, ids, d2, s);
  if (k <= 4) return launch_ext<D, 4>(t, g, q, m, k, ids, d2, s);
  if (k <= 8) return launch_ext<D, 8>(t, g, q, m, k, ids, d2, s);
  if (k <= 16) return launch_ext<D, 16>(t, g, q, m, k, ids, d2, s);
  if (k <= 32) return launch_ext<D, 32>(t, g, q, m, k, ids, d2, s);
  return launch_ext<D, 64>(t, g, q, m, k, ids, d2, s);
}

hipError_t knn_external(int dim, const TreeView &t, const Geometry &g, const double *q,
                        int64_t m, int k, int32_t *out_ids, double *out_d2, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  return dim == 3 ? dispatch_ext<3>(t, g, q, m, k, out_ids, out_d2, s)
                  : dispatch_ext<2>(t, g, q, m, k, out_ids, out_d2, s);
}

}  // namespace zd
