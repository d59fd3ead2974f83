// zd_build.hip -- zd-tree construction on gfx950.
//
// Algorithm 1 (buildTree) recurses top-down: a range of Morton-sorted points
// with more than L points and distinct keys splits on its highest differing
// key bit (found by binary search, splitUsingBit), and empty cuts are skipped
// (Section 2.1).  The resulting tree is the binary radix (Patricia) tree of
// the sorted keys, truncated at nodes of at most L points.  This file builds
// the same tree bottom-up, with no recursion and a constant number of
// launches:
//
//  1. encode:   per point, round to integer cells, add the shift, interleave.
//  2. sort:     radix sort of (key, id)  (zd_sort.hip).
//  3. gather:   coordinates into Morton order (structure of arrays), id map.
//  4. flags:    sorted position i (between points i and i+1) carries the
//               split of the radix node whose highest differing bit is
//               bit(i) = highest bit of key[i] ^ key[i+1]; that node spans
//               the maximal run of points around i sharing key[i]'s prefix
//               above bit(i).  Position i is an internal zd-tree node iff
//               the run holds more than L points (a bounded scan of at most
//               L+1 neighbours each way decides it).
//  5. compact:  scan the flags; internal node x = x-th flagged position,
//               which is the in-order numbering of internal nodes.
//  6. leaves:   in a full binary tree the in-order sequence alternates
//               leaf, internal, ..., leaf, so leaf j is the run of points
//               between internal positions j-1 and j.  One thread per leaf
//               computes its tight box, then climbs: the parent of a node
//               spanning leaves [l, r] is whichever neighbouring internal
//               node (l-1 or r) splits on the lower bit.  Each parent's
//               second arriving child merges the two boxes and continues,
//               so every node is finished exactly once.
#include "zd_internal.h"

namespace zd {

// ----------------------------------------------------------------- encode --

// points per record of the AoS staging copy: 4 doubles (32 B) in 3-D, 2 in 2-D
template <int D>
constexpr int kAos = D == 3 ? 4 : 2;

template <int D>
__global__ void k_encode(Geometry g, const double *__restrict__ xyz, int64_t stride, int64_t n,
                         int32_t id_base, uint64_t *__restrict__ key, int32_t *__restrict__ id,
                         double *__restrict__ aos) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = xyz[i], y = xyz[stride + i];
  double z = D == 3 ? xyz[2 * stride + i] : 0.0;
  key[i] = morton_key<D>(g, x, y, z);
  id[i] = id_base + (int32_t)i;
  if (aos) {
    double2 *r = reinterpret_cast<double2 *>(aos + (int64_t)kAos<D> * i);
    r[0] = make_double2(x, y);
    if (D == 3) r[1] = make_double2(z, 0.0);
  }
}

hipError_t encode_keys(const Geometry &g, const double *xyz, int64_t stride, int64_t n,
                       int32_t id_base, uint64_t *key, int32_t *id, hipStream_t s, double *aos) {
  if (n <= 0) return hipSuccess;
  unsigned grid = (unsigned)((n + 255) / 256);
  if (g.dim == 3)
    k_encode<3><<<grid, 256, 0, s>>>(g, xyz, stride, n, id_base, key, id, aos);
  else
    k_encode<2><<<grid, 256, 0, s>>>(g, xyz, stride, n, id_base, key, id, aos);
  return hipGetLastError();
}

// ------------------------------------------------------- forest: geometry --

// One block per cloud: mark the cloud's positions, reduce its bounding box,
// and derive the cloud's own key geometry the way zd_build does for a single
// tree (lo = minimum, common side = largest extent or 1, S = 2^(B-1)/side;
// with a declared box, that box for every cloud).
template <int D>
__global__ void __launch_bounds__(256) k_seg_geometry(const double *__restrict__ xyz, int64_t n,
                                                      const int64_t *__restrict__ offsets,
                                                      int B, int have_box, Box3 box,
                                                      int32_t *__restrict__ seg,
                                                      double *__restrict__ seg_lo,
                                                      double *__restrict__ seg_S) {
  __shared__ double red[6][256];
  const int c = blockIdx.x;
  const int64_t a = offsets[c], b = offsets[c + 1];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) {
    seg[i] = c;
    for (int d = 0; d < D; ++d) {
      const double v = xyz[d * n + i];
      lo[d] = fmin(lo[d], v);
      hi[d] = fmax(hi[d], v);
    }
  }
  for (int d = 0; d < 3; ++d) {
    red[d][threadIdx.x] = lo[d];
    red[3 + d][threadIdx.x] = hi[d];
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int d = 0; d < 3; ++d) {
        red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + w]);
        red[3 + d][threadIdx.x] = fmax(red[3 + d][threadIdx.x], red[3 + d][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double cells = ldexp(1.0, B - 1);
    if (have_box) {
      for (int d = 0; d < D; ++d) {
        seg_lo[c * 3 + d] = box.lo[d];
        seg_S[c * 3 + d] = cells / (box.hi[d] - box.lo[d]);
      }
    } else {
      double side = 0.0;
      for (int d = 0; d < D; ++d)
        if (red[3 + d][0] - red[d][0] > side) side = red[3 + d][0] - red[d][0];
      if (!(side > 0.0)) side = 1.0;
      for (int d = 0; d < D; ++d) {
        seg_lo[c * 3 + d] = b > a ? red[d][0] : 0.0;
        seg_S[c * 3 + d] = cells / side;
      }
    }
  }
}

template <int D>
__global__ void k_encode_seg(const double *__restrict__ xyz, int64_t n,
                             const int32_t *__restrict__ seg, const double *__restrict__ seg_lo,
                             const double *__restrict__ seg_S, Geometry g,
                             uint64_t *__restrict__ key, int32_t *__restrict__ id) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = seg[i];
  Geometry gc = g;
  for (int d = 0; d < D; ++d) {
    gc.lo[d] = seg_lo[c * 3 + d];
    gc.S[d] = seg_S[c * 3 + d];
  }
  key[i] = morton_key<D>(gc, xyz[i], xyz[n + i], D == 3 ? xyz[2 * n + i] : 0.0);
  id[i] = (int32_t)i;
}

hipError_t forest_geometry(int dim, const double *xyz, int64_t n, const int64_t *offsets, int C,
                           int B, const double *box_lo, const double *box_hi, int32_t *seg,
                           double *seg_lo, double *seg_S, hipStream_t s) {
  if (C <= 0) return hipSuccess;
  Box3 box{};
  const int have = box_lo != nullptr;
  for (int d = 0; d < dim && have; ++d) {
    box.lo[d] = box_lo[d];
    box.hi[d] = box_hi[d];
  }
  if (dim == 3)
    k_seg_geometry<3><<<C, 256, 0, s>>>(xyz, n, offsets, B, have, box, seg, seg_lo, seg_S);
  else
    k_seg_geometry<2><<<C, 256, 0, s>>>(xyz, n, offsets, B, have, box, seg, seg_lo, seg_S);
  return hipGetLastError();
}

hipError_t encode_keys_seg(const Geometry &g, const double *xyz, int64_t n, const int32_t *seg,
                           const double *seg_lo, const double *seg_S, uint64_t *key, int32_t *id,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  unsigned grid = (unsigned)((n + 255) / 256);
  if (g.dim == 3)
    k_encode_seg<3><<<grid, 256, 0, s>>>(xyz, n, seg, seg_lo, seg_S, g, key, id);
  else
    k_encode_seg<2><<<grid, 256, 0, s>>>(xyz, n, seg, seg_lo, seg_S, g, key, id);
  return hipGetLastError();
}

// ----------------------------------------------------------------- gather --

template <int D>
__global__ void k_gather(const double *__restrict__ xyz, int64_t stride,
                         const int32_t *__restrict__ id, int64_t n, double *__restrict__ X,
                         double *__restrict__ Y, double *__restrict__ Z,
                         int32_t *__restrict__ slot_of, const double *__restrict__ aos) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t src = id[i];
  if (aos) {
    const double2 *r = reinterpret_cast<const double2 *>(aos + (int64_t)kAos<D> * src);
    const double2 a = r[0];
    X[i] = a.x;
    Y[i] = a.y;
    if (D == 3) Z[i] = r[1].x;
  } else {
    X[i] = xyz[src];
    Y[i] = xyz[stride + src];
    if (D == 3) Z[i] = xyz[2 * stride + src];
  }
  slot_of[src] = (int32_t)i;
}

hipError_t gather_points(int dim, const double *xyz, int64_t stride, const int32_t *id,
                         int64_t n, double *X, double *Y, double *Z, int32_t *slot_of,
                         hipStream_t s, const double *aos) {
  if (n <= 0) return hipSuccess;
  unsigned grid = (unsigned)((n + 255) / 256);
  if (dim == 3)
    k_gather<3><<<grid, 256, 0, s>>>(xyz, stride, id, n, X, Y, Z, slot_of, aos);
  else
    k_gather<2><<<grid, 256, 0, s>>>(xyz, stride, id, n, X, Y, Z, slot_of, aos);
  return hipGetLastError();
}

// ------------------------------------------------------------------ flags --

// Split bit between sorted positions i and i+1.  In a forest the order is by
// (cloud, key): a change of cloud splits above every key bit, at 64 + the
// highest differing bit of the cloud numbers, so the top of the tree
// separates the clouds and each cloud's subtree is its own zd-tree.
__device__ __forceinline__ int pos_split_bit(const uint64_t *key, const int32_t *seg, int64_t i) {
  if (seg) {
    const uint32_t a = (uint32_t)seg[i], b = (uint32_t)seg[i + 1];
    if (a != b) return 64 + 31 - __clz((int)(a ^ b));
  }
  return split_bit(key[i], key[i + 1]);
}

// Split bit of every adjacent pair (-1 for equal keys, >= 64 between two
// clouds), one byte each: the flag pass scans these instead of keys.
__global__ void k_split_bits(const uint64_t *__restrict__ key, const int32_t *__restrict__ seg,
                             int64_t n, int8_t *__restrict__ sb) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  sb[i] = (int8_t)pos_split_bit(key, seg, i);
}

// Leaf sizes up to kFlagHalo: the workgroup's 256 split bits and kFlagHalo
// on each side are staged in LDS, and the scans read LDS.  Positions outside
// the array read as a split above every bit, which ends a scan where the
// array ends.
constexpr int kFlagBlock = 256;
constexpr int kFlagHalo = 256;

__global__ void __launch_bounds__(kFlagBlock)
    k_split_flags_lds(const int8_t *__restrict__ sb, const int32_t *__restrict__ seg, int64_t n,
                      int L, int H, const int32_t *__restrict__ seg_leaf,
                      int32_t *__restrict__ flag) {
  __shared__ int8_t s[kFlagBlock + 2 * kFlagHalo];
  const int64_t i0 = (int64_t)blockIdx.x * kFlagBlock;
  for (int q = threadIdx.x; q < kFlagBlock + 2 * H; q += kFlagBlock) {
    const int64_t y = i0 - H + q;
    s[q] = (y >= 0 && y < n - 1) ? sb[y] : (int8_t)127;
  }
  __syncthreads();
  const int64_t i = i0 + threadIdx.x;
  if (i >= n - 1) return;
  const int c = H + (int)threadIdx.x;
  const int Li = seg_leaf ? seg_leaf[seg[i]] : L;  // <= H
  flag[i] = leaf_test(s[c], Li, s, c, 0, kFlagBlock + 2 * H);
}

// Any leaf size: the scans read device memory.
__global__ void k_split_flags(const int8_t *__restrict__ sb, const int32_t *__restrict__ seg,
                              int64_t n, int L, const int32_t *__restrict__ seg_leaf,
                              int32_t *__restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  const int Li = seg_leaf ? seg_leaf[seg[i]] : L;
  flag[i] = leaf_test(sb[i], Li, sb, i, 0, n - 1);
}

// ---------------------------------------------------------------- compact --

__global__ void k_compact(const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                          const int8_t *__restrict__ sb, int64_t n, INode *__restrict__ inode) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1 || !flag[i]) return;
  INode &N = inode[pos[i]];
  N.split = (int32_t)i;
  N.bit = sb[i];
  N.visits = 0;
  N.parent = -1;
}

// ------------------------------------------------- leaves + bottom-up links --

constexpr int kLeafBlock = 256;

// One thread per leaf: the leaf's point range and tight box (from points the
// workgroup stages in LDS), then the climb.
// A node spanning leaves [l, r] hangs below the neighbouring split (l-1 or r)
// with the lower bit; each node is finished by the second child to arrive.
// Workgroup w takes leaves [256w, 256w + 256).  An internal node whose whole
// leaf range lies in that window ("local": its nearest higher splits on both
// sides lie in the window, found by a scan of the window's split bits in
// LDS) has both children climbed by this workgroup, so its two children meet
// in LDS; only the nodes above a window's local subtrees meet through device
// memory.
template <int D>
__global__ void __launch_bounds__(kLeafBlock)
    k_leaves(const double *__restrict__ X, const double *__restrict__ Y,
             const double *__restrict__ Z, int64_t n, INode *inode, int32_t *meta,
             int32_t *__restrict__ leaf_begin, int32_t *leaf_parent,
             int32_t *__restrict__ leaf_of, double *root_box) {
  __shared__ int32_t s_bit[kLeafBlock + 1];  // split bits of nodes j0-1 .. j0+255
  __shared__ int32_t s_loc[kLeafBlock];      // node j0+t is local
  __shared__ int32_t s_cnt[kLeafBlock];      // arrivals at local node j0+t
  __shared__ int32_t s_end[kLeafBlock][2];   // outer leaf bound of each child
  __shared__ double s_box[kLeafBlock][2][6]; // box of each child (lo, hi)
  __shared__ double s_pt[3][kLeafBlock];     // a chunk of the window's points
  __shared__ int32_t s_range[2];             // the window's points [P0, P1)
  const int t = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * kLeafBlock;
  const int32_t I = meta[kMetaInternal];
  if (j0 > I) return;
  // nodes outside [0, I) act as splits above every bit: the tree's ends
  for (int q = t; q <= kLeafBlock; q += kLeafBlock) {
    const int64_t x = j0 - 1 + q;
    s_bit[q] = (x >= 0 && x < I) ? inode[x].bit : INT_MAX;
  }
  s_cnt[t] = 0;
  __syncthreads();
  {
    // node x = j0 + t splits leaves x and x+1; its range ends at the nearest
    // higher split on each side (LDS index q holds node j0 - 1 + q)
    bool loc = false;
    const int64_t x = j0 + t;
    if (x < I && t < kLeafBlock - 1) {
      const int32_t bx = s_bit[t + 1];
      bool lok = false, rok = false;
      for (int q = t; q >= 0 && !lok; --q) lok = s_bit[q] > bx;
      for (int q = t + 2; q <= kLeafBlock && !rok; ++q) rok = s_bit[q] > bx;
      loc = lok && rok;
    }
    s_loc[t] = loc ? 1 : 0;
  }
  __syncthreads();
  const int64_t j = j0 + t;
  const bool own = j <= I;  // this thread's leaf exists
  int32_t begin = 0, end = 0;
  if (own) {
    begin = j == 0 ? 0 : inode[j - 1].split + 1;
    end = j == I ? (int32_t)n : inode[j].split + 1;
    leaf_begin[j] = begin;
    // leaf_of[s] for s < n-1 already holds the exclusive count of splits
    // before s, which is the leaf of s; only the last point is left
    if (j == I) {
      leaf_begin[I + 1] = (int32_t)n;
      leaf_of[n - 1] = I;
    }
  }
  // Leaf boxes.  The window's leaves hold the contiguous points [P0, P1);
  // the workgroup reads them in coalesced chunks into LDS and each thread
  // folds in the part of the chunk that belongs to its leaf.
  if (t == 0) s_range[0] = begin;
  if (j == min(j0 + kLeafBlock - 1, (int64_t)I)) s_range[1] = end;
  __syncthreads();
  const int32_t P0 = s_range[0], P1 = s_range[1];
  double lo[3] = {INFINITY, INFINITY, D == 3 ? INFINITY : 0.0};
  double hi[3] = {-INFINITY, -INFINITY, D == 3 ? -INFINITY : 0.0};
  for (int32_t c0 = P0; c0 < P1; c0 += kLeafBlock) {
    const int32_t p = c0 + t;
    if (p < P1) {
      s_pt[0][t] = X[p];
      s_pt[1][t] = Y[p];
      if (D == 3) s_pt[2][t] = Z[p];
    }
    __syncthreads();
    const int32_t a = max(begin, c0), b = min(end, c0 + kLeafBlock);
    for (int32_t s = a; s < b; ++s) {
      const double x = s_pt[0][s - c0], y = s_pt[1][s - c0];
      lo[0] = fmin(lo[0], x); hi[0] = fmax(hi[0], x);
      lo[1] = fmin(lo[1], y); hi[1] = fmax(hi[1], y);
      if (D == 3) {
        const double z = s_pt[2][s - c0];
        lo[2] = fmin(lo[2], z); hi[2] = fmax(hi[2], z);
      }
    }
    __syncthreads();
  }
  if (!own) return;
  auto bit_of = [&](int32_t x) -> int32_t {
    const int64_t q = (int64_t)x - (j0 - 1);
    return (q >= 0 && q <= kLeafBlock) ? s_bit[q] : inode[x].bit;
  };
  int32_t l = (int32_t)j, r = (int32_t)j;
  int32_t node = ~(int32_t)j;
  // every climb ends at the root or hands its node to the sibling's climb
  // within one step per level (at most 64 levels per cloud, plus the levels
  // that separate a forest's clouds); running out of steps is a corruption
  int guard = 0;
  for (; guard < 130; ++guard) {
    if (l == 0 && r == I) {
      meta[kMetaRoot] = node;
      if (node < 0) leaf_parent[~node] = -1;
      else inode[node].parent = -1;
      for (int c = 0; c < 3; ++c) { root_box[c] = lo[c]; root_box[3 + c] = hi[c]; }
      break;
    }
    int32_t p;
    int side;
    if (l == 0) { p = r; side = 0; }
    else if (r == I) { p = l - 1; side = 1; }
    else {
      side = bit_of(r) < bit_of(l - 1) ? 0 : 1;
      p = side ? l - 1 : r;
    }
    INode *P = &inode[p];
    // links are read only by later kernels: plain stores
    P->child[side] = node;
    if (node < 0) leaf_parent[~node] = (p << 1) | side;
    else inode[node].parent = (p << 1) | side;
    const int os = 1 - side;
    const int64_t qp = (int64_t)p - j0;
    if (qp >= 0 && qp < kLeafBlock && s_loc[qp]) {
      // both children of p are climbed in this workgroup: meet in LDS
      for (int c = 0; c < 3; ++c) {
        P->lo[side][c] = lo[c];
        P->hi[side][c] = hi[c];
        s_box[qp][side][c] = lo[c];
        s_box[qp][side][3 + c] = hi[c];
      }
      if (side == 0) P->first_leaf = l; else P->last_leaf = r;
      s_end[qp][side] = side == 0 ? l : r;
      // the box is in LDS before the arrival is counted; the second arrival
      // reads the sibling's box after its count
      if (__hip_atomic_fetch_add(&s_cnt[qp], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) == 0)
        break;
      for (int c = 0; c < 3; ++c) {
        lo[c] = fmin(lo[c], s_box[qp][os][c]);
        hi[c] = fmax(hi[c], s_box[qp][os][3 + c]);
      }
      if (side == 0) r = s_end[qp][os]; else l = s_end[qp][os];
    } else {
      // what the sibling needs now: this child's box and outer bound
      for (int c = 0; c < 3; ++c) {
        publish_f64(&P->lo[side][c], lo[c]);
        publish_f64(&P->hi[side][c], hi[c]);
      }
      publish_i32(side == 0 ? &P->first_leaf : &P->last_leaf, side == 0 ? l : r);
      // every publish has completed before the arrival is counted
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      if (atomicAdd(&P->visits, 1) == 0) break;  // the sibling finishes this node
      for (int c = 0; c < 3; ++c) {
        lo[c] = fmin(lo[c], fetch_f64(&P->lo[os][c]));
        hi[c] = fmax(hi[c], fetch_f64(&P->hi[os][c]));
      }
      if (side == 0) r = fetch_i32(&P->last_leaf); else l = fetch_i32(&P->first_leaf);
    }
    // a corrupted exchange ends the climb instead of indexing out of range
    if (l < 0 || r > I || l > r) {
      atomicAdd(&meta[kMetaBuildErr], 1);
      break;
    }
    node = p;
  }
  if (guard == 130) atomicAdd(&meta[kMetaBuildErr], 1);
}

// One thread per leaf: count the links up to the root.
__global__ void k_leaf_depth(const int32_t *__restrict__ leaf_parent,
                             const INode *__restrict__ inode, int64_t nl, int32_t *depth) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nl) return;
  int32_t d = 0;
  int32_t link = leaf_parent[j];
  while (link >= 0 && d < 1024) {
    ++d;
    link = inode[link >> 1].parent;
  }
  atomicMax(depth, d);
}

hipError_t tree_depth(const int32_t *leaf_parent, const INode *inode, int64_t n_leaves,
                      int32_t *depth, hipStream_t s) {
  hipError_t e = fill_i32(depth, 0, 1, s);
  if (e != hipSuccess || n_leaves <= 0) return e;
  k_leaf_depth<<<(unsigned)((n_leaves + 255) / 256), 256, 0, s>>>(leaf_parent, inode, n_leaves,
                                                                  depth);
  return hipGetLastError();
}

hipError_t build_tree_links(int dim, int leaf_size, int64_t n, const BuildBuffers &b,
                            hipStream_t s) {
  hipError_t e = hipSuccess;
  if (n <= 0) {
    e = fill_i32(b.meta, 0, 1, s);
    if (e == hipSuccess) e = fill_i32(b.meta + kMetaRoot, kNoRoot, 1, s);
    return e;
  }
  const unsigned grid_n = (unsigned)((n + 255) / 256);
  if (n > 1) {
    int8_t *sb = nullptr;
    e = dev_alloc_n(&sb, n, s);
    if (e == hipSuccess) {
      k_split_bits<<<grid_n, 256, 0, s>>>(b.key, b.seg, n, sb);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      const int H = b.max_leaf > 0 ? b.max_leaf : leaf_size;  // largest leaf size in use
      if (H <= kFlagHalo)
        k_split_flags_lds<<<grid_n, kFlagBlock, 0, s>>>(sb, b.seg, n, leaf_size, H, b.seg_leaf,
                                                        b.flag);
      else
        k_split_flags<<<grid_n, 256, 0, s>>>(sb, b.seg, n, leaf_size, b.seg_leaf, b.flag);
      e = hipGetLastError();
    }
    // exclusive split counts: the node number of each split for the
    // compaction, and at the same time leaf_of (the splits before a point
    // number its leaf; the leaf pass adds the last point)
    if (e == hipSuccess)
      e = exclusive_scan_i32(b.flag, b.leaf_of, n - 1, b.meta + kMetaInternal, s);
    if (e == hipSuccess) {
      k_compact<<<grid_n, 256, 0, s>>>(b.flag, b.leaf_of, sb, n, b.inode);
      e = hipGetLastError();
    }
    dev_release(sb, s);
  } else {
    e = fill_i32(b.meta + kMetaInternal, 0, 1, s);
  }
  if (e != hipSuccess) return e;
  if (dim == 3)
    k_leaves<3><<<grid_n, kLeafBlock, 0, s>>>(b.X, b.Y, b.Z, n, b.inode, b.meta, b.leaf_begin,
                                      b.leaf_parent, b.leaf_of, b.root_box);
  else
    k_leaves<2><<<grid_n, kLeafBlock, 0, s>>>(b.X, b.Y, b.Z, n, b.inode, b.meta, b.leaf_begin,
                                      b.leaf_parent, b.leaf_of, b.root_box);
  return hipGetLastError();
}

}  // namespace zd
