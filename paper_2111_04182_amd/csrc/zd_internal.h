// zd_internal.h -- internal types and device helpers of libzd (gfx950).
//
// Everything here is private to the library; the public interface is
// include/zd.h.  All HIP sources are compiled with -ffp-contract=off so that
// no multiply-add is ever fused: squared distances must round exactly as
// ((dx*dx + dy*dy) + dz*dz) does in IEEE binary64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zd.h"

namespace zd {

// ---------------------------------------------------------------------------
// tree layout in device memory
// ---------------------------------------------------------------------------

// One internal node.  The tight boxes of BOTH children are stored in the
// parent, so a single 128-byte line answers "which children does the ball
// reach, and which is nearer" during the search (Algorithm 2 reads the two
// children's boxes and centres together).
//   child[s] >= 0 : internal node index;  child[s] < 0 : leaf ~child[s].
//   parent        : (parent << 1) | side-in-parent, or -1 at the root.
//   bit           : the Morton key bit the node splits on.
//   split         : sorted position p; the left subtree ends at point p.
//   first/last    : the node's leaves, inclusive.
//   visits        : arrival counter of the bottom-up construction.
struct alignas(128) INode {
  double lo[2][3];
  double hi[2][3];
  int32_t child[2];
  int32_t parent;
  int32_t bit;
  int32_t split;
  int32_t first_leaf;
  int32_t last_leaf;
  int32_t visits;
};
static_assert(sizeof(INode) == 128, "INode must fill one cache line");

constexpr int32_t kNoRoot = INT32_MIN;

// Key geometry: rounding to integers (Section 3.1) and the random shift
// (Section 2).  B = 64/dim bits per coordinate; the box maps onto the low
// 2^(B-1) cells, the shift is < 2^(B-1).
struct Geometry {
  double lo[3];
  double S[3];
  uint64_t shift[3];
  int32_t dim;
  int32_t B;
};

// An axis-aligned box, passed to kernels by value.
struct Box3 {
  double lo[3];
  double hi[3];
};

// Device view of a built tree, passed to kernels by value.
struct TreeView {
  const uint64_t *key;      // [n] Morton keys, ascending
  const int32_t *id;        // [n] point id of each sorted position
  const double *X, *Y, *Z;  // [n] coordinates in sorted order
  const int32_t *leaf_of;   // [n] leaf holding each sorted position
  const int32_t *leaf_begin;   // [n_leaves + 1]
  const int32_t *leaf_parent;  // [n_leaves] (parent << 1) | side, -1 if root
  const INode *inode;       // [n_internal]
  const int32_t *meta;      // meta[0] = n_internal, meta[1] = root
  int32_t *walk_err;        // &meta[kMetaWalkErr]: counts searches that gave up
  int64_t n;
  int64_t walk_limit;       // steps a search may take; 0: 4n + 256 (never reached)
  // Points inserted by small batches since the last relink: leaf l holds,
  // besides its sorted range, ovf_cnt[l] points at pool entries
  // [ovf_blk[l] * kOvfBlock, + ovf_cnt[l]).  Null when nothing is pending.
  // Deleted points keep their slot with a NaN x coordinate (a NaN distance
  // never enters a candidate set, and a NaN query answers nothing).
  const int32_t *ovf_blk, *ovf_cnt;
  const double *pX, *pY, *pZ;
  const int32_t *pid;
};

// pool entries per leaf block (at most this many small-batch points per leaf
// before the tree is rebuilt)
constexpr int kOvfBlock = 16;
// slot_of values at or above this encode a pool entry (slot - kPoolSlot)
constexpr int32_t kPoolSlot = int32_t(1) << 30;

// meta[] slots: the internal node count and root of the tree; a status word
// for the validation of updates; the count of corrupted climbs in the build
// and of searches that gave up (both stay zero on a valid tree, and are read
// at the next call that synchronises); the depth, when asked for.
enum {
  kMetaInternal = 0,
  kMetaRoot = 1,
  kMetaCheck = 2,
  kMetaBuildErr = 3,
  kMetaWalkErr = 4,
  kMetaDepth = 5,
  kMetaLocal = 6,   // small insert: points that cannot join their leaf in place
  kMetaBlocks = 7,  // small insert: leaves that need a new pool block
  kMetaCount = 8
};

// Links are stored as (node << 1) | side in int32, so node indices, and
// with them the points of one tree (internal nodes <= points - 1), stay
// below 2^30.
constexpr int64_t kMaxLive = (int64_t(1) << 30) - 1;

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

// highest set bit of a non-zero 64-bit value
__device__ __forceinline__ int high_bit64(uint64_t v) { return 63 - __clzll((long long)v); }

// Split bit between two sorted keys, -1 if equal.
__device__ __forceinline__ int split_bit(uint64_t a, uint64_t b) {
  uint64_t x = a ^ b;
  return x ? high_bit64(x) : -1;
}

// Position i (between sorted points i and i+1) is an internal node iff the
// run of points that share the prefix above its split bit b holds more than
// L points (the leaf test of Algorithm 1).  Point x shares that prefix with
// point i iff no split between them exceeds b, so the run extends from i
// while the adjacent split bits stay <= b, and the scan stops once more than
// L points are seen.
__device__ __forceinline__ int32_t leaf_test(int b, int Li, const int8_t *sb, int64_t i,
                                             int64_t lo, int64_t hi) {
  if (b >= 64) return 1;  // cloud boundaries are always internal: no leaf mixes clouds
  if (b < 0) return 0;
  int64_t left = 1, right = 1;
  for (int64_t y = i - 1; y >= lo && left + right <= Li; --y) {
    if (sb[y] > b) break;
    ++left;
  }
  for (int64_t y = i + 1; y < hi && left + right <= Li; ++y) {
    if (sb[y] > b) break;
    ++right;
  }
  return left + right > Li ? 1 : 0;
}

// Values a child hands to its parent during the climb travel through device-
// scope atomics only (64-bit exchanges to publish, no-op RMWs to read), which
// are coherent across the chip's L2 slices; a __threadfence() here would write
// back and invalidate the whole L2 at every step.
__device__ __forceinline__ void publish_f64(double *p, double v) {
  atomicExch(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}
__device__ __forceinline__ double fetch_f64(double *p) {
  return __longlong_as_double((long long)atomicOr(reinterpret_cast<unsigned long long *>(p), 0ULL));
}
__device__ __forceinline__ void publish_i32(int32_t *p, int32_t v) { atomicExch(p, v); }
__device__ __forceinline__ int32_t fetch_i32(int32_t *p) { return atomicOr(p, 0); }

// One coordinate to its integer cell: u = (x - lo) * S, floor, clamp into
// [0, 2^(B-1) - 1]; monotone non-decreasing in x (NaN goes to cell 0).
__device__ __forceinline__ uint64_t cell_of(double x, double lo, double S, int B) {
  const uint64_t top = (uint64_t(1) << (B - 1)) - 1;
  double u = (x - lo) * S;
  if (!(u >= 0.0)) return 0;
  double f = floor(u);
  if (f >= (double)top) return top;
  return (uint64_t)f;
}

// Spread the low 21 bits of v so bit j lands at 3j (3-D interleave).
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
  v &= 0x1fffffULL;
  v = (v | (v << 32)) & 0x001f00000000ffffULL;
  v = (v | (v << 16)) & 0x001f0000ff0000ffULL;
  v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
  v = (v | (v << 2)) & 0x1249249249249249ULL;
  return v;
}

// Spread the low 32 bits of v so bit j lands at 2j (2-D interleave).
__device__ __forceinline__ uint64_t spread2(uint64_t v) {
  v &= 0xffffffffULL;
  v = (v | (v << 16)) & 0x0000ffff0000ffffULL;
  v = (v | (v << 8)) & 0x00ff00ff00ff00ffULL;
  v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0fULL;
  v = (v | (v << 2)) & 0x3333333333333333ULL;
  v = (v | (v << 1)) & 0x5555555555555555ULL;
  return v;
}

// Morton key (Section 1.1): bit j of coordinate c at key bit d*j + (d-1-c),
// x most significant within each group.
template <int D>
__device__ __forceinline__ uint64_t morton_key(const Geometry &g, double x, double y, double z) {
  if constexpr (D == 3) {
    uint64_t cx = cell_of(x, g.lo[0], g.S[0], 21) + g.shift[0];
    uint64_t cy = cell_of(y, g.lo[1], g.S[1], 21) + g.shift[1];
    uint64_t cz = cell_of(z, g.lo[2], g.S[2], 21) + g.shift[2];
    return (spread3(cx) << 2) | (spread3(cy) << 1) | spread3(cz);
  } else {
    uint64_t cx = cell_of(x, g.lo[0], g.S[0], 32) + g.shift[0];
    uint64_t cy = cell_of(y, g.lo[1], g.S[1], 32) + g.shift[1];
    return (spread2(cx) << 1) | spread2(cy);
  }
}

// Squared distance with the fixed evaluation order (no FMA: the sources are
// built with -ffp-contract=off).
template <int D>
__device__ __forceinline__ double dist2(double px, double py, double pz, double qx, double qy,
                                        double qz) {
  double dx = px - qx;
  double dy = py - qy;
  double s = dx * dx + dy * dy;
  if constexpr (D == 3) {
    double dz = pz - qz;
    s = s + dz * dz;
  }
  return s;
}

// Gap from p to [lo, hi] along one axis (0 inside).  Rounding is monotone, so
// for any point q of the box fl(gap) <= |fl(p - q)|: the box distance never
// exceeds a member's distance, and pruning with it is exact.
__device__ __forceinline__ double axis_gap(double p, double lo, double hi) {
  // at most one of lo - p and p - hi is positive (lo <= hi)
  return fmax(fmax(lo - p, p - hi), 0.0);
}

template <int D>
__device__ __forceinline__ double box_dist2(double px, double py, double pz, const double *lo,
                                            const double *hi) {
  double tx = axis_gap(px, lo[0], hi[0]);
  double ty = axis_gap(py, lo[1], hi[1]);
  double s = tx * tx + ty * ty;
  if constexpr (D == 3) {
    double tz = axis_gap(pz, lo[2], hi[2]);
    s = s + tz * tz;
  }
  return s;
}

// (d, i) < (e, j) in the order on (d2, id).  Bitwise, not short-circuit: the
// three compares combine as lane masks instead of nested divergent branches.
__device__ __forceinline__ bool cand_lt(double d, int32_t i, double e, int32_t j) {
  return (d < e) | ((d == e) & (i < j));
}

// ---------------------------------------------------------------------------
// host-side internals (implemented across the .hip files)
// ---------------------------------------------------------------------------

// device allocation ordered on a stream (cached blocks reused on the same
// stream).  While an arena is
// active on the calling thread (graph capture), allocations are carved from
// it instead and releases are no-ops, so a captured graph calls no
// allocator.
hipError_t dev_alloc(void **p, size_t bytes, hipStream_t s);
void dev_release(void *p, hipStream_t s);
struct Arena {
  char *base;
  size_t size;
  size_t used;
};
void arena_activate(Arena *a);  // nullptr deactivates
// a pinned 64-byte host buffer of the calling thread (nullptr if pinned
// memory is unavailable): destination of device-to-host status words
int32_t *host_flag();

template <typename T>
hipError_t dev_alloc_n(T **p, int64_t n, hipStream_t s) {
  return dev_alloc(reinterpret_cast<void **>(p), sizeof(T) * (size_t)(n > 0 ? n : 1), s);
}

// fill kernels (used instead of hipMemsetAsync, which must not be recorded
// in captured graphs)
hipError_t fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t fill_f64(double *p, double v, int64_t n, hipStream_t s);

// exclusive prefix sum of int32 values; the total goes to *total (device)
// when total != nullptr.  in and out may alias.
hipError_t exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total,
                              hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by key bits [0, key_bits).
// Sorted pairs end in (key, val); key_tmp/val_tmp are scratch of n entries.
// With `tiles` (device, ntiles entries of {start, count <= kSortTileKeys,
// count base, tiles in segment}) each segment of the array is sorted on its
// own.
constexpr int kSortTileKeys = 4096;  // keys per sort workgroup (256 digits each)
hipError_t radix_sort_pairs(uint64_t *key, int32_t *val, uint64_t *key_tmp, int32_t *val_tmp,
                            int64_t n, int key_bits, hipStream_t s, const int4 *tiles = nullptr,
                            int ntiles = 0);

// (key, value) pairs sorted by (key, value) in one workgroup, n <=
// kSmallSortKeys (values distinct)
constexpr int kSmallSortKeys = 2048;
hipError_t sort_pairs_small(uint64_t *key, int32_t *val, int64_t n, hipStream_t s);

// Build kernels.  n points sorted by key in (key, id); the tree arrays have
// room for n leaves and n internal nodes.
struct BuildBuffers {
  uint64_t *key;
  int32_t *id;
  double *X, *Y, *Z;
  int32_t *leaf_of;
  int32_t *leaf_begin;
  int32_t *leaf_parent;
  INode *inode;
  int32_t *meta;
  double *root_box;  // [6]: lo[3], hi[3]
  int32_t *flag;     // scratch [n]
  const int32_t *seg = nullptr;       // forest: cloud of each sorted position
  const int32_t *seg_leaf = nullptr;  // forest: leaf size of each cloud
  int32_t max_leaf = 0;               // forest: the largest entry of seg_leaf
};
// aos (nullable): also write each point as one (x, y, z, 0) / (x, y) record,
// so that the later gather reads one aligned record per point instead of
// one 8-byte value from each coordinate array
hipError_t encode_keys(const Geometry &g, const double *xyz, int64_t stride, int64_t n,
                       int32_t id_base, uint64_t *key, int32_t *id, hipStream_t s,
                       double *aos = nullptr);
// Forest: per-cloud key geometry (seg_lo/seg_S [C][3]) and the cloud of
// every point (seg [n]); offsets is a device copy of the cloud bounds.
hipError_t forest_geometry(int dim, const double *xyz, int64_t n, const int64_t *offsets, int C,
                           int B, const double *box_lo, const double *box_hi, int32_t *seg,
                           double *seg_lo, double *seg_S, hipStream_t s);
hipError_t encode_keys_seg(const Geometry &g, const double *xyz, int64_t n, const int32_t *seg,
                           const double *seg_lo, const double *seg_S, uint64_t *key, int32_t *id,
                           hipStream_t s);
// aos (nullable): read the points from encode_keys' records instead of xyz
hipError_t gather_points(int dim, const double *xyz, int64_t stride, const int32_t *id,
                         int64_t n, double *X, double *Y, double *Z, int32_t *slot_of,
                         hipStream_t s, const double *aos = nullptr);
hipError_t build_tree_links(int dim, int leaf_size, int64_t n, const BuildBuffers &b,
                            hipStream_t s);
// the largest number of edges from the root to a leaf, into *depth (device)
hipError_t tree_depth(const int32_t *leaf_parent, const INode *inode, int64_t n_leaves,
                      int32_t *depth, hipStream_t s);

// Queries.  groups == nullptr: wavefront w answers sorted positions
// [64w, 64w + 64); otherwise wavefront w answers [groups[w].x, groups[w].y],
// which lie in the cloud [groups[w].z, groups[w].w] (a forest's groups never
// span two clouds).  query_waves: wavefronts per workgroup (1, 2 or 4).
// The persistent forest launch (zd_persist_impl.h): the forest's arrays,
// which its builds write and its queries read through a TreeView.
struct PersistTree {
  uint64_t *key;
  int32_t *id;
  double *X, *Y, *Z;
  int32_t *leaf_of, *leaf_begin, *leaf_parent;
  INode *inode;
  int32_t *meta;
};

struct PersistArgs {
  const double *xyz;        // the caller's points, SoA [dim][n]
  int64_t n;
  const int64_t *offsets;   // [C + 1]
  const int32_t *order;     // [C] clouds by decreasing size
  int32_t C;
  const int32_t *leaf_size; // [C], or null: L for every cloud
  int32_t L;
  Geometry g;               // dim, B and shift (lo and S are per cloud)
  int32_t have_box;         // one declared box for every cloud
  Box3 box;
  uint64_t *key2;           // [n] sort scratch
  int32_t *id2;             // [n] sort scratch
  int8_t *sb;               // [n] split bits
  int32_t *slot_of;         // [n]
  int32_t *ctl;             // [0]: next cloud to build, [1]: next query group
  int32_t *ready;           // [C]: builder wavefronts done (zero before the launch)
  const int4 *qgroups;      // {first, last, cloud, 0}, by predicted build completion
  int64_t ngroups;
  int32_t *out_ids;
  double *out_d2;
  int32_t k;
  int64_t wait_ticks;       // bound on one wait, in wall-clock ticks
};

hipError_t forest_persistent_d2(const PersistArgs &a, const PersistTree &pt, const TreeView &t,
                                hipStream_t s);
hipError_t forest_persistent_d3(const PersistArgs &a, const PersistTree &pt, const TreeView &t,
                                hipStream_t s);

hipError_t knn_all_points(int dim, const TreeView &t, int k, int32_t *out_ids, double *out_d2,
                          hipStream_t s, int query_waves, const int4 *groups = nullptr,
                          int64_t ngroups = 0);
hipError_t knn_external(int dim, const TreeView &t, const Geometry &g, const double *q,
                        int64_t m, int k, int32_t *out_ids, double *out_d2, hipStream_t s,
                        int query_waves);
// Root-based search (Section 2: Algorithm 2 from the root, empty candidate
// set): all-points rows when q == nullptr (m ignored), else external queries.
hipError_t knn_root_based(int dim, const TreeView &t, const Geometry &g, const double *q,
                          int64_t m, int k, int32_t *out_ids, double *out_d2, hipStream_t s,
                          int query_waves);
// All-points rows of the pool entries [0, m) (points of small inserts not
// yet merged into the sorted arrays): each entry queries the tree with
// itself excluded; rows go to pid[entry].  pxyz is SoA with stride pstride.
hipError_t knn_pool_rows(int dim, const TreeView &t, const Geometry &g, const double *pxyz,
                         int64_t pstride, const int32_t *pid, int64_t m, int k, int32_t *out_ids,
                         double *out_d2, hipStream_t s, int query_waves, bool root);
hipError_t fill_dead_rows(const int32_t *slot_of, int64_t cap, int k, int32_t *out_ids,
                          double *out_d2, hipStream_t s);

// Backward
hipError_t knn_backward(int dim, const double *xyz, int64_t stride, int64_t rows, int k,
                        const int32_t *ids, const double *g, double *grad, hipStream_t s);
// the same without atomics, in a fixed order (bit-identical between runs)
hipError_t knn_backward_det(int dim, const double *xyz, int64_t stride, int64_t rows, int k,
                            const int32_t *ids, const double *g, double *grad, hipStream_t s);

// Updates
// Backward of a tree's own all-points rows (rows by id, cap of them), in
// the tree's Morton order with in-tile sums in LDS (zd_grad.hip).
hipError_t knn_backward_tree(int dim, const TreeView &t, const int32_t *slot_of, int64_t cap,
                             int64_t pcap, int k, const int32_t *ids, const double *g,
                             double *grad, hipStream_t s);
hipError_t count_outside_box(int dim, const double *xyz, int64_t m, const double *lo,
                             const double *hi, int32_t *counter, hipStream_t s);
hipError_t box_reduce(int dim, const double *xyz, int64_t n, double *out_lo_hi, hipStream_t s);
hipError_t merge_sorted(const uint64_t *ka, const int32_t *ia, int64_t na, const uint64_t *kb,
                        const int32_t *ib, int64_t nb, int32_t *mark_scratch, uint64_t *kout,
                        int32_t *iout, int32_t *src, hipStream_t s);
hipError_t gather_merged(int dim, const int32_t *src, int64_t n, const double *X, const double *Y,
                         const double *Z, const double *bxyz, int64_t nb, int32_t id_base,
                         const int32_t *iout, double *X2, double *Y2, double *Z2,
                         int32_t *slot_of, hipStream_t s);
hipError_t validate_delete(const int32_t *ids, int64_t m, int64_t cap, const int32_t *slot_of,
                           int32_t *mark, int32_t *err, hipStream_t s);
hipError_t unmark_ids(const int32_t *ids, int64_t m, int64_t cap, int32_t *mark, hipStream_t s);
hipError_t kill_ids(const int32_t *ids, int64_t m, int32_t *slot_of, int32_t *mark,
                    int32_t *dead_slot, hipStream_t s);
hipError_t compact_live(int dim, const int32_t *dead_slot, int64_t n, int32_t *scan_scratch,
                        const uint64_t *key, const int32_t *id, const double *X,
                        const double *Y, const double *Z, uint64_t *key2, int32_t *id2,
                        double *X2, double *Y2, double *Z2, int32_t *slot_of, hipStream_t s);
hipError_t iota_i32(int32_t *p, int32_t base, int64_t n, hipStream_t s);

// Small batches in place (see zd_update.hip)
constexpr int kMaxPath = 64;  // internal nodes on a root-to-leaf path of one tree
hipError_t insert_in_place_locate(const INode *inode, const uint64_t *tkey,
                                  const int32_t *leaf_begin, const int32_t *meta,
                                  const uint64_t *bk, int64_t m, const int32_t *ovf_blk,
                                  const int32_t *ovf_cnt, int32_t *leaf, int32_t *path,
                                  int32_t *depth, int32_t *local_fail, int32_t *blocks_needed,
                                  hipStream_t s);
hipError_t insert_in_place_commit(int dim, const int32_t *leaf, int64_t m, const int32_t *path,
                                  const int32_t *depth, const int32_t *bi, const double *bxyz,
                                  int32_t id_base, int32_t *ovf_blk, int32_t *ovf_cnt,
                                  int32_t *blocks_used, double *pxyz, int64_t pcap, int32_t *pid,
                                  int32_t *slot_of, INode *inode, double *root_box,
                                  int32_t *new_ids, hipStream_t s);
// One launch for a batch of at most kSmallSortKeys points: the box check,
// keys, sort, descent with paths and room check of the two calls above
// (counts to meta[kMetaCheck], meta[kMetaLocal], meta[kMetaBlocks]).
hipError_t insert_in_place_prepare(const Geometry &g, const double *lo, const double *hi,
                                   const double *xyz, int64_t m, int32_t id_base,
                                   const INode *inode, const uint64_t *tkey,
                                   const int32_t *leaf_begin, int32_t *meta,
                                   const int32_t *ovf_blk, const int32_t *ovf_cnt, uint64_t *bk,
                                   int32_t *bi, int32_t *leaf, int32_t *path, int32_t *depth,
                                   hipStream_t s);
hipError_t tombstone_ids(const int32_t *ids, int64_t m, int32_t *slot_of, int32_t *mark,
                         double *X, double *pX, hipStream_t s);
// live flags of the sorted slots and the pool entries, scanned (positions
// in scan_scratch[n + np], the count in *nlive_dev)
hipError_t count_live(const double *X, int64_t n, const double *pX, int64_t np,
                      int32_t *scan_scratch, int32_t *nlive_dev, hipStream_t s);
// Folding pending small batches back into the sorted arrays (zd_update.hip)
// (key, id) pairs (ids distinct) into (key, id) order; ktmp, itmp, k2, i2:
// scratch of n entries each
hipError_t sort_key_id(uint64_t *key, int32_t *id, int64_t n, int key_bits, uint64_t *ktmp,
                       int32_t *itmp, uint64_t *k2, int32_t *i2, hipStream_t s);
hipError_t fold_main(int dim, const int32_t *pos, int64_t n, const uint64_t *key,
                     const int32_t *id, const double *X, const double *Y, const double *Z,
                     uint64_t *key2, int32_t *id2, double *X2, double *Y2, double *Z2,
                     hipStream_t s);
hipError_t fold_extra(int dim, const int32_t *pos, int64_t n, int64_t np, int64_t na,
                      const double *pxyz, int64_t pcap, const int32_t *pid, const double *bxyz,
                      int64_t nb, int32_t id_base, int64_t ne, double *out, int32_t *out_id,
                      hipStream_t s);
hipError_t fold_gather(int dim, const int32_t *src, int64_t n2, int64_t na, const double *X,
                       const double *Y, const double *Z, const double *pxyz, int64_t pcap,
                       const double *bxyz, int64_t nb, int32_t id_base, const int32_t *iout,
                       double *X2, double *Y2, double *Z2, int32_t *slot_of, hipStream_t s);

}  // namespace zd
