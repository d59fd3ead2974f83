// zd_persist_impl.h -- the batched forest in one persistent launch.
//
// Each cloud is its own zd-tree (Section 2: Morton sort, buildTree of
// Algorithm 1 with the leaf size as its cut-off, tight boxes), and its
// all-points rows are searched from each point's leaf (Algorithms 2 and
// 3).  One kernel does all of it:
//
//  * builds: every workgroup takes clouds from a counter, largest first, and
//    builds each one alone, with workgroup barriers only -- bounding cube and
//    key geometry, Morton keys, a stable LSD radix sort of (key, id) inside
//    the cloud's range of the sorted arrays, the coordinates in key order,
//    split bits, the leaf test and the in-order numbering of the internal
//    nodes (a workgroup scan), then the leaves' boxes and the bottom-up
//    links.  A cloud that starts at sorted position o numbers its internal
//    nodes o + x and its leaves o + j, so no number depends on another cloud
//    and clouds build in any order, on any workgroup.  Each wavefront of the
//    builder releases its stores and then counts itself into the cloud's
//    ready word.
//  * queries: once the cloud counter runs out, every wavefront takes 64-point
//    query groups, in the order the host predicts the clouds to be built,
//    from a second counter, waits
//    for the group's cloud to be ready (every builder wavefront counted; an
//    acquire fence the first time it meets that cloud) and answers the
//    group like the all-points kernel.
//
// Every wait is bounded by the wall clock; one that runs out counts a build
// error and skips its group, so the launch always ends.  Every claimed
// cloud is built by the workgroup that claimed it, which is running, so a
// wait only ever waits on running work.
#pragma once

#include "zd_knn_impl.h"

namespace zd {

constexpr int kPWaves = 4;
constexpr int kPThreads = 64 * kPWaves;  // one radix digit per thread
constexpr int kPItems = 8;
constexpr int kPChunk = kPThreads * kPItems;  // keys ranked per sort step
constexpr int kPHalo = 256;                   // leaf sizes the leaf test serves from LDS

struct PBuildLds {
  int32_t hist[256];              // digit counts, then running output bases
  int32_t wc[kPWaves][256];       // per-wave digit counters of a sort step
  int8_t sbw[kPThreads + 2 * kPHalo];  // split bits of a leaf-test step
  int32_t wsum[kPWaves];
  double box[kPWaves][6];         // per-wave bounding box
  double geo[6];                  // the cloud's lo[3], S[3]
  int32_t task;
};

// Exclusive prefix sum over the workgroup's threads (thread order); the
// total goes to every thread.
__device__ __forceinline__ int32_t p_exscan(int32_t x, PBuildLds &S, int32_t &total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) S.wsum[w] = inc;
  __syncthreads();
  int32_t add = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kPWaves; ++i) {
    add += i < w ? S.wsum[i] : 0;
    all += S.wsum[i];
  }
  total = all;
  __syncthreads();
  return inc - x + add;
}

__device__ __forceinline__ uint32_t p_digit(uint64_t k, int shift) {
  return (uint32_t)(k >> shift) & 255u;
}

// One stable LSD pass over the cloud's range [o, o + m): (kin, vin) ->
// (kout, vout) by the 8 key bits at `shift`.  A histogram of the range
// gives each digit's first output position; the range is then ranked in
// steps of kPChunk keys in order (wave w, round r, lane l holds key
// (w * kPItems + r) * 64 + l of the step; ballots rank equal digits within
// a round, per-wave counters across rounds, and each digit's running base
// carries across steps), so equal digits keep their order.
__device__ void p_pass(PBuildLds &S, const uint64_t *kin, const int32_t *vin, uint64_t *kout,
                       int32_t *vout, int64_t o, int32_t m, int shift) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  S.hist[t] = 0;
  __syncthreads();
  for (int32_t i0 = 0; i0 < m; i0 += kPThreads * 8) {
    uint32_t d[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int32_t i = i0 + r * kPThreads + t;
      d[r] = i < m ? p_digit(kin[o + i], shift) : 256u;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r)
      if (d[r] < 256u) atomicAdd(&S.hist[d[r]], 1);
  }
  __syncthreads();
  {
    int32_t total;
    const int32_t base = p_exscan(S.hist[t], S, total);
    S.hist[t] = base;
  }
  __syncthreads();
  const uint64_t lt = lane ? (~0ULL >> (64 - lane)) : 0ULL;
  for (int32_t c0 = 0; c0 < m; c0 += kPChunk) {
    uint64_t k[kPItems];
    int32_t v[kPItems], rank[kPItems];
    for (int c = lane; c < 256; c += 64) S.wc[w][c] = 0;
#pragma unroll
    for (int r = 0; r < kPItems; ++r) {
      const int32_t i = c0 + (w * kPItems + r) * 64 + lane;
      k[r] = i < m ? kin[o + i] : 0;
      v[r] = i < m ? vin[o + i] : 0;
    }
#pragma unroll
    for (int r = 0; r < kPItems; ++r) {
      const int32_t i = c0 + (w * kPItems + r) * 64 + lane;
      const bool valid = i < m;
      const uint32_t d = p_digit(k[r], shift);
      uint64_t mm = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        mm &= bit ? bb : ~bb;
      }
      const int lower = __popcll(mm & lt), cnt = __popcll(mm);
      const int32_t before = valid ? S.wc[w][d] : 0;
      rank[r] = before + lower;
      if (valid && lower == cnt - 1) S.wc[w][d] = before + cnt;
    }
    __syncthreads();
    {
      // digit t: this step's slots per wave, after the earlier steps' slots
      int32_t run = S.hist[t];
#pragma unroll
      for (int i = 0; i < kPWaves; ++i) {
        const int32_t c = S.wc[i][t];
        S.wc[i][t] = run;
        run += c;
      }
      S.hist[t] = run;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPItems; ++r) {
      const int32_t i = c0 + (w * kPItems + r) * 64 + lane;
      if (i < m) {
        const int64_t p = o + S.wc[w][p_digit(k[r], shift)] + rank[r];
        kout[p] = k[r];
        vout[p] = v[r];
      }
    }
    __syncthreads();
  }
}

// The cloud's key geometry, as a separate zd_build of the cloud would take
// it: the declared box, else the bounding cube (lo = minimum, common side =
// the largest extent, or 1 if it is 0).
template <int D>
__device__ void p_geometry(PBuildLds &S, const PersistArgs &a, int64_t o, int32_t m,
                           Geometry &gc) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (!a.have_box) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t i = t; i < m; i += kPThreads)
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const double v = a.xyz[d * a.n + o + i];
        lo[d] = fmin(lo[d], v);
        hi[d] = fmax(hi[d], v);
      }
#pragma unroll
    for (int d = 0; d < D; ++d)
      for (int off = 32; off > 0; off >>= 1) {
        lo[d] = fmin(lo[d], __shfl_xor(lo[d], off));
        hi[d] = fmax(hi[d], __shfl_xor(hi[d], off));
      }
    if (lane == 0)
      for (int d = 0; d < 3; ++d) {
        S.box[w][d] = lo[d];
        S.box[w][3 + d] = hi[d];
      }
    __syncthreads();
  }
  if (t == 0) {
    const double cells = ldexp(1.0, a.g.B - 1);
    if (a.have_box) {
      for (int d = 0; d < D; ++d) {
        S.geo[d] = a.box.lo[d];
        S.geo[3 + d] = cells / (a.box.hi[d] - a.box.lo[d]);
      }
    } else {
      double lo[3], hi[3];
      for (int d = 0; d < 3; ++d) {
        lo[d] = S.box[0][d];
        hi[d] = S.box[0][3 + d];
        for (int i = 1; i < kPWaves; ++i) {
          lo[d] = fmin(lo[d], S.box[i][d]);
          hi[d] = fmax(hi[d], S.box[i][3 + d]);
        }
      }
      double side = 0.0;
      for (int d = 0; d < D; ++d)
        if (hi[d] - lo[d] > side) side = hi[d] - lo[d];
      if (!(side > 0.0)) side = 1.0;
      for (int d = 0; d < D; ++d) {
        S.geo[d] = m > 0 ? lo[d] : 0.0;
        S.geo[3 + d] = cells / side;
      }
    }
  }
  __syncthreads();
  gc = a.g;
  for (int d = 0; d < D; ++d) {
    gc.lo[d] = S.geo[d];
    gc.S[d] = S.geo[3 + d];
  }
  __syncthreads();
}

// Build cloud c (m >= 1 points from sorted position o) in the forest's
// arrays; the workgroup's threads all call it.
template <int D>
__device__ void p_build_cloud(PBuildLds &S, const PersistArgs &a, const PersistTree &pt,
                              int32_t c, int64_t o, int32_t m) {
  const int t = threadIdx.x;
  Geometry gc;
  p_geometry<D>(S, a, o, m, gc);
  // keys, ids in input order
  for (int32_t i = t; i < m; i += kPThreads) {
    const int64_t p = o + i;
    pt.key[p] = morton_key<D>(gc, a.xyz[p], a.xyz[a.n + p], D == 3 ? a.xyz[2 * a.n + p] : 0.0);
    pt.id[p] = (int32_t)p;
  }
  __syncthreads();
  // stable sort by key: 8 passes of 8 bits over the 63 (3-D) or 64 (2-D)
  // key bits, back and forth between the arrays and the scratch
  if (m > 1)
    for (int sh = 0; sh < 64; sh += 16) {
      p_pass(S, pt.key, pt.id, a.key2, a.id2, o, m, sh);
      p_pass(S, a.key2, a.id2, pt.key, pt.id, o, m, sh + 8);
    }
  // coordinates in key order, id -> slot (four points in flight per thread)
  for (int32_t r0 = 0; r0 < m; r0 += 4 * kPThreads) {
    int32_t src[4];
    double x[4], y[4], z[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t r = r0 + u * kPThreads + t;
      src[u] = r < m ? pt.id[o + r] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t r = r0 + u * kPThreads + t;
      if (r < m) {
        x[u] = a.xyz[src[u]];
        y[u] = a.xyz[a.n + src[u]];
        z[u] = D == 3 ? a.xyz[2 * a.n + src[u]] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t r = r0 + u * kPThreads + t;
      if (r < m) {
        const int64_t p = o + r;
        pt.X[p] = x[u];
        pt.Y[p] = y[u];
        if (D == 3) pt.Z[p] = z[u];
        a.slot_of[src[u]] = (int32_t)p;
      }
    }
  }
  // split bits between neighbours
  for (int32_t r = t; r + 1 < m; r += kPThreads)
    a.sb[o + r] = (int8_t)split_bit(pt.key[o + r], pt.key[o + r + 1]);
  __syncthreads();
  // leaf test and in-order numbering of the internal nodes: the x-th split
  // that fails the leaf test is internal node o + x, and the splits before
  // a point number its leaf
  const int Li = a.leaf_size ? a.leaf_size[c] : a.L;
  // split bits of a step and Li on each side in LDS (outside the cloud: a
  // split above every bit, which ends a scan where the cloud ends)
  const int H = Li <= kPHalo ? Li : 0;
  int32_t I = 0;
  for (int32_t c0 = 0; c0 < m - 1; c0 += kPThreads) {
    const int32_t r = c0 + t;
    if (H > 0) {
      for (int q = t; q < kPThreads + 2 * H; q += kPThreads) {
        const int64_t y = (int64_t)c0 - H + q;
        S.sbw[q] = (y >= 0 && y < m - 1) ? a.sb[o + y] : (int8_t)127;
      }
      __syncthreads();
    }
    int32_t f = 0;
    int b = -1;
    if (r < m - 1) {
      if (H > 0) {
        b = S.sbw[H + t];
        f = leaf_test(b, Li, S.sbw, H + t, 0, kPThreads + 2 * H);
      } else {
        b = a.sb[o + r];
        f = leaf_test(b, Li, a.sb, o + r, o, o + m - 1);
      }
    }
    int32_t total;
    const int32_t ex = p_exscan(f, S, total);
    if (r < m - 1) {
      pt.leaf_of[o + r] = (int32_t)o + I + ex;
      if (f) {
        INode &N = pt.inode[o + I + ex];
        N.split = (int32_t)(o + r);
        N.bit = b;
        N.visits = 0;
        N.parent = -1;
      }
    }
    I += total;
  }
  if (t == 0) pt.leaf_of[o + m - 1] = (int32_t)o + I;
  __syncthreads();
  // leaves: range and tight box, then the climb (as the single-tree build:
  // a node spanning leaves [l, r] hangs below the neighbouring split with
  // the lower bit; the second child to arrive finishes the node)
  for (int32_t j0 = 0; j0 <= I; j0 += kPThreads) {
    const int32_t j = j0 + t;
    if (j > I) continue;
    const int32_t begin = j == 0 ? (int32_t)o : pt.inode[o + j - 1].split + 1;
    const int32_t end = j == I ? (int32_t)(o + m) : pt.inode[o + j].split + 1;
    pt.leaf_begin[o + j] = begin;
    if (j == I) pt.leaf_begin[o + I + 1] = (int32_t)(o + m);
    double lo[3] = {INFINITY, INFINITY, D == 3 ? INFINITY : 0.0};
    double hi[3] = {-INFINITY, -INFINITY, D == 3 ? -INFINITY : 0.0};
    for (int32_t s = begin; s < end; ++s) {
      lo[0] = fmin(lo[0], pt.X[s]);
      hi[0] = fmax(hi[0], pt.X[s]);
      lo[1] = fmin(lo[1], pt.Y[s]);
      hi[1] = fmax(hi[1], pt.Y[s]);
      if (D == 3) {
        lo[2] = fmin(lo[2], pt.Z[s]);
        hi[2] = fmax(hi[2], pt.Z[s]);
      }
    }
    int32_t l = j, r = j;  // cloud-local leaf range of the current node
    int32_t node = ~(int32_t)(o + j);
    int guard = 0;
    for (; guard < 130; ++guard) {
      if (l == 0 && r == I) {
        if (node < 0) pt.leaf_parent[~node] = -1;
        else pt.inode[node].parent = -1;
        break;
      }
      int32_t p;
      int side;
      if (l == 0) {
        p = r;
        side = 0;
      } else if (r == I) {
        p = l - 1;
        side = 1;
      } else {
        side = pt.inode[o + r].bit < pt.inode[o + l - 1].bit ? 0 : 1;
        p = side ? l - 1 : r;
      }
      const int32_t gp = (int32_t)o + p;
      INode *P = &pt.inode[gp];
      P->child[side] = node;
      if (node < 0) pt.leaf_parent[~node] = (gp << 1) | side;
      else pt.inode[node].parent = (gp << 1) | side;
      for (int d = 0; d < 3; ++d) {
        publish_f64(&P->lo[side][d], lo[d]);
        publish_f64(&P->hi[side][d], hi[d]);
      }
      publish_i32(side == 0 ? &P->first_leaf : &P->last_leaf,
                  (int32_t)o + (side == 0 ? l : r));
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      if (atomicAdd(&P->visits, 1) == 0) break;  // the sibling finishes this node
      const int os = 1 - side;
      for (int d = 0; d < 3; ++d) {
        lo[d] = fmin(lo[d], fetch_f64(&P->lo[os][d]));
        hi[d] = fmax(hi[d], fetch_f64(&P->hi[os][d]));
      }
      if (side == 0) r = fetch_i32(&P->last_leaf) - (int32_t)o;
      else l = fetch_i32(&P->first_leaf) - (int32_t)o;
      if (l < 0 || r > I || l > r) {
        atomicAdd(&pt.meta[kMetaBuildErr], 1);
        break;
      }
      node = gp;
    }
    if (guard == 130) atomicAdd(&pt.meta[kMetaBuildErr], 1);
  }
  __syncthreads();
}

template <int K>
constexpr size_t persist_lds_bytes(int waves) {
  const size_t q = (size_t)waves * all_lds_bytes<K>();
  return q > sizeof(PBuildLds) ? q : sizeof(PBuildLds);
}

// Register caps of the all-points kernel that leave room for the build
// code (the k = 10 and 12 caps of 80 and 96 VGPRs would spill it).
template <int K>
constexpr int persist_min_waves() {
  return K == 20 || K == 24 || K == 32 ? 3 : 1;
}

template <int D, int K>
__global__ void __launch_bounds__(kPThreads)
    __attribute__((amdgpu_waves_per_eu(persist_min_waves<K>())))
        k_forest_persistent(PersistArgs a, PersistTree pt, TreeView t, int qwaves) {
  extern __shared__ __align__(16) char smem[];
  PBuildLds &S = *reinterpret_cast<PBuildLds *>(smem);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // builds, one cloud per workgroup at a time
  for (;;) {
    if (threadIdx.x == 0) S.task = atomicAdd(&a.ctl[0], 1);
    __syncthreads();
    const int32_t ci = S.task;
    __syncthreads();
    if (ci >= a.C) break;
    const int32_t c = a.order[ci];
    const int64_t o = a.offsets[c];
    const int32_t m = (int32_t)(a.offsets[c + 1] - o);
    if (m > 0) p_build_cloud<D>(S, a, pt, c, o, m);
    // Publication: the workgroup barrier orders the wavefronts' stores only
    // within the workgroup (it does not wait for them to reach L2), so each
    // wavefront releases its own stores at agent scope and then counts
    // itself into the cloud's ready word; a reader waits for all of them.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0) __hip_atomic_fetch_add(&a.ready[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // queries, one 64-point group per wavefront at a time (wavefronts beyond
  // the LDS that the k bucket needs per wavefront sit this phase out)
  if (w >= qwaves) return;
  int32_t seen = -1;
  bool skip = false;
  for (;;) {
    int32_t gi = 0;
    if (lane == 0) gi = atomicAdd(&a.ctl[1], 1);
    gi = uni(gi);
    if (gi >= a.ngroups) return;
    const int4 G = a.qgroups[gi];
    const int32_t c = uni(G.z);
    if (c != seen) {
      int32_t late = 0;
      if (lane == 0) {
        const int64_t t0 = wall_clock64();
        while (__hip_atomic_load(&a.ready[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
               kPWaves) {
          if (wall_clock64() - t0 > a.wait_ticks) {
            atomicAdd(&pt.meta[kMetaBuildErr], 1);
            late = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(32);
        }
      }
      skip = uni(late) != 0;
      // the cloud's tree as its builder published it
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      seen = c;
    }
    if (skip) continue;
    all_points_group<D, K, false>(t, a.k, a.out_ids, a.out_d2, uni(G.x), uni(G.y),
                                  a.offsets[c], a.offsets[c + 1] - 1, smem, w);
  }
}

// Host: one launch over every resident workgroup slot.
template <int D, int K>
hipError_t launch_forest_persistent(const PersistArgs &a, const PersistTree &pt,
                                    const TreeView &t, hipStream_t s) {
  const int qw = fit_waves<K, true>(kPWaves);
  const size_t lds = persist_lds_bytes<K>(qw);
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_forest_persistent<D, K>,
                                                     kPThreads, lds);
  if (e != hipSuccess) return e;
  const unsigned grid = (unsigned)std::max(1, cus * std::max(1, per_cu));
  k_forest_persistent<D, K><<<grid, kPThreads, lds, s>>>(a, pt, t, qw);
  return hipGetLastError();
}

}  // namespace zd
