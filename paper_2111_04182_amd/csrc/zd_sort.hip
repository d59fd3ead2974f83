// zd_sort.hip -- stable LSD radix sort of (Morton key, id) pairs.
//
// The Morton sort of Section 2 ("Construction"); the paper notes a radix sort
// gives linear work (Section 2.1, Theorem 1).  Each pass handles 8 key bits
// in three kernels: per-tile digit counts, an exclusive scan of the counts in
// digit-major order (which gives every (digit, tile) its output base), and a
// stable scatter.  Inside a tile, each 64-lane wavefront ranks 64 keys at a
// time: eight ballots find the lanes holding the same digit, and a per-wave
// digit counter in LDS carries the running rank across rounds, so equal keys
// keep their input order (ties stay in ascending id order).  The tile is
// reordered by digit in LDS before it is written, so the stores coalesce.
#include "zd_internal.h"

namespace zd {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortThreads = 1024;  // 16 wavefronts
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortItems = 4;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 keys
static_assert(kSortTile == kSortTileKeys, "tile tables assume kSortTileKeys keys per tile");
static_assert(kSortThreads >= kRadix, "a thread per digit");
constexpr int kWaveSpan = 64 * kSortItems;            // keys per wave per tile

__device__ __forceinline__ uint32_t digit_of(uint64_t k, int shift) {
  return (uint32_t)(k >> shift) & (kRadix - 1);
}

// A tile is at most kSortTile consecutive keys inside one segment; its
// digit counts live at cbase + digit * nts (nts = tiles of its segment), so
// one exclusive scan over all counts in (segment, digit, tile) order gives
// every (tile, digit) its output base.  With tiles == nullptr the whole
// array is one segment cut into uniform tiles.
struct TileInfo {
  int64_t start, end, cbase, nts;
};

__device__ __forceinline__ TileInfo tile_info(const int4 *tiles, int64_t n, int ntiles) {
  TileInfo ti;
  if (tiles) {
    const int4 d = tiles[blockIdx.x];
    ti.start = d.x;
    ti.end = (int64_t)d.x + d.y;
    ti.cbase = d.z;
    ti.nts = d.w;
  } else {
    ti.start = (int64_t)blockIdx.x * kSortTile;
    ti.end = min(ti.start + kSortTile, n);
    ti.cbase = blockIdx.x;
    ti.nts = ntiles;
  }
  return ti;
}

__global__ void __launch_bounds__(kSortThreads) k_radix_count(const uint64_t *key, int64_t n,
                                                              int shift, int32_t *counts,
                                                              int ntiles, const int4 *tiles) {
  __shared__ int32_t hist[kRadix];
  if (threadIdx.x < kRadix) hist[threadIdx.x] = 0;
  __syncthreads();
  const TileInfo ti = tile_info(tiles, n, ntiles);
#pragma unroll 4
  for (int j = 0; j < kSortItems; ++j) {
    int64_t i = ti.start + (int64_t)j * kSortThreads + threadIdx.x;
    if (i < ti.end) atomicAdd(&hist[digit_of(key[i], shift)], 1);
  }
  __syncthreads();
  if (threadIdx.x < kRadix) counts[ti.cbase + (int64_t)threadIdx.x * ti.nts] = hist[threadIdx.x];
}

// Exclusive prefix sum of one int per thread over the workgroup; `wsum`
// holds one int per wavefront.  (Threads past the 256 digits pass 0.)
__device__ __forceinline__ int32_t digit_exclusive_scan(int32_t x, int32_t *wsum) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  int32_t inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int32_t add = 0;
#pragma unroll
  for (int i = 0; i < kSortWaves; ++i) add += i < w ? wsum[i] : 0;
  return inc - x + add;
}

// Stable scatter of one tile.  The tile's pairs are first ordered by digit
// in LDS (local position = tile-local start of the digit + the pair's rank
// among the tile's pairs of that digit), then written out in that order, so
// consecutive lanes store to consecutive addresses of one digit's run.
__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(
    const uint64_t *__restrict__ key_in, const int32_t *__restrict__ val_in,
    uint64_t *__restrict__ key_out, int32_t *__restrict__ val_out, int64_t n, int shift,
    const int32_t *__restrict__ offsets, int ntiles, const int4 *tiles) {
  __shared__ int32_t wcount[kSortWaves][kRadix];
  __shared__ int32_t gbase[kRadix];  // output position of local slot 0 of each digit
  __shared__ int32_t wsum[kSortWaves];
  __shared__ uint64_t skey[kSortTile];
  __shared__ int32_t sval[kSortTile];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  if (threadIdx.x < kRadix)
#pragma unroll
    for (int i = 0; i < kSortWaves; ++i) wcount[i][threadIdx.x] = 0;
  __syncthreads();

  const TileInfo ti = tile_info(tiles, n, ntiles);
  const int64_t base = ti.start + (int64_t)w * kWaveSpan;
  const uint64_t lt_mask = lane ? (~0ULL >> (64 - lane)) : 0ULL;
  uint64_t k[kSortItems];
  int32_t v[kSortItems];
  int32_t rank[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    int64_t i = base + r * 64 + lane;
    bool valid = i < ti.end;
    k[r] = valid ? key_in[i] : 0;
    v[r] = valid ? val_in[i] : 0;
    uint32_t d = digit_of(k[r], shift);
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      bool bit = (d >> b) & 1u;
      uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    int lower = __popcll(m & lt_mask);
    int cnt = __popcll(m);
    int32_t before = valid ? wcount[w][d] : 0;
    rank[r] = before + lower;
    if (valid && lower == cnt - 1) wcount[w][d] = before + cnt;
  }
  __syncthreads();
  {
    // thread d: the digit's per-wave starts, then its start in the tile
    const int d = threadIdx.x;
    int32_t run = 0;
    if (d < kRadix) {
#pragma unroll
      for (int i = 0; i < kSortWaves; ++i) {
        int32_t t = wcount[i][d];
        wcount[i][d] = run;
        run += t;
      }
    }
    const int32_t start = digit_exclusive_scan(run, wsum);
    if (d < kRadix) {
#pragma unroll
      for (int i = 0; i < kSortWaves; ++i) wcount[i][d] += start;
      gbase[d] = offsets[ti.cbase + (int64_t)d * ti.nts] - start;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    int64_t i = base + r * 64 + lane;
    if (i < ti.end) {
      const int32_t lp = wcount[w][digit_of(k[r], shift)] + rank[r];
      skey[lp] = k[r];
      sval[lp] = v[r];
    }
  }
  __syncthreads();
  const int32_t cnt = (int32_t)(ti.end - ti.start);
  for (int32_t i = threadIdx.x; i < cnt; i += kSortThreads) {
    const uint64_t kk = skey[i];
    const int64_t pos = (int64_t)gbase[digit_of(kk, shift)] + i;
    key_out[pos] = kk;
    val_out[pos] = sval[i];
  }
}

hipError_t radix_sort_pairs(uint64_t *key, int32_t *val, uint64_t *key_tmp, int32_t *val_tmp,
                            int64_t n, int key_bits, hipStream_t s, const int4 *tiles,
                            int ntiles_seg) {
  if (n <= 1) return hipSuccess;
  const int ntiles = tiles ? ntiles_seg : (int)((n + kSortTile - 1) / kSortTile);
  const int64_t ncounts = (int64_t)kRadix * ntiles;
  int32_t *counts = nullptr;
  hipError_t e = dev_alloc_n(&counts, ncounts, s);
  if (e != hipSuccess) return e;
  uint64_t *ka = key, *kb = key_tmp;
  int32_t *va = val, *vb = val_tmp;
  int passes = 0;
  for (int shift = 0; shift < key_bits && e == hipSuccess; shift += kRadixBits) {
    k_radix_count<<<ntiles, kSortThreads, 0, s>>>(ka, n, shift, counts, ntiles, tiles);
    e = hipGetLastError();
    if (e == hipSuccess) e = exclusive_scan_i32(counts, counts, ncounts, nullptr, s);
    if (e == hipSuccess) {
      k_radix_scatter<<<ntiles, kSortThreads, 0, s>>>(ka, va, kb, vb, n, shift, counts, ntiles,
                                                      tiles);
      e = hipGetLastError();
    }
    uint64_t *tk = ka; ka = kb; kb = tk;
    int32_t *tv = va; va = vb; vb = tv;
    ++passes;
  }
  if (e == hipSuccess && (passes & 1)) {
    e = hipMemcpyAsync(key, ka, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(val, va, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s);
  }
  dev_release(counts, s);
  return e;
}

}  // namespace zd

namespace zd {

// A batch of at most kSmallSortKeys pairs sorted by one workgroup in LDS
// (bitonic sort on (key, value), values distinct, padding above every real
// pair): one launch instead of the radix sort's three per pass, for the
// small batches whose cost is launch latency.  With values given in
// ascending order (batch ids), the order equals a stable sort by key.
__global__ void __launch_bounds__(1024) k_sort_small(uint64_t *key, int32_t *val, int m, int np2) {
  __shared__ uint64_t sk[kSmallSortKeys];
  __shared__ int32_t sv[kSmallSortKeys];
  // np2: the power of two >= m that the network spans
  for (int i = threadIdx.x; i < np2; i += blockDim.x) {
    sk[i] = i < m ? key[i] : ~uint64_t(0);
    sv[i] = i < m ? val[i] : INT_MAX;
  }
  __syncthreads();
  for (int size = 2; size <= np2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < np2 / 2; i += blockDim.x) {
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
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    key[i] = sk[i];
    val[i] = sv[i];
  }
}

hipError_t sort_pairs_small(uint64_t *key, int32_t *val, int64_t n, hipStream_t s) {
  if (n <= 1) return hipSuccess;
  if (n > kSmallSortKeys) return hipErrorInvalidValue;
  int np2 = 2;
  while (np2 < n) np2 <<= 1;
  k_sort_small<<<1, np2 / 2 < 1024 ? (np2 / 2 + 63) / 64 * 64 : 1024, 0, s>>>(key, val, (int)n,
                                                                             np2);
  return hipGetLastError();
}

}  // namespace zd
