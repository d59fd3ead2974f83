// zd_scan.hip -- device memory, fills and the device-wide exclusive scan.
#include "zd_internal.h"

#include <cstdint>
#include <mutex>
#include <unordered_map>
#include <vector>

namespace zd {

// ---------------------------------------------------------------------------
// device memory: a caching allocator.  Released blocks are kept per device
// and handed out again to a request on the same stream whose size is within
// [need, need + need/4]; stream order then makes the reuse safe without
// events.  This keeps the runtime's allocator out of repeated builds and
// updates (its stream-ordered free costs about 0.2 ms per block here).
// Cached bytes per device are capped; beyond the cap, and when an
// allocation fails, cached blocks go back to the runtime (hipFree, which
// waits for the device).
// ---------------------------------------------------------------------------

namespace {

struct Block {
  void *p;
  size_t bytes;
  hipStream_t s;
  uint64_t tick;
};

struct DevCache {
  std::vector<Block> free;                   // released, reusable
  std::unordered_map<void *, size_t> live;   // handed out -> capacity
  size_t cached = 0;
  uint64_t tick = 0;
};

constexpr int kMaxDev = 64;
constexpr size_t kCacheCap = size_t(32) << 30;
std::mutex g_mu;
DevCache g_cache[kMaxDev];

size_t round_bytes(size_t b) {
  const size_t g = b <= (size_t(1) << 20) ? 256 : (size_t(1) << 20);
  return (b + g - 1) / g * g;
}

// evict until the cache holds at most `keep` bytes (caller holds g_mu)
void evict_locked(DevCache &c, size_t keep) {
  while (c.cached > keep && !c.free.empty()) {
    size_t oldest = 0;
    for (size_t i = 1; i < c.free.size(); ++i)
      if (c.free[i].tick < c.free[oldest].tick) oldest = i;
    const Block b = c.free[oldest];
    c.free[oldest] = c.free.back();
    c.free.pop_back();
    c.cached -= b.bytes;
    (void)hipFree(b.p);
  }
}

}  // namespace

static thread_local Arena *tl_arena = nullptr;

void arena_activate(Arena *a) { tl_arena = a; }

hipError_t dev_alloc(void **p, size_t bytes, hipStream_t s) {
  if (tl_arena) {
    const size_t off = (tl_arena->used + 255) & ~size_t(255);
    if (off + bytes > tl_arena->size) return hipErrorOutOfMemory;
    *p = tl_arena->base + off;
    tl_arena->used = off + bytes;
    return hipSuccess;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
  const size_t need = round_bytes(bytes);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    DevCache &c = g_cache[dev];
    size_t best = SIZE_MAX;
    for (size_t i = 0; i < c.free.size(); ++i) {
      const Block &b = c.free[i];
      if (b.s == s && b.bytes >= need && b.bytes <= need + need / 4 &&
          (best == SIZE_MAX || b.bytes < c.free[best].bytes))
        best = i;
    }
    if (best != SIZE_MAX) {
      const Block b = c.free[best];
      c.free[best] = c.free.back();
      c.free.pop_back();
      c.cached -= b.bytes;
      c.live[b.p] = b.bytes;
      *p = b.p;
      return hipSuccess;
    }
  }
  e = hipMalloc(p, need);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> lk(g_mu);
      evict_locked(g_cache[dev], 0);
    }
    e = hipMalloc(p, need);
  }
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[dev].live[*p] = need;
  return hipSuccess;
}

void dev_release(void *p, hipStream_t s) {
  if (!p) return;
  if (tl_arena && (char *)p >= tl_arena->base && (char *)p < tl_arena->base + tl_arena->size)
    return;
  std::lock_guard<std::mutex> lk(g_mu);
  for (int dev = 0; dev < kMaxDev; ++dev) {
    DevCache &c = g_cache[dev];
    auto it = c.live.find(p);
    if (it == c.live.end()) continue;
    const size_t bytes = it->second;
    c.live.erase(it);
    c.free.push_back(Block{p, bytes, s, c.tick++});
    c.cached += bytes;
    evict_locked(c, kCacheCap);
    return;
  }
}

int32_t *host_flag() {
  // a small pinned buffer per host thread for device-to-host status words
  static thread_local int32_t *buf = nullptr;
  if (!buf && hipHostMalloc(reinterpret_cast<void **>(&buf), 64, hipHostMallocDefault) != hipSuccess)
    buf = nullptr;
  return buf;
}

// ---------------------------------------------------------------------------
// fills
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_fill(T *p, T v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

static unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}

hipError_t fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill<int32_t><<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

hipError_t fill_f64(double *p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill<double><<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

__global__ void k_iota(int32_t *p, int32_t base, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = base + (int32_t)i;
}

hipError_t iota_i32(int32_t *p, int32_t base, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_iota<<<grid_for(n, 256), 256, 0, s>>>(p, base, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exclusive scan: reduce per block -> scan of block sums (recursive) ->
// per-block scan with the block offset.  4096 elements per 256-thread block.
// ---------------------------------------------------------------------------

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

// inclusive scan across a 64-wide wavefront
__device__ __forceinline__ int32_t wave_inclusive_scan(int32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int32_t t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread; returns the exclusive
// prefix and writes the block total to *total.
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t *total) {
  __shared__ int32_t wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t inc = wave_inclusive_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int32_t before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kScanThreads / 64; ++i) {
    int32_t x = wsum[i];
    if (i < w) before += x;
    all += x;
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const int32_t *in, int64_t n,
                                                              int32_t *sums) {
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int32_t acc = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + (int64_t)j * kScanThreads + threadIdx.x;
    if (i < n) acc += in[i];
  }
  int32_t total;
  (void)block_exclusive_scan(acc, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// The tile passes through LDS twice so that global loads and stores are
// coalesced while each thread scans kScanItems consecutive entries (one
// padding slot per 32 entries keeps the strided LDS accesses conflict-free).
__device__ __forceinline__ int scan_slot(int idx) { return idx + (idx >> 5); }

__global__ void __launch_bounds__(kScanThreads) k_scan_down(const int32_t *in, int32_t *out,
                                                            int64_t n, const int32_t *offsets,
                                                            int32_t *total_out) {
  __shared__ int32_t tile[kScanTile + kScanTile / 32];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int idx = j * kScanThreads + threadIdx.x;
    tile[scan_slot(idx)] = base + idx < n ? in[base + idx] : 0;
  }
  __syncthreads();
  int32_t v[kScanItems];
  int32_t acc = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = tile[scan_slot(threadIdx.x * kScanItems + j)];
    acc += v[j];
  }
  int32_t total;
  int32_t run = block_exclusive_scan(acc, &total) + (offsets ? offsets[blockIdx.x] : 0);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    tile[scan_slot(threadIdx.x * kScanItems + j)] = run;
    run += v[j];
  }
  if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1)
    *total_out = run;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int idx = j * kScanThreads + threadIdx.x;
    if (base + idx < n) out[base + idx] = tile[scan_slot(idx)];
  }
}

hipError_t exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total,
                              hipStream_t s) {
  if (n <= 0) {
    if (total) return fill_i32(total, 0, 1, s);
    return hipSuccess;
  }
  int64_t nblk = (n + kScanTile - 1) / kScanTile;
  if (nblk == 1) {
    k_scan_down<<<1, kScanThreads, 0, s>>>(in, out, n, nullptr, total);
    return hipGetLastError();
  }
  int32_t *sums = nullptr;
  hipError_t e = dev_alloc_n(&sums, nblk, s);
  if (e != hipSuccess) return e;
  k_scan_reduce<<<(unsigned)nblk, kScanThreads, 0, s>>>(in, n, sums);
  e = hipGetLastError();
  if (e == hipSuccess) e = exclusive_scan_i32(sums, sums, nblk, nullptr, s);
  if (e == hipSuccess) {
    k_scan_down<<<(unsigned)nblk, kScanThreads, 0, s>>>(in, out, n, sums, total);
    e = hipGetLastError();
  }
  dev_release(sums, s);
  return e;
}

}  // namespace zd
