// zd_scan.hip -- device memory, fills and the device-wide exclusive scan.
#include "zd_internal.h"

#include <mutex>

namespace zd {

// ---------------------------------------------------------------------------
// stream-ordered allocation from the device's default memory pool; the pool
// keeps freed blocks (release threshold = max), so repeated builds and
// queries do not return to the driver.
// ---------------------------------------------------------------------------

static std::once_flag g_pool_once[64];

static void configure_pool(int dev) {
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
}

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
  if (dev >= 0 && dev < 64) std::call_once(g_pool_once[dev], configure_pool, dev);
  return hipMallocAsync(p, bytes, s);
}

void dev_release(void *p, hipStream_t s) {
  if (!p) return;
  if (tl_arena && (char *)p >= tl_arena->base && (char *)p < tl_arena->base + tl_arena->size)
    return;
  (void)hipFreeAsync(p, s);
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

__global__ void __launch_bounds__(kScanThreads) k_scan_down(const int32_t *in, int32_t *out,
                                                            int64_t n, const int32_t *offsets,
                                                            int32_t *total_out) {
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int32_t acc = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + j;
    v[j] = i < n ? in[i] : 0;
    acc += v[j];
  }
  int32_t total;
  int32_t run = block_exclusive_scan(acc, &total) + (offsets ? offsets[blockIdx.x] : 0);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + j;
    if (i < n) out[i] = run;
    run += v[j];
  }
  if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1)
    *total_out = run;
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
