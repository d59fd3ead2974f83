// zd_grad.hip -- backward of the k-NN squared distances.
//
// For a fixed neighbour table the loss L = sum_{r,j} g[r][j] * d2(p_r, p_q),
// q = ids[r][j], is quadratic in the coordinates:
//   dL/dp_r += 2 (p_r - p_q) g,   dL/dp_q -= 2 (p_r - p_q) g.
// One thread per (row, slot) forms the term once and scatter-adds it to both
// endpoints with hardware FP64 atomics.  Neighbour selection is untouched.
#include "zd_internal.h"

namespace zd {

template <int D>
__global__ void k_knn_backward(const double *__restrict__ xyz, int64_t stride, int64_t rows,
                               int k, const int32_t *__restrict__ ids,
                               const double *__restrict__ g, double *grad) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * k) return;
  const int32_t q = ids[e];
  if (q < 0 || q >= stride) return;
  const int64_t r = e / k;
  const double w = g[e];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    double t = 2.0 * (xyz[c * stride + r] - xyz[c * stride + q]) * w;
    unsafeAtomicAdd(&grad[c * stride + r], t);
    unsafeAtomicAdd(&grad[c * stride + q], -t);
  }
}

hipError_t knn_backward(int dim, const double *xyz, int64_t stride, int64_t rows, int k,
                        const int32_t *ids, const double *g, double *grad, hipStream_t s) {
  hipError_t e = fill_f64(grad, 0.0, (int64_t)dim * stride, s);
  if (e != hipSuccess || rows <= 0) return e;
  const int64_t total = rows * k;
  unsigned grid = (unsigned)((total + 255) / 256);
  if (dim == 3) k_knn_backward<3><<<grid, 256, 0, s>>>(xyz, stride, rows, k, ids, g, grad);
  else k_knn_backward<2><<<grid, 256, 0, s>>>(xyz, stride, rows, k, ids, g, grad);
  return hipGetLastError();
}

}  // namespace zd
