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
