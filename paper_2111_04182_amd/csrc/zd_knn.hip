// zd_knn.hip -- host side of the k-NN queries: kernel choice per dimension
// and k, the Morton presort of external queries (Section 3.1), the
// root-based variant, and the padding of rows that belong to deleted ids.  The search kernels themselves
// are in zd_knn_impl.h.
#include "zd_internal.h"

namespace zd {

hipError_t knn_all_d2(const TreeView &t, int k, int32_t *ids, double *d2, hipStream_t s,
                      const int4 *groups, int64_t ngroups, int query_waves);
hipError_t knn_all_d3(const TreeView &t, int k, int32_t *ids, double *d2, hipStream_t s,
                      const int4 *groups, int64_t ngroups, int query_waves);
hipError_t knn_ext_d2(const TreeView &t, const double *q, int64_t qs, const uint64_t *qkey,
                      const int32_t *order, int64_t m, int k, int32_t *ids, double *d2,
                      const int32_t *row_ids, hipStream_t s, int query_waves);
hipError_t knn_ext_d3(const TreeView &t, const double *q, int64_t qs, const uint64_t *qkey,
                      const int32_t *order, int64_t m, int k, int32_t *ids, double *d2,
                      const int32_t *row_ids, hipStream_t s, int query_waves);

hipError_t knn_root_d2(const TreeView &t, const double *q, int64_t qs, const uint64_t *qkey,
                       const int32_t *order, int64_t m, int k, int32_t *ids, double *d2,
                       const int32_t *row_ids, hipStream_t s, int query_waves);
hipError_t knn_root_d3(const TreeView &t, const double *q, int64_t qs, const uint64_t *qkey,
                       const int32_t *order, int64_t m, int k, int32_t *ids, double *d2,
                       const int32_t *row_ids, hipStream_t s, int query_waves);

hipError_t knn_all_points(int dim, const TreeView &t, int k, int32_t *out_ids, double *out_d2,
                          hipStream_t s, int query_waves, const int4 *groups, int64_t ngroups) {
  if (t.n <= 0 || (groups && ngroups <= 0)) return hipSuccess;
  return dim == 3 ? knn_all_d3(t, k, out_ids, out_d2, s, groups, ngroups, query_waves)
                  : knn_all_d2(t, k, out_ids, out_d2, s, groups, ngroups, query_waves);
}

// External queries are sorted by their Morton keys so that a wavefront's 64
// queries are neighbours in space (Section 3.1); rows are still written in
// query order (or at row_ids[query], for the tree's own pool entries).
// `root` selects the root-based start instead of the bit-based descent.
static hipError_t knn_presorted(int dim, const TreeView &t, const Geometry &g, const double *q,
                                int64_t qs, int64_t m, int k, int32_t *out_ids, double *out_d2,
                                const int32_t *row_ids, hipStream_t s, int query_waves,
                                bool root) {
  uint64_t *key = nullptr, *key_tmp = nullptr;
  int32_t *order = nullptr, *order_tmp = nullptr;
  hipError_t e = dev_alloc_n(&key, m, s);
  if (e == hipSuccess) e = dev_alloc_n(&order, m, s);
  if (e == hipSuccess) e = dev_alloc_n(&key_tmp, m, s);
  if (e == hipSuccess) e = dev_alloc_n(&order_tmp, m, s);
  if (e == hipSuccess) e = encode_keys(g, q, qs, m, 0, key, order, s);
  if (e == hipSuccess) e = radix_sort_pairs(key, order, key_tmp, order_tmp, m, dim * g.B, s);
  if (e == hipSuccess) {
    if (root)
      e = dim == 3 ? knn_root_d3(t, q, qs, key, order, m, k, out_ids, out_d2, row_ids, s,
                                 query_waves)
                   : knn_root_d2(t, q, qs, key, order, m, k, out_ids, out_d2, row_ids, s,
                                 query_waves);
    else
      e = dim == 3 ? knn_ext_d3(t, q, qs, key, order, m, k, out_ids, out_d2, row_ids, s,
                                query_waves)
                   : knn_ext_d2(t, q, qs, key, order, m, k, out_ids, out_d2, row_ids, s,
                                query_waves);
  }
  dev_release(key, s);
  dev_release(order, s);
  dev_release(key_tmp, s);
  dev_release(order_tmp, s);
  return e;
}

hipError_t knn_external(int dim, const TreeView &t, const Geometry &g, const double *q,
                        int64_t m, int k, int32_t *out_ids, double *out_d2, hipStream_t s,
                        int query_waves) {
  if (m <= 0) return hipSuccess;
  return knn_presorted(dim, t, g, q, m, m, k, out_ids, out_d2, nullptr, s, query_waves, false);
}

hipError_t knn_root_based(int dim, const TreeView &t, const Geometry &g, const double *q,
                          int64_t m, int k, int32_t *out_ids, double *out_d2, hipStream_t s,
                          int query_waves) {
  if (q) {
    if (m <= 0) return hipSuccess;
    return knn_presorted(dim, t, g, q, m, m, k, out_ids, out_d2, nullptr, s, query_waves, true);
  }
  if (t.n <= 0) return hipSuccess;
  return dim == 3 ? knn_root_d3(t, nullptr, 0, nullptr, nullptr, t.n, k, out_ids, out_d2,
                                nullptr, s, query_waves)
                  : knn_root_d2(t, nullptr, 0, nullptr, nullptr, t.n, k, out_ids, out_d2,
                                nullptr, s, query_waves);
}

hipError_t knn_pool_rows(int dim, const TreeView &t, const Geometry &g, const double *pxyz,
                         int64_t pstride, const int32_t *pid, int64_t m, int k, int32_t *out_ids,
                         double *out_d2, hipStream_t s, int query_waves, bool root) {
  if (m <= 0) return hipSuccess;
  return knn_presorted(dim, t, g, pxyz, pstride, m, k, out_ids, out_d2, pid, s, query_waves,
                       root);
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

}  // namespace zd
