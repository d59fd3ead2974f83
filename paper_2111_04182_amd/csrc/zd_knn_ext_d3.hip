// zd_knn_ext_d3.hip -- external-query search kernels for 3-D trees, one per k bucket.
#include "zd_knn_impl.h"

namespace zd {

hipError_t knn_ext_d3(const TreeView &t, const double *q, int64_t qs, const uint64_t *qkey,
                      const int32_t *order, int64_t m, int k, int32_t *ids, double *d2,
                      const int32_t *row_ids, hipStream_t s, int query_waves) {
  switch (k_bucket(k)) {
#define X(KK) \
  case KK: return launch_knn_ext<3, KK>(t, q, qs, qkey, order, m, k, ids, d2, row_ids, s, query_waves);
    ZD_FOR_EACH_K(X)
#undef X
  }
  return hipErrorInvalidValue;
}

}  // namespace zd
