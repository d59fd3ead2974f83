// zd_knn_all_d2.hip -- all-points search kernels for 2-D trees, one per k bucket.
#include "zd_knn_impl.h"

namespace zd {

hipError_t knn_all_d2(const TreeView &t, int k, int32_t *ids, double *d2, hipStream_t s,
                      const int4 *groups, int64_t ngroups, int query_waves) {
  switch (k_bucket(k)) {
#define X(KK) \
  case KK: return launch_knn_all<2, KK>(t, k, ids, d2, s, groups, ngroups, query_waves);
    ZD_FOR_EACH_K(X)
#undef X
  }
  return hipErrorInvalidValue;
}

}  // namespace zd
