// zd_persist_d3.hip -- the persistent forest kernel for 3-D clouds, one per k bucket.
#include "zd_persist_impl.h"

namespace zd {

hipError_t forest_persistent_d3(const PersistArgs &a, const PersistTree &pt, const TreeView &t,
                                hipStream_t s) {
  switch (k_bucket(a.k)) {
#define X(KK) \
  case KK: return launch_forest_persistent<3, KK>(a, pt, t, s);
    ZD_FOR_EACH_K(X)
#undef X
  }
  return hipErrorInvalidValue;
}

}  // namespace zd
