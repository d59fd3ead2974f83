// zd_persist_d2.hip -- the persistent forest kernel for 2-D clouds, one per k bucket.
#include "zd_persist_impl.h"

namespace zd {

hipError_t forest_persistent_d2(const PersistArgs &a, const PersistTree &pt, const TreeView &t,
                                hipStream_t s) {
  switch (k_bucket(a.k)) {
#define X(KK) \
  case KK: return launch_forest_persistent<2, KK>(a, pt, t, s);
    ZD_FOR_EACH_K(X)
#undef X
  }
  return hipErrorInvalidValue;
}

}  // namespace zd
