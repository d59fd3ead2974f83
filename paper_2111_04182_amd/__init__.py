"""zd-tree exact k-nearest neighbours on MI355X (gfx950).

The compute path is libzd.so (hand-written HIP kernels behind the C ABI in
include/zd.h); this package is its thin binding.  PyTorch provides device
memory and streams only.
"""
from ._lib import (ZD_KMAX, ZdError, ZdForest, ZdForestPlan, ZdTree, lib, soa, zd_build,
                   zd_check, zd_delete_batch, zd_export, zd_forest_build, zd_forest_free, zd_forest_knn,
                   zd_forest_plan, zd_forest_plan_persistent, zd_forest_run, zd_free, zd_info, zd_insert_batch, zd_knn,
                   zd_knn_backward, zd_knn_backward_tree, zd_knn_root, zd_set_walk_limit)
from .autograd import ZdKnnSqDist, knn_sq_dist

__all__ = ["ZD_KMAX", "ZdError", "ZdForest", "ZdForestPlan", "ZdTree", "ZdKnnSqDist",
           "knn_sq_dist", "lib", "soa", "zd_build", "zd_check", "zd_delete_batch", "zd_export",
           "zd_forest_build", "zd_forest_free", "zd_forest_knn", "zd_forest_plan",
           "zd_forest_plan_persistent",
           "zd_forest_run", "zd_free", "zd_info", "zd_insert_batch", "zd_knn",
           "zd_knn_backward", "zd_knn_backward_tree", "zd_knn_root", "zd_set_walk_limit"]
