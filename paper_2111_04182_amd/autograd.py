"""Differentiable k-NN squared distances.

``ZdKnnSqDist.apply(xyz, tree, k)`` returns (d2, ids) for the all-points
k-NN rows of ``tree``; d2 is differentiable with respect to the SoA point
tensor ``xyz`` (d, cap), which must hold the tree's points by id.  The
neighbour set is chosen exactly and held fixed: the backward pass is the
library's scatter-add kernel,
    dL/dp += 2 (p - q) g,   dL/dq -= 2 (p - q) g,
for every row p, neighbour q and upstream gradient g: in the tree's Morton
order (zd_knn_backward_tree) when the tree is unchanged since the forward
pass, else over the rows in id order (zd_knn_backward), or without atomics
in a fixed order when deterministic=True (zd_knn_backward_det).  Selection itself is not
differentiated, as usual for nearest-neighbour losses.
"""
from __future__ import annotations

import torch

from ._lib import ZdTree, zd_knn_backward


class ZdKnnSqDist(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xyz: torch.Tensor, tree: ZdTree, k: int, deterministic: bool = False):
        ids, d2 = tree.knn(k)
        ctx.save_for_backward(xyz, ids)
        ctx.mark_non_differentiable(ids)
        ctx.deterministic = deterministic
        ctx.tree = tree
        ctx.version = tree.version
        return d2, ids

    @staticmethod
    def backward(ctx, grad_d2, grad_ids):
        xyz, ids = ctx.saved_tensors
        g = torch.zeros(ids.shape, dtype=torch.float64, device=xyz.device) if grad_d2 is None \
            else grad_d2.contiguous()
        tree = ctx.tree
        if (not ctx.deterministic and tree.handle is not None and tree.version == ctx.version
                and tree.cap == xyz.shape[1]):
            grad = tree.knn_backward(ids, g)
        else:
            grad = zd_knn_backward(xyz.detach(), ids, g, deterministic=ctx.deterministic)
        return grad, None, None, None


def knn_sq_dist(xyz: torch.Tensor, tree: ZdTree, k: int, deterministic: bool = False):
    """Functional form of ZdKnnSqDist.  deterministic=True makes the backward
    sum in a fixed order without atomics (the same bits on every run)."""
    return ZdKnnSqDist.apply(xyz, tree, k, deterministic)
