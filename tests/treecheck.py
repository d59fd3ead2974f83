"""Structural checks of an exported zd-tree (in-order canonical form).

The export lists the live (key, id) pairs in tree order, the size and box of
every leaf, and the split bit and box of every internal node, in order.  In a
full binary tree the in-order sequence alternates leaf, internal, ..., leaf, and
a node's range is the maximal run of leaves around it whose internal nodes have
smaller bits; these checks rebuild that structure and test the zd-tree's
defining properties (paper Section 2, "Data structure", and Algorithm 1).
"""
import numpy as np


def node_ranges(bits):
    """For each internal node i (between leaf i and leaf i+1), the leaf range
    [a, b] of its subtree: the nearest internal nodes with a larger bit to the
    left and right bound it (a Cartesian tree on the bits)."""
    ni = len(bits)
    left = np.zeros(ni, dtype=np.int64)
    right = np.zeros(ni, dtype=np.int64)
    st = []
    for i in range(ni):
        while st and bits[st[-1]] < bits[i]:
            st.pop()
        left[i] = st[-1] + 1 if st else 0
        st.append(i)
    st = []
    for i in range(ni - 1, -1, -1):
        while st and bits[st[-1]] < bits[i]:
            st.pop()
        right[i] = st[-1] if st else ni
        st.append(i)
    return left, right


def check_tree(ex, pts, L, live_ids=None):
    """Assert the zd-tree invariants on an export dict.

    pts: (cap, d) points by id.  live_ids: ids that must be present (default
    all)."""
    keys = np.asarray(ex["keys"], dtype=np.uint64)
    ids = np.asarray(ex["ids"], dtype=np.int64)
    cnt = np.asarray(ex["leaf_count"], dtype=np.int64)
    bits = np.asarray(ex["int_bit"], dtype=np.int64)
    d = pts.shape[1]
    n = keys.shape[0]
    if live_ids is None:
        live_ids = np.arange(pts.shape[0])
    # every live point in exactly one leaf
    assert np.array_equal(np.sort(ids), np.sort(np.asarray(live_ids))), "ids are not the live set"
    if n == 0:
        assert len(cnt) == 0 and len(bits) == 0
        return
    assert len(cnt) == len(bits) + 1, "a full binary tree has one more leaf than internal nodes"
    assert cnt.sum() == n and (cnt >= 1).all(), "leaf sizes must partition the points, no empty leaf"
    # Morton order: keys ascending, equal keys by ascending id
    assert (keys[1:] >= keys[:-1]).all(), "keys not sorted"
    eq = keys[1:] == keys[:-1]
    assert (ids[1:][eq] > ids[:-1][eq]).all(), "equal keys not in id order"
    starts = np.concatenate([[0], np.cumsum(cnt)])
    P = pts[ids]
    # leaves: at most L points unless every key is equal; tight boxes
    for j in range(len(cnt)):
        a, b = starts[j], starts[j + 1]
        if b - a > L:
            assert keys[a] == keys[b - 1], f"leaf {j} oversized with distinct keys"
        assert np.array_equal(ex["leaf_lo"][j], P[a:b].min(axis=0)), f"leaf {j} lo"
        assert np.array_equal(ex["leaf_hi"][j], P[a:b].max(axis=0)), f"leaf {j} hi"
    # internal nodes: more than L points, distinct keys, split on their bit
    lr, rr = node_ranges(bits)
    for i in range(len(bits)):
        a, m, b = starts[lr[i]], starts[i + 1], starts[rr[i] + 1]
        assert b - a > L, f"internal node {i} has only {b - a} points"
        x = int(keys[a]) ^ int(keys[b - 1])
        assert x != 0 and x.bit_length() - 1 == bits[i], f"node {i} bit is not the highest differing bit"
        bi = int(bits[i])
        kk = keys[a:b]
        assert ((kk[: m - a] >> np.uint64(bi)) & np.uint64(1) == 0).all(), f"node {i} left side"
        assert ((kk[m - a:] >> np.uint64(bi)) & np.uint64(1) == 1).all(), f"node {i} right side"
        assert np.array_equal(ex["int_lo"][i], P[a:b].min(axis=0)), f"node {i} lo"
        assert np.array_equal(ex["int_hi"][i], P[a:b].max(axis=0)), f"node {i} hi"
    return lr, rr


def tree_depth(bits):
    """Depth (edges root -> deepest leaf) of the tree given by in-order bits."""
    ni = len(bits)
    if ni == 0:
        return 0
    lr, rr = node_ranges(np.asarray(bits))
    # parent of internal i: the smaller-bit of its two bounding internal nodes
    depth = np.zeros(ni, dtype=np.int64)
    order = np.argsort(-np.asarray(bits), kind="stable")
    parent = np.full(ni, -1)
    for i in range(ni):
        cands = []
        if lr[i] > 0:
            cands.append(lr[i] - 1)
        if rr[i] < ni:
            cands.append(rr[i])
        if cands:
            parent[i] = min(cands, key=lambda c: bits[c])
    for i in order:
        depth[i] = 0 if parent[i] < 0 else depth[parent[i]] + 1
    return int(depth.max()) + 1
