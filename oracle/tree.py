"""Cluster tree by literal recursive bisection (oracle only).

Paper reference: Definition 1 (Sec. 3.1) -- every non-leaf cluster is the
disjoint union of two sons and a leaf holds fewer than C_leaf indices; the
clusters come from geometric bisection of bounding boxes, first along x, then
along y (and z in 3-D), as Fig. 2 shows.

Readings where the paper is silent (each listed in the design notes):
  * the root box is a cube of power-of-two edge 2^e > the largest extent of the
    centres, anchored at their per-axis minimum; boxes are halved at their
    midpoint, cycling x -> y -> z. With 21 levels per axis this is exactly one
    bit of a 21-bit quantised coordinate per split;
  * a split that leaves one half empty creates no node: bisection continues on
    the next axis;
  * a cluster that cannot be split any further (all quantised coordinates
    equal) becomes a forced leaf even if it holds C_leaf or more indices;
  * inside a leaf, indices are ordered by (Morton key, original index);
  * nodes are numbered in pre-order (a node, then its low half, then its high
    half), and every node covers a contiguous range [begin, end) of the
    resulting particle order.

Quantisation: lo_d = min_i x_id; E = max_d (max_i x_id - lo_d) in FP64;
e = the smallest integer with 2^e > E; q_id = floor((x_id - lo_d) * 2^(21-e)),
capped at 2^21 - 1. Every step is exact except the correctly rounded
subtraction.
"""
from __future__ import annotations

import math

import numpy as np

BITS = 21


def quantize(X):
    """Quantised coordinates q [N, 3] (int64) of the centres."""
    X = np.asarray(X, dtype=np.float64)
    lo = X.min(axis=0)
    hi = X.max(axis=0)
    E = max(float(hi[0] - lo[0]), float(hi[1] - lo[1]), float(hi[2] - lo[2]))
    if E > 0.0:
        _, e = math.frexp(E)          # E = m 2^e with m in [0.5, 1): 2^(e-1) <= E < 2^e
    else:
        e = 0
    q = np.floor(np.ldexp(X - lo, BITS - e)).astype(np.int64)
    return np.minimum(q, (1 << BITS) - 1)


def morton_keys(q):
    """63-bit Morton keys: bit 3k+2 is bit k of q_x, 3k+1 of q_y, 3k of q_z."""
    q = np.asarray(q, dtype=np.int64)
    key = np.zeros(q.shape[0], dtype=np.uint64)
    for k in range(BITS):
        for d in range(3):
            bit = ((q[:, d] >> k) & 1).astype(np.uint64)
            key |= bit << np.uint64(3 * k + (2 - d))
    return key


class Tree:
    """perm[s] = original index at sorted position s; keys[s] its Morton key;
    nodes[n] = (begin, end, left, right) with -1 children for leaves;
    bbox[n] = (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z) of the member centres."""

    def __init__(self, perm, keys, nodes, bbox, c_leaf):
        self.perm = perm
        self.keys = keys
        self.nodes = nodes
        self.bbox = bbox
        self.c_leaf = c_leaf

    @property
    def n_nodes(self):
        return self.nodes.shape[0]

    def is_leaf(self, n):
        return self.nodes[n, 2] < 0

    def sons(self, n):
        return int(self.nodes[n, 2]), int(self.nodes[n, 3])

    def size(self, n):
        return int(self.nodes[n, 1] - self.nodes[n, 0])

    def leaves(self):
        return np.nonzero(self.nodes[:, 2] < 0)[0]


def build_tree(X, c_leaf: int) -> Tree:
    """Literal top-down bisection (Definition 1 with the readings above)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    assert n >= 1 and c_leaf >= 2
    q = quantize(X)
    keys = morton_keys(q)
    nodes = []      # (begin, end, left, right), filled in pre-order
    order = []      # particle order, leaves appended left to right

    def rec(idx, b):
        me = len(nodes)
        nodes.append([len(order), -1, -1, -1])
        split = None
        if idx.size >= c_leaf:
            bb = b
            while bb >= 0:
                d = 2 - bb % 3            # bit 3k+2 -> x, 3k+1 -> y, 3k -> z
                bit = (q[idx, d] >> (bb // 3)) & 1
                nz = int(bit.sum())
                if 0 < nz < idx.size:
                    split = (bb, bit)
                    break
                bb -= 1
        if split is None:                  # leaf (regular or forced)
            o = np.lexsort((idx, keys[idx]))
            order.extend(idx[o].tolist())
        else:
            bb, bit = split
            lo_idx = idx[bit == 0]
            hi_idx = idx[bit == 1]
            nodes[me][2] = rec(lo_idx, bb - 1)
            nodes[me][3] = rec(hi_idx, bb - 1)
        nodes[me][1] = len(order)
        return me

    rec(np.arange(n, dtype=np.int64), 3 * BITS - 1)
    perm = np.asarray(order, dtype=np.int64)
    nodes = np.asarray(nodes, dtype=np.int64)
    Xs = X[perm]
    bbox = np.empty((nodes.shape[0], 6))
    for t in range(nodes.shape[0]):
        m = Xs[nodes[t, 0]:nodes[t, 1]]
        bbox[t, :3] = m.min(axis=0)
        bbox[t, 3:] = m.max(axis=0)
    return Tree(perm, keys[perm], nodes, bbox, c_leaf)
