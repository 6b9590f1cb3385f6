"""BuildPartition, Algorithm 1, with the admissibility condition Eq. (7).

Paper reference: Sec. 3.1, Definition 2 / Eq. (7): a block (tau, sigma) is
admissible when max{diam(tau), diam(sigma)} <= eta dist(tau, sigma), eta > 0,
with diam and dist approximated on bounding boxes (Fig. 3b). Algorithm 1
starts at (I, I): an admissible block goes to P^G; otherwise a pair of leaves
goes to P^H; otherwise the block is split into the sons of the non-leaf
side(s) and each son block is visited recursively.

Readings (listed in the design notes):
  * bounding boxes are the tight boxes of the member centres; diam is the box
    diagonal, dist the Euclidean gap between the boxes (0 if they touch or
    overlap);
  * the test is evaluated on squares without fused multiply-add, in a fixed
    order: diam^2 = (dx*dx + dy*dy) + dz*dz, dist^2 likewise over the per-axis
    gaps g_d = max(0, lo_sigma - hi_tau, lo_tau - hi_sigma); admissible iff
    dist^2 > 0 and max(diam_tau^2, diam_sigma^2) <= (eta*eta) * dist^2;
  * "leaf" is the tree's leaf flag (covers clusters that cannot be split);
  * the output lists are sorted by (tau, sigma) node id.
"""
from __future__ import annotations

import numpy as np


def diam2(bb):
    dx = float(bb[3]) - float(bb[0])
    dy = float(bb[4]) - float(bb[1])
    dz = float(bb[5]) - float(bb[2])
    return (dx * dx + dy * dy) + dz * dz


def dist2(bt, bs):
    g = []
    for d in range(3):
        a = float(bs[d]) - float(bt[d + 3])
        b = float(bt[d]) - float(bs[d + 3])
        g.append(max(0.0, a, b))
    return (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2]


def admissible(bt, bs, eta: float) -> bool:
    d2 = dist2(bt, bs)
    if not d2 > 0.0:
        return False
    return max(diam2(bt), diam2(bs)) <= (eta * eta) * d2


def build_partition(tree, eta: float = 1.0, dense_mode: bool = False):
    """Returns (G, H): int64 arrays [nG, 2] and [nH, 2] of (tau, sigma) node ids.

    dense_mode treats no block as admissible (every leaf pair is near), which
    makes the H-matrix product equal to the dense one.
    """
    assert eta > 0.0
    G, H = [], []
    stack = [(0, 0)]
    while stack:
        t, s = stack.pop()
        if not dense_mode and admissible(tree.bbox[t], tree.bbox[s], eta):
            G.append((t, s))
            continue
        lt, ls = tree.is_leaf(t), tree.is_leaf(s)
        if lt and ls:
            H.append((t, s))
            continue
        if ls:
            kids = [(t2, s) for t2 in tree.sons(t)]
        elif lt:
            kids = [(t, s2) for s2 in tree.sons(s)]
        else:
            kids = [(t2, s2) for t2 in tree.sons(t) for s2 in tree.sons(s)]
        stack.extend(reversed(kids))
    G = np.asarray(sorted(G), dtype=np.int64).reshape(-1, 2)
    H = np.asarray(sorted(H), dtype=np.int64).reshape(-1, 2)
    return G, H
