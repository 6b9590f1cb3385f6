"""Rotational mobility: the 6N product [U; w] = M [F; T] of Eq. (1) (oracle only).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Eq. (1) couples translational and rotational velocities (U, w) to forces and
torques (F, T) through the 6N x 6N mobility; the paper restricts itself to
translation and notes the extension (end of Sec. 2.2). The two-body blocks
here are the Rotne-Prager forms for spheres of radius a in a fluid of
viscosity mu, with r = x_i - x_j (target minus source), r_hat = r / |r|:

  M^tt_ij = the RPY tensor (kernels.rpy), self 1/(6 pi mu a) I;
  M^rt_ij = -1/(8 pi mu |r|^2) [r_hat]_x      (w_i from F_j: half the curl
            of the Stokeslet flow of F_j at x_i, i.e. F_j x r_hat / (8 pi mu |r|^2));
  M^tr_ij = (M^rt_ji)^T, which is the same matrix function of r;
  M^rr_ij = -1/(16 pi mu |r|^3) (I - 3 r_hat r_hat^T)   (half the curl of the
            rotlet flow of T_j), self 1/(8 pi mu a^3) I;
[v]_x is the cross-product matrix ([v]_x u = v x u). These are the
non-overlapping forms; they are used at every separation (the workloads keep
centres at least 2.05 a apart).

  U_i = a_t F_i + sum_{j != i} M^tt_ij F_j + M^tr_ij T_j
  w_i = a_r T_i + sum_{j != i} M^rt_ij F_j + M^rr_ij T_j
"""
from __future__ import annotations

import math

import numpy as np

from .kernels import rpy


def cross_matrix(v):
    """[..., 3] -> [..., 3, 3] with cross_matrix(v) @ u = v x u."""
    v = np.asarray(v, dtype=np.float64)
    z = np.zeros(v.shape[:-1])
    return np.stack([np.stack([z, -v[..., 2], v[..., 1]], -1),
                     np.stack([v[..., 2], z, -v[..., 0]], -1),
                     np.stack([-v[..., 1], v[..., 0], z], -1)], -2)


def coupling(r, mu: float = 1.0):
    """M^rt(r) = M^tr(r) = -[r_hat]_x / (8 pi mu |r|^2) for r = x_i - x_j."""
    r = np.asarray(r, dtype=np.float64)
    d = np.sqrt(np.sum(r * r, axis=-1))
    return -cross_matrix(r / d[..., None]) / (8.0 * math.pi * mu * d * d)[..., None, None]


def rotation(r, mu: float = 1.0):
    """M^rr(r) = -(I - 3 r_hat r_hat^T) / (16 pi mu |r|^3)."""
    r = np.asarray(r, dtype=np.float64)
    d = np.sqrt(np.sum(r * r, axis=-1))
    rh = r / d[..., None]
    out = np.eye(3) - 3.0 * rh[..., :, None] * rh[..., None, :]
    return -out / (16.0 * math.pi * mu * d ** 3)[..., None, None]


def self_rotation(a: float = 1.0, mu: float = 1.0) -> float:
    return 1.0 / (8.0 * math.pi * mu * a ** 3)


def u6(X, F, T, a: float = 1.0, mu: float = 1.0, rows=None):
    """(U, w) of the dense 6N product at the rows `rows` (all by default)."""
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    n = X.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    U = np.empty((rows.size, 3))
    W = np.empty((rows.size, 3))
    for a_, i in enumerate(rows):
        others = np.arange(n)
        others = others[others != i]
        r = X[i] - X[others]
        Ktt, Kc, Krr = rpy(r, a, mu), coupling(r, mu), rotation(r, mu)
        U[a_] = (F[i] / (6 * math.pi * mu * a) + np.einsum("pab,pb->a", Ktt, F[others]) +
                 np.einsum("pab,pb->a", Kc, T[others]))
        W[a_] = (self_rotation(a, mu) * T[i] + np.einsum("pab,pb->a", Kc, F[others]) +
                 np.einsum("pab,pb->a", Krr, T[others]))
    return U, W


def mobility6(X, a: float = 1.0, mu: float = 1.0):
    """The 6N x 6N matrix (small N), unknowns ordered (F_1..F_N, T_1..T_N)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    M = np.zeros((6 * n, 6 * n))
    for i in range(n):
        M[3 * i:3 * i + 3, 3 * i:3 * i + 3] = np.eye(3) / (6 * math.pi * mu * a)
        M[3 * n + 3 * i:3 * n + 3 * i + 3, 3 * n + 3 * i:3 * n + 3 * i + 3] = \
            self_rotation(a, mu) * np.eye(3)
        for j in range(n):
            if j == i:
                continue
            r = X[i] - X[j]
            M[3 * i:3 * i + 3, 3 * j:3 * j + 3] = rpy(r[None], a, mu)[0]
            M[3 * i:3 * i + 3, 3 * n + 3 * j:3 * n + 3 * j + 3] = coupling(r, mu)
            M[3 * n + 3 * i:3 * n + 3 * i + 3, 3 * j:3 * j + 3] = coupling(r, mu)
            M[3 * n + 3 * i:3 * n + 3 * i + 3, 3 * n + 3 * j:3 * n + 3 * j + 3] = rotation(r, mu)
    return M


# ------------------------------------------------------- the 6N H-matrix
#
# The H-matrix of Sec. 3 over the 6N mobility, read as the grid of 3x3
# entries that Eq. (1) describes: every particle contributes two rows
# (translation / force, then rotation / torque), so a cluster of m particles
# spans 2m rows, local row 2p + r being row r of its p-th particle in cluster
# order. The tree and the partition are those of the particles (Definition 1,
# Algorithm 1 with Eq. (7)); every admissible block is approximated by
# Algorithm 2 on its 2c x 2q entries. The translation-rotation entries are
# antisymmetric 3x3 matrices, hence singular, so the pivot magnitude is |det|
# (the reading of Eq. (9) that never picks a singular pivot).


def entry6(r, si: int, sj: int, a: float = 1.0, mu: float = 1.0):
    """3x3 entries of the rows of types si (0: U, 1: w) and columns sj (0: F,
    1: T) at displacements r [..., 3]."""
    if si == 0 and sj == 0:
        return rpy(r, a, mu)
    if si != sj:
        return coupling(r, mu)
    return rotation(r, mu)


def _gen_block(Xt, Xs, a, mu):
    """col(j) -> [2c, 3, 3] and row(i) -> [2q, 3, 3] of the block's 6N entries."""
    c, q = 2 * Xt.shape[0], 2 * Xs.shape[0]

    def col(j):
        out = np.empty((c, 3, 3))
        for s in (0, 1):
            out[s::2] = entry6(Xt - Xs[j // 2], s, j % 2, a, mu)
        return out

    def row(i):
        out = np.empty((q, 3, 3))
        for s in (0, 1):
            out[s::2] = entry6(Xt[i // 2] - Xs, i % 2, s, a, mu)
        return out

    return col, row, c, q


class HMatrix6:
    def __init__(self, tree, G, H, blocks, n_fallback, a, mu):
        self.tree, self.G, self.H = tree, G, H
        self.blocks = blocks            # ACAResult per admissible block, None for fallbacks
        self.n_fallback = n_fallback
        self.a, self.mu = a, mu


def build6(X, c_leaf, eta=1.0, eps=1e-6, l_max=48, a=1.0, mu=1.0, dense_mode=False,
           pivot="determinant"):
    from .aca import aca_entries
    from .partition import build_partition
    from .tree import build_tree
    X = np.asarray(X, dtype=np.float64)
    tree = build_tree(X, c_leaf)
    G, H = build_partition(tree, eta, dense_mode)
    Xs = X[tree.perm]
    blocks, nfb = [], 0
    for t, s in G:
        bt, et = tree.nodes[t, 0], tree.nodes[t, 1]
        bs, es = tree.nodes[s, 0], tree.nodes[s, 1]
        col, row, c, q = _gen_block(Xs[bt:et], Xs[bs:es], a, mu)
        res = aca_entries(col, row, c, q, eps, l_max, None, pivot)
        if not res.converged:
            res, nfb = None, nfb + 1
        blocks.append(res)
    return HMatrix6(tree, G, H, blocks, nfb, a, mu)


def _dense6(Xt, Xs, G6s, a, mu, diag: bool):
    """sum over the block's columns of the 6N entries times G6s [2q, 3]."""
    c = 2 * Xt.shape[0]
    out = np.zeros((c, 3))
    r = Xt[:, None, :] - Xs[None, :, :]
    if diag:
        eye = np.eye(Xt.shape[0], dtype=bool)
        r = np.where(eye[..., None], 1.0, r)
    for si in (0, 1):
        for sj in (0, 1):
            K = entry6(r, si, sj, a, mu)
            if diag:
                K[eye] = 0.0
            out[si::2] += np.einsum("ijab,jb->ia", K, G6s[sj::2])
    return out


def apply6(hm: HMatrix6, X, F, T):
    """(U, w) of the 6N H-matrix product in the input particle order."""
    from .aca import lowrank_apply
    X = np.asarray(X, dtype=np.float64)
    tree = hm.tree
    n = X.shape[0]
    Xs = X[tree.perm]
    G6 = np.empty((2 * n, 3))
    G6[0::2] = np.asarray(F, dtype=np.float64)[tree.perm]
    G6[1::2] = np.asarray(T, dtype=np.float64)[tree.perm]
    Y6 = np.zeros_like(G6)
    for t, s in hm.H:
        bt, et = tree.nodes[t, 0], tree.nodes[t, 1]
        bs, es = tree.nodes[s, 0], tree.nodes[s, 1]
        Y6[2 * bt:2 * et] += _dense6(Xs[bt:et], Xs[bs:es], G6[2 * bs:2 * es], hm.a, hm.mu, t == s)
    for (t, s), res in zip(hm.G, hm.blocks):
        bt, et = tree.nodes[t, 0], tree.nodes[t, 1]
        bs, es = tree.nodes[s, 0], tree.nodes[s, 1]
        if res is None:
            Y6[2 * bt:2 * et] += _dense6(Xs[bt:et], Xs[bs:es], G6[2 * bs:2 * es], hm.a, hm.mu,
                                         False)
        else:
            Y6[2 * bt:2 * et] += lowrank_apply(res, G6[2 * bs:2 * es])
    Y6[0::2] += G6[0::2] / (6.0 * math.pi * hm.mu * hm.a)
    Y6[1::2] += self_rotation(hm.a, hm.mu) * G6[1::2]
    U = np.empty((n, 3))
    W = np.empty((n, 3))
    U[tree.perm] = Y6[0::2]
    W[tree.perm] = Y6[1::2]
    return U, W
