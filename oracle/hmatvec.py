"""The H-matrix mobility product, assembled step by step (oracle only).

Paper reference: Sec. 3. M^(t,2) is split into admissible blocks P^G
(Algorithm 1), each approximated by ACA (Algorithm 2) and applied as C (Q F)
(Sec. 3, low-rank product), and inadmissible leaf blocks P^H, evaluated
densely (Sec. 3.3.1). The one-body term M^(1) F is diagonal (Eq. (6)).

  U = alpha_1 F + sum_{(tau,sigma) in P^H} H F_sigma (j != i)
                + sum_{(tau,sigma) in P^G} C (Q F_sigma)

Blocks whose ACA falls back (see aca.py) are applied densely. The relative
error of Eq. (11) is provided as `eps_r`.
"""
from __future__ import annotations

import numpy as np

from .aca import aca_block, lowrank_apply
from .partition import build_partition
from .tree import build_tree


class HMatrix:
    def __init__(self, tree, G, H, blocks, n_fallback):
        self.tree, self.G, self.H = tree, G, H
        self.blocks = blocks            # list of ACAResult (None for fallbacks)
        self.n_fallback = n_fallback


def build(X, kern, c_leaf, eta=1.0, eps=1e-6, l_max=48, dense_mode=False, tree=None, part=None,
          pivot="frobenius"):
    X = np.asarray(X, dtype=np.float64)
    if tree is None:
        tree = build_tree(X, c_leaf)
    if part is None:
        G, H = build_partition(tree, eta, dense_mode)
    else:
        G, H = part
    Xs = X[tree.perm]
    blocks = []
    nfb = 0
    for t, s in G:
        bt, et = tree.nodes[t, 0], tree.nodes[t, 1]
        bs, es = tree.nodes[s, 0], tree.nodes[s, 1]
        res = aca_block(kern, Xs[bt:et], Xs[bs:es], eps, l_max, pivot=pivot)
        if not res.converged:
            res = None
            nfb += 1
        blocks.append(res)
    return HMatrix(tree, G, H, blocks, nfb)


def _dense_block(kern, Xt, Xs, Fs, diag: bool):
    r = Xt[:, None, :] - Xs[None, :, :]
    if diag:
        n = Xt.shape[0]
        eye = np.eye(n, dtype=bool)
        r = np.where(eye[..., None], 1.0, r)
        K = kern(r)
        K[eye] = 0.0
    else:
        K = kern(r)
    return np.einsum("ijab,jb->ia", K, Fs)


def apply(hm: HMatrix, X, F, kern, two_body_only: bool = False):
    """U in the input particle order."""
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    tree = hm.tree
    Xs = X[tree.perm]
    Fs = F[tree.perm]
    Us = np.zeros_like(Fs)
    for t, s in hm.H:
        bt, et = tree.nodes[t, 0], tree.nodes[t, 1]
        bs, es = tree.nodes[s, 0], tree.nodes[s, 1]
        Us[bt:et] += _dense_block(kern, Xs[bt:et], Xs[bs:es], Fs[bs:es], t == s)
    for (t, s), res in zip(hm.G, hm.blocks):
        bt, et = tree.nodes[t, 0], tree.nodes[t, 1]
        bs, es = tree.nodes[s, 0], tree.nodes[s, 1]
        if res is None:
            Us[bt:et] += _dense_block(kern, Xs[bt:et], Xs[bs:es], Fs[bs:es], False)
        else:
            Us[bt:et] += lowrank_apply(res, Fs[bs:es])
    if not two_body_only:
        Us += kern.alpha1 * Fs
    U = np.empty_like(Us)
    U[tree.perm] = Us
    return U


def hmatvec(X, F, kern, c_leaf, eta=1.0, eps=1e-6, l_max=48, dense_mode=False):
    hm = build(X, kern, c_leaf, eta, eps, l_max, dense_mode)
    return apply(hm, X, F, kern), hm


def eps_r(u_h, u_ref):
    """Eq. (11): ||u_ref - u_h||_2 / ||u_ref||_2 over all 3N components."""
    u_h = np.asarray(u_h, dtype=np.float64)
    u_ref = np.asarray(u_ref, dtype=np.float64)
    return float(np.linalg.norm(u_ref - u_h) / np.linalg.norm(u_ref))
