"""Dense FP64 gradients of L = sum_i w_i . U_i (oracle only).

U is the dense product of dense.py (Eq. (2) restricted to alpha_1 and the
two-body term). Gradients, by the chain rule written out by hand:

  dL/dF_j = alpha_1 w_j + sum_{i != j} K(x_i - x_j)^T w_i

For a pair (i, j) with r = x_i - x_j, f = w_i^T K(r) F_j. For the seeded MLP
kernel K = s(r) (O + O^T)/2 with s = 1/(8 pi |r|) and O the 3x3 reshaped MLP
output at input v, f = s(r) * (o . g) where g is the row-major flattening of
G = (w_i F_j^T + F_j w_i^T)/2. Back-propagating delta_out = s g through the
layers (tanh' = 1 - tanh^2) gives the parameter gradients and grad_v f =
W1^T delta_1. With v = r/|r| (direction input), grad_r of v^T u is
(u - v (v . u))/|r|; with v = r it is u. Then
grad_r f = (grad through v) - r/(8 pi |r|^3) (o . g);
dL/dx_i += grad_r f and dL/dx_j -= grad_r f.
"""
from __future__ import annotations

import math

import numpy as np


def dense_grad_F(X, w, kern):
    """dL/dF for any kernel: alpha_1 w_j + sum_{i != j} K(x_i - x_j)^T w_i."""
    X = np.asarray(X, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n = X.shape[0]
    out = kern.alpha1 * w.copy()
    per = max(1, (1 << 20) // max(n, 1))
    for s in range(0, n, per):
        cols = np.arange(s, min(n, s + per))
        r = X[:, None, :] - X[None, cols, :]                 # [n, b, 3]: x_i - x_j
        mask = np.ones((n, cols.size), dtype=bool)
        mask[cols, np.arange(cols.size)] = False
        r = np.where(mask[..., None], r, 1.0)
        K = kern(r)
        K[~mask] = 0.0
        out[cols] += np.einsum("ibac,ia->bc", K, w)          # K^T w_i
    return out


def dense_grad_mlp(X, F, w, mlp, chunk_pairs: int = 1 << 16, inp: str = "direction"):
    """(dL/dX [N,3], dW list, db list) for the MLP kernel."""
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n = X.shape[0]
    W, b = mlp.W, mlp.b
    nl = len(W)
    dW = [np.zeros_like(m) for m in W]
    db = [np.zeros_like(v) for v in b]
    dX = np.zeros((n, 3))
    ii, jj = np.nonzero(~np.eye(n, dtype=bool)) if n <= 4096 else (None, None)

    def pairs():
        if ii is not None:
            for s in range(0, ii.size, chunk_pairs):
                yield ii[s:s + chunk_pairs], jj[s:s + chunk_pairs]
        else:
            per = max(1, chunk_pairs // n)
            for s in range(0, n, per):
                rows = np.arange(s, min(n, s + per))
                I = np.repeat(rows, n)
                J = np.tile(np.arange(n), rows.size)
                keep = I != J
                yield I[keep], J[keep]

    for I, J in pairs():
        r = X[I] - X[J]
        d = np.sqrt(np.sum(r * r, axis=1))
        v = r / d[:, None] if inp == "direction" else r
        o, acts = mlp.forward(v, keep=True)
        wi, fj = w[I], F[J]
        G = 0.5 * (wi[:, :, None] * fj[:, None, :] + fj[:, :, None] * wi[:, None, :])
        g = G.reshape(-1, 9)
        s = 1.0 / (8.0 * math.pi * d)
        delta = s[:, None] * g
        for l in range(nl - 1, -1, -1):
            dW[l] += delta.T @ acts[l]
            db[l] += delta.sum(axis=0)
            up = delta @ W[l]
            if l > 0:
                delta = up * (1.0 - acts[l] ** 2)
            else:
                grad_r = up
        if inp == "direction":
            grad_r = (grad_r - v * np.sum(v * grad_r, axis=1)[:, None]) / d[:, None]
        og = np.sum(o * g, axis=1)
        grad_r = grad_r - r * (og / (8.0 * math.pi * d ** 3))[:, None]
        np.add.at(dX, I, grad_r)
        np.add.at(dX, J, -grad_r)
    return dX, dW, db


def dense_grad_rows(X, F, w, kern, rows):
    """Rows `rows` of the dense gradients, for sizes where the full sums are
    too costly: (dL/dF [k, 3], dL/dX [k, 3] or None for a kernel other than
    the MLP). dL/dF_j = alpha_1 w_j + sum_{i != j} K(x_i - x_j)^T w_i, and
    dL/dx_i = sum_{j != i} grad_r (w_i^T K(r) F_j)|_{r = x_i - x_j}
            - sum_{j != i} grad_r (w_j^T K(r) F_i)|_{r = x_j - x_i}
    (the particle is the target of the first pairs and the source of the
    second), each pair term back-propagated by kernel_vjp."""
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    n = X.shape[0]
    dF = np.empty((rows.size, 3))
    dX = np.empty((rows.size, 3)) if kern.mlp is not None else None
    for a, i in enumerate(rows):
        others = np.arange(n)
        others = others[others != i]
        K = kern(X[others] - X[i])                          # K(x_o - x_i), i the source
        dF[a] = kern.alpha1 * w[i] + np.einsum("pab,pa->b", K, w[others])
        if dX is None:
            continue
        g_t = np.einsum("a,pb->pab", w[i], F[others])       # i the target: w_i F_j^T
        dr_t, _, _ = kernel_vjp(X[i] - X[others], g_t, kern.mlp, kern.inp)
        g_s = np.einsum("pa,b->pab", w[others], F[i])       # i the source: w_j F_i^T
        dr_s, _, _ = kernel_vjp(X[others] - X[i], g_s, kern.mlp, kern.inp)
        dX[a] = dr_t.sum(axis=0) - dr_s.sum(axis=0)
    return dF, dX


# --------------------------------------------------------------------------
# Adjoint of the H-matrix product with its structure frozen: the tree, the
# partition, the ACA pivots and ranks (and which blocks fell back) stay as in
# the forward pass, so the product is a smooth function of X, F and theta and
# its gradient is exact (finite differences of the frozen product agree).


def kernel_vjp(r, Gbar, mlp, inp: str = "direction"):
    """Cotangents of sum_p sum_ab Gbar_p,ab K_ab(r_p) for the MLP kernel.

    r: [P, 3], Gbar: [P, 3, 3]. Returns (d/dr [P, 3], dW list, db list).
    Since K is symmetric only the symmetric part of Gbar contributes.
    """
    r = np.asarray(r, dtype=np.float64)
    d = np.sqrt(np.sum(r * r, axis=1))
    v = r / d[:, None] if inp == "direction" else r
    o, acts = mlp.forward(v, keep=True)
    g = (0.5 * (Gbar + np.swapaxes(Gbar, 1, 2))).reshape(-1, 9)
    s = 1.0 / (8.0 * math.pi * d)
    W = mlp.W
    nl = len(W)
    dW = [np.zeros_like(m) for m in W]
    db = [np.zeros_like(v_) for v_ in mlp.b]
    delta = s[:, None] * g
    for l in range(nl - 1, -1, -1):
        dW[l] += delta.T @ acts[l]
        db[l] += delta.sum(axis=0)
        up = delta @ W[l]
        if l > 0:
            delta = up * (1.0 - acts[l] ** 2)
        else:
            grad_v = up
    if inp == "direction":
        grad_v = (grad_v - v * np.sum(v * grad_v, axis=1)[:, None]) / d[:, None]
    og = np.sum(o * g, axis=1)
    dr = grad_v - r * (og / (8.0 * math.pi * d ** 3))[:, None]
    return dr, dW, db


def aca_replay(col, row, c, q, piv_i, piv_j):
    """Algorithm 2's recursion with the pivots given (no search, no stopping test).

    Returns C [l, c, 3, 3], Q [l, q, 3, 3] and the intermediates the adjoint
    needs: the residual columns a_k [l, c, 3, 3] and the pivot inverses."""
    l = len(piv_i)
    C, Q, A, Pinv = [], [], [], []
    for k in range(l):
        a = np.array(col(piv_j[k]), dtype=np.float64)
        for m in range(k):
            a = a - C[m] @ Q[m][piv_j[k]]
        P = a[piv_i[k]]
        Pi = np.linalg.inv(P)
        C.append(a @ Pi)
        b = np.array(row(piv_i[k]), dtype=np.float64)
        for m in range(k):
            b = b - C[m][piv_i[k]] @ Q[m]
        Q.append(b)
        A.append(a)
        Pinv.append(Pi)
    sh = lambda L_, n: np.asarray(L_).reshape(-1, n, 3, 3)
    return sh(C, c), sh(Q, q), sh(A, c), np.asarray(Pinv).reshape(-1, 3, 3)


def aca_adjoint(C, Q, A, Pinv, piv_i, piv_j, wt, Fs):
    """Reverse mode through Algorithm 2 (frozen pivots) for the block output
    u_i = sum_k c_k(i) t_k, t_k = sum_j q_k(j) F_j, against the cotangent wt.

    Returns (cotangents of the sampled columns G(:, j_k) [l, c, 3, 3], of the
    sampled rows G(i_k, :) [l, q, 3, 3], and dL/dF_sigma [q, 3])."""
    l = C.shape[0]
    t = np.einsum("kjab,jb->ka", Q, Fs)
    Cb = np.einsum("ia,kb->kiab", wt, t)             # d/dc_k(i) of w_i . c_k(i) t_k
    tb = np.einsum("kiba,ib->ka", C, wt)              # sum_i c_k(i)^T w_i
    Qb = np.einsum("ka,jb->kjab", tb, Fs)
    dF = np.einsum("kjba,kb->ja", Q, tb)              # sum_k q_k(j)^T tb_k
    gcol = np.zeros_like(C)
    grow = np.zeros_like(Q)
    for k in range(l - 1, -1, -1):
        ik, jk = piv_i[k], piv_j[k]
        # q_k = G(i_k, :) - sum_{m<k} c_m(i_k) q_m
        grow[k] = Qb[k]
        for m in range(k):
            Cb[m, ik] -= np.einsum("jab,jcb->ac", Qb[k], Q[m])
            Qb[m] -= np.einsum("ba,jbc->jac", C[m, ik], Qb[k])
        # c_k = a_k P^-1 with P = a_k(i_k)
        ab = Cb[k] @ Pinv[k].T
        S = np.einsum("iba,ibc->ac", A[k], Cb[k])     # sum_i a_k(i)^T cbar_k(i)
        ab[ik] -= Pinv[k].T @ S @ Pinv[k].T
        # a_k = G(:, j_k) - sum_{m<k} c_m q_m(j_k)
        gcol[k] = ab
        for m in range(k):
            Cb[m] -= np.einsum("iab,cb->iac", ab, Q[m, jk])
            Qb[m, jk] -= np.einsum("iba,ibc->ac", C[m], ab)
    return gcol, grow, dF


def hmatvec_grad(hm, X, F, w, kern):
    """Gradients of L = sum_i w_i . U_i for the H-matrix product `hm` (oracle
    hmatvec.HMatrix) with its structure frozen: (dF [N,3], dX [N,3], dW, db).
    dX and dtheta need the MLP kernel; dF works for any kernel."""
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    tree = hm.tree
    perm = tree.perm
    Xs, Fs, ws = X[perm], F[perm], w[perm]
    n = X.shape[0]
    mlp = kern.mlp
    dFs = kern.alpha1 * ws.copy()
    dXs = np.zeros((n, 3))
    dW = [np.zeros_like(m) for m in mlp.W] if mlp is not None else None
    db = [np.zeros_like(v) for v in mlp.b] if mlp is not None else None

    def add_pairs(ti, sj, Gbar):
        if mlp is None:
            return
        dr, gW, gb = kernel_vjp(Xs[ti] - Xs[sj], Gbar, mlp, kern.inp)
        np.add.at(dXs, ti, dr)
        np.add.at(dXs, sj, -dr)
        for l in range(len(dW)):
            dW[l] += gW[l]
            db[l] += gb[l]

    def dense_block(bt, et, bs, es):
        I, J = np.meshgrid(np.arange(bt, et), np.arange(bs, es), indexing="ij")
        I, J = I.ravel(), J.ravel()
        keep = I != J
        I, J = I[keep], J[keep]
        K = kern(Xs[I] - Xs[J])
        np.add.at(dFs, J, np.einsum("pab,pa->pb", K, ws[I]))      # K^T w_i
        add_pairs(I, J, np.einsum("pa,pb->pab", ws[I], Fs[J]))

    for t, s in hm.H:
        dense_block(tree.nodes[t, 0], tree.nodes[t, 1], tree.nodes[s, 0], tree.nodes[s, 1])
    for (t, s), res in zip(hm.G, hm.blocks):
        bt, et = tree.nodes[t, 0], tree.nodes[t, 1]
        bs, es = tree.nodes[s, 0], tree.nodes[s, 1]
        if res is None:
            dense_block(bt, et, bs, es)
            continue
        if res.rank == 0:
            continue
        xt, xsr = Xs[bt:et], Xs[bs:es]
        C, Q, A, Pinv = aca_replay(lambda j: kern(xt - xsr[j]), lambda i: kern(xt[i] - xsr),
                                   et - bt, es - bs, res.piv_i, res.piv_j)
        gcol, grow, dfs = aca_adjoint(C, Q, A, Pinv, res.piv_i, res.piv_j, ws[bt:et], Fs[bs:es])
        dFs[bs:es] += dfs
        c, q = et - bt, es - bs
        for k in range(len(res.piv_i)):
            add_pairs(np.arange(bt, et), np.full(c, bs + res.piv_j[k]), gcol[k])
            add_pairs(np.full(q, bt + res.piv_i[k]), np.arange(bs, es), grow[k])
    dF = np.empty_like(dFs)
    dF[perm] = dFs
    dX = np.empty_like(dXs)
    dX[perm] = dXs
    return dF, dX, dW, db


def frozen_apply(hm, X, F, kern):
    """The H-matrix product at positions X with hm's structure and pivots frozen
    (for finite-difference checks of hmatvec_grad)."""
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    tree = hm.tree
    Xs, Fs = X[tree.perm], F[tree.perm]
    Us = kern.alpha1 * Fs.copy()
    for t, s in list(hm.H) + [g for g, r in zip(hm.G, hm.blocks) if r is None]:
        bt, et, bs, es = tree.nodes[t, 0], tree.nodes[t, 1], tree.nodes[s, 0], tree.nodes[s, 1]
        for i in range(bt, et):
            J = np.arange(bs, es)
            J = J[J != i]
            if J.size:
                Us[i] += np.einsum("jab,jb->a", kern(Xs[i] - Xs[J]), Fs[J])
    for (t, s), res in zip(hm.G, hm.blocks):
        if res is None or res.rank == 0:
            continue
        bt, et, bs, es = tree.nodes[t, 0], tree.nodes[t, 1], tree.nodes[s, 0], tree.nodes[s, 1]
        xt, xsr = Xs[bt:et], Xs[bs:es]
        C, Q, _, _ = aca_replay(lambda j: kern(xt - xsr[j]), lambda i: kern(xt[i] - xsr),
                                et - bt, es - bs, res.piv_i, res.piv_j)
        t_ = np.einsum("kjab,jb->ka", Q, Fs[bs:es])
        Us[bt:et] += np.einsum("kiab,kb->ia", C, t_)
    U = np.empty_like(Us)
    U[tree.perm] = Us
    return U
