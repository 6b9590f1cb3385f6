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
