"""Exact dense FP64 mobility product (oracle only).

U_i = alpha_1 F_i + sum_{j != i} K(x_i - x_j) F_j

This is Eq. (2) restricted to the one-body and the two-body off-diagonal terms,
equivalently M^(1) F + M^(t,2) F of Eq. (6): the quantity the H-matrix product
approximates (Sec. 3). The diagonal of M^(t,2) is empty (j != i in Eq. (2)).
"""
from __future__ import annotations

import numpy as np


def two_body_rows(X, F, kern, rows, chunk_pairs: int = 1 << 20):
    """sum_{j != i} K(x_i - x_j) F_j for each i in `rows` ([len(rows), 3])."""
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    n = X.shape[0]
    out = np.zeros((rows.size, 3))
    per = max(1, chunk_pairs // max(n, 1))
    for s in range(0, rows.size, per):
        rr = rows[s:s + per]
        r = X[rr][:, None, :] - X[None, :, :]            # [b, n, 3]
        mask = np.ones((rr.size, n), dtype=bool)
        mask[np.arange(rr.size), rr] = False
        r = np.where(mask[..., None], r, 1.0)             # placeholder, dropped below
        K = kern(r)                                       # [b, n, 3, 3]
        K[~mask] = 0.0
        out[s:s + per] = np.einsum("bnij,nj->bi", K, F)
    return out


def dense_u(X, F, kern, rows=None):
    """Full dense product U (or its rows `rows`)."""
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    if rows is None:
        rows = np.arange(X.shape[0])
    rows = np.asarray(rows, dtype=np.int64)
    return kern.alpha1 * F[rows] + two_body_rows(X, F, kern, rows)


def dense_matrix(X, kern):
    """The 3N x 3N matrix M = M^(1) + M^(t,2) (small N only)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    r = X[:, None, :] - X[None, :, :]
    eye = np.eye(n, dtype=bool)
    r = np.where(eye[..., None], 1.0, r)
    K = kern(r)
    K[eye] = 0.0
    K[eye] += kern.alpha1 * np.eye(3)
    return K.transpose(0, 2, 1, 3).reshape(3 * n, 3 * n)


def rel_err(u, ref):
    """Relative 2-norm error over all components, the form of Eq. (11)."""
    u = np.asarray(u, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(u - ref) / np.linalg.norm(ref))
