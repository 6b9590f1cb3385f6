"""Short-range many-body terms of the velocity, written out directly (oracle only).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Eq. (6) splits U into M^(1) F + M^(t,2) F + M^(s,2) F + M^(t,3) F + M^(s,3) F.
The H-matrix product covers the first two; this module computes the other
three from Eq. (2) and its normalised form Eq. (4):

  U_i^short = sum_{j in N(i)} alpha_2^(s)(x_i, x_j) F_i
            + sum_{(j,k,i)} [ alpha_3^(s)(x_i, x_k, x_j) F_i + alpha_3^(t)(x_i, x_k, x_j) F_j ]

N(i) is the set of particles within the cut-off R_cut of particle i (Sec. 2.2,
R_cut = 5 from Sec. 2.4); a 3-clique (j, k, i) exists when i and j are both
neighbours of k, with j != i and k != i (Sec. 2.3), so j need not be a
neighbour of i. Following Eq. (4), with d_j = x_j - x_i and d_k = x_k - x_i:

  alpha_2^(s) = h_s(d_j) / |d_j|,
  [alpha_3^(s), alpha_3^(t)] = g(d_j, d_k) / (|x_j - x_k| |x_k - x_i|).

The trained networks are not available; seeded stand-ins take their place
(the reading is recorded with the library's design notes):
  h_s: MLP 3 -> 64 -> 64 -> 64 -> 9 on the unit direction d_j / |d_j|, output
       reshaped row-major to 3x3, symmetrised, divided by 8 pi (as the
       two-body stand-in of kernels.py);
  g:   MLP 6 -> 64 -> 64 -> 64 -> 18 (tanh hidden layers, linear output) on
       (d_j, d_k) / R_cut; outputs 0..8 and 9..17 reshaped row-major to the
       3x3 blocks of alpha_3^(s) and alpha_3^(t), each symmetrised, divided
       by 8 pi.
Everything is FP64; the loops follow the definitions (brute-force distances,
explicit clique enumeration), for small N.
"""
from __future__ import annotations

import math

import numpy as np

R_CUT = 5.0


class Net:
    """A tanh MLP: W[l] of shape [out, in], b[l] of shape [out]; tanh after
    every layer but the last."""

    def __init__(self, Ws, bs):
        self.W = [np.asarray(w, dtype=np.float64) for w in Ws]
        self.b = [np.asarray(v, dtype=np.float64) for v in bs]

    def __call__(self, v):
        h = np.asarray(v, dtype=np.float64)
        for l in range(len(self.W)):
            z = h @ self.W[l].T + self.b[l]
            h = np.tanh(z) if l < len(self.W) - 1 else z
        return h


def _sym(O):
    return 0.5 * (O + np.swapaxes(O, -1, -2))


def alpha2_s(d, hs: Net):
    """Two-body self term alpha_2^(s) for displacements d = x_j - x_i: [P, 3] -> [P, 3, 3]."""
    d = np.asarray(d, dtype=np.float64).reshape(-1, 3)
    r = np.sqrt(np.sum(d * d, axis=1))
    O = hs(d / r[:, None]).reshape(-1, 3, 3)
    return _sym(O) / (8.0 * math.pi * r)[:, None, None]


def alpha3(dj, dk, g: Net, r_cut: float = R_CUT):
    """Three-body blocks (alpha_3^(s), alpha_3^(t)) for d_j = x_j - x_i and
    d_k = x_k - x_i: [P, 3] each -> two [P, 3, 3]."""
    dj = np.asarray(dj, dtype=np.float64).reshape(-1, 3)
    dk = np.asarray(dk, dtype=np.float64).reshape(-1, 3)
    o = g(np.concatenate([dj, dk], axis=1) / r_cut)
    rjk = np.sqrt(np.sum((dj - dk) ** 2, axis=1))     # |x_j - x_k|
    rki = np.sqrt(np.sum(dk * dk, axis=1))            # |x_k - x_i|
    s = 1.0 / (8.0 * math.pi * rjk * rki)
    As = _sym(o[:, :9].reshape(-1, 3, 3)) * s[:, None, None]
    At = _sym(o[:, 9:].reshape(-1, 3, 3)) * s[:, None, None]
    return As, At


def neighbours(X, r_cut: float = R_CUT):
    """N(i) for every i: the particles j != i with |x_i - x_j| < r_cut (brute
    force over all pairs), each list ascending. The test is taken on squares
    in FP64, (dx^2 + dy^2) + dz^2 < r_cut^2 with each operation rounded (no
    fused multiply-add), so that a pair at the cut-off is decided the same way
    by every implementation that follows this order."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    rc2 = float(r_cut) * float(r_cut)
    out = []
    for i in range(n):
        d = X - X[i]
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        nb = np.nonzero(d2 < rc2)[0]
        out.append(nb[nb != i])
    return out


def cliques(X, r_cut: float = R_CUT, nb=None):
    """All 3-cliques (j, k, i): k in N(i), j in N(k), j != i. [M, 3] int array
    of (j, k, i), ordered by i, then k, then j."""
    if nb is None:
        nb = neighbours(X, r_cut)
    rows = []
    for i in range(len(nb)):
        for k in nb[i]:
            for j in nb[k]:
                if j != i:
                    rows.append((j, k, i))
    return np.asarray(rows, dtype=np.int64).reshape(-1, 3)


def short_u(X, F, hs: Net, g: Net, r_cut: float = R_CUT):
    """M^(s,2) F + M^(t,3) F + M^(s,3) F for positions X [N, 3] and forces F [N, 3]."""
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    n = X.shape[0]
    U = np.zeros((n, 3))
    nb = neighbours(X, r_cut)
    for i in range(n):
        if nb[i].size:
            K = alpha2_s(X[nb[i]] - X[i], hs)
            U[i] += np.einsum("pab,b->a", K, F[i])
    C = cliques(X, r_cut, nb)
    for s in range(0, C.shape[0], 1 << 16):
        c = C[s:s + (1 << 16)]
        j, k, i = c[:, 0], c[:, 1], c[:, 2]
        As, At = alpha3(X[j] - X[i], X[k] - X[i], g, r_cut)
        contrib = np.einsum("pab,pb->pa", As, F[i]) + np.einsum("pab,pb->pa", At, F[j])
        np.add.at(U, i, contrib)
    return U


def short_u_rows(X, F, hs: Net, g: Net, rows, r_cut: float = R_CUT):
    """short_u at the particles `rows` only (for large N): N(i) of each row and
    N(k) of each of its neighbours by the brute-force test of neighbours(),
    one particle at a time; the cliques (j, k, i) of each row in the order of
    cliques()."""
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    rc2 = float(r_cut) * float(r_cut)
    cache = {}

    def nb_of(i):
        if i not in cache:
            d = X - X[i]
            d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
            nb = np.nonzero(d2 < rc2)[0]
            cache[i] = nb[nb != i]
        return cache[i]

    rows = np.asarray(rows, dtype=np.int64)
    U = np.zeros((rows.size, 3))
    for a, i in enumerate(rows):
        ni = nb_of(int(i))
        if ni.size:
            U[a] += np.einsum("pab,b->a", alpha2_s(X[ni] - X[i], hs), F[i])
        js, ks = [], []
        for k in ni:
            for j in nb_of(int(k)):
                if j != i:
                    js.append(j)
                    ks.append(k)
        if js:
            js, ks = np.asarray(js), np.asarray(ks)
            As, At = alpha3(X[js] - X[i], X[ks] - X[i], g, r_cut)
            U[a] += np.einsum("pab,b->a", As, F[i]) + np.einsum("pab,pb->a", At, F[js])
    return U
