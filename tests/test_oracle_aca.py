"""Pins of the oracle ACA, Algorithm 2 with 3x3 entries (CPU only).

A block that is exactly a sum of r separable 3x3 terms is recovered with rank
r; with zero tolerance ACA interpolates the full block; after every step the
residual vanishes on the chosen rows and columns; the incremental nu^2 and
lambda^2 equal brute-force Frobenius norms; on admissible RPY and MLP blocks
the block error stays within 10 zeta. The pivot guard: the 2-norm condition
number of a 3x3 entry is at most ||P||_F^3 / |det P|, and the determinant rule
refuses a column whose entries are all conditioned worse than 1e8 (the
Frobenius rule only refuses singular entries).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import aca, kernels, partition, tree


def _sep_block(c, q, r, seed):
    rng = wl.Rng(seed, "misc")
    A = rng.normal(r * c * 9).reshape(r, c, 3, 3)
    B = rng.normal(r * q * 9).reshape(r, q, 3, 3)
    G = np.einsum("sIab,sJbc->IJac", A, B)
    return G


@pytest.mark.parametrize("pivot", ["frobenius", "determinant"])
@pytest.mark.parametrize("r", [1, 2, 5])
def test_exact_rank_recovered(r, pivot):
    c, q = 40, 33
    G = _sep_block(c, q, r, 30 + r)
    res = aca.aca_entries(lambda j: G[:, j], lambda i: G[i, :], c, q, 1e-10, 20, pivot=pivot)
    assert res.converged
    assert res.rank in (r, r + 1)
    err = np.linalg.norm(aca.lowrank_dense(res) - G) / np.linalg.norm(G)
    assert err < 1e-12


def _rpy_block(seed=0):
    X = wl.rsa_cube(2000, 0.1, seed=seed)
    tr = tree.build_tree(X, 64)
    G, _ = partition.build_partition(tr, 1.0)
    Xs = X[tr.perm]
    out = []
    for t, s in G[:: max(1, len(G) // 12)]:
        out.append((Xs[tr.nodes[t, 0]:tr.nodes[t, 1]], Xs[tr.nodes[s, 0]:tr.nodes[s, 1]]))
    return out


@pytest.mark.parametrize("pivot", ["frobenius", "determinant"])
def test_zero_tolerance_interpolates_block(pivot):
    kern = kernels.Kernel("rpy")
    Xt, Xs = _rpy_block()[0]
    Xt, Xs = Xt[:12], Xs[:9]
    res = aca.aca_block(kern, Xt, Xs, 0.0, 100, pivot=pivot)
    G = kern(Xt[:, None] - Xs[None])
    assert res.converged and res.rank == 9
    assert np.linalg.norm(aca.lowrank_dense(res) - G) <= 1e-10 * np.linalg.norm(G)


@pytest.mark.parametrize("pivot", ["frobenius", "determinant"])
def test_residual_zero_on_pivots_and_norms_match(pivot):
    kern = kernels.Kernel("rpy")
    Xt, Xs = _rpy_block()[3]
    G = kern(Xt[:, None] - Xs[None])
    res = aca.aca_block(kern, Xt, Xs, 1e-8, 30, pivot=pivot)
    gnorm = np.linalg.norm(G)
    for k in range(1, res.rank + 1):
        approx = np.einsum("kiab,kjbc->ijac", res.C[:k], res.Q[:k])
        E = G - approx
        for m in range(k):
            assert np.linalg.norm(E[res.piv_i[m]]) <= 1e-11 * gnorm
            assert np.linalg.norm(E[:, res.piv_j[m]]) <= 1e-11 * gnorm
        term = np.einsum("iab,jbc->ijac", res.C[k - 1], res.Q[k - 1])
        assert res.nu2[k - 1] == pytest.approx(np.sum(term * term), rel=1e-10)
        assert res.lam2[k - 1] == pytest.approx(np.sum(approx * approx), rel=1e-10)


@pytest.mark.parametrize("pivot", ["frobenius", "determinant"])
@pytest.mark.parametrize("kind,eps", [("rpy", 1e-4), ("rpy", 1e-6), ("mlp", 1e-4)])
def test_block_error_within_ten_zeta(kind, eps, pivot):
    if kind == "rpy":
        kern = kernels.Kernel("rpy")
    else:
        Ws, bs = wl.mlp_weights(1)
        kern = kernels.Kernel("mlp", kernels.MLP(Ws, bs))
    for Xt, Xs in _rpy_block(1):
        G = kern(Xt[:, None] - Xs[None])
        res = aca.aca_block(kern, Xt, Xs, eps, 48, pivot=pivot)
        assert res.converged
        err = np.linalg.norm(aca.lowrank_dense(res) - G) / np.linalg.norm(G)
        assert err <= 10 * eps


def test_determinant_pivot_prefers_well_conditioned_entries():
    # two candidate rows: a large nearly singular entry and a smaller regular
    # one; the Frobenius rule takes the first, the determinant rule the second
    big = np.diag([10.0, 10.0, 1e-9])
    small = np.eye(3)
    G = np.stack([np.stack([big, 2 * big]), np.stack([small, 3 * small])])   # [2, 2, 3, 3]
    rf = aca.aca_entries(lambda j: G[:, j], lambda i: G[i, :], 2, 2, 0.0, 1, pivot="frobenius")
    rd = aca.aca_entries(lambda j: G[:, j], lambda i: G[i, :], 2, 2, 0.0, 1, pivot="determinant")
    assert rd.rank == 1 and rd.piv_i[0] == 1
    assert rf.rank == 0 or rf.piv_i[0] == 0


def test_condition_bound_of_the_pivot_guard():
    # for a 3x3 matrix |det P| = s1 s2 s3 <= s1^2 s3, so the 2-norm condition
    # number never exceeds ||P||_F^3 / |det P| (the quantity the guard caps)
    rng = np.random.default_rng(4)
    for scale in (1.0, 1e-3, 1e-6, 1e-9):
        for _ in range(200):
            U, _, Vt = np.linalg.svd(rng.normal(size=(3, 3)))
            s = np.sort(rng.uniform(0.1, 10.0, 3))[::-1] * np.array([1.0, 1.0, scale])
            P = U @ np.diag(s) @ Vt
            assert np.linalg.cond(P) <= np.linalg.norm(P) ** 3 / abs(np.linalg.det(P)) * (1 + 1e-9)


@pytest.mark.parametrize("small,usable", [(1e-9, False), (1e-6, True)])
def test_determinant_rule_refuses_ill_conditioned_columns(small, usable):
    # every entry of the first column has condition number 1 / small: under the
    # determinant rule a column whose best entry is conditioned worse than 1e8
    # holds no usable pivot (dense fallback); the Frobenius rule only refuses
    # singular entries
    D = np.diag([1.0, 1.0, small])
    G = np.stack([np.stack([D, np.eye(3)]), np.stack([2.0 * D, 3.0 * np.eye(3)])])   # [2, 2, 3, 3]
    col, row = (lambda j: G[:, j]), (lambda i: G[i, :])
    rd = aca.aca_entries(col, row, 2, 2, 0.0, 2, piv_j1=0, pivot="determinant")
    rf = aca.aca_entries(col, row, 2, 2, 0.0, 2, piv_j1=0, pivot="frobenius")
    assert rf.rank >= 1
    if usable:
        assert rd.rank >= 1
    else:
        assert rd.rank == 0 and not rd.converged
