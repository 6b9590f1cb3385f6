"""Pins of the oracle kernels against closed forms and invariants (CPU only).

RPY: the textbook parallel / perpendicular mobilities of two equal spheres,
continuity at contact r = 2a, the Oseen limit, zero divergence and positive
definiteness of the assembled mobility. MLP stand-in: a hand-evaluated network
with one active unit per layer, the all-bias special case I/(8 pi |r|),
symmetry and homogeneity of degree -1 in the direction-input reading.
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import dense, kernels

A = 1.0


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("d", [0.3, 1.0, 1.7, 2.0, 2.5, 4.0, 17.0, 300.0])
def test_rpy_parallel_perpendicular(d):
    # Two equal spheres: along the line of centres the mobility is
    #   r >= 2a: (1/(4 pi r)) (1 - 2a^2/(3 r^2)),   r < 2a: (1/(6 pi a)) (1 - 3r/(16a))
    # and across it
    #   r >= 2a: (1/(8 pi r)) (1 + 2a^2/(3 r^2)),   r < 2a: (1/(6 pi a)) (1 - 9r/(32a)).
    n = _unit([0.3, -0.7, 0.64])
    K = kernels.rpy(d * n)
    t = _unit(np.cross(n, [1.0, 0.0, 0.0]))
    par, perp = n @ K @ n, t @ K @ t
    if d >= 2 * A:
        ep = (1.0 / (4 * math.pi * d)) * (1 - 2 * A * A / (3 * d * d))
        eq = (1.0 / (8 * math.pi * d)) * (1 + 2 * A * A / (3 * d * d))
    else:
        ep = (1.0 / (6 * math.pi * A)) * (1 - 3 * d / (16 * A))
        eq = (1.0 / (6 * math.pi * A)) * (1 - 9 * d / (32 * A))
    assert par == pytest.approx(ep, rel=1e-13)
    assert perp == pytest.approx(eq, rel=1e-13)
    assert abs(t @ K @ n) < 1e-15            # no cross coupling


def test_rpy_continuity_at_contact():
    n = _unit([1.0, 2.0, -0.5])
    lo = kernels.rpy((2 * A - 1e-12) * n)
    hi = kernels.rpy((2 * A) * n)
    expect = 7.0 / (96 * math.pi * A) * np.eye(3) + 1.0 / (32 * math.pi * A) * np.outer(n, n)
    assert np.allclose(lo, expect, atol=1e-12, rtol=0)
    assert np.allclose(hi, expect, atol=1e-15, rtol=0)


def test_rpy_oseen_limit():
    n = _unit([-0.2, 0.9, 0.4])
    for d in (1e4, 1e6):
        K = kernels.rpy(d * n) * (8 * math.pi * d)
        assert np.allclose(K, np.eye(3) + np.outer(n, n), atol=3 / d ** 2)


@pytest.mark.parametrize("d", [0.9, 1.6, 3.0, 11.0])
def test_rpy_divergence_free(d):
    # sum_j dK_ij/dr_j = 0 in both branches (central differences).
    r0 = d * _unit([0.4, -0.3, 0.85])
    h = 1e-5
    div = np.zeros(3)
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        div += (kernels.rpy(r0 + e)[:, j] - kernels.rpy(r0 - e)[:, j]) / (2 * h)
    assert np.max(np.abs(div)) < 1e-8


def test_rpy_symmetry_and_evenness():
    rng = wl.Rng(11, "misc")
    r = rng.normal(300).reshape(100, 3) * 3
    K = kernels.rpy(r)
    assert np.array_equal(K, np.swapaxes(K, 1, 2)) or np.allclose(K, np.swapaxes(K, 1, 2), atol=1e-17)
    assert np.allclose(kernels.rpy(-r), K, atol=0, rtol=1e-15)


def test_rpy_mobility_positive_definite():
    X = wl.rsa_cube(200, 0.3, seed=5)
    M = dense.dense_matrix(X, kernels.Kernel("rpy"))
    assert np.allclose(M, M.T, atol=1e-16)
    np.linalg.cholesky(M)                       # raises if not SPD


def _one_unit_mlp(alpha, beta, gamma, delta, omega):
    W1 = np.zeros((64, 3)); b1 = np.zeros(64)
    W2 = np.zeros((64, 64)); b2 = np.zeros(64)
    W3 = np.zeros((64, 64)); b3 = np.zeros(64)
    W4 = np.zeros((9, 64)); b4 = np.zeros(9)
    W1[0] = alpha; b1[0] = beta
    W2[0, 0] = gamma
    W3[0, 0] = delta
    W4[:, 0] = omega
    return kernels.MLP([W1, W2, W3, W4], [b1, b2, b3, b4])


@pytest.mark.parametrize("inp", ["direction", "displacement"])
def test_mlp_one_active_unit_by_hand(inp):
    alpha = np.array([0.7, -0.2, 0.4])
    beta, gamma, delta = 0.3, -1.3, 0.9
    omega = np.arange(1.0, 10.0) / 10.0          # O = [[.1,.2,.3],[.4,.5,.6],[.7,.8,.9]]
    mlp = _one_unit_mlp(alpha, beta, gamma, delta, omega)
    r = np.array([1.5, -2.0, 0.5])
    d = math.sqrt(1.5 ** 2 + 2.0 ** 2 + 0.5 ** 2)
    v = r / d if inp == "direction" else r
    h1 = math.tanh(0.7 * v[0] - 0.2 * v[1] + 0.4 * v[2] + 0.3)
    h2 = math.tanh(-1.3 * h1)
    h3 = math.tanh(0.9 * h2)
    O = np.array([[0.1, 0.2, 0.3], [0.4, 0.5, 0.6], [0.7, 0.8, 0.9]]) * h3
    expect = 0.5 * (O + O.T) / (8 * math.pi * d)
    K = kernels.mlp_kernel(r[None], mlp, inp)[0]
    assert np.allclose(K, expect, rtol=1e-14, atol=0)


def test_mlp_bias_only_is_scaled_identity():
    W = [np.zeros((64, 3)), np.zeros((64, 64)), np.zeros((64, 64)), np.zeros((9, 64))]
    b = [np.full(64, 0.3), np.full(64, -0.1), np.full(64, 0.2), np.eye(3).ravel()]
    mlp = kernels.MLP(W, b)
    rng = wl.Rng(12, "misc")
    r = rng.normal(60).reshape(20, 3) * 5
    K = kernels.mlp_kernel(r, mlp)
    d = np.linalg.norm(r, axis=1)
    assert np.allclose(K, np.eye(3)[None] / (8 * math.pi * d)[:, None, None], rtol=1e-14, atol=0)


def test_mlp_kernel_symmetric_and_homogeneous():
    Ws, bs = wl.mlp_weights(1)
    mlp = kernels.MLP(Ws, bs)
    rng = wl.Rng(13, "misc")
    r = rng.normal(300).reshape(100, 3) * 4
    K = kernels.mlp_kernel(r, mlp, "direction")
    assert np.allclose(K, np.swapaxes(K, 1, 2), rtol=0, atol=1e-18)
    K7 = kernels.mlp_kernel(7.0 * r, mlp, "direction")
    assert np.allclose(7.0 * K7, K, rtol=1e-12, atol=0)


def test_self_mobility_value():
    assert kernels.self_mobility(1.0, 1.0) == pytest.approx(0.05305164769729845, rel=1e-15)
    assert kernels.self_mobility(2.0, 0.5) == pytest.approx(1.0 / (6 * math.pi), rel=1e-15)
