"""Pins of the dense FP64 product (CPU only): two-particle closed form, the
excluded diagonal, linearity, translation invariance, permutation equivariance,
and agreement with the assembled 3N x 3N matrix."""
import math

import numpy as np

import workloads as wl
from oracle import dense, kernels

RPY = kernels.Kernel("rpy")


def _mlp_kernel():
    Ws, bs = wl.mlp_weights(1)
    return kernels.Kernel("mlp", kernels.MLP(Ws, bs))


def test_two_particles_closed_form():
    # U_1 = F_1/(6 pi) + K(x_1 - x_2) F_2 with K from the textbook
    # parallel/perpendicular form (r >= 2a).
    x1, x2 = np.array([0.0, 0.0, 0.0]), np.array([3.0, 4.0, 0.0])   # r = 5
    F1, F2 = np.array([1.0, -2.0, 0.5]), np.array([0.3, 0.1, -1.0])
    U = dense.dense_u(np.stack([x1, x2]), np.stack([F1, F2]), RPY)
    n = (x1 - x2) / 5.0
    par = (1 / (4 * math.pi * 5)) * (1 - 2 / 75)
    perp = (1 / (8 * math.pi * 5)) * (1 + 2 / 75)
    f_par = (F2 @ n) * n
    expect1 = F1 / (6 * math.pi) + par * f_par + perp * (F2 - f_par)
    f_par2 = (F1 @ n) * n
    expect2 = F2 / (6 * math.pi) + par * f_par2 + perp * (F1 - f_par2)
    assert np.allclose(U[0], expect1, rtol=1e-14, atol=1e-16)
    assert np.allclose(U[1], expect2, rtol=1e-14, atol=1e-16)


def test_self_pair_excluded():
    X = wl.rsa_cube(50, 0.1, seed=3)
    F = np.zeros((50, 3))
    F[17] = [1.0, 2.0, 3.0]
    U = dense.dense_u(X, F, RPY)
    assert np.allclose(U[17], F[17] / (6 * math.pi), rtol=1e-15, atol=0)


def test_linear_translation_permutation():
    X = wl.rsa_cube(120, 0.15, seed=4)
    F1 = wl.normal_forces(120, seed=1)
    F2 = wl.normal_forces(120, seed=2)
    for kern in (RPY, _mlp_kernel()):
        U1 = dense.dense_u(X, F1, kern)
        U2 = dense.dense_u(X, F2, kern)
        U12 = dense.dense_u(X, 2.0 * F1 - 3.0 * F2, kern)
        assert np.allclose(U12, 2.0 * U1 - 3.0 * U2, rtol=1e-12, atol=1e-14)
        Ut = dense.dense_u(X + np.array([10.0, -4.0, 7.0]), F1, kern)
        assert np.allclose(Ut, U1, rtol=1e-11, atol=1e-13)
        p = np.random.default_rng(0).permutation(120)
        Up = dense.dense_u(X[p], F1[p], kern)
        assert np.allclose(Up, U1[p], rtol=1e-13, atol=1e-15)


def test_matrix_and_rows_agree():
    X = wl.rsa_cube(80, 0.1, seed=6)
    F = wl.normal_forces(80, seed=7)
    kern = _mlp_kernel()
    M = dense.dense_matrix(X, kern)
    U = dense.dense_u(X, F, kern)
    assert np.allclose(M @ F.ravel(), U.ravel(), rtol=1e-13, atol=1e-15)
    rows = np.array([3, 40, 79])
    assert np.allclose(dense.dense_u(X, F, kern, rows), U[rows], rtol=1e-14, atol=0)
