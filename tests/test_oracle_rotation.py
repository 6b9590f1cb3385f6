"""Pins of the oracle's rotational mobility (CPU only).

* M^rt F is half the curl of the Stokeslet (Oseen) flow of F, taken by
  central differences of the flow field;
* M^rr T is half the curl of the rotlet flow T x r / (8 pi mu |r|^3), by
  central differences;
* M^tr T is the rotlet flow itself at the target;
* the 6N matrix is symmetric (M^tr_ij = (M^rt_ji)^T) and positive definite for
  non-overlapping spheres;
* the cross-product matrix and the self mobilities;
* the 6N H-matrix: dense mode is the 6N matrix, the translation block is the
  3N RPY product, Eq. (11) holds, and with two-particle leaves (where columns
  of singular coupling entries leave only poorly conditioned pivots) the
  product is the dense sum to rounding.
"""
import math

import numpy as np

import workloads as wl
from oracle import rotation as OR


def _curl(field, x, h=1e-4):
    J = np.zeros((3, 3))   # J[a, b] = d field_a / d x_b
    for b in range(3):
        e = np.zeros(3)
        e[b] = h
        J[:, b] = (field(x + e) - field(x - e)) / (2 * h)
    return np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])


def test_coupling_is_half_curl_of_stokeslet_and_rotlet_flow():
    mu = 1.3
    xj = np.array([0.3, -1.0, 2.0])
    F = np.array([0.4, -1.1, 0.7])
    T = np.array([-0.2, 0.5, 1.3])
    oseen = lambda x: ((np.eye(3) + np.outer(x - xj, x - xj) / np.sum((x - xj) ** 2)) @ F /
                       (8 * math.pi * mu * np.linalg.norm(x - xj)))
    rotlet = lambda x: np.cross(T, x - xj) / (8 * math.pi * mu * np.linalg.norm(x - xj) ** 3)
    for xi in (np.array([4.0, 1.0, -2.0]), np.array([-3.0, 2.5, 5.0])):
        r = xi - xj
        w_from_F = 0.5 * _curl(oseen, xi)
        assert np.allclose(OR.coupling(r, mu) @ F, w_from_F, rtol=1e-7, atol=1e-11)
        assert np.allclose(OR.coupling(r, mu) @ T, rotlet(xi), rtol=1e-13, atol=1e-16)
        assert np.allclose(OR.rotation(r, mu) @ T, 0.5 * _curl(rotlet, xi), rtol=1e-7, atol=1e-11)


def test_mobility6_symmetric_positive_definite():
    X = wl.rsa_cube(60, 0.2, seed=3)
    M = OR.mobility6(X, 1.0, 1.0)
    assert np.allclose(M, M.T, rtol=0, atol=1e-15)
    np.linalg.cholesky(M)   # raises if not positive definite
    F = wl.normal_forces(60, seed=1)
    T = wl.normal_forces(60, seed=2)
    U, W = OR.u6(X, F, T)
    y = M @ np.concatenate([F.ravel(), T.ravel()])
    assert np.allclose(np.concatenate([U.ravel(), W.ravel()]), y, rtol=1e-12, atol=1e-15)


def test_cross_matrix_and_self_terms():
    v = np.array([1.0, -2.0, 0.5])
    u = np.array([0.3, 0.7, -1.1])
    assert np.allclose(OR.cross_matrix(v) @ u, np.cross(v, u), rtol=0, atol=1e-15)
    assert OR.self_rotation(2.0, 0.5) == 1.0 / (8 * math.pi * 0.5 * 8.0)
    # rotation block: traceless and symmetric; coupling: antisymmetric
    r = np.array([1.0, 2.0, -3.0])
    R = OR.rotation(r)
    C = OR.coupling(r)
    assert abs(np.trace(R)) < 1e-16 and np.allclose(R, R.T) and np.allclose(C, -C.T)


def test_hmatrix6_dense_mode_is_the_6n_matrix():
    # no admissible block: the assembly (sorted rows, interleaved types, self
    # terms, the zero pair term of a particle's own two rows) against the
    # explicit 6N matrix
    n = 150
    X = wl.rsa_cube(n, 0.2, seed=5)
    F = wl.normal_forces(n, seed=3)
    T = wl.normal_forces(n, seed=4)
    hm = OR.build6(X, 16, dense_mode=True)
    assert len(hm.G) == 0
    U, W = OR.apply6(hm, X, F, T)
    y = OR.mobility6(X) @ np.concatenate([F.ravel(), T.ravel()])
    assert np.allclose(np.concatenate([U.ravel(), W.ravel()]), y, rtol=1e-13, atol=1e-16)


def test_translation_block_is_the_3n_rpy_product():
    from oracle import dense as OD
    from oracle import kernels as OK
    n = 300
    X = wl.rsa_cube(n, 0.2, seed=6)
    F = wl.normal_forces(n, seed=5)
    U, W = OR.u6(X, F, np.zeros_like(F))
    assert np.allclose(U, OD.dense_u(X, F, OK.Kernel("rpy")), rtol=1e-13, atol=1e-16)
    # torques alone move the particles through the coupling only: no self term
    U2, W2 = OR.u6(X[:2], np.zeros((2, 3)), np.array([[0, 0, 1.0], [0, 0, 0]]))
    r = X[1] - X[0]
    assert np.allclose(U2[1], np.cross([0, 0, 1.0], r) / (8 * math.pi * np.linalg.norm(r) ** 3),
                       rtol=1e-14, atol=0)
    assert np.allclose(W2[0], [0, 0, OR.self_rotation()], rtol=1e-15, atol=0)


def test_hmatrix6_within_eq11_bound():
    # Algorithm 2 on the 6N grid with |det| pivots, and the relative error of
    # Eq. (11) over all 6N components below 10 zeta. A block with a single
    # particle on one side (two rows) may end on a singular residual pivot
    # (the rotation row's residual at a force column is built from the
    # singular coupling entries) and falls back to dense evaluation; no
    # larger block does
    n = 700
    X = wl.rsa_cube(n, 0.2, seed=3)
    F = wl.normal_forces(n, seed=1)
    T = wl.normal_forces(n, seed=2)
    U, W = OR.u6(X, F, T)
    hm = OR.build6(X, 32, 1.0, 1e-6, 48)
    nodes = hm.tree.nodes
    sizes = [min(nodes[t, 1] - nodes[t, 0], nodes[s, 1] - nodes[s, 0]) for t, s in hm.G]
    assert len(hm.G) > 0 and sum(m > 1 for m in sizes) > 50
    assert all(m == 1 for m, b in zip(sizes, hm.blocks) if b is None)
    Uh, Wh = OR.apply6(hm, X, F, T)
    ref = np.concatenate([U.ravel(), W.ravel()])
    e = np.linalg.norm(np.concatenate([Uh.ravel(), Wh.ravel()]) - ref) / np.linalg.norm(ref)
    assert e < 1e-5


def test_hmatrix6_small_leaves_no_ill_conditioned_pivots():
    # 65 particles in 4-row leaves (two particles): blocks small enough that a
    # column of coupling entries (singular) leaves only poorly conditioned
    # pivots. With the determinant rule's conditioning cap those blocks are
    # evaluated densely and the product is the dense sum to rounding; a cap at
    # the bare singularity level (1e-14) gave 2.5e-9 here, and 5e-7 with the
    # inverse taken through the adjugate instead of LU
    n = 65
    X = wl.rsa_cube(n, 0.05, seed=84)
    F = wl.normal_forces(n, seed=85)
    T = wl.normal_forces(n, seed=86)
    U, W = OR.u6(X, F, T)
    ref = np.hstack([U, W])
    o = OR.build6(X, 4, 1.0, 1e-8, 48)
    Uo, Wo = OR.apply6(o, X, F, T)
    Y = np.hstack([Uo, Wo])
    assert np.linalg.norm(Y - ref) / np.linalg.norm(ref) < 1e-10
    assert np.max(np.linalg.norm(Y - ref, axis=1)) / np.max(np.linalg.norm(ref, axis=1)) < 1e-10
