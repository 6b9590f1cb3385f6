"""Pins of the oracle adjoint of the H-matrix product (CPU only).

With the structure frozen (tree, partition, pivots, ranks, fallbacks) the
H-matrix product is a smooth function of X, F and theta; its oracle gradient
is checked against central finite differences of that frozen product, the
replayed ACA against the searched one, dL/dF against the explicitly
materialised transposed H-matrix, and the kernel cotangent routine against
the dense gradient written out independently.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import aca, dense, grad, hmatvec, kernels


def _setup(n=260, eps=1e-5, seed=6, build=True):
    X = wl.rsa_cube(n, 0.15, seed=seed)
    F = wl.normal_forces(n, seed=seed)
    w = wl.normal_forces(n, seed=seed + 50)
    mlp = kernels.MLP(*wl.mlp_weights(1))
    kern = kernels.Kernel("mlp", mlp)
    hm = hmatvec.build(X, kern, 16, 1.0, eps, 48) if build else None
    assert hm is None or len(hm.G) > 10
    return X, F, w, kern, hm


def test_replay_reproduces_search():
    X, F, w, kern, hm = _setup()
    Xs = X[hm.tree.perm]
    for (t, s), res in list(zip(hm.G, hm.blocks))[:20]:
        bt, et = hm.tree.nodes[t, :2]
        bs, es = hm.tree.nodes[s, :2]
        xt, xsr = Xs[bt:et], Xs[bs:es]
        C, Q, _, _ = grad.aca_replay(lambda j: kern(xt - xsr[j]), lambda i: kern(xt[i] - xsr),
                                     et - bt, es - bs, res.piv_i, res.piv_j)
        assert np.allclose(C, res.C, rtol=1e-12, atol=1e-14) and np.allclose(Q, res.Q, rtol=1e-12, atol=1e-14)
    U1 = hmatvec.apply(hm, X, F, kern)
    U2 = grad.frozen_apply(hm, X, F, kern)
    assert np.allclose(U1, U2, rtol=1e-12, atol=1e-15)


def test_kernel_vjp_matches_dense_gradient():
    X, F, w, kern, _ = _setup(n=40, build=False)
    n = X.shape[0]
    I, J = np.nonzero(~np.eye(n, dtype=bool))
    dr, dW, db = grad.kernel_vjp(X[I] - X[J], np.einsum("pa,pb->pab", w[I], F[J]), kern.mlp)
    dX = np.zeros((n, 3))
    np.add.at(dX, I, dr)
    np.add.at(dX, J, -dr)
    rX, rW, rb = grad.dense_grad_mlp(X, F, w, kern.mlp)
    assert np.allclose(dX, rX, rtol=1e-12, atol=1e-15)
    for l in range(4):
        assert np.allclose(dW[l], rW[l], rtol=1e-12, atol=1e-15)


def test_grad_F_is_transposed_hmatrix():
    # U is linear in F: dF . e = w . (M_H e) for any probe e
    X, F, w, kern, hm = _setup()
    dF, _, _, _ = grad.hmatvec_grad(hm, X, F, w, kern)
    for seed in (11, 12, 13):
        e = wl.normal_forces(X.shape[0], seed=seed)
        lhs = float(np.sum(dF * e))
        rhs = float(np.sum(w * grad.frozen_apply(hm, X, e, kern)))
        assert abs(lhs - rhs) <= 1e-11 * abs(rhs)


@pytest.mark.slow
def test_grad_X_theta_finite_differences():
    X, F, w, kern, hm = _setup(n=160, seed=7)
    dF, dX, dW, db = grad.hmatvec_grad(hm, X, F, w, kern)
    L = lambda X_, k_: float(np.sum(w * grad.frozen_apply(hm, X_, F, k_)))
    h = 1e-5
    rng = np.random.default_rng(4)
    for _ in range(4):
        p, d = int(rng.integers(X.shape[0])), int(rng.integers(3))
        Xp, Xm = X.copy(), X.copy()
        Xp[p, d] += h
        Xm[p, d] -= h
        fd = (L(Xp, kern) - L(Xm, kern)) / (2 * h)
        assert abs(fd - dX[p, d]) <= 1e-6 * max(1.0, abs(fd)), (p, d, fd, dX[p, d])
    Ws, bs = [m.copy() for m in kern.mlp.W], [v.copy() for v in kern.mlp.b]
    for (l, idx) in [(1, (3, 17)), (3, (4, 30)), (0, (10, 2))]:
        def Lw(delta):
            W2 = [m.copy() for m in Ws]
            W2[l][idx] += delta
            return L(X, kernels.Kernel("mlp", kernels.MLP(W2, bs)))
        fd = (Lw(h) - Lw(-h)) / (2 * h)
        assert abs(fd - dW[l][idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx, fd, dW[l][idx])


def test_adjoint_displacement_input_finite_differences():
    """The frozen-structure adjoint with the raw-displacement MLP input (the
    kernel is then not asymptotically smooth and many blocks fall back)."""
    X = wl.rsa_cube(260, 0.15, seed=21)
    F = wl.normal_forces(260, seed=21)
    w = wl.normal_forces(260, seed=71)
    mlp = kernels.MLP(*wl.mlp_weights(1))
    kern = kernels.Kernel("mlp", mlp, inp="displacement")
    hm = hmatvec.build(X, kern, 16, 1.0, 1e-5, 48)
    assert len(hm.G) > 10
    dF, dX, dW, db = grad.hmatvec_grad(hm, X, F, w, kern)
    L = lambda X_, k_: float(np.sum(w * grad.frozen_apply(hm, X_, F, k_)))
    h = 1e-5
    for (p, d) in [(3, 0), (77, 2)]:
        Xp, Xm = X.copy(), X.copy()
        Xp[p, d] += h
        Xm[p, d] -= h
        fd = (L(Xp, kern) - L(Xm, kern)) / (2 * h)
        assert abs(fd - dX[p, d]) <= 1e-6 * max(1.0, abs(fd)), (p, d, fd, dX[p, d])
    W2 = [m.copy() for m in mlp.W]
    W2[2][5, 9] += h
    W3 = [m.copy() for m in mlp.W]
    W3[2][5, 9] -= h
    fd = (L(X, kernels.Kernel("mlp", kernels.MLP(W2, mlp.b), inp="displacement")) -
          L(X, kernels.Kernel("mlp", kernels.MLP(W3, mlp.b), inp="displacement"))) / (2 * h)
    assert abs(fd - dW[2][5, 9]) <= 1e-6 * max(1.0, abs(fd))
    # dL/dF is the transposed frozen product
    e = wl.normal_forces(260, seed=5)
    assert abs(float(np.sum(dF * e)) - float(np.sum(w * grad.frozen_apply(hm, X, e, kern)))) \
        <= 1e-11 * abs(float(np.sum(dF * e)))
