"""Pins of the oracle gradients (CPU only): dL/dF against the transposed dense
matrix, and dL/dX, dL/dtheta against torch-CPU float64 autograd of an
independently written forward pass and against central finite differences,
for both MLP inputs (unit direction and raw displacement); the sampled-row
gradients against the full ones."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import dense, grad, kernels


def _setup(n=30, seed=9):
    X = wl.rsa_cube(n, 0.2, seed=seed)
    F = wl.normal_forces(n, seed=seed)
    w = wl.normal_forces(n, seed=seed + 100)
    Ws, bs = wl.mlp_weights(1)
    return X, F, w, kernels.MLP(Ws, bs)


def test_grad_F_is_transposed_matrix():
    X, F, w, mlp = _setup()
    for kern in (kernels.Kernel("rpy"), kernels.Kernel("mlp", mlp)):
        M = dense.dense_matrix(X, kern)
        g = grad.dense_grad_F(X, w, kern)
        assert np.allclose(g.ravel(), M.T @ w.ravel(), rtol=1e-13, atol=1e-16)


def _torch_loss(X, F, w, Ws, bs, inp="direction"):
    n = X.shape[0]
    i, j = torch.meshgrid(torch.arange(n), torch.arange(n), indexing="ij")
    keep = i != j
    i, j = i[keep], j[keep]
    r = X[i] - X[j]
    d = torch.linalg.norm(r, dim=1)
    h = r / d[:, None] if inp == "direction" else r
    for l in range(4):
        h = torch.nn.functional.linear(h, Ws[l], bs[l])
        if l < 3:
            h = torch.tanh(h)
    O = h.reshape(-1, 3, 3)
    K = 0.5 * (O + O.transpose(1, 2)) / (8 * math.pi * d)[:, None, None]
    U = torch.zeros_like(F).index_add(0, i, torch.einsum("pab,pb->pa", K, F[j]))
    U = U + F / (6 * math.pi)
    return torch.sum(w * U)


@pytest.mark.parametrize("inp", ["direction", "displacement"])
def test_mlp_grads_match_torch_autograd(inp):
    X, F, w, mlp = _setup()
    Xt = torch.tensor(X, dtype=torch.float64, requires_grad=True)
    Ft = torch.tensor(F, dtype=torch.float64)
    wt = torch.tensor(w, dtype=torch.float64)
    Wt = [torch.tensor(m, requires_grad=True) for m in mlp.W]
    bt = [torch.tensor(v, requires_grad=True) for v in mlp.b]
    L = _torch_loss(Xt, Ft, wt, Wt, bt, inp)
    L.backward()
    dX, dW, db = grad.dense_grad_mlp(X, F, w, mlp, inp=inp)
    assert np.allclose(dX, Xt.grad.numpy(), rtol=1e-11, atol=1e-14)
    for l in range(4):
        assert np.allclose(dW[l], Wt[l].grad.numpy(), rtol=1e-11, atol=1e-14)
        assert np.allclose(db[l], bt[l].grad.numpy(), rtol=1e-11, atol=1e-14)
    # the loss itself agrees with the dense oracle
    U = dense.dense_u(X, F, kernels.Kernel("mlp", mlp, inp=inp))
    assert abs(L.item() - np.sum(w * U)) < 1e-12 * max(1.0, abs(L.item()))


@pytest.mark.parametrize("inp", ["direction", "displacement"])
def test_kernel_vjp_matches_torch_autograd(inp):
    """The pair-level VJP that the H-matrix adjoint uses, against autograd of
    sum_p <Gbar_p, K(r_p)> written independently in torch."""
    X, F, w, mlp = _setup(n=12, seed=11)
    rng = np.random.default_rng(0)
    r = rng.normal(size=(40, 3)) * 3.0
    Gb = rng.normal(size=(40, 3, 3))
    rt = torch.tensor(r, requires_grad=True)
    Wt = [torch.tensor(m, requires_grad=True) for m in mlp.W]
    bt = [torch.tensor(v, requires_grad=True) for v in mlp.b]
    d = torch.linalg.norm(rt, dim=1)
    h = rt / d[:, None] if inp == "direction" else rt
    for l in range(4):
        h = torch.nn.functional.linear(h, Wt[l], bt[l])
        if l < 3:
            h = torch.tanh(h)
    O = h.reshape(-1, 3, 3)
    K = 0.5 * (O + O.transpose(1, 2)) / (8 * math.pi * d)[:, None, None]
    torch.sum(K * torch.tensor(Gb)).backward()
    dr, dW, db = grad.kernel_vjp(r, Gb, mlp, inp)
    assert np.allclose(dr, rt.grad.numpy(), rtol=1e-11, atol=1e-15)
    for l in range(4):
        assert np.allclose(dW[l], Wt[l].grad.numpy(), rtol=1e-11, atol=1e-15)
        assert np.allclose(db[l], bt[l].grad.numpy(), rtol=1e-11, atol=1e-15)


@pytest.mark.parametrize("inp", ["direction", "displacement"])
def test_sampled_row_grads_equal_full(inp):
    X, F, w, mlp = _setup(n=40, seed=13)
    kern = kernels.Kernel("mlp", mlp, inp=inp)
    dX, _, _ = grad.dense_grad_mlp(X, F, w, mlp, inp=inp)
    dF = grad.dense_grad_F(X, w, kern)
    rows = np.array([0, 7, 39, 21])
    gF, gX = grad.dense_grad_rows(X, F, w, kern, rows)
    assert np.allclose(gF, dF[rows], rtol=1e-12, atol=1e-15)
    assert np.allclose(gX, dX[rows], rtol=1e-11, atol=1e-15)
    gF2, gX2 = grad.dense_grad_rows(X, F, w, kernels.Kernel("rpy"), rows)
    assert gX2 is None
    assert np.allclose(gF2, grad.dense_grad_F(X, w, kernels.Kernel("rpy"))[rows], rtol=1e-12)


@pytest.mark.parametrize("inp", ["direction", "displacement"])
def test_mlp_grad_X_finite_differences(inp):
    X, F, w, mlp = _setup(n=20, seed=4)
    kern = kernels.Kernel("mlp", mlp, inp=inp)
    dX, _, _ = grad.dense_grad_mlp(X, F, w, mlp, inp=inp)
    h = 1e-5
    for (p, d) in [(0, 0), (7, 2), (19, 1)]:
        Xp, Xm = X.copy(), X.copy()
        Xp[p, d] += h
        Xm[p, d] -= h
        fd = (np.sum(w * dense.dense_u(Xp, F, kern)) - np.sum(w * dense.dense_u(Xm, F, kern))) / (2 * h)
        assert abs(fd - dX[p, d]) <= 1e-7 * max(1.0, abs(fd))
