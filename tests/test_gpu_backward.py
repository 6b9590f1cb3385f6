"""GPU parity of the backward pass (hh_matvec_backward) against the oracle's
adjoint of the frozen-structure H-matrix product, plus the linearity pin of
dL/dF and the autograd wrapper."""
import numpy as np
import pytest
import torch

import paper_2505_08174_amd as hh
import workloads as wl
from oracle import grad as OG
from oracle import hmatvec as OH

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _case(n=600, c_leaf=32, eps=1e-5, seed=3):
    X = wl.rsa_cube(n, 0.15, seed=seed)
    F = wl.normal_forces(n, seed=seed)
    w = wl.normal_forces(n, seed=seed + 77)
    return X, F, w, c_leaf, eps


def test_backward_matches_oracle_fp64():
    from gpu_common import ctx, dev, kernels, say
    X, F, w, c_leaf, eps = _case()
    ko, kg = kernels("mlp")
    hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=c_leaf, eta=1.0, eps=eps, prec="fp64")
    ref = OH.build(X, ko, c_leaf, 1.0, eps, 48)
    ex = hm.lr.export()
    same = all(b is not None and ex["rank"][i] == b.rank and
               np.array_equal(ex["piv_i"][i, :b.rank], b.piv_i) and
               np.array_equal(ex["piv_j"][i, :b.rank], b.piv_j)
               for i, b in enumerate(ref.blocks))
    say("blocks", len(ref.blocks), "all pivots equal", same)
    assert same and len(ref.blocks) > 20
    dF, dX, dth = hh.matvec_backward(ctx(), hm.tree, hm.part, hm.lr, kg, dev(F), dev(w), "fp64")
    rF, rX, rW, rb = OG.hmatvec_grad(ref, X, F, w, ko)
    rth = hh.pack_mlp((rW, rb))
    eF, eX, et = _rel(dF.cpu().numpy(), rF), _rel(dX.cpu().numpy(), rX), _rel(dth.cpu().numpy(), rth)
    say("dF", eF, "dX", eX, "dtheta", et)
    assert eF < 1e-10 and eX < 1e-9 and et < 1e-9


def test_backward_dF_is_transpose_fp32():
    """U is linear in F: dF . e == w . (M_H e) for the same frozen H-matrix."""
    from gpu_common import ctx, dev, kernels, say
    X, F, w, c_leaf, eps = _case(n=3000, c_leaf=64, eps=1e-4, seed=5)
    _, kg = kernels("mlp")
    hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=c_leaf, eta=1.0, eps=eps, prec="fp32")
    dF, _, _ = hh.matvec_backward(ctx(), hm.tree, hm.part, hm.lr, kg, dev(F, torch.float32),
                                  dev(w, torch.float32), "fp32", want=("F",))
    for s in (1, 2):
        e = wl.normal_forces(3000, seed=40 + s)
        lhs = float(np.sum(dF.double().cpu().numpy() * e))
        rhs = float(np.sum(w * (hm @ dev(e, torch.float32)).double().cpu().numpy()))
        say("linearity", lhs, rhs)
        assert abs(lhs - rhs) <= 1e-5 * abs(rhs)


def test_autograd_wrapper():
    from gpu_common import ctx, dev, say
    X, F, w, c_leaf, eps = _case(n=400, c_leaf=32, eps=1e-6, seed=8)
    theta = torch.tensor(hh.pack_mlp(wl.mlp_weights(1)), dtype=torch.float64, requires_grad=True)
    Xt = dev(X).requires_grad_(True)
    Ft = dev(F).requires_grad_(True)
    U = hh.hmatvec_autograd(ctx(), Xt, Ft, theta, c_leaf=c_leaf, eps=eps, prec="fp64")
    L = torch.sum(dev(w) * U)
    L.backward()
    assert Xt.grad is not None and Ft.grad is not None and theta.grad is not None
    assert theta.grad.shape == (9161,) and torch.isfinite(Xt.grad).all()
