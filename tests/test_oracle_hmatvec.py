"""Pins of the oracle H-matrix product against the exact dense sum (CPU only):
dense mode reproduces the dense product to rounding, and the error of Eq. (11)
stays within 10 zeta and falls as zeta falls (RPY and MLP kernels)."""
import numpy as np
import pytest

import workloads as wl
from oracle import dense, hmatvec, kernels


def test_dense_mode_equals_dense():
    X = wl.rsa_cube(600, 0.1, seed=8)
    F = wl.normal_forces(600, seed=8)
    for kern in (kernels.Kernel("rpy"), kernels.Kernel("mlp", kernels.MLP(*wl.mlp_weights(1)))):
        U, hm = hmatvec.hmatvec(X, F, kern, 64, dense_mode=True)
        assert len(hm.G) == 0
        assert hmatvec.eps_r(U, dense.dense_u(X, F, kern)) < 1e-13


def test_error_within_ten_zeta_and_monotone():
    X = wl.rsa_cube(2000, 0.1, seed=0)
    F = wl.normal_forces(2000, seed=0)
    kern = kernels.Kernel("rpy")
    Ud = dense.dense_u(X, F, kern)
    errs = []
    for eps in (1e-2, 1e-4, 1e-6):
        U, hm = hmatvec.hmatvec(X, F, kern, 64, 1.0, eps)
        e = hmatvec.eps_r(U, Ud)
        assert e <= 10 * eps
        errs.append(e)
    assert errs[0] > errs[1] > errs[2]


@pytest.mark.slow
def test_mlp_error_within_ten_zeta():
    X = wl.rsa_cube(1500, 0.2, seed=0)
    F = wl.normal_forces(1500, seed=0)
    kern = kernels.Kernel("mlp", kernels.MLP(*wl.mlp_weights(1)))
    U, hm = hmatvec.hmatvec(X, F, kern, 32, 1.0, 1e-4)
    assert len(hm.G) > 0 and hm.n_fallback == 0
    assert hmatvec.eps_r(U, dense.dense_u(X, F, kern)) <= 1e-3
