"""The allocation-free product hh_matvec_noalloc against hh_matvec.

Two calls in a row on one device, the second on a smaller input, each equal
bit for bit to hh_matvec on the same handles (same kernels, workspaces in the
library's static scratch instead of the low-rank handle); the size limit and
the streamed-mode refusal are errors, checked before any work.
"""
import pytest
import torch

import paper_2505_08174_amd as hh
import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,prec", [("mlp", "bf16"), ("rpy", "fp64"), ("mlp", "fp32")])
def test_noalloc_equals_matvec(kind, prec):
    from gpu_common import ctx, dev, kernels, say
    _, kg = kernels(kind)
    fdt = torch.float64 if prec == "fp64" else torch.float32
    for n in (30000, 4000):   # the second call on a smaller input
        say("noalloc", kind, prec, n)
        X = wl.rsa_cube(n, 0.15, seed=n)
        F = dev(wl.normal_forces(n, seed=n + 1), fdt)
        hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, eta=1.0,
                        eps=1e-6 if prec == "fp64" else 1e-4, prec=prec)
        assert hm.lr.info()["bytes"] > 0   # stored factors
        ref = hm @ F
        U = torch.full_like(ref, float("nan"))
        hh.matvec_noalloc(ctx(), hm.tree, hm.part, hm.lr, kg, F, U, prec)
        torch.cuda.synchronize()
        assert torch.equal(U, ref)
        # again, after other work on the device, with new forces
        F2 = dev(wl.normal_forces(n, seed=n + 2), fdt)
        ref2 = hm @ F2
        hh.matvec_noalloc(ctx(), hm.tree, hm.part, hm.lr, kg, F2, U, prec)
        torch.cuda.synchronize()
        assert torch.equal(U, ref2)


def test_noalloc_errors():
    from gpu_common import ctx, dev, kernels, say
    _, kg = kernels("rpy")
    # streamed mode is refused
    n = 6000
    X = wl.rsa_cube(n, 0.15, seed=3)
    ctx().set_budget(2 << 20)
    try:
        hs = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, eps=1e-6, prec="fp64")
    finally:
        ctx().set_budget(64 << 30)
    assert hs.lr.info()["bytes"] == 0
    U = torch.empty((n, 3), dtype=torch.float64, device="cuda:0")
    with pytest.raises(hh.HHError, match="INVALID_ARG"):
        hh.matvec_noalloc(ctx(), hs.tree, hs.part, hs.lr, kg, dev(wl.normal_forces(n)), U, "fp64")
    # beyond the scratch: 1.5M particles in FP64 need 72 MB (checked first)
    n = 1_500_000
    say("noalloc capacity", n)
    X = wl.lattice_sphere(n, 0.1, seed=0)
    ctx().set_budget(1 << 30)
    try:
        big = hh.HMatrix(ctx(), dev(X), kg, c_leaf=128, eps=1e-6, prec="fp64")
    finally:
        ctx().set_budget(64 << 30)
    Fb = torch.zeros((n, 3), dtype=torch.float64, device="cuda:0")
    Ub = torch.empty_like(Fb)
    with pytest.raises(hh.HHError, match="CAPACITY"):
        hh.matvec_noalloc(ctx(), big.tree, big.part, big.lr, kg, Fb, Ub, "fp64")
