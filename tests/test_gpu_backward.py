"""GPU parity of the backward pass (hh_matvec_backward).

* against the oracle's adjoint of the frozen-structure H-matrix product
  (oracle.grad.hmatvec_grad): FP64 and FP32 forms, element by element, with
  the factors built on the oracle's own pivots (hh_aca_build_pivots), so that
  no pivot choice of the single-precision search can make the two products
  different functions; also with blocks that fall back to dense evaluation;
* the pivot replay (hh_aca_build with freeze_pivots_from) reproduces the
  searched build at the same positions;
* central finite differences of the frozen GPU product (hh_tree_refit +
  replay) at N = 5,000 in FP64, 64 coordinates each of X, F and theta;
* the dense FP64 gradient at N = 5,000 (stored by tests/golden/make_grad.py
  from the oracle): dF within 10 zeta, dX and dtheta within 100 zeta;
* sampled rows of the dense gradient at N = 50,000 (FP32 form);
* the autograd wrapper's gradients equal the oracle adjoint.
"""
import hashlib
import os

import numpy as np
import pytest
import torch

import paper_2505_08174_amd as hh
import workloads as wl
from oracle import grad as OG
from oracle import hmatvec as OH

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


def _maxrel(a, b):
    """Largest component error relative to the largest reference component."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _case(n=600, c_leaf=32, eps=1e-5, seed=3):
    X = wl.rsa_cube(n, 0.15, seed=seed)
    F = wl.normal_forces(n, seed=seed)
    w = wl.normal_forces(n, seed=seed + 77)
    return X, F, w, c_leaf, eps


def _oracle_pivots(ref):
    """The oracle's pivots, ranks and fallbacks in the layout of hh_lowrank_export."""
    nb = len(ref.blocks)
    rank = np.zeros(nb, np.int32)
    fb = np.zeros(nb, np.int32)
    pi = np.full((nb, 64), -1, np.int32)
    pj = np.full((nb, 64), -1, np.int32)
    for b, blk in enumerate(ref.blocks):
        if blk is None:
            fb[b] = 1
            continue
        rank[b] = blk.rank
        pi[b, :blk.rank] = blk.piv_i
        pj[b, :blk.rank] = blk.piv_j
    return rank, fb, pi, pj


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
    mX, mt = _maxrel(dX.cpu().numpy(), rX), _maxrel(dth.cpu().numpy(), rth)
    say("dF", eF, "dX", eX, "dtheta", et, "max", mX, mt)
    # dX and dtheta carry the cancellation of the ACA adjoint (see below)
    assert eF < 1e-10 and eX < 1e-9 and et < 1e-9
    assert mX < 1e-8 and mt < 1e-8


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_replay_reproduces_build(prec):
    """Factors replayed with a build's own pivots at the same positions are
    the build's factors (same arithmetic and summation order)."""
    from gpu_common import ctx, dev, kernels, say
    X = wl.rsa_cube(3000, 0.15, seed=9)
    F = wl.normal_forces(3000, seed=9)
    _, kg = kernels("mlp")
    fdt = torch.float64 if prec == "fp64" else torch.float32
    hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, eta=1.0, eps=1e-5, prec=prec)
    lr2 = hh.aca_build(ctx(), hm.tree, hm.part, kg, prec, freeze_pivots_from=hm.lr)
    i1, i2 = hm.lr.info(), lr2.info()
    e1, e2 = hm.lr.export(), lr2.export()
    assert i1["rank_sum"] == i2["rank_sum"] and i1["n_fallback"] == i2["n_fallback"]
    assert np.array_equal(e1["piv_i"], e2["piv_i"]) and np.array_equal(e1["piv_j"], e2["piv_j"])
    U1 = hh.matvec(ctx(), hm.tree, hm.part, hm.lr, kg, dev(F, fdt), prec).double().cpu().numpy()
    U2 = hh.matvec(ctx(), hm.tree, hm.part, lr2, kg, dev(F, fdt), prec).double().cpu().numpy()
    worst = 0.0
    G = hm.part.export()[0]
    nodes = hm.tree.export()["nodes"]
    for b in range(0, i1["n_blocks"], max(1, i1["n_blocks"] // 20)):
        if e1["fallback"][b] or e1["rank"][b] == 0:
            continue
        g = G[b]
        c = nodes[g[0], 1] - nodes[g[0], 0]
        q = nodes[g[1], 1] - nodes[g[1], 0]
        k = e1["rank"][b] - 1
        c1, q1 = hm.lr.factor(b, k, c, q)
        c2, q2 = lr2.factor(b, k, c, q)
        worst = max(worst, _rel(c2, c1), _rel(q2, q1))
    say("replay", prec, "U diff", _rel(U2, U1), "worst last factor", worst)
    tol = 1e-13 if prec == "fp64" else 1e-5
    assert _rel(U2, U1) <= tol and worst <= (1e-10 if prec == "fp64" else 1e-3)


@pytest.mark.parametrize("prec,l_max", [("fp64", 48), ("fp32", 48), ("fp64", 3)])
def test_backward_on_oracle_pivots(prec, l_max):
    """Factors replayed on the oracle's pivots (|det| rule); every gradient
    element by element against the oracle adjoint. l_max = 3 makes blocks
    fall back, so the dense-fallback adjoint runs too.
    Bounds. FP64: rounding only (measured 1e-14): dF 1e-13, dX and dtheta
    1e-11. FP32 (u = 6e-8): dF 2e-5 (kernel values to ~1e-6 per entry). The
    factors of a late ACA term are cut from a residual of size nu_k out of
    entries of size lambda, so their relative rounding error is ~u lambda /
    nu_k <= u / zeta (6e-4 at zeta = 1e-4); they add little to U but the
    adjoint gives their samples cotangents of order |w||F|, so dX and dtheta
    carry that error: bound 3 u / zeta = 2e-3 in norm and 1e-2 of the
    largest entry per component."""
    from gpu_common import ctx, dev, kernels, say
    n = 3000 if l_max > 3 else 1500
    X, F, w, _, _ = _case(n=n, seed=12)
    eps = 1e-4
    ko, kg = kernels("mlp")
    ref = OH.build(X, ko, 64, 1.0, eps, l_max, pivot="determinant")
    rank, fb, pi, pj = _oracle_pivots(ref)
    say("oracle blocks", len(ref.blocks), "fallbacks", int(fb.sum()), "rank sum", int(rank.sum()))
    if l_max == 3:
        assert fb.sum() > 0
    fdt = torch.float64 if prec == "fp64" else torch.float32
    tree = hh.build_tree(ctx(), dev(X), 64)
    part = hh.partition(ctx(), tree, 1.0)
    G, _ = part.export()
    assert np.array_equal(G, np.asarray(ref.G))
    lr = hh.aca_build_pivots(ctx(), tree, part, kg, prec, rank, fb, pi, pj)
    assert lr.info()["n_fallback"] == int(fb.sum())
    dF, dX, dth = hh.matvec_backward(ctx(), tree, part, lr, kg, dev(F, fdt), dev(w, fdt), prec)
    rF, rX, rW, rb = OG.hmatvec_grad(ref, X, F, w, ko)
    rth = hh.pack_mlp((rW, rb))
    got = {"dF": dF.double().cpu().numpy(), "dX": dX.cpu().numpy(), "dtheta": dth.cpu().numpy()}
    want = {"dF": rF, "dX": rX, "dtheta": rth}
    errs = {k: (_rel(got[k], want[k]), _maxrel(got[k], want[k])) for k in got}
    say(prec, "l_max", l_max, errs)
    # the forward of the same factors against the oracle's frozen product
    U = hh.matvec(ctx(), tree, part, lr, kg, dev(F, fdt), prec).double().cpu().numpy()
    eU = _rel(U, OH.apply(ref, X, F, ko))
    say("forward on oracle pivots", eU)
    if prec == "fp64":
        assert eU < 1e-13
        assert errs["dF"][0] < 1e-13 and errs["dF"][1] < 1e-13
        assert all(errs[k][0] < 1e-11 and errs[k][1] < 1e-11 for k in ("dX", "dtheta"))
    else:
        assert eU < 2e-5
        assert errs["dF"][0] < 2e-5 and errs["dF"][1] < 2e-5
        assert all(errs[k][0] < 2e-3 and errs[k][1] < 1e-2 for k in ("dX", "dtheta"))


def test_fp32_pivots_against_oracle_determinant_rule():
    """The single-precision search picks the pivots of the oracle's |det| rule
    on (nearly) every block; the share that match is reported."""
    from gpu_common import ctx, dev, kernels, say
    X = wl.rsa_cube(4000, 0.2, seed=0)
    ko, kg = kernels("mlp")
    ref = OH.build(X, ko, 64, 1.0, 1e-4, 48, pivot="determinant")
    share = {}
    for prec in ("fp32", "bf16"):
        hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, eta=1.0, eps=1e-4, prec=prec)
        ex = hm.lr.export()
        same = same_rank = 0
        for b, blk in enumerate(ref.blocks):
            if blk is None:
                continue
            m = min(ex["rank"][b], blk.rank)
            if np.array_equal(ex["piv_i"][b, :m], blk.piv_i[:m]) and \
                    np.array_equal(ex["piv_j"][b, :m], blk.piv_j[:m]):
                same += 1
                same_rank += int(ex["rank"][b] == blk.rank)
        nb = sum(b is not None for b in ref.blocks)
        say(prec, "blocks", nb, "pivot match share", same / nb, "and same rank", same_rank / nb)
        share[prec] = same / nb
    # a near tie of two candidates' |det| may go either way in single
    # precision, and the factors differ from there on; the products agree to
    # the ACA tolerance either way (accuracy tests)
    assert share["fp32"] >= 0.75 and share["bf16"] >= 0.15


def _golden_grad():
    d = np.load(os.path.join(GOLDEN, "grad_diff_5k.npz"))
    return d


def test_backward_dense_gradient_5k():
    """The H-matrix gradient (its own ACA, zeta = 1e-4) against the dense FP64
    gradient of the exact product: dF within 10 zeta, dX and dtheta within
    100 zeta (relative 2-norm), FP64 and FP32 forms."""
    from gpu_common import ctx, dev, kernels, say
    X, F, cfg = wl.workload("diff_5k")
    g = _golden_grad()
    w = wl.normal_forces(X.shape[0], seed=int(g["w_seed"]))
    assert _digest(X) == str(g["sha_X"]) and _digest(F) == str(g["sha_F"])
    assert _digest(w) == str(g["sha_w"])
    _, kg = kernels("mlp")
    zeta = cfg["eps"]
    for prec in ("fp64", "fp32"):
        fdt = torch.float64 if prec == "fp64" else torch.float32
        hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=cfg["c_leaf"], eta=1.0, eps=zeta, prec=prec)
        dF, dX, dth = hh.matvec_backward(ctx(), hm.tree, hm.part, hm.lr, kg, dev(F, fdt),
                                         dev(w, fdt), prec)
        eF = _rel(dF.double().cpu().numpy(), g["dF"])
        eX = _rel(dX.cpu().numpy(), g["dX"])
        et = _rel(dth.cpu().numpy(), g["dtheta"])
        say(prec, "vs dense gradient: dF", eF, "dX", eX, "dtheta", et,
            "max", _maxrel(dX.cpu().numpy(), g["dX"]), hm.lr.info())
        assert eF <= 10 * zeta and eX <= 100 * zeta and et <= 100 * zeta


def test_backward_finite_differences_frozen_5k():
    """Central differences (h = 1e-4) of the frozen FP64 GPU product at 64
    coordinates each of X, F and theta (seed 4) against the backward: the
    tree, partition, pivots and fallbacks stay those of the unperturbed
    build (hh_tree_refit, freeze_pivots_from). Each coordinate within 1e-6 of
    the largest gradient entry of its kind (FD truncation ~h^2, rounding of
    L ~1e-16 |L| / h). The pivots are those of the |det| search (an FP32
    build) replayed in FP64: the largest-Frobenius pivots of the FP64 search
    can be nearly singular 3x3 entries for this indefinite kernel, and a
    perturbation of theta moves every entry, so P^-1 would change faster than
    a difference step resolves."""
    from gpu_common import ctx, dev, kernels, mlp_params, say
    X, F, cfg = wl.workload("diff_5k")
    n = X.shape[0]
    w = wl.normal_forces(n, seed=5)
    _, kg = kernels("mlp")
    theta = hh.pack_mlp(mlp_params())
    hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=cfg["c_leaf"], eta=1.0, eps=cfg["eps"], prec="fp32")
    lr0 = hh.aca_build(ctx(), hm.tree, hm.part, kg, "fp64", freeze_pivots_from=hm.lr)
    Fd, wd = dev(F), dev(w)
    dF, dX, dth = hh.matvec_backward(ctx(), hm.tree, hm.part, lr0, kg, Fd, wd, "fp64")
    dF, dX, dth = dF.cpu().numpy(), dX.cpu().numpy(), dth.cpu().numpy()

    def loss(lr, kern, Fv=Fd):
        U = hh.matvec(ctx(), hm.tree, hm.part, lr, kern, Fv, "fp64")
        return float(torch.sum(wd * U).item())

    h = 1e-4
    rng = wl.Rng(4, "fd")
    pts = (rng.raw(64) % (3 * n)).astype(np.int64)
    worst = {"X": 0.0, "F": 0.0, "theta": 0.0}
    say("fd: backward done, blocks", lr0.info())
    for a_, p in enumerate(pts):
        if a_ % 16 == 0:
            say("fd X", a_)
        i, d = divmod(int(p), 3)
        vals = []
        for sgn in (1.0, -1.0):
            Xp = X.copy()
            Xp[i, d] += sgn * h
            hh.tree_refit(ctx(), hm.tree, dev(Xp))
            lr = hh.aca_build(ctx(), hm.tree, hm.part, kg, "fp64", freeze_pivots_from=lr0)
            vals.append(loss(lr, kg))
        fd = (vals[0] - vals[1]) / (2 * h)
        worst["X"] = max(worst["X"], abs(fd - dX[i, d]) / np.max(np.abs(dX)))
    hh.tree_refit(ctx(), hm.tree, dev(X))
    for p in pts:
        i, d = divmod(int(p), 3)
        vals = []
        for sgn in (1.0, -1.0):
            Fp = F.copy()
            Fp[i, d] += sgn * h
            vals.append(loss(lr0, kg, dev(Fp)))
        fd = (vals[0] - vals[1]) / (2 * h)
        worst["F"] = max(worst["F"], abs(fd - dF[i, d]) / np.max(np.abs(dF)))
    say("fd F done", worst)
    tpts = (wl.Rng(4, "misc").raw(64) % theta.size).astype(np.int64)
    for a_, p in enumerate(tpts):
        if a_ % 16 == 0:
            say("fd theta", a_)
        vals = []
        for sgn in (1.0, -1.0):
            th = theta.copy()
            th[p] += sgn * h
            k2 = hh.Kernel.mlp(ctx(), th, "direction")
            lr = hh.aca_build(ctx(), hm.tree, hm.part, k2, "fp64", freeze_pivots_from=lr0)
            vals.append(loss(lr, k2))
        fd = (vals[0] - vals[1]) / (2 * h)
        worst["theta"] = max(worst["theta"], abs(fd - dth[p]) / np.max(np.abs(dth)))
    say("finite differences, worst error relative to the largest entry", worst)
    assert all(v <= 1e-6 for v in worst.values())


def test_backward_sampled_rows_50k():
    """The FP32 backward on the differentiation workload's geometry (cube,
    15% volume fraction) at N = 50,000: rows of dF and dX at 16 sampled
    particles against the dense FP64 gradient rows (oracle.grad.
    dense_grad_rows): within 10 zeta and 100 zeta. (The full N = 200,000 is
    timed by bench.py --workload diff_200k --backward.)"""
    from gpu_common import ctx, dev, kernels, say
    X, F, cfg = wl.workload("diff_200k", 50000)
    n = X.shape[0]
    w = wl.normal_forces(n, seed=5)
    ko, kg = kernels("mlp")
    ctx().set_budget(200 << 30)   # stored factors (the backward needs them)
    try:
        hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=cfg["c_leaf"], eta=1.0, eps=cfg["eps"],
                        prec="fp32")
    finally:
        ctx().set_budget(64 << 30)
    dF, dX, _ = hh.matvec_backward(ctx(), hm.tree, hm.part, hm.lr, kg, dev(F, torch.float32),
                                   dev(w, torch.float32), "fp32", want=("F", "X"))
    rows = wl.sample_rows(n, 16, seed=3)
    rF, rX = OG.dense_grad_rows(X, F, w, ko, rows)
    eF = _rel(dF.double().cpu().numpy()[rows], rF)
    eX = _rel(dX.cpu().numpy()[rows], rX)
    say("50k sampled rows: dF", eF, "dX", eX, hm.lr.info())
    assert eF <= 10 * cfg["eps"] and eX <= 100 * cfg["eps"]


def test_autograd_wrapper():
    """torch.autograd through HMatvecFn returns the oracle adjoint."""
    from gpu_common import ctx, dev, kernels, say
    X, F, w, c_leaf, eps = _case(n=400, c_leaf=32, eps=1e-6, seed=8)
    ko, _ = kernels("mlp")
    theta = torch.tensor(hh.pack_mlp(wl.mlp_weights(1)), dtype=torch.float64, requires_grad=True)
    Xt = dev(X).requires_grad_(True)
    Ft = dev(F).requires_grad_(True)
    U = hh.hmatvec_autograd(ctx(), Xt, Ft, theta, c_leaf=c_leaf, eps=eps, prec="fp64")
    L = torch.sum(dev(w) * U)
    L.backward()
    ref = OH.build(X, ko, c_leaf, 1.0, eps, 48)
    rF, rX, rW, rb = OG.hmatvec_grad(ref, X, F, w, ko)
    e = (_rel(Ft.grad.cpu().numpy(), rF), _rel(Xt.grad.cpu().numpy(), rX),
         _rel(theta.grad.numpy(), hh.pack_mlp((rW, rb))))
    say("autograd vs oracle adjoint", e)
    assert max(e) < 1e-8
