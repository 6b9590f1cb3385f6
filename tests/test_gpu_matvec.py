"""GPU parity of the H-matrix product against the FP64 oracle.

* dense mode (no admissible block) reproduces the exact dense sum: FP64
  within 1e-10 relative (RPY and MLP);
* FP64 H-matvec with RPY at zeta = 1e-6 is within 10 zeta of the dense sum
  and within zeta of the oracle's own H-matrix product (a borderline stopping
  test may add or drop one term of size ~zeta lambda), with the ACA pivots and
  ranks equal to the oracle's on (almost) every block;
* FP32 with the MLP kernel within 1e-3 of the dense sum;
* where the pivots agree with the oracle's, the factors c_k, q_k agree with
  the oracle's to rounding, scaled by (k + 1)^2, lambda_k / nu_k and the
  condition of the pivot entries met so far (Frobenius, per factor);
* every product test bounds the worst particle's error as well as the 2-norm.
"""
import numpy as np
import pytest
import torch

import paper_2505_08174_amd as hh
import workloads as wl
from oracle import dense as OD
from oracle import hmatvec as OH

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _row(a, b):
    """Largest per-particle error relative to the largest reference row."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.linalg.norm(a - b, axis=1)) / np.max(np.linalg.norm(b, axis=1)))


@pytest.mark.parametrize("kind", ["rpy", "mlp"])
def test_dense_mode_fp64(kind):
    from gpu_common import ctx, dev, kernels, say
    say("dense mode fp64", kind)
    n = 2000 if kind == "rpy" else 700
    X = wl.rsa_cube(n, 0.1, seed=0)
    F = wl.normal_forces(n, seed=0)
    ko, kg = kernels(kind)
    Ud = OD.dense_u(X, F, ko)
    hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, prec="fp64", dense_mode=True)
    U = (hm @ dev(F)).cpu().numpy()
    assert _rel(U, Ud) < 1e-10 and _row(U, Ud) < 1e-10


@pytest.mark.parametrize("inp", ["direction", "displacement"])
def test_dense_mode_fp32_mlp(inp):
    """The plain FP32 form's near field (the MLP on FP32 MFMA tiles, FP32
    operands and accumulation) over every pair. Per entry the FP32 rounding
    of four layers of 64-term sums is a few 1e-7; the sum over sources adds at
    most the ratio sum|K F| / |sum K F| (below ~10 for these forces), so the
    bound is 1e-5 on the 2-norm and on the worst particle."""
    from gpu_common import ctx, dev, kernels, say
    n = 900
    X = wl.rsa_cube(n, 0.1, seed=2)
    F = wl.normal_forces(n, seed=2)
    ko, kg = kernels("mlp", inp)
    Ud = OD.dense_u(X, F, ko)
    hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, prec="fp32", dense_mode=True)
    U = (hm @ dev(F, torch.float32)).double().cpu().numpy()
    say("dense mode fp32 mlp", inp, "rel", _rel(U, Ud), "worst row", _row(U, Ud))
    assert _rel(U, Ud) < 1e-5 and _row(U, Ud) < 1e-5


def test_hmatvec_fp64_rpy_plain_small():
    from gpu_common import ctx, dev, kernels, say
    say("plain small fp64 rpy")
    X, F, cfg = wl.workload("plain_small")
    ko, kg = kernels("rpy")
    Ud = OD.dense_u(X, F, ko)
    hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, eta=1.0, eps=1e-6, prec="fp64")
    U = (hm @ dev(F)).cpu().numpy()
    e = _rel(U, Ud)
    say("eps_r", e, "worst row", _row(U, Ud))
    assert e <= 1e-5 and _row(U, Ud) <= 1e-5
    # against the oracle's literal H-matrix product: pivots and ranks first
    ref = OH.build(X, ko, 64, 1.0, 1e-6, 48)
    ex = hm.lr.export()
    ranks = np.array([0 if b is None else b.rank for b in ref.blocks])
    same = same_piv = 0
    for b, blk in enumerate(ref.blocks):
        r = ex["rank"][b]
        if blk is None:
            continue
        m = min(r, blk.rank)
        if np.array_equal(ex["piv_i"][b, :m], blk.piv_i[:m]) and \
                np.array_equal(ex["piv_j"][b, :m], blk.piv_j[:m]):
            same_piv += 1
            same += int(r == blk.rank)
    say("blocks", len(ref.blocks), "same pivots", same_piv, "same pivots and rank", same,
        "rank sums", int(ex["rank"].sum()), int(ranks.sum()))
    assert same_piv >= 0.99 * len(ref.blocks)
    assert same >= 0.95 * len(ref.blocks)
    assert ex["fallback"].sum() == ref.n_fallback
    # a borderline stopping test may end a block one term earlier or later
    # (a term of size ~ zeta * lambda), so the two H products agree to ~zeta
    Uo = OH.apply(ref, X, F, ko)
    d = _rel(U, Uo)
    say("gpu vs oracle H", d, "worst row", _row(U, Uo))
    assert d < 1e-6 and _row(U, Uo) < 1e-6


def test_factors_match_oracle_fp64():
    from gpu_common import ctx, dev, kernels, say
    say("factors fp64")
    X = wl.rsa_cube(1500, 0.15, seed=5)
    ko, kg = kernels("rpy")
    hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=32, eta=1.0, eps=1e-5, prec="fp64")
    ref = OH.build(X, ko, 32, 1.0, 1e-5, 48)
    ex = hm.lr.export()
    t = ref.tree
    checked = 0
    worst = 0.0
    for b in range(0, len(ref.blocks), max(1, len(ref.blocks) // 25)):
        blk = ref.blocks[b]
        r = ex["rank"][b]
        if blk is None or r != blk.rank or not np.array_equal(ex["piv_i"][b, :r], blk.piv_i):
            continue
        tau, sig = ref.G[b]
        c = t.nodes[tau, 1] - t.nodes[tau, 0]
        q = t.nodes[sig, 1] - t.nodes[sig, 0]
        # condition of the pivot entries P_m = q_m(j_m) met so far
        conds = np.maximum.accumulate([np.linalg.cond(blk.Q[m][blk.piv_j[m]]) for m in range(r)])
        for k in range(r):
            ck, qk = hm.lr.factor(b, k, c, q)
            # Bound: the residual of step k is entries of size ~lambda minus
            # k earlier terms, so its absolute rounding error is ~k u lambda,
            # and every earlier term carries the error of its own step into
            # it (~k^2 u lambda after k steps); term k is cut from a residual
            # of size ~nu_k, and the solve with P_k scales by cond(P_k):
            # rel(c_k), rel(q_k) <= C (k + 1)^2 u cond_k max(1, lambda_k / nu_k),
            # u = 2^-53; C = 16 covers the constants of the 3x3 products and
            # of the adjugate inverse
            bound = (k + 1) ** 2 * U64 * conds[k] * max(1.0, np.sqrt(blk.lam2[k] / blk.nu2[k]))
            rc, rq = _rel(ck, blk.C[k]), _rel(qk, blk.Q[k])
            worst = max(worst, rc / bound, rq / bound)
            assert rc <= 16 * bound, (b, k, rc, bound)
            assert rq <= 16 * bound, (b, k, rq, bound)
        checked += 1
    say("factors: worst error / (k^2 u cond lambda/nu)", worst)
    assert checked >= 5


@pytest.mark.parametrize("inp", ["direction", "displacement"])
def test_hmatvec_fp32_mlp(inp):
    from gpu_common import ctx, dev, kernels, say
    say("fp32 mlp", inp)
    n = 4000
    X = wl.rsa_cube(n, 0.2, seed=0)
    F = wl.normal_forces(n, seed=0)
    ko, kg = kernels("mlp", inp)
    rows = wl.sample_rows(n, 300)
    Ud = OD.dense_u(X, F, ko, rows)
    hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, eta=1.0, eps=1e-4, prec="fp32")
    U = (hm @ dev(F, torch.float32)).cpu().numpy().astype(np.float64)
    e = _rel(U[rows], Ud)
    say("eps_r", e, "worst row", _row(U[rows], Ud), hm.lr.info())
    assert e <= 1e-3 and _row(U[rows], Ud) <= 1e-3


def test_hmatvec_edge_sizes():
    from gpu_common import ctx, dev, kernels, say
    ko, kg = kernels("rpy")
    for n in (1, 2, 5, 64, 65, 300):
        say("edge", n)
        X = wl.rsa_cube(n, 0.05, seed=n) if n > 1 else np.zeros((1, 3))
        F = wl.normal_forces(n, seed=n)
        hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=8, eps=1e-8, prec="fp64")
        U = (hm @ dev(F)).cpu().numpy()
        Ud = OD.dense_u(X, F, ko)
        assert _rel(U, Ud) < 1e-6 and _row(U, Ud) < 1e-6


@pytest.mark.parametrize("kind,prec,n,eps,tol,l_max", [("rpy", "fp64", 2000, 1e-6, 1e-12, 48),
                                                       ("mlp", "fp32", 4000, 1e-4, 2e-5, 48),
                                                       ("mlp", "fp32", 4000, 1e-4, 2e-5, 2),
                                                       ("mlp", "bf16", 4000, 1e-4, 2e-5, 2)])
def test_streamed_equals_stored(kind, prec, n, eps, tol, l_max):
    """Batches of blocks with the apply fused into the ACA (factors discarded)
    give the product of the stored factors, to rounding of the summation order.
    l_max = 2 makes most blocks fall back, so the fused path's dense
    evaluation of fallback blocks is checked too, also against the dense sum."""
    from gpu_common import ctx, dev, kernels, say
    say("streamed vs stored", kind, prec, n, l_max)
    X = wl.rsa_cube(n, 0.15, seed=1)
    F = wl.normal_forces(n, seed=1)
    ko, kg = kernels(kind)
    fdt = torch.float64 if prec == "fp64" else torch.float32
    hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, eta=1.0, eps=eps, prec=prec, l_max=l_max)
    U1 = (hm @ dev(F, fdt)).double().cpu().numpy()
    info1 = hm.lr.info()
    ctx().set_budget(2 << 20)           # 2 MiB: forces many small batches
    try:
        hs = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, eta=1.0, eps=eps, prec=prec, l_max=l_max)
        U2 = (hs @ dev(F, fdt)).double().cpu().numpy()
        info2 = hs.lr.info()
    finally:
        ctx().set_budget(64 << 30)
    say("stored", info1, "streamed", info2, "diff", _rel(U2, U1), "worst row", _row(U2, U1))
    assert info2["n_blocks"] == info1["n_blocks"]
    assert abs(info2["rank_sum"] - info1["rank_sum"]) <= 0.002 * info1["rank_sum"]
    assert info2["n_fallback"] == info1["n_fallback"]
    if l_max == 2:
        assert info1["n_fallback"] >= 0.5 * info1["n_blocks"]
        rows = wl.sample_rows(n, 200, seed=4)
        Ud = OD.dense_u(X, F, ko, rows)
        e = _rel(U2[rows], Ud)
        say("fallback-heavy streamed vs dense", e)
        assert e <= (5e-3 if prec == "bf16" else 1e-3)
    assert _rel(U2, U1) < tol and _row(U2, U1) < 10 * tol
    with pytest.raises(hh.HHError, match="streamed"):
        hs.lr.factor(0, 0, 1, 1)


@pytest.mark.parametrize("inp", ["direction", "displacement"])
def test_bf16_dense_mode(inp):
    """BF16 MFMA near field (every leaf pair dense) against the FP64 dense sum.
    Split BF16 weights keep the error far below the 5e-3 bar."""
    from gpu_common import ctx, dev, kernels, say
    n = 3000
    X = wl.rsa_cube(n, 0.2, seed=2)
    F = wl.gravity_forces(n, seed=2)
    ko, kg = kernels("mlp", inp)
    hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, prec="bf16", dense_mode=True)
    U = (hm @ dev(F, torch.float32)).cpu().numpy()
    assert U.dtype == np.float64
    rows = wl.sample_rows(n, 400, seed=3)
    Ud = OD.dense_u(X, F, ko, rows)
    e = _rel(U[rows], Ud)
    say("bf16 dense mode", inp, e, "worst row", _row(U[rows], Ud))
    assert e <= 5e-4 and _row(U[rows], Ud) <= 5e-4


def test_bf16_hmatvec():
    from gpu_common import ctx, dev, kernels, say
    n = 8000
    X = wl.lattice_sphere(n, 0.1, seed=0)
    F = wl.gravity_forces(n, seed=0)
    ko, kg = kernels("mlp")
    hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=128, eta=1.0, eps=1e-4, prec="bf16")
    U = (hm @ dev(F, torch.float32)).cpu().numpy()
    rows = wl.sample_rows(n, 300, seed=3)
    Ud = OD.dense_u(X, F, ko, rows)
    e = _rel(U[rows], Ud)
    say("bf16 hmatvec", e, "worst row", _row(U[rows], Ud), hm.lr.info())
    assert e <= 5e-3 and _row(U[rows], Ud) <= 5e-3


@pytest.mark.parametrize("kind,prec,eps,tol", [("rpy", "fp64", 1e-6, 1e-5),
                                               ("mlp", "bf16", 1e-4, 5e-3)])
def test_workgroup_teams_match_single_waves(kind, prec, eps, tol):
    """Blocks approximated by whole workgroups (the threshold lowered so that
    every block takes that path) follow the same pivots and ranks as the
    single-wave path: only the order of the Gram sums differs, so a rank can
    change only where the stopping test is a near tie. Stored and streamed
    (fused apply) both checked, and the dense sum within the form's bound."""
    from gpu_common import ctx, dev, kernels, say
    n = 6000
    X = wl.rsa_cube(n, 0.15, seed=4)
    F = wl.gravity_forces(n, seed=4)
    ko, kg = kernels(kind)
    fdt = torch.float64 if prec == "fp64" else torch.float32
    hm1 = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, eps=eps, prec=prec)
    U1 = (hm1 @ dev(F, fdt)).double().cpu().numpy()
    r1 = hm1.lr.export()["rank"] if prec == "fp64" else None
    ctx().set_team_min(64)
    try:
        hm2 = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, eps=eps, prec=prec)
        U2 = (hm2 @ dev(F, fdt)).double().cpu().numpy()
        ctx().set_budget(2 << 20)
        hm3 = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, eps=eps, prec=prec)
        U3 = (hm3 @ dev(F, fdt)).double().cpu().numpy()
    finally:
        ctx().set_team_min(4096)
        ctx().set_budget(64 << 30)
    rows = wl.sample_rows(n, 300, seed=5)
    Ud = OD.dense_u(X, F, ko, rows)
    say("teams", kind, prec, "vs waves", _rel(U2, U1), "streamed", _rel(U3, U1),
        "dense", _rel(U2[rows], Ud), _rel(U3[rows], Ud))
    if r1 is not None:
        r2 = hm2.lr.export()["rank"]
        assert np.mean(r1 == r2) >= 0.999
    assert hm2.lr.info()["n_fallback"] == hm1.lr.info()["n_fallback"]
    assert _rel(U2, U1) < 10 * eps
    assert _rel(U3, U1) < 10 * eps
    assert _rel(U2[rows], Ud) <= tol and _rel(U3[rows], Ud) <= tol
    assert _row(U2[rows], Ud) <= tol and _row(U3[rows], Ud) <= tol


def test_bf16_split_dense_mode():
    """Near field with hi + lo BF16 activations: per-entry error ~1e-6, far
    below the once-rounded BF16 near field."""
    from gpu_common import ctx, dev, kernels, say
    n = 3000
    X = wl.rsa_cube(n, 0.2, seed=2)
    F = wl.normal_forces(n, seed=2)
    ko, kg = kernels("mlp")
    rows = wl.sample_rows(n, 400, seed=3)
    Ud = OD.dense_u(X, F, ko, rows)
    errs = {}
    for prec in ("bf16", "bf16_split"):
        hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, prec=prec, dense_mode=True)
        U = (hm @ dev(F, torch.float32)).cpu().numpy()
        errs[prec] = _rel(U[rows], Ud)
    say("dense mode, random forces", errs)
    assert errs["bf16_split"] <= 5e-5
    assert errs["bf16_split"] < errs["bf16"]


def test_bf16_split_as_accurate_as_fp32():
    """With zero-mean random forces (no coherent flow to hide the kernel
    error) the split BF16 form reaches the plain FP32 form's accuracy."""
    from gpu_common import ctx, dev, kernels, say
    n = 8000
    X = wl.rsa_cube(n, 0.2, seed=6)
    F = wl.normal_forces(n, seed=6)
    ko, kg = kernels("mlp")
    rows = wl.sample_rows(n, 300, seed=3)
    Ud = OD.dense_u(X, F, ko, rows)
    errs = {}
    for prec in ("fp32", "bf16_split", "bf16"):
        hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, eta=1.0, eps=1e-4, prec=prec)
        U = (hm @ dev(F, torch.float32)).double().cpu().numpy()
        errs[prec] = _rel(U[rows], Ud)
    say("eps_r by form", errs)
    assert errs["bf16_split"] <= max(2 * errs["fp32"], 1e-4)
    assert errs["bf16"] <= 5e-3
