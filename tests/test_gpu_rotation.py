"""GPU parity of the 6N mobility product [U; w] = M [F; T] (forces and torques).

The library's 6N kernel on a tree of hh_build_tree6 against the oracle's
dense 6N product and its H-matrix over the grid of 3x3 entries:
* dense mode (no admissible block): FP64 within 1e-10 of the dense sum;
* FP64 at zeta = 1e-6: within 10 zeta of the dense sum (Eq. (11) over all 6N
  components, and per particle), pivots and ranks equal to the oracle's
  H-matrix on (almost) every block, and within zeta of its product;
* FP32: within 1e-4 of the dense sum (the FP32 RPY entries carry ~1e-7
  relative rounding; the |det| pivots keep c_k = a P^-1 well conditioned);
* the pivot replay, the workgroup-team ACA, the streamed (fused) product with
  its dense fallbacks and the allocation-free product agree with the stored
  product;
* refit at unchanged positions keeps the product;
* 1, 2, 5, 65 and 400 particles in two-particle leaves, FP64 and FP32, against
  the dense sum;
* the 6N kernel is refused on a particle tree (and a 3N kernel on a 6N tree),
  in BF16, in the backward and in the short-range terms.
"""
import numpy as np
import pytest
import torch

import paper_2505_08174_amd as hh
import workloads as wl
from oracle import rotation as OR

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _row(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.linalg.norm(a - b, axis=1)) / np.max(np.linalg.norm(b, axis=1)))


def _case(n, seed=3, phi=0.2):
    X = wl.rsa_cube(n, phi, seed=seed)
    F = wl.normal_forces(n, seed=seed + 1)
    T = wl.normal_forces(n, seed=seed + 2)
    return X, F, T


def _ref(X, F, T, rows=None):
    U, W = OR.u6(X, F, T, rows=rows)
    return np.hstack([U, W])


def _g6(F, T, dtype=torch.float64):
    from gpu_common import dev
    return dev(np.hstack([F, T]), dtype)


def test_dense_mode_fp64():
    from gpu_common import ctx, dev, say
    say("6N dense mode fp64")
    X, F, T = _case(1200)
    k6 = hh.Kernel.rpy6(ctx())
    hm = hh.HMatrix(ctx(), dev(X), k6, c_leaf=32, prec="fp64", dense_mode=True)
    assert hm.tree.info()[0] == 2 * 1200
    Y = (hm @ _g6(F, T)).cpu().numpy()
    ref = _ref(X, F, T)
    say("rel", _rel(Y, ref), "worst row", _row(Y, ref))
    assert Y.shape == (1200, 6)
    assert _rel(Y, ref) < 1e-10 and _row(Y, ref) < 1e-10


def test_hmatvec6_fp64_against_dense_and_oracle_hmatrix():
    from gpu_common import ctx, dev, say
    say("6N fp64 eps 1e-6 n=1500")
    n = 1500
    X, F, T = _case(n)
    k6 = hh.Kernel.rpy6(ctx())
    hm = hh.HMatrix(ctx(), dev(X), k6, c_leaf=32, eta=1.0, eps=1e-6, prec="fp64")
    Y = (hm @ _g6(F, T)).cpu().numpy()
    ref = _ref(X, F, T)
    e = _rel(Y, ref)
    say("eps_r", e, "worst row", _row(Y, ref), "U", _rel(Y[:, :3], ref[:, :3]),
        "w", _rel(Y[:, 3:], ref[:, 3:]))
    assert e <= 1e-5 and _row(Y, ref) <= 1e-5
    assert _rel(Y[:, 3:], ref[:, 3:]) <= 1e-5
    # the oracle's H-matrix on the same 6N grid: pivots, ranks, fallbacks
    say("oracle 6N H-matrix")
    o = OR.build6(X, 32, 1.0, 1e-6, 48)
    ex = hm.lr.export()
    assert len(o.blocks) == ex["rank"].shape[0]
    same = same_piv = 0
    for b, blk in enumerate(o.blocks):
        if blk is None:
            continue
        r = ex["rank"][b]
        m = min(r, blk.rank)
        if np.array_equal(ex["piv_i"][b, :m], blk.piv_i[:m]) and \
                np.array_equal(ex["piv_j"][b, :m], blk.piv_j[:m]):
            same_piv += 1
            same += int(r == blk.rank)
    nb = sum(b is not None for b in o.blocks)
    say("blocks", len(o.blocks), "same pivots", same_piv, "and rank", same, "fallbacks",
        int(ex["fallback"].sum()), o.n_fallback)
    assert same_piv >= 0.99 * nb and same >= 0.95 * nb
    assert ex["fallback"].sum() == o.n_fallback
    Uo, Wo = OR.apply6(o, X, F, T)
    d = _rel(Y, np.hstack([Uo, Wo]))
    say("vs oracle H-matrix", d)
    assert d < 1e-6


def test_hmatvec6_fp32():
    from gpu_common import ctx, dev, say
    say("6N fp32 eps 1e-5 n=4000")
    n = 4000
    X, F, T = _case(n, seed=7)
    k6 = hh.Kernel.rpy6(ctx())
    hm = hh.HMatrix(ctx(), dev(X), k6, c_leaf=64, eps=1e-5, prec="fp32")
    Y = (hm @ _g6(F, T, torch.float32)).double().cpu().numpy()
    rows = wl.sample_rows(n, 400, seed=2)
    ref = _ref(X, F, T, rows)
    say("eps_r", _rel(Y[rows], ref), "worst row", _row(Y[rows], ref), "info", hm.lr.info())
    assert _rel(Y[rows], ref) <= 1e-4 and _row(Y[rows], ref) <= 1e-4


@pytest.mark.parametrize("prec,l_max", [("fp64", 48), ("fp32", 48), ("fp64", 2)])
def test_paths_agree(prec, l_max):
    """Replayed pivots, workgroup teams, the streamed product (l_max = 2: most
    blocks fall back and are evaluated densely inside the fused apply) and
    the allocation-free product against the stored product."""
    from gpu_common import ctx, dev, say
    say("6N paths", prec, l_max)
    n = 5000
    X, F, T = _case(n, seed=11, phi=0.15)
    k6 = hh.Kernel.rpy6(ctx())
    fdt = torch.float64 if prec == "fp64" else torch.float32
    tol = 1e-12 if prec == "fp64" else 2e-5
    G = _g6(F, T, fdt)
    hm = hh.HMatrix(ctx(), dev(X), k6, c_leaf=64, eps=1e-6 if prec == "fp64" else 1e-5,
                    prec=prec, l_max=l_max)
    Y1 = (hm @ G).double().cpu().numpy()
    info1 = hm.lr.info()
    # pivot replay (the recursion recomputed with the exported pivots)
    lr2 = hh.aca_build(ctx(), hm.tree, hm.part, k6, prec, freeze_pivots_from=hm.lr)
    Y2 = hh.matvec(ctx(), hm.tree, hm.part, lr2, k6, G, prec).double().cpu().numpy()
    # allocation-free product
    Y3 = torch.empty_like(G, dtype=torch.float64 if prec == "fp64" else torch.float32)
    hh.matvec_noalloc(ctx(), hm.tree, hm.part, hm.lr, k6, G, Y3, prec)
    Y3 = Y3.double().cpu().numpy()
    ctx().set_team_min(64)
    try:
        hmt = hh.HMatrix(ctx(), dev(X), k6, c_leaf=64, eps=1e-6 if prec == "fp64" else 1e-5,
                         prec=prec, l_max=l_max)
        Y4 = (hmt @ G).double().cpu().numpy()
        ctx().set_budget(2 << 20)
        hms = hh.HMatrix(ctx(), dev(X), k6, c_leaf=64, eps=1e-6 if prec == "fp64" else 1e-5,
                         prec=prec, l_max=l_max)
        Y5 = (hms @ G).double().cpu().numpy()
        info5 = hms.lr.info()
    finally:
        ctx().set_team_min(4096)
        ctx().set_budget(64 << 30)
    say("info", info1, "replay", _rel(Y2, Y1), "noalloc", _rel(Y3, Y1), "teams", _rel(Y4, Y1),
        "streamed", _rel(Y5, Y1), info5)
    assert np.array_equal(Y3, Y1)
    assert _rel(Y2, Y1) < tol
    assert info5["n_blocks"] == info1["n_blocks"] and info5["n_fallback"] == info1["n_fallback"]
    if l_max == 2:
        assert info1["n_fallback"] >= 0.5 * info1["n_blocks"]
    assert _rel(Y5, Y1) < 10 * tol
    eps = 1e-6 if prec == "fp64" else 1e-5
    assert _rel(Y4, Y1) < 10 * eps
    rows = wl.sample_rows(n, 300, seed=6)
    ref = _ref(X, F, T, rows)
    bound = 1e-5 if prec == "fp64" else 1e-4
    for Y in (Y1, Y2, Y4, Y5):
        assert _rel(Y[rows], ref) <= bound and _row(Y[rows], ref) <= bound


def test_refit_keeps_product():
    from gpu_common import ctx, dev, say
    say("6N refit")
    X, F, T = _case(2000, seed=13)
    k6 = hh.Kernel.rpy6(ctx())
    hm = hh.HMatrix(ctx(), dev(X), k6, c_leaf=32, eps=1e-6, prec="fp64")
    Y1 = (hm @ _g6(F, T)).cpu().numpy()
    hh.tree_refit(ctx(), hm.tree, dev(X))
    lr = hh.aca_build(ctx(), hm.tree, hm.part, k6, "fp64", freeze_pivots_from=hm.lr)
    Y2 = hh.matvec(ctx(), hm.tree, hm.part, lr, k6, _g6(F, T), "fp64").cpu().numpy()
    assert _rel(Y2, Y1) < 1e-13


def test_refusals():
    from gpu_common import ctx, dev, kernels, say
    say("6N refusals")
    X, F, T = _case(600, seed=17)
    k6 = hh.Kernel.rpy6(ctx())
    _, k3 = kernels("rpy")
    t3 = hh.build_tree(ctx(), dev(X), 32)
    p3 = hh.partition(ctx(), t3)
    with pytest.raises(hh.HHError, match="6N"):
        hh.aca_build(ctx(), t3, p3, k6, "fp64")
    t6 = hh.build_tree6(ctx(), dev(X), 32)
    p6 = hh.partition(ctx(), t6)
    assert t6.info()[0] == 1200 and t6.info()[1:] == t3.info()[1:]
    assert p6.info() == p3.info()
    with pytest.raises(hh.HHError, match="6N"):
        hh.aca_build(ctx(), t6, p6, k3, "fp64")
    with pytest.raises(hh.HHError, match="6N"):
        hh.aca_build(ctx(), t6, p6, k6, "bf16")
    lr = hh.aca_build(ctx(), t6, p6, k6, "fp64")
    with pytest.raises(hh.HHError, match="3N"):
        hh.matvec_backward(ctx(), t6, p6, lr, k6, _g6(F, T).view(-1, 3),
                           torch.ones(1200, 3, dtype=torch.float64, device="cuda:0"), "fp64",
                           want=("F",))
    s2, g3 = wl.mlp_weights(11), wl.mlp_weights(12, widths=(6, 64, 64, 64, 18))
    with pytest.raises(hh.HHError, match="particles"):
        hh.ShortRange(ctx(), t6, s2, g3, 5.0)


@pytest.mark.parametrize("prec,eps,tol", [("fp64", 1e-8, 1e-6), ("fp32", 1e-5, 1e-4)])
def test_edge_sizes(prec, eps, tol):
    """1, 2, 5, 65 and 400 particles in two-particle leaves (a single leaf,
    ragged leaves, blocks whose coupling columns leave only poorly conditioned
    pivots): the 6N product against the dense 6N sum, globally and per
    particle, FP64 within 100 zeta and FP32 within the FP32 bound."""
    from gpu_common import ctx, dev, say
    k6 = hh.Kernel.rpy6(ctx())
    dt = torch.float64 if prec == "fp64" else torch.float32
    for n in (1, 2, 5, 65, 400):
        X, F, T = _case(n, seed=19 + n, phi=0.05)
        say("6N edge", prec, n)
        hm = hh.HMatrix(ctx(), dev(X), k6, c_leaf=4, eps=eps, prec=prec)
        Y = (hm @ _g6(F, T, dt)).double().cpu().numpy()
        ref = _ref(X, F, T)
        say("rel", _rel(Y, ref), "worst row", _row(Y, ref), "info", hm.lr.info())
        assert Y.shape == (n, 6)
        assert _rel(Y, ref) < tol and _row(Y, ref) < tol
