"""GPU parity of the batched form: several independent systems in one tree,
one partition and the same ACA and apply launches.

* the batched tree and block lists are, system by system, the oracle's
  single-system tree and lists with node ids and positions shifted (bit-exact);
* no block couples two systems: zero forces on one system give exactly zero
  velocities there, whatever the other systems carry;
* each system's velocities equal its own single-system product (FP64 RPY,
  BF16 MLP) and the FP64 dense sum within the single-system tolerances;
* the backward pass on the batched tree gives each system's own gradients.
"""
import numpy as np
import pytest
import torch

import paper_2505_08174_amd as hh
import workloads as wl
from oracle import dense as OD
from oracle import partition as OP
from oracle import tree as OT

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _systems(sizes, seed0=40):
    """Alternating sphere packings and filaments of the given sizes."""
    Xs = []
    for s, n in enumerate(sizes):
        if s % 2 == 1 and n % 50 == 0:
            Xs.append(wl.filament_chains(n, 0.1, seed=seed0 + s))
        else:
            Xs.append(wl.lattice_cube(n, 0.05 + 0.05 * (s % 5), seed=seed0 + s))
    off = np.concatenate([[0], np.cumsum([x.shape[0] for x in Xs])]).astype(np.int64)
    return Xs, np.concatenate(Xs), off


SIZES = [700, 3000, 1, 64, 2500, 65, 150, 4000]


@pytest.mark.parametrize("c_leaf", [64, 32])
def test_batched_tree_and_partition_equal_per_system_oracle(c_leaf):
    from gpu_common import ctx, dev, say
    say("batched tree", SIZES, c_leaf)
    Xs, X, off = _systems(SIZES)
    t = hh.build_tree_batch(ctx(), dev(X), off, c_leaf)
    ex = t.export()
    g, h = hh.partition(ctx(), t, 1.0).export()
    node0 = 0
    Gs, Hs, nodes, bbox = [], [], [], []
    for s, Xk in enumerate(Xs):
        ref = OT.build_tree(Xk, c_leaf)
        a, b = off[s], off[s + 1]
        assert np.array_equal(ex["perm"][a:b], ref.perm + a), s
        assert np.array_equal(ex["keys"][a:b], ref.keys), s
        nd = ref.nodes.copy()
        nd[:, :2] += a
        nd[:, 2:] = np.where(nd[:, 2:] >= 0, nd[:, 2:] + node0, -1)
        nodes.append(nd)
        bbox.append(ref.bbox)
        G, H = OP.build_partition(ref, 1.0)
        Gs.append(G + node0)
        Hs.append(H + node0)
        node0 += ref.nodes.shape[0]
    assert np.array_equal(ex["nodes"], np.concatenate(nodes))
    assert np.array_equal(ex["bbox"], np.concatenate(bbox))
    G = np.concatenate(Gs).reshape(-1, 2)
    H = np.concatenate(Hs).reshape(-1, 2)
    assert np.array_equal(g, G) and np.array_equal(h, H)


def test_per_system_leaf_sizes_equal_per_system_oracle():
    """Each system with its own C_leaf: its subtree and blocks are the
    oracle's single-system ones built with that leaf size."""
    from gpu_common import ctx, dev, say
    cls = [16, 64, 2, 32, 128, 8, 48, 100]
    say("per-system leaf sizes", cls)
    Xs, X, off = _systems(SIZES)
    t = hh.build_tree_batch(ctx(), dev(X), off, np.array(cls))
    ex = t.export()
    g, h = hh.partition(ctx(), t, 1.0).export()
    node0 = 0
    Gs, Hs, nodes = [], [], []
    for s, Xk in enumerate(Xs):
        ref = OT.build_tree(Xk, cls[s])
        a = off[s]
        assert np.array_equal(ex["perm"][a:off[s + 1]], ref.perm + a), s
        nd = ref.nodes.copy()
        nd[:, :2] += a
        nd[:, 2:] = np.where(nd[:, 2:] >= 0, nd[:, 2:] + node0, -1)
        nodes.append(nd)
        G, H = OP.build_partition(ref, 1.0)
        Gs.append(G + node0)
        Hs.append(H + node0)
        node0 += ref.nodes.shape[0]
    assert np.array_equal(ex["nodes"], np.concatenate(nodes))
    assert np.array_equal(g, np.concatenate(Gs).reshape(-1, 2))
    assert np.array_equal(h, np.concatenate(Hs).reshape(-1, 2))
    with pytest.raises(hh.HHError):
        hh.build_tree_batch(ctx(), dev(X), off, np.array([1] + cls[1:]))


def test_batched_tree_rejects_bad_offsets():
    from gpu_common import ctx, dev, say
    say("batched tree errors")
    X = wl.lattice_cube(100, 0.1, seed=1)
    for off in ([0, 50, 50, 100], [0, 60, 40, 100]):
        with pytest.raises(hh.HHError):
            hh.build_tree_batch(ctx(), dev(X), np.array(off), 16)


def test_no_cross_system_leakage():
    from gpu_common import ctx, dev, kernels, say
    say("batched leakage")
    Xs, X, off = _systems(SIZES)
    F = wl.normal_forces(X.shape[0], seed=7)
    _, kg = kernels("rpy")
    hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=32, eps=1e-6, prec="fp64", offsets=off)
    for s in (1, 4):
        Fz = F.copy()
        Fz[off[s]:off[s + 1]] = 0.0
        U = (hm @ dev(Fz)).cpu().numpy()
        assert np.all(U[off[s]:off[s + 1]] == 0.0), s
        assert np.any(U[off[s + 1]:] != 0.0)


@pytest.mark.parametrize("kind,prec,tol_self,tol_dense", [("rpy", "fp64", 1e-12, 1e-5),
                                                          ("mlp", "bf16", 1e-6, 5e-3)])
def test_batched_product_equals_per_system(kind, prec, tol_self, tol_dense):
    from gpu_common import ctx, dev, kernels, say
    say("batched product", kind, prec)
    Xs, X, off = _systems(SIZES)
    F = wl.gravity_forces(X.shape[0], seed=8)
    ko, kg = kernels(kind)
    fdt = torch.float64 if prec == "fp64" else torch.float32
    eps = 1e-6 if prec == "fp64" else 1e-4
    hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, eps=eps, prec=prec, offsets=off)
    U = (hm @ dev(F, fdt)).double().cpu().numpy()
    for s, Xk in enumerate(Xs):
        a, b = off[s], off[s + 1]
        hs = hh.HMatrix(ctx(), dev(Xk), kg, c_leaf=64, eps=eps, prec=prec)
        Us = (hs @ dev(F[a:b], fdt)).double().cpu().numpy()
        rows = wl.sample_rows(b - a, min(b - a, 200), seed=s)
        Ud = OD.dense_u(Xk, F[a:b], ko, rows)
        d_self, d_dense = _rel(U[a:b], Us), _rel(U[a:b][rows], Ud)
        say("system", s, b - a, "vs single", d_self, "vs dense", d_dense)
        assert d_self <= tol_self, s
        assert d_dense <= tol_dense, s


def test_batched_backward_equals_per_system():
    from gpu_common import ctx, dev, kernels, say
    say("batched backward fp64 mlp")
    sizes = [900, 1500, 300]
    Xs, X, off = _systems(sizes, seed0=60)
    F = wl.normal_forces(X.shape[0], seed=9)
    W = wl.normal_forces(X.shape[0], seed=10)
    _, kg = kernels("mlp")
    hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=32, eps=1e-8, prec="fp64", offsets=off)
    dF, dX, dth = hh.matvec_backward(ctx(), hm.tree, hm.part, hm.lr, kg, dev(F), dev(W), prec="fp64")
    dF, dX, dth = (v.cpu().numpy() for v in (dF, dX, dth))
    dth_sum = np.zeros_like(dth)
    for s, Xk in enumerate(Xs):
        a, b = off[s], off[s + 1]
        hs = hh.HMatrix(ctx(), dev(Xk), kg, c_leaf=32, eps=1e-8, prec="fp64")
        g = hh.matvec_backward(ctx(), hs.tree, hs.part, hs.lr, kg, dev(F[a:b]), dev(W[a:b]),
                               prec="fp64")
        gF, gX, gt = (v.cpu().numpy() for v in g)
        say("system", s, _rel(dF[a:b], gF), _rel(dX[a:b], gX))
        assert _rel(dF[a:b], gF) < 1e-12
        assert _rel(dX[a:b], gX) < 1e-11
        dth_sum += gt
    assert _rel(dth, dth_sum) < 1e-11
