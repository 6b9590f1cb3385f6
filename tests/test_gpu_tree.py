"""GPU parity: Morton order, cluster tree and block partition bit-exact against
the oracle, plus error paths of the two entry points."""
import numpy as np
import pytest

import paper_2505_08174_amd as hh
import workloads as wl
from oracle import partition as OP
from oracle import tree as OT

pytestmark = pytest.mark.gpu

CASES = [
    ("cube", 2000, 0.10, 64, 0),      # plain small configuration
    ("cube", 777, 0.20, 32, 3),       # ragged sizes
    ("cube", 5000, 0.30, 50, 1),
    ("sphere", 20000, 0.10, 128, 0),  # lattice drop
    ("cube", 100000, 0.20, 128, 0),   # plain FP32 configuration geometry
]


def _pos(geom, n, phi, seed):
    return wl.rsa_cube(n, phi, seed=seed) if geom == "cube" else wl.lattice_sphere(n, phi, seed=seed)


@pytest.mark.parametrize("geom,n,phi,c_leaf,seed", CASES)
def test_tree_and_partition_bit_exact(geom, n, phi, c_leaf, seed):
    from gpu_common import ctx, dev, say
    say("tree", geom, n, phi, c_leaf, seed)
    X = _pos(geom, n, phi, seed)
    ref = OT.build_tree(X, c_leaf)
    t = hh.build_tree(ctx(), dev(X), c_leaf)
    ex = t.export()
    assert np.array_equal(ex["perm"], ref.perm)
    assert np.array_equal(ex["keys"], ref.keys)
    assert np.array_equal(ex["nodes"], ref.nodes)
    assert np.array_equal(ex["bbox"], ref.bbox)
    for eta in (1.0, 0.5):
        say("partition", n, eta)
        G, H = OP.build_partition(ref, eta)
        p = hh.partition(ctx(), t, eta)
        g, h = p.export()
        assert np.array_equal(g, G) and np.array_equal(h, H)


def test_small_and_degenerate_sizes():
    from gpu_common import ctx, dev, say
    for n, c_leaf in [(1, 2), (2, 2), (3, 64), (63, 64), (64, 64), (65, 64), (130, 2)]:
        say("small", n, c_leaf)
        X = wl.rsa_cube(n, 0.05, seed=n) if n > 1 else np.array([[0.5, -1.0, 2.0]])
        ref = OT.build_tree(X, c_leaf)
        t = hh.build_tree(ctx(), dev(X), c_leaf)
        ex = t.export()
        assert np.array_equal(ex["perm"], ref.perm)
        assert np.array_equal(ex["nodes"], ref.nodes)
        G, H = OP.build_partition(ref, 1.0)
        g, h = hh.partition(ctx(), t, 1.0).export()
        assert np.array_equal(g, G) and np.array_equal(h, H)


def test_line_example_and_dense_mode():
    from gpu_common import ctx, dev, say
    say("line example")
    X = np.array([[float(x), 0.0, 0.0] for x in [5, 2, 7, 0, 3, 6, 1, 4]])
    t = hh.build_tree(ctx(), dev(X), 2)
    ref = OT.build_tree(X, 2)
    assert np.array_equal(t.export()["nodes"], ref.nodes)
    g, h = hh.partition(ctx(), t, 1.0).export()
    G, H = OP.build_partition(ref, 1.0)
    assert np.array_equal(g, G) and np.array_equal(h, H)
    g, h = hh.partition(ctx(), t, 1.0, dense_mode=True).export()
    assert g.shape[0] == 0 and h.shape[0] == 64


def test_error_paths():
    from gpu_common import ctx, dev, say
    say("error paths")
    X = wl.rsa_cube(100, 0.1, seed=2)
    Xd = X.copy()
    Xd[57] = Xd[12]
    with pytest.raises(hh.HHError, match="DUPLICATE"):
        hh.build_tree(ctx(), dev(Xd), 16)
    Xn = X.copy()
    Xn[3, 1] = np.nan
    with pytest.raises(hh.HHError, match="INVALID_ARG"):
        hh.build_tree(ctx(), dev(Xn), 16)
    with pytest.raises(hh.HHError, match="INVALID_ARG"):
        hh.build_tree(ctx(), dev(X), 1)
    t = hh.build_tree(ctx(), dev(X), 16)
    with pytest.raises(hh.HHError, match="INVALID_ARG"):
        hh.partition(ctx(), t, 0.0)
    with pytest.raises(hh.HHError, match="INVALID_ARG"):
        hh.partition(ctx(), t, -1.0)
