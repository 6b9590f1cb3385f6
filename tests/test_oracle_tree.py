"""Pins of the oracle cluster tree and Morton order (CPU only).

A hand-worked 1-D example fixes the node table; brute-force bit interleaving
fixes the Morton keys; invariants of Definition 1 are checked on seeded
workloads; identical points exercise the forced-leaf reading.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import tree as T


def _interleave_by_string(qx, qy, qz):
    bx, by, bz = (format(int(v), "021b") for v in (qx, qy, qz))
    return int("".join(x + y + z for x, y, z in zip(bx, by, bz)), 2)


def test_morton_against_string_interleave():
    rng = wl.Rng(21, "misc")
    q = (rng.raw(600).reshape(200, 3) >> np.uint64(43)).astype(np.int64)   # 21-bit values
    keys = T.morton_keys(q)
    for i in range(200):
        assert int(keys[i]) == _interleave_by_string(*q[i])


def test_quantize_by_hand():
    X = np.array([[1.0, 2.0, 3.0], [4.0, 2.5, 3.25], [2.0, 2.0, 5.0]])
    # extents (3, .5, 2): E = 3 -> e = 2 -> scale 2^19
    q = T.quantize(X)
    expect = np.array([[0, 0, 0], [3 << 19, 1 << 18, 1 << 17], [1 << 19, 0, 1 << 20]])
    assert np.array_equal(q, expect)


def test_line_example_by_hand():
    xs = [5, 2, 7, 0, 3, 6, 1, 4]
    X = np.array([[float(x), 0.0, 0.0] for x in xs])
    tr = T.build_tree(X, 2)
    expect_nodes = np.array([
        [0, 8, 1, 8], [0, 4, 2, 5], [0, 2, 3, 4], [0, 1, -1, -1], [1, 2, -1, -1],
        [2, 4, 6, 7], [2, 3, -1, -1], [3, 4, -1, -1], [4, 8, 9, 12], [4, 6, 10, 11],
        [4, 5, -1, -1], [5, 6, -1, -1], [6, 8, 13, 14], [6, 7, -1, -1], [7, 8, -1, -1]])
    assert np.array_equal(tr.nodes, expect_nodes)
    assert np.array_equal(tr.perm, [3, 6, 1, 4, 7, 0, 5, 2])
    assert np.array_equal(tr.bbox[5], [2.0, 0, 0, 3.0, 0, 0])


def test_identical_points_make_a_forced_leaf():
    X = np.tile([[1.0, 2.0, 3.0]], (5, 1))
    tr = T.build_tree(X, 2)
    assert np.array_equal(tr.nodes, [[0, 5, -1, -1]])
    assert np.array_equal(tr.perm, np.arange(5))


@pytest.mark.parametrize("n,phi,c_leaf,geom", [(2000, 0.1, 64, "cube"), (5000, 0.2, 128, "cube"),
                                               (3000, 0.1, 50, "sphere")])
def test_tree_invariants(n, phi, c_leaf, geom):
    X = wl.rsa_cube(n, phi) if geom == "cube" else wl.lattice_sphere(n, phi)
    tr = T.build_tree(X, c_leaf)
    keys_all = T.morton_keys(T.quantize(X))
    # particle order is the stable Morton sort
    assert np.array_equal(tr.perm, np.lexsort((np.arange(n), keys_all)))
    assert np.array_equal(tr.keys, keys_all[tr.perm])
    nodes = tr.nodes
    assert nodes[0, 0] == 0 and nodes[0, 1] == n
    Xs = X[tr.perm]
    for t in range(tr.n_nodes):
        b, e, l, r = nodes[t]
        assert b < e
        assert np.array_equal(tr.bbox[t, :3], Xs[b:e].min(axis=0))
        assert np.array_equal(tr.bbox[t, 3:], Xs[b:e].max(axis=0))
        if l < 0:
            assert r < 0
            assert e - b < c_leaf or np.all(tr.keys[b:e] == tr.keys[b])
        else:
            assert e - b >= c_leaf
            assert l == t + 1 and r > l                   # pre-order
            assert nodes[l, 0] == b and nodes[l, 1] == nodes[r, 0] and nodes[r, 1] == e
            # the split is a Morton bit: the sons share the parent's prefix and
            # differ exactly at the highest bit where the node's keys differ
            kk = tr.keys[b:e]
            hb = int(kk[0] ^ kk[-1]).bit_length() - 1
            assert np.all((tr.keys[b:nodes[l, 1]] >> np.uint64(hb)) & np.uint64(1) == 0)
            assert np.all((tr.keys[nodes[r, 0]:e] >> np.uint64(hb)) & np.uint64(1) == 1)
