"""Pins of the oracle block partition, Algorithm 1 with Eq. (7) (CPU only).

A hand-worked 1-D example fixes P^G and P^H exactly; on seeded workloads every
(i, j) is covered exactly once, the lists are symmetric, every admissible
block satisfies Eq. (7) and every inadmissible block is a leaf pair that fails
it (checked with an independent norm-based evaluation).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import partition as P
from oracle import tree as T


def test_line_example_by_hand():
    xs = [5, 2, 7, 0, 3, 6, 1, 4]
    X = np.array([[float(x), 0.0, 0.0] for x in xs])
    tr = T.build_tree(X, 2)
    G, H = P.build_partition(tr, 1.0)
    leaves = [3, 4, 6, 7, 10, 11, 13, 14]
    assert [tuple(h) for h in H] == [(l, l) for l in leaves]
    expect_G = sorted([(3, 4), (4, 3), (6, 7), (7, 6), (10, 11), (11, 10), (13, 14), (14, 13),
                       (2, 5), (5, 2), (9, 12), (12, 9),
                       (2, 9), (2, 12), (5, 9), (5, 12), (9, 2), (12, 2), (9, 5), (12, 5)])
    assert [tuple(g) for g in G] == expect_G


def _eq7_margin(bt, bs, eta):
    """(max diam) - eta dist, by norms (independent of the squared form)."""
    dt = np.linalg.norm(bt[3:] - bt[:3])
    ds = np.linalg.norm(bs[3:] - bs[:3])
    gap = np.maximum(0.0, np.maximum(bs[:3] - bt[3:], bt[:3] - bs[3:]))
    return max(dt, ds) - eta * np.linalg.norm(gap), np.linalg.norm(gap)


@pytest.mark.parametrize("n,phi,c_leaf,eta", [(2000, 0.1, 64, 1.0), (1500, 0.25, 32, 0.7),
                                              (2000, 0.1, 64, 2.0)])
def test_partition_properties(n, phi, c_leaf, eta):
    X = wl.rsa_cube(n, phi, seed=1)
    tr = T.build_tree(X, c_leaf)
    G, H = P.build_partition(tr, eta)
    cover = np.zeros((n, n), dtype=np.int32)
    for lst in (G, H):
        for t, s in lst:
            cover[tr.nodes[t, 0]:tr.nodes[t, 1], tr.nodes[s, 0]:tr.nodes[s, 1]] += 1
    assert np.all(cover == 1)
    sG = {tuple(x) for x in G}
    sH = {tuple(x) for x in H}
    assert sG == {(s, t) for t, s in sG}
    assert sH == {(s, t) for t, s in sH}
    scale = np.abs(tr.bbox).max()
    for t, s in G:
        m, gap = _eq7_margin(tr.bbox[t], tr.bbox[s], eta)
        assert gap > 0 and m <= 1e-12 * scale
    for t, s in H:
        assert tr.is_leaf(t) and tr.is_leaf(s)
        m, gap = _eq7_margin(tr.bbox[t], tr.bbox[s], eta)
        assert gap == 0 or m >= -1e-12 * scale


def test_dense_mode_has_only_leaf_pairs():
    X = wl.rsa_cube(700, 0.1, seed=2)
    tr = T.build_tree(X, 64)
    G, H = P.build_partition(tr, 1.0, dense_mode=True)
    nl = len(tr.leaves())
    assert G.shape[0] == 0 and H.shape[0] == nl * nl
