"""Pins of the oracle's short-range many-body terms (CPU only).

* a hand-worked three-particle line with constant networks: every neighbour
  pair and every 3-clique (j, k, i) written out by hand, with the
  normalisations of Eq. (4);
* the cut-off is strict (a particle exactly R_cut away is no neighbour) and
  an isolated particle gets and gives nothing;
* an independent brute-force enumeration over all ordered triples (the
  definition of a 3-clique checked literally) gives the same cliques and the
  same velocities with seeded networks;
* translation invariance and permutation equivariance;
* the stand-in networks: a hand-evaluated single active unit, and symmetric
  3x3 blocks.
"""
import itertools
import math

import numpy as np

import workloads as wl
from oracle import short as OS


def _const_nets(cs=1.0, c3s=1.0, c3t=1.0):
    """Networks whose outputs are constants: zero weights, output bias set."""
    Ws, bs = wl.mlp_weights(11)
    Ws = [np.zeros_like(w) for w in Ws]
    bs = [np.zeros_like(b) for b in bs]
    bs[-1] = cs * np.eye(3).ravel()
    Wg, bg = wl.mlp_weights(12, widths=(6, 64, 64, 64, 18))
    Wg = [np.zeros_like(w) for w in Wg]
    bg = [np.zeros_like(b) for b in bg]
    bg[-1] = np.concatenate([c3s * np.eye(3).ravel(), c3t * np.eye(3).ravel()])
    return OS.Net(Ws, bs), OS.Net(Wg, bg)


def _seeded_nets():
    return OS.Net(*wl.mlp_weights(11)), OS.Net(*wl.mlp_weights(12, widths=(6, 64, 64, 64, 18)))


def test_hand_worked_line():
    # x0 = 0, x1 = 2, x2 = 4 on the x axis: every pair is within R_cut = 5
    X = np.array([[0.0, 0, 0], [2.0, 0, 0], [4.0, 0, 0]])
    F = np.array([[1.0, 2.0, 3.0], [-1.0, 0.5, 0.25], [0.0, -2.0, 1.0]])
    hs, g = _const_nets(cs=1.0, c3s=2.0, c3t=3.0)
    p = 8.0 * math.pi
    # two-body self terms: I / (8 pi |d|), summed over the neighbours, times F_i
    s2 = [(1 / 2 + 1 / 4) / p, (1 / 2 + 1 / 2) / p, (1 / 4 + 1 / 2) / p]
    U = np.array([s2[i] * F[i] for i in range(3)])
    # 3-cliques (j, k, i), weight 1 / (8 pi |x_j - x_k| |x_k - x_i|):
    #   i=0: (2,1,0) 1/(2*2), (1,2,0) 1/(2*4)
    #   i=1: (2,0,1) 1/(4*2), (0,2,1) 1/(4*2)
    #   i=2: (0,1,2) 1/(2*2), (1,0,2) 1/(2*4)
    for (j, k, i, w) in [(2, 1, 0, 1 / 4), (1, 2, 0, 1 / 8), (2, 0, 1, 1 / 8), (0, 2, 1, 1 / 8),
                         (0, 1, 2, 1 / 4), (1, 0, 2, 1 / 8)]:
        U[i] += (w / p) * (2.0 * F[i] + 3.0 * F[j])
    got = OS.short_u(X, F, hs, g)
    assert np.allclose(got, U, rtol=1e-14, atol=1e-16)
    C = OS.cliques(X)
    assert sorted(map(tuple, C)) == sorted([(2, 1, 0), (1, 2, 0), (2, 0, 1), (0, 2, 1),
                                            (0, 1, 2), (1, 0, 2)])


def test_cutoff_is_strict_and_isolated_particles_do_nothing():
    X = np.array([[0.0, 0, 0], [5.0, 0, 0], [0.0, 4.999, 0], [40.0, 40, 40]])
    F = wl.normal_forces(4, seed=1)
    nb = OS.neighbours(X)
    assert list(nb[0]) == [2] and list(nb[1]) == [] and list(nb[3]) == []
    hs, g = _seeded_nets()
    U = OS.short_u(X, F, hs, g)
    assert np.all(U[1] == 0) and np.all(U[3] == 0)
    # moving the isolated particle's force changes nothing elsewhere
    F2 = F.copy()
    F2[3] = [9.0, -9.0, 9.0]
    assert np.array_equal(OS.short_u(X, F2, hs, g)[:3], U[:3])


def test_brute_force_triples():
    X = wl.rsa_cube(40, 0.3, seed=5)
    F = wl.normal_forces(40, seed=6)
    hs, g = _seeded_nets()
    n = X.shape[0]
    D = np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1))
    # the definition, literally: ordered triples of distinct particles with
    # |x_i - x_k| < R_cut and |x_j - x_k| < R_cut
    want = []
    for j, k, i in itertools.permutations(range(n), 3):
        if D[i, k] < OS.R_CUT and D[j, k] < OS.R_CUT:
            want.append((j, k, i))
    C = OS.cliques(X)
    assert sorted(want) == sorted(map(tuple, C)) and len(want) > 100
    U = np.zeros((n, 3))
    for i in range(n):
        for j in range(n):
            if j != i and D[i, j] < OS.R_CUT:
                U[i] += OS.alpha2_s((X[j] - X[i])[None], hs)[0] @ F[i]
    for (j, k, i) in want:
        As, At = OS.alpha3((X[j] - X[i])[None], (X[k] - X[i])[None], g)
        U[i] += As[0] @ F[i] + At[0] @ F[j]
    assert np.allclose(OS.short_u(X, F, hs, g), U, rtol=1e-13, atol=1e-16)


def test_invariances():
    X = wl.rsa_cube(60, 0.25, seed=7)
    F = wl.normal_forces(60, seed=8)
    hs, g = _seeded_nets()
    U = OS.short_u(X, F, hs, g)
    assert np.allclose(OS.short_u(X + np.array([3.5, -1e3, 7.25]), F, hs, g), U, rtol=1e-9,
                       atol=1e-13)
    p = np.random.default_rng(0).permutation(60)
    assert np.allclose(OS.short_u(X[p], F[p], hs, g), U[p], rtol=1e-12, atol=1e-16)


def test_networks_hand_evaluated_and_symmetric():
    # one active unit per hidden layer: o = w4 * tanh(w3 * tanh(w2 * tanh(w1 . v)))
    Wg, bg = wl.mlp_weights(12, widths=(6, 64, 64, 64, 18))
    Wg = [np.zeros_like(w) for w in Wg]
    bg = [np.zeros_like(b) for b in bg]
    Wg[0][0, 3] = 0.7          # unit 0 of layer 1 reads the x component of d_k / R_cut
    Wg[1][0, 0] = 1.3
    Wg[2][0, 0] = -0.4
    Wg[3][13, 0] = 2.0         # alpha_3^(t) block, row 1, column 1
    g = OS.Net(Wg, bg)
    dj = np.array([[1.0, 2.0, -0.5]])
    dk = np.array([[3.0, 0.0, 1.0]])
    As, At = OS.alpha3(dj, dk, g)
    h = math.tanh(-0.4 * math.tanh(1.3 * math.tanh(0.7 * 3.0 / 5.0)))
    scale = 1.0 / (8 * math.pi * np.linalg.norm(dj - dk) * np.linalg.norm(dk))
    want = np.zeros((3, 3))
    want[1, 1] = 2.0 * h * scale
    assert np.allclose(At[0], want, rtol=1e-14, atol=1e-18) and np.all(As == 0)
    hs, g2 = _seeded_nets()
    d = np.random.default_rng(1).normal(size=(20, 3)) * 3
    K = OS.alpha2_s(d, hs)
    A1, A2 = OS.alpha3(d, d[::-1] + 0.5, g2)
    for M in (K, A1, A2):
        assert np.allclose(M, np.swapaxes(M, 1, 2), rtol=0, atol=0)


def test_rows_variant_equals_full():
    # the large-N row evaluation against the full sum (same definitions,
    # separate neighbour and clique enumeration)
    X = wl.rsa_cube(400, 0.2, seed=31)
    F = wl.normal_forces(400, seed=32)
    hs, g = _seeded_nets()
    full = OS.short_u(X, F, hs, g)
    rows = np.array([0, 7, 123, 399])
    got = OS.short_u_rows(X, F, hs, g, rows)
    assert np.allclose(got, full[rows], rtol=1e-12, atol=1e-15)
