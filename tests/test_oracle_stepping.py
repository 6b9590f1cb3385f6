"""Pins of the oracle's time stepping and filament forces (CPU only).

* tension: a hand-worked stretched bond, and zero at the rest length;
* bending: zero on a straight chain, and a hand-worked right angle;
* the internal forces of a chain sum to zero and turn with the chain
  (rotation equivariance), and do not depend on its position;
* one Euler step of an isolated particle under gravity moves it by
  dt / (6 pi) (its self mobility, Eq. (2)), and a free particle far from a
  filament is unaffected by the filament's internal forces.
"""
import math

import numpy as np

import workloads as wl
from oracle import dense as OD
from oracle import kernels as OK
from oracle import stepping as OS


def test_tension_hand_worked():
    X = np.array([[0.0, 0, 0], [3.0, 0, 0]])
    F = OS.filament_forces(X, 1, 2, k_t=20.0, l0=2.2, k_b=50.0)
    # f = 20 * (3 - 2.2) along +x on bead 0, the opposite on bead 1
    assert np.allclose(F, [[16.0, 0, 0], [-16.0, 0, 0]], rtol=1e-14, atol=0)
    X2 = np.array([[0.0, 0, 0], [0, 0, 2.2], [0, 0, 4.4]])
    assert np.allclose(OS.filament_forces(X2, 1, 3, 20.0, 2.2, 50.0), 0, atol=1e-13)


def test_bending_hand_worked():
    # right angle at bead 1: t1 = +x, t2 = +y, t1 x t2 = +z, sin = 1, T = -k_b z
    X = np.array([[-1.0, 0, 0], [0.0, 0, 0], [0.0, 1, 0]])
    kb = 50.0
    F = OS.filament_forces(X, 1, 3, k_t=0.0, l0=1.0, k_b=kb)
    # f_0 = T x t1 = -kb (z x x) = -kb y; f_2 = -T x t2 = kb (z x y) = -kb x
    want = np.array([[0.0, -kb, 0], [kb, kb, 0], [-kb, 0, 0]])
    assert np.allclose(F, want, rtol=1e-14, atol=1e-12)
    Xs = np.array([[0.0, 0, 0], [1.5, 0, 0], [3.0, 0, 0], [4.5, 0, 0]])
    assert np.allclose(OS.filament_forces(Xs, 1, 4, 0.0, 1.5, kb), 0, atol=1e-12)


def test_chain_forces_sum_to_zero_and_rotate():
    X = wl.filament_chains(100, 0.1, seed=4)[:100]
    F = OS.filament_forces(X, 2, 50, 20.0, 2.0, 50.0)
    assert np.allclose(F.sum(axis=0), 0, atol=1e-10)
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    FR = OS.filament_forces(X @ R.T, 2, 50, 20.0, 2.0, 50.0)
    assert np.allclose(FR, F @ R.T, rtol=1e-10, atol=1e-10)
    assert np.allclose(OS.filament_forces(X + 123.5, 2, 50, 20.0, 2.0, 50.0), F, rtol=1e-9,
                       atol=1e-9)


def test_euler_step_of_isolated_particle_and_far_filament():
    kern = OK.Kernel("rpy")
    vel = lambda X_, F_: OD.dense_u(X_, F_, kern)
    X = np.array([[0.0, 0, 0]])
    X1, F, U = OS.step(X, 0.01, vel)
    assert np.allclose(X1, [[0, 0, -0.01 / (6 * math.pi)]], rtol=1e-15, atol=0)
    # a free particle 1e6 away: the filament forces sum to zero and the
    # filament is far, so the particle moves as if alone to ~1e-6
    chain = np.array([[0.0, 0, 0], [2.2, 0.3, 0], [4.0, 1.5, 0.2]])
    Xb = np.vstack([chain, [[1e6, 0, 0]]])
    _, Fb, Ub = OS.step(Xb, 0.01, vel, n_fil=1, n_beads=3, k_t=20.0, l0=2.2, k_b=50.0)
    assert np.allclose(Fb[3], [0, 0, -1])
    assert np.allclose(Ub[3], [0, 0, -1 / (6 * math.pi)], rtol=0, atol=1e-6)
