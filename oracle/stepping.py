"""Time stepping of a suspension with flexible filaments (oracle only).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 4.3: the velocities U = M(X) F are predicted at every time step and the
positions advanced by the explicit Euler scheme, X <- X + dt U. Every
particle carries the gravitational force (0, 0, -1) (Sec. 4.3.1). A filament
is a chain of N_b beads (consecutive indices) with two internal forces
(Sec. 4.3.2, the two displayed force laws):
  tension on each bond (i, i+1), r = x_{i+1} - x_i:
      f = k_t (|r| - l_0) r / |r|,  F_i += f,  F_{i+1} -= f;
  COS bending on each interior bead i of the triple (i-1, i, i+1):
      t_1 = (x_i - x_{i-1}) / |.|, t_2 = (x_{i+1} - x_i) / |.|,
      sin(theta) = |t_1 x t_2|, T = -k_b (t_1 x t_2) sin(theta),
      f_{i-1} = T x t_1, f_{i+1} = -T x t_2, f_i = -(f_{i-1} + f_{i+1}).
The filaments are the first n_fil * n_beads particles, chain c holding
particles [c n_beads, (c + 1) n_beads); the remaining particles are free.
"""
from __future__ import annotations

import numpy as np


def filament_forces(X, n_fil: int, n_beads: int, k_t: float, l0: float, k_b: float):
    """Tension and bending forces of the chains (zero on free particles)."""
    X = np.asarray(X, dtype=np.float64)
    F = np.zeros_like(X)
    for c in range(n_fil):
        b0 = c * n_beads
        for i in range(b0, b0 + n_beads - 1):
            r = X[i + 1] - X[i]
            d = np.linalg.norm(r)
            f = k_t * (d - l0) * r / d
            F[i] += f
            F[i + 1] -= f
        for i in range(b0 + 1, b0 + n_beads - 1):
            a = X[i] - X[i - 1]
            b = X[i + 1] - X[i]
            t1 = a / np.linalg.norm(a)
            t2 = b / np.linalg.norm(b)
            c12 = np.cross(t1, t2)
            T = -k_b * c12 * np.linalg.norm(c12)
            f_prev = np.cross(T, t1)
            f_next = -np.cross(T, t2)
            F[i - 1] += f_prev
            F[i + 1] += f_next
            F[i] += -(f_prev + f_next)
    return F


def forces(X, n_fil: int = 0, n_beads: int = 0, k_t: float = 20.0, l0: float = 3.0,
           k_b: float = 50.0, gravity=(0.0, 0.0, -1.0)):
    """Gravity on every particle plus the filaments' internal forces."""
    X = np.asarray(X, dtype=np.float64)
    F = np.tile(np.asarray(gravity, dtype=np.float64), (X.shape[0], 1))
    if n_fil > 0:
        F += filament_forces(X, n_fil, n_beads, k_t, l0, k_b)
    return F


def euler(X, U, dt: float):
    """One explicit Euler step of dX/dt = U."""
    return np.asarray(X, dtype=np.float64) + dt * np.asarray(U, dtype=np.float64)


def step(X, dt: float, velocity, **fparams):
    """Forces at X, velocities velocity(X, F), then the Euler update:
    returns (X_next, F, U)."""
    F = forces(X, **fparams)
    U = velocity(X, F)
    return euler(X, U, dt), F, U
