"""Time stepping of a suspension (Sec. 4.3): every step computes the forces
(gravity plus filament tension and bending, hh_filament_forces), rebuilds the
H-matrix on the current positions (tree, partition, ACA) and takes the
product U = M(X) F, optionally adds the short-range many-body terms, and
advances the positions by one explicit Euler step (hh_euler_step). Every
step of the path runs in libhh.so; this module only sequences the calls."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from . import api


class Suspension:
    """Particles X (device FP64 [n, 3], advanced in place) whose first
    n_fil * n_beads particles form filaments of n_beads consecutive beads."""

    def __init__(self, ctx: api.Context, X: torch.Tensor, kern: api.Kernel, prec="bf16",
                 dt: float = 0.01, n_fil: int = 0, n_beads: int = 0, k_t: float = 20.0,
                 l0: float = 3.0, k_b: float = 50.0, gravity=(0.0, 0.0, -1.0),
                 c_leaf: int = 128, eta: float = 1.0, eps: float = 1e-4, l_max: int = 48,
                 short=None):
        assert X.is_cuda and X.dtype == torch.float64 and X.is_contiguous()
        self.ctx, self.X, self.kern = ctx, X, kern
        self.prec = api._prec(prec)
        self.dt, self.n_fil, self.n_beads = float(dt), int(n_fil), int(n_beads)
        self.k_t, self.l0, self.k_b = float(k_t), float(l0), float(k_b)
        self.gravity = np.ascontiguousarray(gravity, dtype=np.float64)
        self.c_leaf, self.eta, self.eps, self.l_max = c_leaf, eta, eps, l_max
        self.short = short            # (s2_params, g3_params, r_cut) or None
        n = X.shape[0]
        self.F = torch.empty((n, 3), dtype=api.F_DTYPE[self.prec], device=X.device)
        self.U = torch.empty((n, 3), dtype=api.U_DTYPE[self.prec], device=X.device)
        self.steps = 0

    def forces(self):
        n = self.X.shape[0]
        self.ctx.check(L.load().hh_filament_forces(
            self.ctx.h, api._ptr(self.X), n, self.n_fil, self.n_beads, self.k_t, self.l0,
            self.k_b, self.gravity.ctypes.data_as(C.POINTER(C.c_double)), self.prec,
            api._ptr(self.F)))
        return self.F

    def velocities(self):
        hm = api.HMatrix(self.ctx, self.X, self.kern, self.c_leaf, self.eta, self.eps, self.prec,
                         self.l_max)
        self.hm = hm     # the H-matrix of the last step (for statistics)
        api.matvec(self.ctx, hm.tree, hm.part, hm.lr, self.kern, self.F, self.prec, self.U)
        if self.short is not None:
            s2, g3, rc = self.short
            api.ShortRange(self.ctx, hm.tree, s2, g3, rc).matvec(self.F, self.U, self.prec)
        return self.U

    def step(self):
        """One time step; returns the velocities it used."""
        self.forces()
        self.velocities()
        self.ctx.check(L.load().hh_euler_step(self.ctx.h, api._ptr(self.X), api._ptr(self.U),
                                              self.X.shape[0], self.dt, self.prec))
        self.steps += 1
        return self.U
