"""Two-body 3x3 mobility kernels and the self mobility, in FP64 (oracle only).

Paper reference: the velocity expansion Eq. (2) (Sec. 2.2) has a one-body term
alpha_1 = (6 pi mu a)^-1 I for spheres in an unbounded fluid and a two-body
off-diagonal term alpha_2^(t)(X_i, X_j) that decays like 1/r; its learned
surrogate is h(X_j - X_i)/|X_j - X_i| (Eq. (4), Sec. 2.3). The matrix M^(t,2)
of Eq. (6) holds these 3x3 blocks (Sec. 3, footnote: entries are 3x3 blocks).

Two stand-ins for the learned h are provided:
  * the Rotne-Prager-Yamakawa tensor, which the paper cites as the classical
    dilute two-body mobility (Sec. 1); textbook closed form, both branches;
  * a seeded MLP 3 -> 64 -> 64 -> 64 -> 9 with tanh after the three hidden
    layers and a linear output, reshaped row-major to 3x3 (the row-major
    flattening of 3x3 entries follows Sec. 3.3.2), symmetrised and scaled by
    1/(8 pi |r|) so that it decays like 1/r as Eq. (4) prescribes.

Displacement convention: r = x_i - x_j (target minus source).
"""
from __future__ import annotations

import math

import numpy as np

EYE = np.eye(3)


def self_mobility(a: float = 1.0, mu: float = 1.0) -> float:
    """Scalar s with alpha_1 = s I, s = 1/(6 pi mu a) (Eq. (2))."""
    return 1.0 / (6.0 * math.pi * mu * a)


def rpy(r: np.ndarray, a: float = 1.0, mu: float = 1.0) -> np.ndarray:
    """Rotne-Prager-Yamakawa tensor for equal spheres of radius a.

    r: [..., 3] displacements (nonzero). Returns [..., 3, 3].
      |r| >= 2a: 1/(8 pi mu |r|) [(1 + 2a^2/(3r^2)) I + (1 - 2a^2/r^2) rr^T/r^2]
      |r| <  2a: 1/(6 pi mu a)  [(1 - 9r/(32a)) I + (3r/(32a)) rr^T/r^2]
    """
    r = np.asarray(r, dtype=np.float64)
    d = np.sqrt(np.sum(r * r, axis=-1))
    rh = r / d[..., None]
    outer = rh[..., :, None] * rh[..., None, :]
    far_i = (1.0 + 2.0 * a * a / (3.0 * d * d)) / (8.0 * math.pi * mu * d)
    far_o = (1.0 - 2.0 * a * a / (d * d)) / (8.0 * math.pi * mu * d)
    near_i = (1.0 - 9.0 * d / (32.0 * a)) / (6.0 * math.pi * mu * a)
    near_o = (3.0 * d / (32.0 * a)) / (6.0 * math.pi * mu * a)
    far = d >= 2.0 * a
    ci = np.where(far, far_i, near_i)
    co = np.where(far, far_o, near_o)
    return ci[..., None, None] * EYE + co[..., None, None] * outer


class MLP:
    """Parameters of the seeded kernel MLP: weights W[l] of shape [out, in] and
    biases b[l] of shape [out]; tanh after every layer except the last."""

    def __init__(self, Ws, bs):
        self.W = [np.asarray(w, dtype=np.float64) for w in Ws]
        self.b = [np.asarray(v, dtype=np.float64) for v in bs]
        assert self.W[0].shape[1] == 3 and self.W[-1].shape[0] == 9

    def forward(self, r: np.ndarray, keep: bool = False):
        """r: [P, 3] -> raw outputs o: [P, 9]; optionally the hidden activations."""
        h = np.asarray(r, dtype=np.float64)
        acts = [h]
        nl = len(self.W)
        for l in range(nl):
            z = h @ self.W[l].T + self.b[l]
            h = np.tanh(z) if l < nl - 1 else z
            acts.append(h)
        return (h, acts) if keep else h


def mlp_kernel(r: np.ndarray, mlp: MLP, inp: str = "direction",
               chunk: int = 65536) -> np.ndarray:
    """K(r) = (O + O^T)/2 / (8 pi |r|) with O = reshape(MLP(v), 3, 3) row-major.

    v is the unit direction r/|r| (inp="direction") or the displacement r
    itself (inp="displacement"). r: [..., 3]; returns [..., 3, 3].
    """
    assert inp in ("direction", "displacement")
    r = np.asarray(r, dtype=np.float64)
    shp = r.shape[:-1]
    rf = r.reshape(-1, 3)
    out = np.empty((rf.shape[0], 3, 3))
    for s in range(0, rf.shape[0], chunk):
        rc = rf[s:s + chunk]
        d = np.sqrt(np.sum(rc * rc, axis=1))
        v = rc / d[:, None] if inp == "direction" else rc
        O = mlp.forward(v).reshape(-1, 3, 3)
        out[s:s + chunk] = 0.5 * (O + np.swapaxes(O, 1, 2)) / (8.0 * math.pi * d)[:, None, None]
    return out.reshape(shp + (3, 3))


class Kernel:
    """A two-body kernel K(r) plus its self mobility, as used by the oracle."""

    def __init__(self, kind: str, mlp: MLP | None = None, a: float = 1.0, mu: float = 1.0,
                 inp: str = "direction"):
        assert kind in ("rpy", "mlp")
        self.kind, self.mlp, self.a, self.mu, self.inp = kind, mlp, a, mu, inp
        if kind == "mlp":
            assert mlp is not None

    def __call__(self, r: np.ndarray) -> np.ndarray:
        if self.kind == "rpy":
            return rpy(r, self.a, self.mu)
        return mlp_kernel(r, self.mlp, self.inp)

    @property
    def alpha1(self) -> float:
        return self_mobility(self.a, self.mu)
