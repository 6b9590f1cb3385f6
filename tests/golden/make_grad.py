"""Writes the dense FP64 oracle gradient of the differentiation workload at
N = 5,000 for the backward checks.

L = sum_i w_i . U_i with U the exact dense product (Eq. (2) restricted to the
one-body and two-body terms), the seeded MLP kernel on the unit direction,
F ~ N(0, I3) and w ~ N(0, I3) (seed 5). Stores dL/dF, dL/dX and dL/dtheta
(packed W1, b1, ..., W4, b4, each row-major [out][in]) from oracle.grad, with
SHA-256 digests of X, F and w, in tests/golden/grad_diff_5k.npz. Only oracle/
and the input generators are called.

Usage: python tests/golden/make_grad.py
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as wl  # noqa: E402
from oracle import grad as OG  # noqa: E402
from oracle import kernels as OK  # noqa: E402

W_SEED = 5


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


def main():
    X, F, cfg = wl.workload("diff_5k")
    n = X.shape[0]
    w = wl.normal_forces(n, seed=W_SEED)
    mlp = OK.MLP(*wl.mlp_weights(1))
    kern = OK.Kernel("mlp", mlp, inp="direction")
    t0 = time.perf_counter()
    dF = OG.dense_grad_F(X, w, kern)
    dX, dW, db = OG.dense_grad_mlp(X, F, w, mlp, inp="direction")
    dth = np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in zip(dW, db)])
    out = os.path.join(HERE, "grad_diff_5k.npz")
    np.savez_compressed(out, dF=dF, dX=dX, dtheta=dth, w_seed=W_SEED, sha_X=digest(X),
                        sha_F=digest(F), sha_w=digest(w), mlp_input="direction")
    print("wrote %s in %.0f s" % (out, time.perf_counter() - t0))


if __name__ == "__main__":
    main()
