"""Writes FP64 dense-oracle rows of named workloads for the accuracy checks.

For a workload (workloads.workload(name)) and k rows sampled uniformly
without replacement (workloads.sample_rows(n, k, seed=3)), stores the exact
dense product U_i = alpha_1 F_i + sum_{j != i} K(x_i - x_j) F_j of those rows
(Eq. (2) restricted to the one-body and two-body terms), as computed by
oracle.dense (for the 6N kernel: the rows (U_i, w_i) of oracle.rotation's
dense 6N product), in tests/golden/rows_<workload>.npz together with SHA-256
digests of X and F, so a reader can check that it compares against the same
inputs. For a workload of many independent systems, k / n_sys rows are
sampled in each system (workloads.sample_rows(n_s, k / n_sys, seed=3)) and
the sum runs over the row's own system. Only oracle/ and the input
generators are called.

Usage: python tests/golden/make_rows.py WORKLOAD [WORKLOAD ...] [--rows K] [--procs P]
"""
from __future__ import annotations

import argparse
import hashlib
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import dense as OD  # noqa: E402
from oracle import kernels as OK  # noqa: E402
from oracle import rotation as OR  # noqa: E402

_X = _F = _K = None


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


def oracle_kernel(cfg):
    if cfg["kernel"] == "rpy6":
        return "rpy6"
    if cfg["kernel"] == "rpy":
        return OK.Kernel("rpy")
    return OK.Kernel("mlp", OK.MLP(*wl.mlp_weights(1)), inp="direction")


def _init(X, F, kind):
    global _X, _F, _K
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass
    _X, _F = X, F
    _K = oracle_kernel({"kernel": kind})


def _rows(task):
    a, b, rows = task   # particles [a, b) form the row's system; rows are local
    if isinstance(_K, str):   # the 6N kernel
        U, W = OR.u6(_X[a:b], _F[a:b, :3], _F[a:b, 3:], rows=rows)
        return np.hstack([U, W])
    return OD.dense_u(_X[a:b], _F[a:b], _K, rows)


def make(name: str, k: int, procs: int) -> str:
    X, F, cfg = wl.workload(name)
    n = X.shape[0]
    off = cfg.get("offsets")
    if off is None:
        rows = wl.sample_rows(n, min(k, n), seed=3)
        chunks = [(0, n, rows[i:i + 8]) for i in range(0, rows.size, 8)]
    else:
        per = max(1, k // (len(off) - 1))
        rows, chunks = [], []
        for s_ in range(len(off) - 1):
            a, b = int(off[s_]), int(off[s_ + 1])
            loc = wl.sample_rows(b - a, min(per, b - a), seed=3)
            rows.append(loc + a)
            chunks += [(a, b, loc[i:i + 8]) for i in range(0, loc.size, 8)]
        rows = np.concatenate(rows)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs, _init, (X, F, cfg["kernel"])) as pool:
        parts = []
        for i, u in enumerate(pool.imap(_rows, chunks)):
            parts.append(u)
            if i % 32 == 0:
                print("%s: %d / %d chunks, %.0f s" % (name, i + 1, len(chunks),
                                                    time.perf_counter() - t0), flush=True)
    U = np.concatenate(parts)
    out = os.path.join(HERE, "rows_%s.npz" % name)
    np.savez_compressed(out, workload=name, n=n, rows=rows, U=U, sha_X=digest(X),
                        sha_F=digest(F), seed=3, kernel=cfg["kernel"], mlp_input="direction")
    print("wrote %s (%d rows, %.0f s)" % (out, rows.size, time.perf_counter() - t0), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="+")
    ap.add_argument("--rows", type=int, default=4096)
    ap.add_argument("--procs", type=int, default=max(1, (os.cpu_count() or 2) - 2))
    a = ap.parse_args()
    for name in a.workloads:
        make(name, a.rows, a.procs)


if __name__ == "__main__":
    main()
