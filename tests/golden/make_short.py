"""Writes FP64 oracle rows of the short-range terms at a named workload.

For the workload's positions and forces (workloads.workload(name)) and k rows
sampled uniformly without replacement (workloads.sample_rows(n, k, seed=3)),
stores M^(s,2) F + M^(t,3) F + M^(s,3) F of those rows (Eq. (6), the seeded
stand-in networks h_s = mlp_weights(11), g = mlp_weights(12, widths
(6, 64, 64, 64, 18)), R_cut = 5) as computed by oracle.short.short_u_rows, in
tests/golden/short_<workload>.npz with SHA-256 digests of X and F. Only
oracle/ and the input generators are called.

Usage: python tests/golden/make_short.py WORKLOAD [--rows K] [--procs P]
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
from oracle import short as OS  # noqa: E402

_X = _F = _NETS = None


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


def _init(X, F):
    global _X, _F, _NETS
    _X, _F = X, F
    _NETS = (OS.Net(*wl.mlp_weights(11)), OS.Net(*wl.mlp_weights(12, widths=(6, 64, 64, 64, 18))))


def _rows(rows):
    return OS.short_u_rows(_X, _F, _NETS[0], _NETS[1], rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--rows", type=int, default=256)
    ap.add_argument("--procs", type=int, default=max(1, (os.cpu_count() or 2) - 2))
    a = ap.parse_args()
    X, F, cfg = wl.workload(a.workload)
    n = X.shape[0]
    rows = wl.sample_rows(n, min(a.rows, n), seed=3)
    chunks = [rows[i:i + 8] for i in range(0, rows.size, 8)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(a.procs, _init, (X, F)) as pool:
        parts = []
        for i, u in enumerate(pool.imap(_rows, chunks)):
            parts.append(u)
            print("%s: %d / %d chunks, %.0f s" % (a.workload, i + 1, len(chunks),
                                                time.perf_counter() - t0), flush=True)
    U = np.concatenate(parts)
    out = os.path.join(HERE, "short_%s.npz" % a.workload)
    np.savez_compressed(out, workload=a.workload, n=n, rows=rows, U=U, sha_X=digest(X),
                        sha_F=digest(F), seed=3, r_cut=OS.R_CUT)
    print("wrote %s (%d rows, %.0f s)" % (out, rows.size, time.perf_counter() - t0), flush=True)


if __name__ == "__main__":
    main()
