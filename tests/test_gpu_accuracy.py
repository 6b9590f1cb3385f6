"""Accuracy of the product at full workload size against stored oracle rows.

Eq. (11) over 4,096 rows sampled uniformly (seed 3), against the dense FP64
oracle rows that tests/golden/make_rows.py wrote for the same inputs (SHA-256
of X and F checked), in the launch configuration the benchmark times:
* the plain FP32 form at N = 100,000 (seeded MLP, leaf 128, zeta = 1e-4):
  within 1e-3;
* the BF16 precision form at N = 1,000,000 (spherical drop, gravity-like
  forces): within 5e-3;
* the 6N product with torques at N = 1,000,000 (rotation_1m: FP32, zeta =
  1e-5; 512 rows of (U, w)): within 10 zeta;
* the short-range terms of the same 1M drop in the BF16 form (FP32 MFMA
  networks), against 256 oracle rows of tests/golden/make_short.py: within
  1e-5 (FP32 rounding of the two networks, as at small N).
Besides the global relative error, every sampled row's error is bounded by
the same tolerance relative to the largest sampled row (a few wrong rows
cannot hide in the 2-norm).
"""
import hashlib
import os

import numpy as np
import pytest
import torch

import paper_2505_08174_amd as hh
import workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


@pytest.mark.parametrize("workload,tol", [("plain_fp32", 1e-3), ("precision_1m", 5e-3)])
def test_full_size_against_oracle_rows(workload, tol):
    from gpu_common import ctx, dev, kernels, say
    X, F, cfg = wl.workload(workload)
    d = np.load(os.path.join(GOLDEN, "rows_%s.npz" % workload))
    assert _digest(X) == str(d["sha_X"]) and _digest(F) == str(d["sha_F"])
    rows, ref = d["rows"], d["U"]
    assert rows.size == 4096
    _, kg = kernels(cfg["kernel"])
    prec = cfg["precision"]
    hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=cfg["c_leaf"], eta=cfg["eta"], eps=cfg["eps"],
                    prec=prec)
    U = (hm @ dev(F, torch.float32)).double().cpu().numpy()
    diff = U[rows] - ref
    e = float(np.linalg.norm(diff) / np.linalg.norm(ref))
    row_err = np.linalg.norm(diff, axis=1) / np.max(np.linalg.norm(ref, axis=1))
    own = np.linalg.norm(diff, axis=1) / np.linalg.norm(ref, axis=1)
    say(workload, prec, "n", X.shape[0], "eps_r", e, "worst row (of the largest row)",
        float(row_err.max()), "worst row (own norm)", float(own.max()), hm.lr.info())
    assert e <= tol
    assert row_err.max() <= tol


def _check(name, got, ref, tol):
    from gpu_common import say
    diff = got - ref
    e = float(np.linalg.norm(diff) / np.linalg.norm(ref))
    row_err = np.linalg.norm(diff, axis=1) / np.max(np.linalg.norm(ref, axis=1))
    say(name, "eps_r", e, "worst row (of the largest row)", float(row_err.max()))
    assert e <= tol and row_err.max() <= tol


def test_rotation_full_size_against_oracle_rows():
    from gpu_common import ctx, dev, say
    X, G, cfg = wl.workload("rotation_1m")
    d = np.load(os.path.join(GOLDEN, "rows_rotation_1m.npz"))
    assert _digest(X) == str(d["sha_X"]) and _digest(G) == str(d["sha_F"])
    say("rotation_1m", X.shape[0])
    k6 = hh.Kernel.rpy6(ctx())
    hm = hh.HMatrix(ctx(), dev(X), k6, c_leaf=cfg["c_leaf"], eta=cfg["eta"], eps=cfg["eps"],
                    prec=cfg["precision"])
    Y = (hm @ dev(G, torch.float32)).double().cpu().numpy()
    _check("rotation_1m", Y[d["rows"]], d["U"], 10 * cfg["eps"])


def test_short_range_full_size_against_oracle_rows():
    from gpu_common import ctx, dev, say
    X, F, cfg = wl.workload("precision_1m")
    d = np.load(os.path.join(GOLDEN, "short_precision_1m.npz"))
    assert _digest(X) == str(d["sha_X"]) and _digest(F) == str(d["sha_F"])
    say("short-range precision_1m", X.shape[0])
    tree = hh.build_tree(ctx(), dev(X), cfg["c_leaf"])
    s2, g3 = wl.mlp_weights(11), wl.mlp_weights(12, widths=(6, 64, 64, 64, 18))
    sh = hh.ShortRange(ctx(), tree, s2, g3, float(d["r_cut"]))
    U = torch.zeros(X.shape[0], 3, dtype=torch.float64, device="cuda:0")
    sh.matvec(dev(F, torch.float32), U, "bf16")
    _check("short-range precision_1m", U.cpu().numpy()[d["rows"]], d["U"], 1e-5)
