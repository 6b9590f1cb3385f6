"""Accuracy of the product at full workload size against stored oracle rows.

Eq. (11) over 4,096 rows sampled uniformly (seed 3), against the dense FP64
oracle rows that tests/golden/make_rows.py wrote for the same inputs (SHA-256
of X and F checked), in the launch configuration the benchmark times:
* the plain FP32 form at N = 100,000 (seeded MLP, leaf 128, zeta = 1e-4):
  within 1e-3;
* the BF16 precision form at N = 1,000,000 (spherical drop, gravity-like
  forces): within 5e-3.
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
