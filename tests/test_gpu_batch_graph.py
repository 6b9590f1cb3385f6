"""The batched form through its C-ABI handle (hh_batch_create, hh_batch_matvec).

* the product recorded in a HIP graph and replayed (one graph launch per
  call) equals the eager batched product bit for bit, on new forces copied
  into the recorded input between replays with other device work in between,
  in stored and streamed mode; and every system's rows equal the FP64 dense
  sum over that system within the form's bound;
* the batch workload at full size (64 systems, N log-uniform in [5k, 200k],
  spheres and filaments, BF16): 64 rows per system against the dense FP64
  oracle rows stored by tests/golden/make_rows.py, within 5e-3 in total and
  per system;
* leaf sizes chosen by the autotuner keep the product within that bound.
"""
import hashlib
import os

import numpy as np
import pytest
import torch

import paper_2505_08174_amd as hh
import workloads as wl
from oracle import dense as OD

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


def _systems(sizes, seed0=40):
    Xs = []
    for s, n in enumerate(sizes):
        if s % 2 == 1 and n % 50 == 0:
            Xs.append(wl.filament_chains(n, 0.1, seed=seed0 + s))
        else:
            Xs.append(wl.lattice_cube(n, 0.05 + 0.05 * (s % 5), seed=seed0 + s))
    off = np.concatenate([[0], np.cumsum([x.shape[0] for x in Xs])]).astype(np.int64)
    return Xs, np.concatenate(Xs), off


@pytest.mark.parametrize("kind,prec,mode", [("mlp", "bf16", "stored"), ("mlp", "bf16", "streamed"),
                                            ("rpy", "fp64", "stored"), ("mlp", "fp32", "streamed")])
def test_batch_graph_replay(kind, prec, mode):
    from gpu_common import ctx, dev, kernels, say
    sizes = [700, 3000, 1, 6400, 2500, 65, 150, 4000]
    Xs, X, off = _systems(sizes)
    n = X.shape[0]
    ko, kg = kernels(kind)
    fdt = torch.float64 if prec == "fp64" else torch.float32
    eps = 1e-6 if prec == "fp64" else 1e-4
    cls = np.array([32, 64, 8, 64, 48, 16, 32, 64], dtype=np.int32)
    if mode == "streamed":
        ctx().set_budget(2 << 20)
    try:
        b = hh.Batch(ctx(), dev(X), off, kg, c_leaf=cls, eta=1.0, eps=eps, prec=prec)
        ref_h = hh.HMatrix(ctx(), dev(X), kg, c_leaf=cls, eta=1.0, eps=eps, prec=prec, offsets=off)
    finally:
        ctx().set_budget(64 << 30)
    assert (b.lr.info()["bytes"] == 0) == (mode == "streamed")
    Fb = dev(wl.gravity_forces(n, seed=1), fdt)
    U = b.matvec(Fb)                      # eager product, then the graph is recorded
    info = b.info()
    say("batch graph", kind, prec, mode, info)
    assert info["graph_nodes"] > 0 and info["graph_launches"] == 0
    assert torch.equal(U, ref_h @ Fb)
    for rep in range(3):
        F = wl.gravity_forces(n, seed=10 + rep)
        Fb.copy_(dev(F, fdt))
        junk = torch.randn(4096, device="cuda:0").sum()   # other work between replays
        b.matvec(Fb, U)                   # one graph launch
        torch.cuda.synchronize()
        got = U.clone()
        ref = ref_h @ Fb
        torch.cuda.synchronize()
        assert torch.equal(got, ref), rep
        assert float(junk) == float(junk)
    assert b.info()["graph_launches"] == 3
    Ug = got.double().cpu().numpy()
    tol = 1e-5 if prec == "fp64" else (5e-3 if prec == "bf16" else 1e-3)
    for s, Xk in enumerate(Xs):
        a, e = off[s], off[s + 1]
        rows = wl.sample_rows(e - a, min(e - a, 64), seed=s)
        Ud = OD.dense_u(Xk, F[a:e], ko, rows)
        err = _rel(Ug[a:e][rows], Ud)
        assert err <= tol, (s, err)


def test_batch64_full_size_against_oracle_rows():
    from gpu_common import ctx, dev, kernels, say
    X, F, cfg = wl.workload("batch64")
    d = np.load(os.path.join(GOLDEN, "rows_batch64.npz"))
    assert _digest(X) == str(d["sha_X"]) and _digest(F) == str(d["sha_F"])
    off = cfg["offsets"]
    _, kg = kernels("mlp")
    b = hh.Batch(ctx(), dev(X), off, kg, c_leaf=cfg["c_leaf"], eta=cfg["eta"], eps=cfg["eps"],
                 prec="bf16")
    Fd = dev(F, torch.float32)
    U = b.matvec(Fd)
    b.matvec(Fd, U)                       # a replay of the recorded graph
    torch.cuda.synchronize()
    Ug = U.double().cpu().numpy()
    rows, ref = d["rows"], d["U"]
    e = _rel(Ug[rows], ref)
    sys_of = np.searchsorted(off, rows, side="right") - 1
    per_sys = [_rel(Ug[rows[sys_of == s]], ref[sys_of == s]) for s in range(len(off) - 1)]
    row_err = np.linalg.norm(Ug[rows] - ref, axis=1) / np.max(np.linalg.norm(ref, axis=1))
    say("batch64", X.shape[0], "eps_r", e, "worst system", max(per_sys), "worst row",
        float(row_err.max()), b.info(), b.lr.info())
    assert e <= 5e-3 and max(per_sys) <= 5e-3 and row_err.max() <= 5e-3


def test_autotuned_batch_within_bound():
    from gpu_common import ctx, dev, kernels, say
    from paper_2505_08174_amd import autotune as AT
    sizes = [5000, 9000, 6000, 14000]
    Xs, X, off = _systems(sizes, seed0=70)
    F = wl.normal_forces(X.shape[0], seed=3)
    ko, kg = kernels("mlp")
    Xd, Fd = dev(X), dev(F, torch.float32)
    r = AT.tune_batch(ctx(), Xd, Fd, off, kg, "bf16", 1e-4, 1.0,
                      kinds=["s" if s % 2 == 0 else "f" for s in range(len(sizes))],
                      leaf_candidates=(64, 128, 256), team_candidates=(2048, 4096))
    try:
        say("autotuned", r["c_leafs"].tolist(), r["team_min"])
        assert set(r["c_leafs"].tolist()) <= {64, 128, 256}
        b = hh.Batch(ctx(), Xd, off, kg, c_leaf=r["c_leafs"], eta=1.0, eps=1e-4, prec="bf16")
        Ug = b.matvec(Fd).double().cpu().numpy()
    finally:
        ctx().set_team_min(4096)
    for s, Xk in enumerate(Xs):
        a, e = off[s], off[s + 1]
        rows = wl.sample_rows(e - a, 64, seed=s)
        err = _rel(Ug[a:e][rows], OD.dense_u(Xk, F[a:e], ko, rows))
        say("system", s, "leaf", int(r["c_leafs"][s]), "eps_r", err)
        assert err <= 5e-3
