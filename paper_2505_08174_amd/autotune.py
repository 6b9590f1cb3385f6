"""Autotuner for the leaf size C_leaf and the workgroup threshold.

The leaf size sets the shape of every near-field tile (|tau| x |sigma| < C_leaf^2)
and of the admissible blocks, so it trades near-field pairs against ACA
samples; the workgroup threshold decides which blocks one 8-wave workgroup
approximates instead of a single wave. Both change the time of a step, never
its definition (the H-matrix error stays bounded by the ACA tolerance).

The tuner times whole steps (tree, partition, ACA and product) on the caller's
own data, as device time from HIP events, and keeps the fastest setting. For a batch of
systems it tunes the leaf size once per size class (systems whose sizes share
a power of two and kind of geometry), on the largest system of the class, then
the threshold on the whole batch.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import api

LEAF_CANDIDATES = (64, 96, 128, 192, 256)
TEAM_CANDIDATES = (2048, 4096, 8192)


def _time_step(ctx, X, F, kern, prec, eps, eta, c_leaf, offsets=None, reps=1):
    """Device seconds of one step (median of reps, after one untimed step):
    the sum of the phases' HIP-event times, so that host overheads of small
    systems do not decide (in a batch they are paid once for all systems)."""
    def step():
        if offsets is None:
            t = api.build_tree(ctx, X, c_leaf)
        else:
            t = api.build_tree_batch(ctx, X, offsets, c_leaf)
        p = api.partition(ctx, t, eta)
        lr = api.aca_build(ctx, t, p, kern, prec, eps)
        api.matvec(ctx, t, p, lr, kern, F, prec)

    step()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        ctx.set_profiling(True)
        ctx.phase_times(reset=True)
        step()
        torch.cuda.synchronize()
        ts.append(sum(ms for ms, _ in ctx.phase_times(reset=True).values()) * 1e-3)
        ctx.set_profiling(False)
    return float(np.median(ts))


def tune_leaf(ctx, X, F, kern, prec="bf16", eps=1e-4, eta=1.0, candidates=LEAF_CANDIDATES):
    """Fastest leaf size for one system; returns (c_leaf, {c_leaf: seconds})."""
    times = {c: _time_step(ctx, X, F, kern, prec, eps, eta, c) for c in candidates}
    return min(times, key=times.get), times


def size_classes(offsets, kinds=None):
    """Groups systems by the power of two of their size (and their kind)."""
    off = np.asarray(offsets, dtype=np.int64)
    sizes = np.diff(off)
    groups = {}
    for s, n in enumerate(sizes):
        key = (int(math.floor(math.log2(max(int(n), 1)))), None if kinds is None else kinds[s])
        groups.setdefault(key, []).append(s)
    return groups


def tune_batch(ctx, X, F, offsets, kern, prec="bf16", eps=1e-4, eta=1.0, kinds=None,
               leaf_candidates=LEAF_CANDIDATES, team_candidates=TEAM_CANDIDATES):
    """Per-system leaf sizes and the workgroup threshold for a batch.

    X, F: device tensors of the concatenated systems; offsets: host array of
    n_sys + 1 particle offsets; kinds: optional label per system (e.g. the
    geometry) that splits size classes further. Returns a dict with
    c_leafs (int32 [n_sys]), team_min and the timings."""
    off = np.asarray(offsets, dtype=np.int64)
    c_leafs = np.zeros(len(off) - 1, dtype=np.int32)
    leaf_times = {}
    for key, members in size_classes(off, kinds).items():
        s = max(members, key=lambda m: off[m + 1] - off[m])
        a, b = int(off[s]), int(off[s + 1])
        best, times = tune_leaf(ctx, X[a:b].contiguous(), F[a:b].contiguous(), kern, prec, eps,
                                eta, leaf_candidates)
        c_leafs[members] = best
        leaf_times[str(key)] = {"system": int(s), "n": b - a, "times": times, "best": best}
    team_times = {}
    for tm in team_candidates:
        ctx.set_team_min(tm)
        team_times[tm] = _time_step(ctx, X, F, kern, prec, eps, eta, c_leafs, off)
    team_min = min(team_times, key=team_times.get)
    ctx.set_team_min(team_min)
    return {"c_leafs": c_leafs, "team_min": int(team_min), "leaf_times": leaf_times,
            "team_times": team_times}
