"""A product recorded in a hipGraph replays to the eager result.

Stored mode (factors kept) and streamed mode (the ACA with the fused apply
inside the graph), the latter also with most blocks given to workgroups so
that huge blocks form tiers and the two ACA kernels run concurrently (the
team kernel on the context's second stream, forked and joined inside the
graph), each replayed several times with new forces copied into
the captured input between replays and with eager library and torch work in
between; every replay must equal the eager product bit for bit (the kernels
and their summation order are the same)."""
import numpy as np
import pytest
import torch

import paper_2505_08174_amd as hh
import workloads as wl
from oracle import dense as OD

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["stored", "streamed", "streamed_teams"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_graph_replay_equals_eager(mode, prec):
    from gpu_common import ctx, dev, kernels, say
    say("graph", prec, mode)
    # streamed_teams: at N = 20000 the 2 MiB budget, leaf 64 and a workgroup
    # threshold of 64 give 2456 huge blocks in 3 size-class tiers, and 64 of the
    # 218 launch ranges run the two ACA kernels concurrently (huge blocks hold
    # 5% or more of their rows; counted from the oracle's tree and partition)
    n = 20000 if mode == "streamed_teams" else 5000
    X = wl.rsa_cube(n, 0.15, seed=11)
    ko, kg = kernels("mlp")
    streamed = mode != "stored"
    if streamed:
        ctx().set_budget(2 << 20)
    if mode == "streamed_teams":
        ctx().set_team_min(64)
    try:
        hm = hh.HMatrix(ctx(), dev(X), kg, c_leaf=64, eps=1e-4, prec=prec)
        assert hm.lr.info()["bytes"] == 0 if streamed else hm.lr.info()["bytes"] > 0
        Fs = dev(wl.normal_forces(n, seed=0), torch.float32)
        g, U = hm.capture(Fs)
        for rep in range(4):
            F = dev(wl.normal_forces(n, seed=100 + rep), torch.float32)
            Fs.copy_(F)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = U.clone()
            # eager work between replays: another product and torch ops
            ref = hm @ F
            junk = torch.randn(1000, device="cuda:0").sum()
            torch.cuda.synchronize()
            say("replay", rep, float(junk) == float(junk))
            assert torch.equal(got, ref), rep
            assert float(torch.linalg.norm(ref)) > 0
        if mode == "streamed_teams":
            # the tiered, concurrent path against the FP64 dense sum
            rows = wl.sample_rows(n, 200, seed=7)
            Ud = OD.dense_u(X, F.double().cpu().numpy(), ko, rows)
            Ug = got.double().cpu().numpy()[rows]
            e = float(np.linalg.norm(Ug - Ud) / np.linalg.norm(Ud))
            say("streamed_teams eps_r", prec, e)
            assert e <= (5e-3 if prec == "bf16" else 1e-3)
    finally:
        ctx().set_budget(64 << 30)
        ctx().set_team_min(4096)
