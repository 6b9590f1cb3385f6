"""A product recorded in a hipGraph replays to the eager result.

Stored mode (factors kept) and streamed mode (the ACA with the fused apply
inside the graph), each replayed several times with new forces copied into
the captured input between replays and with eager library and torch work in
between; every replay must equal the eager product bit for bit (the kernels
and their summation order are the same)."""
import numpy as np
import pytest
import torch

import paper_2505_08174_amd as hh
import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("streamed", [False, True])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_graph_replay_equals_eager(streamed, prec):
    from gpu_common import ctx, dev, kernels, say
    say("graph", prec, "streamed" if streamed else "stored")
    n = 5000
    X = wl.rsa_cube(n, 0.15, seed=11)
    _, kg = kernels("mlp")
    if streamed:
        ctx().set_budget(2 << 20)
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
    finally:
        ctx().set_budget(64 << 30)
