"""Shared set-up of the GPU tests (imports torch lazily, prints the case)."""
import sys

import numpy as np
import torch

import paper_2505_08174_amd as hh
import workloads as wl
from oracle import kernels as OK

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        _CTX = hh.Context(0)
    return _CTX


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def mlp_params(seed=1):
    return wl.mlp_weights(seed)


def kernels(kind, inp="direction"):
    """(oracle kernel, library kernel) of the same definition."""
    if kind == "rpy":
        return OK.Kernel("rpy"), hh.Kernel.rpy(ctx())
    Ws, bs = mlp_params()
    return OK.Kernel("mlp", OK.MLP(Ws, bs), inp=inp), hh.Kernel.mlp(ctx(), (Ws, bs), inp)
