"""Python face of the C ABI: same call names, torch tensors for device memory
and the current torch stream for ordering. Every step runs in libhh.so."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L

PRECISION = {"fp64": L.HH_FP64, "fp32": L.HH_FP32, "bf16": L.HH_BF16,
             "bf16_split": L.HH_BF16_SPLIT}
F_DTYPE = {L.HH_FP64: torch.float64, L.HH_FP32: torch.float32, L.HH_BF16: torch.float32,
           L.HH_BF16_SPLIT: torch.float32}
U_DTYPE = {L.HH_FP64: torch.float64, L.HH_FP32: torch.float32, L.HH_BF16: torch.float64,
           L.HH_BF16_SPLIT: torch.float64}


def _prec(p):
    return PRECISION[p] if isinstance(p, str) else int(p)


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


class Context:
    """A library context bound to a device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        lib = L.load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        h = C.c_void_p()
        st = lib.hh_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != L.HH_OK:
            raise L.HHError(st, "hh_ctx_create failed")
        self.h = h

    def check(self, status):
        L.check(self.h, status)

    def set_stream(self, stream):
        self.check(L.load().hh_ctx_set_stream(self.h, C.c_void_p(stream.cuda_stream)))

    def synchronize(self):
        self.check(L.load().hh_synchronize(self.h))

    def set_budget(self, nbytes: int):
        self.check(L.load().hh_ctx_set_budget(self.h, int(nbytes)))

    def set_team_min(self, team_min: int):
        """Blocks with c + q >= team_min go to whole workgroups (default 4096)."""
        self.check(L.load().hh_ctx_set_team_min(self.h, int(team_min)))

    def set_profiling(self, on: bool):
        self.check(L.load().hh_ctx_set_profiling(self.h, int(bool(on))))

    def phase_times(self, reset: bool = False):
        """{phase: (ms, count)} accumulated while profiling was on."""
        ms = (C.c_double * L.HH_NPHASE)()
        cnt = (C.c_int64 * L.HH_NPHASE)()
        self.check(L.load().hh_ctx_phase_times(self.h, ms, cnt, int(bool(reset))))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(L.PHASES)}

    def __del__(self):
        try:
            if getattr(self, "h", None):
                L.load().hh_ctx_destroy(self.h)
                self.h = None
        except Exception:
            pass


class _Handle:
    _free = None

    def __init__(self, ctx, h, keep=()):
        self.ctx, self.h, self._keep = ctx, h, keep

    def __del__(self):
        try:
            if getattr(self, "h", None):
                getattr(L.load(), self._free)(self.h)
                self.h = None
        except Exception:   # interpreter shutdown: the library is already gone
            pass


class Kernel(_Handle):
    _free = "hh_kernel_free"

    @staticmethod
    def rpy(ctx: Context, a: float = 1.0, mu: float = 1.0):
        h = C.c_void_p()
        ctx.check(L.load().hh_kernel_create_rpy(ctx.h, a, mu, C.byref(h)))
        k = Kernel(ctx, h)
        k.kind, k.a, k.mu = "rpy", a, mu
        return k

    @staticmethod
    def rpy6(ctx: Context, a: float = 1.0, mu: float = 1.0):
        """The 6N mobility with rotations (forces and torques); goes with
        build_tree6."""
        h = C.c_void_p()
        ctx.check(L.load().hh_kernel_create_rpy6(ctx.h, a, mu, C.byref(h)))
        k = Kernel(ctx, h)
        k.kind, k.a, k.mu = "rpy6", a, mu
        return k

    @staticmethod
    def mlp(ctx: Context, params, input_mode: str = "direction", a: float = 1.0, mu: float = 1.0):
        """params: packed FP64 vector (W1,b1,...,W4,b4) or (Ws, bs) lists."""
        p = pack_mlp(params) if isinstance(params, (tuple, list)) else np.ascontiguousarray(
            params, dtype=np.float64)
        assert p.size == L.HH_MLP_NPARAM
        mode = {"direction": L.HH_MLP_INPUT_DIRECTION,
                "displacement": L.HH_MLP_INPUT_DISPLACEMENT}[input_mode]
        h = C.c_void_p()
        ctx.check(L.load().hh_kernel_create_mlp(ctx.h, p.ctypes.data_as(C.POINTER(C.c_double)),
                                                mode, a, mu, C.byref(h)))
        k = Kernel(ctx, h)
        k.kind, k.a, k.mu, k.params, k.input_mode = "mlp", a, mu, p, input_mode
        return k


def pack_mlp(params):
    Ws, bs = params
    parts = []
    for W, b in zip(Ws, bs):
        parts.append(np.asarray(W, dtype=np.float64).ravel())
        parts.append(np.asarray(b, dtype=np.float64).ravel())
    return np.ascontiguousarray(np.concatenate(parts))


class Tree(_Handle):
    _free = "hh_tree_free"

    def info(self):
        n, nn, nl = C.c_int64(), C.c_int64(), C.c_int64()
        self.ctx.check(L.load().hh_tree_info(self.h, C.byref(n), C.byref(nn), C.byref(nl)))
        return n.value, nn.value, nl.value

    def export(self):
        n, nn, _ = self.info()
        perm = np.empty(n, np.int64)
        keys = np.empty(n, np.uint64)
        nodes = np.empty((nn, 4), np.int32)
        bbox = np.empty((nn, 6), np.float64)
        self.ctx.check(L.load().hh_tree_export(
            self.h, perm.ctypes.data_as(C.POINTER(C.c_int64)),
            keys.ctypes.data_as(C.POINTER(C.c_uint64)), nodes.ctypes.data_as(C.POINTER(C.c_int32)),
            bbox.ctypes.data_as(C.POINTER(C.c_double))))
        return {"perm": perm, "keys": keys, "nodes": nodes, "bbox": bbox}


class Partition(_Handle):
    _free = "hh_part_free"

    def info(self):
        g, h = C.c_int64(), C.c_int64()
        self.ctx.check(L.load().hh_part_info(self.h, C.byref(g), C.byref(h)))
        return g.value, h.value

    def stats(self):
        a, b = C.c_int64(), C.c_int64()
        self.ctx.check(L.load().hh_part_stats(self.h, C.byref(a), C.byref(b)))
        return {"near_pairs": a.value, "far_entries": b.value}

    def export(self):
        ng, nh = self.info()
        G = np.empty((ng, 2), np.int32)
        H = np.empty((nh, 2), np.int32)
        self.ctx.check(L.load().hh_part_export(self.h, G.ctypes.data_as(C.POINTER(C.c_int32)),
                                               H.ctypes.data_as(C.POINTER(C.c_int32))))
        return G, H


class LowRank(_Handle):
    _free = "hh_lowrank_free"

    def info(self):
        v = [C.c_int64() for _ in range(5)]
        self.ctx.check(L.load().hh_lowrank_info(self.h, *[C.byref(x) for x in v]))
        keys = ("n_blocks", "rank_sum", "n_fallback", "samples", "bytes")
        return dict(zip(keys, [x.value for x in v]))

    def export(self):
        nb = self.info()["n_blocks"]
        rank = np.empty(nb, np.int32)
        fb = np.empty(nb, np.int32)
        pi = np.empty((nb, L.LMAX_CAP), np.int32)
        pj = np.empty((nb, L.LMAX_CAP), np.int32)
        p32 = C.POINTER(C.c_int32)
        self.ctx.check(L.load().hh_lowrank_export(self.h, rank.ctypes.data_as(p32),
                                                  fb.ctypes.data_as(p32), pi.ctypes.data_as(p32),
                                                  pj.ctypes.data_as(p32)))
        return {"rank": rank, "fallback": fb, "piv_i": pi, "piv_j": pj}

    def factor(self, b: int, k: int, c: int, q: int):
        ck = np.empty((c, 3, 3))
        qk = np.empty((q, 3, 3))
        pd = C.POINTER(C.c_double)
        self.ctx.check(L.load().hh_lowrank_factor(self.h, b, k, ck.ctypes.data_as(pd),
                                                  qk.ctypes.data_as(pd)))
        return ck, qk


def build_tree(ctx: Context, X: torch.Tensor, c_leaf: int) -> Tree:
    assert X.is_cuda and X.dtype == torch.float64 and X.dim() == 2 and X.shape[1] == 3
    X = X.contiguous()
    h = C.c_void_p()
    ctx.check(L.load().hh_build_tree(ctx.h, _ptr(X), X.shape[0], int(c_leaf), C.byref(h)))
    return Tree(ctx, h)


def build_tree6(ctx: Context, X: torch.Tensor, c_leaf: int) -> Tree:
    """Tree of the 2n rows (translation, rotation of every particle) of the
    6N mobility; c_leaf counts particles."""
    assert X.is_cuda and X.dtype == torch.float64 and X.dim() == 2 and X.shape[1] == 3
    X = X.contiguous()
    h = C.c_void_p()
    ctx.check(L.load().hh_build_tree6(ctx.h, _ptr(X), X.shape[0], int(c_leaf), C.byref(h)))
    t = Tree(ctx, h)
    t.six = True
    return t


def build_tree_batch(ctx: Context, X: torch.Tensor, offsets, c_leaf) -> Tree:
    """One tree over several independent systems (concatenated in X); c_leaf
    is one leaf size or one per system."""
    assert X.is_cuda and X.dtype == torch.float64 and X.dim() == 2 and X.shape[1] == 3
    X = X.contiguous()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    assert off[0] == 0 and off[-1] == X.shape[0]
    h = C.c_void_p()
    p64 = off.ctypes.data_as(C.POINTER(C.c_int64))
    if np.ndim(c_leaf) == 0:
        ctx.check(L.load().hh_build_tree_batch(ctx.h, _ptr(X), p64, len(off) - 1, int(c_leaf),
                                               C.byref(h)))
    else:
        cl = np.ascontiguousarray(c_leaf, dtype=np.int32)
        assert cl.shape == (len(off) - 1,)
        ctx.check(L.load().hh_build_tree_batch_leaf(ctx.h, _ptr(X), p64, len(off) - 1,
                                                    cl.ctypes.data_as(C.POINTER(C.c_int32)),
                                                    C.byref(h)))
    return Tree(ctx, h)


def partition(ctx: Context, tree: Tree, eta: float = 1.0, dense_mode: bool = False) -> Partition:
    h = C.c_void_p()
    ctx.check(L.load().hh_partition(ctx.h, tree.h, float(eta), int(bool(dense_mode)), C.byref(h)))
    return Partition(ctx, h, keep=(tree,))


def aca_build(ctx: Context, tree: Tree, part: Partition, kern: Kernel, prec="fp64",
              eps: float = 1e-6, l_max: int = 48, freeze_pivots_from: LowRank | None = None
              ) -> LowRank:
    """ACA of every admissible block; with freeze_pivots_from, the recursion
    replayed with that handle's pivots, ranks and fallbacks."""
    h = C.c_void_p()
    fz = freeze_pivots_from.h if freeze_pivots_from is not None else C.c_void_p(0)
    ctx.check(L.load().hh_aca_build(ctx.h, tree.h, part.h, kern.h, _prec(prec), float(eps),
                                    int(l_max), fz, C.byref(h)))
    return LowRank(ctx, h, keep=(tree, part, kern))


def aca_build_pivots(ctx: Context, tree: Tree, part: Partition, kern: Kernel, prec, rank,
                     fallback, piv_i, piv_j) -> LowRank:
    """Factors from the ACA recursion with the given pivots (host arrays:
    rank [nG], fallback [nG], piv_i and piv_j [nG, 64])."""
    ng = part.info()[0]
    rk = np.ascontiguousarray(rank, dtype=np.int32)
    fb = np.ascontiguousarray(fallback, dtype=np.int32)
    pi = np.full((max(ng, 1), L.LMAX_CAP), -1, np.int32)
    pj = np.full((max(ng, 1), L.LMAX_CAP), -1, np.int32)
    if ng:
        pi[:ng, :np.shape(piv_i)[1]] = piv_i
        pj[:ng, :np.shape(piv_j)[1]] = piv_j
    assert rk.shape == (ng,) and fb.shape == (ng,)
    p32 = C.POINTER(C.c_int32)
    h = C.c_void_p()
    ctx.check(L.load().hh_aca_build_pivots(ctx.h, tree.h, part.h, kern.h, _prec(prec),
                                           rk.ctypes.data_as(p32), fb.ctypes.data_as(p32),
                                           pi.ctypes.data_as(p32), pj.ctypes.data_as(p32),
                                           C.byref(h)))
    return LowRank(ctx, h, keep=(tree, part, kern))


def tree_refit(ctx: Context, tree: Tree, X: torch.Tensor) -> Tree:
    """New positions for `tree`, keeping its order and nodes (in place)."""
    rows = tree.info()[0] // (2 if getattr(tree, "six", False) else 1)
    assert X.is_cuda and X.dtype == torch.float64 and X.shape == (rows, 3)
    X = X.contiguous()
    ctx.check(L.load().hh_tree_refit(ctx.h, tree.h, _ptr(X)))
    return tree


def matvec(ctx: Context, tree: Tree, part: Partition, lr: LowRank, kern: Kernel, F: torch.Tensor,
           prec="fp64", U: torch.Tensor | None = None) -> torch.Tensor:
    p = _prec(prec)
    # [n][3], or [n/2][6] = (F_i, T_i) on a tree of build_tree6
    assert F.is_cuda and F.dtype == F_DTYPE[p] and F.numel() == 3 * tree.info()[0]
    assert F.shape[-1] == (6 if getattr(tree, "six", False) else 3)
    F = F.contiguous()
    if U is None:
        U = torch.empty(F.shape, dtype=U_DTYPE[p], device=F.device)
    assert U.dtype == U_DTYPE[p] and U.is_contiguous() and U.shape == F.shape
    ctx.check(L.load().hh_matvec(ctx.h, tree.h, part.h, lr.h, kern.h, p, _ptr(F), _ptr(U)))
    return U


def matvec_noalloc(ctx: Context, tree: Tree, part: Partition, lr: LowRank, kern: Kernel,
                   F: torch.Tensor, U: torch.Tensor, prec="fp64") -> torch.Tensor:
    """hh_matvec_noalloc: the stored-mode product with its workspaces in the
    library's static device scratch (U must be given: nothing is allocated)."""
    p = _prec(prec)
    assert F.is_cuda and F.dtype == F_DTYPE[p] and F.is_contiguous()
    assert F.numel() == 3 * tree.info()[0]
    assert U.dtype == U_DTYPE[p] and U.is_contiguous() and U.shape == F.shape
    ctx.check(L.load().hh_matvec_noalloc(ctx.h, tree.h, part.h, lr.h, kern.h, p, _ptr(F),
                                         _ptr(U)))
    return U


def matvec_backward(ctx: Context, tree: Tree, part: Partition, lr: LowRank, kern: Kernel,
                    F: torch.Tensor, dU: torch.Tensor, prec="fp64", want=("F", "X", "theta")):
    """(dF, dX, dtheta) of L = sum dU . U with the structure frozen (None where
    not requested). dtheta is the packed FP64 parameter vector."""
    p = _prec(prec)
    n = tree.info()[0]
    F, dU = F.contiguous(), dU.contiguous()
    assert F.dtype == F_DTYPE[p] and dU.dtype == U_DTYPE[p] and F.shape == dU.shape == (n, 3)
    dF = torch.empty_like(F) if "F" in want else None
    dX = torch.empty((n, 3), dtype=torch.float64, device=F.device) if "X" in want else None
    dth = (torch.zeros(L.HH_MLP_NPARAM, dtype=torch.float64, device=F.device)
           if "theta" in want else None)
    nul = C.c_void_p(0)
    ctx.check(L.load().hh_matvec_backward(
        ctx.h, tree.h, part.h, lr.h, kern.h, p, _ptr(F), _ptr(dU),
        _ptr(dF) if dF is not None else nul, _ptr(dX) if dX is not None else nul,
        _ptr(dth) if dth is not None else nul))
    return dF, dX, dth


class HMatvecFn(torch.autograd.Function):
    """U = M_H(X; theta) F with the H-matrix rebuilt from X in the forward and
    its structure frozen for the backward. theta: packed FP64 MLP parameters
    (a CPU tensor). cfg: dict(c_leaf, eta, eps, prec, l_max, input_mode)."""

    @staticmethod
    def forward(fctx, X, F, theta, ctx, cfg):
        kern = Kernel.mlp(ctx, theta.detach().cpu().double().numpy(), cfg.get("input_mode", "direction"))
        hm = HMatrix(ctx, X.detach(), kern, cfg.get("c_leaf", 64), cfg.get("eta", 1.0),
                     cfg.get("eps", 1e-6), cfg.get("prec", "fp64"), cfg.get("l_max", 48))
        U = hm @ F.detach()
        fctx.hm = hm
        fctx.save_for_backward(F)
        fctx.theta_device = theta.device
        return U

    @staticmethod
    def backward(fctx, gU):
        (F,) = fctx.saved_tensors
        hm = fctx.hm
        want = []
        if fctx.needs_input_grad[1]:
            want.append("F")
        if fctx.needs_input_grad[0]:
            want.append("X")
        if fctx.needs_input_grad[2]:
            want.append("theta")
        dF, dX, dth = matvec_backward(hm.ctx, hm.tree, hm.part, hm.lr, hm.kern, F,
                                      gU.contiguous().to(U_DTYPE[hm.prec]), hm.prec, tuple(want))
        if dth is not None:
            dth = dth.to(fctx.theta_device)
        return dX, dF, dth, None, None


def hmatvec_autograd(ctx, X, F, theta, **cfg):
    return HMatvecFn.apply(X, F, theta, ctx, cfg)


class HMatrix:
    """Tree + partition + factors for one configuration X (rebuilt when X moves).
    offsets: optional particle offsets of several independent systems in X."""

    def __init__(self, ctx, X, kern, c_leaf=64, eta=1.0, eps=1e-6, prec="fp64", l_max=48,
                 dense_mode=False, offsets=None):
        self.ctx, self.kern, self.prec = ctx, kern, _prec(prec)
        if getattr(kern, "kind", None) == "rpy6":
            assert offsets is None
            self.tree = build_tree6(ctx, X, c_leaf)
        elif offsets is None:
            self.tree = build_tree(ctx, X, c_leaf)
        else:
            self.tree = build_tree_batch(ctx, X, offsets, c_leaf)
        self.part = partition(ctx, self.tree, eta, dense_mode)
        self.lr = aca_build(ctx, self.tree, self.part, kern, self.prec, eps, l_max)

    def __matmul__(self, F):
        return matvec(self.ctx, self.tree, self.part, self.lr, self.kern, F, self.prec)

    def capture(self, F: torch.Tensor):
        """Record the product U = M F in a hipGraph (a torch.cuda.CUDAGraph).

        One eager product runs first (it sizes every workspace, so the
        recorded launches allocate nothing); replaying the graph recomputes U
        (returned) from the current contents of F. In streamed mode the graph
        holds the whole ACA with the fused apply. F and U must keep their
        storage while the graph is in use; products on one H-matrix must not
        overlap in time. Returns (graph, U)."""
        assert F.is_contiguous()
        U = torch.empty(F.shape, dtype=U_DTYPE[self.prec], device=F.device)
        matvec(self.ctx, self.tree, self.part, self.lr, self.kern, F, self.prec, U)
        torch.cuda.synchronize(F.device)
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(F.device)
        home = torch.cuda.current_stream(F.device)
        try:
            with torch.cuda.graph(g, stream=side):
                self.ctx.set_stream(side)
                matvec(self.ctx, self.tree, self.part, self.lr, self.kern, F, self.prec, U)
        finally:
            self.ctx.set_stream(home)
        return g, U


class _Borrowed:
    """A handle owned by another object (not freed here)."""

    def __del__(self):
        pass


class _BTree(_Borrowed, Tree):
    pass


class _BPart(_Borrowed, Partition):
    pass


class _BLowRank(_Borrowed, LowRank):
    pass


class Batch(_Handle):
    """Many independent systems in one handle (hh_batch_create); the product
    is recorded once in a HIP graph and replayed by one graph launch per call
    (hh_batch_matvec). c_leaf: one leaf size or one per system."""
    _free = "hh_batch_free"

    def __init__(self, ctx: Context, X: torch.Tensor, offsets, kern: Kernel, c_leaf=128,
                 eta: float = 1.0, eps: float = 1e-4, prec="bf16", l_max: int = 48):
        assert X.is_cuda and X.dtype == torch.float64 and X.dim() == 2 and X.shape[1] == 3
        X = X.contiguous()
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        assert off[0] == 0 and off[-1] == X.shape[0]
        prm = L.BatchParams()
        prm.n_sys = len(off) - 1
        prm.offsets = off.ctypes.data_as(C.POINTER(C.c_int64))
        cl = None
        if np.ndim(c_leaf) == 0:
            prm.c_leafs = C.POINTER(C.c_int32)()
            prm.c_leaf = int(c_leaf)
        else:
            cl = np.ascontiguousarray(c_leaf, dtype=np.int32)
            assert cl.shape == (prm.n_sys,)
            prm.c_leafs = cl.ctypes.data_as(C.POINTER(C.c_int32))
            prm.c_leaf = 0
        prm.eta, prm.eps, prm.l_max, prm.prec = float(eta), float(eps), int(l_max), _prec(prec)
        h = C.c_void_p()
        ctx.check(L.load().hh_batch_create(ctx.h, _ptr(X), C.byref(prm), kern.h, C.byref(h)))
        super().__init__(ctx, h, keep=(kern,))
        self.kern, self.prec, self.offsets = kern, _prec(prec), off
        tree, part, lr = C.c_void_p(), C.c_void_p(), C.c_void_p()
        ctx.check(L.load().hh_batch_info(h, None, None, None, None, C.byref(tree), C.byref(part),
                                         C.byref(lr)))
        self.tree = _BTree(ctx, tree)
        self.part = _BPart(ctx, part)
        self.lr = _BLowRank(ctx, lr)

    def info(self):
        n, ns, nodes, launches = C.c_int64(), C.c_int32(), C.c_int64(), C.c_int64()
        self.ctx.check(L.load().hh_batch_info(self.h, C.byref(n), C.byref(ns), C.byref(nodes),
                                              C.byref(launches), None, None, None))
        return {"n": n.value, "n_sys": ns.value, "graph_nodes": nodes.value,
                "graph_launches": launches.value}

    def matvec(self, F: torch.Tensor, U: torch.Tensor | None = None) -> torch.Tensor:
        """U = M F; the first call with these buffers records the graph, later
        calls replay it (F and U must keep their storage)."""
        n = int(self.offsets[-1])
        assert F.is_cuda and F.dtype == F_DTYPE[self.prec] and F.shape == (n, 3)
        assert F.is_contiguous()
        if U is None:
            U = torch.empty(F.shape, dtype=U_DTYPE[self.prec], device=F.device)
        assert U.dtype == U_DTYPE[self.prec] and U.is_contiguous() and U.shape == F.shape
        self.ctx.check(L.load().hh_batch_matvec(self.ctx.h, self.h, _ptr(F), _ptr(U)))
        return U


class ShortRange(_Handle):
    """The short-range many-body terms M^(s,2) F + M^(t,3) F + M^(s,3) F of a
    tree's current positions (hh_short_create); s2 and g3 are packed FP64
    parameter vectors or (Ws, bs) lists of the two stand-in networks."""
    _free = "hh_short_free"

    def __init__(self, ctx: Context, tree: Tree, s2, g3, r_cut: float = 5.0):
        p2 = pack_mlp(s2) if isinstance(s2, (tuple, list)) else np.ascontiguousarray(s2, np.float64)
        p3 = pack_mlp(g3) if isinstance(g3, (tuple, list)) else np.ascontiguousarray(g3, np.float64)
        assert p2.size == L.HH_MLP_NPARAM and p3.size == L.HH_G3_NPARAM
        pd = C.POINTER(C.c_double)
        h = C.c_void_p()
        ctx.check(L.load().hh_short_create(ctx.h, tree.h, p2.ctypes.data_as(pd),
                                           p3.ctypes.data_as(pd), float(r_cut), C.byref(h)))
        super().__init__(ctx, h, keep=(tree,))
        self.n = tree.info()[0]

    def info(self):
        a, b = C.c_int64(), C.c_int64()
        self.ctx.check(L.load().hh_short_info(self.h, C.byref(a), C.byref(b)))
        return {"n_pairs": a.value, "n_cliques": b.value}

    def matvec(self, F: torch.Tensor, U: torch.Tensor, prec="fp64") -> torch.Tensor:
        """U += M^(s,2) F + M^(t,3) F + M^(s,3) F (in place)."""
        p = _prec(prec)
        assert F.is_cuda and F.dtype == F_DTYPE[p] and F.is_contiguous() and F.shape == (self.n, 3)
        assert U.dtype == U_DTYPE[p] and U.is_contiguous() and U.shape == F.shape
        self.ctx.check(L.load().hh_short_matvec(self.ctx.h, self.h, p, _ptr(F), _ptr(U)))
        return U


def hmatvec(ctx, X, F, kern, c_leaf=64, eta=1.0, eps=1e-6, prec="fp64", l_max=48):
    """One full step: tree, partition, ACA and product."""
    return HMatrix(ctx, X, kern, c_leaf, eta, eps, prec, l_max) @ F
