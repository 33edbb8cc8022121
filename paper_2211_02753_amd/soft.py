"""Relaxed (differentiable) filter and grouped aggregation, exposed as
torch.autograd.Functions whose forward and backward both run libtdp kernels.

``SoftFilterGroupBy`` saves only its inputs (x, v, g, c) and recomputes the
logistic mask in the backward kernel.
"""
from __future__ import annotations

import torch

from . import _lib as L

_WS = {}


def new_soft_workspace(device) -> torch.Tensor:
    """Allocate and prepare a workspace for the soft calls (on the current stream)."""
    lib = L.load()
    ws = L.workspace(lib.tdp_soft_workspace_size(), device)
    L.check("tdp_soft_workspace_init", lib.tdp_soft_workspace_init(L.ptr(ws), ws.numel(), L.stream_handle(device)))
    return ws


def soft_workspace(device) -> torch.Tensor:
    """The shared workspace of this device (calls using it run on one stream)."""
    key = str(torch.device(device))
    if key not in _WS:
        _WS[key] = new_soft_workspace(device)
    return _WS[key]


def _s(dev):
    return L.stream_handle(dev)


def _need(t, dtype, name, dims=None):
    """Raise unless t is a contiguous device tensor of dtype (and of dims dimensions)."""
    if t is None:
        return
    if not torch.is_tensor(t) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        got = (t.dtype, t.device, t.is_contiguous()) if torch.is_tensor(t) else type(t)
        raise TypeError(f"{name} must be a contiguous {dtype} tensor on the GPU, got {got}")
    if dims is not None and t.dim() not in dims:
        raise ValueError(f"{name} must have {' or '.join(map(str, dims))} dimensions, got {t.dim()}")


def _raise_flags(st, what):
    """Synchronise on the status word of a call and raise on any device flag."""
    v = int(st.item())
    if v:
        names = [n for n, bit in [("KEY_DOMAIN", L.FLAG_KEY_DOMAIN), ("GROUP_RANGE", L.FLAG_GROUP_RANGE),
                                  ("SPIN", L.FLAG_SPIN), ("BAD_PARAM", L.FLAG_BAD_PARAM)] if v & bit]
        raise L.TdpError(what, L.TDP_EINVAL, "device flags " + ("|".join(names) or hex(v)))


def soft_filter(x: torch.Tensor, c: torch.Tensor, tau: float) -> torch.Tensor:
    lib = L.load()
    _need(x, torch.float32, "x")
    _need(c, torch.float32, "c")
    w = torch.empty_like(x)
    L.check("tdp_soft_filter", lib.tdp_soft_filter(L.ptr(x), x.numel(), L.ptr(c), float(tau), L.ptr(w), _s(x.device)))
    return w


def soft_filter_bwd(x, c, tau, dw, want_dx=True, want_dtau=False):
    """(dx, dc), or (dx, dc, dtau) when want_dtau."""
    lib = L.load()
    for t, name in ((x, "x"), (c, "c"), (dw, "dw")):
        _need(t, torch.float32, name)
    dx = torch.empty_like(x) if want_dx else None
    dc = torch.empty(1, dtype=torch.float32, device=x.device)
    dtau = torch.empty(1, dtype=torch.float32, device=x.device) if want_dtau else None
    ws = soft_workspace(x.device)
    L.check("tdp_soft_filter_bwd", lib.tdp_soft_filter_bwd(L.ptr(x), x.numel(), L.ptr(c), float(tau), L.ptr(dw),
                                                           L.ptr(dx), L.ptr(dc), L.ptr(dtau), L.ptr(ws), ws.numel(),
                                                           _s(x.device)))
    return (dx, dc, dtau) if want_dtau else (dx, dc)


def soft_groupby(g, w, v, G, status=None):
    """S[G, K] (or [G] for 1-d v) with S[g, k] = sum_{g_i = g} w_i v[i, k].

    Without a status tensor the call synchronises and raises when a group id
    falls outside [0, G); with one, the flags are left in it for the caller."""
    lib = L.load()
    _need(g, torch.int32, "g", (1,))
    _need(w, torch.float32, "w", (1,))
    _need(v, torch.float32, "v", (1, 2))
    if v.shape[0] != g.numel() or (w is not None and w.numel() != g.numel()):
        raise ValueError("g, w and the rows of v must have the same length")
    K = 1 if v.dim() == 1 else v.shape[1]
    S = torch.empty((G, K), dtype=torch.float32, device=v.device)
    st = torch.zeros(1, dtype=torch.int32, device=v.device) if status is None else status
    ws = soft_workspace(v.device)
    L.check("tdp_soft_groupby", lib.tdp_soft_groupby(L.ptr(g), L.ptr(w), L.ptr(v), g.numel(), K, G, L.ptr(S), L.ptr(st),
                                                     L.ptr(ws), ws.numel(), _s(v.device)))
    if status is None:
        _raise_flags(st, "tdp_soft_groupby")
    return S[:, 0] if v.dim() == 1 else S


def soft_groupby_bwd(g, w, v, dS, want_dw=True, want_dv=True):
    lib = L.load()
    _need(g, torch.int32, "g", (1,))
    _need(w, torch.float32, "w", (1,))
    _need(v, torch.float32, "v", (1, 2))
    dS = dS.contiguous()
    _need(dS, torch.float32, "dS", (1, 2))
    K = 1 if v.dim() == 1 else v.shape[1]
    G = dS.shape[0]
    dw = torch.empty(g.numel(), dtype=torch.float32, device=v.device) if want_dw else None
    dS = dS.contiguous()  # a copy must outlive the asynchronous call
    dv = torch.empty_like(v) if want_dv else None
    L.check("tdp_soft_groupby_bwd", lib.tdp_soft_groupby_bwd(L.ptr(g), L.ptr(w), L.ptr(v), L.ptr(dS),
                                                             g.numel(), K, G, L.ptr(dw), L.ptr(dv), _s(v.device)))
    return dw, dv


def soft_pe_groupby(p, q=None, seg=None, G=1, status=None):
    """S[G, K1, K2] with S[g, a, b] = sum over segment g's rows of p[i, a] q[i, b]
    (q None: q = 1, K2 = 1; seg None: one segment of all rows, G = 1)."""
    lib = L.load()
    _need(p, torch.float32, "p", (2,))
    _need(q, torch.float32, "q", (2,))
    _need(seg, torch.int64, "seg", (1,))
    if q is not None and q.shape[0] != p.shape[0]:
        raise ValueError("p and q must have the same rows")
    if seg is not None and seg.numel() != G + 1:
        raise ValueError("seg must hold G + 1 offsets")
    K1 = p.shape[1]
    K2 = 1 if q is None else q.shape[1]
    S = torch.empty((G, K1, K2), dtype=torch.float32, device=p.device)
    st = torch.zeros(1, dtype=torch.int32, device=p.device) if status is None else status
    ws = soft_workspace(p.device)
    L.check("tdp_soft_pe_groupby",
            lib.tdp_soft_pe_groupby(L.ptr(seg), G, L.ptr(p), K1, L.ptr(q), K2, p.shape[0], L.ptr(S), L.ptr(st),
                                    L.ptr(ws), ws.numel(), _s(p.device)))
    if status is None:
        _raise_flags(st, "tdp_soft_pe_groupby")
    return S


def soft_pe_groupby_bwd(p, q, seg, dS, want_dp=True, want_dq=True):
    """(dp, dq) from dS[G, K1, K2]; dq is None when q is None or not wanted."""
    lib = L.load()
    dS = dS.contiguous()
    for t, name, dt, dims in ((p, "p", torch.float32, (2,)), (q, "q", torch.float32, (2,)),
                              (seg, "seg", torch.int64, (1,)), (dS, "dS", torch.float32, (3,))):
        _need(t, dt, name, dims)
    G, K1, K2 = dS.shape
    dp = torch.empty_like(p) if want_dp else None
    dq = torch.empty_like(q) if (want_dq and q is not None) else None
    dS = dS.contiguous()  # a copy must outlive the asynchronous call
    L.check("tdp_soft_pe_groupby_bwd",
            lib.tdp_soft_pe_groupby_bwd(L.ptr(seg), G, L.ptr(p), K1, L.ptr(q), K2, p.shape[0], L.ptr(dS),
                                        L.ptr(dp), L.ptr(dq), _s(p.device)))
    return dp, dq


class SoftPEGroupBy(torch.autograd.Function):
    """S[g, a, b] = sum over segment g's rows of p[i, a] q[i, b]: the soft COUNT
    grouped by two probability-encoded attributes, differentiable in p and q."""

    @staticmethod
    def forward(ctx, p, q, seg, G: int):
        S = soft_pe_groupby(p, q, seg, G)
        ctx.save_for_backward(p, q, seg)
        return S

    @staticmethod
    def backward(ctx, dS):
        p, q, seg = ctx.saved_tensors
        dp, dq = soft_pe_groupby_bwd(p, q, seg, dS, ctx.needs_input_grad[0], ctx.needs_input_grad[1])
        return dp, dq, None, None


class SoftFilterGroupBy(torch.autograd.Function):
    """S_g = sum_{i: g_i = g} sigmoid((c - x_i) / tau) v_i, differentiable in c, v and x, and in tau when tau is
    a one-element tensor that requires grad (a float tau is a fixed hyperparameter)."""

    @staticmethod
    def forward(ctx, x, v, g, c, tau, G: int):
        lib = L.load()
        for t, name in ((x, "x"), (v, "v"), (c, "c")):
            _need(t, torch.float32, name, (1,))
        _need(g, torch.int32, "g", (1,))
        if v.numel() != x.numel() or g.numel() != x.numel() or c.numel() != 1:
            raise ValueError("x, v and g must have the same length and c one element")
        S = torch.empty(G, dtype=torch.float32, device=x.device)
        st = torch.zeros(1, dtype=torch.int32, device=x.device)
        ws = soft_workspace(x.device)
        L.check("tdp_soft_filter_groupby",
                lib.tdp_soft_filter_groupby(L.ptr(x), L.ptr(v), L.ptr(g), x.numel(), L.ptr(c), float(tau), G, L.ptr(S),
                                            None, None, None, L.ptr(st), L.ptr(ws), ws.numel(), _s(x.device)))
        _raise_flags(st, "tdp_soft_filter_groupby")
        ctx.save_for_backward(x, v, g, c)
        ctx.tau, ctx.G = float(tau), G
        ctx.tau_shape = tau.shape if torch.is_tensor(tau) else None
        return S

    @staticmethod
    def backward(ctx, dS):
        x, v, g, c = ctx.saved_tensors
        lib = L.load()
        dv = torch.empty_like(v)
        dx = torch.empty_like(x) if ctx.needs_input_grad[0] else None
        dc = torch.empty(1, dtype=torch.float32, device=x.device)
        want_tau = ctx.tau_shape is not None and ctx.needs_input_grad[4]
        dtau = torch.empty(1, dtype=torch.float32, device=x.device) if want_tau else None
        ws = soft_workspace(x.device)
        dS = dS.contiguous()  # a copy must outlive the asynchronous call
        L.check("tdp_soft_filter_groupby_bwd",
                lib.tdp_soft_filter_groupby_bwd(L.ptr(x), L.ptr(v), L.ptr(g), x.numel(), L.ptr(c), ctx.tau, ctx.G,
                                                L.ptr(dS), L.ptr(dv), L.ptr(dx), L.ptr(dc), L.ptr(dtau),
                                                L.ptr(ws), ws.numel(), _s(x.device)))
        return dx, dv, None, dc.reshape(c.shape), (dtau.reshape(ctx.tau_shape) if want_tau else None), None


class MSELoss(torch.autograd.Function):
    """(1/G) sum (S - T)^2, the loss of the paper's training loop."""

    @staticmethod
    def forward(ctx, S, T):
        lib = L.load()
        loss = torch.empty(1, dtype=torch.float32, device=S.device)
        dS = torch.empty_like(S)
        L.check("tdp_mse_loss", lib.tdp_mse_loss(L.ptr(S), L.ptr(T), S.numel(), L.ptr(loss), L.ptr(dS), _s(S.device)))
        ctx.save_for_backward(dS)
        return loss[0]

    @staticmethod
    def backward(ctx, dL):
        (dS,) = ctx.saved_tensors
        return dS * dL, None


class SoftQueryStep:
    """One forward + backward of the soft query with preallocated buffers:
    S = soft group-by of soft-filtered v, L = MSE(S, T), then dv and dc."""

    def __init__(self, x, v, g, c, tau, G, T, want_dx=False):
        self.x, self.v, self.g, self.c, self.tau, self.G, self.T = x, v, g, c, float(tau), G, T
        dev = x.device
        f32 = dict(dtype=torch.float32, device=dev)
        self.S = torch.empty(G, **f32)
        self.dS = torch.empty(G, **f32)
        self.loss = torch.empty(1, **f32)
        self.dv = torch.empty_like(v)
        self.dx = torch.empty_like(x) if want_dx else None
        self.dc = torch.empty(1, **f32)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.ws = new_soft_workspace(dev)

    def forward(self, stream=None):
        lib = L.load()
        s = L.stream_handle(self.x.device) if stream is None else stream
        L.check("tdp_soft_filter_groupby",
                lib.tdp_soft_filter_groupby(L.ptr(self.x), L.ptr(self.v), L.ptr(self.g), self.x.numel(), L.ptr(self.c),
                                            self.tau, self.G, L.ptr(self.S), L.ptr(self.T), L.ptr(self.loss),
                                            L.ptr(self.dS), L.ptr(self.status), L.ptr(self.ws), self.ws.numel(), s))

    def backward(self, stream=None):
        lib = L.load()
        s = L.stream_handle(self.x.device) if stream is None else stream
        L.check("tdp_soft_filter_groupby_bwd",
                lib.tdp_soft_filter_groupby_bwd(L.ptr(self.x), L.ptr(self.v), L.ptr(self.g), self.x.numel(),
                                                L.ptr(self.c), self.tau, self.G, L.ptr(self.dS), L.ptr(self.dv),
                                                L.ptr(self.dx), L.ptr(self.dc), None, L.ptr(self.ws), self.ws.numel(), s))

    def __call__(self):
        self.forward()
        self.backward()
