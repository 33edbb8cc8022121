"""One query description, run exact or relaxed by one flag.

Section 4 of the paper makes a query trainable by a flag at compilation: the
comparison steps of its WHERE clause and its grouped aggregate are relaxed
into differentiable operators (a logistic in place of each step, the
conjunction as a product, the grouped sum with + and * only), their
thresholds become parameters trained by gradient descent, and at inference
the exact operators come back.  ``TrainableQuery`` holds the description

    SELECT key0[, key1], SUM(value) | COUNT(*) FROM t
    WHERE col_1 op_1 c_1 AND ... AND col_J op_J c_J GROUP BY key0[, key1]

and ``compile(trainable=...)`` returns the relaxed plan (``tdp_soft_query``
and its backward, an autograd Function over the thresholds and
temperatures) or the exact plan (``tdp_groupby_agg`` with the thresholds
folded into literals).  Both run the same libtdp descriptor.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import torch

from . import _lib as L
from .query import GroupbyQuery, Key
from .soft import _need, _raise_flags, _s, soft_workspace

RELAXABLE = ("<", "<=", ">", ">=")


@dataclass
class Where:
    """One conjunct ``col op threshold``; the threshold is learnable when the
    query is compiled trainable."""
    col: torch.Tensor
    op: str
    threshold: float


def exact_literal(op: str, c: float, is_float: bool):
    """The literal of the exact comparison that agrees with ``x op c`` for
    every value of the column: for an integer column x < c and x >= c turn
    on ceil(c), x <= c and x > c on floor(c) (so a learned threshold of
    1277.3 on an integer day column is the literal 1278 of "<"); a float32
    column keeps c (compared in float32)."""
    if is_float:
        return float(c)
    if not math.isfinite(c):
        raise ValueError(f"threshold {c} is not finite")
    if op in ("<", ">="):
        return int(math.ceil(c))
    if op in ("<=", ">"):
        return int(math.floor(c))
    if float(c) != int(c):
        raise ValueError(f"'{op}' on an integer column needs an integral threshold, got {c}")
    return int(c)


class TrainableQuery:
    def __init__(self, n_rows: int, keys: list, where: list, value: torch.Tensor | None = None,
                 tau=1.0, device=None):
        if not 1 <= len(keys) <= 2:
            raise ValueError("one or two group keys")
        if len(where) > L.MAX_MORE_PREDS + 1:
            raise ValueError(f"at most {L.MAX_MORE_PREDS + 1} conjuncts")
        self.n_rows = int(n_rows)
        self.keys = list(keys)
        self.where = list(where)
        self.value = value
        self.device = keys[0].col.device if device is None else torch.device(device)
        J = len(self.where)
        taus = [float(tau)] * J if not isinstance(tau, (list, tuple)) else [float(t) for t in tau]
        if len(taus) != J:
            raise ValueError("one temperature per conjunct")
        f32 = dict(dtype=torch.float32, device=self.device)
        # learnable thresholds and (hyperparameter) temperatures, one per conjunct
        self.c = torch.tensor([float(w.threshold) for w in self.where], **f32)
        self.tau = torch.tensor(taus, **f32)
        self.G = 1
        for k in self.keys:
            self.G *= int(k.card)

    def compile(self, trainable: bool):
        """The relaxed plan (trainable=True) or the exact plan."""
        return SoftPlan(self) if trainable else ExactPlan(self)


def _desc(q: TrainableQuery):
    """The groupby descriptor of the relaxed plan (its thresholds come from
    the device tensor, so the literals are left 0)."""
    d = L.GroupbyDesc()
    keep = []
    d.n_rows = q.n_rows
    d.n_keys = len(q.keys)
    for i, k in enumerate(q.keys):
        d.key[i] = L.col(k.col)
        d.key_lo[i] = k.lo
        d.key_card[i] = k.card
    if q.value is not None:
        d.expr = L.EXPR_COL
        d.a = L.col(q.value)
    else:
        d.expr = L.EXPR_NONE
    if q.where:
        # the first conjunct takes the descriptor's own predicate slot, the
        # rest go to more_preds (the relaxed run accepts any column type there)
        first = q.where[0]
        d.has_pred = 1
        d.pred_cmp = L.CMP[first.op]
        d.pred = L.col(first.col)
        rest = q.where[1:]
        if rest:
            arr = (L.Pred * len(rest))()
            for i, w in enumerate(rest):
                arr[i] = L.Pred(L.col(w.col), L.CMP[w.op], 0, 0, 0.0)
            keep.append(arr)
            d.more_preds = C.cast(arr, C.POINTER(L.Pred))
            d.n_more_preds = len(rest)
    return d, keep


class _SoftQueryFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, tau, plan):
        lib = L.load()
        q = plan.q
        S = torch.empty(q.G, dtype=torch.float32, device=q.device)
        st = torch.zeros(1, dtype=torch.int32, device=q.device)
        _need(tau, torch.float32, "tau", (1,))
        taus = tau.detach()
        ws = soft_workspace(q.device)
        L.check("tdp_soft_query", lib.tdp_soft_query(C.byref(plan.desc), L.ptr(c), L.ptr(taus), L.ptr(S), None, None,
                                                     None, L.ptr(st), L.ptr(ws), ws.numel(), _s(q.device)))
        _raise_flags(st, "tdp_soft_query")
        ctx.plan = plan
        ctx.taus = taus
        ctx.save_for_backward(c)
        return S

    @staticmethod
    def backward(ctx, dS):
        lib = L.load()
        plan = ctx.plan
        q = plan.q
        (c,) = ctx.saved_tensors
        J = len(q.where)
        dc = torch.empty(max(J, 1), dtype=torch.float32, device=q.device)
        dtau = torch.empty(max(J, 1), dtype=torch.float32, device=q.device) if ctx.needs_input_grad[1] else None
        ws = soft_workspace(q.device)
        dS = dS.contiguous()  # a copy must outlive the asynchronous call
        L.check("tdp_soft_query_bwd", lib.tdp_soft_query_bwd(C.byref(plan.desc), L.ptr(c), L.ptr(ctx.taus),
                                                             L.ptr(dS), L.ptr(dc), L.ptr(dtau), None,
                                                             L.ptr(ws), ws.numel(), _s(q.device)))
        return dc[:J], (dtau[:J] if dtau is not None else None), None


class SoftPlan:
    """The relaxed plan: ``plan(c, tau)`` returns S[G] (float32, every group)
    differentiable in the thresholds c and the temperatures tau."""

    def __init__(self, q: TrainableQuery):
        for w in q.where:
            if w.op not in RELAXABLE:
                raise ValueError(f"'{w.op}' has no logistic relaxation")
        self.q = q
        self.desc, self._keep = _desc(q)

    def __call__(self, c: torch.Tensor | None = None, tau: torch.Tensor | None = None):
        c = self.q.c if c is None else c
        tau = self.q.tau if tau is None else tau
        _need(c.detach(), torch.float32, "c", (1,))
        return _SoftQueryFn.apply(c, tau, self)

    def step_buffers(self):
        f32 = dict(dtype=torch.float32, device=self.q.device)
        J = max(len(self.q.where), 1)
        self._S = torch.empty(self.q.G, **f32)
        self._dS = torch.empty(self.q.G, **f32)
        self._loss = torch.empty(1, **f32)
        self._dc = torch.empty(J, **f32)
        self._dtau = torch.empty(J, **f32)
        self._st = torch.zeros(1, dtype=torch.int32, device=self.q.device)

    def loss_and_grad(self, T: torch.Tensor, want_dtau: bool = False):
        """One training evaluation against target answers T[G] (float32): the
        forward with the mean squared error and its dS fused into the final
        reduction, then the backward.  Returns device tensors (loss[1],
        dc[J], dtau[J] or None); nothing is synchronised."""
        lib = L.load()
        q = self.q
        if not hasattr(self, "_S"):
            self.step_buffers()
        _need(T, torch.float32, "T", (1,))
        taus = L.ptr(q.tau)  # device temperatures: nothing here waits for the GPU
        ws = soft_workspace(q.device)
        s = _s(q.device)
        L.check("tdp_soft_query", lib.tdp_soft_query(C.byref(self.desc), L.ptr(q.c), taus, L.ptr(self._S), L.ptr(T),
                                                     L.ptr(self._loss), L.ptr(self._dS), L.ptr(self._st), L.ptr(ws),
                                                     ws.numel(), s))
        dtau = self._dtau if want_dtau else None
        L.check("tdp_soft_query_bwd", lib.tdp_soft_query_bwd(C.byref(self.desc), L.ptr(q.c), taus, L.ptr(self._dS),
                                                             L.ptr(self._dc), L.ptr(dtau), None, L.ptr(ws), ws.numel(),
                                                             s))
        return self._loss, self._dc, dtau

    def value_grad(self, dS: torch.Tensor, c: torch.Tensor | None = None) -> torch.Tensor:
        """dL/dvalue [n_rows] from dL/dS (the value column as a parameter)."""
        lib = L.load()
        q = self.q
        c = q.c if c is None else c
        J = len(q.where)
        taus = L.ptr(q.tau)
        dc = torch.empty(max(J, 1), dtype=torch.float32, device=q.device)
        de = torch.empty(q.n_rows, dtype=torch.float32, device=q.device)
        ws = soft_workspace(q.device)
        dS = dS.contiguous()  # a copy must outlive the asynchronous call
        L.check("tdp_soft_query_bwd", lib.tdp_soft_query_bwd(C.byref(self.desc), L.ptr(c.detach()), taus,
                                                             L.ptr(dS), L.ptr(dc), None, L.ptr(de),
                                                             L.ptr(ws), ws.numel(), _s(q.device)))
        return de


class ExactPlan:
    """The exact plan: the thresholds (read once, at compilation) become the
    literals of the exact comparisons, and ``plan()`` returns the exact
    groups (non-empty ones, in key order) of tdp_groupby_agg."""

    def __init__(self, q: TrainableQuery):
        self.q = q
        c = q.c.detach().cpu().tolist()
        self.literals = [exact_literal(w.op, c[i], w.col.dtype == torch.float32) for i, w in enumerate(q.where)]
        preds = [(w.col, w.op, self.literals[i]) for i, w in enumerate(q.where)]
        self.query = GroupbyQuery(q.n_rows, [Key(k.col, k.lo, k.card) for k in q.keys],
                                  expr=L.EXPR_COL if q.value is not None else L.EXPR_NONE,
                                  a=None if q.value is None else _operand(q.value), pred=preds or None)

    def __call__(self):
        return self.query()


def _operand(col):
    from .query import Operand
    if col.dtype == torch.float32:
        raise ValueError("the exact plan sums integer columns only (COUNT works on any table)")
    return Operand(col)
