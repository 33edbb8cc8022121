"""Exact relational operators over device columns: filter, hash join and
grouped SUM / COUNT / AVG (thin wrappers over libtdp)."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import torch

from . import _lib as L


def _status(device):
    return torch.zeros(1, dtype=torch.int32, device=device)


def check_flags(d_status: torch.Tensor, what: str):
    v = int(d_status.item())
    if v:
        names = [n for n, b in [("KEY_DOMAIN", L.FLAG_KEY_DOMAIN), ("DUP_BUILD", L.FLAG_DUP_BUILD),
                                ("GROUP_RANGE", L.FLAG_GROUP_RANGE), ("TABLE_FULL", L.FLAG_TABLE_FULL),
                                ("SPIN", L.FLAG_SPIN)] if v & b]
        raise L.TdpError(what, L.TDP_EINVAL, "device flags " + "|".join(names))


def filter(col: torch.Tensor, op: str, literal: int, sel: torch.Tensor | None = None) -> torch.Tensor:
    """Row ids (int32, ascending candidate order) with ``col[row] op literal``."""
    lib = L.load()
    dev = col.device
    n_cand = col.numel() if sel is None else sel.numel()
    out = torch.empty(max(n_cand, 1), dtype=torch.int32, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    st = _status(dev)
    ws = L.workspace(lib.tdp_filter_workspace_size(n_cand), dev)
    c = L.col(col)
    L.check("tdp_filter", lib.tdp_filter(C.byref(c), L.CMP[op], int(literal), L.ptr(sel), n_cand if sel is not None else 0,
                                         L.ptr(out), out.numel(), L.ptr(n_out), L.ptr(st), L.ptr(ws), ws.numel(),
                                         L.stream_handle(dev)))
    m = int(n_out.item())
    check_flags(st, "tdp_filter")
    return out[:m]


def hash_join(build_key: torch.Tensor, probe_key: torch.Tensor, probe_sel: torch.Tensor | None = None,
              count_only: bool = False, build_unique: bool = False, load_pct: int = 0, max_distinct: int = 0):
    """Inner equi-join pairs (probe_row, build_row) in unspecified order, or
    the pair count.  max_distinct (0 = build rows) bounds the distinct build
    keys and sizes the hash table."""
    lib = L.load()
    dev = probe_key.device
    d = L.JoinDesc(build_key.data_ptr(), build_key.numel(), probe_key.data_ptr(), probe_key.numel(),
                   None if probe_sel is None else probe_sel.data_ptr(), 0 if probe_sel is None else probe_sel.numel(),
                   int(build_unique), int(load_pct), int(max_distinct))
    ws = L.workspace(lib.tdp_hash_join_workspace_size(C.byref(d)), dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    st = _status(dev)
    s = L.stream_handle(dev)
    if count_only:
        L.check("tdp_hash_join", lib.tdp_hash_join(C.byref(d), L.JOIN_COUNT, None, None, 0, L.ptr(n_out), L.ptr(st),
                                                   L.ptr(ws), ws.numel(), s))
        total = int(n_out.item())
        check_flags(st, "tdp_hash_join")
        return total
    L.check("tdp_hash_join", lib.tdp_hash_join(C.byref(d), L.JOIN_COUNT, None, None, 0, L.ptr(n_out), L.ptr(st),
                                               L.ptr(ws), ws.numel(), s))
    total = int(n_out.item())
    check_flags(st, "tdp_hash_join")
    a = torch.empty(max(total, 1), dtype=torch.int32, device=dev)
    b = torch.empty(max(total, 1), dtype=torch.int32, device=dev)
    L.check("tdp_hash_join", lib.tdp_hash_join(C.byref(d), L.JOIN_PAIRS, L.ptr(a), L.ptr(b), total, L.ptr(n_out),
                                               L.ptr(st), L.ptr(ws), ws.numel(), s))
    got = int(n_out.item())
    check_flags(st, "tdp_hash_join")
    assert got == total
    return a[:total], b[:total]


@dataclass
class Key:
    col: torch.Tensor
    lo: int
    card: int
    side: int = L.PROBE


@dataclass
class Operand:
    col: torch.Tensor
    side: int = L.PROBE


@dataclass
class GroupbyQuery:
    """SELECT keys, SUM(e), COUNT(*), AVG(e) FROM probe [JOIN build] WHERE pred
    GROUP BY keys, prepared once (descriptor, workspace, outputs) so that
    ``launch()`` only enqueues kernels."""
    n_rows: int
    keys: list
    expr: int = L.EXPR_NONE
    a: Operand | None = None
    b: Operand | None = None
    k: int = 0
    pred: tuple | list | None = None   # (col, op, literal) or a list of them (a conjunction)
    sel: torch.Tensor | None = None
    join: tuple | None = None          # (build_key, probe_key, build_unique[, load_pct[, max_distinct]])
    topk: int = 0
    strategy: int = L.PROBE_AUTO
    _keep: list = field(default_factory=list, repr=False)

    def __post_init__(self):
        lib = L.load()
        d = L.GroupbyDesc()
        d.n_rows = self.n_rows
        dev = self.keys[0].col.device
        self.device = dev
        conj = [] if self.pred is None else (list(self.pred) if isinstance(self.pred, list) else [self.pred])
        first_int = next((i for i, p in enumerate(conj) if p[0].dtype != torch.float32), None)
        if first_int is not None:
            # an integer conjunct takes the descriptor's own predicate slot
            first = conj.pop(first_int)
            d.has_pred = 1
            d.pred_cmp = L.CMP[first[1]]
            d.pred_literal = int(first[2])
            d.pred = L.col(first[0])
        if len(conj) > L.MAX_MORE_PREDS:
            raise ValueError(f"at most {L.MAX_MORE_PREDS + 1} conjuncts")
        if conj:
            arr = (L.Pred * len(conj))()
            for i, (col, op, lit) in enumerate(conj):
                is_f = col.dtype == torch.float32
                arr[i] = L.Pred(L.col(col), L.CMP[op], 0, 0 if is_f else int(lit), float(lit) if is_f else 0.0)
            self._keep.append(arr)
            d.more_preds = C.cast(arr, C.POINTER(L.Pred))
            d.n_more_preds = len(conj)
        if self.sel is not None:
            d.sel = self.sel.data_ptr()
            d.n_sel = self.sel.numel()
        if self.join is not None:
            bk, pk = self.join[0], self.join[1]
            unique = self.join[2] if len(self.join) > 2 else False
            load_pct = self.join[3] if len(self.join) > 3 else 0
            max_distinct = self.join[4] if len(self.join) > 4 else 0
            jd = L.JoinDesc(bk.data_ptr(), bk.numel(), pk.data_ptr(), pk.numel(), None, 0, int(unique), int(load_pct),
                            int(max_distinct))
            self._keep.append(jd)
            d.join = C.pointer(jd)
        d.n_keys = len(self.keys)
        d.expr = self.expr
        for i, kk in enumerate(self.keys):
            d.key[i] = L.col(kk.col, kk.side)
            d.key_lo[i] = kk.lo
            d.key_card[i] = kk.card
        if self.a is not None:
            d.a = L.col(self.a.col, self.a.side)
        if self.b is not None:
            d.b = L.col(self.b.col, self.b.side)
        d.k = self.k
        d.topk = self.topk
        d.strategy = self.strategy
        self.desc = d
        G = 1
        for kk in self.keys:
            G *= kk.card
        self.cap = G
        ws_bytes = lib.tdp_groupby_workspace_size(C.byref(d))
        if ws_bytes == 0:
            L.check("tdp_groupby_workspace_size", lib.tdp_groupby_agg(C.byref(d), None, None, None, 0, None))
        self.ws = L.workspace(ws_bytes, dev)
        i64 = dict(dtype=torch.int64, device=dev)
        self.n_groups = torch.zeros(1, **i64)
        self.key0 = torch.empty(self.cap, **i64)
        self.key1 = torch.empty(self.cap, **i64)
        self.sum = torch.empty(self.cap, **i64)
        self.count = torch.empty(self.cap, **i64)
        self.avg = torch.empty(self.cap, dtype=torch.float64, device=dev)
        self.status = _status(dev)
        self.out = L.GroupbyOut(self.cap, self.n_groups.data_ptr(), self.key0.data_ptr(), self.key1.data_ptr(),
                                self.sum.data_ptr(), self.count.data_ptr(), self.avg.data_ptr())

    def launch(self, stream=None):
        lib = L.load()
        s = L.stream_handle(self.device) if stream is None else C.c_void_p(stream)
        L.check("tdp_groupby_agg", lib.tdp_groupby_agg(C.byref(self.desc), C.byref(self.out), L.ptr(self.status),
                                                       L.ptr(self.ws), self.ws.numel(), s))

    def launch_build(self, stream=None):
        lib = L.load()
        s = L.stream_handle(self.device) if stream is None else C.c_void_p(stream)
        L.check("tdp_groupby_build", lib.tdp_groupby_build(C.byref(self.desc), L.ptr(self.status), L.ptr(self.ws),
                                                           self.ws.numel(), s))

    def launch_probe(self, stream=None):
        lib = L.load()
        s = L.stream_handle(self.device) if stream is None else C.c_void_p(stream)
        L.check("tdp_groupby_probe", lib.tdp_groupby_probe(C.byref(self.desc), C.byref(self.out), L.ptr(self.status),
                                                           L.ptr(self.ws), self.ws.numel(), s))

    def result(self):
        m = int(self.n_groups.item())
        check_flags(self.status, "tdp_groupby_agg")
        r = {"k0": self.key0[:m], "sum": self.sum[:m], "count": self.count[:m], "avg": self.avg[:m]}
        if len(self.keys) > 1:
            r["k1"] = self.key1[:m]
        return r

    def __call__(self):
        self.launch()
        return self.result()


def groupby_agg(n_rows, keys, **kw):
    return GroupbyQuery(n_rows, keys, **kw)()
