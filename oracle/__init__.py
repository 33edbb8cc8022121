"""CPU oracle (test infrastructure only).

Plain, single-threaded C++ statement of every operator on the hot path, loaded
through ctypes.  Only the test suite, the smoke check and the benchmark's CPU
baseline use it; the GPU library neither imports nor links it, and it shares
no code with the GPU library.

Paper: "The Tensor Data Platform: Towards an AI-centric Database System"
(arXiv 2211.02753).  Each wrapper names the passage it follows; the C++ file
holds the arithmetic.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

I8, I32, I64, F32 = 1, 2, 3, 4
LT, LE, GT, GE, EQ, NE = range(6)
EXPR_COL, EXPR_MUL, EXPR_MUL_CONST_SUB, EXPR_NONE = range(4)
_DT = {np.dtype(np.int8): I8, np.dtype(np.int32): I32, np.dtype(np.int64): I64, np.dtype(np.float32): F32}
_CMP = {"<": LT, "<=": LE, ">": GT, ">=": GE, "==": EQ, "!=": NE}


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (plain -O2, no parallelism)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


def _declare(L):
    p, i64, i32, d = C.c_void_p, C.c_int64, C.c_int, C.c_double
    sig = {
        "orc_filter": (i64, [p, i32, i64, i32, i64, p, i64, p]),
        "orc_join_pairs": (i64, [p, i64, p, i64, p, i64, i64, p, p]),
        "orc_filter_f32": (i64, [p, i64, i32, d, p, i64, p]),
        "orc_soft_where": (None, [p, p, p, p, i32, p, p, i64, i64, p]),
        "orc_soft_where_bwd": (None, [p, p, p, p, i32, p, p, i64, p, p, p, p]),
        "orc_llp_forward": (None, [p, i64, i32, p, p, i32, i64, p]),
        "orc_llp_backward": (None, [p, i64, i32, p, p, i32, i64, p, p, p]),
        "orc_llp_predict": (None, [p, i64, i32, p, p, i32, p]),
        "orc_query": (i64, [i64, p, i64, p, i32, i32, i64, p, p, i64, i32, p, i32, i32, p, i32, i32,
                            i32, p, i32, i32, p, i32, i32, i64, i64, p, p, p, p, p, p]),
        "orc_mn_group": (None, [i64, p, p, p, i64, p, p, i64, p, p]),
        "orc_topk": (i64, [p, p, i64, i64, p]),
        "orc_soft_filter": (None, [p, i64, d, d, p]),
        "orc_soft_filter_bwd": (None, [p, i64, d, d, p, p, p, p]),
        "orc_soft_groupby": (None, [p, p, p, i64, i32, i32, p]),
        "orc_soft_groupby_bwd": (None, [p, p, p, p, i64, i32, p, p]),
        "orc_soft_pe_groupby": (None, [p, i32, p, i32, p, i32, i64, p]),
        "orc_soft_pe_groupby_bwd": (None, [p, i32, p, i32, p, i32, i64, p, p, p]),
        "orc_mse": (d, [p, p, i64, p]),
        "orc_bf16_round": (None, [p, p, i64]),
        "orc_conv3x3_fwd": (None, [p, p, p, i32, i32, i32, i32, i32, i32, p]),
        "orc_conv3x3_dgrad": (None, [p, p, i32, i32, i32, i32, i32, p]),
        "orc_conv3x3_wgrad": (None, [p, p, i32, i32, i32, i32, i32, p, p]),
        "orc_maxpool2_fwd": (None, [p, i32, i32, i32, i32, p]),
        "orc_maxpool2_bwd": (None, [p, p, i32, i32, i32, i32, p]),
        "orc_linear_fwd": (None, [p, p, p, i32, i32, i32, i32, p]),
        "orc_linear_bwd": (None, [p, p, p, i32, i32, i32, p, p, p]),
        "orc_softmax_expect": (None, [p, i32, i32, p, p]),
        "orc_softmax_expect_bwd": (None, [p, p, i32, i32, p]),
        "orc_softmax_bwd": (None, [p, p, i32, i32, p]),
        "orc_argmax": (None, [p, i32, i32, p]),
        "orc_adam": (None, [p, p, p, p, i64, d, d, d, d, i32, p, p, p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------------------
# Exact operators
# ---------------------------------------------------------------------------

def filter(col, op, lit, sel=None):
    """Ascending row ids with ``col[row] op lit`` (SQL WHERE; Section 2)."""
    col = np.ascontiguousarray(col)
    n_cand = len(col) if sel is None else len(sel)
    out = np.empty(max(n_cand, 1), dtype=np.int32)
    sel_c = None if sel is None else _c(sel, np.int32)
    m = lib().orc_filter(_p(col), _DT[col.dtype], len(col), _CMP[op], int(lit), _p(sel_c),
                         0 if sel is None else len(sel), _p(out))
    return out[:m].copy()


def filter_f32(col, op, lit, sel=None):
    """Ascending row ids with ``col[row] op lit`` on a float32 column, the
    literal rounded to float32 (SQL WHERE; Section 2)."""
    col = _c(col, np.float32)
    n_cand = len(col) if sel is None else len(sel)
    out = np.empty(max(n_cand, 1), dtype=np.int32)
    sel_c = None if sel is None else _c(sel, np.int32)
    m = lib().orc_filter_f32(_p(col), len(col), _CMP[op], float(lit), _p(sel_c), 0 if sel is None else len(sel),
                             _p(out))
    return out[:m].copy()


def where(n_rows, preds):
    """Rows satisfying every conjunct (col, op, lit) of a WHERE clause, as
    successive filters each over the survivors of the ones before it."""
    sel = None
    for col, op, lit in preds:
        col = np.ascontiguousarray(col)
        sel = filter_f32(col, op, lit, sel) if col.dtype == np.float32 else filter(col, op, lit, sel)
    return np.arange(n_rows, dtype=np.int32) if sel is None else sel


def join_pairs(build_key, probe_key, probe_sel=None):
    """All (probe_row, build_row) pairs of the inner equi-join, in probe order
    then ascending build row."""
    bk, pk = _c(build_key, np.int32), _c(probe_key, np.int32)
    ps = None if probe_sel is None else _c(probe_sel, np.int32)
    nps = 0 if ps is None else len(ps)
    L = lib()
    total = L.orc_join_pairs(_p(bk), len(bk), _p(pk), len(pk), _p(ps), nps, 0, None, None)
    a = np.empty(max(total, 1), np.int32)
    b = np.empty(max(total, 1), np.int32)
    L.orc_join_pairs(_p(bk), len(bk), _p(pk), len(pk), _p(ps), nps, total, _p(a), _p(b))
    return a[:total].copy(), b[:total].copy()


def query(n_fact, keys, expr=EXPR_NONE, a=None, b=None, K=0, pred=None, join=None):
    """Filter -> join -> group-by with SUM/COUNT/AVG (Section 2; Section 3's
    grouped COUNT; Section 5.2's AVG).

    pred = (col, op, lit), a list of such conjuncts, or None (a list runs as
    successive filters, the last inside the query); join = (fact_fk, dim_pk) or None;
    keys = [(col, side), ...] (1 or 2, side 0 fact / 1 dim);
    a, b = (col, side) operands of the value expression.
    Returns a dict of numpy arrays (k0, k1, sum, count, avg, wrapped)."""
    hold = []

    def arr(x):
        if x is None:
            return None, 0
        x = np.ascontiguousarray(x)
        hold.append(x)
        return x, _DT[x.dtype]

    pc, pdt, pcmp, plit = None, 0, 0, 0
    sel = None
    if isinstance(pred, list):
        if pred and np.asarray(pred[-1][0]).dtype != np.float32:
            sel = where(n_fact, pred[:-1]) if len(pred) > 1 else None
            pred = pred[-1]
        else:
            sel = where(n_fact, pred) if pred else None
            pred = None
        if sel is not None:
            sel = _c(sel, np.int32)
            hold.append(sel)
    if pred is not None:
        pc, pdt = arr(pred[0])
        pcmp, plit = _CMP[pred[1]], int(pred[2])
    fk = pkk = None
    n_dim = 0
    if join is not None:
        fk, _ = arr(_c(join[0], np.int32))
        pkk, _ = arr(_c(join[1], np.int32))
        n_dim = len(pkk)
    k0, k0d = arr(keys[0][0])
    k0s = keys[0][1]
    k1, k1d, k1s = None, 0, 0
    if len(keys) > 1:
        k1, k1d = arr(keys[1][0])
        k1s = keys[1][1]
    ac, ad, asd = None, 0, 0
    bc, bd, bsd = None, 0, 0
    if a is not None:
        ac, ad = arr(a[0])
        asd = a[1]
    if b is not None:
        bc, bd = arr(b[0])
        bsd = b[1]
    L = lib()
    args = [n_fact, _p(sel), 0 if sel is None else len(sel), _p(pc), pdt, pcmp, plit, _p(fk), _p(pkk), n_dim, len(keys), _p(k0), k0d, k0s,
            _p(k1), k1d, k1s, expr, _p(ac), ad, asd, _p(bc), bd, bsd, int(K)]
    m = L.orc_query(*args, 0, None, None, None, None, None, None)
    out = {k: np.empty(max(m, 1), dt) for k, dt in
           [("k0", np.int64), ("k1", np.int64), ("sum", np.int64), ("count", np.int64),
            ("avg", np.float64), ("wrapped", np.int32)]}
    L.orc_query(*args, m, _p(out["k0"]), _p(out["k1"]), _p(out["sum"]), _p(out["count"]),
                _p(out["avg"]), _p(out["wrapped"]))
    res = {k: v[:m].copy() for k, v in out.items()}
    if len(keys) < 2:
        del res["k1"]
    return res


class MNGroupOracle:
    """Per-group enumeration of the many-to-many join aggregate
    SUM(l.payload * r.payload), COUNT(*) ... GROUP BY l.gkey."""

    def __init__(self, lkey, lgkey, lpay, rkey, rpay):
        # left rows ordered by group so that one group's rows are one slice
        lo = np.argsort(np.asarray(lgkey), kind="stable")
        self.l = [_c(np.asarray(lkey)[lo], np.int32), _c(np.asarray(lgkey)[lo], np.int32),
                  _c(np.asarray(lpay)[lo], np.int64)]
        order = np.argsort(rkey, kind="stable")
        self.r = [_c(np.asarray(rkey)[order], np.int32), _c(np.asarray(rpay)[order], np.int64)]

    def group(self, g):
        g32 = np.int32(g)  # a Python int would make searchsorted convert the whole column
        a = int(np.searchsorted(self.l[1], g32, side="left"))
        b = int(np.searchsorted(self.l[1], g32, side="right"))
        s, c = C.c_int64(), C.c_int64()
        k, gk, pay = (x[a:b] for x in self.l)
        lib().orc_mn_group(int(g), _p(k), _p(gk), _p(pay), b - a, _p(self.r[0]), _p(self.r[1]), len(self.r[0]),
                           C.byref(s), C.byref(c))
        return s.value, c.value


def topk(keys, sums, k):
    keys, sums = _c(keys, np.int64), _c(sums, np.int64)
    out = np.empty(max(min(k, len(keys)), 1), np.int64)
    m = lib().orc_topk(_p(keys), _p(sums), len(keys), k, _p(out))
    return out[:m].copy()


# ---------------------------------------------------------------------------
# Relaxed operators (Section 4)
# ---------------------------------------------------------------------------

def soft_filter(x, c, tau):
    x = _c(x, np.float32)
    w = np.empty(len(x), np.float64)
    lib().orc_soft_filter(_p(x), len(x), float(c), float(tau), _p(w))
    return w


def soft_filter_bwd(x, c, tau, dw, want_dx=True):
    x, dw = _c(x, np.float32), _c(dw, np.float64)
    dx = np.empty(len(x), np.float64) if want_dx else None
    dc = C.c_double()
    lib().orc_soft_filter_bwd(_p(x), len(x), float(c), float(tau), _p(dw), _p(dx), C.byref(dc), None)
    return dx, dc.value


def soft_filter_bwd_tau(x, c, tau, dw):
    """dL/dtau of the soft filter from dL/dw (the temperature as a parameter)."""
    x, dw = _c(x, np.float32), _c(dw, np.float64)
    dc, dtau = C.c_double(), C.c_double()
    lib().orc_soft_filter_bwd(_p(x), len(x), float(c), float(tau), _p(dw), None, C.byref(dc), C.byref(dtau))
    return dtau.value


_SIGN = {"<": 1, "<=": 1, ">": -1, ">=": -1}


def _soft_where_args(xs, ops, c, tau, v, gid):
    J = len(xs)
    n = len(gid)
    x = np.empty((J, n), np.float64)
    for j, col in enumerate(xs):
        x[j] = np.asarray(col).astype(np.float64)   # the float32 (or integer) column value, exactly
    s = _c([_SIGN[o] for o in ops], np.int32)
    c = _c(c, np.float64)
    tau = _c(tau, np.float64)
    v = None if v is None else _c(np.asarray(v).astype(np.float64), np.float64)
    return x, s, c, tau, v, _c(gid, np.int64), J, n


def soft_where(xs, ops, c, tau, v, gid, G):
    """Relaxed WHERE x_1 op_1 c_1 AND ... GROUP BY gid with SUM(v) (COUNT
    when v is None): S[g] = sum_i prod_j sigma(s_j (c_j - x_ij) / tau_j) v_i
    (Section 4).  xs: J columns; ops in <, <=, >, >=; c, tau: J values."""
    x, s, c, tau, v, gid, J, n = _soft_where_args(xs, ops, c, tau, v, gid)
    S = np.empty(G, np.float64)
    lib().orc_soft_where(_p(x), _p(s), _p(c), _p(tau), J, _p(v), _p(gid), n, G, _p(S))
    return S


def soft_where_bwd(xs, ops, c, tau, v, gid, dS):
    """Gradients of soft_where from dS: (dc[J], dtau[J], dv[n])."""
    x, s, c, tau, v, gid, J, n = _soft_where_args(xs, ops, c, tau, v, gid)
    dS = _c(dS, np.float64)
    dc = np.empty(J, np.float64)
    dtau = np.empty(J, np.float64)
    dv = np.empty(n, np.float64)
    lib().orc_soft_where_bwd(_p(x), _p(s), _p(c), _p(tau), J, _p(v), _p(gid), n, _p(dS), _p(dc), _p(dtau), _p(dv))
    return dc, dtau, dv


def group_ids(keys):
    """Dense group id of each row from 1 or 2 key columns with declared
    domains: keys = [(col, lo, card), ...]; gid = (k0 - lo0) * card1 + (k1 - lo1).
    Rows outside a domain get -1."""
    k0, lo0, c0 = keys[0]
    u0 = np.asarray(k0).astype(np.int64) - lo0
    ok = (u0 >= 0) & (u0 < c0)
    gid = u0
    if len(keys) > 1:
        k1, lo1, c1 = keys[1]
        u1 = np.asarray(k1).astype(np.int64) - lo1
        ok &= (u1 >= 0) & (u1 < c1)
        gid = u0 * c1 + u1
    return np.where(ok, gid, -1)


def soft_groupby(g, w, v, G):
    g = _c(g, np.int32)
    v = _c(v, np.float64)
    K = 1 if v.ndim == 1 else v.shape[1]
    w = None if w is None else _c(w, np.float64)
    S = np.empty((G, K), np.float64)
    lib().orc_soft_groupby(_p(g), _p(w), _p(v), len(g), K, G, _p(S))
    return S[:, 0].copy() if v.ndim == 1 else S


def soft_groupby_bwd(g, w, v, dS):
    g = _c(g, np.int32)
    v = _c(v, np.float64)
    K = 1 if v.ndim == 1 else v.shape[1]
    w = None if w is None else _c(w, np.float64)
    dS = _c(dS, np.float64)
    dw = np.empty(len(g), np.float64)
    dv = np.empty(v.shape, np.float64)
    lib().orc_soft_groupby_bwd(_p(g), _p(w), _p(v), _p(dS), len(g), K, _p(dw), _p(dv))
    return dw, dv


def soft_pe_groupby(seg, p, q, G):
    """S[g][a][b] = sum over segment g's rows of p[i][a] q[i][b] (q None: q = 1,
    K2 = 1); seg None is one segment of all rows.  Returns [G][K1][K2]."""
    p = _c(p, np.float64)
    n, K1 = p.shape
    q = None if q is None else _c(q, np.float64)
    K2 = 1 if q is None else q.shape[1]
    seg = None if seg is None else _c(seg, np.int64)
    S = np.empty((G, K1, K2), np.float64)
    lib().orc_soft_pe_groupby(_p(seg), G, _p(p), K1, _p(q), K2, n, _p(S))
    return S


def soft_pe_groupby_bwd(seg, p, q, dS):
    """dp[i][a] = sum_b dS[g_i][a][b] q[i][b], dq[i][b] = sum_a dS[g_i][a][b] p[i][a]
    (dq None when q is None)."""
    p = _c(p, np.float64)
    n, K1 = p.shape
    q = None if q is None else _c(q, np.float64)
    K2 = 1 if q is None else q.shape[1]
    dS = _c(dS, np.float64)
    G = dS.shape[0]
    seg = None if seg is None else _c(seg, np.int64)
    dp = np.empty((n, K1), np.float64)
    dq = None if q is None else np.empty((n, K2), np.float64)
    lib().orc_soft_pe_groupby_bwd(_p(seg), G, _p(p), K1, _p(q), K2, n, _p(dS), _p(dp), _p(dq))
    return dp, dq


def mse(S, T):
    S, T = _c(S, np.float64), _c(T, np.float64)
    dS = np.empty(len(S), np.float64)
    L = lib().orc_mse(_p(S), _p(T), len(S), _p(dS))
    return L, dS


def soft_query(x, v, g, c, tau, G, T):
    """Soft filter then soft group-by SUM(v), MSE against T, and the
    gradients with respect to c, tau and v, all in float64."""
    w = soft_filter(x, c, tau)
    S = soft_groupby(g, w, v, G)
    L, dS = mse(S, T)
    dw, dv = soft_groupby_bwd(g, w, v, dS)
    _, dc = soft_filter_bwd(x, c, tau, dw, want_dx=False)
    dtau = soft_filter_bwd_tau(x, c, tau, dw)
    return {"w": w, "S": S, "loss": L, "dS": dS, "dv": dv, "dc": dc, "dtau": dtau}


# ---------------------------------------------------------------------------
# Classifier layers
# ---------------------------------------------------------------------------

def bf16_round(a):
    a = _c(a, np.float32)
    out = np.empty_like(a)
    lib().orc_bf16_round(_p(a), _p(out), a.size)
    return out


def conv3x3_fwd(x, w, bias, relu):
    x, w = _c(x, np.float32), _c(w, np.float32)
    bias = None if bias is None else _c(bias, np.float32)
    B, H, W, Cin = x.shape
    Cout = w.shape[0]
    y = np.empty((B, H - 2, W - 2, Cout), np.float64)
    lib().orc_conv3x3_fwd(_p(x), _p(w), _p(bias), B, H, W, Cin, Cout, int(relu), _p(y))
    return y


def conv3x3_dgrad(dy, w, H, W):
    dy, w = _c(dy, np.float32), _c(w, np.float32)
    B, Cout, Cin = dy.shape[0], w.shape[0], w.shape[3]
    dx = np.empty((B, H, W, Cin), np.float64)
    lib().orc_conv3x3_dgrad(_p(dy), _p(w), B, H, W, Cin, Cout, _p(dx))
    return dx


def conv3x3_wgrad(x, dy):
    x, dy = _c(x, np.float32), _c(dy, np.float32)
    B, H, W, Cin = x.shape
    Cout = dy.shape[3]
    dw = np.empty((Cout, 3, 3, Cin), np.float64)
    db = np.empty(Cout, np.float64)
    lib().orc_conv3x3_wgrad(_p(x), _p(dy), B, H, W, Cin, Cout, _p(dw), _p(db))
    return dw, db


def maxpool2_fwd(x):
    x = _c(x, np.float32)
    B, H, W, Cc = x.shape
    y = np.empty((B, H // 2, W // 2, Cc), np.float64)
    lib().orc_maxpool2_fwd(_p(x), B, H, W, Cc, _p(y))
    return y


def maxpool2_bwd(x, dy):
    x, dy = _c(x, np.float32), _c(dy, np.float32)
    B, H, W, Cc = x.shape
    dx = np.empty(x.shape, np.float64)
    lib().orc_maxpool2_bwd(_p(x), _p(dy), B, H, W, Cc, _p(dx))
    return dx


def linear_fwd(x, w, bias, relu):
    x, w = _c(x, np.float32), _c(w, np.float32)
    bias = None if bias is None else _c(bias, np.float32)
    M, K = x.shape
    N = w.shape[0]
    y = np.empty((M, N), np.float64)
    lib().orc_linear_fwd(_p(x), _p(w), _p(bias), M, N, K, int(relu), _p(y))
    return y


def linear_bwd(x, w, dy):
    x, w, dy = _c(x, np.float32), _c(w, np.float32), _c(dy, np.float32)
    M, K = x.shape
    N = w.shape[0]
    dx = np.empty((M, K), np.float64)
    dw = np.empty((N, K), np.float64)
    db = np.empty(N, np.float64)
    lib().orc_linear_bwd(_p(x), _p(w), _p(dy), M, N, K, _p(dx), _p(dw), _p(db))
    return dx, dw, db


def softmax_expect(logits):
    z = _c(logits, np.float32)
    M, K = z.shape
    p = np.empty((M, K), np.float64)
    e = np.empty(M, np.float64)
    lib().orc_softmax_expect(_p(z), M, K, _p(p), _p(e))
    return p, e


def softmax_expect_bwd(p, dE):
    p, dE = _c(p, np.float64), _c(dE, np.float64)
    M, K = p.shape
    dz = np.empty((M, K), np.float64)
    lib().orc_softmax_expect_bwd(_p(p), _p(dE), M, K, _p(dz))
    return dz


def softmax_bwd(p, dP):
    p, dP = _c(p, np.float64), _c(dP, np.float64)
    M, K = p.shape
    dz = np.empty((M, K), np.float64)
    lib().orc_softmax_bwd(_p(p), _p(dP), M, K, _p(dz))
    return dz


def argmax(p):
    p = _c(p, np.float32)
    M, K = p.shape
    out = np.empty(M, np.int8)
    lib().orc_argmax(_p(p), M, K, _p(out))
    return out


def adam(p, g, m, v, lr, b1, b2, eps, step):
    p, g, m, v = (_c(a, np.float32) for a in (p, g, m, v))
    po, mo, vo = (np.empty(p.shape, np.float64) for _ in range(3))
    lib().orc_adam(_p(p), _p(g), _p(m), _p(v), p.size, lr, b1, b2, eps, int(step), _p(po), _p(mo), _p(vo))
    return po, mo, vo


# ---------------------------------------------------------------------------
# Learning from label proportions (Section 5.3) and its Label-DP form (5.4)
# ---------------------------------------------------------------------------

def llp_forward(X, W, b, bag):
    """Soft COUNT per (bag, class) of a linear classifier's softmax over
    consecutive bags of `bag` rows: S[j][c] = sum_{i in bag j} p_i[c]."""
    X = _c(X, np.float32)
    n, F = X.shape
    W = _c(W, np.float64)
    C = W.shape[0]
    b = _c(b, np.float64)
    S = np.empty(((n + bag - 1) // bag, C), np.float64)
    lib().orc_llp_forward(_p(X), n, F, _p(W), _p(b), C, int(bag), _p(S))
    return S


def llp_backward(X, W, b, bag, dS):
    """(dW, db) of llp_forward from dS[n_bags][C]."""
    X = _c(X, np.float32)
    n, F = X.shape
    W = _c(W, np.float64)
    C = W.shape[0]
    b = _c(b, np.float64)
    dS = _c(dS, np.float64)
    dW = np.empty((C, F), np.float64)
    db = np.empty(C, np.float64)
    lib().orc_llp_backward(_p(X), n, F, _p(W), _p(b), C, int(bag), _p(dS), _p(dW), _p(db))
    return dW, db


def llp_predict(X, W, b):
    """Argmax labels of the linear classifier (ties to the smallest class)."""
    X = _c(X, np.float32)
    n, F = X.shape
    W = _c(W, np.float64)
    out = np.empty(n, np.int8)
    lib().orc_llp_predict(_p(X), n, F, _p(W), _p(_c(b, np.float64)), W.shape[0], _p(out))
    return out


def noisy_counts(counts, noise):
    """The Laplace mechanism's released counts: each count plus its noise
    draw, in float32 (the precision the training targets are kept in)."""
    return (np.asarray(counts).astype(np.float32) + np.asarray(noise, np.float32)).astype(np.float32)


def cnn_forward(images, params):
    """Class probabilities of the image classifier (Sections 3 and 5.5), the
    oracle's layers composed in order: pixels / 255, conv3x3 + ReLU (32),
    conv3x3 + ReLU (64), 2x2 max pool, fully connected + ReLU (128), fully
    connected (10), softmax.  Operands are passed on as float32."""
    x = (np.asarray(images, np.float32) / np.float32(255.0))[..., None]
    h = conv3x3_fwd(x, params["conv1_w"], params["conv1_b"], True).astype(np.float32)
    h = conv3x3_fwd(h, params["conv2_w"], params["conv2_b"], True).astype(np.float32)
    h = maxpool2_fwd(h).astype(np.float32)
    h = linear_fwd(h.reshape(h.shape[0], -1), params["fc1_w"], params["fc1_b"], True).astype(np.float32)
    z = linear_fwd(h, params["fc2_w"], params["fc2_b"], False).astype(np.float32)
    return softmax_expect(z)[0]


# ---------------------------------------------------------------------------
# Order-preserving dictionary encoding of string columns (Section 2, storage
# and encodings): the dictionary is the sorted list of distinct strings (one
# string per row of a 2-d byte tensor) and a string's code is its position.
# ---------------------------------------------------------------------------

def _strings(rows):
    """Byte strings of a zero-padded [n][L] uint8 matrix (padding removed)."""
    rows = np.asarray(rows, np.uint8)
    return [bytes(r).rstrip(b"\0") for r in rows]


def dict_build(rows):
    """(dictionary [d][L] uint8, codes int32 [n]): the sorted distinct strings
    and each row's position among them, by Python's own byte-string order."""
    rows = np.asarray(rows, np.uint8)
    L = rows.shape[1]
    strs = _strings(rows)
    uniq = sorted(set(strs))
    pos = {s: i for i, s in enumerate(uniq)}
    d = np.zeros((len(uniq), L), np.uint8)
    for i, s in enumerate(uniq):
        d[i, :len(s)] = np.frombuffer(s, np.uint8)
    return d, np.array([pos[s] for s in strs], np.int32)


def dict_lookup(dictionary, rows):
    """(lower bound int32, found int8) of each string in the sorted
    dictionary: the number of entries below it, and whether it is one."""
    keys = _strings(dictionary)
    out, found = [], []
    for s in _strings(rows):
        lo = sum(1 for k in keys if k < s)
        out.append(lo)
        found.append(1 if lo < len(keys) and keys[lo] == s else 0)
    return np.array(out, np.int32), np.array(found, np.int8)
