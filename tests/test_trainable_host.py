"""Host logic of the exact/soft switch (no GPU): threshold -> literal folding
for the exact plan, and argument checks of tdp_soft_query that return before
any launch."""
import ctypes as C
import math

import numpy as np
import pytest
import torch

from paper_2211_02753_amd import _lib as L
from paper_2211_02753_amd.trainable import exact_literal


@pytest.mark.parametrize("op", ["<", "<=", ">", ">="])
@pytest.mark.parametrize("c", [1277.3, 1278.0, 1277.5, -3.2, -3.0, 0.0])
def test_exact_literal_agrees_with_the_real_comparison_on_integers(op, c):
    lit = exact_literal(op, c, is_float=False)
    assert isinstance(lit, int)
    xs = np.arange(math.floor(c) - 5, math.ceil(c) + 6)
    real = {"<": xs < c, "<=": xs <= c, ">": xs > c, ">=": xs >= c}[op]
    folded = {"<": xs < lit, "<=": xs <= lit, ">": xs > lit, ">=": xs >= lit}[op]
    assert np.array_equal(real, folded)


def test_exact_literal_float_column_and_errors():
    assert exact_literal("<", 0.25, is_float=True) == 0.25
    assert exact_literal("==", 4.0, is_float=False) == 4
    with pytest.raises(ValueError):
        exact_literal("==", 4.5, is_float=False)
    with pytest.raises(ValueError):
        exact_literal("<", float("inf"), is_float=False)


def _desc(n, col, cmp, more=None, expr=L.EXPR_NONE, a=None, join=None):
    d = L.GroupbyDesc()
    d.n_rows = n
    d.has_pred = 1
    d.pred_cmp = cmp
    d.pred = col
    d.n_keys = 1
    d.key[0] = L.Col(0x1000, L.I32, 0, n)
    d.key_lo[0] = 0
    d.key_card[0] = 10
    d.expr = expr
    if a is not None:
        d.a = a
    if more:
        arr = (L.Pred * len(more))(*more)
        d.more_preds = C.cast(arr, C.POINTER(L.Pred))
        d.n_more_preds = len(more)
        d._arr = arr
    if join is not None:
        d.join = C.pointer(join)
    return d


def test_soft_query_rejects_what_has_no_relaxation():
    lib = L.load()
    col = L.Col(0x2000, L.F32, 0, 100)
    tau = C.c_void_p(0x5000)  # device pointers: nothing below reaches a launch
    c = C.c_void_p(0x3000)
    S = C.c_void_p(0x4000)
    ws = C.c_void_p(0x10000)
    nbytes = lib.tdp_soft_workspace_size()
    call = lambda d: lib.tdp_soft_query(C.byref(d), c, tau, S, None, None, None, None, ws, nbytes, None)
    assert call(_desc(100, col, L.EQ)) == L.TDP_EUNSUPPORTED          # == has no logistic
    jd = L.JoinDesc(0x2000, 5, 0x3000, 10, None, 0, 1, 0, 0)
    assert call(_desc(100, col, L.LT, join=jd)) == L.TDP_EUNSUPPORTED  # no relaxed join here
    assert call(_desc(100, col, L.LT, expr=L.EXPR_MUL)) == L.TDP_EUNSUPPORTED
    # the temperatures are device data (their values are checked by the kernel); a missing array is an error
    assert lib.tdp_soft_query(C.byref(_desc(100, col, L.LT)), c, None, S, None, None, None, None, ws, nbytes,
                              None) == L.TDP_EINVAL
    more = [L.Pred(L.Col(0x2000, L.I32, 0, 100), L.GE, 0, 0, 0.0)] * 4    # 5 conjuncts in all
    assert call(_desc(100, col, L.LT, more=more)) == L.TDP_EINVAL
    short = L.Col(0x2000, L.F32, 0, 50)                                   # shorter than n_rows
    assert call(_desc(100, short, L.LT)) == L.TDP_EINVAL


def test_groupby_checks_more_preds_on_the_host():
    lib = L.load()
    col = L.Col(0x2000, L.I32, 0, 100)
    bad_cmp = [L.Pred(L.Col(0x2000, L.F32, 0, 100), 9, 0, 0, 0.0)]
    d = _desc(100, col, L.LT, more=bad_cmp, expr=L.EXPR_NONE)
    assert lib.tdp_groupby_workspace_size(C.byref(d)) == 0
    too_many = [L.Pred(L.Col(0x2000, L.F32, 0, 100), L.LT, 0, 0, 0.0)] * 4
    d = _desc(100, col, L.LT, more=too_many)
    assert lib.tdp_groupby_workspace_size(C.byref(d)) == 0
    build_side = [L.Pred(L.Col(0x2000, L.I32, 1, 100), L.LT, 0, 0, 0.0)]
    d = _desc(100, col, L.LT, more=build_side)
    assert lib.tdp_groupby_workspace_size(C.byref(d)) == 0
    ok = [L.Pred(L.Col(0x2000, L.F32, 0, 100), L.GE, 0, 0, 0.5)]
    d = _desc(100, col, L.LT, more=ok)
    assert lib.tdp_groupby_workspace_size(C.byref(d)) > 0
