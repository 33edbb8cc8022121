"""The allocation-free filter entry point against the workspace one, through
the C ABI: two calls in a row on one GPU (the second on a smaller input, so
stale tile states of the first would show), for each column dtype, with and
without a selection vector, and the host-side limit."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _run(fn, col, op, lit, sel=None):
    import torch

    from paper_2211_02753_amd import _lib as L
    lib = L.load()
    dev = col.device
    n_cand = col.numel() if sel is None else sel.numel()
    out = torch.full((max(n_cand, 1),), -7, dtype=torch.int32, device=dev)
    n_out = torch.full((1,), -1, dtype=torch.int64, device=dev)
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    c = L.col(col)
    args = [C.byref(c), L.CMP[op], int(lit), L.ptr(sel), n_cand if sel is not None else 0, L.ptr(out), out.numel(),
            L.ptr(n_out), L.ptr(st)]
    if fn == "tdp_filter_noalloc":
        rc = lib.tdp_filter_noalloc(*args, L.stream_handle(dev))
    else:
        ws = L.workspace(lib.tdp_filter_workspace_size(n_cand), dev)
        rc = lib.tdp_filter(*args, L.ptr(ws), ws.numel(), L.stream_handle(dev))
    L.check(fn, rc)
    torch.cuda.synchronize()
    m = int(n_out.item())
    assert int(st.item()) == 0
    return out[:m].cpu().numpy()


@pytest.mark.parametrize("dtype", ["int8", "int32", "int64"])
@pytest.mark.parametrize("with_sel", [False, True])
def test_noalloc_filter_matches_workspace_filter_twice(dtype, with_sel):
    import torch

    rng = np.random.default_rng(20240 + (3 if with_sel else 0) + len(dtype))
    lo, hi = (-100, 100) if dtype == "int8" else (-5000, 5000)
    # first call: several tiles and a ragged tail; second: smaller, ragged
    for n, lit in [(1_000_003, 17), (70_001, -40)]:
        host = rng.integers(lo, hi, size=n).astype(dtype)
        col = torch.from_numpy(host).cuda()
        sel = None
        if with_sel:
            sel_h = np.sort(rng.choice(n, size=n // 3, replace=False)).astype(np.int32)
            sel = torch.from_numpy(sel_h).cuda()
        got = _run("tdp_filter_noalloc", col, "<", lit, sel)
        want = _run("tdp_filter", col, "<", lit, sel)
        assert np.array_equal(got, want)
        cand = np.arange(n) if sel is None else sel.cpu().numpy()
        assert np.array_equal(got, cand[host[cand] < lit])


def test_noalloc_filter_empty_and_limit():
    import torch

    from paper_2211_02753_amd import _lib as L
    lib = L.load()
    empty = torch.empty(0, dtype=torch.int32, device="cuda")
    assert _run("tdp_filter_noalloc", empty, "<", 0).size == 0
    assert lib.tdp_filter_noalloc_max_candidates() == 2**31 - 1
    # more candidates than the static scratch covers: rejected on the host, before any launch
    c = L.Col(0x1000, L.I32, 0, 2**31)
    n_out = torch.zeros(1, dtype=torch.int64, device="cuda")
    rc = lib.tdp_filter_noalloc(C.byref(c), L.LT, 0, None, 0, C.c_void_p(0x2000), 2**31, L.ptr(n_out), None,
                                L.stream_handle("cuda"))
    assert rc == L.TDP_EINVAL
    assert b"exceed the limit" in lib.tdp_last_error()
