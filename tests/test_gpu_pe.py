"""Soft COUNT grouped by two probability-encoded attributes (tdp_soft_pe_groupby
and its backward) against the float64 oracle: segments of the grid-of-images
shape, ragged and empty segments, rows outside every segment, an invalid
segment, the ungrouped form, every (K1, K2) edge, autograd, and sampled groups
of the 10M-row workload the benchmark times."""
import numpy as np
import pytest
import torch

import oracle
import tdp_datagen as gen

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = 1e-5  # normwise relative, float32 against the float64 oracle


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def say(*a):
    print(*a, flush=True)


def rel_err(got, want):
    got = got.detach().cpu().double().numpy() if torch.is_tensor(got) else got
    return float(np.abs(got - want).max() / max(np.abs(want).max(), 1e-30))


def _prob(rng, n, k):
    z = rng.standard_normal((n, k)) * 2.0
    e = np.exp(z - z.max(1, keepdims=True))
    return (e / e.sum(1, keepdims=True)).astype(np.float32)


def _run(seg, p, q, G, dS=None):
    from paper_2211_02753_amd import soft
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    ps, qs = dev(p), (None if q is None else dev(q))
    sg = None if seg is None else dev(seg)
    S = soft.soft_pe_groupby(ps, qs, sg, G, status=st)
    out = {"S": S, "status": int(st.item())}
    if dS is not None:
        dp, dq = soft.soft_pe_groupby_bwd(ps, qs, sg, dev(dS))
        torch.cuda.synchronize()
        out["dp"], out["dq"] = dp, dq
    return out


@pytest.mark.parametrize("K1,K2", [(10, 2), (1, 1), (16, 4), (4, 16), (7, 3), (3, 5)])
def test_pe_groupby_segments_against_oracle(K1, K2):
    rng = np.random.default_rng(100 + K1 * 17 + K2)
    lens = np.concatenate([[81] * 40, [0, 1, 2, 63, 64, 65, 5000, 0, 129]])
    rng.shuffle(lens)
    seg = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    n = int(seg[-1]) + 37  # a tail outside every segment
    G = len(lens)
    p, q = _prob(rng, n, K1), _prob(rng, n, K2)
    dS = rng.standard_normal((G, K1, K2)).astype(np.float32)
    say("pe segments", K1, K2, "G", G, "n", n)
    r = _run(seg, p, q, G, dS)
    want = oracle.soft_pe_groupby(seg, p, q, G)
    assert r["status"] == 0
    assert rel_err(r["S"], want) <= TOL
    # float32 sums over at most a tile's rows per lane, float64 beyond: every cell close to float32 rounding
    np.testing.assert_allclose(r["S"].cpu().double().numpy(), want, rtol=1e-6, atol=1e-6)
    wp, wq = oracle.soft_pe_groupby_bwd(seg, p, q, dS)
    m = int(seg[-1])
    assert rel_err(r["dp"][:m], wp[:m]) <= TOL
    assert rel_err(r["dq"][:m], wq[:m]) <= TOL


@pytest.mark.parametrize("n", [1, 63, 1000, 1_000_003])
@pytest.mark.parametrize("K1,K2,with_q", [(10, 2, True), (7, 1, False), (16, 4, True), (1, 1, True)])
def test_pe_groupby_ungrouped_against_oracle(n, K1, K2, with_q):
    rng = np.random.default_rng(n % 1000 + K1)
    p = _prob(rng, n, K1)
    q = _prob(rng, n, K2) if with_q else None
    dS = rng.standard_normal((1, K1, K2)).astype(np.float32)
    say("pe ungrouped", n, K1, K2, with_q)
    r = _run(None, p, q, 1, dS)
    want = oracle.soft_pe_groupby(None, p, q, 1)
    assert r["status"] == 0
    assert rel_err(r["S"], want) <= TOL
    wp, wq = oracle.soft_pe_groupby_bwd(None, p, q, dS)
    assert rel_err(r["dp"], wp) <= TOL
    if with_q:
        assert rel_err(r["dq"], wq) <= TOL
    else:
        assert r["dq"] is None


def test_pe_groupby_invalid_segment_flags_and_zeroes():
    rng = np.random.default_rng(7)
    n = 500
    p, q = _prob(rng, n, 10), _prob(rng, n, 2)
    seg = np.array([0, 100, 50, 300, n + 1], np.int64)  # segment 1 inverted, segment 3 past the end
    say("pe invalid segments")
    r = _run(seg, p, q, 4)
    from paper_2211_02753_amd import _lib as L
    assert r["status"] & L.FLAG_GROUP_RANGE
    S = r["S"].cpu().double().numpy()
    want = oracle.soft_pe_groupby(seg, p, q, 4)
    assert not S[1].any() and not S[3].any()
    np.testing.assert_allclose(S[[0, 2]], want[[0, 2]], rtol=1e-6, atol=1e-6)
    # the next call on the same workspace starts with clear flags
    r2 = _run(np.array([0, n], np.int64), p, q, 1)
    assert r2["status"] == 0


def test_pe_groupby_argument_errors():
    from paper_2211_02753_amd import _lib as L
    lib = L.load()
    from paper_2211_02753_amd import soft
    p = dev(np.ones((8, 10), np.float32))
    S = torch.empty(100, device=DEV)
    ws = soft.soft_workspace(DEV)
    s = L.stream_handle(DEV)
    call = lambda seg, G, K1, q, K2: lib.tdp_soft_pe_groupby(seg, G, L.ptr(p), K1, q, K2, 8, L.ptr(S), None,
                                                             L.ptr(ws), ws.numel(), s)
    assert call(None, 1, 10, L.ptr(p), 7) == L.TDP_EINVAL     # K1 * K2 > 64
    assert call(None, 1, 17, L.ptr(p), 1) == L.TDP_EINVAL     # K1 > 16
    assert call(None, 1, 10, None, 2) == L.TDP_EINVAL         # q == NULL needs K2 == 1
    assert call(None, 2, 10, L.ptr(p), 1) == L.TDP_EINVAL     # G != 1 without segments
    assert lib.tdp_soft_pe_groupby(None, 1, L.ptr(p), 10, None, 1, 8, L.ptr(S), None, L.ptr(ws), 16, s) == L.TDP_EWORKSPACE
    assert lib.tdp_soft_pe_groupby_bwd(None, 1, L.ptr(p), 10, None, 1, 8, L.ptr(S), L.ptr(S), L.ptr(S), s) == L.TDP_EINVAL


def test_pe_groupby_autograd_matches_oracle():
    from paper_2211_02753_amd import soft
    rng = np.random.default_rng(21)
    G, tiles = 50, 81
    seg = (np.arange(G + 1) * tiles).astype(np.int64)
    n = G * tiles
    p, q = _prob(rng, n, 10), _prob(rng, n, 2)
    T = rng.random((G, 10, 2)) * 8
    say("pe autograd")
    pt = dev(p).requires_grad_(True)
    qt = dev(q).requires_grad_(True)
    S = soft.SoftPEGroupBy.apply(pt, qt, dev(seg), G)
    loss = ((S.double() - dev(T)) ** 2).mean()
    gp, gq = torch.autograd.grad(loss, (pt, qt))
    Sw = oracle.soft_pe_groupby(seg, p, q, G)
    dS = 2.0 * (Sw - T) / Sw.size
    wp, wq = oracle.soft_pe_groupby_bwd(seg, p, q, dS)
    assert rel_err(S, Sw) <= TOL
    assert rel_err(gp, wp) <= TOL and rel_err(gq, wq) <= TOL


def test_pe_groupby_full_size_sampled():
    """The benchmark's workload: 123,457 grid images of 81 tiles (10M rows),
    10 digit and 2 size probabilities.  Sampled segments against the oracle
    (run on those rows alone), every segment's cell total against its tile
    count (rows are distributions), and the backward on sampled segments."""
    from paper_2211_02753_amd import soft
    c = gen.pe_grid_columns()
    seg, p, q = c["seg"], c["p"], c["q"]
    G = len(seg) - 1
    say("pe full size: G", G, "n", len(p))
    ps, qs, sg = dev(p), dev(q), dev(seg)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    S = soft.soft_pe_groupby(ps, qs, sg, G, status=st)
    rng = np.random.default_rng(5)
    dS = rng.standard_normal((G, 10, 2)).astype(np.float32)
    dp, dq = soft.soft_pe_groupby_bwd(ps, qs, sg, dev(dS))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    tot = S.double().sum((1, 2)).cpu().numpy()
    assert np.abs(tot - 81).max() <= 81 * 1e-5
    Sh, dph, dqh = S.cpu().double().numpy(), dp.cpu().double().numpy(), dq.cpu().double().numpy()
    for g in [0, 1, G // 2, G - 2, G - 1] + list(rng.integers(0, G, 20)):
        lo, hi = seg[g], seg[g + 1]
        local = np.array([0, hi - lo], np.int64)
        want = oracle.soft_pe_groupby(local, p[lo:hi], q[lo:hi], 1)[0]
        assert rel_err(Sh[g], want) <= TOL, g
        wp, wq = oracle.soft_pe_groupby_bwd(local, p[lo:hi], q[lo:hi], dS[g:g + 1])
        assert rel_err(dph[lo:hi], wp) <= TOL and rel_err(dqh[lo:hi], wq) <= TOL, g
