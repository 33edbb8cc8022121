"""Parity of the relaxed operators (soft filter, soft group-by, their fused
pair, MSE and the backward kernels) with the float64 oracle.

Tolerances (float32 kernels against float64): normwise relative 1e-5 for S,
dS, dv and w (max-norm of the error over max-norm of the reference); for the
mixed-sign scalar dc, |dc_gpu - dc_ref| <= 1e-5 * sum_i |t_i| where t_i are
its terms.  Quantities computed from S (loss, dS and through dS the
gradients) also admit the error S propagates into them, which matters only
when they are near zero (S close to its target)."""
import numpy as np
import pytest
import torch

import oracle
import tdp_datagen as gen

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-5


def S():
    from paper_2211_02753_amd import soft
    return soft


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def normwise(got, ref):
    ref = np.asarray(ref, np.float64)
    return float(np.max(np.abs(np.asarray(got, np.float64) - ref)) / max(np.max(np.abs(ref)), 1e-300))


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("n", [1, 5, 4099, 1_000_003])
@pytest.mark.parametrize("tau", [1.0, 0.1])
def test_soft_filter_and_bwd(n, tau):
    c = gen.soft_query_columns(n=n, n_groups=10)
    x = c["x"]
    cc = dev(np.array([0.3], np.float32))
    say("soft filter", n, tau)
    w = S().soft_filter(dev(x), cc, tau)
    ref = oracle.soft_filter(x, 0.3, tau)
    assert normwise(host(w), ref) <= TOL
    dw = gen.float_uniform(gen.stream_seed(99, n), n, -1, 1)
    dx, dc = S().soft_filter_bwd(dev(x), cc, tau, dev(dw))
    rdx, rdc = oracle.soft_filter_bwd(x, 0.3, tau, dw.astype(np.float64))
    assert normwise(host(dx), rdx) <= TOL
    assert abs(float(host(dc)[0]) - rdc) <= TOL * float(np.sum(np.abs(rdx)))


@pytest.mark.parametrize("K,G,n,weights", [(1, 1000, 1_000_003, True), (10, 30, 50_001, False), (10, 7, 3, True),
                                           (16, 4096, 200_000, True), (1, 30_000, 120_000, False)])
def test_soft_groupby_and_bwd(K, G, n, weights):
    rng = np.random.default_rng(K * 1000 + G)
    g = rng.integers(0, G, n).astype(np.int32)
    v = rng.random((n, K)).astype(np.float32)
    w = rng.random(n).astype(np.float32) if weights else None
    say("soft groupby", K, G, n, weights)
    Sg = S().soft_groupby(dev(g), None if w is None else dev(w), dev(v), G)
    ref = oracle.soft_groupby(g, None if w is None else w.astype(np.float64), v.astype(np.float64), G)
    assert normwise(host(Sg), ref) <= TOL
    dS = rng.standard_normal((G, K)).astype(np.float32)
    dw, dv = S().soft_groupby_bwd(dev(g), None if w is None else dev(w), dev(v), dev(dS))
    rdw, rdv = oracle.soft_groupby_bwd(g, None if w is None else w.astype(np.float64), v.astype(np.float64),
                                       dS.astype(np.float64))
    assert normwise(host(dv), rdv) <= TOL
    assert normwise(host(dw), rdw) <= TOL


def _soft_case(n, G, tau):
    c = gen.soft_query_columns(n=n, n_groups=G)
    T = oracle.soft_groupby(c["g"], (c["x"] < 0.5).astype(np.float64), c["v"].astype(np.float64), G)
    return c, T.astype(np.float32)


@pytest.mark.parametrize("tau", [1.0, 0.1])
@pytest.mark.parametrize("n,G", [(10_000_000, 1000), (12_345, 17), (1, 1)])
def test_soft_query_step(n, G, tau):
    c, T = _soft_case(n, G, tau)
    say("soft query step", n, G, tau)
    step = S().SoftQueryStep(dev(c["x"]), dev(c["v"]), dev(c["g"]), dev(np.array([0.3], np.float32)), tau, G, dev(T),
                             want_dx=True)
    step()
    torch.cuda.synchronize()
    ref = oracle.soft_query(c["x"], c["v"], c["g"], 0.3, tau, G, T.astype(np.float64))
    assert normwise(host(step.S), ref["S"]) <= TOL
    # S carries a normwise error of at most e_S = TOL * max|S|; the loss,
    # dS = 2 (S - T) / G, dv = dS_g w and dc propagate it (plus their own
    # float32 rounding, bounded relative to their references).
    e_S = TOL * float(np.max(np.abs(ref["S"])))
    d = ref["S"] - T.astype(np.float64)
    assert abs(float(host(step.loss)[0]) - ref["loss"]) <= TOL * ref["loss"] + 2 * float(np.max(np.abs(d))) * e_S + e_S ** 2
    e_dS = TOL * float(np.max(np.abs(ref["dS"]))) + 2 * e_S / G
    assert float(np.max(np.abs(host(step.dS) - ref["dS"]))) <= e_dS
    assert float(np.max(np.abs(host(step.dv) - ref["dv"]))) <= TOL * float(np.max(np.abs(ref["dv"]))) + e_dS
    # dc: terms t_i = dS_g v_i w_i (1 - w_i) / tau; bound by their absolute sum
    w = ref["w"]
    wd = c["v"].astype(np.float64) * w * (1 - w) / tau
    t = ref["dS"][c["g"]] * wd
    assert abs(float(host(step.dc)[0]) - ref["dc"]) <= TOL * float(np.sum(np.abs(t))) + e_dS * float(np.sum(wd))
    assert float(np.max(np.abs(host(step.dx) + t))) <= TOL * float(np.max(np.abs(t))) + e_dS * float(np.max(wd))
    assert int(step.status.item()) == 0


def test_autograd_path_matches_direct_calls():
    c, T = _soft_case(100_000, 50, 0.1)
    x, v, g = dev(c["x"]), dev(c["v"]).requires_grad_(True), dev(c["g"])
    cc = dev(np.array([0.3], np.float32)).requires_grad_(True)
    Sg = S().SoftFilterGroupBy.apply(x, v, g, cc, 0.1, 50)
    loss = S().MSELoss.apply(Sg, dev(T))
    loss.backward()
    ref = oracle.soft_query(c["x"], c["v"], c["g"], 0.3, 0.1, 50, T.astype(np.float64))
    assert normwise(host(Sg), ref["S"]) <= TOL
    assert normwise(host(v.grad), ref["dv"]) <= TOL
    w = ref["w"]
    t = ref["dS"][c["g"]] * c["v"].astype(np.float64) * w * (1 - w) / 0.1
    assert abs(float(host(cc.grad)[0]) - ref["dc"]) <= TOL * float(np.sum(np.abs(t)))


@pytest.mark.parametrize("n", [1, 4099, 1_000_003])
@pytest.mark.parametrize("tau", [1.0, 0.1])
def test_soft_filter_temperature_gradient(n, tau):
    c = gen.soft_query_columns(n=n, n_groups=10)
    x = c["x"]
    cc = dev(np.array([0.3], np.float32))
    dw = gen.float_uniform(gen.stream_seed(98, n), n, -1, 1)
    say("soft filter dtau", n, tau)
    dx, dc, dtau = S().soft_filter_bwd(dev(x), cc, tau, dev(dw), want_dtau=True)
    rdx, rdc = oracle.soft_filter_bwd(x, 0.3, tau, dw.astype(np.float64))
    rdtau = oracle.soft_filter_bwd_tau(x, 0.3, tau, dw.astype(np.float64))
    z = (0.3 - x.astype(np.float64)) / tau
    assert abs(float(host(dc)[0]) - rdc) <= TOL * float(np.sum(np.abs(rdx)))
    # the mixed-sign sum's bound: tolerance times the sum of its terms' magnitudes
    assert abs(float(host(dtau)[0]) - rdtau) <= TOL * float(np.sum(np.abs(rdx * z)))


def test_backward_scalars_stable_across_repeated_calls():
    """dc and dtau reduce through one shared LDS scratch per kernel; every
    call must give the oracle's value (a missing barrier between the two
    block sums once corrupted dc on some calls only)."""
    n, G, tau = 1_000_003, 100, 0.1
    c, T = _soft_case(n, G, tau)
    ref = oracle.soft_query(c["x"], c["v"], c["g"], 0.3, tau, G, T.astype(np.float64))
    w = ref["w"]
    t = ref["dS"][c["g"]] * c["v"].astype(np.float64) * w * (1 - w) / tau
    z = (0.3 - c["x"].astype(np.float64)) / tau
    x, v, g = dev(c["x"]), dev(c["v"]), dev(c["g"])
    cc = dev(np.array([0.3], np.float32))
    dS = dev(ref["dS"].astype(np.float32))
    say("repeated backward scalars")
    for rep in range(8):
        _, dc, dtau = S().soft_filter_bwd(x, cc, tau, dS[g] * v, want_dx=False, want_dtau=True)
        assert abs(float(host(dc)[0]) - ref["dc"]) <= TOL * float(np.sum(np.abs(t))), rep
        assert abs(float(host(dtau)[0]) - ref["dtau"]) <= TOL * float(np.sum(np.abs(t * z))), rep


def test_autograd_temperature_gradient():
    c, T = _soft_case(100_000, 50, 0.5)
    x, v, g = dev(c["x"]), dev(c["v"]), dev(c["g"])
    cc = dev(np.array([0.3], np.float32)).requires_grad_(True)
    tau = torch.tensor([0.5], dtype=torch.float32, device=DEV, requires_grad=True)
    say("autograd dtau")
    Sg = S().SoftFilterGroupBy.apply(x, v, g, cc, tau, 50)
    loss = S().MSELoss.apply(Sg, dev(T))
    loss.backward()
    ref = oracle.soft_query(c["x"], c["v"], c["g"], 0.3, 0.5, 50, T.astype(np.float64))
    w = ref["w"]
    t = ref["dS"][c["g"]] * c["v"].astype(np.float64) * w * (1 - w) / 0.5
    z = (0.3 - c["x"].astype(np.float64)) / 0.5
    assert abs(float(host(cc.grad)[0]) - ref["dc"]) <= TOL * float(np.sum(np.abs(t)))
    assert tau.grad is not None and tau.grad.shape == tau.shape
    assert abs(float(host(tau.grad)[0]) - ref["dtau"]) <= TOL * float(np.sum(np.abs(t * z)))
    # a float temperature stays a fixed hyperparameter
    cc2 = dev(np.array([0.3], np.float32)).requires_grad_(True)
    S().MSELoss.apply(S().SoftFilterGroupBy.apply(x, v, g, cc2, 0.5, 50), dev(T)).backward()
    assert abs(float(host(cc2.grad)[0]) - float(host(cc.grad)[0])) <= TOL * float(np.sum(np.abs(t)))


def test_soft_reduces_to_exact_at_small_tau():
    """As tau -> 0 the soft query equals the exact filter + group-by SUM."""
    c = gen.soft_query_columns(n=200_000, n_groups=20)
    x = c["x"].copy()
    x[np.abs(x - 0.5) < 1e-2] = 0.0  # keep every row far from the threshold
    Sg = S().SoftFilterGroupBy.apply(dev(x), dev(c["v"]), dev(c["g"]), dev(np.array([0.5], np.float32)), 1e-4, 20)
    exact = oracle.soft_groupby(c["g"], (x < 0.5).astype(np.float64), c["v"].astype(np.float64), 20)
    assert normwise(host(Sg), exact) <= TOL


def test_group_range_flag():
    from paper_2211_02753_amd import _lib
    g = dev(np.array([0, 1, 5, 2], np.int32))
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    Sg = S().soft_groupby(g, None, dev(np.ones(4, np.float32)), 3, status=st)
    assert int(st.item()) & _lib.FLAG_GROUP_RANGE
    assert host(Sg).tolist() == [1.0, 1.0, 1.0]


@pytest.mark.parametrize("tau", [1.0, 0.1])
def test_soft_backward_full_size_from_the_oracle_dS(tau):
    """The fused backward over the full 10M-row workload, fed the oracle's dS
    (rounded to float32) instead of its own forward's, so no forward error
    enters: dv and dx within 1e-5 normwise, dc and dtau within 1e-5 of the
    absolute sums of their terms."""
    from paper_2211_02753_amd import _lib as L
    n, G = 10_000_000, 1000
    c, T = _soft_case(n, G, tau)
    ref = oracle.soft_query(c["x"], c["v"], c["g"], 0.3, tau, G, T.astype(np.float64))
    dS32 = ref["dS"].astype(np.float32)
    # the oracle's backward for exactly that dS: the group-by's, then the filter's
    w = oracle.soft_filter(c["x"], 0.3, tau)
    dw, dv = oracle.soft_groupby_bwd(c["g"], w, c["v"].astype(np.float64), dS32.astype(np.float64))
    dx, dc = oracle.soft_filter_bwd(c["x"], 0.3, tau, dw, want_dx=True)
    dtau = oracle.soft_filter_bwd_tau(c["x"], 0.3, tau, dw)
    lib = L.load()
    x, v, g = dev(c["x"]), dev(c["v"]), dev(c["g"])
    gdv, gdx = torch.empty_like(x), torch.empty_like(x)
    gdc = torch.empty(1, dtype=torch.float32, device=x.device)
    gdt = torch.empty(1, dtype=torch.float32, device=x.device)
    ws = S().soft_workspace(x.device)
    say("soft backward full size from the oracle's dS", tau)
    cd, dSd = dev(np.array([0.3], np.float32)), dev(dS32)   # held until the call has run
    L.check("bwd", lib.tdp_soft_filter_groupby_bwd(L.ptr(x), L.ptr(v), L.ptr(g), n, L.ptr(cd),
                                                   tau, G, L.ptr(dSd), L.ptr(gdv), L.ptr(gdx), L.ptr(gdc), L.ptr(gdt),
                                                   L.ptr(ws), ws.numel(), L.stream_handle(x.device)))
    torch.cuda.synchronize()
    assert normwise(host(gdv), dv) <= TOL
    assert normwise(host(gdx), dx) <= TOL
    t = dw * w * (1 - w) / tau                      # the terms of dc
    z = (0.3 - c["x"].astype(np.float64)) / tau      # and z t those of dtau
    assert abs(float(host(gdc)[0]) - dc) <= TOL * float(np.sum(np.abs(t)))
    assert abs(float(host(gdt)[0]) - dtau) <= TOL * float(np.sum(np.abs(t * z)))
