"""The library's calls captured into a HIP graph (torch.cuda.CUDAGraph) and
replayed: every replay, with eager work and synchronisations between the
replays, must reproduce the eager result.  No call enqueues a memset or a
host synchronisation, so a whole query step can be captured."""
import numpy as np
import pytest
import torch

import tdp_datagen as gen

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def say(*a):
    print(*a, flush=True)


def _small_query():
    from paper_2211_02753_amd import _lib as L
    from paper_2211_02753_amd import query as Q
    f, d = gen.small_query_tables()
    fd = {k: dev(v) for k, v in f.items()}
    dd = {k: dev(v) for k, v in d.items()}
    return Q.GroupbyQuery(len(f["key"]), keys=[Q.Key(dd["region"], 0, 25, L.BUILD), Q.Key(fd["flag"], 0, 3)],
                          expr=L.EXPR_COL, a=Q.Operand(fd["price"]), pred=(fd["day"], "<", 1278),
                          join=(dd["pk"], fd["key"], True)), (fd, dd)


def _snapshot(q):
    r = q.result()
    return {k: v.clone() for k, v in r.items()}


def test_exact_query_graph_replays_match_eager():
    q, keep = _small_query()
    say("graph: exact small query")
    q.launch_build()
    q.launch_probe()
    ref = _snapshot(q)
    assert ref["k0"].numel() == 75
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        q.launch_build()  # warm the capture stream once, eagerly
        q.launch_probe()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        q.launch_build()
        q.launch_probe()
    other, _ = _small_query()
    for rep in range(4):
        # eager work between the replays, then clear the outputs so a replay
        # that wrote nothing would show
        other.launch()
        other.result()
        for t in (q.sum, q.count, q.key0, q.key1):
            t.zero_()
        q.n_groups.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = q.result()
        for k in ref:
            assert torch.equal(got[k], ref[k]), (rep, k)


def test_soft_step_graph_replays_match_eager():
    from paper_2211_02753_amd import soft
    n, G = 1_000_003, 1000
    c = gen.soft_query_columns(n=n, n_groups=G)
    T = np.zeros(G)
    np.add.at(T, c["g"], np.where(c["x"] < 0.5, c["v"].astype(np.float64), 0.0))
    say("graph: soft step")
    step = soft.SoftQueryStep(dev(c["x"]), dev(c["v"]), dev(c["g"]), dev(np.array([0.3], np.float32)), 1.0, G,
                              dev(T.astype(np.float32)))
    step.forward()
    step.backward()
    torch.cuda.synchronize()
    ref = {k: getattr(step, k).clone() for k in ("S", "loss", "dS", "dv", "dc")}
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step.forward()
        step.backward()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step.forward()
        step.backward()
    for rep in range(4):
        step.forward()  # eager work between replays
        torch.cuda.synchronize()
        for k in ("S", "dS", "dv", "dc"):
            getattr(step, k).fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        # LDS float atomics add in arrival order, so runs agree to rounding
        for k, v in ref.items():
            got = getattr(step, k)
            assert torch.isfinite(got).all(), (rep, k)
            scale = max(float(v.abs().max()), 1e-30)
            assert float((got - v).abs().max()) <= 1e-5 * scale, (rep, k)


@pytest.mark.parametrize("grouped", [True, False])
def test_grouped_soft_count_graph_replays_match_eager(grouped):
    """The grouped soft COUNT (forward and backward) in a graph: every replay
    reproduces the eager outputs bit for bit (fixed summation order, no
    atomics), including the flags the forward's finishing kernel returns."""
    from paper_2211_02753_amd import soft
    c = gen.pe_grid_columns(n_grids=2000)
    p, q = dev(c["p"]), dev(c["q"])
    seg = dev(c["seg"]) if grouped else None
    G = 2000 if grouped else 1
    dS = torch.linspace(-1.0, 1.0, G * 20, device=DEV).reshape(G, 10, 2)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    say("graph: grouped soft count", grouped)

    def step():
        S = soft.soft_pe_groupby(p, q, seg, G, status=st)
        dp, dq = soft.soft_pe_groupby_bwd(p, q, seg, dS)
        return S, dp, dq

    ref = [t.clone() for t in step()]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        outs = step()
    for rep in range(4):
        step()  # eager work between replays
        torch.cuda.synchronize()
        for t in outs:
            t.fill_(float("nan"))
        st.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(st.item()) == 0, rep
        for k, (got, want) in enumerate(zip(outs, ref)):
            assert torch.equal(got, want), (rep, k)
