"""One query description run exact or relaxed (Section 4's trainable flag):
conjunctive WHERE clauses in the exact fused group-by against the oracle
(bit-exact, every probe strategy), the relaxed query's forward and backward
against the float64 oracle (1e-5), and thresholds learned from grouped
counts that swap back into the exact query's answer."""
import ctypes as C

import numpy as np
import pytest
import scipy.special as sp
import torch

import oracle
import tdp_datagen as gen
from paper_2211_02753_amd import _lib as L
from paper_2211_02753_amd import query as Q
from paper_2211_02753_amd import trainable as TR

pytestmark = pytest.mark.gpu
DEV = "cuda"


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _same(got, want, keys=("k0", "k1", "sum", "count")):
    for k in keys:
        if k in want:
            assert np.array_equal(got[k].cpu().numpy(), want[k]), k
    assert np.array_equal(got["avg"].cpu().numpy().view(np.int64), want["avg"].view(np.int64))


CONJ = [("day", "<", 1700), ("x", "<", 0.25), ("qty", ">=", 12), ("price", "!=", 5000)]


@pytest.mark.parametrize("n", [1, 4099, 300_007])
def test_exact_conjunction_matches_oracle(n):
    tab = gen.where_table(n)
    td = {k: t(v) for k, v in tab.items()}
    print(f"exact conjunction n={n}", flush=True)
    got = Q.GroupbyQuery(n, [Q.Key(td["region"], 0, 25), Q.Key(td["flag"], 0, 3)], expr=L.EXPR_COL,
                         a=Q.Operand(td["price"]), pred=[(td[c], op, lit) for c, op, lit in CONJ])()
    want = oracle.query(n, keys=[(tab["region"], 0), (tab["flag"], 0)], expr=oracle.EXPR_COL, a=(tab["price"], 0),
                        pred=[(tab[c], op, lit) for c, op, lit in CONJ])
    _same(got, want)
    # COUNT over two int8 keys with an int32 first conjunct: the kernel built for exactly these columns
    got3 = Q.GroupbyQuery(n, [Q.Key(td["region"], 0, 25), Q.Key(td["flag"], 0, 3)],
                          pred=[(td[c], op, lit) for c, op, lit in CONJ])()
    want3 = oracle.query(n, keys=[(tab["region"], 0), (tab["flag"], 0)], pred=[(tab[c], op, lit) for c, op, lit in CONJ])
    _same(got3, want3)
    # a float conjunct first: the integer one still takes the first slot
    got2 = Q.GroupbyQuery(n, [Q.Key(td["region"], 0, 25)], pred=[(td["x"], ">=", -0.5), (td["qty"], "<=", 30)])()
    want2 = oracle.query(n, keys=[(tab["region"], 0)], pred=[(tab["x"], ">=", -0.5), (tab["qty"], "<=", 30)])
    _same(got2, want2)


def test_exact_conjunction_with_join_selection_and_partitioned_paths():
    f, d = gen.small_query_tables(n_fact=200_000, n_dim=1000)
    fd, dd = {k: t(v) for k, v in f.items()}, {k: t(v) for k, v in d.items()}
    conj = [("day", "<", 2000), ("price", ">=", 20000), ("flag", "!=", 2)]
    print("conjunction with a join", flush=True)
    got = Q.GroupbyQuery(len(f["key"]), [Q.Key(dd["region"], 0, 25, L.BUILD), Q.Key(fd["flag"], 0, 3)],
                         expr=L.EXPR_COL, a=Q.Operand(fd["price"]), pred=[(fd[c], o, v) for c, o, v in conj],
                         join=(dd["pk"], fd["key"], True))()
    want = oracle.query(len(f["key"]), keys=[(d["region"], 1), (f["flag"], 0)], expr=oracle.EXPR_COL,
                        a=(f["price"], 0), pred=[(f[c], o, v) for c, o, v in conj], join=(f["key"], d["pk"]))
    _same(got, want)
    # selection vector + conjuncts (generic kernel, candidates from sel)
    sel_h = np.arange(0, len(f["key"]), 3, dtype=np.int32)
    got = Q.GroupbyQuery(len(f["key"]), [Q.Key(fd["flag"], 0, 3)], pred=[(fd[c], o, v) for c, o, v in conj],
                         sel=t(sel_h))()
    want = oracle.query(len(sel_h), keys=[(f["flag"][sel_h], 0)],
                        pred=[(f[c][sel_h], o, v) for c, o, v in conj])
    _same(got, want)
    # staged probe of a keys-only join
    s, sd = gen.scaled_query_tables(n_fact=400_000, n_dim=120_000)
    st, sdd = {k: t(v) for k, v in s.items()}, {k: t(v) for k, v in sd.items()}
    conj2 = [("shipday", "<=", 2000), ("discount", "<", 7), ("extprice", ">", 200_000)]
    for strategy in (L.PROBE_DIRECT, L.PROBE_STAGED):
        print(f"scaled conjunction strategy={strategy}", flush=True)
        got = Q.GroupbyQuery(len(s["orderkey"]), [Q.Key(st["returnflag"], 0, 3), Q.Key(st["linestatus"], 0, 2)],
                             expr=L.EXPR_MUL_CONST_SUB, a=Q.Operand(st["extprice"]), b=Q.Operand(st["discount"]),
                             k=100, pred=[(st[c], o, v) for c, o, v in conj2],
                             join=(sdd["orderkey"], st["orderkey"], True), strategy=strategy)()
        want = oracle.query(len(s["orderkey"]), keys=[(s["returnflag"], 0), (s["linestatus"], 0)],
                            expr=oracle.EXPR_MUL_CONST_SUB, a=(s["extprice"], 0), b=(s["discount"], 0), K=100,
                            pred=[(s[c], o, v) for c, o, v in conj2], join=(s["orderkey"], sd["orderkey"]))
        _same(got, want)
    # partitioned aggregation of a large dense table (AUTO picks it at 2^20 rows, 300K groups)
    n = (1 << 20) + 5
    rng = np.random.default_rng(7)
    gk = rng.integers(0, 300_000, n).astype(np.int32)
    val = rng.integers(-1000, 1000, n).astype(np.int64)
    xf = rng.standard_normal(n).astype(np.float32)
    day = rng.integers(0, 2556, n).astype(np.int32)
    print("conjunction with partitioned aggregation", flush=True)
    got = Q.GroupbyQuery(n, [Q.Key(t(gk), 0, 300_000)], expr=L.EXPR_COL, a=Q.Operand(t(val)),
                         pred=[(t(day), ">", 600), (t(xf), "<=", 1.0)])()
    want = oracle.query(n, keys=[(gk, 0)], expr=oracle.EXPR_COL, a=(val, 0), pred=[(day, ">", 600), (xf, "<=", 1.0)])
    _same(got, want)


# ------------------------------------------------------------------ relaxed

def _soft_setup(n, value, big_groups=False):
    tab = gen.where_table(n)
    td = {k: t(v) for k, v in tab.items()}
    where = [TR.Where(td["x"], "<", 0.25), TR.Where(td["day"], "<", 1700.5), TR.Where(td["qty"], ">=", 11.5),
             TR.Where(td["flag"], ">", 0.5)]
    taus = [0.5, 60.0, 2.0, 0.3]
    if big_groups:
        gk = gen.uniform_int(gen.stream_seed(gen.SEED_WHERE, 9), n, 0, 39_999, np.int32)
        keys_h, keys = [(gk, 0, 40_000)], [Q.Key(t(gk), 0, 40_000)]
    else:
        keys_h = [(tab["region"], 0, 25), (tab["flag"], 0, 3)]
        keys = [Q.Key(td["region"], 0, 25), Q.Key(td["flag"], 0, 3)]
    v_h = None if value is None else tab[value]
    q = TR.TrainableQuery(n, keys, where, value=None if value is None else td[value], tau=taus)
    xs = [tab["x"], tab["day"], tab["qty"], tab["flag"]]
    ops = [w.op for w in where]
    c = [0.25, 1700.5, 11.5, 0.5]
    return q, xs, ops, c, taus, v_h, oracle.group_ids(keys_h)


@pytest.mark.parametrize("n,value,big", [(5, "price", False), (100_003, "price", False), (100_003, None, False),
                                         (2_000_001, "price", False), (300_001, "x", True)])
def test_soft_query_forward_matches_oracle(n, value, big):
    q, xs, ops, c, taus, v_h, gid = _soft_setup(n, value, big)
    print(f"soft query forward n={n} value={value} groups={q.G}", flush=True)
    S = q.compile(trainable=True)().cpu().numpy().astype(np.float64)
    want = oracle.soft_where(xs, ops, c, taus, v_h, gid, q.G)
    assert np.max(np.abs(S - want)) <= 1e-5 * np.max(np.abs(want))


def _bounds(xs, ops, c, taus, v, gid, dS):
    """Tolerance scales of the mixed-sign sums: sum_i |t_ij| and sum_i |t_ij z_ij|."""
    z = [np.array([1.0 if o in ("<", "<=") else -1.0])[0] * (c[j] - xs[j].astype(np.float64)) / taus[j]
         for j, o in enumerate(ops)]
    sg = [sp.expit(zz) for zz in z]
    w = np.prod(sg, axis=0)
    e = np.ones(len(gid)) if v is None else v.astype(np.float64)
    base = np.abs(dS[gid] * e * w)
    bc = [np.sum(base * (1 - sg[j]) / taus[j]) for j in range(len(ops))]
    bt = [np.sum(base * (1 - sg[j]) * np.abs(z[j]) / taus[j]) for j in range(len(ops))]
    return bc, bt


@pytest.mark.parametrize("n,value,big", [(4099, "price", False), (2_000_001, "price", False), (100_003, None, False),
                                         (300_001, "x", True)])
def test_soft_query_backward_matches_oracle(n, value, big):
    q, xs, ops, c, taus, v_h, gid = _soft_setup(n, value, big)
    rng = np.random.default_rng(n)
    dS = rng.standard_normal(q.G).astype(np.float32)
    print(f"soft query backward n={n} value={value} groups={q.G}", flush=True)
    lib = L.load()
    plan = q.compile(trainable=True)
    J = len(ops)
    dc = torch.empty(J, dtype=torch.float32, device=DEV)
    dtau = torch.empty(J, dtype=torch.float32, device=DEV)
    de = torch.empty(n, dtype=torch.float32, device=DEV)
    from paper_2211_02753_amd.soft import soft_workspace
    ws = soft_workspace(DEV)
    tau_arr = torch.tensor(taus, dtype=torch.float32, device=DEV)
    dSd = t(dS)   # held until the call has run
    L.check("bwd", lib.tdp_soft_query_bwd(C.byref(plan.desc), L.ptr(q.c), L.ptr(tau_arr), L.ptr(dSd), L.ptr(dc),
                                          L.ptr(dtau), L.ptr(de), L.ptr(ws), ws.numel(), L.stream_handle(DEV)))
    torch.cuda.synchronize()
    wdc, wdt, wdv = oracle.soft_where_bwd(xs, ops, c, taus, v_h, gid, dS.astype(np.float64))
    bc, bt = _bounds(xs, ops, c, taus, v_h, gid, dS.astype(np.float64))
    gdc, gdt = dc.cpu().numpy(), dtau.cpu().numpy()
    for j in range(J):
        assert abs(gdc[j] - wdc[j]) <= 1e-5 * bc[j] + 1e-30, (j, gdc[j], wdc[j], bc[j])
        assert abs(gdt[j] - wdt[j]) <= 1e-5 * bt[j] + 1e-30, (j, gdt[j], wdt[j], bt[j])
    gde = de.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(gde - wdv)) <= 1e-5 * np.max(np.abs(wdv))


def test_soft_query_autograd_and_key_domain_flag():
    n = 50_000
    q, xs, ops, c, taus, v_h, gid = _soft_setup(n, "price")
    plan = q.compile(trainable=True)
    cc = q.c.clone().requires_grad_(True)
    tt = q.tau.clone().requires_grad_(True)
    r = torch.from_numpy(np.random.default_rng(3).standard_normal(q.G).astype(np.float32)).to(DEV)
    S = plan(cc, tt)
    (S * r).sum().backward()
    wdc, wdt, _ = oracle.soft_where_bwd(xs, ops, c, taus, v_h, gid, r.cpu().numpy().astype(np.float64))
    bc, bt = _bounds(xs, ops, c, taus, v_h, gid, r.cpu().numpy().astype(np.float64))
    for j in range(len(ops)):
        assert abs(cc.grad[j].item() - wdc[j]) <= 1e-5 * bc[j]
        assert abs(tt.grad[j].item() - wdt[j]) <= 1e-5 * bt[j]
    # a group key outside its declared domain raises the device flag
    tab = gen.where_table(1000)
    reg = tab["region"].copy()
    reg[17] = 30
    bad = TR.TrainableQuery(1000, [Q.Key(t(reg), 0, 25)], [TR.Where(t(tab["x"]), "<", 0.0)])
    with pytest.raises(L.TdpError):
        bad.compile(trainable=True)()
    # a temperature that is not positive and finite (device data) raises its flag
    good = TR.TrainableQuery(1000, [Q.Key(t(tab["region"]), 0, 25)], [TR.Where(t(tab["x"]), "<", 0.0)])
    gp = good.compile(trainable=True)
    for bad_tau in (0.0, -1.0, float("inf")):
        with pytest.raises(L.TdpError, match="BAD_PARAM"):
            gp(good.c, torch.tensor([bad_tau], dtype=torch.float32, device=DEV))
    assert torch.isfinite(gp(good.c, good.tau)).all()


def _dense_counts(groups, card1):
    k0, k1, cnt = (groups[k].cpu().numpy() for k in ("k0", "k1", "count"))
    out = np.zeros(25 * card1, np.float32)
    out[k0 * card1 + k1] = cnt
    return out


def test_learned_thresholds_swap_to_the_exact_answer():
    """Train the two thresholds of WHERE day < c1 AND qty >= c2 through the
    relaxed query against the exact engine's COUNT per (region, flag), then
    compile the same query exact: the learned thresholds fold into the true
    literals and the exact answer equals the target bit for bit."""
    n = 1_000_000
    tab = gen.where_table(n)
    td = {k: t(v) for k, v in tab.items()}
    keys = [Q.Key(td["region"], 0, 25), Q.Key(td["flag"], 0, 3)]
    truth = TR.TrainableQuery(n, keys, [TR.Where(td["day"], "<", 1278), TR.Where(td["qty"], ">=", 20)])
    target = truth.compile(trainable=False)()
    T = t(_dense_counts(target, 3))
    q = TR.TrainableQuery(n, keys, [TR.Where(td["day"], "<", 2000.0), TR.Where(td["qty"], ">=", 5.0)],
                          tau=[100.0, 5.0])
    before = _dense_counts(q.compile(trainable=False)(), 3)
    plan = q.compile(trainable=True)
    lib = L.load()
    m = torch.zeros(2, dtype=torch.float32, device=DEV)
    v = torch.zeros(2, dtype=torch.float32, device=DEV)
    # temperatures annealed from (100, 5) to (1, 0.3) and learning rates from
    # (30, 0.5) to (2, 0.05), geometrically: the relaxed loss's minimum at the
    # final temperatures lies at (1277.46, 19.50), inside the cells that fold
    # to the literals 1278 and 20
    steps = 3000
    s = L.stream_handle(DEV)
    for it in range(steps):
        f = it / (steps - 1)
        q.tau.copy_(torch.tensor([100.0 * 0.01 ** f, 5.0 * 0.06 ** f]))
        loss, dc, _ = plan.loss_and_grad(T)
        for j, lr in enumerate((30.0 * (2.0 / 30.0) ** f, 0.5 * 0.1 ** f)):
            L.check("adam", lib.tdp_adam_step(L.ptr(q.c[j:j + 1]), L.ptr(dc[j:j + 1]), L.ptr(m[j:j + 1]),
                                              L.ptr(v[j:j + 1]), 1, lr, 0.9, 0.999, 1e-8, it + 1, None, s))
    learned = q.c.cpu().tolist()
    exact = q.compile(trainable=False)
    print(f"learned thresholds {learned} -> literals {exact.literals}; final soft loss {loss.item():.3g}", flush=True)
    got = _dense_counts(exact(), 3)
    T_h = T.cpu().numpy()
    assert np.abs(before - T_h).sum() > 0.2 * T_h.sum()        # the starting thresholds were far off
    assert exact.literals == [1278, 20]
    assert np.array_equal(got, T_h)
