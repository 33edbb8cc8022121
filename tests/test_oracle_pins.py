"""Pins of the CPU oracle against facts fixed outside it: hand-worked
examples (tests/golden), brute force on tiny inputs, closed forms, algebraic
identities and library routines.  No GPU needed."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
import tdp_datagen as gen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


OPS = {"<": lambda a, b: a < b, "<=": lambda a, b: a <= b, ">": lambda a, b: a > b,
       ">=": lambda a, b: a >= b, "==": lambda a, b: a == b, "!=": lambda a, b: a != b}


# ---------------------------------------------------------------------------
# filter
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [np.int8, np.int32, np.int64])
@pytest.mark.parametrize("op", list(OPS))
def test_filter_brute_force(dtype, op):
    rng = np.random.default_rng(1)
    col = rng.integers(-100, 100, size=257).astype(dtype)
    for lit in (-101, -3, 0, 42, 100):
        want = [i for i in range(len(col)) if OPS[op](int(col[i]), lit)]
        assert oracle.filter(col, op, lit).tolist() == want


def test_filter_special_cases():
    col = np.arange(10, 20, dtype=np.int32)
    assert oracle.filter(col, "<", 10).size == 0              # literal at the minimum
    assert oracle.filter(col, "<", 20).tolist() == list(range(10))
    assert oracle.filter(col, "<=", 10).tolist() == [0]       # boundary equality
    assert oracle.filter(np.zeros(0, np.int32), "<", 5).size == 0
    # conjunction through an input selection
    sel = oracle.filter(col, ">=", 13)
    assert oracle.filter(col, "<", 16, sel=sel).tolist() == [3, 4, 5]


def test_filter_count_matches_popcount():
    f, _ = gen.small_query_tables(n_fact=20000, n_dim=100)
    rows = oracle.filter(f["day"], "<", 1278)
    assert rows.size == int(np.count_nonzero(f["day"] < 1278))
    assert np.all(np.diff(rows) > 0)


# ---------------------------------------------------------------------------
# join
# ---------------------------------------------------------------------------

def test_join_golden():
    g = _gold("join_pairs.json")
    a, b = oracle.join_pairs(g["build_key"], g["probe_key"])
    assert list(map(list, zip(a.tolist(), b.tolist()))) == g["expected_pairs"]


def test_join_nested_loop_and_count_closed_form():
    rng = np.random.default_rng(2)
    for nb, npb, kr in [(0, 5, 3), (7, 0, 3), (50, 80, 10), (300, 200, 40), (64, 64, 1)]:
        bk = rng.integers(0, kr, nb).astype(np.int32)
        pk = rng.integers(0, kr + 2, npb).astype(np.int32)
        want = [(i, j) for i in range(npb) for j in range(nb) if pk[i] == bk[j]]
        a, b = oracle.join_pairs(bk, pk)
        assert list(zip(a.tolist(), b.tolist())) == want
        ub, cb = np.unique(bk, return_counts=True)
        up, cp = np.unique(pk, return_counts=True)
        common = np.intersect1d(ub, up)
        closed = int(sum(cb[np.searchsorted(ub, k)] * cp[np.searchsorted(up, k)] for k in common))
        assert len(a) == closed


def test_join_int32_extremes():
    bk = np.array([np.iinfo(np.int32).min, np.iinfo(np.int32).max, 0], np.int32)
    pk = np.array([0, np.iinfo(np.int32).max, np.iinfo(np.int32).min, 7], np.int32)
    a, b = oracle.join_pairs(bk, pk)
    assert list(zip(a.tolist(), b.tolist())) == [(0, 2), (1, 1), (2, 0)]


# ---------------------------------------------------------------------------
# group-by query
# ---------------------------------------------------------------------------

def test_query_golden():
    g = _gold("tiny_query.json")
    f = {k: np.array(v, dtype=np.int64) for k, v in g["fact"].items()}
    d = {k: np.array(v, dtype=np.int64) for k, v in g["dim"].items()}
    r = oracle.query(len(f["key"]), keys=[(d["region"].astype(np.int8), 1), (f["flag"].astype(np.int8), 0)],
                     expr=oracle.EXPR_COL, a=(f["price"], 0), pred=(f["day"].astype(np.int32), "<", 10),
                     join=(f["key"], d["pk"]))
    e = g["expected"]
    assert r["k0"].tolist() == e["region"] and r["k1"].tolist() == e["flag"]
    assert r["sum"].tolist() == e["sum"] and r["count"].tolist() == e["count"]
    assert r["avg"].tolist() == e["avg"]


def _naive_query(fact, dim, pred, keyspec, value):
    """Nested-loop join and naive grouping in pure Python (tiny tables only)."""
    pairs = []
    for i in range(len(fact["key"])):
        if not pred(i):
            continue
        for j in range(len(dim["pk"])):
            if fact["key"][i] == dim["pk"][j]:
                pairs.append((i, j))
    groups = {}
    for i, j in pairs:
        k = keyspec(i, j)
        groups.setdefault(k, []).append(value(i, j))
    out = []
    for k in sorted(groups):
        vals = groups[k]
        s = sum(vals) % (1 << 64)
        s = s - (1 << 64) if s >= (1 << 63) else s
        out.append((k, s, len(vals)))
    return out, pairs


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_query_against_naive_small_config(seed):
    f, d = gen.small_query_tables(n_fact=600, n_dim=40, seed=gen.SEED_SMALL + 1000 + seed)
    # make the build side non-unique and partly missing to exercise M:N and misses
    d["pk"] = (np.arange(40) % 30).astype(np.int32)
    f["key"] = f["key"].copy()
    f["key"][::7] = 999
    ref, pairs = _naive_query(
        {k: v.tolist() for k, v in f.items()}, {k: v.tolist() for k, v in d.items()},
        lambda i: f["day"][i] < 1278, lambda i, j: (int(d["region"][j]), int(f["flag"][i])),
        lambda i, j: int(f["price"][i]))
    r = oracle.query(len(f["key"]), keys=[(d["region"], 1), (f["flag"], 0)], expr=oracle.EXPR_COL,
                     a=(f["price"], 0), pred=(f["day"], "<", 1278), join=(f["key"], d["pk"]))
    got = [((int(a), int(b)), int(s), int(c)) for a, b, s, c in zip(r["k0"], r["k1"], r["sum"], r["count"])]
    assert got == ref
    # invariants: counts add up to the join cardinality; sums add up mod 2^64; min <= avg <= max
    assert int(r["count"].sum()) == len(pairs)
    tot = sum(int(f["price"][i]) for i, _ in pairs) % (1 << 64)
    assert int(r["sum"].astype(np.uint64).sum(dtype=np.uint64)) == tot
    assert np.all(r["avg"] >= 100) and np.all(r["avg"] <= 100000)


def test_query_scaled_expression_against_naive():
    f, d = gen.scaled_query_tables(n_fact=500, n_dim=60)
    ref, _ = _naive_query(
        {"key": f["orderkey"].tolist()}, {"pk": d["orderkey"].tolist()},
        lambda i: f["shipday"][i] <= 2450, lambda i, j: (int(f["returnflag"][i]), int(f["linestatus"][i])),
        lambda i, j: int(f["extprice"][i]) * (100 - int(f["discount"][i])))
    r = oracle.query(len(f["orderkey"]), keys=[(f["returnflag"], 0), (f["linestatus"], 0)],
                     expr=oracle.EXPR_MUL_CONST_SUB, a=(f["extprice"], 0), b=(f["discount"], 0), K=100,
                     pred=(f["shipday"], "<=", 2450), join=(f["orderkey"], d["orderkey"]))
    got = [((int(a), int(b)), int(s), int(c)) for a, b, s, c in zip(r["k0"], r["k1"], r["sum"], r["count"])]
    assert got == ref
    # every fact key is a dim key, so the join keeps every filtered row
    assert int(r["count"].sum()) == int(np.count_nonzero(f["shipday"] <= 2450))


def test_query_int64_wrap_golden():
    g = _gold("int64_wrap.json")
    v = np.array(g["values"], dtype=np.int64)
    r = oracle.query(len(v), keys=[(np.zeros(len(v), np.int32), 0)], expr=oracle.EXPR_COL, a=(v, 0))
    assert r["sum"].tolist() == [g["expected_sum"]] and r["count"].tolist() == [3]
    assert r["avg"][0] == float(g["expected_sum"]) / 3.0
    assert r["wrapped"].tolist() == [1]


def test_query_empty_and_single():
    z = np.zeros(0, np.int32)
    r = oracle.query(0, keys=[(z, 0)], expr=oracle.EXPR_COL, a=(np.zeros(0, np.int64), 0))
    assert r["sum"].size == 0
    r = oracle.query(1, keys=[(np.array([5], np.int32), 0)], expr=oracle.EXPR_COL, a=(np.array([-9], np.int64), 0))
    assert r["k0"].tolist() == [5] and r["sum"].tolist() == [-9] and r["avg"].tolist() == [-9.0]


# ---------------------------------------------------------------------------
# many-to-many join aggregate and top-k
# ---------------------------------------------------------------------------

def test_mn_group_against_nested_loop_and_factorisation():
    l, r = gen.mn_join_tables(n_left=400, n_right=300, n_keys=50, n_groups=20)
    mo = oracle.MNGroupOracle(l["key"], l["gkey"], l["payload"], r["key"], r["payload"])
    # pre-aggregated route (distributivity mod 2^64), computed independently with numpy
    rsum = np.zeros(50, np.uint64)
    rcnt = np.zeros(50, np.int64)
    np.add.at(rsum, r["key"], r["payload"].astype(np.uint64))
    np.add.at(rcnt, r["key"], 1)
    for g in range(20):
        li = np.nonzero(l["gkey"] == g)[0]
        s_nl = 0
        c_nl = 0
        for i in li:
            for j in range(len(r["key"])):
                if l["key"][i] == r["key"][j]:
                    s_nl += int(l["payload"][i]) * int(r["payload"][j])
                    c_nl += 1
        s_nl %= 1 << 64
        s, c = mo.group(g)
        assert (s % (1 << 64), c) == (s_nl, c_nl)
        s_fac = int((l["payload"][li].astype(np.uint64) * rsum[l["key"][li]]).sum(dtype=np.uint64))
        assert s % (1 << 64) == s_fac and c == int(rcnt[l["key"][li]].sum())


def test_mn_query_matches_group_enumeration():
    l, r = gen.mn_join_tables(n_left=300, n_right=300, n_keys=30, n_groups=15)
    q = oracle.query(len(l["key"]), keys=[(l["gkey"], 0)], expr=oracle.EXPR_MUL, a=(l["payload"], 0),
                     b=(r["payload"], 1), join=(l["key"], r["key"]))
    mo = oracle.MNGroupOracle(l["key"], l["gkey"], l["payload"], r["key"], r["payload"])
    for g, s, c in zip(q["k0"], q["sum"], q["count"]):
        assert mo.group(g) == (int(s), int(c))


def test_mn_full_digest_totals_match_closed_forms():
    """The stored digest of the full 20M x 20M enumeration: its totals agree
    with COUNT = sum_l cntR(key_l) and SUM = sum_l p_l * sumR(key_l) (mod 2^64),
    computed with numpy from the same seeded tables, and its top-100 is
    ranked (SUM desc, key asc)."""
    dg = _gold("mn_full_digest.json")
    l, r = gen.mn_join_tables()
    cnt_r = np.bincount(r["key"], minlength=2_000_000).astype(np.int64)
    sum_r = np.zeros(2_000_000, np.uint64)
    np.add.at(sum_r, r["key"], r["payload"].astype(np.uint64))
    assert dg["count_total"] == int(cnt_r[l["key"]].sum())
    with np.errstate(over="ignore"):
        tot = (l["payload"].astype(np.uint64) * sum_r[l["key"]]).sum(dtype=np.uint64)
    assert dg["sum_total_mod_2_64"] == int(tot)
    # groups with at least one joined pair: those holding a left row whose key occurs on the right
    hit = cnt_r[l["key"]] > 0
    assert dg["groups"] == len(np.unique(l["gkey"][hit]))
    t = dg["top100"]
    assert all((-a[1], a[0]) < (-b[1], b[0]) for a, b in zip(t, t[1:]))


def test_topk_against_sorted():
    rng = np.random.default_rng(5)
    keys = rng.permutation(500).astype(np.int64)
    sums = rng.integers(-20, 20, 500).astype(np.int64)  # many ties
    want = sorted(range(500), key=lambda i: (-int(sums[i]), int(keys[i])))[:37]
    assert oracle.topk(keys, sums, 37).tolist() == want
    assert oracle.topk(keys[:5], sums[:5], 37).size == 5


# ---------------------------------------------------------------------------
# relaxed operators
# ---------------------------------------------------------------------------

def test_soft_filter_golden_closed_forms():
    g = _gold("soft_filter.json")
    for case in g["cases"]:
        x = np.array([g["c"] + case["x_minus_c"]], np.float32)
        w = oracle.soft_filter(x, g["c"], case["tau"])
        # x is rounded to float32; the logistic's slope bounds the effect
        assert abs(w[0] - case["w"]) < 1e-6 / case["tau"]
        _, dc = oracle.soft_filter_bwd(x, g["c"], case["tau"], np.ones(1), want_dx=False)
        assert abs(dc - case["dw_dc"]) < 1e-5 / case["tau"] ** 2


def test_soft_filter_symmetry_and_limit():
    x = np.linspace(-3, 3, 1001).astype(np.float32)
    c = 0.25
    w = oracle.soft_filter(x, c, 0.7)
    w_m = oracle.soft_filter((2 * c - x.astype(np.float64)).astype(np.float32), c, 0.7)
    assert np.all(np.abs(w + w_m - 1.0) < 1e-6)
    # tau -> 0: the exact step 1[x < c] wherever |x - c| >> tau
    w0 = oracle.soft_filter(x, c, 1e-4)
    far = np.abs(x - c) > 0.01
    assert np.array_equal(w0[far] > 0.5, (x < c)[far])
    assert np.all((w0[far] < 1e-30) | (w0[far] > 1 - 1e-15))
    # extreme arguments stay finite
    assert np.all(np.isfinite(oracle.soft_filter(np.array([-1e30, 1e30], np.float32), 0.0, 1e-3)))


def test_soft_groupby_reduces_to_exact_and_count():
    c = gen.soft_query_columns(n=5000, n_groups=37)
    w01 = (c["x"] < 0.5).astype(np.float64)
    S = oracle.soft_groupby(c["g"], w01, c["v"], 37)
    # exact filter + group-by SUM through the exact path (values scaled to integers)
    vi = np.round(c["v"].astype(np.float64) * 2 ** 24).astype(np.int64)
    ex = oracle.query(len(vi), keys=[(c["g"], 0)], expr=oracle.EXPR_COL, a=(vi, 0), pred=(
        (c["x"] < 0.5).astype(np.int8), "==", 1))
    S_exact = np.zeros(37)
    S_exact[ex["k0"]] = ex["sum"] / 2 ** 24
    assert np.allclose(S, S_exact, rtol=0, atol=1e-9)
    # v = 1 gives the soft count; the total is sum_i w_i v_i
    cnt = oracle.soft_groupby(c["g"], w01, np.ones(5000), 37)
    assert np.array_equal(cnt, np.bincount(c["g"], weights=w01, minlength=37))
    w = oracle.soft_filter(c["x"], 0.3, 1.0)
    S = oracle.soft_groupby(c["g"], w, c["v"], 37)
    assert abs(S.sum() - float(np.dot(w, c["v"].astype(np.float64)))) < 1e-9
    # K columns at once equal K single-column calls
    V = np.stack([c["v"], 1 - c["v"], np.ones(5000)], axis=1)
    SK = oracle.soft_groupby(c["g"], w, V, 37)
    for k in range(3):
        assert np.allclose(SK[:, k], oracle.soft_groupby(c["g"], w, V[:, k], 37), rtol=1e-14, atol=0)


def test_soft_query_gradients_finite_difference():
    cols = gen.soft_query_columns(n=3000, n_groups=25)
    x, v, g = cols["x"], cols["v"], cols["g"]
    T = oracle.soft_groupby(g, (x < 0.5).astype(np.float64), v, 25)
    for tau in (1.0, 0.1):
        r = oracle.soft_query(x, v, g, 0.3, tau, 25, T)
        h = 1e-6
        Lp = oracle.soft_query(x, v, g, 0.3 + h, tau, 25, T)["loss"]
        Lm = oracle.soft_query(x, v, g, 0.3 - h, tau, 25, T)["loss"]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - r["dc"]) <= 1e-6 * max(1.0, abs(r["dc"]))
        # L is quadratic in v: a central difference is exact up to rounding
        vd = v.astype(np.float64)
        for i in (0, 17, 2999):
            w = r["w"]
            def loss(vv):
                S = oracle.soft_groupby(g, w, vv, 25)
                return oracle.mse(S, T)[0]
            e = np.zeros_like(vd)
            e[i] = 1e-3
            fdv = (loss(vd + e) - loss(vd - e)) / 2e-3
            assert abs(fdv - r["dv"][i]) <= 1e-8 * max(1.0, abs(r["dv"][i]))


def _pe_case(rng, n, K1, K2, G):
    """Random probability rows (each sums to 1) and G segments with an empty
    one and a tail of rows outside every segment."""
    p = rng.random((n, K1)) + 1e-3
    p /= p.sum(1, keepdims=True)
    q = rng.random((n, K2)) + 1e-3
    q /= q.sum(1, keepdims=True)
    cuts = np.sort(rng.integers(0, n - 5, G - 1))
    seg = np.concatenate([[0], cuts, [n - 5]]).astype(np.int64)
    seg[G // 2 + 1] = seg[G // 2]  # segment G // 2 is empty
    seg[G // 2 + 1:] = np.maximum.accumulate(seg[G // 2 + 1:])
    return p, q, seg


def test_soft_pe_groupby_one_hot_is_the_exact_count():
    # one-hot probability rows turn the soft COUNT into the exact COUNT per
    # (segment, a, b), counted here from the integer labels directly
    rng = np.random.default_rng(11)
    n, K1, K2, G = 400, 5, 3, 7
    a = rng.integers(0, K1, n)
    b = rng.integers(0, K2, n)
    _, _, seg = _pe_case(rng, n, K1, K2, G)
    S = oracle.soft_pe_groupby(seg, np.eye(K1)[a], np.eye(K2)[b], G)
    want = np.zeros((G, K1, K2))
    for g in range(G):
        for i in range(seg[g], seg[g + 1]):
            want[g, a[i], b[i]] += 1
    assert np.array_equal(S, want)
    assert S.sum() == seg[G] - seg[0]  # rows past seg[G] belong to no segment


def test_soft_pe_groupby_special_cases():
    rng = np.random.default_rng(12)
    n, K1, K2, G = 300, 4, 2, 6
    p, q, seg = _pe_case(rng, n, K1, K2, G)
    S = oracle.soft_pe_groupby(seg, p, q, G)
    for g in range(G):
        lo, hi = seg[g], seg[g + 1]
        # rows are distributions, so each segment's cells add up to its row count
        assert abs(S[g].sum() - (hi - lo)) <= 1e-12 * max(1, hi - lo)
        # q = 1 (K2 = 1): the soft COUNT per class is the column sum
        S1 = oracle.soft_pe_groupby(seg, p, None, G)
        assert np.allclose(S1[g, :, 0], p[lo:hi].sum(0), rtol=1e-13, atol=1e-13)
    assert not S[G // 2].any()  # the empty segment
    # no segments: one group of all rows
    S0 = oracle.soft_pe_groupby(None, p, q, 1)
    assert np.allclose(S0[0], np.einsum("ia,ib->ab", p, q), rtol=1e-13)
    # an inverted or out-of-range segment is left 0
    bad = np.array([0, 50, 20, n + 1], np.int64)
    Sb = oracle.soft_pe_groupby(bad, p, q, 3)
    assert Sb[0].sum() > 0 and not Sb[1].any() and not Sb[2].any()


def test_soft_pe_groupby_backward_adjoint_and_finite_difference():
    rng = np.random.default_rng(13)
    n, K1, K2, G = 200, 6, 3, 5
    p, q, seg = _pe_case(rng, n, K1, K2, G)
    dS = rng.standard_normal((G, K1, K2))
    dp, dq = oracle.soft_pe_groupby_bwd(seg, p, q, dS)
    # S is bilinear: its derivative along (ep, eq) is S(ep, q) + S(p, eq), so
    # <dS, S(ep, q) + S(p, eq)> = <dp, ep> + <dq, eq> for any directions
    ep, eq = rng.standard_normal(p.shape), rng.standard_normal(q.shape)
    lhs = np.sum(dS * (oracle.soft_pe_groupby(seg, ep, q, G) + oracle.soft_pe_groupby(seg, p, eq, G)))
    rhs = np.sum(dp * ep) + np.sum(dq * eq)
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))
    # central differences of L = <dS, S> (exact up to rounding: L is linear in each row)
    L = lambda pp, qq: np.sum(dS * oracle.soft_pe_groupby(seg, pp, qq, G))
    for i, a, b in ((0, 0, 0), (77, 5, 2), (n - 6, 3, 1)):
        e = np.zeros_like(p)
        e[i, a] = 1e-3
        assert abs((L(p + e, q) - L(p - e, q)) / 2e-3 - dp[i, a]) <= 1e-9
        e = np.zeros_like(q)
        e[i, b] = 1e-3
        assert abs((L(p, q + e) - L(p, q - e)) / 2e-3 - dq[i, b]) <= 1e-9
    # rows outside every segment get zero gradients
    assert not dp[seg[G]:].any() and not dq[seg[G]:].any()
    # q = 1: dp[i][a] = dS[g_i][a][0]
    dp1, dq1 = oracle.soft_pe_groupby_bwd(seg, p, None, dS[:, :, :1])
    g_of = np.repeat(np.arange(G), np.diff(seg))
    assert dq1 is None and np.array_equal(dp1[:seg[G]], dS[g_of, :, 0])


def test_soft_query_temperature_gradient():
    # central differences of the loss in tau (h = 1e-6 relative)
    cols = gen.soft_query_columns(n=3000, n_groups=25)
    x, v, g = cols["x"], cols["v"], cols["g"]
    T = oracle.soft_groupby(g, (x < 0.5).astype(np.float64), v, 25)
    for tau in (1.0, 0.1):
        r = oracle.soft_query(x, v, g, 0.3, tau, 25, T)
        h = 1e-6 * tau
        Lp = oracle.soft_query(x, v, g, 0.3, tau + h, 25, T)["loss"]
        Lm = oracle.soft_query(x, v, g, 0.3, tau - h, 25, T)["loss"]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - r["dtau"]) <= 1e-5 * max(1.0, abs(r["dtau"])), (tau, fd, r["dtau"])
    # one element, dL/dw = 1: dw/dtau = -w (1 - w) (c - x) / tau^2 in closed form
    x1 = np.array([0.8], np.float32)
    for tau in (0.5, 2.0):
        z = (0.3 - float(x1[0])) / tau
        w = 1.0 / (1.0 + math.exp(-z))
        want = -w * (1.0 - w) * (0.3 - float(x1[0])) / tau ** 2
        assert abs(oracle.soft_filter_bwd_tau(x1, 0.3, tau, np.ones(1)) - want) <= 1e-15


def test_mse_closed_form():
    L, dS = oracle.mse(np.array([1.0, 2.0, 4.0]), np.array([1.0, 0.0, 1.0]))
    assert L == (0 + 4 + 9) / 3 and dS.tolist() == [0.0, 4 / 3, 2.0]


# ---------------------------------------------------------------------------
# classifier layers
# ---------------------------------------------------------------------------

def _bits(a):
    return np.asarray(a, np.float32).view(np.uint32)


def test_bf16_round_cases():
    u = np.array([0x3F800000, 0x3F808000, 0x3F818000, 0x3F808001, 0x7F7FFFFF, 0x7F800000,
                  0xFF800000, 0x80000000, 0x7FC00001, 0x7F800001, 0x00000001, 0x3F80FFFF], np.uint32)
    want = np.array([0x3F800000, 0x3F800000, 0x3F820000, 0x3F810000, 0x7F800000, 0x7F800000,
                     0xFF800000, 0x80000000, None, None, 0x00000000, 0x3F810000], dtype=object)
    got = _bits(oracle.bf16_round(u.view(np.float32)))
    for i in range(len(u)):
        if want[i] is None:
            assert np.isnan(got.view(np.float32)[i]) and (got[i] & 0xFFFF) == 0
        else:
            assert got[i] == want[i], hex(int(u[i]))


def test_bf16_round_matches_library():
    import torch
    x = gen.float_normal(123, 100000, 50.0)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(_bits(oracle.bf16_round(x)), _bits(ref))


def _im2col_conv(x, w, b):
    B, H, W, Cin = x.shape
    cols = np.stack([x[:, ky:ky + H - 2, kx:kx + W - 2, :] for ky in range(3) for kx in range(3)], axis=3)
    return np.tensordot(cols.astype(np.float64), w.reshape(w.shape[0], 9, Cin).astype(np.float64),
                        axes=([3, 4], [1, 2])) + b


def test_conv_forward_against_im2col_and_identity():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((2, 7, 6, 5)).astype(np.float32)
    w = rng.standard_normal((4, 3, 3, 5)).astype(np.float32)
    b = rng.standard_normal(4).astype(np.float32)
    y = oracle.conv3x3_fwd(x, w, b, relu=False)
    assert np.allclose(y, _im2col_conv(x, w, b), rtol=1e-12, atol=1e-12)
    assert np.array_equal(oracle.conv3x3_fwd(x, w, b, relu=True), np.maximum(y, 0))
    # a centre tap picks out the shifted input
    wid = np.zeros((5, 3, 3, 5), np.float32)
    for c in range(5):
        wid[c, 1, 1, c] = 1
    assert np.array_equal(oracle.conv3x3_fwd(x, wid, None, False), x[:, 1:-1, 1:-1, :].astype(np.float64))


def test_conv_ramp_golden():
    # x[b, y, x, 0] = x; kernel row [-1, 0, 1] in every row -> 3 * (x+1 - (x-1)) = 6 everywhere
    x = np.tile(np.arange(8, dtype=np.float32)[None, None, :, None], (1, 5, 1, 1))
    w = np.tile(np.array([-1, 0, 1], np.float32)[None, None, :, None], (1, 3, 1, 1))
    assert np.all(oracle.conv3x3_fwd(x, w, None, False) == 6.0)


def test_conv_backward_adjoint():
    rng = np.random.default_rng(8)
    B, H, W, Cin, Cout = 2, 6, 7, 3, 4
    x = rng.standard_normal((B, H, W, Cin)).astype(np.float32)
    w = rng.standard_normal((Cout, 3, 3, Cin)).astype(np.float32)
    r = rng.standard_normal((B, H - 2, W - 2, Cout)).astype(np.float32)
    y = oracle.conv3x3_fwd(x, w, None, False)
    dx = oracle.conv3x3_dgrad(r, w, H, W)
    dw, db = oracle.conv3x3_wgrad(x, r)
    lhs = float(np.sum(y * r))
    assert math.isclose(lhs, float(np.sum(dx * x)), rel_tol=1e-12)
    assert math.isclose(lhs, float(np.sum(dw * w)), rel_tol=1e-12)
    assert np.allclose(db, r.astype(np.float64).sum(axis=(0, 1, 2)), rtol=1e-13)


def test_maxpool_brute_force_and_grad_routing():
    rng = np.random.default_rng(9)
    x = rng.standard_normal((2, 6, 4, 3)).astype(np.float32)
    x[0, 0, 0, 0] = x[0, 1, 1, 0] = 5.0  # a tie: the first in row-major order wins
    y = oracle.maxpool2_fwd(x)
    for b, oy, ox, c in itertools.product(range(2), range(3), range(2), range(3)):
        assert y[b, oy, ox, c] == x[b, 2 * oy:2 * oy + 2, 2 * ox:2 * ox + 2, c].max()
    dy = rng.standard_normal(y.shape).astype(np.float32)
    dx = oracle.maxpool2_bwd(x, dy)
    assert dx[0, 0, 0, 0] == dy[0, 0, 0, 0] and dx[0, 1, 1, 0] == 0
    assert np.allclose(dx.sum(), dy.astype(np.float64).sum())
    assert np.count_nonzero(dx) == dy.size


def test_linear_against_matmul_and_adjoint():
    rng = np.random.default_rng(10)
    x = rng.standard_normal((5, 7)).astype(np.float32)
    w = rng.standard_normal((3, 7)).astype(np.float32)
    b = rng.standard_normal(3).astype(np.float32)
    y = oracle.linear_fwd(x, w, b, False)
    assert np.allclose(y, x.astype(np.float64) @ w.T.astype(np.float64) + b, rtol=1e-12, atol=1e-12)
    dy = rng.standard_normal((5, 3)).astype(np.float32)
    dx, dw, db = oracle.linear_bwd(x, w, dy)
    lhs = float(np.sum((y - b) * dy))
    assert math.isclose(lhs, float(np.sum(dx * x)), rel_tol=1e-12)
    assert math.isclose(lhs, float(np.sum(dw * w)), rel_tol=1e-12)
    assert np.allclose(db, dy.astype(np.float64).sum(0))


def test_softmax_expectation_closed_forms_and_fd():
    p, e = oracle.softmax_expect(np.zeros((1, 10), np.float32))
    assert np.allclose(p, 0.1) and abs(e[0] - 4.5) < 1e-14
    z = np.zeros((1, 10), np.float32)
    z[0, 7] = 100
    p, e = oracle.softmax_expect(z)
    assert abs(e[0] - 7) < 1e-30 + 1e-35 or abs(e[0] - 7) < 1e-12
    rng = np.random.default_rng(11)
    z = rng.standard_normal((4, 10)).astype(np.float32)
    p, e = oracle.softmax_expect(z)
    assert np.allclose(p.sum(1), 1.0)
    dE = rng.standard_normal(4)
    dz = oracle.softmax_expect_bwd(p, dE)
    # finite differences in float64 on the expectation, through an independent softmax
    def E64(zz):
        q = np.exp(zz - zz.max(1, keepdims=True))
        q /= q.sum(1, keepdims=True)
        return q @ np.arange(10.0)
    z64 = z.astype(np.float64)
    for m, k in [(0, 0), (1, 5), (3, 9)]:
        d = np.zeros_like(z64)
        d[m, k] = 1e-6
        fd = (E64(z64 + d) - E64(z64 - d))[m] / 2e-6 * dE[m]
        assert abs(fd - dz[m, k]) < 1e-8


def test_softmax_backward_finite_difference_and_expectation_case():
    rng = np.random.default_rng(12)
    z = rng.standard_normal((3, 10))
    dP = rng.standard_normal((3, 10))
    def sm(zz):
        q = np.exp(zz - zz.max(1, keepdims=True))
        return q / q.sum(1, keepdims=True)
    p = sm(z)
    dz = oracle.softmax_bwd(p, dP)
    for m, k in [(0, 0), (1, 4), (2, 9)]:
        d = np.zeros_like(z)
        d[m, k] = 1e-6
        fd = np.sum((sm(z + d) - sm(z - d)) * dP) / 2e-6
        assert abs(fd - dz[m, k]) < 1e-8
    # with dP_k = k * dE it reduces to the expectation backward
    dE = rng.standard_normal(3)
    assert np.allclose(oracle.softmax_bwd(p, dE[:, None] * np.arange(10.0)), oracle.softmax_expect_bwd(p, dE),
                       rtol=1e-12, atol=1e-14)


def test_argmax_ties_smallest_index():
    p = np.array([[0.1, 0.4, 0.4, 0.1], [0.25, 0.25, 0.25, 0.25], [0, 0, 0, 1]], np.float32)
    assert oracle.argmax(p).tolist() == [1, 0, 3]


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3], np.float32)
    p = np.array([1.0, 1.0, 1.0], np.float32)
    z = np.zeros(3, np.float32)
    po, mo, vo = oracle.adam(p, g, z, z, lr=0.01, b1=0.9, b2=0.999, eps=1e-8, step=1)
    g64 = g.astype(np.float64)
    assert np.allclose(mo, 0.1 * g64) and np.allclose(vo, 0.001 * g64 ** 2)
    assert np.allclose(po, 1.0 - 0.01 * g64 / (np.abs(g64) + 1e-8), rtol=1e-12)


def test_soft_filter_input_gradient_finite_difference():
    # dL/dx_i of L = sum_i dw_i w_i(x) by central differences in x_i alone
    # (float32 inputs: the step is the one the rounded points actually take)
    rng = np.random.default_rng(21)
    x = rng.standard_normal(64).astype(np.float32)
    dw = rng.standard_normal(64)
    c = 0.3
    for tau in (1.0, 0.1):
        dx, dc = oracle.soft_filter_bwd(x, c, tau, dw, want_dx=True)
        for i in (0, 9, 33, 63):
            xp, xm = x.copy(), x.copy()
            xp[i] = np.float32(x[i] + np.float32(1e-3 * tau))
            xm[i] = np.float32(x[i] - np.float32(1e-3 * tau))
            h = float(xp[i]) - float(xm[i])
            fd = dw[i] * (oracle.soft_filter(xp, c, tau)[i] - oracle.soft_filter(xm, c, tau)[i]) / h
            assert abs(fd - dx[i]) <= 1e-5 * max(abs(dx[i]), 1e-3 / tau), (tau, i, fd, dx[i])
        # moving the threshold c is moving every x the other way
        assert abs(dc + dx.sum()) <= 1e-12 * np.abs(dx).sum()


@pytest.mark.parametrize("K", [3, 10])
def test_soft_groupby_backward_adjoint_multi_column(K):
    # S(w, V) is linear in V and in w, so for any directions V', w':
    #   <dS, S(w, V')> = <dv, V'>   and   <dS, S(w', V)> = <dw, w'>
    rng = np.random.default_rng(22 + K)
    n, G = 500, 7
    g = rng.integers(0, G, n).astype(np.int32)
    w = rng.random(n)
    V = rng.standard_normal((n, K))
    dS = rng.standard_normal((G, K))
    dw, dv = oracle.soft_groupby_bwd(g, w, V, dS)
    Vp, wp = rng.standard_normal((n, K)), rng.standard_normal(n)
    lhs_v = np.sum(dS * oracle.soft_groupby(g, w, Vp, G))
    assert abs(lhs_v - np.sum(dv * Vp)) <= 1e-10 * max(1.0, abs(lhs_v))
    lhs_w = np.sum(dS * oracle.soft_groupby(g, wp, V, G))
    assert abs(lhs_w - np.sum(dw * wp)) <= 1e-10 * max(1.0, abs(lhs_w))
    # w = None means w = 1: dv[i, k] = dS[g_i, k]
    _, dv1 = oracle.soft_groupby_bwd(g, None, V, dS)
    assert np.array_equal(dv1, dS[g])


def test_adam_constant_gradient_over_several_steps():
    # With a constant gradient g the moments after t steps from zero are the
    # geometric sums m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the bias
    # corrections recover g and g^2 exactly and every step moves p by
    # lr * g / (|g| + eps).  Steps 2..5 start from the non-zero moments of the
    # step before; b1 and b2 are far apart so that swapping them shows.
    g = np.array([0.5, -2.0, 1e-3, 3.0], np.float32)
    g64 = g.astype(np.float64)
    lr, b1, b2, eps = 0.01, 0.6, 0.95, 1e-8
    p = np.ones(4, np.float32)
    m = np.zeros(4, np.float32)
    v = np.zeros(4, np.float32)
    for t in range(1, 6):
        po, mo, vo = oracle.adam(p, g, m, v, lr=lr, b1=b1, b2=b2, eps=eps, step=t)
        # the inputs were float32 roundings of the previous moments, so compare
        # the recurrence's fixed point within float32 input error
        assert np.allclose(mo, (1 - b1 ** t) * g64, rtol=1e-6, atol=0)
        assert np.allclose(vo, (1 - b2 ** t) * g64 ** 2, rtol=1e-6, atol=0)
        assert np.allclose(p.astype(np.float64) - po, lr * g64 / (np.abs(g64) + eps), rtol=1e-5, atol=0)
        p, m, v = po.astype(np.float32), mo.astype(np.float32), vo.astype(np.float32)


def test_adam_two_steps_expanded():
    # two steps from zero with gradients g1 then g2, expanded by hand:
    #   m2 = b1 (1 - b1) g1 + (1 - b1) g2,  v2 = b2 (1 - b2) g1^2 + (1 - b2) g2^2
    g1 = np.array([1.0, -0.5, 0.25], np.float32)
    g2 = np.array([-1.0, 2.0, 0.0], np.float32)
    lr, b1, b2, eps = 0.1, 0.5, 0.75, 0.0
    p0 = np.zeros(3, np.float32)
    z = np.zeros(3, np.float32)
    p1, m1, v1 = oracle.adam(p0, g1, z, z, lr=lr, b1=b1, b2=b2, eps=eps, step=1)
    p2, m2, v2 = oracle.adam(p1.astype(np.float32), g2, m1.astype(np.float32), v1.astype(np.float32),
                             lr=lr, b1=b1, b2=b2, eps=eps, step=2)
    # these constants and gradients are exact in binary, so every value is exact
    assert m2.tolist() == [0.25 * 1.0 + 0.5 * -1.0, 0.25 * -0.5 + 0.5 * 2.0, 0.25 * 0.25]
    assert v2.tolist() == [0.1875 * 1.0 + 0.25 * 1.0, 0.1875 * 0.25 + 0.25 * 4.0, 0.1875 * 0.0625]
    # step 1 moves every coordinate by lr * sign(g1) (eps = 0); step 2 by
    # lr * (m2 / (1 - b1^2)) / sqrt(v2 / (1 - b2^2))
    assert p1.tolist() == [-0.1, 0.1, -0.1]
    want = p1 - lr * (m2 / 0.75) / np.sqrt(v2 / 0.4375)
    assert np.allclose(p2, want, rtol=0, atol=1e-7)


# ---------------------------------------------------------------------------
# conjunctive WHERE (exact) and its relaxation (Section 4), one query
# description run exact or soft
# ---------------------------------------------------------------------------

def test_filter_f32_rounds_the_literal_to_float32():
    # 0.1 is not a float32; the column value float32(0.1) equals the rounded
    # literal, so it passes "<= 0.1" and fails "< 0.1" (a float64 comparison
    # would reverse the first)
    x = np.array([np.float32(0.1), np.float32(0.05), np.float32(0.2), -np.inf, np.inf], np.float32)
    assert oracle.filter_f32(x, "<=", 0.1).tolist() == [0, 1, 3]
    assert oracle.filter_f32(x, "<", 0.1).tolist() == [1, 3]
    assert oracle.filter_f32(x, "==", 0.1).tolist() == [0]
    assert oracle.filter_f32(x, ">", 0.1).tolist() == [2, 4]
    # against numpy's own float32 comparison on a larger column
    rng = np.random.default_rng(5)
    y = rng.standard_normal(5000).astype(np.float32)
    for op, f in OPS.items():
        assert np.array_equal(oracle.filter_f32(y, op, 0.3), np.nonzero(f(y, np.float32(0.3)))[0])


def test_where_conjunction_is_the_intersection_in_any_order():
    rng = np.random.default_rng(11)
    n = 4000
    a = rng.integers(0, 100, n).astype(np.int32)
    b = rng.integers(-50, 50, n).astype(np.int8)
    x = rng.standard_normal(n).astype(np.float32)
    conj = [(a, "<", 60), (b, ">=", -10), (x, "<", 0.25)]
    rows = oracle.where(n, conj)
    each = [set(oracle.filter(a, "<", 60)), set(oracle.filter(b, ">=", -10)), set(oracle.filter_f32(x, "<", 0.25))]
    assert rows.tolist() == sorted(set.intersection(*each))
    for perm in itertools.permutations(conj):
        assert np.array_equal(oracle.where(n, list(perm)), rows)
    assert np.array_equal(oracle.where(n, []), np.arange(n))


def test_query_with_conjunctive_predicates_against_naive():
    f, d = gen.small_query_tables(n_fact=700, n_dim=50, seed=gen.SEED_SMALL + 2024)
    conds = [(f["day"], "<", 1800), (f["price"], ">=", 30000), (f["flag"], "!=", 1)]
    keep = lambda i: f["day"][i] < 1800 and f["price"][i] >= 30000 and f["flag"][i] != 1
    ref, pairs = _naive_query(
        {k: v.tolist() for k, v in f.items()}, {k: v.tolist() for k, v in d.items()}, keep,
        lambda i, j: (int(d["region"][j]), int(f["flag"][i])), lambda i, j: int(f["price"][i]))
    r = oracle.query(len(f["key"]), keys=[(d["region"], 1), (f["flag"], 0)], expr=oracle.EXPR_COL,
                     a=(f["price"], 0), pred=conds, join=(f["key"], d["pk"]))
    got = [((int(a), int(b)), int(s), int(c)) for a, b, s, c in zip(r["k0"], r["k1"], r["sum"], r["count"])]
    assert got == ref
    assert int(r["count"].sum()) == len(pairs) > 0


def _soft_case(seed, n=2000, G=7):
    rng = np.random.default_rng(seed)
    x1 = rng.standard_normal(n).astype(np.float32)
    x2 = rng.integers(0, 50, n).astype(np.int32)
    v = rng.random(n).astype(np.float32)
    gid = rng.integers(0, G, n)
    return x1, x2, v, gid


def test_soft_where_hand_worked_example():
    # one group, v = 1: sigma(1) + sigma(0) + sigma(-1) = 1.5 from the first
    # conjunct, and sigma(0) = 1/2 for each row from the second
    x1 = np.array([0, 1, 2], np.float32)
    x2 = np.array([5, 5, 5], np.int32)
    S = oracle.soft_where([x1, x2], ["<", ">="], [1.0, 5.0], [1.0, 3.0], None, np.zeros(3, np.int64), 1)
    assert abs(S[0] - 0.75) <= 1e-15


def test_soft_where_single_conjunct_is_the_soft_filter_groupby():
    x1, _, v, gid = _soft_case(1)
    for tau in (1.0, 0.1):
        S = oracle.soft_where([x1], ["<"], [0.3], [tau], v, gid, 7)
        w = oracle.soft_filter(x1, 0.3, tau)
        want = oracle.soft_groupby(gid.astype(np.int32), w, v, 7)
        assert np.allclose(S, want, rtol=1e-13, atol=0)


def test_soft_where_directions_are_complementary_and_limits():
    x1, x2, v, gid = _soft_case(2)
    lt = oracle.soft_where([x1], ["<"], [0.3], [0.5], None, gid, 7)
    gt = oracle.soft_where([x1], [">"], [0.3], [0.5], None, gid, 7)
    counts = np.bincount(gid, minlength=7).astype(np.float64)
    assert np.allclose(lt + gt, counts, rtol=1e-14)
    # a conjunct that every row passes by a wide margin changes nothing
    far = np.full(len(x1), -1e4, np.float32)
    one = oracle.soft_where([x1], ["<"], [0.3], [0.5], v, gid, 7)
    two = oracle.soft_where([x1, far], ["<", "<"], [0.3, 0.0], [0.5, 1.0], v, gid, 7)
    assert np.allclose(one, two, rtol=1e-14)
    # tau -> 0 gives the exact conjunctive SUM (the Section 4 swap), for rows
    # away from their thresholds (integer column, half-integer threshold)
    keep = np.abs(x1 - 0.3) > 1e-3
    x1k, x2k, vk, gk = x1[keep], x2[keep], v[keep], gid[keep]
    S0 = oracle.soft_where([x1k, x2k], ["<", ">="], [0.3, 19.5], [1e-6, 1e-6], vk, gk, 7)
    rows = oracle.where(len(gk), [(x1k, "<", 0.3), (x2k, ">=", 20)])
    exact = np.bincount(gk[rows], weights=vk[rows].astype(np.float64), minlength=7)
    assert np.allclose(S0, exact, rtol=1e-12, atol=0)


@pytest.mark.parametrize("taus", [(1.0, 4.0), (0.1, 1.5)])
def test_soft_where_backward_finite_differences(taus):
    x1, x2, v, gid = _soft_case(3)
    ops = ["<", ">="]
    c = np.array([0.2, 21.5])
    tau = np.array(taus)
    r = np.random.default_rng(4).standard_normal(7)   # dL/dS of L = <r, S>
    dc, dtau, dv = oracle.soft_where_bwd([x1, x2], ops, c, tau, v, gid, r)

    def L(cc, tt, vv=v):
        return float(r @ oracle.soft_where([x1, x2], ops, cc, tt, vv, gid, 7))

    for j in range(2):
        for which, base, grad in (("c", c, dc), ("tau", tau, dtau)):
            h = 1e-6 * max(1.0, abs(base[j]))
            e = np.zeros(2)
            e[j] = h
            if which == "c":
                fd = (L(c + e, tau) - L(c - e, tau)) / (2 * h)
            else:
                fd = (L(c, tau + e) - L(c, tau - e)) / (2 * h)
            assert abs(fd - grad[j]) <= 1e-6 * max(1.0, np.abs(grad[j])), (which, j, fd, grad[j])
    # L is linear in v: the difference quotient is exact up to rounding
    vd = v.astype(np.float64)
    for i in (0, 99, 1999):
        e = np.zeros_like(vd)
        e[i] = 0.25
        fd = (L(c, tau, vd + e) - L(c, tau, vd - e)) / 0.5
        assert abs(fd - dv[i]) <= 1e-12 * max(1.0, abs(dv[i]))
    # one conjunct: the threshold gradient is the soft filter's
    dc1, _, _ = oracle.soft_where_bwd([x1], ["<"], [0.2], [taus[0]], v, gid, r)
    _, want = oracle.soft_filter_bwd(x1, 0.2, taus[0], r[gid] * v.astype(np.float64), want_dx=False)
    assert abs(dc1[0] - want) <= 1e-12 * max(1.0, abs(want))


def test_group_ids_against_ravel_multi_index():
    rng = np.random.default_rng(8)
    k0 = rng.integers(-3, 12, 500).astype(np.int8)
    k1 = rng.integers(100, 140, 500).astype(np.int32)
    gid = oracle.group_ids([(k0, -2, 12), (k1, 101, 38)])
    inside = (k0 >= -2) & (k0 < 10) & (k1 >= 101) & (k1 < 139)
    want = np.ravel_multi_index((k0[inside].astype(np.int64) + 2, k1[inside].astype(np.int64) - 101), (12, 38))
    assert np.array_equal(gid[inside], want)
    assert np.all(gid[~inside] == -1)


# ---------------------------------------------------------------------------
# learning from label proportions (Section 5.3)
# ---------------------------------------------------------------------------

def _llp_case(n=1000, F=6, C=2, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, F)).astype(np.float32)
    W = rng.standard_normal((C, F)) * 0.7
    b = rng.standard_normal(C) * 0.3
    return X, W, b


def test_llp_forward_closed_forms_and_invariants():
    import scipy.special as sp
    X, W, b = _llp_case(n=997, C=3)
    # bag of one row: the softmax itself (a library routine)
    S1 = oracle.llp_forward(X, W, b, 1)
    assert np.allclose(S1, sp.softmax(X.astype(np.float64) @ W.T + b, axis=1), rtol=1e-13, atol=1e-15)
    # every bag's soft counts add up to its size (the last bag is short)
    for bag in (8, 64, 256):
        S = oracle.llp_forward(X, W, b, bag)
        sizes = np.minimum(bag, 997 - bag * np.arange(len(S)))
        assert np.allclose(S.sum(1), sizes, rtol=1e-13)
    # constant classifier: p = (1/4, 3/4) on every row
    S = oracle.llp_forward(X, np.zeros((2, 6)), np.array([0.0, np.log(3.0)]), 100)
    assert np.allclose(S[0], [25.0, 75.0], rtol=1e-14)
    assert np.allclose(S[-1], [97 / 4, 97 * 3 / 4], rtol=1e-14)


@pytest.mark.parametrize("C,bag", [(2, 16), (3, 1), (2, 128)])
def test_llp_backward_finite_differences(C, bag):
    X, W, b = _llp_case(n=500, F=5, C=C, seed=C + bag)
    r = np.random.default_rng(9).standard_normal(((500 + bag - 1) // bag, C))
    dW, db = oracle.llp_backward(X, W, b, bag, r)
    L = lambda WW, bb: float(np.sum(r * oracle.llp_forward(X, WW, bb, bag)))
    h = 1e-6
    for c in range(C):
        for f in range(5):
            E = np.zeros_like(W)
            E[c, f] = h
            fd = (L(W + E, b) - L(W - E, b)) / (2 * h)
            assert abs(fd - dW[c, f]) <= 1e-6 * max(1.0, abs(dW[c, f]))
        e = np.zeros(C)
        e[c] = h
        fd = (L(W, b + e) - L(W, b - e)) / (2 * h)
        assert abs(fd - db[c]) <= 1e-6 * max(1.0, abs(db[c]))
    # the softmax's rows sum to one, so adding the same constant to every
    # class's bias changes nothing: the bias gradients sum to zero
    assert abs(db.sum()) <= 1e-9 * max(1.0, np.abs(db).sum())


def test_llp_predict_ties_and_argmax():
    X, W, b = _llp_case(n=300, C=3)
    got = oracle.llp_predict(X, W, b)
    assert np.array_equal(got, np.argmax(X.astype(np.float64) @ W.T + b, axis=1))
    # equal logits: the smallest class wins
    assert oracle.llp_predict(X[:5], np.zeros((3, 6)), np.zeros(3)).tolist() == [0] * 5


def test_noisy_counts_are_float32_sums():
    c = np.array([0, 3, 1 << 25], np.int64)
    z = np.array([0.5, -10.25, 1.0], np.float32)
    got = oracle.noisy_counts(c, z)
    assert got.dtype == np.float32
    assert got.tolist() == [0.5, -7.25, float(np.float32(1 << 25) + np.float32(1.0))]


# ---------------------------------------------------------------------------
# order-preserving dictionary encoding (Section 2)
# ---------------------------------------------------------------------------

def test_dictionary_hand_worked_and_order_preserving():
    words = [b"pear", b"apple", b"fig", b"apple", b"", b"apples", b"fig", b"zz"]
    rows = np.zeros((len(words), 8), np.uint8)
    for i, w in enumerate(words):
        rows[i, :len(w)] = np.frombuffer(w, np.uint8)
    d, codes = oracle.dict_build(rows)
    assert [bytes(r).rstrip(b"\0") for r in d] == [b"", b"apple", b"apples", b"fig", b"pear", b"zz"]
    assert codes.tolist() == [4, 1, 3, 1, 0, 2, 3, 5]
    # codes compare exactly as the strings do, and decode back
    for i, j in itertools.product(range(len(words)), repeat=2):
        assert (words[i] < words[j]) == (codes[i] < codes[j])
        assert (words[i] == words[j]) == (codes[i] == codes[j])
    assert np.array_equal(d[codes], rows)
    lb, found = oracle.dict_lookup(d, rows[[1, 2]])
    assert lb.tolist() == [1, 3] and found.tolist() == [1, 1]
    probe = np.zeros((4, 8), np.uint8)
    for i, w in enumerate([b"b", b"apple", b"zzz", b"a"]):
        probe[i, :len(w)] = np.frombuffer(w, np.uint8)
    lb, found = oracle.dict_lookup(d, probe)
    assert lb.tolist() == [3, 1, 6, 1] and found.tolist() == [0, 1, 0, 0]


def test_dictionary_against_numpy_unique():
    rng = np.random.default_rng(12)
    n, L = 3000, 12
    lens = rng.integers(1, L + 1, n)
    rows = rng.integers(97, 101, (n, L)).astype(np.uint8)   # a small alphabet: many repeats
    rows[np.arange(L)[None, :] >= lens[:, None]] = 0
    d, codes = oracle.dict_build(rows)
    # numpy's fixed-width byte strings compare with the padding removed
    u, inv = np.unique(rows.view(f"S{L}").ravel(), return_inverse=True)
    assert np.array_equal(d.view(f"S{L}").ravel(), u)
    assert np.array_equal(codes, inv.astype(np.int32))
