"""Parity of the exact operators (filter, hash join, grouped aggregate) with
the CPU oracle: bit-exact for every integer result, and AVG as the same
rounded float64 division."""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import oracle
import tdp_datagen as gen

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def q():
    from paper_2211_02753_amd import query
    return query


def L():
    from paper_2211_02753_amd import _lib
    return _lib


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)


# ---------------------------------------------------------------------- filter

@pytest.mark.parametrize("dtype", [np.int8, np.int32, np.int64])
@pytest.mark.parametrize("n", [0, 1, 17, 16384, 16385, 100_003])
def test_filter_parity(dtype, n):
    rng = np.random.default_rng(n + 7)
    col = rng.integers(-100, 100, size=n).astype(dtype)
    d = dev(col)
    for op in ["<", "<=", ">", ">=", "==", "!="]:
        for lit in (-101, 0, 37, 100):
            say("filter", dtype.__name__, n, op, lit)
            got = host(q().filter(d, op, lit))
            assert np.array_equal(got, oracle.filter(col, op, lit)), (op, lit)


def test_filter_selection_chain_and_extremes():
    rng = np.random.default_rng(3)
    col = rng.integers(-2**40, 2**40, size=70_001).astype(np.int64)
    d = dev(col)
    sel = q().filter(d, ">", -2**39)
    got = host(q().filter(d, "<", 2**39, sel=sel))
    want = oracle.filter(col, "<", 2**39, sel=oracle.filter(col, ">", -2**39))
    assert np.array_equal(got, want)
    assert q().filter(d, "<", -2**41).numel() == 0                  # none pass
    assert np.array_equal(host(q().filter(d, ">=", -2**41)), np.arange(len(col)))  # all pass


def test_filter_full_scaled_column():
    f, _ = gen.scaled_query_tables(n_fact=60_000_000, n_dim=16)  # only shipday is used here
    say("filter full 60M shipday<=2450")
    got = host(q().filter(dev(f["shipday"]), "<=", 2450))
    want = oracle.filter(f["shipday"], "<=", 2450)
    assert got.shape == want.shape and np.array_equal(got, want)


# ------------------------------------------------------------------- hash join

def _sorted_pairs(a, b):
    a, b = np.asarray(a, np.int64), np.asarray(b, np.int64)
    o = np.lexsort((b, a))
    return a[o], b[o]


@pytest.mark.parametrize("nb,np_,kr", [(0, 10, 3), (10, 0, 3), (1, 1, 1), (1000, 5000, 700), (20000, 30000, 500),
                                       (4096, 4096, 1)])
def test_join_pairs_parity(nb, np_, kr):
    rng = np.random.default_rng(nb * 7 + np_)
    bk = rng.integers(0, kr, nb).astype(np.int32)
    pk = rng.integers(0, kr + 50, np_).astype(np.int32)
    if nb > 2:
        bk[0] = np.iinfo(np.int32).min   # the table's empty marker value is a valid key
        bk[1] = np.iinfo(np.int32).max
    if np_ > 3:
        pk[:3] = [np.iinfo(np.int32).min, np.iinfo(np.int32).max, np.iinfo(np.int32).min]
    say("join pairs", nb, np_, kr)
    wa, wb = oracle.join_pairs(bk, pk)
    if nb == 0 or np_ == 0:
        assert q().hash_join(dev(bk), dev(pk), count_only=True) == 0
        return
    ga, gb = q().hash_join(dev(bk), dev(pk))
    assert q().hash_join(dev(bk), dev(pk), count_only=True) == len(wa)
    x = _sorted_pairs(host(ga), host(gb))
    y = _sorted_pairs(wa, wb)
    assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])


def test_join_with_probe_selection_and_unique_flag():
    rng = np.random.default_rng(11)
    bk = rng.permutation(5000).astype(np.int32)
    pk = rng.integers(0, 6000, 20000).astype(np.int32)
    sel = oracle.filter(pk, "<", 3000)
    ga, gb = q().hash_join(dev(bk), dev(pk), probe_sel=dev(sel), build_unique=True)
    wa, wb = oracle.join_pairs(bk, pk, probe_sel=sel)
    x, y = _sorted_pairs(host(ga), host(gb)), _sorted_pairs(wa, wb)
    assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
    dup = bk.copy()
    dup[7] = dup[8]
    with pytest.raises(L().TdpError, match="DUP_BUILD"):
        q().hash_join(dev(dup), dev(pk), build_unique=True)


# -------------------------------------------------------------- grouped query

def _cmp(got, want, keys=2):
    assert np.array_equal(host(got["k0"]), want["k0"])
    if keys > 1:
        assert np.array_equal(host(got["k1"]), want["k1"])
    assert np.array_equal(host(got["sum"]), want["sum"])
    assert np.array_equal(host(got["count"]), want["count"])
    assert np.array_equal(host(got["avg"]).view(np.uint64), want["avg"].view(np.uint64))


def _small_query(f, d, Q):
    Key, Op = Q.Key, Q.Operand
    fd = {k: dev(v) for k, v in f.items()}
    dd = {k: dev(v) for k, v in d.items()}
    gq = Q.GroupbyQuery(len(f["key"]), keys=[Key(dd["region"], 0, 25, L().BUILD), Key(fd["flag"], 0, 3)],
                        expr=L().EXPR_COL, a=Op(fd["price"]), pred=(fd["day"], "<", 1278),
                        join=(dd["pk"], fd["key"], True))
    return gq


def test_small_query_full_size():
    f, d = gen.small_query_tables()
    say("small query 1M x 10K")
    got = _small_query(f, d, q())()
    want = oracle.query(len(f["key"]), keys=[(d["region"], 1), (f["flag"], 0)], expr=oracle.EXPR_COL,
                        a=(f["price"], 0), pred=(f["day"], "<", 1278), join=(f["key"], d["pk"]))
    _cmp(got, want)
    assert len(want["k0"]) == 75


def _scaled(Q, f, d, load_pct=0, strategy=0, fd=None, dk=None):
    Key, Op = Q.Key, Q.Operand
    fd = {k: dev(v) for k, v in f.items()} if fd is None else fd
    dk = dev(d["orderkey"]) if dk is None else dk
    return Q.GroupbyQuery(len(f["orderkey"]), keys=[Key(fd["returnflag"], 0, 3), Key(fd["linestatus"], 0, 2)],
                          expr=L().EXPR_MUL_CONST_SUB, a=Op(fd["extprice"]), b=Op(fd["discount"]), k=100,
                          pred=(fd["shipday"], "<=", 2450), join=(dk, fd["orderkey"], True, load_pct),
                          strategy=strategy)


def _scaled_oracle(f, d):
    return oracle.query(len(f["orderkey"]), keys=[(f["returnflag"], 0), (f["linestatus"], 0)],
                        expr=oracle.EXPR_MUL_CONST_SUB, a=(f["extprice"], 0), b=(f["discount"], 0), K=100,
                        pred=(f["shipday"], "<=", 2450), join=(f["orderkey"], d["orderkey"]))


@pytest.mark.parametrize("zipf", [None, 1.1])
@pytest.mark.parametrize("load_pct", [0, 85])
def test_scaled_query_reduced(zipf, load_pct):
    f, d = gen.scaled_query_tables(n_fact=2_000_003, n_dim=500_000, zipf_s=zipf)
    say("scaled query reduced", zipf, load_pct)
    _cmp(_scaled(q(), f, d, load_pct)(), _scaled_oracle(f, d))


@pytest.mark.parametrize("zipf", [None, 1.1])
def test_scaled_query_full_size(zipf):
    f, d = gen.scaled_query_tables(zipf_s=zipf)
    fd = {k: dev(v) for k, v in f.items()}
    dk = dev(d["orderkey"])
    want = _scaled_oracle(f, d)
    # the strategy AUTO picks (the fused probe), and the partitioned probe
    for strategy in (L().PROBE_AUTO, L().PROBE_DIRECT, L().PROBE_PARTITIONED):
        say("scaled query full", zipf, "strategy", strategy)
        got = _scaled(q(), f, d, strategy=strategy, fd=fd, dk=dk)()
        _cmp(got, want)
        # invariant: every filtered row finds its key, so counts add up to the filter count
        assert int(host(got["count"]).sum()) == int(np.count_nonzero(f["shipday"] <= 2450))


def test_query_golden_and_edges():
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tiny_query.json")))
    Q = q()
    f = {k: np.array(v) for k, v in g["fact"].items()}
    fd = {"key": dev(f["key"].astype(np.int32)), "price": dev(f["price"].astype(np.int64)),
          "day": dev(f["day"].astype(np.int32)), "flag": dev(f["flag"].astype(np.int8))}
    pk = dev(np.array(g["dim"]["pk"], np.int32))
    region = dev(np.array(g["dim"]["region"], np.int8))
    r = Q.GroupbyQuery(8, keys=[Q.Key(region, 0, 10, L().BUILD), Q.Key(fd["flag"], 0, 3)], expr=L().EXPR_COL,
                       a=Q.Operand(fd["price"]), pred=(fd["day"], "<", 10), join=(pk, fd["key"], True))()
    e = g["expected"]
    assert host(r["k0"]).tolist() == e["region"] and host(r["k1"]).tolist() == e["flag"]
    assert host(r["sum"]).tolist() == e["sum"] and host(r["count"]).tolist() == e["count"]
    assert host(r["avg"]).tolist() == e["avg"]
    # empty probe side
    z = dev(np.zeros(0, np.int32))
    r = Q.GroupbyQuery(0, keys=[Q.Key(z, 0, 5)], expr=L().EXPR_NONE)()
    assert r["k0"].numel() == 0
    # one group, int64 wrap
    w = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "int64_wrap.json")))
    v = dev(np.array(w["values"], np.int64))
    r = Q.GroupbyQuery(3, keys=[Q.Key(dev(np.zeros(3, np.int32)), 0, 1)], expr=L().EXPR_COL, a=Q.Operand(v))()
    assert host(r["sum"]).tolist() == [w["expected_sum"]] and host(r["count"]).tolist() == [3]
    # key outside its declared domain raises the device flag
    with pytest.raises(L().TdpError, match="KEY_DOMAIN"):
        Q.GroupbyQuery(4, keys=[Q.Key(dev(np.array([0, 1, 5, 2], np.int32)), 0, 4)], expr=L().EXPR_NONE)()


@pytest.mark.parametrize("G", [1, 7, 8, 9, 100, 2048, 2049, 5000, 100_000])
def test_groupby_accumulator_modes(G):
    """Register, LDS and global accumulators and both finalize paths agree
    with the oracle (no join, selection vector on odd G)."""
    rng = np.random.default_rng(G)
    n = 300_001
    k = rng.integers(-3, G - 3, n).astype(np.int32)
    v = rng.integers(-2**40, 2**40, n).astype(np.int64)
    Q = q()
    sel = None
    if G % 2:
        sel_h = oracle.filter(v, ">", -2**39)
        sel = dev(sel_h)
    say("groupby modes", G)
    got = Q.GroupbyQuery(n, keys=[Q.Key(dev(k), -3, G)], expr=L().EXPR_COL, a=Q.Operand(dev(v)), sel=sel)()
    if sel is None:
        want = oracle.query(n, keys=[(k, 0)], expr=oracle.EXPR_COL, a=(v, 0))
    else:
        want = oracle.query(len(sel_h), keys=[(k[sel_h], 0)], expr=oracle.EXPR_COL, a=(v[sel_h], 0))
    _cmp(got, want, keys=1)


@pytest.mark.parametrize("G,join,topk", [(3000, "none", 0), (70_000, "keys", 0), (1_000_000, "agg", 0),
                                         (1_000_000, "none", 25), (65_536, "rowid", 0)])
def test_partitioned_aggregation(G, join, topk):
    """Dense tables beyond LDS over more than 2^20 rows aggregate through
    group-range partitions (histogram, LDS-sorted records, per-partition LDS
    reduce).  Two-key groups, a predicate, keys outside their domain (rows
    dropped, flag checked separately), rows without a join partner, ragged
    partition and row counts; the forced single-kernel path must agree."""
    rng = np.random.default_rng(G + len(join))
    n = (1 << 20) + 12_345
    c1 = 5
    g = rng.integers(0, G, n)
    k0 = (g // c1).astype(np.int32)
    k1 = (g % c1).astype(np.int32)
    v = rng.integers(-2**40, 2**40, n).astype(np.int64)
    day = rng.integers(0, 100, n).astype(np.int32)
    Q = q()
    kw = dict(keys=[Q.Key(dev(k0), 0, -(-G // c1)), Q.Key(dev(k1), 0, c1)], expr=L().EXPR_COL, a=Q.Operand(dev(v)),
              pred=(dev(day), "<", 80), topk=topk)
    okw = dict(keys=[(k0, 0), (k1, 0)], expr=oracle.EXPR_COL, a=(v, 0), pred=(day, "<", 80))
    if join != "none":
        nb = 50_000
        bk = gen.scattered_keys(nb)
        pk = bk[rng.integers(0, nb, n)]
        pk[::7] = 777  # absent from the build side
        if join == "agg":
            bk = np.concatenate([bk, bk[:20_000]])  # duplicates: pre-aggregated build side
        kw["join"] = (dev(bk), dev(pk), join != "agg")
        okw["join"] = (pk, bk)
        if join == "rowid":  # a build-side operand makes the join return build rows
            bpay = rng.integers(-1000, 1000, len(bk)).astype(np.int64)
            kw.update(expr=L().EXPR_MUL, b=Q.Operand(dev(bpay), L().BUILD))
            okw.update(expr=oracle.EXPR_MUL, b=(bpay, 1))
    say("partitioned aggregation", G, join, topk)
    got = Q.GroupbyQuery(n, strategy=L().PROBE_AUTO, **kw)()
    want = oracle.query(n, **okw)
    _cmp(got, _topk_ref2(want, topk) if topk else want, keys=2)
    direct = Q.GroupbyQuery(n, strategy=L().PROBE_DIRECT, **kw)()
    for key in ("k0", "k1", "sum", "count", "avg"):
        assert torch.equal(direct[key], got[key])


@pytest.mark.parametrize("nb", [70_000, 300_000])
def test_row_id_lds_build(nb):
    """A unique build side large enough for the LDS build of a row-id table
    (the join then reads a build-side operand): bucketed keys and row ids,
    probe keys absent from the build, a group key from the build side, and a
    duplicated build key raising DUP_BUILD."""
    rng = np.random.default_rng(nb)
    n = 500_003
    bk = gen.scattered_keys(nb)[gen.permutation(gen.stream_seed(5, nb), nb)]
    bpay = rng.integers(-10**6, 10**6, nb).astype(np.int64)
    breg = rng.integers(0, 7, nb).astype(np.int8)
    pk = bk[rng.integers(0, nb, n)]
    pk[::11] = 12345  # absent from the build side
    a = rng.integers(-1000, 1000, n).astype(np.int64)
    flag = rng.integers(0, 3, n).astype(np.int8)
    Q = q()
    say("row-id LDS build", nb)
    got = Q.GroupbyQuery(n, keys=[Q.Key(dev(breg), 0, 7, L().BUILD), Q.Key(dev(flag), 0, 3)], expr=L().EXPR_MUL,
                         a=Q.Operand(dev(a)), b=Q.Operand(dev(bpay), L().BUILD), join=(dev(bk), dev(pk), True))()
    want = oracle.query(n, keys=[(breg, 1), (flag, 0)], expr=oracle.EXPR_MUL, a=(a, 0), b=(bpay, 1), join=(pk, bk))
    _cmp(got, want, keys=2)
    dup = bk.copy()
    dup[nb // 2] = dup[7]
    with pytest.raises(L().TdpError, match="DUP_BUILD"):
        Q.GroupbyQuery(n, keys=[Q.Key(dev(breg), 0, 7, L().BUILD)], expr=L().EXPR_COL, a=Q.Operand(dev(a)),
                       join=(dev(dup), dev(pk), True))()


def _topk_ref2(want, k):
    idx = oracle.topk(want["k0"] * 5 + want["k1"], want["sum"], k)
    return {key: want[key][idx] for key in ("k0", "k1", "sum", "count", "avg")}


def test_partitioned_aggregation_key_domain_flag():
    n = (1 << 20) + 3
    k = np.arange(n, dtype=np.int32) % 10_000
    k[123_457] = 10_000  # outside [0, 10000)
    Q = q()
    with pytest.raises(RuntimeError, match="KEY_DOMAIN"):
        Q.GroupbyQuery(n, keys=[Q.Key(dev(k), 0, 10_000)], expr=L().EXPR_NONE)()


@pytest.mark.parametrize("n_right,max_distinct", [(200_000, 0), (200_000, 20_000), (60_000, 0)])
def test_many_to_many_join_aggregate_reduced(n_right, max_distinct):
    """Pre-aggregated build side: LDS block build (table sized by the build
    rows or by the distinct-key bound) and the atomic build (small side)."""
    l, r = gen.mn_join_tables(n_left=200_000, n_right=n_right, n_keys=20_000, n_groups=10_000)
    Q = q()
    ld = {k: dev(v) for k, v in l.items()}
    rd = {k: dev(v) for k, v in r.items()}
    say("M:N join aggregate reduced", n_right, max_distinct)
    got = Q.GroupbyQuery(len(l["key"]), keys=[Q.Key(ld["gkey"], 0, 10_000)], expr=L().EXPR_MUL,
                         a=Q.Operand(ld["payload"]), b=Q.Operand(rd["payload"], L().BUILD),
                         join=(rd["key"], ld["key"], False, 0, max_distinct))()
    want = oracle.query(len(l["key"]), keys=[(l["gkey"], 0)], expr=oracle.EXPR_MUL, a=(l["payload"], 0),
                        b=(r["payload"], 1), join=(l["key"], r["key"]))
    _cmp(got, want, keys=1)
    # COUNT only and a*(k-b) forms through the same pre-aggregated build side
    got = Q.GroupbyQuery(len(l["key"]), keys=[Q.Key(ld["gkey"], 0, 10_000)], expr=L().EXPR_MUL_CONST_SUB,
                         a=Q.Operand(ld["payload"]), b=Q.Operand(rd["payload"], L().BUILD), k=1 << 20,
                         join=(rd["key"], ld["key"], False, 0, max_distinct))()
    want = oracle.query(len(l["key"]), keys=[(l["gkey"], 0)], expr=oracle.EXPR_MUL_CONST_SUB, a=(l["payload"], 0),
                        b=(r["payload"], 1), K=1 << 20, join=(l["key"], r["key"]))
    _cmp(got, want, keys=1)


@pytest.mark.parametrize("with_sum,max_distinct", [(False, 0), (True, 0), (True, 100_003)])
def test_many_to_many_lds_build_skew_and_extremes(with_sum, max_distinct):
    """LDS block build of a pre-aggregated side: one key on 40% of the build
    rows (folded per wave), the int32 extremes as keys (INT32_MIN is the
    table's empty marker and lives in the extra slot), a ragged block tail."""
    rng = np.random.default_rng(11 + 2 * with_sum + (max_distinct > 0))
    lo, hi = np.iinfo(np.int32).min, np.iinfo(np.int32).max
    nb, npr = 300_001, 250_003
    bkey = rng.integers(-50_000, 50_000, nb).astype(np.int32)
    bkey[:120_000] = 77
    bkey[120_000:120_500] = lo
    bkey[120_500:121_000] = hi
    rng.shuffle(bkey)
    bval = rng.integers(-2**40, 2**40, nb).astype(np.int64)
    pkey = rng.integers(-50_000, 50_000, npr).astype(np.int32)
    pkey[::997] = 77
    pkey[1::1009] = lo
    pkey[2::1013] = hi
    grp = rng.integers(0, 300, npr).astype(np.int32)
    pval = rng.integers(-1000, 1000, npr).astype(np.int64)
    Q = q()
    say("M:N LDS build", with_sum, max_distinct)
    if with_sum:
        got = Q.GroupbyQuery(npr, keys=[Q.Key(dev(grp), 0, 300)], expr=L().EXPR_MUL, a=Q.Operand(dev(pval)),
                             b=Q.Operand(dev(bval), L().BUILD), join=(dev(bkey), dev(pkey), False, 0, max_distinct))()
        want = oracle.query(npr, keys=[(grp, 0)], expr=oracle.EXPR_MUL, a=(pval, 0), b=(bval, 1), join=(pkey, bkey))
    else:
        got = Q.GroupbyQuery(npr, keys=[Q.Key(dev(grp), 0, 300)], expr=L().EXPR_COL, a=Q.Operand(dev(pval)),
                             join=(dev(bkey), dev(pkey), False, 0, max_distinct))()
        want = oracle.query(npr, keys=[(grp, 0)], expr=oracle.EXPR_COL, a=(pval, 0), join=(pkey, bkey))
    _cmp(got, want, keys=1)


def test_max_distinct_too_small_raises_table_full():
    rng = np.random.default_rng(5)
    bkey = rng.permutation(200_000).astype(np.int32)
    pkey = rng.integers(0, 200_000, 100_000).astype(np.int32)
    grp = np.zeros(100_000, np.int32)
    Q = q()
    say("table full flag")
    with pytest.raises(RuntimeError, match="TABLE_FULL|table full"):
        Q.GroupbyQuery(100_000, keys=[Q.Key(dev(grp), 0, 1)], expr=L().EXPR_NONE,
                       join=(dev(bkey), dev(pkey), False, 0, 5000))()


def test_skewed_aggregate_build_over_its_bound_raises_table_full():
    # a pre-aggregated build side whose table is one 4096-slot block (distinct
    # bound 2000) but whose rows hold 4097 distinct keys, each repeated, so the
    # block's rows run past one build segment into the merge workgroups: some
    # key cannot be placed, and wherever that happens the flag must be raised
    rng = np.random.default_rng(6)
    bkey = rng.permutation(np.repeat(np.arange(4097, dtype=np.int32) * 7919, 25)).astype(np.int32)
    bval = rng.integers(0, 100, bkey.size).astype(np.int64)
    pkey = rng.choice(bkey, 50_000).astype(np.int32)
    grp = np.zeros(50_000, np.int32)
    pval = np.ones(50_000, np.int64)
    Q = q()
    say("aggregate build over its distinct-key bound")
    with pytest.raises(RuntimeError, match="TABLE_FULL|table full"):
        Q.GroupbyQuery(50_000, keys=[Q.Key(dev(grp), 0, 1)], expr=L().EXPR_MUL, a=Q.Operand(dev(pval)),
                       b=Q.Operand(dev(bval), L().BUILD), join=(dev(bkey), dev(pkey), False, 0, 2000))()


# ------------------------------------------------------------------- top-k

def _topk_ref(want, k):
    idx = oracle.topk(want["k0"], want["sum"], k)
    return {key: want[key][idx] for key in ("k0", "sum", "count", "avg")}


@pytest.mark.parametrize("G,k", [(50, 10), (2048, 100), (2049, 100), (300_000, 100), (300_000, 1024), (5, 100)])
def test_groupby_topk_with_ties(G, k):
    rng = np.random.default_rng(G + k)
    n = 400_003
    key = rng.integers(0, G, n).astype(np.int32)
    val = rng.integers(-3, 4, n).astype(np.int64)  # small values: many equal sums, ties broken by key
    Q = q()
    say("topk", G, k)
    got = Q.GroupbyQuery(n, keys=[Q.Key(dev(key), 0, G)], expr=L().EXPR_COL, a=Q.Operand(dev(val)), topk=k)()
    want = _topk_ref(oracle.query(n, keys=[(key, 0)], expr=oracle.EXPR_COL, a=(val, 0)), k)
    _cmp(got, want, keys=1)


def test_many_to_many_topk_reduced():
    l, r = gen.mn_join_tables(n_left=300_000, n_right=300_000, n_keys=30_000, n_groups=20_000)
    Q = q()
    ld = {k: dev(v) for k, v in l.items()}
    rd = {k: dev(v) for k, v in r.items()}
    got = Q.GroupbyQuery(len(l["key"]), keys=[Q.Key(ld["gkey"], 0, 20_000)], expr=L().EXPR_MUL,
                         a=Q.Operand(ld["payload"]), b=Q.Operand(rd["payload"], L().BUILD),
                         join=(rd["key"], ld["key"], False), topk=100)()
    want = oracle.query(len(l["key"]), keys=[(l["gkey"], 0)], expr=oracle.EXPR_MUL, a=(l["payload"], 0),
                        b=(r["payload"], 1), join=(l["key"], r["key"]))
    _cmp(got, _topk_ref(want, 100), keys=1)


@pytest.mark.parametrize("max_distinct", [0, 2_000_000])
def test_many_to_many_full_size_sampled(max_distinct):
    """20M x 20M Zipf(0.8) join aggregated over 1M groups: the join output
    (~1.2e11 pairs) is never materialised.  Every group is checked bit-exactly
    against the stored digest of the oracle's enumeration of all pairs
    (tests/golden/make_mn_digest.py); on top of that, exact per-group
    enumeration on a sample (and on the top 100), the top-100 against the
    full table, and closed-form totals."""
    l, r = gen.mn_join_tables()
    Q = q()
    ld = {k: dev(v) for k, v in l.items()}
    rd = {k: dev(v) for k, v in r.items()}
    say("M:N full size", max_distinct)
    mk = lambda topk: Q.GroupbyQuery(len(l["key"]), keys=[Q.Key(ld["gkey"], 0, 1_000_000)], expr=L().EXPR_MUL,
                                     a=Q.Operand(ld["payload"]), b=Q.Operand(rd["payload"], L().BUILD),
                                     join=(rd["key"], ld["key"], False, 0, max_distinct), topk=topk)
    full = {k: host(v) for k, v in mk(0)().items()}
    top = {k: host(v) for k, v in mk(100)().items()}
    # top-100 is the first 100 of the full table ranked by (SUM desc, key asc)
    idx = oracle.topk(full["k0"], full["sum"], 100)
    for key in ("k0", "sum", "count"):
        assert np.array_equal(top[key], full[key][idx])
    # closed forms: COUNT = sum_l cntR(key_l); SUM = sum_l p_l * sumR(key_l)  (mod 2^64)
    cnt_r = np.bincount(r["key"], minlength=2_000_000).astype(np.int64)
    sum_r = np.zeros(2_000_000, np.uint64)
    np.add.at(sum_r, r["key"], r["payload"].astype(np.uint64))
    assert int(full["count"].sum()) == int(cnt_r[l["key"]].sum())
    with np.errstate(over="ignore"):
        tot = (l["payload"].astype(np.uint64) * sum_r[l["key"]]).sum(dtype=np.uint64)
        assert full["sum"].astype(np.uint64).sum(dtype=np.uint64) == tot
    # every group against the digest of the oracle's full pair enumeration
    with open(os.path.join(GOLDEN, "mn_full_digest.json")) as f:
        dg = json.load(f)
    o = np.argsort(full["k0"], kind="stable")
    k0, sums, counts = (np.asarray(full[k], np.int64)[o] for k in ("k0", "sum", "count"))
    assert len(k0) == dg["groups"] and int(counts.sum()) == dg["count_total"]
    assert int(sums.astype(np.uint64).sum(dtype=np.uint64)) == dg["sum_total_mod_2_64"]
    canon = np.ascontiguousarray(np.stack([k0, sums, counts], axis=1)).astype("<i8").tobytes()
    assert hashlib.sha256(canon).hexdigest() == dg["sha256"]
    assert [[int(top["k0"][i]), int(top["sum"][i]), int(top["count"][i])] for i in range(100)] == dg["top100"]
    # exact enumeration of sampled groups and of the top 100
    mo = oracle.MNGroupOracle(l["key"], l["gkey"], l["payload"], r["key"], r["payload"])
    pos = {int(g): i for i, g in enumerate(full["k0"])}
    sample = np.random.default_rng(1).choice(1_000_000, 150, replace=False).tolist() + top["k0"].tolist()
    for g in sample:
        s, c = mo.group(int(g))
        if c == 0:
            assert int(g) not in pos
        else:
            i = pos[int(g)]
            assert (int(full["sum"][i]), int(full["count"][i])) == (s, c)


@pytest.mark.parametrize("G,topk", [(6, 0), (1000, 0), (60_000, 0), (60_000, 50)])
def test_staged_probe_accumulators(G, topk):
    """Large keys-only join through the partitioned, XCD-aware probe (forced
    by the strategy hint) with every accumulator mode, a generic column
    signature, misses and a ragged tail."""
    rng = np.random.default_rng(G + topk)
    n, nd = 4_200_003, 9_000_000
    pk = gen.scattered_keys(nd)
    fk = pk[rng.integers(0, nd, n)]
    fk[::11] = 12345  # mostly absent from the build side
    grp = rng.integers(0, G, n).astype(np.int32)
    val = rng.integers(-2**40, 2**40, n).astype(np.int64)
    day = rng.integers(0, 100, n).astype(np.int16).astype(np.int32)
    Q = q()
    say("staged probe", G, topk)
    got = Q.GroupbyQuery(n, keys=[Q.Key(dev(grp), 0, G)], expr=L().EXPR_COL, a=Q.Operand(dev(val)),
                         pred=(dev(day), "<", 90), join=(dev(pk), dev(fk), True), topk=topk,
                         strategy=L().PROBE_STAGED)()
    want = oracle.query(n, keys=[(grp, 0)], expr=oracle.EXPR_COL, a=(val, 0), pred=(day, "<", 90), join=(fk, pk))
    _cmp(got, _topk_ref(want, topk) if topk else want, keys=1)


def test_staged_probe_rejects_wide_group_ids():
    """Staged records hold 16-bit group ids: forcing the staged probe with
    65535 or more groups is refused on the host."""
    n = 100_000
    pk = gen.scattered_keys(70_000)
    Q = q()
    with pytest.raises(RuntimeError, match="status -4"):
        Q.GroupbyQuery(n, keys=[Q.Key(dev(np.zeros(n, np.int32)), 0, 70_000)], expr=L().EXPR_NONE,
                       join=(dev(pk), dev(pk[np.arange(n) % 70_000]), True), strategy=L().PROBE_STAGED)
