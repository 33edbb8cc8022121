"""The radix-partitioned probe (TDP_PROBE_PARTITIONED) against the oracle,
bit-exact: ragged sizes over several partitions and chunks, register and
LDS accumulators, extra conjuncts, Zipf skew (one partition split over
many work items), a partition holding more build keys than one LDS
sub-table, an empty build side, keys absent from the build side, and the
duplicate-key flag."""
import numpy as np
import pytest
import torch

import oracle
import tdp_datagen as gen
from paper_2211_02753_amd import _lib as L
from paper_2211_02753_amd import query as Q

pytestmark = pytest.mark.gpu
DEV = "cuda"


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _cmp(got, want):
    for k in ("k0", "k1", "sum", "count"):
        if k in want:
            assert np.array_equal(got[k].cpu().numpy(), want[k]), k
    assert np.array_equal(got["avg"].cpu().numpy().view(np.uint64), want["avg"].view(np.uint64))


def _fmix32(h):
    """murmur3's 32-bit finaliser on a uint32 numpy array (the partitioning
    hash; the test uses it only to build a skewed build side)."""
    h = h.astype(np.uint64)
    m = np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(16)
    h = (h * np.uint64(0x85EBCA6B)) & m
    h ^= h >> np.uint64(13)
    h = (h * np.uint64(0xC2B2AE35)) & m
    h ^= h >> np.uint64(16)
    return h.astype(np.uint32)


def _scaled_q(f, d, strategy, preds=None, keys=None):
    fd = {k: t(v) for k, v in f.items()}
    keys = keys or [Q.Key(fd["returnflag"], 0, 3), Q.Key(fd["linestatus"], 0, 2)]
    return Q.GroupbyQuery(len(f["orderkey"]), keys=keys, expr=L.EXPR_MUL_CONST_SUB, a=Q.Operand(fd["extprice"]),
                          b=Q.Operand(fd["discount"]), k=100,
                          pred=preds(fd) if preds else (fd["shipday"], "<=", 2450),
                          join=(t(d["orderkey"]), fd["orderkey"], True), strategy=strategy)


def _scaled_o(f, d, preds=None, keys=None):
    return oracle.query(len(f["orderkey"]), keys=keys or [(f["returnflag"], 0), (f["linestatus"], 0)],
                        expr=oracle.EXPR_MUL_CONST_SUB, a=(f["extprice"], 0), b=(f["discount"], 0), K=100,
                        pred=preds(f) if preds else (f["shipday"], "<=", 2450), join=(f["orderkey"], d["orderkey"]))


@pytest.mark.parametrize("n_fact,n_dim,zipf", [(1, 5, None), (8191, 3000, None), (1_000_003, 700_001, None),
                                               (2_500_007, 4_300_001, None), (3_000_001, 500_000, 1.1)])
def test_partitioned_probe_matches_oracle(n_fact, n_dim, zipf):
    f, d = gen.scaled_query_tables(n_fact=n_fact, n_dim=n_dim, zipf_s=zipf)
    print(f"partitioned probe {n_fact} x {n_dim} zipf={zipf}", flush=True)
    _cmp(_scaled_q(f, d, L.PROBE_PARTITIONED)(), _scaled_o(f, d))


def test_partitioned_probe_lds_accumulators_conjuncts_and_misses():
    f, d = gen.scaled_query_tables(n_fact=1_200_001, n_dim=300_000)
    # a third of the fact keys miss the build side
    f["orderkey"] = f["orderkey"].copy()
    absent = gen.scattered_keys(400_000)[300_000:]   # keys the build side does not hold
    f["orderkey"][::3] = np.resize(absent, len(f["orderkey"][::3]))
    preds = lambda c: [(c["shipday"], "<", 200), (c["discount"], ">=", 2), (c["extprice"], "!=", 100_000)]
    keys_d = lambda c: [Q.Key(c["shipday"], 0, 200)]
    fd = {k: t(v) for k, v in f.items()}
    got = Q.GroupbyQuery(len(f["orderkey"]), keys=keys_d(fd), expr=L.EXPR_MUL_CONST_SUB,
                         a=Q.Operand(fd["extprice"]), b=Q.Operand(fd["discount"]), k=100, pred=preds(fd),
                         join=(t(d["orderkey"]), fd["orderkey"], True), strategy=L.PROBE_PARTITIONED)()
    want = _scaled_o(f, d, preds, [(f["shipday"], 0)])
    print("partitioned probe: 200 groups, LDS accumulators", flush=True)
    _cmp(got, want)
    assert int(want["count"].sum()) < int(np.count_nonzero(f["shipday"] < 200))  # misses really missed


def test_partitioned_probe_oversized_partition_and_empty_build():
    # 40,000 build keys whose hash lands in partition 0 of 64 (more than one
    # LDS sub-table of 30,720 tags) plus 10,000 others
    cand = np.arange(0, 1 << 24, dtype=np.uint32)
    top = _fmix32(cand) >> np.uint32(26)
    hot = cand[top == 0][:40_000].astype(np.int32)
    cold = cand[top != 0][:10_000].astype(np.int32)
    pk = np.concatenate([hot, cold])
    rng = np.random.default_rng(1)
    pk = pk[rng.permutation(len(pk))]
    n = 300_001
    fk = pk[rng.integers(0, len(pk), n)].astype(np.int32)
    fk[::5] = -7  # absent
    gk = rng.integers(0, 5, n).astype(np.int8)
    val = rng.integers(-10**12, 10**12, n).astype(np.int64)
    got = Q.GroupbyQuery(n, [Q.Key(t(gk), 0, 5)], expr=L.EXPR_COL, a=Q.Operand(t(val)),
                         join=(t(pk), t(fk), True), strategy=L.PROBE_PARTITIONED)()
    want = oracle.query(n, keys=[(gk, 0)], expr=oracle.EXPR_COL, a=(val, 0), join=(fk, pk))
    print("partitioned probe: two sub-tables in one partition", flush=True)
    _cmp(got, want)
    # empty build side: no row joins
    got = Q.GroupbyQuery(n, [Q.Key(t(gk), 0, 5)], expr=L.EXPR_COL, a=Q.Operand(t(val)),
                         join=(t(np.zeros(0, np.int32)), t(fk), True), strategy=L.PROBE_PARTITIONED)()
    assert int(got["count"].numel()) == 0


def test_partitioned_probe_duplicate_build_key_flag_and_refusals():
    f, d = gen.scaled_query_tables(n_fact=100_000, n_dim=50_000)
    d["orderkey"] = d["orderkey"].copy()
    d["orderkey"][7] = d["orderkey"][40_000]
    with pytest.raises(L.TdpError, match="DUP_BUILD"):
        _scaled_q(f, d, L.PROBE_PARTITIONED)()
    # a selection vector has no partitioned form
    fd = {k: t(v) for k, v in f.items()}
    with pytest.raises(L.TdpError):
        Q.GroupbyQuery(len(f["orderkey"]), keys=[Q.Key(fd["returnflag"], 0, 3)], sel=t(np.arange(10, dtype=np.int32)),
                       join=(t(d["orderkey"]), fd["orderkey"], True), strategy=L.PROBE_PARTITIONED)()


def test_auto_takes_the_partitioned_probe_for_large_keys_only_joins():
    """AUTO routes a keys-only join of 2^22 probe rows with more than 2^18
    build keys to the partitioned probe (its scatter kernel runs), DIRECT to
    the fused kernel, both equal to the oracle bit for bit; with fewer build
    keys AUTO keeps the fused kernel."""
    n = (1 << 22) + 12_345
    f, d = gen.scaled_query_tables(n_fact=n, n_dim=(1 << 22) + 77)
    want = _scaled_o(f, d)
    for strategy, stage in ((L.PROBE_AUTO, L.STAGE_RP_SCATTER), (L.PROBE_DIRECT, L.STAGE_FUSED_PROBE)):
        q = _scaled_q(f, d, strategy)
        L.stage_timer(stage)
        got = q()
        torch.cuda.synchronize()
        ms, launches = L.stage_time()
        L.stage_timer(L.STAGE_NONE)
        print(f"strategy {strategy}: stage {stage} launches {launches}, {ms:.3f} ms", flush=True)
        assert launches >= 1
        _cmp(got, want)
    # under DIRECT the partitioned scatter never runs
    q = _scaled_q(f, d, L.PROBE_DIRECT)
    L.stage_timer(L.STAGE_RP_SCATTER)
    q()
    torch.cuda.synchronize()
    assert L.stage_time()[1] == 0
    L.stage_timer(L.STAGE_NONE)
    # below 2^18 build keys AUTO keeps the fused kernel
    f2, d2 = gen.scaled_query_tables(n_fact=n, n_dim=(1 << 18) - 1000)
    q = _scaled_q(f2, d2, L.PROBE_AUTO)
    L.stage_timer(L.STAGE_RP_SCATTER)
    got = q()
    torch.cuda.synchronize()
    assert L.stage_time()[1] == 0
    L.stage_timer(L.STAGE_NONE)
    _cmp(got, _scaled_o(f2, d2))
