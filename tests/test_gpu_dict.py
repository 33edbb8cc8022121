"""Dictionary-encoded string columns on the GPU: the dictionary and the codes
bit-exact against the oracle, lookup and decode, and the codes as keys of
the exact filter, join and group-by against the oracle's query over the
oracle's codes."""
import numpy as np
import pytest
import torch

import oracle
import tdp_datagen as gen
from paper_2211_02753_amd import _lib as L
from paper_2211_02753_amd import dictenc
from paper_2211_02753_amd import query as Q

pytestmark = pytest.mark.gpu
DEV = "cuda"


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("n,nd,width", [(1, 1, 4), (1000, 37, 8), (1_000_003, 50_000, 16), (300_001, 150_000, 32)])
def test_dictionary_build_matches_oracle(n, nd, width):
    rows, _ = gen.string_column(n, nd, width)
    print(f"dictionary n={n} distinct={nd} width={width}", flush=True)
    d, codes = dictenc.encode(t(rows), max_distinct=nd)
    wd, wc = oracle.dict_build(rows)
    assert np.array_equal(d.cpu().numpy(), wd)
    assert np.array_equal(codes.cpu().numpy(), wc)
    assert np.array_equal(dictenc.decode(d, codes).cpu().numpy(), rows)


def test_dictionary_edges_lookup_and_capacity_flag():
    # empty strings, full-width strings, a single distinct string
    words = [b"", b"abcdefgh", b"", b"abcdefgh", b"abcdefg", b"b"]
    rows = dictenc.pad(words, 8).numpy()
    d, codes = dictenc.encode(t(rows))
    wd, wc = oracle.dict_build(rows)
    assert np.array_equal(d.cpu().numpy(), wd) and np.array_equal(codes.cpu().numpy(), wc)
    same = dictenc.pad([b"same"] * 5000, 4).numpy()
    d1, c1 = dictenc.encode(t(same), max_distinct=1)
    assert d1.shape[0] == 1 and int(c1.max()) == 0
    # lookup of present and absent strings
    probe = dictenc.pad([b"", b"a", b"abcdefg", b"abcdefgh", b"abcdefgi", b"zzzz"], 8).numpy()
    pos, found = dictenc.lookup(d, t(probe))
    wp, wf = oracle.dict_lookup(wd, probe)
    assert np.array_equal(pos.cpu().numpy(), wp) and np.array_equal(found.cpu().numpy(), wf)
    # more distinct strings than the bound: the flag
    rows2, _ = gen.string_column(20_000, 5000, 8)
    with pytest.raises(L.TdpError, match="TABLE_FULL"):
        dictenc.encode(t(rows2), max_distinct=1000)


def test_codes_as_keys_of_filter_join_and_groupby():
    """SELECT city, SUM(amount), COUNT(*) FROM sales JOIN stores ON sales.store = stores.store
    WHERE city >= 'm' GROUP BY city, with city and store names dictionary-encoded."""
    rng = np.random.default_rng(4)
    n = 400_003
    store_names, _ = gen.string_column(3000, 3000, 12, seed=gen.SEED_STR + 1)
    store_names = np.unique(store_names.view("S12").ravel()).view(np.uint8).reshape(-1, 12)
    cities, _ = gen.string_column(len(store_names), 120, 8, seed=gen.SEED_STR + 2)
    pick = rng.integers(0, len(store_names) + 200, n)   # some sales name stores that do not exist
    others, _ = gen.string_column(200, 200, 12, seed=gen.SEED_STR + 3)
    sale_store = np.where(pick[:, None] < len(store_names), store_names[np.minimum(pick, len(store_names) - 1)],
                          others[np.maximum(pick - len(store_names), 0) % len(others)])
    amount = rng.integers(1, 10_000, n).astype(np.int64)
    # encode: store names through the stores' dictionary, sales looked up in it
    sd, scode = dictenc.encode(t(store_names))
    spos, sfound = dictenc.lookup(sd, t(sale_store))
    sale_code = torch.where(sfound.bool(), spos, torch.full_like(spos, -1)).contiguous()
    cd, ccode = dictenc.encode(t(cities))
    op, lit = dictenc.literal_predicate(cd, ">=", b"m")
    # city per sale comes from the store (build side), so the filter applies after the join:
    # express it as a filter on the build side's city codes, then the join and group-by
    keep = Q.filter(ccode, op, lit)
    build_keys = scode[keep.long()].contiguous()
    build_city = ccode[keep.long()].contiguous()
    got = Q.GroupbyQuery(n, [Q.Key(build_city, 0, cd.shape[0], L.BUILD)], expr=L.EXPR_COL, a=Q.Operand(t(amount)),
                         join=(build_keys, sale_code, True))()
    # oracle: the same query over the oracle's codes, then keys decoded to strings
    od_s, oc_s = oracle.dict_build(store_names)
    od_c, oc_c = oracle.dict_build(cities)
    opos, ofound = oracle.dict_lookup(od_s, sale_store)
    osale = np.where(ofound == 1, opos, -1).astype(np.int32)
    city_str = [bytes(r).rstrip(b"\0") for r in cities]
    kept = np.array([i for i, c in enumerate(city_str) if c >= b"m"], np.int32)
    want = oracle.query(n, keys=[(oc_c[kept], 1)], expr=oracle.EXPR_COL, a=(amount, 0),
                        join=(osale, oc_s[kept].astype(np.int32)))
    assert np.array_equal(got["k0"].cpu().numpy(), want["k0"])
    assert np.array_equal(got["sum"].cpu().numpy(), want["sum"])
    assert np.array_equal(got["count"].cpu().numpy(), want["count"])
    names = dictenc.decode(cd, got["k0"].to(torch.int32).contiguous()).cpu().numpy()
    assert all(bytes(r).rstrip(b"\0") >= b"m" for r in names)
    assert np.array_equal(names, od_c[want["k0"]])
