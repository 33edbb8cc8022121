"""Seeded synthetic inputs for the exact query, the soft query and the image column.

This module is shared by the HIP path's tests/benchmark and by the CPU oracle's
tests.  It holds only random-number generation and table shaping: no filter,
join, aggregation, relaxation or network arithmetic lives here.

Every random column is a counter-based SplitMix64 stream (Steele, Lea & Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014): element ``i`` of
a stream with seed ``s`` is ``mix64(s + (i + 1) * GAMMA)`` (all arithmetic mod
2**64), which is the state of SplitMix64 after ``i + 1`` steps, so any element
can be produced independently of the others.

Derived draws:
  * integers uniform in ``[lo, hi]`` (inclusive): Lemire's multiply-shift on the
    top 32 bits, ``lo + ((z >> 32) * (hi - lo + 1)) >> 32`` (no rejection; the
    bias is below 2**-32 relative and the map is deterministic);
  * ``U(0,1)`` float32 from the top 24 bits;
  * ``N(0,1)`` by Box-Muller in float64 from two streams, rounded to float32;
  * bounded Zipf ranks (``P(k) ~ k**-s``, ``k = 1..N``) by binary search of the
    float64 CDF with a 53-bit uniform;
  * seeded permutations as the argsort of one stream (ties broken by index).
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_COL = np.uint64(0xD1B54A32D192ED03)

# Base seeds of the workloads (exact small query, exact scaled query, skewed
# many-to-many join, soft query, image column, probability-encoded tile
# columns).  Skew variants add 0x100.
SEED_SMALL, SEED_SCALED, SEED_MN, SEED_SOFT, SEED_IMAGES, SEED_PE = (0x7D0D0000 + i for i in range(1, 7))
SKEW_OFFSET = 0x100

_CHUNK = 1 << 22
_THREADS = 8


def _parallel_chunks(n, fn):
    """Run fn(lo, hi) over [0, n) in chunks on a small thread pool (numpy
    releases the GIL inside its kernels, so chunks run concurrently)."""
    spans = [(lo, min(n, lo + _CHUNK)) for lo in range(0, n, _CHUNK)]
    if len(spans) <= 1:
        for lo, hi in spans:
            fn(lo, hi)
        return
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=_THREADS) as ex:
        list(ex.map(lambda s: fn(*s), spans))


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (the variant-13 finaliser) on uint64 arrays."""
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_seed(base: int, column: int) -> np.uint64:
    """Seed of column ``column`` of a workload with base seed ``base``."""
    with np.errstate(over="ignore"):
        s = np.array([base], dtype=np.uint64) + np.uint64(column) * _COL
    return np.uint64(mix64(s)[0])


def draws(seed: np.uint64, n: int, start: int = 0) -> np.ndarray:
    """Raw 64-bit draws ``start .. start+n-1`` of the stream ``seed``."""
    out = np.empty(n, dtype=np.uint64)

    def fill(lo, hi):
        ctr = np.arange(start + lo + 1, start + hi + 1, dtype=np.uint64)
        out[lo:hi] = mix64(np.uint64(seed) + ctr * GAMMA)

    _parallel_chunks(n, fill)
    return out


def uniform_int(seed, n, lo, hi, dtype=np.int64, start=0):
    """Integers uniform in the inclusive range ``[lo, hi]`` (``hi - lo < 2**32``)."""
    span = int(hi) - int(lo) + 1
    assert 0 < span <= (1 << 32)
    out = np.empty(n, dtype=dtype)

    def fill(a, b):
        ctr = np.arange(start + a + 1, start + b + 1, dtype=np.uint64)
        z = mix64(np.uint64(seed) + ctr * GAMMA)
        r = ((z >> np.uint64(32)) * np.uint64(span)) >> np.uint64(32)
        out[a:b] = (r.astype(np.int64) + int(lo)).astype(dtype)

    _parallel_chunks(n, fill)
    return out


def uniform01_f32(seed, n, start=0):
    """Float32 uniform in ``[0, 1)`` from the top 24 bits of each draw."""
    z = draws(seed, n, start)
    return ((z >> np.uint64(40)).astype(np.float32) * np.float32(2.0 ** -24)).astype(np.float32)


def _uniform01_f64(seed, n, start=0):
    z = draws(seed, n, start)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal_f32(seed_a, seed_b, n):
    """Standard normal float32 by Box-Muller from two independent streams."""
    u1 = 1.0 - _uniform01_f64(seed_a, n)  # in (0, 1]
    u2 = _uniform01_f64(seed_b, n)
    return (np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)).astype(np.float32)


def permutation(seed, n):
    """A seeded permutation of ``0..n-1`` (argsort of one stream, stable)."""
    return np.argsort(draws(seed, n), kind="stable").astype(np.int64)


def zipf_ranks(seed, n, n_ranks, s):
    """``n`` bounded-Zipf ranks in ``[0, n_ranks)`` (rank 0 is the most frequent)."""
    w = np.arange(1, n_ranks + 1, dtype=np.float64) ** (-float(s))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    out = np.empty(n, dtype=np.int64)

    def fill(a, b):
        ctr = np.arange(a + 1, b + 1, dtype=np.uint64)
        u = (mix64(np.uint64(seed) + ctr * GAMMA) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        out[a:b] = np.minimum(np.searchsorted(cdf, u, side="right"), n_ranks - 1)

    _parallel_chunks(n, fill)
    return out


# ---------------------------------------------------------------------------
# Workload tables.  ``scale`` shrinks row counts for CPU-sized test cases while
# keeping every value distribution.
# ---------------------------------------------------------------------------

def small_query_tables(n_fact=1_000_000, n_dim=10_000, seed=SEED_SMALL):
    """Fact(key i32 U[0,n_dim), price i64 U[100,100000], day i32 U[0,2556), flag i8 U{0,1,2});
    Dim(pk i32 = 0..n_dim-1, region i8 U[0,25))."""
    s = lambda c: stream_seed(seed, c)
    fact = {
        "key": uniform_int(s(0), n_fact, 0, n_dim - 1, np.int32),
        "price": uniform_int(s(1), n_fact, 100, 100_000, np.int64),
        "day": uniform_int(s(2), n_fact, 0, 2555, np.int32),
        "flag": uniform_int(s(3), n_fact, 0, 2, np.int8),
    }
    dim = {
        "pk": np.arange(n_dim, dtype=np.int32),
        "region": uniform_int(s(4), n_dim, 0, 24, np.int8),
    }
    return fact, dim


def scattered_keys(n):
    """``n`` distinct int32 keys: the image of ``0..n-1`` under the bijection
    ``j -> j * 0x9E3779B1 + 0x7F4A7C15 (mod 2**32)``, reinterpreted as signed."""
    j = np.arange(n, dtype=np.uint64)
    u = (j * np.uint64(0x9E3779B1) + np.uint64(0x7F4A7C15)) & np.uint64(0xFFFFFFFF)
    return u.astype(np.uint32).view(np.int32)


def scaled_query_tables(n_fact=60_000_000, n_dim=15_000_000, zipf_s=None, seed=SEED_SCALED):
    """Fact(orderkey i32, extprice i64 U[90000,10500000], discount i64 U[0,10],
    shipday i32 U[0,2556), returnflag i8 U{0,1,2}, linestatus i8 U{0,1});
    Dim(orderkey i32 distinct scattered keys in shuffled order, orderday i32 U[0,2556)).

    Fact orderkeys are dim keys picked uniformly, or by Zipf(``zipf_s``) rank
    over a seeded permutation of the dim rows (so hot keys are not adjacent)."""
    if zipf_s is not None:
        seed = seed + SKEW_OFFSET
    s = lambda c: stream_seed(seed, c)
    pk = scattered_keys(n_dim)[permutation(s(10), n_dim)]
    if zipf_s is None:
        idx = uniform_int(s(0), n_fact, 0, n_dim - 1, np.int64)
    else:
        idx = permutation(s(11), n_dim)[zipf_ranks(s(0), n_fact, n_dim, zipf_s)]
    fact = {
        "orderkey": pk[idx],
        "extprice": uniform_int(s(1), n_fact, 90_000, 10_500_000, np.int64),
        "discount": uniform_int(s(2), n_fact, 0, 10, np.int64),
        "shipday": uniform_int(s(3), n_fact, 0, 2555, np.int32),
        "returnflag": uniform_int(s(4), n_fact, 0, 2, np.int8),
        "linestatus": uniform_int(s(5), n_fact, 0, 1, np.int8),
    }
    dim = {
        "orderkey": pk,
        "orderday": uniform_int(s(6), n_dim, 0, 2555, np.int32),
    }
    return fact, dim


def mn_join_tables(n_left=20_000_000, n_right=20_000_000, n_keys=2_000_000, n_groups=1_000_000,
                   zipf_s=0.8, seed=SEED_MN):
    """Left(key i32 ~ Zipf(s) over n_keys values, gkey i32 U[0,n_groups), payload i64 U[0,2**20));
    Right(key i32 same law from an independent stream, payload i64 U[0,2**20)).
    Rank -> key value through one seeded permutation shared by both sides."""
    s = lambda c: stream_seed(seed, c)
    perm = permutation(s(10), n_keys).astype(np.int32)
    left = {
        "key": perm[zipf_ranks(s(0), n_left, n_keys, zipf_s)],
        "gkey": uniform_int(s(1), n_left, 0, n_groups - 1, np.int32),
        "payload": uniform_int(s(2), n_left, 0, (1 << 20) - 1, np.int64),
    }
    right = {
        "key": perm[zipf_ranks(s(3), n_right, n_keys, zipf_s)],
        "payload": uniform_int(s(4), n_right, 0, (1 << 20) - 1, np.int64),
    }
    return left, right


def soft_query_columns(n=10_000_000, n_groups=1000, seed=SEED_SOFT):
    """x f32 ~ N(0,1), v f32 ~ U(0,1), g i32 ~ U[0,n_groups)."""
    s = lambda c: stream_seed(seed, c)
    return {
        "x": normal_f32(s(0), s(1), n),
        "v": uniform01_f32(s(2), n),
        "g": uniform_int(s(3), n, 0, n_groups - 1, np.int32),
    }


def _prob_rows(seed_a, seed_b, n, k, scale):
    """Float32 rows of k positive entries summing to 1 (up to rounding): the
    normalised exponentials of N(0, scale^2) draws, like a classifier's
    output.  An input shape, drawn once for both sides."""
    z = normal_f32(seed_a, seed_b, n * k).astype(np.float64).reshape(n, k) * scale
    e = np.exp(z - z.max(1, keepdims=True))
    return (e / e.sum(1, keepdims=True)).astype(np.float32)


def pe_grid_columns(n_grids=123_457, tiles=81, k_digit=10, k_size=2, seed=SEED_PE):
    """Probability-encoded columns of a table of image tiles: ``tiles`` rows
    per grid image (9 x 9), p f32 [n][k_digit] and q f32 [n][k_size] peaked
    probability rows, and seg i64 [n_grids + 1] the first row of each grid."""
    n = n_grids * tiles
    s = lambda c: stream_seed(seed, c)
    return {
        "p": _prob_rows(s(0), s(1), n, k_digit, 2.0),
        "q": _prob_rows(s(2), s(3), n, k_size, 2.0),
        "seg": (np.arange(n_grids + 1, dtype=np.int64) * tiles),
    }


SEED_WHERE = 0x7D0D0000 + 0x200


def where_table(n=1_000_000, seed=SEED_WHERE):
    """A table for learning WHERE thresholds from grouped counts: region i8
    U[0,25), flag i8 U{0,1,2}, day i32 uniform on [50 * region,
    50 * region + 2000) and qty i32 uniform on [1, 30 + 15 * flag] (each
    column's range depends on one group key, so the ratios of the counts per
    (region, flag) identify a threshold on each; the range ends lie away from
    thresholds near the middle), price i64 U[100,100000], x f32 N(0,1)."""
    s = lambda c: stream_seed(seed, c)
    region = uniform_int(s(0), n, 0, 24, np.int8)
    flag = uniform_int(s(1), n, 0, 2, np.int8)
    day_lo = 50 * region.astype(np.int64)
    qty_hi = 30 + 15 * flag.astype(np.int64)
    day = (day_lo + np.floor(_uniform01_f64(s(2), n) * 2000)).astype(np.int32)
    qty = (1 + np.floor(_uniform01_f64(s(3), n) * qty_hi)).astype(np.int32)
    return {
        "region": region, "flag": flag, "day": day, "qty": qty,
        "price": uniform_int(s(4), n, 100, 100_000, np.int64),
        "x": normal_f32(s(5), s(6), n),
    }


SEED_LLP = 0x7D0D0000 + 0x300


def tabular_income(n=49_152, F=8, seed=SEED_LLP):
    """A synthetic stand-in for a census-income table: F standard-normal
    features per row (float32, row-major) and a binary label drawn from a
    logistic model over them (a fixed weight vector of this generator, a
    bias giving about three positives in ten, unit logistic noise); rows come
    in a seeded random order."""
    s = lambda c: stream_seed(seed, c)
    X = np.empty((n, F), np.float32)
    for f in range(F):
        X[:, f] = normal_f32(s(2 * f), s(2 * f + 1), n)
    w = np.linspace(1.5, -1.0, F)
    z = X.astype(np.float64) @ w - 1.5
    u = np.clip(_uniform01_f64(s(100), n), 1e-12, 1 - 1e-12)
    y = (z + np.log(u / (1 - u)) > 0).astype(np.int8)   # logistic noise by inversion
    return X, y


def laplace_f32(seed, n, scale):
    """Laplace(0, scale) draws by inversion of a uniform, float32."""
    u = _uniform01_f64(seed, n) - 0.5
    u = np.clip(u, -0.5 + 1e-16, 0.5 - 1e-16)
    return (-scale * np.sign(u) * np.log1p(-2.0 * np.abs(u))).astype(np.float32)


SEED_STR = 0x7D0D0000 + 0x400


def string_column(n=1_000_000, n_distinct=50_000, width=16, seed=SEED_STR):
    """A string column: exactly n_distinct distinct words of 1 .. width
    lowercase letters (seeded; the drawing is repeated with more words until
    enough distinct ones exist, since short words repeat often), each row one
    of them, uniformly; as a zero-padded uint8 [n][width] matrix, plus the
    words' own matrix."""
    s = lambda c: stream_seed(seed, c)
    m = int(n_distinct * 1.25) + 64
    while True:
        lens = uniform_int(s(0), m, 1, width, np.int64)
        letters = uniform_int(s(1), m * width, ord("a"), ord("z"), np.uint8).reshape(m, width)
        letters[np.arange(width)[None, :] >= lens[:, None]] = 0
        words = np.unique(letters.view(f"S{width}").ravel())
        if len(words) >= n_distinct:
            break
        if m > 16 * n_distinct + 1024:
            raise ValueError(f"cannot draw {n_distinct} distinct words of at most {width} letters")
        m *= 2
    order = np.argsort(draws(s(2), len(words)), kind="stable")[:n_distinct]
    wmat = np.zeros((len(order), width), np.uint8)
    wmat.view(f"S{width}").ravel()[:] = words[order]
    pick = uniform_int(s(3), n, 0, len(order) - 1, np.int64)
    return np.ascontiguousarray(wmat[pick]), wmat


def float_uniform(seed, n, lo, hi):
    """Float32 uniform in ``[lo, hi)``."""
    return (np.float32(lo) + (np.float32(hi) - np.float32(lo)) * uniform01_f32(seed, n)).astype(np.float32)


def float_normal(seed, n, scale=1.0):
    return (normal_f32(stream_seed(int(seed), 0), stream_seed(int(seed), 1), n) * np.float32(scale)).astype(np.float32)


from .glyphs import GLYPH_SIZE, glyph_templates, image_column, cnn_init  # noqa: E402,F401
