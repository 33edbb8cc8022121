// Fused filter -> hash probe -> grouped SUM / COUNT / AVG.
//
// One streaming kernel reads each probe-side row once: it evaluates the
// predicate, probes the build table, forms the dense group id from the keys'
// declared domains and adds the row's value and count to a privatised
// accumulator:
//   G <= 8     per-thread registers, wave-reduced, one partial per workgroup;
//   G <= 2048  an LDS table per workgroup, merged with global atomics;
//   larger     global atomics on the dense table, or (many rows, at most
//              2^20 groups) the partitioned aggregation further below.
// For G <= 4096 one workgroup of a separate finishing kernel emits the
// non-empty groups in key order; larger tables are emitted by three small
// kernels (count per chunk, scan of the chunk counts, write), or ranked by
// the top-k kernels.  The opt-in partitioned (staged) probe is also below.
#include <type_traits>

#include "hash.hpp"

namespace tdp {

int table_clear_zero(const HashView& t, bool all_slots, int32_t* d_status, unsigned int* d_done,
                     unsigned long long* zero, int64_t n_zero, hipStream_t s);

namespace {

enum AccMode { ACC_REG = 0, ACC_LDS = 1, ACC_GLOBAL = 2 };
enum JoinMode { J_NONE = 0, J_KEYS = 1, J_ROWID = 2, J_AGG = 3 };
// Per-row value forms when the build side is pre-aggregated per key
// (cnt = build rows with the key, sum = their sum of the build operand).
enum AggForm { F_ACNT = 0, F_SUM = 1, F_ASUM = 2, F_AKCNT_SUM = 3, F_NONE = 4, F_ABCNT = 5, F_AKBCNT = 6 };

constexpr int kThreads = 256;
constexpr int kRegMaxG = 8;
constexpr int kFinRegThreads = 1024;  // threads of the finalize over register partials
constexpr int kLdsMaxG = 2048;
constexpr int kLastBlockMaxG = 4096;
constexpr int kFinChunk = kThreads * 16;

struct ColDev {
    const void* p = nullptr;
    int32_t dt = 0;
    int32_t side = 0;
};

// A further conjunct of the WHERE clause (integer or float32 column).
struct PredDev {
    ColDev col;
    int32_t cmp = 0;
    int64_t lit = 0;
    float litf = 0.0f;
};

struct GbDev {
    int64_t n_cand;
    const int32_t* sel;
    int32_t has_pred, pred_cmp;
    int64_t pred_lit;
    ColDev pred;
    int32_t n_more;                       // further conjuncts (generic signature only)
    PredDev more[TDP_MAX_MORE_PREDS];
    const int32_t* probe_key;
    HashView t;
    int32_t n_keys, expr, form;
    ColDev key[2];
    int64_t lo[2], card[2];
    ColDev a, b;
    int64_t k;
    int64_t G;
    unsigned long long* gtab;   // [G][sum, count] (LDS / GLOBAL modes): one 16-byte record per group
    unsigned long long* part;   // [nblocks][G][2] (REG mode)
    unsigned int* done;
    int32_t* status;
    int32_t last_block_fin;
    const uint32_t* n_parts_dev;  // REG partials: when set, only the first *n_parts_dev rows were written
    // outputs
    int64_t* d_n_groups;
    int64_t *okey0, *okey1, *osum, *ocnt;
    double* oavg;
};

__device__ __forceinline__ void read4(const ColDev& c, bool contiguous, int64_t r0, int64_t n, const int64_t rows[4],
                                      const int64_t brows[4], const bool ok[4], int64_t v[4]) {
    if (c.side == TDP_SIDE_PROBE && contiguous) {
        load4_int(c.p, c.dt, r0, n, v);
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            v[e] = ok[e] ? load_int(c.p, c.dt, c.side == TDP_SIDE_PROBE ? rows[e] : brows[e]) : 0;
    }
}

__device__ __forceinline__ bool cmp_f32(float a, int cmp, float b) {
    switch (cmp) {
        case TDP_LT: return a < b;
        case TDP_LE: return a <= b;
        case TDP_GT: return a > b;
        case TDP_GE: return a >= b;
        case TDP_EQ: return a == b;
        default: return a != b;
    }
}

// The further conjuncts of four candidate rows (probe side): clears ok[e]
// of a row that fails any of them.
__device__ __forceinline__ void more_preds4(const GbDev& d, bool contiguous, int64_t r0, const int64_t rows[4],
                                            const int64_t brows[4], bool ok[4]) {
    for (int j = 0; j < d.n_more; ++j) {
        const PredDev& q = d.more[j];
        if (q.col.dt == TDP_F32) {
            const float* f = (const float*)q.col.p;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (ok[e]) ok[e] = cmp_f32(f[contiguous ? r0 + e : rows[e]], q.cmp, q.litf);
        } else {
            int64_t v[4];
            read4(q.col, contiguous, r0, d.n_cand, rows, brows, ok, v);
#pragma unroll
            for (int e = 0; e < 4; ++e) ok[e] = ok[e] && cmp_i64(v[e], q.cmp, q.lit);
        }
    }
}

// Probe N keys at once.  Slots are read as aligned groups of four (one
// 16-byte load covers the home slot and the slots linear probing visits
// next, so most keys resolve from their first load), and the first group of
// every key is loaded before any comparison, so the N random reads are in
// flight together.
template <int N>
__device__ __forceinline__ void probeN(const int32_t* __restrict__ keys, uint32_t mask, uint32_t bmask,
                                       const int32_t* pk, bool* ok, int64_t* slot) {
    uint32_t h[N];
    int4 grp[N];
#pragma unroll
    for (int e = 0; e < N; ++e) h[e] = hash32((uint32_t)pk[e]) & mask;
#pragma unroll
    for (int e = 0; e < N; ++e)
        grp[e] = (ok[e] && pk[e] != kEmpty) ? *(const int4*)(keys + (h[e] & ~3u)) : make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
#pragma unroll
    for (int e = 0; e < N; ++e) {
        slot[e] = -1;
        if (!ok[e]) continue;
        if (pk[e] == kEmpty) {
            slot[e] = keys[(int64_t)mask + 1] ? (int64_t)mask + 1 : -1;
        } else {
            uint32_t s = h[e];
            int4 g = grp[e];
            uint32_t seen = 0;
            bool done = false;
            while (!done && seen <= bmask) {
                const int32_t kq[4] = {g.x, g.y, g.z, g.w};
                for (uint32_t q = s & 3u; q < 4; ++q) {
                    ++seen;
                    if (kq[q] == pk[e]) {
                        slot[e] = (s & ~3u) + q;
                        done = true;
                        break;
                    }
                    if (kq[q] == kEmpty) {
                        done = true;
                        break;
                    }
                }
                if (!done) {
                    s = ht_next(s | 3u, bmask);  // first slot of the next group (wraps inside the block)
                    g = *(const int4*)(keys + s);
                }
            }
        }
        if (slot[e] < 0) ok[e] = false;
    }
}

__device__ __forceinline__ void probe4(const int32_t* __restrict__ keys, uint32_t mask, uint32_t bmask,
                                       const int32_t pk[4], bool ok[4], int64_t slot[4]) {
    probeN<4>(keys, mask, bmask, pk, ok, slot);
}

// Probe four keys in an aggregate table: the record at each key's home slot
// is loaded before any comparison; a found record carries the key's count
// and sum.
__device__ __forceinline__ void probe_agg4(const HashView& t, const int32_t pk[4], bool ok[4],
                                           unsigned long long cnt[4], unsigned long long sum[4]) {
    uint32_t h[4];
    uint4 r[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) h[e] = pk[e] == kEmpty ? t.mask + 1 : hash32((uint32_t)pk[e]) & t.mask;
#pragma unroll
    for (int e = 0; e < 4; ++e) r[e] = ok[e] ? *(const uint4*)&t.rec[h[e]] : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if (!ok[e]) continue;
        bool found = false;
        if (pk[e] == kEmpty) {
            found = r[e].x != 0;  // the extra slot: key field is the presence flag
        } else {
            uint32_t s = h[e];
            uint4 q = r[e];
            for (uint32_t probe = 0; probe <= t.bmask; ++probe) {
                if ((int32_t)q.x == pk[e]) {
                    found = true;
                    break;
                }
                if ((int32_t)q.x == kEmpty) break;
                s = ht_next(s, t.bmask);
                q = *(const uint4*)&t.rec[s];
            }
            r[e] = q;
        }
        ok[e] = found;
        if (found) {
            cnt[e] = r[e].y;
            sum[e] = (unsigned long long)r[e].z | ((unsigned long long)r[e].w << 32);
        }
    }
}

// Column signatures.  A signature fixes, at compile time, the dtype (and
// table side) of each column the kernel reads, so that the loads of one
// group of rows are issued back to back with no data-dependent branch
// between them.  -1 = read the dtype at run time (the generic kernel),
// 0 = column absent.  MORE: the kernel also evaluates the further conjuncts
// of the WHERE clause (their dtypes read at run time).
struct SigGeneric {
    static constexpr int P = -1, K0 = -1, K1 = -1, A = -1, B = -1;
    static constexpr int K0S = -1, K1S = -1, AS = -1, BS = -1;
    static constexpr bool MORE = true;
};
// predicate i32; keys i8, i8 (probe side); value a*(k-b) or a*b with i64 a, b
struct SigPredI32KeysI8I8ValI64I64 {
    static constexpr int P = TDP_I32, K0 = TDP_I8, K1 = TDP_I8, A = TDP_I64, B = TDP_I64;
    static constexpr int K0S = TDP_SIDE_PROBE, K1S = TDP_SIDE_PROBE, AS = TDP_SIDE_PROBE, BS = TDP_SIDE_PROBE;
    static constexpr bool MORE = false;
};
// predicate i32; first key i8 from the build side, second key i8 from the probe side; value i64
struct SigPredI32BuildKeyI8KeyI8ValI64 {
    static constexpr int P = TDP_I32, K0 = TDP_I8, K1 = TDP_I8, A = TDP_I64, B = 0;
    static constexpr int K0S = TDP_SIDE_BUILD, K1S = TDP_SIDE_PROBE, AS = TDP_SIDE_PROBE, BS = -1;
    static constexpr bool MORE = false;
};
// no predicate; one i32 key; value i64 (or a pre-aggregated build-side sum)
struct SigKeyI32ValI64 {
    static constexpr int P = 0, K0 = TDP_I32, K1 = 0, A = TDP_I64, B = 0;
    static constexpr int K0S = TDP_SIDE_PROBE, K1S = -1, AS = TDP_SIDE_PROBE, BS = -1;
    static constexpr bool MORE = false;
};
// predicate i32 and further conjuncts; keys i8, i8 (probe side); COUNT only
// (the exact plan of a trainable WHERE ... GROUP BY two small keys)
struct SigPredI32KeysI8I8Count {
    static constexpr int P = TDP_I32, K0 = TDP_I8, K1 = TDP_I8, A = 0, B = 0;
    static constexpr int K0S = TDP_SIDE_PROBE, K1S = TDP_SIDE_PROBE, AS = -1, BS = -1;
    static constexpr bool MORE = true;
};

template <int DT>
__device__ __forceinline__ int64_t load1s(const void* p, int64_t i) {
    if constexpr (DT == TDP_I8) return ((const int8_t*)p)[i];
    else if constexpr (DT == TDP_I32) return ((const int32_t*)p)[i];
    else return ((const int64_t*)p)[i];
}

// Four consecutive rows from r0 (full group, 16-byte aligned column).
template <int DT>
__device__ __forceinline__ void load4s(const void* p, int64_t r0, int64_t v[4]) {
    if constexpr (DT == TDP_I32) {
        const int4 q = *(const int4*)((const int32_t*)p + r0);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else if constexpr (DT == TDP_I64) {
        const longlong2 a = *(const longlong2*)((const int64_t*)p + r0);
        const longlong2 b = *(const longlong2*)((const int64_t*)p + r0 + 2);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else {
        const char4 q = *(const char4*)((const int8_t*)p + r0);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    }
}

// Read one column for a group of four rows: static dtype (DT > 0) or the
// run-time path (DT < 0).
template <int DT, int SIDE, bool SEL, bool FULL>
__device__ __forceinline__ void colread(const ColDev& c, int64_t r0, int64_t n, const int64_t rows[4],
                                        const int64_t brows[4], const bool ok[4], int64_t v[4]) {
    if constexpr (DT < 0) {
        read4(c, !SEL, r0, n, rows, brows, ok, v);
    } else if constexpr (DT == 0) {
        v[0] = v[1] = v[2] = v[3] = 0;
    } else if constexpr (SIDE == TDP_SIDE_PROBE && !SEL) {
        if (FULL) {
            load4s<DT>(c.p, r0, v);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = r0 + e < n ? load1s<DT>(c.p, r0 + e) : 0;
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            v[e] = ok[e] ? load1s<DT>(c.p, SIDE == TDP_SIDE_PROBE ? rows[e] : brows[e]) : 0;
    }
}

// Emit group g (non-empty) at output position pos.
__device__ __forceinline__ void emit_group(const GbDev& d, int64_t g, int64_t pos, unsigned long long s,
                                           unsigned long long c) {
    const int64_t c1 = d.n_keys > 1 ? d.card[1] : 1;
    d.okey0[pos] = d.lo[0] + g / c1;
    if (d.okey1) d.okey1[pos] = d.n_keys > 1 ? d.lo[1] + g % c1 : 0;
    d.osum[pos] = (int64_t)s;
    d.ocnt[pos] = (int64_t)c;
    d.oavg[pos] = (double)(int64_t)s / (double)(int64_t)c;
}

// Block-wide exclusive scan of one 32-bit value per thread (256 threads).
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t& total, uint32_t* s_w) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    uint32_t incl = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t u = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += u;
    }
    if (lane == kWave - 1) s_w[wave] = incl;
    __syncthreads();
    uint32_t woff = 0;
    total = 0;
    for (int w = 0; w < kThreads / kWave; ++w) {
        if (w < wave) woff += s_w[w];
        total += s_w[w];
    }
    __syncthreads();
    return woff + incl - v;
}

// Emit the groups of a small table from one workgroup, after the
// aggregation kernel: REG partials ([n_parts][G][sum, count]) or the dense
// global table.
template <int ACC>
__device__ void finalize_last_block(const GbDev& d, int n_parts) {
    __shared__ uint32_t s_w[kThreads / kWave];
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    if (ACC == ACC_REG) {
        // every thread sums whole partial rows, so all loads are independent
        __shared__ unsigned long long s_acc[2][kFinRegThreads / kWave][kRegMaxG];
        unsigned long long s[kRegMaxG], c[kRegMaxG];
#pragma unroll
        for (int g = 0; g < kRegMaxG; ++g) s[g] = c[g] = 0;
        if (d.n_parts_dev) n_parts = min(n_parts, (int)*d.n_parts_dev);
        for (int64_t b = threadIdx.x; b < n_parts; b += blockDim.x) {
            const unsigned long long* row = d.part + b * d.G * 2;
#pragma unroll
            for (int g = 0; g < kRegMaxG; ++g) {
                if (g < d.G) {
                    s[g] += row[2 * g];
                    c[g] += row[2 * g + 1];
                }
            }
        }
#pragma unroll
        for (int g = 0; g < kRegMaxG; ++g) {
            const unsigned long long ws = wave_sum_u64(s[g]);
            const unsigned long long wc = wave_sum_u64(c[g]);
            if (lane == 0) {
                s_acc[0][wave][g] = ws;
                s_acc[1][wave][g] = wc;
            }
        }
        __syncthreads();
        // thread g adds group g over the waves, then thread 0 numbers the non-empty groups
        __shared__ unsigned long long s_tot[2][kRegMaxG];
        if (threadIdx.x < d.G) {
            unsigned long long ts = 0, tc = 0;
            for (int w = 0; w < (int)blockDim.x / kWave; ++w) {
                ts += s_acc[0][w][threadIdx.x];
                tc += s_acc[1][w][threadIdx.x];
            }
            s_tot[0][threadIdx.x] = ts;
            s_tot[1][threadIdx.x] = tc;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t m = 0;
            for (int64_t g = 0; g < d.G; ++g)
                if (s_tot[1][g]) emit_group(d, g, m++, s_tot[0][g], s_tot[1][g]);
            *d.d_n_groups = m;
        }
    } else {
        int64_t base = 0;
        for (int64_t g0 = 0; g0 < d.G; g0 += kThreads) {
            const int64_t g = g0 + threadIdx.x;
            unsigned long long s = 0, c = 0;
            if (g < d.G) {
                s = d.gtab[2 * g];
                c = d.gtab[2 * g + 1];
            }
            uint32_t total;
            const uint32_t pre = block_excl_scan(c ? 1u : 0u, total, s_w);
            if (c) {
                emit_group(d, g, base + pre, s, c);
                d.gtab[2 * g] = 0;  // leave the workspace ready for the next probe
                d.gtab[2 * g + 1] = 0;
            }
            base += total;
        }
        if (threadIdx.x == 0) *d.d_n_groups = base;
    }
}

template <int ACC>
__device__ void merge_and_finish(const GbDev& d, const unsigned long long* rs, const unsigned long long* rc,
                                 unsigned long long* s_tab);

// Add one row's (group, value, count) to the workgroup's accumulators.
template <int ACC>
__device__ __forceinline__ void acc_row(const GbDev& d, unsigned long long* rs, unsigned long long* rc,
                                        unsigned long long* s_tab, int64_t gid, unsigned long long v,
                                        unsigned long long c) {
    if (ACC == ACC_REG) {
#pragma unroll
        for (int g = 0; g < kRegMaxG; ++g) {
            const bool hit = gid == g;
            rs[g] += hit ? v : 0ull;
            rc[g] += hit ? c : 0ull;
        }
    } else if (ACC == ACC_LDS) {
        atomicAdd(&s_tab[gid], v);
        atomicAdd(&s_tab[d.G + gid], c);
    } else {
        atomicAdd(&d.gtab[2 * gid], v);
        atomicAdd(&d.gtab[2 * gid + 1], c);
    }
}

// Evaluate four consecutive candidate rows r0..r0+3: predicate, join probe,
// group id, value and the count each row adds (the matched build rows for a
// pre-aggregated build side, else 1).  ok: the row contributes; qual: the row
// passes range, predicate and group-key domain (whether or not it joins).
template <int JM, bool SEL, class S, bool FULL>
__device__ __forceinline__ void eval_rows(const GbDev& d, int64_t r0, bool ok[4], bool qual[4], int64_t gid[4],
                                          unsigned long long val[4], unsigned long long cnt[4]) {
    constexpr bool STATIC = S::P >= 0;
    const bool has_pred = STATIC ? S::P > 0 : d.has_pred != 0;
    const int n_keys = STATIC ? (S::K1 > 0 ? 2 : 1) : d.n_keys;
    const bool need_a = STATIC ? S::A > 0
                               : (JM == J_AGG ? (d.form == F_ACNT || d.form == F_ASUM || d.form == F_AKCNT_SUM ||
                                                 d.form == F_ABCNT || d.form == F_AKBCNT)
                                              : d.expr != TDP_EXPR_NONE);
    const bool need_b = STATIC ? S::B > 0
                               : (JM == J_AGG ? (d.form == F_ABCNT || d.form == F_AKBCNT)
                                              : (d.expr == TDP_EXPR_MUL || d.expr == TDP_EXPR_MUL_CONST_SUB));
    const int64_t c1 = n_keys > 1 ? d.card[1] : 1;
    int64_t rows[4], brows[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) brows[e] = 0;
    if (SEL) {
        if (FULL) {
            const int4 q = *(const int4*)(d.sel + r0);
            rows[0] = q.x; rows[1] = q.y; rows[2] = q.z; rows[3] = q.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) rows[e] = r0 + e < d.n_cand ? d.sel[r0 + e] : 0;
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) rows[e] = r0 + e;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) ok[e] = FULL || r0 + e < d.n_cand;
    int64_t pv[4], k0[4], k1[4], av[4], bv[4];
    int32_t pk[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) pv[e] = k0[e] = k1[e] = av[e] = bv[e] = 0, pk[e] = 0;
    // probe-side columns of a static signature: all loads issued together
    if constexpr (STATIC) {
        if constexpr (S::P > 0) colread<S::P, TDP_SIDE_PROBE, SEL, FULL>(d.pred, r0, d.n_cand, rows, brows, ok, pv);
        if constexpr (S::K0S == TDP_SIDE_PROBE) colread<S::K0, TDP_SIDE_PROBE, SEL, FULL>(d.key[0], r0, d.n_cand, rows, brows, ok, k0);
        if constexpr (S::K1 > 0 && S::K1S == TDP_SIDE_PROBE)
            colread<S::K1, TDP_SIDE_PROBE, SEL, FULL>(d.key[1], r0, d.n_cand, rows, brows, ok, k1);
        if constexpr (S::A > 0 && S::AS == TDP_SIDE_PROBE) colread<S::A, TDP_SIDE_PROBE, SEL, FULL>(d.a, r0, d.n_cand, rows, brows, ok, av);
        if constexpr (S::B > 0 && S::BS == TDP_SIDE_PROBE) colread<S::B, TDP_SIDE_PROBE, SEL, FULL>(d.b, r0, d.n_cand, rows, brows, ok, bv);
    }
    if (JM != J_NONE) {
        if (!SEL && FULL) {
            const int4 q = *(const int4*)(d.probe_key + r0);
            pk[0] = q.x; pk[1] = q.y; pk[2] = q.z; pk[3] = q.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) pk[e] = ok[e] ? d.probe_key[rows[e]] : 0;
        }
    }
    if (has_pred) {
        if constexpr (!STATIC) read4(d.pred, !SEL, r0, d.n_cand, rows, brows, ok, pv);
#pragma unroll
        for (int e = 0; e < 4; ++e) ok[e] = ok[e] && cmp_i64(pv[e], d.pred_cmp, d.pred_lit);
    }
    if constexpr (S::MORE) {
        if (d.n_more > 0) more_preds4(d, !SEL, r0, rows, brows, ok);
    }
    // qualifying rows (range, predicate), before the join
#pragma unroll
    for (int e = 0; e < 4; ++e) qual[e] = ok[e];
    unsigned long long bcnt[4], bsum[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) bcnt[e] = 1, bsum[e] = 0;
    if (JM == J_AGG) {
        probe_agg4(d.t, pk, ok, bcnt, bsum);
    } else if (JM != J_NONE) {
        int64_t slot[4];
        probeN<4>(d.t.keys, d.t.mask, d.t.bmask, pk, ok, slot);
        if (JM == J_ROWID) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (ok[e]) brows[e] = d.t.rowid[slot[e]];
        }
    }
    // build-side columns (static) or every column (run-time path)
    if constexpr (STATIC) {
        if constexpr (S::K0S == TDP_SIDE_BUILD) colread<S::K0, TDP_SIDE_BUILD, SEL, FULL>(d.key[0], r0, d.n_cand, rows, brows, ok, k0);
        if constexpr (S::K1 > 0 && S::K1S == TDP_SIDE_BUILD)
            colread<S::K1, TDP_SIDE_BUILD, SEL, FULL>(d.key[1], r0, d.n_cand, rows, brows, ok, k1);
        if constexpr (S::A > 0 && S::AS == TDP_SIDE_BUILD) colread<S::A, TDP_SIDE_BUILD, SEL, FULL>(d.a, r0, d.n_cand, rows, brows, ok, av);
        if constexpr (S::B > 0 && S::BS == TDP_SIDE_BUILD) colread<S::B, TDP_SIDE_BUILD, SEL, FULL>(d.b, r0, d.n_cand, rows, brows, ok, bv);
    } else {
        read4(d.key[0], !SEL, r0, d.n_cand, rows, brows, ok, k0);
        if (n_keys > 1) read4(d.key[1], !SEL, r0, d.n_cand, rows, brows, ok, k1);
        if (need_a) read4(d.a, !SEL, r0, d.n_cand, rows, brows, ok, av);
        if (need_b) read4(d.b, !SEL, r0, d.n_cand, rows, brows, ok, bv);
    }
    // group id
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t u0 = k0[e] - d.lo[0];
        const int64_t u1 = n_keys > 1 ? k1[e] - d.lo[1] : 0;
        const bool in = u0 >= 0 && u0 < d.card[0] && u1 >= 0 && u1 < c1;
        if (ok[e] && !in) raise_flag(d.status, TDP_FLAG_KEY_DOMAIN);
        if (!in) {
            ok[e] = false;
            qual[e] = false;
        }
        gid[e] = u0 * c1 + u1;
    }
    // value
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const unsigned long long a = (unsigned long long)av[e], b = (unsigned long long)bv[e];
        const unsigned long long K = (unsigned long long)d.k;
        val[e] = 0;
        if (JM == J_AGG) {
            switch (d.form) {
                case F_ACNT: val[e] = a * bcnt[e]; break;
                case F_SUM: val[e] = bsum[e]; break;
                case F_ASUM: val[e] = a * bsum[e]; break;
                case F_AKCNT_SUM: val[e] = a * (K * bcnt[e] - bsum[e]); break;
                case F_ABCNT: val[e] = a * b * bcnt[e]; break;
                case F_AKBCNT: val[e] = a * (K - b) * bcnt[e]; break;
                default: val[e] = 0; break;
            }
        } else {
            switch (d.expr) {
                case TDP_EXPR_COL: val[e] = a; break;
                case TDP_EXPR_MUL: val[e] = a * b; break;
                case TDP_EXPR_MUL_CONST_SUB: val[e] = a * (K - b); break;
                default: val[e] = 0; break;
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) cnt[e] = JM == J_AGG ? bcnt[e] : 1ull;
}

template <int ACC, int JM, bool SEL, class S>
__global__ __launch_bounds__(kThreads) void groupby_kernel(GbDev d) {
    extern __shared__ unsigned long long s_tab[];  // ACC_LDS: [G] sums then [G] counts
    unsigned long long rs[kRegMaxG], rc[kRegMaxG];
    if (ACC == ACC_REG) {
#pragma unroll
        for (int g = 0; g < kRegMaxG; ++g) rs[g] = rc[g] = 0;
    }
    if (ACC == ACC_LDS) {
        for (int64_t i = threadIdx.x; i < 2 * d.G; i += kThreads) s_tab[i] = 0;
        __syncthreads();
    }
    // four consecutive rows per thread and step (eight measured no faster:
    // the probe is bound by table lines fetched, not by reads in flight, and
    // the extra registers cost occupancy)
    auto rows4 = [&](int64_t r0, auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        bool ok[4], qual[4];
        int64_t gid[4];
        unsigned long long val[4], cnt[4];
        eval_rows<JM, SEL, S, FULL>(d, r0, ok, qual, gid, val, cnt);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (ok[e]) acc_row<ACC>(d, rs, rc, s_tab, gid[e], val[e], cnt[e]);
    };
    const int64_t stride = (int64_t)gridDim.x * kThreads * 4;
    int64_t r0 = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * 4;
    for (; r0 + 4 <= d.n_cand; r0 += stride) rows4(r0, std::true_type{});
    if (r0 < d.n_cand) rows4(r0, std::false_type{});

    merge_and_finish<ACC>(d, rs, rc, s_tab);
}

// Merge one workgroup's accumulators into its partial row (REG) or the
// global table (LDS).
template <int ACC>
__device__ void merge_and_finish(const GbDev& d, const unsigned long long* rs, const unsigned long long* rc,
                                 unsigned long long* s_tab) {
    if (ACC == ACC_REG) {
        __shared__ unsigned long long s_acc[2][1024 / kWave][kRegMaxG];
        const int lane = lane_id(), wave = threadIdx.x / kWave;
#pragma unroll
        for (int g = 0; g < kRegMaxG; ++g) {
            const unsigned long long s = wave_sum_u64(rs[g]);
            const unsigned long long c = wave_sum_u64(rc[g]);
            if (lane == 0) {
                s_acc[0][wave][g] = s;
                s_acc[1][wave][g] = c;
            }
        }
        __syncthreads();
        if (threadIdx.x < d.G) {
            unsigned long long s = 0, c = 0;
            for (int w = 0; w < (int)blockDim.x / kWave; ++w) {
                s += s_acc[0][w][threadIdx.x];
                c += s_acc[1][w][threadIdx.x];
            }
            d.part[((int64_t)blockIdx.x * d.G + threadIdx.x) * 2] = s;
            d.part[((int64_t)blockIdx.x * d.G + threadIdx.x) * 2 + 1] = c;
        }
    } else if (ACC == ACC_LDS) {
        __syncthreads();
        for (int64_t g = threadIdx.x; g < d.G; g += kThreads) {
            const unsigned long long c = s_tab[d.G + g];
            if (c) {
                atomicAdd(&d.gtab[2 * g], s_tab[g]);
                atomicAdd(&d.gtab[2 * g + 1], c);
            }
        }
    }
}

// Emits the groups of a small table (G <= 4096) after the aggregation
// kernel: one workgroup reads the partials or the dense table.  A separate
// launch orders it after every aggregation workgroup without a device-wide
// fence in each of them.
template <int ACC>
__global__ __launch_bounds__(ACC == ACC_REG ? kFinRegThreads : kThreads) void finalize_small_kernel(GbDev d,
                                                                                                    int n_parts) {
    finalize_last_block<ACC>(d, n_parts);
}

__global__ void gb_init_kernel(unsigned long long* zero, int64_t n_zero, int32_t* d_status, unsigned int* done) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_zero; i += stride) zero[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (d_status) *d_status = 0;
        *done = 0;
    }
}

// Large tables: non-empty count per chunk of kFinChunk groups.  Thread t
// reads groups t, t + 256, ... of its chunk, so every load is coalesced.
__global__ __launch_bounds__(kThreads) void fin_count_kernel(GbDev d, uint32_t* chunk_cnt) {
    __shared__ uint32_t s_w[kThreads / kWave];
    const int64_t g0 = (int64_t)blockIdx.x * kFinChunk + threadIdx.x;
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < kFinChunk / kThreads; ++i) {
        const int64_t g = g0 + (int64_t)i * kThreads;
        if (g < d.G && d.gtab[2 * g + 1]) ++m;
    }
    uint32_t total;
    block_excl_scan(m, total, s_w);
    if (threadIdx.x == 0) chunk_cnt[blockIdx.x] = total;
}

// Exclusive scan of the chunk counts (one workgroup) and the group total.
__global__ __launch_bounds__(kThreads) void fin_scan_kernel(uint32_t* chunk_cnt, int64_t n_chunks, int64_t* d_n_groups) {
    __shared__ uint32_t s_w[kThreads / kWave];
    uint32_t base = 0;
    for (int64_t c0 = 0; c0 < n_chunks; c0 += kThreads) {
        const int64_t c = c0 + threadIdx.x;
        const uint32_t v = c < n_chunks ? chunk_cnt[c] : 0;
        uint32_t total;
        const uint32_t pre = block_excl_scan(v, total, s_w);
        if (c < n_chunks) chunk_cnt[c] = base + pre;
        base += total;
    }
    if (threadIdx.x == 0) *d_n_groups = base;
}

// Rank of a set flag among the workgroup's threads (thread order) and the
// number of set flags, from wave ballots.
__device__ __forceinline__ uint32_t block_flag_rank(bool f, uint32_t& total, uint32_t* s_w) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const unsigned long long bal = __ballot(f);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
    if (lane == 0) s_w[wave] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t woff = 0;
    total = 0;
    for (int w = 0; w < kThreads / kWave; ++w) {
        if (w < wave) woff += s_w[w];
        total += s_w[w];
    }
    __syncthreads();
    return woff + below;
}

// Writes the chunk's non-empty groups in ascending order, one row of 256
// groups at a time (coalesced reads and nearly contiguous writes).
__global__ __launch_bounds__(kThreads) void fin_write_kernel(GbDev d, const uint32_t* chunk_off) {
    __shared__ uint32_t s_w[kThreads / kWave];
    const int64_t g0 = (int64_t)blockIdx.x * kFinChunk + threadIdx.x;
    ulonglong2 e[kFinChunk / kThreads];
#pragma unroll
    for (int i = 0; i < kFinChunk / kThreads; ++i) {
        const int64_t g = g0 + (int64_t)i * kThreads;
        e[i] = g < d.G ? *(const ulonglong2*)&d.gtab[2 * g] : make_ulonglong2(0ull, 0ull);
    }
    int64_t pos = chunk_off[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kFinChunk / kThreads; ++i) {
        const int64_t g = g0 + (int64_t)i * kThreads;
        const bool f = e[i].y != 0;
        uint32_t total;
        const uint32_t rank = block_flag_rank(f, total, s_w);
        if (f) {
            emit_group(d, g, pos + rank, e[i].x, e[i].y);
            *(ulonglong2*)&d.gtab[2 * g] = make_ulonglong2(0ull, 0ull);  // ready for the next probe
        }
        pos += total;
    }
}


// ------------------------------------------------------- staged probe
// For hash tables far beyond one XCD's L2 (4 MiB), probing in row order
// pulls a 128-byte table line per row through the fabric.  The staged probe
// partitions the probe side by table region first:
//   1. stage_hist_kernel: per tile of kStageTile rows, the qualifying rows
//      of each partition (kParts slot ranges of the table; predicate and
//      probe key only);
//   2. stage_colscan_kernel / stage_start_kernel: exclusive offsets per
//      (tile, partition) in partition-major order, each partition's region
//      padded to a multiple of 4 records;
//   3. stage_kernel: evaluates every qualifying row of a tile once (group id
//      and value), sorts the tile's records by partition in LDS and writes
//      each partition's run contiguously at its offset;
//   4. stage_probe_kernel: workgroups claim chunks of records from the
//      partitions of their own XCD first (partition mod 8 = XCD id read from
//      the hardware), so one partition's table slice is shared in that XCD's
//      L2 while its records stream past, then help elsewhere.
constexpr int kParts = 64;             // table partitions
constexpr int kStageTile = 4096;       // rows per staging tile (16 per thread)
constexpr int kStageGrid = 1024;       // workgroups of the histogram and staging passes
constexpr int kProbeGrid = 1024;       // workgroups of the probing pass
constexpr int kChunkRec = 8192;        // records per claimed chunk
constexpr uint16_t kSkipGid = 0xFFFF;  // padding / rejected record
constexpr int64_t kStageMaxG = 0xFFFF; // group ids are stored in 16 bits
constexpr bool kStagedAuto = false;

struct StageDev {
    int32_t* rkey;                 // [n_rec]
    uint16_t* rgid;                // [n_rec]
    unsigned long long* rval;      // [n_rec]
    uint32_t* off;                 // [n_tiles][kParts] counts, then offsets within the partition
    uint32_t* ptot;                // [kParts] records per partition
    uint32_t* pstart;              // [kParts + 1] partition starts (multiples of 4)
    uint32_t* ctr;                 // [kParts] chunks claimed by the probing pass
    int64_t n_tiles;
    int pshift;
};

__device__ __forceinline__ int stage_part(int32_t key, uint32_t mask, int pshift) {
    return key == kEmpty ? 0 : (int)((hash32((uint32_t)key) & mask) >> pshift);
}

// Predicate and probe key of four rows: which rows qualify, and their keys.
template <class S, bool FULL>
__device__ __forceinline__ void stage_keys4(const GbDev& d, int64_t r0, bool ok[4], int32_t pk[4]) {
    constexpr bool STATIC = S::P >= 0;
    const int64_t rows[4] = {r0, r0 + 1, r0 + 2, r0 + 3};
    const int64_t brows[4] = {0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < 4; ++e) ok[e] = FULL || r0 + e < d.n_cand;
    int64_t pv[4] = {0, 0, 0, 0};
    const bool has_pred = STATIC ? S::P > 0 : d.has_pred != 0;
    if constexpr (STATIC) {
        if constexpr (S::P > 0) colread<S::P, TDP_SIDE_PROBE, false, FULL>(d.pred, r0, d.n_cand, rows, brows, ok, pv);
    } else {
        if (d.has_pred) read4(d.pred, true, r0, d.n_cand, rows, brows, ok, pv);
    }
    if (FULL) {
        const int4 q = *(const int4*)(d.probe_key + r0);
        pk[0] = q.x; pk[1] = q.y; pk[2] = q.z; pk[3] = q.w;
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) pk[e] = ok[e] ? d.probe_key[r0 + e] : 0;
    }
    if (has_pred) {
#pragma unroll
        for (int e = 0; e < 4; ++e) ok[e] = ok[e] && cmp_i64(pv[e], d.pred_cmp, d.pred_lit);
    }
    if constexpr (S::MORE) {
        if (d.n_more > 0) more_preds4(d, true, r0, rows, brows, ok);
    }
}

// Every column of four rows: qualification (predicate only: a row whose
// group key is outside its domain still takes its record, marked skipped),
// probe key, group id and value.  All columns are on the probe side.
template <class S, bool FULL>
__device__ __forceinline__ void stage_eval(const GbDev& d, int64_t r0, bool ok[4], int32_t pk[4], uint16_t gid[4],
                                           unsigned long long val[4]) {
    constexpr bool STATIC = S::P >= 0;
    const int64_t rows[4] = {r0, r0 + 1, r0 + 2, r0 + 3};
    const int64_t brows[4] = {0, 0, 0, 0};
    int64_t k0[4] = {0, 0, 0, 0}, k1[4] = {0, 0, 0, 0}, av[4] = {0, 0, 0, 0}, bv[4] = {0, 0, 0, 0};
    const int n_keys = STATIC ? (S::K1 > 0 ? 2 : 1) : d.n_keys;
    const bool need_a = STATIC ? S::A > 0 : d.expr != TDP_EXPR_NONE;
    const bool need_b = STATIC ? S::B > 0 : (d.expr == TDP_EXPR_MUL || d.expr == TDP_EXPR_MUL_CONST_SUB);
    bool in_rows[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) in_rows[e] = FULL || r0 + e < d.n_cand;
    if constexpr (STATIC) {
        colread<S::K0, TDP_SIDE_PROBE, false, FULL>(d.key[0], r0, d.n_cand, rows, brows, in_rows, k0);
        if constexpr (S::K1 > 0) colread<S::K1, TDP_SIDE_PROBE, false, FULL>(d.key[1], r0, d.n_cand, rows, brows, in_rows, k1);
        if constexpr (S::A > 0) colread<S::A, TDP_SIDE_PROBE, false, FULL>(d.a, r0, d.n_cand, rows, brows, in_rows, av);
        if constexpr (S::B > 0) colread<S::B, TDP_SIDE_PROBE, false, FULL>(d.b, r0, d.n_cand, rows, brows, in_rows, bv);
    } else {
        read4(d.key[0], true, r0, d.n_cand, rows, brows, in_rows, k0);
        if (n_keys > 1) read4(d.key[1], true, r0, d.n_cand, rows, brows, in_rows, k1);
        if (need_a) read4(d.a, true, r0, d.n_cand, rows, brows, in_rows, av);
        if (need_b) read4(d.b, true, r0, d.n_cand, rows, brows, in_rows, bv);
    }
    stage_keys4<S, FULL>(d, r0, ok, pk);
    const int64_t c1 = n_keys > 1 ? d.card[1] : 1;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t u0 = k0[e] - d.lo[0];
        const int64_t u1 = n_keys > 1 ? k1[e] - d.lo[1] : 0;
        const bool in = u0 >= 0 && u0 < d.card[0] && u1 >= 0 && u1 < c1;
        if (ok[e] && !in) raise_flag(d.status, TDP_FLAG_KEY_DOMAIN);
        gid[e] = in ? (uint16_t)(u0 * c1 + u1) : kSkipGid;
        const unsigned long long a = (unsigned long long)av[e], b = (unsigned long long)bv[e];
        const unsigned long long K = (unsigned long long)d.k;
        switch (d.expr) {
            case TDP_EXPR_COL: val[e] = a; break;
            case TDP_EXPR_MUL: val[e] = a * b; break;
            case TDP_EXPR_MUL_CONST_SUB: val[e] = a * (K - b); break;
            default: val[e] = 0; break;
        }
    }
}

template <class S>
__global__ __launch_bounds__(kThreads) void stage_hist_kernel(GbDev d, StageDev st) {
    __shared__ uint32_t h[kParts];
    for (int64_t tile = blockIdx.x; tile < st.n_tiles; tile += gridDim.x) {
        if (threadIdx.x < kParts) h[threadIdx.x] = 0;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kStageTile / (kThreads * 4); ++j) {
            const int64_t r0 = tile * kStageTile + j * kThreads * 4 + (int64_t)threadIdx.x * 4;
            bool ok[4];
            int32_t pk[4];
            if (r0 + 4 <= d.n_cand)
                stage_keys4<S, true>(d, r0, ok, pk);
            else
                stage_keys4<S, false>(d, r0, ok, pk);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (ok[e]) atomicAdd(&h[stage_part(pk[e], d.t.mask, st.pshift)], 1u);
        }
        __syncthreads();
        if (threadIdx.x < kParts) st.off[tile * kParts + threadIdx.x] = h[threadIdx.x];
    }
}

// Workgroup p: exclusive prefix of partition p's tile counts (in place),
// and the partition's total.
__global__ __launch_bounds__(256) void stage_colscan_kernel(StageDev st) {
    __shared__ uint32_t s_w[kThreads / kWave];
    const int p = blockIdx.x, lane = lane_id(), wave = threadIdx.x / kWave;
    const int64_t per = ceil_div(st.n_tiles, (int64_t)kThreads);
    const int64_t t0 = threadIdx.x * per, t1 = t0 + per < st.n_tiles ? t0 + per : st.n_tiles;
    uint32_t sum = 0;
    for (int64_t t = t0; t < t1; ++t) sum += st.off[t * kParts + p];
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t u = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += u;
    }
    if (lane == kWave - 1) s_w[wave] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int w = 0; w < wave; ++w) run += s_w[w];
    for (int64_t t = t0; t < t1; ++t) {
        const uint32_t v = st.off[t * kParts + p];
        st.off[t * kParts + p] = run;
        run += v;
    }
    if (threadIdx.x == kThreads - 1) st.ptot[p] = run;
}

// One wave: padded partition starts, the padding records, and the probing
// pass's chunk counters.
__global__ void stage_start_kernel(StageDev st) {
    const int p = threadIdx.x;  // 64 lanes = 64 partitions
    const uint32_t tot = st.ptot[p];
    const uint32_t padded = (tot + 3u) & ~3u;
    uint32_t incl = padded;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t u = __shfl_up(incl, o, kWave);
        if (p >= o) incl += u;
    }
    const uint32_t start = incl - padded;
    st.pstart[p] = start;
    if (p == kParts - 1) st.pstart[kParts] = incl;
    for (uint32_t i = start + tot; i < start + padded; ++i) {
        st.rkey[i] = 0;
        st.rgid[i] = kSkipGid;
        st.rval[i] = 0;
    }
    st.ctr[p] = 0;
}

template <class S>
__global__ __launch_bounds__(kThreads) void stage_kernel(GbDev d, StageDev st) {
    __shared__ int32_t s_key[kStageTile];
    __shared__ unsigned long long s_val[kStageTile];
    __shared__ uint16_t s_gid[kStageTile];
    __shared__ uint8_t s_part[kStageTile];
    __shared__ uint32_t cnt[kParts], pref[kParts], base[kParts];
    for (int64_t tile = blockIdx.x; tile < st.n_tiles; tile += gridDim.x) {
        if (threadIdx.x < kParts) {
            cnt[threadIdx.x] = 0;
            base[threadIdx.x] = st.pstart[threadIdx.x] + st.off[tile * kParts + threadIdx.x];
        }
        __syncthreads();
        // counts of this tile per partition (the histogram pass's numbers)
        if (threadIdx.x < kWave) {
            const int p = threadIdx.x;
            const uint32_t c = (tile + 1 < st.n_tiles ? st.off[(tile + 1) * kParts + p] : st.ptot[p]) -
                               st.off[tile * kParts + p];
            uint32_t incl = c;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const uint32_t u = __shfl_up(incl, o, kWave);
                if (p >= o) incl += u;
            }
            pref[p] = incl - c;
        }
        __syncthreads();
        uint32_t total = 0;
#pragma unroll
        for (int j = 0; j < kStageTile / (kThreads * 4); ++j) {
            const int64_t r0 = tile * kStageTile + j * kThreads * 4 + (int64_t)threadIdx.x * 4;
            bool ok[4];
            int32_t pk[4];
            uint16_t gid[4];
            unsigned long long val[4];
            if (r0 + 4 <= d.n_cand)
                stage_eval<S, true>(d, r0, ok, pk, gid, val);
            else
                stage_eval<S, false>(d, r0, ok, pk, gid, val);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (!ok[e]) continue;
                const int part = stage_part(pk[e], d.t.mask, st.pshift);
                const uint32_t pos = pref[part] + atomicAdd(&cnt[part], 1u);
                s_key[pos] = pk[e];
                s_val[pos] = val[e];
                s_gid[pos] = gid[e];
                s_part[pos] = (uint8_t)part;
            }
        }
        __syncthreads();
        total = pref[kParts - 1] + cnt[kParts - 1];
        for (uint32_t i = threadIdx.x; i < total; i += kThreads) {
            const int part = s_part[i];
            const uint32_t at = base[part] + (i - pref[part]);
            st.rkey[at] = s_key[i];
            st.rval[at] = s_val[i];
            st.rgid[at] = s_gid[i];
        }
        __syncthreads();
    }
}

__device__ __forceinline__ uint32_t xcd_id() {
    uint32_t v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return v & 7u;
}

template <int ACC>
__global__ __launch_bounds__(kThreads) void stage_probe_kernel(GbDev d, StageDev st) {
    extern __shared__ unsigned long long s_tab[];  // ACC_LDS: [G] sums then [G] counts
    unsigned long long rs[kRegMaxG], rc[kRegMaxG];
    if (ACC == ACC_REG) {
#pragma unroll
        for (int g = 0; g < kRegMaxG; ++g) rs[g] = rc[g] = 0;
    }
    if (ACC == ACC_LDS) {
        for (int64_t i = threadIdx.x; i < 2 * d.G; i += kThreads) s_tab[i] = 0;
        __syncthreads();
    }
    __shared__ uint32_t s_chunk;
    const int tid = threadIdx.x;
    const int xcd = (int)xcd_id();
    for (int round = 0; round < 2; ++round) {
        for (int ci = 0; ci < kParts; ++ci) {
            const int p = round == 0 ? xcd + 8 * ci : ci;
            if (p >= kParts) break;
            const uint32_t pbeg = st.pstart[p], pend = st.pstart[p + 1];
            while (true) {
                __syncthreads();
                if (tid == 0) s_chunk = atomicAdd(&st.ctr[p], 1u);
                __syncthreads();
                const uint64_t lo = (uint64_t)pbeg + (uint64_t)s_chunk * kChunkRec;
                if (lo >= pend) break;
                const uint32_t hi = lo + kChunkRec < pend ? (uint32_t)lo + kChunkRec : pend;
                // pbeg, pend and lo are multiples of 4: whole groups of 4 records;
                // each thread takes two groups per step (8 probes in flight)
                for (uint32_t r = (uint32_t)lo + tid * 4; r < hi; r += kThreads * 8) {
                    int32_t pk[8];
                    uint32_t g[8];
                    unsigned long long v[8];
                    bool ok[8];
#pragma unroll
                    for (int hgrp = 0; hgrp < 2; ++hgrp) {
                        const uint32_t rr = r + hgrp * kThreads * 4;
                        const bool in = rr < hi;
                        const uint32_t ra = in ? rr : (uint32_t)lo;  // a valid group; ignored below
                        const int4 q = *(const int4*)(st.rkey + ra);
                        const uint2 gq = *(const uint2*)(st.rgid + ra);
                        const ulonglong2 va = *(const ulonglong2*)(st.rval + ra);
                        const ulonglong2 vb = *(const ulonglong2*)(st.rval + ra + 2);
                        const int o = hgrp * 4;
                        pk[o] = q.x; pk[o + 1] = q.y; pk[o + 2] = q.z; pk[o + 3] = q.w;
                        g[o] = gq.x & 0xFFFFu; g[o + 1] = gq.x >> 16; g[o + 2] = gq.y & 0xFFFFu; g[o + 3] = gq.y >> 16;
                        v[o] = va.x; v[o + 1] = va.y; v[o + 2] = vb.x; v[o + 3] = vb.y;
#pragma unroll
                        for (int e = 0; e < 4; ++e) ok[o + e] = in && g[o + e] != kSkipGid;
                    }
                    int64_t slot[8];
                    probeN<8>(d.t.keys, d.t.mask, d.t.bmask, pk, ok, slot);
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        if (ok[e]) acc_row<ACC>(d, rs, rc, s_tab, (int64_t)g[e], v[e], 1ull);
                }
            }
        }
    }
    merge_and_finish<ACC>(d, rs, rc, s_tab);
}

// ---------------------------------------------- radix-partitioned probe
// For keys-only joins (a unique build side, nothing read from it) whose
// table is far beyond the caches, every probe of the direct kernel fetches
// one random 128-byte table line.  Here both sides are partitioned by the top
// bits of the key's hash (murmur3's finaliser, a bijection on 32 bits, so a
// partition and the remaining bits, the tag, identify the key), and each
// partition is probed against an LDS table of its build tags.  The probe
// traffic becomes one sequential write and one read of 8-byte records.
//   build:  rp_count (build keys per build workgroup and partition, rounded
//           up to whole 64-byte units of 16 tags), rp_colscan, rp_start,
//           rp_build_scatter: the build tags grouped by partition (btag,
//           bstart), each region's last unit padded with kRpPadTag.
//   probe:  rp_count (probe rows per scatter workgroup and partition, rounded
//           up to whole 64-byte units of 8 records), rp_colscan, rp_start
//           (partition starts, work items of at most kRpItemRec records),
//           rp_scatter (every row once: predicate, group id, value and one
//           record in its partition), rp_probe (one work item per workgroup:
//           the partition's tags into an LDS table, then the item's records
//           streamed through it).
// A record is (field << tbits | tag, value).  The field is the group id; a
// row whose value does not fit in int32 sets the field's top bit and stores
// its row index instead (the probe re-reads its value from the columns); a
// field of all ones is a skipped record (a row that does not qualify, or
// padding).  Each scatter workgroup owns one region per partition, sized by
// the histogram.  It keeps fewer than 8 records per partition in LDS between
// sub-chunks and writes only whole, aligned 64-byte units, so no write covers
// part of a unit; the last unit of a region is padded with skipped records.
// The order of records inside a partition follows the workgroups; integer
// sums do not depend on it.
constexpr int kRpThreads = 1024;       // threads of the histogram and build-side kernels
constexpr int kRpMaxP = 1024;          // partitions the scans handle
constexpr int kRpBSub = 8192;          // build keys a workgroup orders at once (8 per thread)
constexpr int kRpTagUnit = 16;         // build tags per written unit (64 bytes)
constexpr uint32_t kRpPadTag = 0xFFFFFFFFu;  // padding of a build region's last unit (above every tag)
constexpr int64_t kRpBuildWgs = 256;   // build scatter workgroups at most (one per CU)
constexpr int kRpMinPBits = 6;         // 64 .. 1024 partitions
constexpr int kRpMaxPBits = 10;
constexpr int kRpScatThreads = 1024;   // threads of the probe-side scatter
constexpr int kRpSub = 4096;           // probe rows a scatter workgroup orders at once (4 per thread)
constexpr int kRpUnit = 8;             // records per written unit (64 bytes)
constexpr int kRpMaxUnits = (kRpSub + (1 << kRpMaxPBits) * (kRpUnit - 1)) / kRpUnit;
constexpr int kRpBMaxUnits = (kRpBSub + (1 << kRpMaxPBits) * (kRpTagUnit - 1)) / kRpTagUnit;
constexpr int kRpScatPerCU = 1;        // scatter workgroups per CU (about 125 KB of LDS each)
constexpr int kRpProbeThreads = 512;   // threads of the probing kernel (two workgroups per CU)
constexpr int kRpBktBits = 12;         // buckets of an LDS sub-table (4096 x 16 bytes)
constexpr int kRpSlots = 8;            // 16-bit slots per bucket
constexpr int kRpMaxTags = 20480;      // tag entries of one LDS sub-table, padding included (load <= 5/8)
constexpr int kRpOvf = 256;            // tags that found both their buckets full
constexpr uint32_t kRpItemRec = 65536;  // probe records per work item
constexpr int64_t kRpTargetTags = 15000;   // build keys per partition the partition count aims at
// AUTO takes the partitioned probe for builds and probes at least this large.
constexpr bool kRpAuto = true;
constexpr int64_t kRpAutoBuild = 1 << 18;  // measured on 60M probe rows: faster than the fused probe from 250K build keys up
constexpr int64_t kRpAutoRows = 1 << 22;

struct RpDev {
    uint32_t* btag = nullptr;            // [n_btag] build tags, partition-major (kRpPadTag pads each region)
    uint32_t* bcnt = nullptr;            // [bw][P] tags per (build workgroup, partition), then offsets
    uint32_t* bstart = nullptr;          // [P + 1] (multiples of kRpTagUnit)
    uint32_t* btot = nullptr;            // [P]
    int64_t bw = 0;                      // build scatter workgroups
    int64_t brows = 0;                   // build keys per build workgroup (a multiple of kRpBSub)
    int64_t n_btag = 0;                  // tag capacity
    uint2* rec = nullptr;                // [n_rec] probe records
    uint32_t* pcnt = nullptr;            // [pw][P] records per (scatter workgroup, partition), then offsets
    uint32_t* pstart = nullptr;          // [P + 1] (multiples of kRpUnit)
    uint32_t* ptot = nullptr;            // [P]
    uint32_t* item = nullptr;            // [P + 1] first work item of each partition
    int64_t pw = 0;                      // scatter workgroups
    int64_t prows = 0;                   // probe rows per scatter workgroup (a multiple of kRpSub)
    int64_t n_rec = 0;                   // record capacity
    int pbits = 0, tbits = 0, P = 0;
    int32_t* status = nullptr;           // the call's flags (build scatter)
};

__device__ __forceinline__ uint32_t rp_skip(const RpDev& r) { return (1u << r.pbits) - 1u; }
__device__ __forceinline__ uint32_t rp_wide(const RpDev& r) { return 1u << (r.pbits - 1); }

// Block-wide exclusive scan of one value per thread (blockDim.x threads);
// *total receives the sum.  Uses s_w[blockDim.x / 64]; its barriers order LDS only.
__device__ __forceinline__ uint32_t rp_block_scan(uint32_t v, uint32_t* s_w, uint32_t* total) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    uint32_t a = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t u = __shfl_up(a, o, kWave);
        if (lane >= o) a += u;
    }
    if (lane == kWave - 1) s_w[wave] = a;
    lds_barrier();
    uint32_t ex = a - v, t = 0;
    for (int w = 0; w < (int)blockDim.x / kWave; ++w) {
        if (w < wave) ex += s_w[w];
        t += s_w[w];
    }
    lds_barrier();
    *total = t;
    return ex;
}

// Keys per (workgroup chunk, partition), rounded up to whole units of
// `unit` entries: workgroup w counts the keys [w * rows, (w + 1) * rows) of
// either side (the build keys for the tag scatter, the probe keys for the
// record scatter), four 16-byte key loads per thread in flight.
__global__ __launch_bounds__(kRpThreads) void rp_count_kernel(const int32_t* __restrict__ keys, int64_t n, int64_t nw,
                                                              int64_t rows, uint32_t* cnt, int P, int tbits,
                                                              uint32_t unit) {
    __shared__ uint32_t h[1 << kRpMaxPBits];
    constexpr int kU = 4;
    for (int64_t w = blockIdx.x; w < nw; w += gridDim.x) {
        for (int q = threadIdx.x; q < P; q += kRpThreads) h[q] = 0;
        __syncthreads();
        const int64_t lo = w * rows, hi = lo + rows < n ? lo + rows : n;
        for (int64_t s = lo; s < hi; s += (int64_t)kRpThreads * 4 * kU) {
            int32_t k[kU][4];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int64_t r0 = s + (int64_t)u * kRpThreads * 4 + threadIdx.x * 4;
                if (r0 + 4 <= hi) {
                    const int4 q = *(const int4*)(keys + r0);
                    k[u][0] = q.x; k[u][1] = q.y; k[u][2] = q.z; k[u][3] = q.w;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) k[u][e] = r0 + e < hi ? keys[r0 + e] : 0;
                }
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int64_t r0 = s + (int64_t)u * kRpThreads * 4 + threadIdx.x * 4;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (r0 + e < hi) atomicAdd(&h[hash32((uint32_t)k[u][e]) >> tbits], 1u);
            }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < P; q += kRpThreads) cnt[w * P + q] = (h[q] + unit - 1) / unit * unit;
        __syncthreads();
    }
}

// Workgroup c: columns 16c .. 16c+15 of the [nw][P] counts, turned into
// exclusive prefixes over the chunks (in place); tot[p] is the column sum.
// 64 slices of chunks per column; each thread loads its slice 8 rows at a
// time, all loads of a batch in flight together.
constexpr int kRpScanCols = 16;
__global__ __launch_bounds__(1024) void rp_colscan_kernel(uint32_t* cnt, int64_t nw, int P, uint32_t* tot) {
    constexpr int kSl = 1024 / kRpScanCols;
    __shared__ uint32_t s_sum[kSl][kRpScanCols];
    const int cl = threadIdx.x % kRpScanCols, sl = threadIdx.x / kRpScanCols;
    const int col = blockIdx.x * kRpScanCols + cl;
    const int64_t per = ceil_div(nw, (int64_t)kSl);
    const int64_t w0 = sl * per, w1 = w0 + per < nw ? w0 + per : nw;
    uint32_t sum = 0;
    for (int64_t w = w0; w < w1; w += 8) {
        uint32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = w + k < w1 ? cnt[(w + k) * P + col] : 0u;
#pragma unroll
        for (int k = 0; k < 8; ++k) sum += v[k];
    }
    s_sum[sl][cl] = sum;
    __syncthreads();
    uint32_t run = 0;
    for (int k = 0; k < sl; ++k) run += s_sum[k][cl];
    for (int64_t w = w0; w < w1; w += 8) {
        uint32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = w + k < w1 ? cnt[(w + k) * P + col] : 0u;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (w + k < w1) cnt[(w + k) * P + col] = run;
            run += v[k];
        }
    }
    if (sl == kSl - 1) tot[col] = run;
}

// One workgroup: partition starts (exclusive prefix of the totals) and, when
// `item` is given, the first work item of each partition (at least one per
// partition, so every build partition is checked, up to kRpItemRec records
// each).
__global__ __launch_bounds__(kRpMaxP) void rp_start_kernel(int P, const uint32_t* tot, uint32_t* start,
                                                           uint32_t* item) {
    __shared__ uint32_t s_w[kRpMaxP / kWave];
    const int q = threadIdx.x;
    const uint32_t t = q < P ? tot[q] : 0u;
    const uint32_t it = q < P ? (t + kRpItemRec - 1) / kRpItemRec + (t == 0 ? 1u : 0u) : 0u;
    uint32_t tc, ti;
    const uint32_t ex = rp_block_scan(t, s_w, &tc);
    const uint32_t iex = rp_block_scan(it, s_w, &ti);
    if (q < P) {
        start[q] = ex;
        if (item) item[q] = iex;
    }
    if (q == 0) {
        start[P] = tc;
        if (item) item[P] = ti;
    }
}

// Build keys -> tags in partition regions, the way the record scatter below
// writes probe records: workgroup w takes the keys [w * brows, (w + 1) *
// brows) in sub-chunks of kRpBSub (two groups of four consecutive keys per
// thread); per sub-chunk each tag is ranked in its partition by an LDS
// counter, the tags are ordered by partition in LDS, every whole 64-byte unit
// of 16 tags is written (the partition's carried tags first) and the rest is
// carried on; the last unit of each region is padded with kRpPadTag.  One
// partition per thread in the per-partition steps (P <= kRpThreads).
__global__ __launch_bounds__(kRpThreads) void rp_build_scatter_kernel(const int32_t* __restrict__ keys, int64_t n,
                                                                      RpDev r) {
    constexpr int kMaxP = 1 << kRpMaxPBits;
    constexpr int kTpu = kRpTagUnit / 4;  // threads per unit, 16 bytes each
    static_assert(kMaxP <= kRpThreads && kRpBSub <= 0xFFFF && kRpBMaxUnits <= 0xFFFF, "per-thread partitions");
    __shared__ uint32_t s_tag[kRpBSub];
    __shared__ uint32_t s_carry[kMaxP][kRpTagUnit + 1];  // rows of 17 words: neighbours start in other banks
    __shared__ uint32_t s_cnt[kMaxP];
    __shared__ uint16_t s_pref[kMaxP];
    __shared__ uint16_t s_uoff[kMaxP];
    __shared__ uint8_t s_cc[kMaxP];
    __shared__ uint32_t s_cur[kMaxP];
    __shared__ uint32_t s_end[kMaxP];
    __shared__ uint16_t s_umap[kRpBMaxUnits];
    __shared__ uint32_t s_w[kRpThreads / kWave];
    __shared__ uint32_t s_units;
    const int64_t w = blockIdx.x;
    const int tid = threadIdx.x, P = r.P;
    const uint32_t tmask = (1u << r.tbits) - 1u;
    if (tid < P) {
        s_cur[tid] = r.bstart[tid] + r.bcnt[w * P + tid];
        s_end[tid] = r.bstart[tid] + (w + 1 < r.bw ? r.bcnt[(w + 1) * P + tid] : r.btot[tid]);
        s_cc[tid] = 0;
        s_cnt[tid] = 0;
    }
    lds_barrier();
    const int64_t lo = w * r.brows, hi = lo + r.brows < n ? lo + r.brows : n;
    for (int64_t base = lo; base < hi; base += kRpBSub) {
        uint32_t tg[8], rk[8];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t r0 = base + (int64_t)j * (kRpBSub / 2) + tid * 4;
            int32_t k[4];
            if (r0 + 4 <= hi) {
                const int4 q = *(const int4*)(keys + r0);
                k[0] = q.x; k[1] = q.y; k[2] = q.z; k[3] = q.w;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) k[e] = r0 + e < hi ? keys[r0 + e] : 0;
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t h = hash32((uint32_t)k[e]);
                tg[j * 4 + e] = h & tmask;
                rk[j * 4 + e] = r0 + e < hi ? (h >> r.tbits) : 0xFFFFFFFFu;
            }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (rk[i] != 0xFFFFFFFFu) rk[i] |= atomicAdd(&s_cnt[rk[i]], 1u) << 16;
        lds_barrier();
        {
            uint32_t cu = 0;
            if (tid < P) {
                const uint32_t c = s_cnt[tid];
                cu = c | (((s_cc[tid] + c) / kRpTagUnit) << 16);
            }
            uint32_t tot;
            const uint32_t ex = rp_block_scan(cu, s_w, &tot);
            if (tid < P) {
                s_pref[tid] = (uint16_t)(ex & 0xFFFFu);
                s_uoff[tid] = (uint16_t)(ex >> 16);
            }
            if (tid == 0) s_units = tot >> 16;
        }
        lds_barrier();
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (rk[i] != 0xFFFFFFFFu) s_tag[s_pref[rk[i] & 0xFFFFu] + (rk[i] >> 16)] = tg[i];
        if (tid < P) {
            const uint32_t u0 = s_uoff[tid], nu = (s_cc[tid] + s_cnt[tid]) / kRpTagUnit;
            for (uint32_t k = 0; k < nu; ++k) s_umap[u0 + k] = (uint16_t)tid;
        }
        lds_barrier();
        const uint32_t n_units = s_units;
        for (uint32_t t = tid; t < n_units * kTpu; t += kRpThreads) {
            const uint32_t u = t / kTpu;
            const uint32_t q = s_umap[u];
            const uint32_t cc = s_cc[q], pf = s_pref[q];
            const uint32_t v0 = (u - s_uoff[q]) * kRpTagUnit + (t % kTpu) * 4;
            uint32_t x[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) x[e] = v0 + e < cc ? s_carry[q][v0 + e] : s_tag[pf + v0 + e - cc];
            const uint32_t at = s_cur[q] + v0;
            if (at + 4 <= s_end[q])
                *(uint4*)(r.btag + at) = make_uint4(x[0], x[1], x[2], x[3]);
            else
                raise_flag(r.status, TDP_FLAG_TABLE_FULL);  // cannot happen: the histogram sized the region
        }
        lds_barrier();
        if (tid < P) {
            const uint32_t c = s_cnt[tid], cc = s_cc[tid], pf = s_pref[tid];
            const uint32_t all = cc + c, used = all / kRpTagUnit * kRpTagUnit;
            if (used > 0) {
                for (uint32_t v = used; v < all; ++v) s_carry[tid][v - used] = s_tag[pf + v - cc];
                s_cur[tid] += used;
            } else {
                for (uint32_t k = 0; k < c; ++k) s_carry[tid][cc + k] = s_tag[pf + k];
            }
            s_cc[tid] = (uint8_t)(all - used);
            s_cnt[tid] = 0;
        }
        lds_barrier();
    }
    if (tid < P && s_cc[tid] > 0) {
        const uint32_t cc = s_cc[tid], at = s_cur[tid];
        if (at + kRpTagUnit <= s_end[tid]) {
#pragma unroll
            for (int k = 0; k < kRpTagUnit; k += 4) {
                uint32_t x[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) x[e] = (uint32_t)(k + e) < cc ? s_carry[tid][k + e] : kRpPadTag;
                *(uint4*)(r.btag + at + k) = make_uint4(x[0], x[1], x[2], x[3]);
            }
        } else {
            raise_flag(r.status, TDP_FLAG_TABLE_FULL);
        }
    }
}

// The columns of four rows as loaded, so a workgroup can issue the loads
// of its next sub-chunk before it orders the current one (the loads stay in
// flight across its barriers).
struct Raw4 {
    int64_t pv[4], k0[4], k1[4], av[4], bv[4];
    int32_t pk[4];
};

template <class S, bool FULL>
__device__ __forceinline__ void rp_load4(const GbDev& d, int64_t r0, Raw4& w) {
    constexpr bool STATIC = S::P >= 0;
    const int64_t rows[4] = {r0, r0 + 1, r0 + 2, r0 + 3};
    const int64_t brows[4] = {0, 0, 0, 0};
    bool in[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) in[e] = FULL || r0 + e < d.n_cand;
    const bool need_a = STATIC ? S::A > 0 : d.expr != TDP_EXPR_NONE;
    const bool need_b = STATIC ? S::B > 0 : (d.expr == TDP_EXPR_MUL || d.expr == TDP_EXPR_MUL_CONST_SUB);
    const bool has_pred = STATIC ? S::P > 0 : d.has_pred != 0;
    const int n_keys = STATIC ? (S::K1 > 0 ? 2 : 1) : d.n_keys;
#pragma unroll
    for (int e = 0; e < 4; ++e) w.pv[e] = w.k1[e] = w.av[e] = w.bv[e] = 0;
    if constexpr (STATIC) {
        if constexpr (S::P > 0) colread<S::P, TDP_SIDE_PROBE, false, FULL>(d.pred, r0, d.n_cand, rows, brows, in, w.pv);
        colread<S::K0, TDP_SIDE_PROBE, false, FULL>(d.key[0], r0, d.n_cand, rows, brows, in, w.k0);
        if constexpr (S::K1 > 0) colread<S::K1, TDP_SIDE_PROBE, false, FULL>(d.key[1], r0, d.n_cand, rows, brows, in, w.k1);
        if constexpr (S::A > 0) colread<S::A, TDP_SIDE_PROBE, false, FULL>(d.a, r0, d.n_cand, rows, brows, in, w.av);
        if constexpr (S::B > 0) colread<S::B, TDP_SIDE_PROBE, false, FULL>(d.b, r0, d.n_cand, rows, brows, in, w.bv);
    } else {
        if (has_pred) read4(d.pred, true, r0, d.n_cand, rows, brows, in, w.pv);
        read4(d.key[0], true, r0, d.n_cand, rows, brows, in, w.k0);
        if (n_keys > 1) read4(d.key[1], true, r0, d.n_cand, rows, brows, in, w.k1);
        if (need_a) read4(d.a, true, r0, d.n_cand, rows, brows, in, w.av);
        if (need_b) read4(d.b, true, r0, d.n_cand, rows, brows, in, w.bv);
    }
    if (FULL) {
        const int4 q = *(const int4*)(d.probe_key + r0);
        w.pk[0] = q.x; w.pk[1] = q.y; w.pk[2] = q.z; w.pk[3] = q.w;
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) w.pk[e] = in[e] ? d.probe_key[r0 + e] : 0;
    }
}

// Qualification, group id and value of four loaded rows, as stage_eval
// computes them (further conjuncts of the WHERE clause are read here).  The
// same arithmetic runs in 32 bits where the operands provably fit: a 32- or
// 8-bit predicate column against a literal that fits in int32, 8-bit group
// keys with domain bounds within +-2^30 (their differences and the dense id,
// at most 2^27, fit in int32), and a value a * (k - b) or a * b whose
// factors fit in int32 on every row of the wave (one 32 x 32 -> 64-bit
// multiply instead of a 64 x 64-bit one).
template <class S>
__device__ __forceinline__ void rp_finish4(const GbDev& d, int64_t r0, const Raw4& w, bool ok[4], uint16_t gid[4],
                                           unsigned long long val[4]) {
    constexpr bool STATIC = S::P >= 0;
    constexpr bool NARROW_P = STATIC && (S::P == TDP_I32 || S::P == TDP_I8);
    constexpr bool NARROW_K = STATIC && S::K0 == TDP_I8 && (S::K1 <= 0 || S::K1 == TDP_I8);
    const bool has_pred = STATIC ? S::P > 0 : d.has_pred != 0;
    const int n_keys = STATIC ? (S::K1 > 0 ? 2 : 1) : d.n_keys;
#pragma unroll
    for (int e = 0; e < 4; ++e) ok[e] = r0 + e < d.n_cand;
    if (has_pred) {
        if (NARROW_P && d.pred_lit == (int64_t)(int32_t)d.pred_lit) {
            const int32_t lit = (int32_t)d.pred_lit;
            int32_t x[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) x[e] = (int32_t)w.pv[e];
            switch (d.pred_cmp) {
                case TDP_LT:
#pragma unroll
                    for (int e = 0; e < 4; ++e) ok[e] = ok[e] && x[e] < lit;
                    break;
                case TDP_LE:
#pragma unroll
                    for (int e = 0; e < 4; ++e) ok[e] = ok[e] && x[e] <= lit;
                    break;
                case TDP_GT:
#pragma unroll
                    for (int e = 0; e < 4; ++e) ok[e] = ok[e] && x[e] > lit;
                    break;
                case TDP_GE:
#pragma unroll
                    for (int e = 0; e < 4; ++e) ok[e] = ok[e] && x[e] >= lit;
                    break;
                case TDP_EQ:
#pragma unroll
                    for (int e = 0; e < 4; ++e) ok[e] = ok[e] && x[e] == lit;
                    break;
                default:
#pragma unroll
                    for (int e = 0; e < 4; ++e) ok[e] = ok[e] && x[e] != lit;
                    break;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) ok[e] = ok[e] && cmp_i64(w.pv[e], d.pred_cmp, d.pred_lit);
        }
    }
    if constexpr (S::MORE) {
        if (d.n_more > 0) {
            const int64_t rows[4] = {r0, r0 + 1, r0 + 2, r0 + 3};
            const int64_t brows[4] = {0, 0, 0, 0};
            more_preds4(d, true, r0, rows, brows, ok);
        }
    }
    const int64_t c1 = n_keys > 1 ? d.card[1] : 1;
    constexpr int64_t kB = (int64_t)1 << 30;
    const bool k32 = NARROW_K && d.lo[0] >= -kB && d.lo[0] <= kB && (n_keys < 2 || (d.lo[1] >= -kB && d.lo[1] <= kB));
    if (k32) {
        const int32_t lo0 = (int32_t)d.lo[0], lo1 = n_keys > 1 ? (int32_t)d.lo[1] : 0;
        const int32_t cd0 = (int32_t)d.card[0], cd1 = (int32_t)c1;  // the product of the domains is at most 2^27
        bool bad = false;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int32_t u0 = (int32_t)w.k0[e] - lo0;
            const int32_t u1 = n_keys > 1 ? (int32_t)w.k1[e] - lo1 : 0;
            const bool in = u0 >= 0 && u0 < cd0 && u1 >= 0 && u1 < cd1;
            bad = bad || (ok[e] && !in);
            gid[e] = in ? (uint16_t)(u0 * cd1 + u1) : kSkipGid;
        }
        if (bad) raise_flag(d.status, TDP_FLAG_KEY_DOMAIN);
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t u0 = w.k0[e] - d.lo[0];
            const int64_t u1 = n_keys > 1 ? w.k1[e] - d.lo[1] : 0;
            const bool in = u0 >= 0 && u0 < d.card[0] && u1 >= 0 && u1 < c1;
            if (ok[e] && !in) raise_flag(d.status, TDP_FLAG_KEY_DOMAIN);
            gid[e] = in ? (uint16_t)(u0 * c1 + u1) : kSkipGid;
        }
    }
    if (d.expr == TDP_EXPR_MUL || d.expr == TDP_EXPR_MUL_CONST_SUB) {
        int64_t f2[4];
        bool fit = true;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            f2[e] = d.expr == TDP_EXPR_MUL ? w.bv[e] : (int64_t)((unsigned long long)d.k - (unsigned long long)w.bv[e]);
            fit = fit && w.av[e] == (int64_t)(int32_t)w.av[e] && f2[e] == (int64_t)(int32_t)f2[e];
        }
        if (ballot(!fit) == 0) {
#pragma unroll
            for (int e = 0; e < 4; ++e) val[e] = (unsigned long long)((int64_t)(int32_t)w.av[e] * (int64_t)(int32_t)f2[e]);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) val[e] = (unsigned long long)w.av[e] * (unsigned long long)f2[e];
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) val[e] = d.expr == TDP_EXPR_COL ? (unsigned long long)w.av[e] : 0ull;
    }
}

// Probe rows -> records in partition regions.  Workgroup w takes the rows
// [w * prows, (w + 1) * prows) in sub-chunks of kRpSub rows (four
// consecutive rows per thread).  Per sub-chunk: every row's record and its
// rank in its partition (LDS counters); one scan gives each partition's
// offset among the new records and among the whole units it can write (the
// carried records first, then the new ones); the records are ordered by
// partition in LDS; kRpUnit / 2 threads write each whole unit (16 bytes
// each); the rest, fewer than kRpUnit records, is carried to the next
// sub-chunk.  Every row in range takes a record, so the regions the
// histogram sized are filled exactly.  Each thread owns kPpt consecutive
// partitions in the per-partition steps.
template <class S>
__global__ __launch_bounds__(kRpScatThreads) void rp_scatter_kernel(GbDev d, RpDev r) {
    constexpr int kMaxP = 1 << kRpMaxPBits;
    constexpr int kPpt = (kMaxP + kRpScatThreads - 1) / kRpScatThreads;  // partitions per thread
    constexpr int kTpu = kRpUnit / 2;                                    // threads per unit
    static_assert(kRpSub <= 0xFFFF && kRpMaxUnits <= 0xFFFF, "16-bit offsets");
    __shared__ uint2 s_rec[kRpSub];
    __shared__ uint2 s_carry[kMaxP][kRpUnit + 1];  // rows of kRpUnit + 1 records: neighbours start in other banks
    __shared__ uint32_t s_cnt[kMaxP];   // new records of the sub-chunk per partition
    __shared__ uint16_t s_pref[kMaxP];  // their exclusive prefix
    __shared__ uint16_t s_uoff[kMaxP];  // exclusive prefix of the whole units
    __shared__ uint8_t s_cc[kMaxP];     // carried records (< kRpUnit)
    __shared__ uint32_t s_cur[kMaxP];   // next record of the partition's region
    __shared__ uint32_t s_end[kMaxP];   // end of the region
    __shared__ uint16_t s_umap[kRpMaxUnits];  // unit -> partition
    __shared__ uint32_t s_w[kRpScatThreads / kWave];
    __shared__ uint32_t s_units;
    const int64_t w = blockIdx.x;
    const int tid = threadIdx.x, P = r.P;
    const uint32_t tmask = (1u << r.tbits) - 1u, skip = rp_skip(r), wide = rp_wide(r);
    for (int q = tid; q < P; q += kRpScatThreads) {
        s_cur[q] = r.pstart[q] + r.pcnt[w * P + q];
        s_end[q] = r.pstart[q] + (w + 1 < r.pw ? r.pcnt[(w + 1) * P + q] : r.ptot[q]);
        s_cc[q] = 0;
        s_cnt[q] = 0;
    }
    lds_barrier();
    const int64_t lo = w * r.prows, hi = lo + r.prows < d.n_cand ? lo + r.prows : d.n_cand;
    Raw4 raw;
    if (lo < hi) {
        const int64_t r0 = lo + (int64_t)tid * 4;
        if (r0 + 4 <= d.n_cand) rp_load4<S, true>(d, r0, raw);
        else rp_load4<S, false>(d, r0, raw);
    }
    for (int64_t base = lo; base < hi; base += kRpSub) {
        const int64_t r0 = base + (int64_t)tid * 4;
        bool ok[4];
        int32_t pk[4];
        uint16_t gid[4];
        unsigned long long val[4];
        rp_finish4<S>(d, r0, raw, ok, gid, val);
#pragma unroll
        for (int e = 0; e < 4; ++e) pk[e] = raw.pk[e];
        // the next sub-chunk's loads, in flight while this one is ordered
        {
            const int64_t n0 = r0 + kRpSub;
            if (base + kRpSub < hi) {
                if (n0 + 4 <= d.n_cand) rp_load4<S, true>(d, n0, raw);
                else rp_load4<S, false>(d, n0, raw);
            }
        }
        uint2 rec[4];
        uint32_t rank[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t h = hash32((uint32_t)pk[e]);
            const int64_t v = (int64_t)val[e];
            const bool use = ok[e] && gid[e] != kSkipGid;
            const bool fits = v == (int64_t)(int32_t)v;
            const uint32_t fld = !use ? skip : (fits ? (uint32_t)gid[e] : (wide | (uint32_t)gid[e]));
            rec[e] = make_uint2((fld << r.tbits) | (h & tmask), fits ? (uint32_t)(int32_t)v : (uint32_t)(r0 + e));
            rank[e] = h >> r.tbits;
        }
        if (r0 + 4 <= d.n_cand) {
#pragma unroll
            for (int e = 0; e < 4; ++e) rank[e] |= atomicAdd(&s_cnt[rank[e]], 1u) << 16;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (r0 + e < d.n_cand) rank[e] |= atomicAdd(&s_cnt[rank[e]], 1u) << 16;
        }
        lds_barrier();
        {
            // the thread's kPpt partitions: record counts (at most kRpSub) in
            // the low half, units in the high half, scanned as one sum
            uint32_t cu[kPpt], sum = 0;
#pragma unroll
            for (int k = 0; k < kPpt; ++k) {
                const int q = tid * kPpt + k;
                cu[k] = 0;
                if (q < P) {
                    const uint32_t c = s_cnt[q];
                    cu[k] = c | (((s_cc[q] + c) / kRpUnit) << 16);
                }
                sum += cu[k];
            }
            uint32_t tot;
            uint32_t ex = rp_block_scan(sum, s_w, &tot);
#pragma unroll
            for (int k = 0; k < kPpt; ++k) {
                const int q = tid * kPpt + k;
                if (q < P) {
                    s_pref[q] = (uint16_t)(ex & 0xFFFFu);
                    s_uoff[q] = (uint16_t)(ex >> 16);
                }
                ex += cu[k];
            }
            if (tid == 0) s_units = tot >> 16;
        }
        lds_barrier();
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (r0 + e < d.n_cand) {
                const uint32_t q = rank[e] & 0xFFFFu;
                s_rec[s_pref[q] + (rank[e] >> 16)] = rec[e];
            }
        }
        for (int q = tid; q < P; q += kRpScatThreads) {
            const uint32_t u0 = s_uoff[q], nu = (s_cc[q] + s_cnt[q]) / kRpUnit;
            for (uint32_t k = 0; k < nu; ++k) s_umap[u0 + k] = (uint16_t)q;
        }
        lds_barrier();
        const uint32_t n_units = s_units;
        for (uint32_t t = tid; t < n_units * kTpu; t += kRpScatThreads) {
            const uint32_t u = t / kTpu;
            const uint32_t q = s_umap[u];
            const uint32_t cc = s_cc[q], pf = s_pref[q];
            const uint32_t v0 = (u - s_uoff[q]) * kRpUnit + (t % kTpu) * 2;
            const uint2 a = v0 < cc ? s_carry[q][v0] : s_rec[pf + v0 - cc];
            const uint2 b = v0 + 1 < cc ? s_carry[q][v0 + 1] : s_rec[pf + v0 + 1 - cc];
            const uint32_t at = s_cur[q] + v0;
            if (at + 2 <= s_end[q])
                *(uint4*)(r.rec + at) = make_uint4(a.x, a.y, b.x, b.y);
            else
                raise_flag(d.status, TDP_FLAG_TABLE_FULL);  // cannot happen: the histogram sized the region
        }
        lds_barrier();
        for (int q = tid; q < P; q += kRpScatThreads) {
            const uint32_t c = s_cnt[q], cc = s_cc[q], pf = s_pref[q];
            const uint32_t all = cc + c, used = all / kRpUnit * kRpUnit;
            if (used > 0) {
                // the carry went out with the first unit; the tail of the new records stays
                for (uint32_t v = used; v < all; ++v) s_carry[q][v - used] = s_rec[pf + v - cc];
                s_cur[q] += used;
            } else {
                for (uint32_t k = 0; k < c; ++k) s_carry[q][cc + k] = s_rec[pf + k];
            }
            s_cc[q] = (uint8_t)(all - used);
            s_cnt[q] = 0;
        }
        lds_barrier();
    }
    // the last, partly filled unit of each region, padded with skipped records
    for (int q = tid; q < P; q += kRpScatThreads) {
        const uint32_t cc = s_cc[q], at = s_cur[q];
        if (cc == 0) continue;
        if (at + kRpUnit <= s_end[q]) {
            const uint2 pad = make_uint2(skip << r.tbits, 0u);
#pragma unroll
            for (int k = 0; k < kRpUnit; k += 2) {
                const uint2 a = (uint32_t)k < cc ? s_carry[q][k] : pad;
                const uint2 b = (uint32_t)k + 1 < cc ? s_carry[q][k + 1] : pad;
                *(uint4*)(r.rec + at + k) = make_uint4(a.x, a.y, b.x, b.y);
            }
        } else {
            raise_flag(d.status, TDP_FLAG_TABLE_FULL);
        }
    }
}

// Second bucket of a tag: the first one XOR an odd function of the tag's
// low bits (so the two always differ).
__device__ __forceinline__ uint32_t rp_alt(uint32_t f) {
    return ((f * 2654435761u) >> (32 - kRpBktBits)) | 1u;
}

// Value of a row whose value did not fit in its record, re-read from the
// probe-side columns (a keys-only join reads nothing from the build side).
__device__ __forceinline__ unsigned long long rp_row_value(const GbDev& d, int64_t row) {
    const bool need_b = d.expr == TDP_EXPR_MUL || d.expr == TDP_EXPR_MUL_CONST_SUB;
    const unsigned long long a = d.expr != TDP_EXPR_NONE ? (unsigned long long)load_int(d.a.p, d.a.dt, row) : 0ull;
    const unsigned long long b = need_b ? (unsigned long long)load_int(d.b.p, d.b.dt, row) : 0ull;
    switch (d.expr) {
        case TDP_EXPR_COL: return a;
        case TDP_EXPR_MUL: return a * b;
        case TDP_EXPR_MUL_CONST_SUB: return a * ((unsigned long long)d.k - b);
        default: return 0ull;
    }
}

// Copies of a tag in an LDS sub-table (both buckets and the overflow list).
__device__ __forceinline__ int rp_count(const uint4* bkt, const uint32_t* ovf, uint32_t no, uint32_t tag, int fbits) {
    const uint32_t f = tag & ((1u << fbits) - 1u);
    const uint32_t b1 = tag >> fbits;
    const uint4 y1 = bkt[b1], y2 = bkt[b1 ^ rp_alt(f)];
    const uint32_t u1[4] = {y1.x, y1.y, y1.z, y1.w}, u2[4] = {y2.x, y2.y, y2.z, y2.w};
    const uint32_t e1 = 0x8000u | f, e2 = 0xC000u | f;
    int c = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        c += ((u1[q] & 0xFFFFu) == e1) + ((u1[q] >> 16) == e1);
        c += ((u2[q] & 0xFFFFu) == e2) + ((u2[q] >> 16) == e2);
    }
    for (uint32_t o = 0; o < no; ++o) c += ovf[o] == tag;
    return c;
}

// Whether any 16-bit half of the four words of a bucket equals e
// (a half of w ^ (e, e) is zero; the borrow of a zero low half can only
// mark the high half too, when the low half already matched).
__device__ __forceinline__ bool rp_has(const uint4& x, uint32_t e) {
    const uint32_t pat = e | (e << 16);
    const uint32_t w[4] = {x.x ^ pat, x.y ^ pat, x.z ^ pat, x.w ^ pat};
    uint32_t z = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) z |= (w[q] - 0x00010001u) & ~w[q];
    return (z & 0x80008000u) != 0;
}

// Whether every slot of a bucket is taken (a stored entry has bit 15 set).
__device__ __forceinline__ bool rp_full(const uint4& x) {
    return (x.x & x.y & x.z & x.w & 0x80008000u) == 0x80008000u;
}

// One work item per workgroup: up to kRpItemRec records of one partition,
// probed against LDS sub-tables of the partition's build tags (one when the
// partition has at most kRpMaxTags keys).  A sub-table is 2^kRpBktBits
// buckets of kRpSlots 16-bit slots, a stored entry being valid bit | choice
// bit | the tag's low bits, which with the bucket identifies the tag.  A tag
// goes to its home bucket (its top bits) while that has a free slot, else to
// a second bucket (the home XOR a function of its low bits), else to a short
// overflow list.  Slots only fill, so a lookup whose home bucket is not full
// is decided by that one 16-byte LDS read; only a full home bucket sends it
// on to the second bucket (and the list).  The first item of a partition
// checks a unique build side: with one sub-table, by a scan of its buckets
// (a repeated tag shows as two equal entries in a bucket, as a second-bucket
// entry whose home bucket holds it too, or as a list entry found twice);
// with several, every tag of the partition must be found once in its own
// sub-table and nowhere else.  Workgroups beyond the last item leave at once
// (register accumulators) or add nothing (LDS accumulators).
template <int ACC>
__global__ __launch_bounds__(kRpProbeThreads) void rp_probe_kernel(GbDev d, RpDev r, int check_dup) {
    __shared__ uint4 bkt[1 << kRpBktBits];   // 8 x uint16 per bucket
    __shared__ uint32_t s_claim[(1 << kRpBktBits) / 2];  // 16-bit claim counters, two per word
    __shared__ uint32_t ovf[kRpOvf];
    __shared__ uint32_t n_ovf;
    __shared__ int s_p;
    extern __shared__ unsigned long long s_tab[];  // ACC_LDS: [G] sums then [G] counts
    unsigned long long rs[kRegMaxG];
    uint32_t rc32[kRegMaxG];
#pragma unroll
    for (int g = 0; g < kRegMaxG; ++g) rs[g] = 0, rc32[g] = 0;
    if (ACC == ACC_LDS) {
        for (int64_t i = threadIdx.x; i < 2 * d.G; i += kRpProbeThreads) s_tab[i] = 0;
    }
    const uint32_t n_items = r.item[r.P];
    const uint32_t b = blockIdx.x;
    if (b < n_items) {
        if (threadIdx.x == 0) {
            int lo = 0, hi = r.P - 1;  // last partition whose first item is <= b
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (r.item[mid] <= b) lo = mid; else hi = mid - 1;
            }
            s_p = lo;
        }
        __syncthreads();
        const int p = s_p;
        const uint32_t k = b - r.item[p];
        const uint32_t pb = r.pstart[p], pe = r.pstart[p] + r.ptot[p];
        const uint32_t lo = pb + k * kRpItemRec;
        const uint32_t hi = lo + kRpItemRec < pe ? lo + kRpItemRec : pe;  // lo and hi are multiples of kRpUnit
        const uint32_t tb = r.bstart[p], te = r.bstart[p + 1];
        const int fbits = r.tbits - kRpBktBits;
        const uint32_t fmask = (1u << fbits) - 1u, tmask = (1u << r.tbits) - 1u;
        const uint32_t skip = rp_skip(r), wide = rp_wide(r);
        const int G = (int)d.G;
        for (uint32_t t0 = tb;; t0 += kRpMaxTags) {
            const uint32_t t1 = te - t0 > (uint32_t)kRpMaxTags ? t0 + kRpMaxTags : te;
            for (int i = threadIdx.x; i < (1 << kRpBktBits); i += kRpProbeThreads) bkt[i] = make_uint4(0, 0, 0, 0);
            for (int i = threadIdx.x; i < (1 << kRpBktBits) / 2; i += kRpProbeThreads) s_claim[i] = 0u;
            if (threadIdx.x == 0) n_ovf = 0;
            __syncthreads();
            // the tags in batches of eight per thread, each batch's loads in
            // flight together before its inserts.  A tag claims a slot of its
            // home bucket by one atomic add on the bucket's 16-bit claim
            // counter (at most kRpMaxTags claims per sub-table: no overflow),
            // then writes its entry; a home bucket already full sends it to
            // its second bucket the same way, then to the overflow list.
            constexpr int kTb = 8;
            uint16_t* slots = (uint16_t*)bkt;
            for (uint32_t i0 = t0 + threadIdx.x; i0 < t1; i0 += kRpProbeThreads * kTb) {
                uint32_t tg[kTb];
#pragma unroll
                for (int j = 0; j < kTb; ++j) {
                    const uint32_t i = i0 + j * kRpProbeThreads;
                    tg[j] = i < t1 ? r.btag[i] : kRpPadTag;
                }
#pragma unroll
                for (int j = 0; j < kTb; ++j) {
                    if (tg[j] == kRpPadTag) continue;  // past the sub-table, or a region's padding
                    const uint32_t tag = tg[j] & tmask;
                    const uint32_t f = tag & fmask;
                    const uint32_t b1 = tag >> fbits;
                    const uint32_t sh1 = (b1 & 1u) * 16u;
                    const uint32_t c1 = (atomicAdd(&s_claim[b1 >> 1], 1u << sh1) >> sh1) & 0xFFFFu;
                    if (c1 < (uint32_t)kRpSlots) {
                        slots[b1 * kRpSlots + c1] = (uint16_t)(0x8000u | f);
                        continue;
                    }
                    const uint32_t b2 = b1 ^ rp_alt(f);
                    const uint32_t sh2 = (b2 & 1u) * 16u;
                    const uint32_t c2 = (atomicAdd(&s_claim[b2 >> 1], 1u << sh2) >> sh2) & 0xFFFFu;
                    if (c2 < (uint32_t)kRpSlots) {
                        slots[b2 * kRpSlots + c2] = (uint16_t)(0xC000u | f);
                        continue;
                    }
                    const uint32_t o = atomicAdd(&n_ovf, 1u);
                    if (o < (uint32_t)kRpOvf) ovf[o] = tag;
                    else raise_flag(d.status, TDP_FLAG_TABLE_FULL);
                }
            }
            __syncthreads();
            const uint32_t no = n_ovf < (uint32_t)kRpOvf ? n_ovf : (uint32_t)kRpOvf;
            if (check_dup && k == 0 && n_ovf <= (uint32_t)kRpOvf) {
                if (t0 == tb && t1 == te) {
                    // the partition's tags are all in this table: two copies of a
                    // tag sit in one bucket (both home or both second), or one in
                    // the home bucket and one in the second bucket or the list
                    for (int bb = threadIdx.x; bb < (1 << kRpBktBits); bb += kRpProbeThreads) {
                        const uint4 x = bkt[bb];
                        const uint32_t wv[4] = {x.x, x.y, x.z, x.w};
                        uint32_t ent[kRpSlots];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            ent[2 * q] = wv[q] & 0xFFFFu;
                            ent[2 * q + 1] = wv[q] >> 16;
                        }
                        bool dup = false;
#pragma unroll
                        for (int a = 0; a < kRpSlots; ++a) {
#pragma unroll
                            for (int c = a + 1; c < kRpSlots; ++c) dup |= ent[a] != 0 && ent[a] == ent[c];
                            if (ent[a] & 0x4000u) {  // a second-bucket entry: is the tag also at home?
                                const uint32_t f = ent[a] & fmask;
                                dup |= rp_has(bkt[(uint32_t)bb ^ rp_alt(f)], 0x8000u | f);
                            }
                        }
                        if (dup) raise_flag(d.status, TDP_FLAG_DUP_BUILD);
                    }
                    for (uint32_t o = threadIdx.x; o < no; o += kRpProbeThreads)
                        if (rp_count(bkt, ovf, no, ovf[o], fbits) != 1) raise_flag(d.status, TDP_FLAG_DUP_BUILD);
                } else {
                    // several sub-tables: every tag of the partition looks itself up
                    // and must be found once in its own sub-table, nowhere else
                    constexpr int kTb = 8;
                    for (uint32_t i0 = tb + threadIdx.x; i0 < te; i0 += kRpProbeThreads * kTb) {
                        uint32_t tg[kTb];
#pragma unroll
                        for (int j = 0; j < kTb; ++j) {
                            const uint32_t i = i0 + j * kRpProbeThreads;
                            tg[j] = i < te ? r.btag[i] : kRpPadTag;
                        }
#pragma unroll
                        for (int j = 0; j < kTb; ++j) {
                            const uint32_t i = i0 + j * kRpProbeThreads;
                            const int want = i >= t0 && i < t1 ? 1 : 0;
                            if (tg[j] != kRpPadTag && rp_count(bkt, ovf, no, tg[j] & tmask, fbits) != want)
                                raise_flag(d.status, TDP_FLAG_DUP_BUILD);
                        }
                    }
                }
            }
            // records: eight per thread and step (four 16-byte loads), the
            // next step's loads issued before this step's lookups.  Counts
            // of the register accumulators go to eight 8-bit fields of one
            // word (at most kRpItemRec / kRpProbeThreads rows per thread and
            // pass), unpacked after the pass.
            static_assert(kRpItemRec / kRpProbeThreads < 256, "8-bit count fields");
            unsigned long long pcnt = 0;
            constexpr int kLd = 4;
            constexpr uint32_t kStep = kRpProbeThreads * 2 * kLd;
            const uint32_t t2 = threadIdx.x * 2;
            const uint4 none = make_uint4(skip << r.tbits, 0, skip << r.tbits, 0);
            uint4 q4[kLd];
#pragma unroll
            for (int h = 0; h < kLd; ++h) {
                const uint32_t i = lo + (uint32_t)h * (kRpProbeThreads * 2) + t2;
                q4[h] = i < hi ? *(const uint4*)(r.rec + i) : none;
            }
            for (uint32_t s = lo; s < hi; s += kStep) {
                // i is even and hi a multiple of kRpUnit: a load covers both records or neither
                uint32_t x[2 * kLd], y[2 * kLd];
#pragma unroll
                for (int h = 0; h < kLd; ++h) {
                    x[2 * h] = q4[h].x;
                    y[2 * h] = q4[h].y;
                    x[2 * h + 1] = q4[h].z;
                    y[2 * h + 1] = q4[h].w;
                }
#pragma unroll
                for (int h = 0; h < kLd; ++h) {
                    const uint32_t i = s + kStep + (uint32_t)h * (kRpProbeThreads * 2) + t2;
                    q4[h] = i < hi ? *(const uint4*)(r.rec + i) : none;
                }
#pragma unroll
              for (int e0 = 0; e0 < 2 * kLd; e0 += 4) {
                uint4 x1[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) x1[e] = bkt[(x[e0 + e] & tmask) >> fbits];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int e = e0 + j;
                    const uint32_t fld = x[e] >> r.tbits;
                    const uint32_t tag = x[e] & tmask;
                    const uint32_t f = tag & fmask;
                    bool hit = fld != skip && rp_has(x1[j], 0x8000u | f);
                    if (fld != skip && !hit && rp_full(x1[j])) {
                        const uint4 x2 = bkt[(tag >> fbits) ^ rp_alt(f)];
                        hit = rp_has(x2, 0xC000u | f);
                        if (!hit && rp_full(x2))
                            for (uint32_t o = 0; o < no; ++o) hit |= ovf[o] == tag;
                    }
                    const uint32_t g = fld & (wide - 1u);
                    const unsigned long long v = (hit && (fld & wide)) ? rp_row_value(d, (int64_t)y[e])
                                                                       : (unsigned long long)(int64_t)(int32_t)y[e];
                    if (ACC == ACC_REG) {
                        pcnt += hit ? 1ull << (8u * g) : 0ull;
#pragma unroll
                        for (int q = 0; q < kRegMaxG; ++q) {
                            if (q >= G) break;
                            rs[q] += hit && g == (uint32_t)q ? v : 0ull;
                        }
                    } else if (hit) {
                        acc_row<ACC>(d, rs, rs, s_tab, (int64_t)g, v, 1ull);
                    }
                }
              }
            }
            if (ACC == ACC_REG) {
#pragma unroll
                for (int q = 0; q < kRegMaxG; ++q) rc32[q] += (uint32_t)(pcnt >> (8 * q)) & 0xFFu;
            }
            __syncthreads();  // the sub-table is rebuilt next
            if (t1 >= te) break;
        }
    }
    if (ACC == ACC_REG && b >= n_items) return;  // the finalize reads the first n_items partial rows only
    unsigned long long rc[kRegMaxG];
#pragma unroll
    for (int g = 0; g < kRegMaxG; ++g) rc[g] = rc32[g];
    merge_and_finish<ACC>(d, rs, rc, s_tab);
}

// -------------------------------------------------- partitioned aggregation
// For dense group tables too large for LDS (G > 2048), adding every row into
// the global table costs two device-scope atomics per row, resolved beyond
// the XCD caches.  Instead, rows are partitioned by group range (kPaggGroups
// groups per partition) and each partition is reduced in LDS:
//   1. pagg_hist_kernel: per tile of kStageTile rows, the qualifying rows of
//      each partition (predicate and probe-side group keys only);
//   2. pagg_colscan_kernel / pagg_start_kernel: offsets per (tile,
//      partition), partition-major;
//   3. pagg_stage_kernel: evaluates every row once (predicate, join probe,
//      group id, value) and writes a (group within partition, count, value)
//      record for each qualifying row, sorted by partition in LDS so each
//      tile writes contiguous runs; a row that finds no join partner leaves
//      a record with count and value 0;
//   4. pagg_reduce_kernel: one workgroup per partition adds its records into
//      an LDS table and writes the partition's slice of the dense table.
constexpr int kPaggGroups = 4096;
constexpr int kPaggShift = 12;
constexpr int kPaggMaxParts = 256;

struct PaggDev {
    uint16_t* rg;                  // [n_rec] group within its partition
    uint32_t* rc;                  // [n_rec] count the record adds
    unsigned long long* rv;        // [n_rec] value it adds
    uint32_t* off;                 // [n_tiles][np] counts, then offsets within the partition
    uint32_t* ptot;                // [np]
    uint32_t* pstart;              // [np + 1]
    int64_t n_tiles;
    int np;
};

// Predicate and probe-side group keys of four rows: which rows qualify and
// their group ids (no join, no flags).
template <class S, bool FULL>
__device__ __forceinline__ void eval_gids(const GbDev& d, int64_t r0, bool qual[4], int64_t gid[4]) {
    constexpr bool STATIC = S::P >= 0;
    const int64_t rows[4] = {r0, r0 + 1, r0 + 2, r0 + 3};
    const int64_t brows[4] = {0, 0, 0, 0};
    const bool has_pred = STATIC ? S::P > 0 : d.has_pred != 0;
    const int n_keys = STATIC ? (S::K1 > 0 ? 2 : 1) : d.n_keys;
    const int64_t c1 = n_keys > 1 ? d.card[1] : 1;
#pragma unroll
    for (int e = 0; e < 4; ++e) qual[e] = FULL || r0 + e < d.n_cand;
    int64_t pv[4] = {0, 0, 0, 0}, k0[4] = {0, 0, 0, 0}, k1[4] = {0, 0, 0, 0};
    if constexpr (STATIC) {
        if constexpr (S::P > 0) colread<S::P, TDP_SIDE_PROBE, false, FULL>(d.pred, r0, d.n_cand, rows, brows, qual, pv);
        colread<S::K0, TDP_SIDE_PROBE, false, FULL>(d.key[0], r0, d.n_cand, rows, brows, qual, k0);
        if constexpr (S::K1 > 0) colread<S::K1, TDP_SIDE_PROBE, false, FULL>(d.key[1], r0, d.n_cand, rows, brows, qual, k1);
    } else {
        if (has_pred) read4(d.pred, true, r0, d.n_cand, rows, brows, qual, pv);
        read4(d.key[0], true, r0, d.n_cand, rows, brows, qual, k0);
        if (n_keys > 1) read4(d.key[1], true, r0, d.n_cand, rows, brows, qual, k1);
    }
    if constexpr (S::MORE) {
        if (d.n_more > 0) more_preds4(d, true, r0, rows, brows, qual);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if (has_pred) qual[e] = qual[e] && cmp_i64(pv[e], d.pred_cmp, d.pred_lit);
        const int64_t u0 = k0[e] - d.lo[0];
        const int64_t u1 = n_keys > 1 ? k1[e] - d.lo[1] : 0;
        qual[e] = qual[e] && u0 >= 0 && u0 < d.card[0] && u1 >= 0 && u1 < c1;
        gid[e] = u0 * c1 + u1;
    }
}

template <class S>
__global__ __launch_bounds__(kThreads) void pagg_hist_kernel(GbDev d, PaggDev pg) {
    __shared__ uint32_t h[kPaggMaxParts];
    for (int64_t tile = blockIdx.x; tile < pg.n_tiles; tile += gridDim.x) {
        for (int p = threadIdx.x; p < pg.np; p += kThreads) h[p] = 0;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kStageTile / (kThreads * 4); ++j) {
            const int64_t r0 = tile * kStageTile + j * kThreads * 4 + (int64_t)threadIdx.x * 4;
            bool qual[4];
            int64_t gid[4];
            if (r0 + 4 <= d.n_cand)
                eval_gids<S, true>(d, r0, qual, gid);
            else
                eval_gids<S, false>(d, r0, qual, gid);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (qual[e]) atomicAdd(&h[gid[e] >> kPaggShift], 1u);
        }
        __syncthreads();
        for (int p = threadIdx.x; p < pg.np; p += kThreads) pg.off[tile * pg.np + p] = h[p];
    }
}

// Workgroup p: exclusive prefix of partition p's tile counts (in place) and
// the partition's total.
__global__ __launch_bounds__(256) void pagg_colscan_kernel(PaggDev pg) {
    __shared__ uint32_t s_w[kThreads / kWave];
    const int p = blockIdx.x, lane = lane_id(), wave = threadIdx.x / kWave;
    const int64_t per = ceil_div(pg.n_tiles, (int64_t)kThreads);
    const int64_t t0 = threadIdx.x * per, t1 = t0 + per < pg.n_tiles ? t0 + per : pg.n_tiles;
    uint32_t sum = 0;
    for (int64_t t = t0; t < t1; ++t) sum += pg.off[t * pg.np + p];
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t u = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += u;
    }
    if (lane == kWave - 1) s_w[wave] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int w = 0; w < wave; ++w) run += s_w[w];
    for (int64_t t = t0; t < t1; ++t) {
        const uint32_t v = pg.off[t * pg.np + p];
        pg.off[t * pg.np + p] = run;
        run += v;
    }
    if (threadIdx.x == kThreads - 1) pg.ptot[p] = run;
}

// One workgroup: partition starts (exclusive prefix of the totals).
__global__ __launch_bounds__(256) void pagg_start_kernel(PaggDev pg) {
    __shared__ uint32_t s_w[kThreads / kWave];
    const int p = threadIdx.x, lane = lane_id(), wave = threadIdx.x / kWave;
    const uint32_t tot = p < pg.np ? pg.ptot[p] : 0u;
    uint32_t incl = tot;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t u = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += u;
    }
    if (lane == kWave - 1) s_w[wave] = incl;
    __syncthreads();
    uint32_t start = incl - tot;
    for (int w = 0; w < wave; ++w) start += s_w[w];
    if (p < pg.np) pg.pstart[p] = start;
    if (p == pg.np - 1) pg.pstart[pg.np] = start + tot;
}

template <int JM, class S>
__global__ __launch_bounds__(kThreads) void pagg_stage_kernel(GbDev d, PaggDev pg) {
    __shared__ unsigned long long s_val[kStageTile];
    __shared__ uint32_t s_cnt[kStageTile];
    __shared__ uint16_t s_grp[kStageTile];
    __shared__ uint8_t s_part[kStageTile];
    __shared__ uint32_t cnt[kPaggMaxParts], pref[kPaggMaxParts], base[kPaggMaxParts];
    __shared__ uint32_t s_w[kThreads / kWave];
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    for (int64_t tile = blockIdx.x; tile < pg.n_tiles; tile += gridDim.x) {
        // this tile's records per partition, from the histogram pass
        uint32_t c = 0;
        const int p = threadIdx.x;
        if (p < pg.np) {
            cnt[p] = 0;
            base[p] = pg.pstart[p] + pg.off[tile * pg.np + p];
            c = (tile + 1 < pg.n_tiles ? pg.off[(tile + 1) * pg.np + p] : pg.ptot[p]) - pg.off[tile * pg.np + p];
        }
        uint32_t incl = c;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t u = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += u;
        }
        if (lane == kWave - 1) s_w[wave] = incl;
        __syncthreads();
        uint32_t ex = incl - c;
        for (int w = 0; w < wave; ++w) ex += s_w[w];
        if (p < pg.np) pref[p] = ex;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kStageTile / (kThreads * 4); ++j) {
            const int64_t r0 = tile * kStageTile + j * kThreads * 4 + (int64_t)threadIdx.x * 4;
            bool ok[4], qual[4];
            int64_t gid[4];
            unsigned long long val[4], rcnt[4];
            if (r0 + 4 <= d.n_cand)
                eval_rows<JM, false, S, true>(d, r0, ok, qual, gid, val, rcnt);
            else
                eval_rows<JM, false, S, false>(d, r0, ok, qual, gid, val, rcnt);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (!qual[e]) continue;
                const int part = (int)(gid[e] >> kPaggShift);
                const uint32_t pos = pref[part] + atomicAdd(&cnt[part], 1u);
                s_val[pos] = ok[e] ? val[e] : 0ull;
                s_cnt[pos] = ok[e] ? (uint32_t)rcnt[e] : 0u;
                s_grp[pos] = (uint16_t)(gid[e] & (kPaggGroups - 1));
                s_part[pos] = (uint8_t)part;
            }
        }
        __syncthreads();
        const uint32_t total = pref[pg.np - 1] + cnt[pg.np - 1];
        for (uint32_t i = threadIdx.x; i < total; i += kThreads) {
            const int part = s_part[i];
            const uint32_t at = base[part] + (i - pref[part]);
            pg.rv[at] = s_val[i];
            pg.rc[at] = s_cnt[i];
            pg.rg[at] = s_grp[i];
        }
        __syncthreads();
    }
}

// Workgroup p: the dense-table slice of groups [p * kPaggGroups, ...).  One
// workgroup per slice leaves a few hundred workgroups for the whole chip, so
// each takes 1024 threads with four records per thread in flight (measured:
// 285 -> 60 us over the 1M-group many-to-many aggregation).
constexpr int kPaggRedThreads = 1024;
__global__ __launch_bounds__(kPaggRedThreads) void pagg_reduce_kernel(GbDev d, PaggDev pg) {
    __shared__ unsigned long long s_sum[kPaggGroups], s_cnt[kPaggGroups];
    const int p = blockIdx.x;
    for (int j = threadIdx.x; j < kPaggGroups; j += kPaggRedThreads) s_sum[j] = s_cnt[j] = 0;
    __syncthreads();
    const uint32_t lo = pg.pstart[p], hi = pg.pstart[p + 1];
    for (uint32_t i0 = lo + threadIdx.x; i0 < hi; i0 += 4 * kPaggRedThreads) {
        uint32_t c[4];
        int g[4];
        unsigned long long v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t i = i0 + k * kPaggRedThreads;
            const bool in = i < hi;
            c[k] = in ? pg.rc[i] : 0u;
            g[k] = in ? pg.rg[i] : 0;
            v[k] = in ? pg.rv[i] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (c[k] == 0) continue;
            atomicAdd(&s_sum[g[k]], v[k]);
            atomicAdd(&s_cnt[g[k]], (unsigned long long)c[k]);
        }
    }
    __syncthreads();
    const int64_t g0 = (int64_t)p * kPaggGroups;
    for (int j = threadIdx.x; j < kPaggGroups && g0 + j < d.G; j += kPaggRedThreads)
        *(ulonglong2*)&d.gtab[2 * (g0 + j)] = make_ulonglong2(s_sum[j], s_cnt[j]);
}

// ------------------------------------------------------------------ top-k
// Exact top-k of the dense group table by (SUM descending, key ascending).
// A candidate packs the order key as hi = SUM with its sign bit flipped (so
// unsigned order is signed order) and lo = ~gid (so a smaller gid ranks
// higher on equal SUM); empty slots are hi = lo = 0, below every group.  The
// 96-bit key (hi, lo) is unique per group.  Each stage loads a chunk of
// kTopChunk candidates into LDS, finds the chunk's k-th largest key by a
// radix select (twelve 8-bit digits from the top, a 256-bin histogram and
// one wave scanning it per digit), and keeps the k candidates at or above it,
// in no particular order, until one chunk remains; the last stage sorts its
// k survivors (bitonic) and emits them.
constexpr int kTopChunk = 2048;
constexpr int kTopMax = 1024;

struct Cand {
    unsigned long long hi;
    unsigned long long cnt;
    unsigned int lo;
    unsigned int pad;
};

__device__ __forceinline__ bool cand_less(const Cand& a, const Cand& b) {
    return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

// Digit d (0 = most significant) of the 96-bit key (hi, lo).
__device__ __forceinline__ uint32_t cand_digit(const Cand& c, int d) {
    const int shift = 88 - 8 * d;  // of the 96-bit key
    return shift >= 32 ? (uint32_t)(c.hi >> (shift - 32)) & 0xFFu : (c.lo >> shift) & 0xFFu;
}

// Whether the top 8d bits of c's key equal those of (phi, plo).
__device__ __forceinline__ bool cand_prefix(const Cand& c, int d, unsigned long long phi, unsigned int plo) {
    if (d == 0) return true;
    if (d <= 8) return (c.hi >> (64 - 8 * d)) == (phi >> (64 - 8 * d));
    return c.hi == phi && (d == 12 || (c.lo >> (96 - 8 * d)) == (plo >> (96 - 8 * d)));
}

// from_dense: read (and zero) the dense accumulators; otherwise read `in`.
// last: emit the best k groups (in order) instead of writing k candidates.
constexpr int kTopThreads = 1024;
__global__ __launch_bounds__(kTopThreads) void topk_stage_kernel(GbDev d, const Cand* in, int64_t n, int k, Cand* out,
                                                                 int from_dense, int last) {
    __shared__ Cand sc[kTopChunk];
    __shared__ Cand sk[kTopMax];              // the k kept candidates
    __shared__ uint32_t s_hist[256];
    __shared__ unsigned long long s_phi;
    __shared__ unsigned int s_plo;
    __shared__ int s_need, s_above, s_tie;
    const int64_t base = (int64_t)blockIdx.x * kTopChunk;
    const int64_t avail = n - base;
    const int m = (int)(avail < kTopChunk ? (avail > 0 ? avail : 0) : kTopChunk);
    for (int i = threadIdx.x; i < m; i += kTopThreads) {
        const int64_t j = base + i;
        Cand c{0ull, 0ull, 0u, 0u};
        if (from_dense) {
            const unsigned long long cnt = d.gtab[2 * j + 1];
            if (cnt) {
                c.hi = d.gtab[2 * j] ^ 0x8000000000000000ull;
                c.lo = ~(unsigned int)j;
                c.cnt = cnt;
                d.gtab[2 * j] = 0;  // leave the workspace ready for the next probe
                d.gtab[2 * j + 1] = 0;
            }
        } else {
            c = in[j];
        }
        sc[i] = c;
    }
    if (threadIdx.x == 0) {
        s_phi = 0ull;
        s_plo = 0u;
        s_need = k;  // rank (from the top) of the wanted key among those matching the prefix
    }
    const int lane = threadIdx.x & (kWave - 1);
    const bool select = m > k;  // otherwise every loaded candidate is kept
    for (int dg = 0; select && dg < 12; ++dg) {
        for (int b = threadIdx.x; b < 256; b += kTopThreads) s_hist[b] = 0;
        __syncthreads();
        const unsigned long long phi = s_phi;
        const unsigned int plo = s_plo;
        for (int i = threadIdx.x; i < m; i += kTopThreads) {
            const Cand c = sc[i];
            if (cand_prefix(c, dg, phi, plo)) atomicAdd(&s_hist[cand_digit(c, dg)], 1u);
        }
        __syncthreads();
        if (threadIdx.x < kWave) {
            // lane l holds bins 255 - 4l .. 252 - 4l (descending); find the bin where the rank falls
            uint32_t h[4], sum = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                h[q] = s_hist[255 - 4 * lane - q];
                sum += h[q];
            }
            uint32_t incl = sum;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const uint32_t t = __shfl_up(incl, off, kWave);
                if (lane >= off) incl += t;
            }
            uint32_t run = incl - sum;
            const uint32_t need = (uint32_t)s_need;
            if (run < need && need <= incl) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (run < need && need <= run + h[q]) {
                        const unsigned long long dig = (unsigned long long)(255 - 4 * lane - q);
                        const int shift = 88 - 8 * dg;
                        if (shift >= 32) s_phi = phi | (dig << (shift - 32));
                        else s_plo = plo | ((unsigned int)dig << shift);
                        s_need = (int)(need - run);
                    }
                    run += h[q];
                }
            }
        }
        __syncthreads();
    }
    // keep the keys above the threshold, then s_need keys equal to it (the
    // threshold itself when keys are unique; empty slots otherwise)
    if (threadIdx.x == 0) {
        s_above = 0;
        s_tie = 0;
    }
    __syncthreads();
    const unsigned long long thi = s_phi;
    const unsigned int tlo = s_plo;
    const int ties = select ? s_need : 0;
    const int n_above = select ? k - ties : m;
    for (int i = threadIdx.x; i < m; i += kTopThreads) {
        const Cand c = sc[i];
        const bool above = !select || c.hi > thi || (c.hi == thi && c.lo > tlo);
        if (above) {
            sk[atomicAdd(&s_above, 1)] = c;
        } else if (c.hi == thi && c.lo == tlo) {
            const int t = atomicAdd(&s_tie, 1);
            if (t < ties) sk[n_above + t] = c;
        }
    }
    __syncthreads();
    const int kept = select ? k : m;  // candidates in sk[0, kept)
    if (!last) {
        for (int i = threadIdx.x; i < k; i += kTopThreads)
            out[(int64_t)blockIdx.x * k + i] = i < kept ? sk[i] : Cand{0ull, 0ull, 0u, 0u};
        return;
    }
    // last stage: sort the kept candidates (descending) and emit the non-empty ones
    int ms = 2;
    while (ms < kept) ms <<= 1;
    for (int i = kept + threadIdx.x; i < ms; i += kTopThreads) sk[i] = Cand{0ull, 0ull, 0u, 0u};
    for (int size = 2; size <= ms; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int i = threadIdx.x; i < ms / 2; i += kTopThreads) {
                const int pos = 2 * i - (i & (stride - 1));
                const int partner = pos + stride;
                const bool desc = (pos & size) == 0;
                const Cand a = sk[pos], b = sk[partner];
                if (desc ? cand_less(a, b) : cand_less(b, a)) {
                    sk[pos] = b;
                    sk[partner] = a;
                }
            }
        }
    }
    __syncthreads();
    __shared__ int s_m;
    if (threadIdx.x == 0) {
        int mm = 0;
        while (mm < kept && mm < k && (sk[mm].hi | sk[mm].lo)) ++mm;
        s_m = mm;
        *d.d_n_groups = mm;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < s_m; i += kTopThreads) {
        const Cand c = sk[i];
        emit_group(d, (int64_t)(~c.lo), i, c.hi ^ 0x8000000000000000ull, c.cnt);
    }
}

// ------------------------------------------------------------------ planning

struct Plan {
    int jm = J_NONE;
    TableKind kind = TABLE_KEYS;
    bool with_sum = false;
    uint32_t cap = 0;
    const void* bvals = nullptr;
    int bdt = 0;
    int form = F_NONE;
    ColDev a, b;
    int expr = TDP_EXPR_NONE;
    int64_t G = 1;
    int acc = ACC_REG;
    int nblocks = 1;
    bool last_block_fin = true;
    int64_t n_cand = 0;
    int topk = 0;
    bool staged = false;   // staged (partitioned) probe for large keys-only tables
    int pshift = 0;
    int64_t stage_tiles = 0;
    bool pagg = false;     // partitioned aggregation of a large dense table
    int pagg_np = 0;
    bool radix = false;    // radix-partitioned probe with LDS tables
    int rp_pbits = 0;
    int64_t rp_bw = 0, rp_pw = 0, rp_prows = 0, rp_nrec = 0, rp_brows = 0, rp_nbtag = 0;
};

ColDev coldev(const tdp_col& c) {
    ColDev r;
    r.p = c.data;
    r.dt = c.dtype;
    r.side = c.side;
    return r;
}

int make_plan(const tdp_groupby_desc* d, Plan& p) {
    if (!d) return fail(TDP_EINVAL, "tdp_groupby_agg: null descriptor");
    if (d->n_rows < 0 || (d->sel && d->n_sel < 0)) return fail(TDP_EINVAL, "tdp_groupby_agg: negative size");
    if (d->n_rows > INT32_MAX) return fail(TDP_EINVAL, "tdp_groupby_agg: more than 2^31-1 rows");
    if (d->n_keys < 1 || d->n_keys > 2) return fail(TDP_EINVAL, "tdp_groupby_agg: n_keys %d", d->n_keys);
    if (d->expr < TDP_EXPR_COL || d->expr > TDP_EXPR_NONE) return fail(TDP_EINVAL, "tdp_groupby_agg: expr %d", d->expr);
    if (d->topk < 0 || d->topk > kTopMax) return fail(TDP_EINVAL, "tdp_groupby_agg: topk %d outside 0..%d", d->topk, kTopMax);
    const tdp_join_desc* j = d->join;
    auto check_col = [&](const tdp_col& c, const char* what) -> int {
        if (!int_dtype(c.dtype)) return fail(TDP_EUNSUPPORTED, "tdp_groupby_agg: %s dtype %d", what, c.dtype);
        if (c.side != TDP_SIDE_PROBE && c.side != TDP_SIDE_BUILD)
            return fail(TDP_EINVAL, "tdp_groupby_agg: %s side %d", what, c.side);
        if (c.side == TDP_SIDE_BUILD && !j) return fail(TDP_EINVAL, "tdp_groupby_agg: %s on the build side without a join", what);
        const int64_t need = c.side == TDP_SIDE_PROBE ? d->n_rows : (j ? j->n_build : 0);
        if (c.n < need) return fail(TDP_EINVAL, "tdp_groupby_agg: %s has %lld rows < %lld", what, (long long)c.n, (long long)need);
        if (need > 0 && !c.data) return fail(TDP_EINVAL, "tdp_groupby_agg: %s data is null", what);
        if ((uintptr_t)c.data & 15) return fail(TDP_EINVAL, "tdp_groupby_agg: %s is not 16-byte aligned", what);
        return TDP_OK;
    };
    int rc;
    if (d->has_pred) {
        if ((rc = check_col(d->pred, "predicate column"))) return rc;
        if (d->pred.side != TDP_SIDE_PROBE) return fail(TDP_EUNSUPPORTED, "tdp_groupby_agg: predicate on the build side");
        if (d->pred_cmp < TDP_LT || d->pred_cmp > TDP_NE) return fail(TDP_EINVAL, "tdp_groupby_agg: comparison %d", d->pred_cmp);
    }
    if (d->n_more_preds < 0 || d->n_more_preds > TDP_MAX_MORE_PREDS)
        return fail(TDP_EINVAL, "tdp_groupby_agg: n_more_preds %d outside 0..%d", d->n_more_preds, TDP_MAX_MORE_PREDS);
    if (d->n_more_preds > 0 && !d->more_preds) return fail(TDP_EINVAL, "tdp_groupby_agg: null more_preds");
    for (int i = 0; i < d->n_more_preds; ++i) {
        const tdp_pred& q = d->more_preds[i];
        if (q.col.dtype == TDP_F32) {
            if (q.col.side != TDP_SIDE_PROBE) return fail(TDP_EUNSUPPORTED, "tdp_groupby_agg: predicate on the build side");
            if (q.col.n < d->n_rows) return fail(TDP_EINVAL, "tdp_groupby_agg: predicate column shorter than n_rows");
            if (d->n_rows > 0 && !q.col.data) return fail(TDP_EINVAL, "tdp_groupby_agg: predicate data is null");
            if ((uintptr_t)q.col.data & 15) return fail(TDP_EINVAL, "tdp_groupby_agg: predicate column is not 16-byte aligned");
        } else {
            if ((rc = check_col(q.col, "predicate column"))) return rc;
            if (q.col.side != TDP_SIDE_PROBE) return fail(TDP_EUNSUPPORTED, "tdp_groupby_agg: predicate on the build side");
        }
        if (q.cmp < TDP_LT || q.cmp > TDP_NE) return fail(TDP_EINVAL, "tdp_groupby_agg: comparison %d", q.cmp);
    }
    p.G = 1;
    for (int i = 0; i < d->n_keys; ++i) {
        if ((rc = check_col(d->key[i], "group key"))) return rc;
        if (d->key_card[i] < 1) return fail(TDP_EINVAL, "tdp_groupby_agg: key_card[%d] < 1", i);
        if (d->key_card[i] > (1ll << 27) || p.G * d->key_card[i] > (1ll << 27))
            return fail(TDP_EUNSUPPORTED, "tdp_groupby_agg: key domains exceed 2^27 groups");
        p.G *= d->key_card[i];
    }
    const bool need_a = d->expr != TDP_EXPR_NONE;
    const bool need_b = d->expr == TDP_EXPR_MUL || d->expr == TDP_EXPR_MUL_CONST_SUB;
    if (need_a && (rc = check_col(d->a, "value operand a"))) return rc;
    if (need_b && (rc = check_col(d->b, "value operand b"))) return rc;
    p.expr = d->expr;
    if (need_a) p.a = coldev(d->a);
    if (need_b) p.b = coldev(d->b);
    if (d->sel && d->n_sel > 0 && (uintptr_t)d->sel & 15) return fail(TDP_EINVAL, "tdp_groupby_agg: sel not 16-byte aligned");
    p.n_cand = d->sel ? d->n_sel : d->n_rows;

    if (j) {
        if (j->n_build < 0 || j->n_build > INT32_MAX) return fail(TDP_EINVAL, "tdp_groupby_agg: build size");
        if (j->n_build > 0 && !j->build_key) return fail(TDP_EINVAL, "tdp_groupby_agg: null build key");
        if (d->n_rows > 0 && !j->probe_key) return fail(TDP_EINVAL, "tdp_groupby_agg: null probe key");
        if (j->n_probe < d->n_rows) return fail(TDP_EINVAL, "tdp_groupby_agg: probe key shorter than n_rows");
        if ((uintptr_t)j->probe_key & 15) return fail(TDP_EINVAL, "tdp_groupby_agg: probe key not 16-byte aligned");
        if (j->probe_sel) return fail(TDP_EINVAL, "tdp_groupby_agg: use the descriptor's sel, not join->probe_sel");
        if (j->load_pct != 0 && (j->load_pct < 10 || j->load_pct > 90)) return fail(TDP_EINVAL, "tdp_groupby_agg: load_pct");
        if (j->max_distinct < 0) return fail(TDP_EINVAL, "tdp_groupby_agg: negative max_distinct");
        bool build_ref = false;
        for (int i = 0; i < d->n_keys; ++i) build_ref |= d->key[i].side == TDP_SIDE_BUILD;
        if (need_a) build_ref |= d->a.side == TDP_SIDE_BUILD;
        if (need_b) build_ref |= d->b.side == TDP_SIDE_BUILD;
        p.cap = table_cap(distinct_bound(j), j->load_pct);
        if (j->build_unique) {
            p.jm = build_ref ? J_ROWID : J_KEYS;
            p.kind = build_ref ? TABLE_ROWID : TABLE_KEYS;
        } else {
            p.jm = J_AGG;
            p.kind = TABLE_AGG;
            for (int i = 0; i < d->n_keys; ++i)
                if (d->key[i].side == TDP_SIDE_BUILD)
                    return fail(TDP_EUNSUPPORTED, "tdp_groupby_agg: build-side group key needs build_unique");
            const bool ab = need_a && d->a.side == TDP_SIDE_BUILD, bb = need_b && d->b.side == TDP_SIDE_BUILD;
            switch (d->expr) {
                case TDP_EXPR_NONE: p.form = F_NONE; break;
                case TDP_EXPR_COL:
                    if (ab) {
                        p.form = F_SUM;
                        p.bvals = d->a.data;
                        p.bdt = d->a.dtype;
                    } else {
                        p.form = F_ACNT;
                    }
                    break;
                case TDP_EXPR_MUL:
                    if (ab && bb) return fail(TDP_EUNSUPPORTED, "tdp_groupby_agg: MUL of two build columns over a non-unique build");
                    if (!ab && !bb) {
                        p.form = F_ABCNT;
                    } else {
                        p.form = F_ASUM;
                        const tdp_col& bc = ab ? d->a : d->b;
                        p.bvals = bc.data;
                        p.bdt = bc.dtype;
                        p.a = coldev(ab ? d->b : d->a);
                    }
                    break;
                case TDP_EXPR_MUL_CONST_SUB:
                    if (ab) return fail(TDP_EUNSUPPORTED, "tdp_groupby_agg: a*(k-b) with a on a non-unique build side");
                    if (bb) {
                        p.form = F_AKCNT_SUM;
                        p.bvals = d->b.data;
                        p.bdt = d->b.dtype;
                    } else {
                        p.form = F_AKBCNT;
                    }
                    break;
            }
            p.with_sum = p.bvals != nullptr;
        }
    } else {
        p.jm = J_NONE;
    }
    p.topk = d->topk;
    // top-k ranks the dense table, so it needs the LDS or global accumulators
    p.acc = (p.G <= kRegMaxG && !p.topk) ? ACC_REG : (p.G <= kLdsMaxG ? ACC_LDS : ACC_GLOBAL);
    p.nblocks = (int)std::min<int64_t>(std::max<int64_t>(ceil_div(p.n_cand, kThreads * 4), 1), 8 * kCUs);
    // LDS accumulators merge into the global table with 2G atomics per
    // workgroup, all on the same G slots: one workgroup per CU (measured on
    // the 1M-row, 75-group query: probe 55 -> 36 us; 128 workgroups 51 us),
    // four from 4M candidate rows, where the scan outweighs the merge.
    if (p.acc == ACC_LDS) p.nblocks = std::min(p.nblocks, p.n_cand >= (4 << 20) ? 4 * kCUs : kCUs);
    p.last_block_fin = p.G <= kLastBlockMaxG && !p.topk;
    // Tables well beyond one XCD's L2 with many probe rows take the staged probe.
    if (d->strategy < TDP_PROBE_AUTO || d->strategy > TDP_PROBE_PARTITIONED)
        return fail(TDP_EINVAL, "tdp_groupby_agg: strategy %d", d->strategy);
    // Radix-partitioned probe: keys-only joins whose probe side is read in
    // order (no selection vector) and whose group ids fit beside the tag (the
    // field's top bit marks a wide value, all ones a skipped record).
    {
        const int64_t nb = j ? j->n_build : 0;
        int pb = kRpMinPBits;
        while (pb < kRpMaxPBits && ((int64_t)1 << pb) * kRpTargetTags < nb) ++pb;
        while (pb < kRpMaxPBits && p.G > ((int64_t)1 << (pb - 1)) - 1) ++pb;
        const int64_t P = (int64_t)1 << pb;
        const int64_t prows = std::max<int64_t>(
            kRpSub, ceil_div(ceil_div(std::max<int64_t>(p.n_cand, 1), (int64_t)kRpScatPerCU * kCUs), (int64_t)kRpSub) *
                        kRpSub);
        const int64_t pw = ceil_div(std::max<int64_t>(p.n_cand, 1), prows);
        const int64_t n_rec = p.n_cand + (kRpUnit - 1) * P * pw;
        const int64_t nbtag_bound = nb + (kRpTagUnit - 1) * P * (ceil_div(std::max<int64_t>(nb, 1), (int64_t)kRpBSub));
        const bool can_radix = p.jm == J_KEYS && !d->sel && p.n_cand > 0 && p.G <= (P >> 1) - 1 &&
                               p.G <= kLdsMaxG && n_rec < (1ll << 31) && nbtag_bound < (1ll << 31);
        if (d->strategy == TDP_PROBE_PARTITIONED && !can_radix)
            return fail(TDP_EUNSUPPORTED, "tdp_groupby_agg: the partitioned probe needs a keys-only join without a "
                                          "selection vector, rows, and at most %d groups",
                        (1 << (kRpMaxPBits - 1)) - 1);
        p.radix = d->strategy == TDP_PROBE_PARTITIONED ||
                  (d->strategy == TDP_PROBE_AUTO && can_radix && kRpAuto && nb >= kRpAutoBuild &&
                   p.n_cand >= kRpAutoRows);
        if (p.radix) {
            p.rp_pbits = pb;
            // at most kRpBuildWgs build workgroups, so the padding of their regions
            // (under 16 tags each) stays a small part of a partition's sub-table
            p.rp_brows = std::max<int64_t>(kRpBSub, ceil_div(ceil_div(std::max<int64_t>(nb, 1), (int64_t)kRpBuildWgs),
                                                             (int64_t)kRpBSub) * kRpBSub);
            p.rp_bw = ceil_div(std::max<int64_t>(nb, 1), p.rp_brows);
            p.rp_nbtag = nb + (kRpTagUnit - 1) * P * p.rp_bw;
            p.rp_pw = pw;
            p.rp_prows = prows;
            p.rp_nrec = n_rec;
            // at most one item per partition plus one per kRpItemRec records
            p.nblocks = (int)(P + ceil_div(n_rec, (int64_t)kRpItemRec) + 1);
            if (p.acc == ACC_GLOBAL) p.acc = ACC_LDS;
        }
    }
    const bool can_stage = !p.radix && p.jm == J_KEYS && !d->sel && p.cap >= (1u << 16) &&
                           p.n_cand < (1ll << 31) - 4 * kParts && p.G < kStageMaxG;
    if (d->strategy == TDP_PROBE_STAGED && !can_stage)
        return fail(TDP_EUNSUPPORTED, "tdp_groupby_agg: the staged probe needs a keys-only join without a selection, "
                                      "a table of at least 65536 slots and fewer than 65535 groups");
    p.staged = d->strategy == TDP_PROBE_STAGED ||
               (d->strategy == TDP_PROBE_AUTO && can_stage && kStagedAuto && (int64_t)p.cap * 4 >= (32ll << 20) &&
                p.n_cand >= (1 << 22));
    if (p.staged) {
        int cbits = 0;
        while ((1u << cbits) < p.cap) ++cbits;
        p.pshift = cbits - 6;  // kParts = 64 slot ranges
        p.stage_tiles = std::max<int64_t>(1, ceil_div(p.n_cand, kStageTile));
        p.nblocks = kProbeGrid;
    }
    // Large dense tables over many rows with probe-side group keys aggregate
    // through group-range partitions instead of global atomics.
    bool keys_probe = true;
    for (int i = 0; i < d->n_keys; ++i) keys_probe &= d->key[i].side == TDP_SIDE_PROBE;
    p.pagg = !p.staged && !p.radix && p.acc == ACC_GLOBAL && !d->sel && keys_probe && d->strategy != TDP_PROBE_DIRECT &&
             p.G <= (int64_t)kPaggMaxParts * kPaggGroups && p.n_cand >= (1 << 20) && p.n_cand < (1ll << 31);
    if (p.pagg) {
        p.pagg_np = (int)ceil_div(p.G, kPaggGroups);
        p.stage_tiles = ceil_div(p.n_cand, kStageTile);
    }
    return TDP_OK;
}

struct WsLayout {
    HashView t;
    unsigned long long* gtab = nullptr;  // [G][sum, count]
    unsigned long long* part = nullptr;
    unsigned int* done = nullptr;
    uint32_t* chunk = nullptr;
    Cand* cand[2] = {nullptr, nullptr};
    BuildScratch bs;
    StageDev st{};
    PaggDev pg{};
    RpDev rp{};
    unsigned long long* zblock = nullptr;  // zeroed by the build: the accumulators
    int64_t n_zero = 0;
    size_t bytes = 0;
};

WsLayout layout(const Plan& p, const tdp_groupby_desc* d, void* ws) {
    WsLayout L;
    WsAlloc wa(ws);
    L.done = wa.take<unsigned int>(64);
    const int64_t n_acc = p.acc == ACC_REG ? 0 : 2 * p.G;
    L.n_zero = n_acc;
    L.zblock = wa.take<unsigned long long>((size_t)std::max<int64_t>(L.n_zero, 1));
    if (p.acc == ACC_REG) {
        L.part = wa.take<unsigned long long>((size_t)p.nblocks * p.G * 2);
    } else {
        L.gtab = L.zblock;
    }
    if (p.staged) {
        StageDev& st = L.st;
        const size_t nrec = (size_t)p.n_cand + 4 * kParts;
        st.rkey = wa.take<int32_t>(nrec);
        st.rgid = wa.take<uint16_t>(nrec);
        st.rval = wa.take<unsigned long long>(nrec);
        st.off = wa.take<uint32_t>((size_t)p.stage_tiles * kParts);
        st.ptot = wa.take<uint32_t>(kParts);
        st.pstart = wa.take<uint32_t>(kParts + 1);
        st.ctr = wa.take<uint32_t>(kParts);
        st.n_tiles = p.stage_tiles;
        st.pshift = p.pshift;
    }
    if (p.pagg) {
        PaggDev& pg = L.pg;
        const size_t nrec = (size_t)p.n_cand;
        pg.rg = wa.take<uint16_t>(nrec);
        pg.rc = wa.take<uint32_t>(nrec);
        pg.rv = wa.take<unsigned long long>(nrec);
        pg.off = wa.take<uint32_t>((size_t)p.stage_tiles * p.pagg_np);
        pg.ptot = wa.take<uint32_t>(p.pagg_np);
        pg.pstart = wa.take<uint32_t>(p.pagg_np + 1);
        pg.n_tiles = p.stage_tiles;
        pg.np = p.pagg_np;
    }
    if (p.radix) {
        RpDev& r = L.rp;
        r.pbits = p.rp_pbits;
        r.tbits = 32 - p.rp_pbits;
        r.P = 1 << p.rp_pbits;
        r.bw = p.rp_bw;
        r.pw = p.rp_pw;
        r.prows = p.rp_prows;
        r.n_rec = p.rp_nrec;
        const int64_t nb = d->join->n_build;
        r.brows = p.rp_brows;
        r.n_btag = p.rp_nbtag;
        r.btag = wa.take<uint32_t>((size_t)std::max<int64_t>(r.n_btag, 1));
        r.bcnt = wa.take<uint32_t>((size_t)r.bw * r.P);
        r.bstart = wa.take<uint32_t>(r.P + 1);
        r.btot = wa.take<uint32_t>(r.P);
        r.rec = wa.take<uint2>((size_t)r.n_rec);
        r.pcnt = wa.take<uint32_t>((size_t)r.pw * r.P);
        r.pstart = wa.take<uint32_t>(r.P + 1);
        r.ptot = wa.take<uint32_t>(r.P);
        r.item = wa.take<uint32_t>(r.P + 1);
    }
    if (!p.last_block_fin && !p.topk) L.chunk = wa.take<uint32_t>((size_t)ceil_div(p.G, kFinChunk));
    if (p.topk) {
        const size_t nc = (size_t)ceil_div(p.G, kTopChunk) * p.topk;
        L.cand[0] = wa.take<Cand>(nc);
        L.cand[1] = wa.take<Cand>(nc);
    }
    if (p.jm != J_NONE && !p.radix) {
        L.t = table_alloc(wa, p.kind, d->join->n_build, p.cap, p.with_sum);
        L.bs = build_scratch_alloc(wa, p.kind, d->join->n_build, p.cap, p.with_sum);
    }
    L.bytes = wa.bytes();
    return L;
}

enum SigId { SIG_GENERIC = 0, SIG_SCALED = 1, SIG_SMALL = 2, SIG_ONEKEY = 3, SIG_WHERE = 4 };

// The static signature the descriptor matches (the fast kernels read the
// probe side contiguously, so a selection vector takes the generic path).
int pick_sig(const Plan& p, const tdp_groupby_desc* d) {
    auto is = [](const tdp_col& c, int dt, int side) { return c.dtype == dt && c.side == side; };
    if (d->sel) return SIG_GENERIC;
    if (d->n_more_preds > 0) {
        if (d->has_pred && d->pred.dtype == TDP_I32 && d->n_keys == 2 && is(d->key[0], TDP_I8, TDP_SIDE_PROBE) &&
            is(d->key[1], TDP_I8, TDP_SIDE_PROBE) && p.jm == J_NONE && p.expr == TDP_EXPR_NONE)
            return SIG_WHERE;
        return SIG_GENERIC;
    }
    const bool a64 = p.a.dt == TDP_I64 && p.a.side == TDP_SIDE_PROBE;
    if (d->has_pred && d->pred.dtype == TDP_I32 && d->n_keys == 2 && is(d->key[0], TDP_I8, TDP_SIDE_PROBE) &&
        is(d->key[1], TDP_I8, TDP_SIDE_PROBE) && a64 && p.b.dt == TDP_I64 && p.b.side == TDP_SIDE_PROBE &&
        (p.jm == J_AGG ? (p.form == F_ABCNT || p.form == F_AKBCNT)
                       : (p.expr == TDP_EXPR_MUL || p.expr == TDP_EXPR_MUL_CONST_SUB)))
        return SIG_SCALED;
    if (d->has_pred && d->pred.dtype == TDP_I32 && d->n_keys == 2 && is(d->key[0], TDP_I8, TDP_SIDE_BUILD) &&
        is(d->key[1], TDP_I8, TDP_SIDE_PROBE) && a64 && p.jm == J_ROWID && p.expr == TDP_EXPR_COL)
        return SIG_SMALL;
    if (!d->has_pred && d->n_keys == 1 && is(d->key[0], TDP_I32, TDP_SIDE_PROBE) && a64 &&
        (p.jm == J_AGG ? (p.form == F_ACNT || p.form == F_ASUM || p.form == F_AKCNT_SUM) : p.expr == TDP_EXPR_COL))
        return SIG_ONEKEY;
    return SIG_GENERIC;
}

template <int ACC, int JM>
void launch_gb(const GbDev& g, bool sel, int sig, int nblocks, size_t lds, hipStream_t s) {
    if (sel) {
        groupby_kernel<ACC, JM, true, SigGeneric><<<nblocks, kThreads, lds, s>>>(g);
        return;
    }
    switch (sig) {
        case SIG_SCALED:
            groupby_kernel<ACC, JM, false, SigPredI32KeysI8I8ValI64I64><<<nblocks, kThreads, lds, s>>>(g);
            break;
        case SIG_SMALL:
            groupby_kernel<ACC, JM, false, SigPredI32BuildKeyI8KeyI8ValI64><<<nblocks, kThreads, lds, s>>>(g);
            break;
        case SIG_ONEKEY:
            groupby_kernel<ACC, JM, false, SigKeyI32ValI64><<<nblocks, kThreads, lds, s>>>(g);
            break;
        case SIG_WHERE:
            if constexpr (JM == J_NONE) {
                groupby_kernel<ACC, JM, false, SigPredI32KeysI8I8Count><<<nblocks, kThreads, lds, s>>>(g);
                break;
            }
            [[fallthrough]];
        default:
            groupby_kernel<ACC, JM, false, SigGeneric><<<nblocks, kThreads, lds, s>>>(g);
            break;
    }
}

template <int JM, class S>
void launch_pagg_sig(const GbDev& g, const PaggDev& pg, hipStream_t s) {
    const int nw = (int)std::min<int64_t>(pg.n_tiles, kStageGrid);
    pagg_hist_kernel<S><<<nw, kThreads, 0, s>>>(g, pg);
    pagg_colscan_kernel<<<pg.np, 256, 0, s>>>(pg);
    pagg_start_kernel<<<1, 256, 0, s>>>(pg);
    pagg_stage_kernel<JM, S><<<nw, kThreads, 0, s>>>(g, pg);
    pagg_reduce_kernel<<<pg.np, kPaggRedThreads, 0, s>>>(g, pg);
}

template <int JM>
void launch_pagg_jm(const GbDev& g, const PaggDev& pg, int sig, hipStream_t s) {
    switch (sig) {
        case SIG_SCALED: launch_pagg_sig<JM, SigPredI32KeysI8I8ValI64I64>(g, pg, s); break;
        case SIG_ONEKEY: launch_pagg_sig<JM, SigKeyI32ValI64>(g, pg, s); break;
        default: launch_pagg_sig<JM, SigGeneric>(g, pg, s); break;
    }
}

void launch_pagg(const GbDev& g, const PaggDev& pg, int jm, int sig, hipStream_t s) {
    switch (jm) {
        case J_NONE: launch_pagg_jm<J_NONE>(g, pg, sig, s); break;
        case J_KEYS: launch_pagg_jm<J_KEYS>(g, pg, sig, s); break;
        case J_ROWID: launch_pagg_jm<J_ROWID>(g, pg, sig, s); break;
        default: launch_pagg_jm<J_AGG>(g, pg, sig, s); break;
    }
}

template <int ACC>
void launch_gb_acc(const GbDev& g, int jm, bool sel, int sig, int nblocks, size_t lds, hipStream_t s) {
    switch (jm) {
        case J_NONE: launch_gb<ACC, J_NONE>(g, sel, sig, nblocks, lds, s); break;
        case J_KEYS: launch_gb<ACC, J_KEYS>(g, sel, sig, nblocks, lds, s); break;
        case J_ROWID: launch_gb<ACC, J_ROWID>(g, sel, sig, nblocks, lds, s); break;
        default: launch_gb<ACC, J_AGG>(g, sel, sig, nblocks, lds, s); break;
    }
}

}  // namespace

}  // namespace tdp

using namespace tdp;

extern "C" size_t tdp_groupby_workspace_size(const tdp_groupby_desc* d) {
    Plan p;
    if (make_plan(d, p)) return 0;
    return layout(p, d, nullptr).bytes;
}

namespace {

GbDev make_dev(const Plan& p, const WsLayout& L, const tdp_groupby_desc* d, const tdp_groupby_out* o,
               int32_t* d_status) {
    GbDev g{};
    g.n_cand = p.n_cand;
    g.sel = d->sel;
    g.has_pred = d->has_pred;
    g.pred_cmp = d->pred_cmp;
    g.pred_lit = d->pred_literal;
    g.pred = coldev(d->pred);
    g.n_more = d->n_more_preds;
    for (int i = 0; i < d->n_more_preds; ++i) {
        g.more[i].col = coldev(d->more_preds[i].col);
        g.more[i].cmp = d->more_preds[i].cmp;
        g.more[i].lit = d->more_preds[i].literal;
        g.more[i].litf = (float)d->more_preds[i].literal_f;
    }
    g.probe_key = d->join ? d->join->probe_key : nullptr;
    g.t = L.t;
    g.n_keys = d->n_keys;
    g.expr = p.expr;
    g.form = p.form;
    for (int i = 0; i < 2; ++i) {
        g.key[i] = i < d->n_keys ? coldev(d->key[i]) : ColDev();
        g.lo[i] = i < d->n_keys ? d->key_lo[i] : 0;
        g.card[i] = i < d->n_keys ? d->key_card[i] : 1;
    }
    g.a = p.a;
    g.b = p.b;
    g.k = d->k;
    g.G = p.G;
    g.gtab = L.gtab;
    g.part = L.part;
    g.done = L.done;
    g.status = d_status;
    g.last_block_fin = p.last_block_fin || p.n_cand == 0;  // no rows: one workgroup emits zero groups
    g.n_parts_dev = p.radix ? L.rp.item + (1 << p.rp_pbits) : nullptr;  // the partitioned probe's work items
    g.d_n_groups = o->d_n_groups;
    g.okey0 = o->key0;
    g.okey1 = o->key1;
    g.osum = o->sum;
    g.ocnt = o->count;
    g.oavg = o->avg;
    return g;
}

int check_out(const Plan& p, const tdp_groupby_desc* d, const tdp_groupby_out* o) {
    if (!o || !o->d_n_groups || !o->key0 || !o->sum || !o->count || !o->avg)
        return fail(TDP_EINVAL, "tdp_groupby_agg: null output");
    if (d->n_keys > 1 && !o->key1) return fail(TDP_EINVAL, "tdp_groupby_agg: key1 output is null");
    const int64_t need = p.topk ? std::min<int64_t>(p.G, p.topk) : p.G;
    if (o->cap < need) return fail_need(TDP_ECAPACITY, need, "tdp_groupby_agg: cap %lld < %lld groups", (long long)o->cap, (long long)need);
    return TDP_OK;
}

int prepare(const tdp_groupby_desc* d, void* ws, size_t ws_bytes, Plan& p, WsLayout& L) {
    int rc = make_plan(d, p);
    if (rc) return rc;
    L = layout(p, d, nullptr);
    if (!ws || ws_bytes < L.bytes) return fail_need(TDP_EWORKSPACE, (int64_t)L.bytes, "tdp_groupby_agg: workspace %zu < %zu", ws_bytes, L.bytes);
    if ((uintptr_t)ws & 255) return fail(TDP_EINVAL, "tdp_groupby_agg: workspace not 256-byte aligned");
    L = layout(p, d, ws);
    return TDP_OK;
}

// Clear the table and the accumulators, then insert the build side.  Every
// probe leaves the accumulators zero again, so one build serves many probes.
int run_build(const Plan& p, const WsLayout& L, const tdp_groupby_desc* d, int32_t* d_status, hipStream_t stream) {
    const int64_t n_zero = L.n_zero;
    if (p.radix) {
        const int ib = (int)std::min<int64_t>(std::max<int64_t>(ceil_div(n_zero, 256), 1), 1024);
        gb_init_kernel<<<ib, 256, 0, stream>>>(L.zblock, n_zero, d_status, L.done);
        RpDev r = L.rp;
        r.status = d_status;
        const int64_t nb = d->join->n_build;
        rp_count_kernel<<<(uint32_t)r.bw, kRpThreads, 0, stream>>>(d->join->build_key, nb, r.bw, r.brows, r.bcnt, r.P,
                                                                   r.tbits, kRpTagUnit);
        rp_colscan_kernel<<<r.P / kRpScanCols, 1024, 0, stream>>>(r.bcnt, r.bw, r.P, r.btot);
        rp_start_kernel<<<1, kRpMaxP, 0, stream>>>(r.P, r.btot, r.bstart, nullptr);
        if (nb > 0) rp_build_scatter_kernel<<<(uint32_t)r.bw, kRpThreads, 0, stream>>>(d->join->build_key, nb, r);
        return launch_status("tdp_groupby_build");
    }
    if (p.jm != J_NONE) {
        int rc = table_clear_zero(L.t, !L.bs.lds, d_status, L.done, L.zblock, n_zero, stream);
        if (rc) return rc;
        return table_build(L.t, L.bs, p.kind, d->join->build_key, d->join->n_build, d->join->build_unique != 0,
                           p.bvals, p.bdt, d_status, stream);
    }
    const int ib = (int)std::min<int64_t>(std::max<int64_t>(ceil_div(n_zero, 256), 1), 1024);
    gb_init_kernel<<<ib, 256, 0, stream>>>(L.zblock, n_zero, d_status, L.done);
    return launch_status("tdp_groupby_build");
}

int run_probe(const Plan& p, const WsLayout& L, const tdp_groupby_desc* d, const tdp_groupby_out* o,
              int32_t* d_status, hipStream_t stream) {
    GbDev g = make_dev(p, L, d, o, d_status);
    const size_t lds = p.acc == ACC_LDS ? (size_t)p.G * 2 * sizeof(unsigned long long) : 0;
    const bool sel = d->sel != nullptr;
    const int sig = pick_sig(p, d);
    if (p.radix) {
        const RpDev& r = L.rp;
        rp_count_kernel<<<(uint32_t)r.pw, kRpThreads, 0, stream>>>(d->join->probe_key, p.n_cand, r.pw, r.prows, r.pcnt,
                                                                   r.P, r.tbits, kRpUnit);
        rp_colscan_kernel<<<r.P / kRpScanCols, 1024, 0, stream>>>(r.pcnt, r.pw, r.P, r.ptot);
        rp_start_kernel<<<1, kRpMaxP, 0, stream>>>(r.P, r.ptot, r.pstart, r.item);
        stage_mark(TDP_STAGE_RP_SCATTER, 0, stream);
        switch (sig) {
            case SIG_SCALED: rp_scatter_kernel<SigPredI32KeysI8I8ValI64I64><<<(uint32_t)r.pw, kRpScatThreads, 0, stream>>>(g, r); break;
            case SIG_ONEKEY: rp_scatter_kernel<SigKeyI32ValI64><<<(uint32_t)r.pw, kRpScatThreads, 0, stream>>>(g, r); break;
            default: rp_scatter_kernel<SigGeneric><<<(uint32_t)r.pw, kRpScatThreads, 0, stream>>>(g, r); break;
        }
        stage_mark(TDP_STAGE_RP_SCATTER, 1, stream);
        const int dup = d->join->build_unique ? 1 : 0;
        stage_mark(TDP_STAGE_RP_PROBE, 0, stream);
        if (p.acc == ACC_REG)
            rp_probe_kernel<ACC_REG><<<p.nblocks, kRpProbeThreads, 0, stream>>>(g, r, dup);
        else
            rp_probe_kernel<ACC_LDS><<<p.nblocks, kRpProbeThreads, lds, stream>>>(g, r, dup);
        stage_mark(TDP_STAGE_RP_PROBE, 1, stream);
    } else if (p.staged && p.n_cand > 0) {
        const int nw = (int)std::min<int64_t>(L.st.n_tiles, kStageGrid);
        switch (sig) {
            case SIG_SCALED: stage_hist_kernel<SigPredI32KeysI8I8ValI64I64><<<nw, kThreads, 0, stream>>>(g, L.st); break;
            case SIG_ONEKEY: stage_hist_kernel<SigKeyI32ValI64><<<nw, kThreads, 0, stream>>>(g, L.st); break;
            default: stage_hist_kernel<SigGeneric><<<nw, kThreads, 0, stream>>>(g, L.st); break;
        }
        stage_colscan_kernel<<<kParts, 256, 0, stream>>>(L.st);
        stage_start_kernel<<<1, kWave, 0, stream>>>(L.st);
        switch (sig) {
            case SIG_SCALED: stage_kernel<SigPredI32KeysI8I8ValI64I64><<<nw, kThreads, 0, stream>>>(g, L.st); break;
            case SIG_ONEKEY: stage_kernel<SigKeyI32ValI64><<<nw, kThreads, 0, stream>>>(g, L.st); break;
            default: stage_kernel<SigGeneric><<<nw, kThreads, 0, stream>>>(g, L.st); break;
        }
        switch (p.acc) {
            case ACC_REG: stage_probe_kernel<ACC_REG><<<kProbeGrid, kThreads, lds, stream>>>(g, L.st); break;
            case ACC_LDS: stage_probe_kernel<ACC_LDS><<<kProbeGrid, kThreads, lds, stream>>>(g, L.st); break;
            default: stage_probe_kernel<ACC_GLOBAL><<<kProbeGrid, kThreads, lds, stream>>>(g, L.st); break;
        }
    } else if (p.pagg && p.n_cand > 0) {
        launch_pagg(g, L.pg, p.jm, sig, stream);
    } else {
        stage_mark(TDP_STAGE_FUSED_PROBE, 0, stream);
        switch (p.acc) {
            case ACC_REG: launch_gb_acc<ACC_REG>(g, p.jm, sel, sig, p.nblocks, lds, stream); break;
            case ACC_LDS: launch_gb_acc<ACC_LDS>(g, p.jm, sel, sig, p.nblocks, lds, stream); break;
            default: launch_gb_acc<ACC_GLOBAL>(g, p.jm, sel, sig, p.nblocks, lds, stream); break;
        }
        stage_mark(TDP_STAGE_FUSED_PROBE, 1, stream);
    }
    const int n_parts = p.staged && p.n_cand > 0 ? kProbeGrid : p.nblocks;  // radix: one partial per item workgroup
    if (g.last_block_fin) {
        switch (p.acc) {
            case ACC_REG: finalize_small_kernel<ACC_REG><<<1, kFinRegThreads, 0, stream>>>(g, n_parts); break;
            case ACC_LDS: finalize_small_kernel<ACC_LDS><<<1, kThreads, 0, stream>>>(g, n_parts); break;
            default: finalize_small_kernel<ACC_GLOBAL><<<1, kThreads, 0, stream>>>(g, n_parts); break;
        }
    } else if (p.topk && p.n_cand > 0) {
        int64_t n = p.G;
        int64_t nb = ceil_div(n, kTopChunk);
        if (nb == 1) {
            topk_stage_kernel<<<1, kTopThreads, 0, stream>>>(g, nullptr, n, p.topk, nullptr, 1, 1);
        } else {
            topk_stage_kernel<<<(uint32_t)nb, kTopThreads, 0, stream>>>(g, nullptr, n, p.topk, L.cand[0], 1, 0);
            n = nb * p.topk;
            int cur = 0;
            while (n > kTopChunk) {
                nb = ceil_div(n, kTopChunk);
                topk_stage_kernel<<<(uint32_t)nb, kTopThreads, 0, stream>>>(g, L.cand[cur], n, p.topk, L.cand[1 - cur], 0, 0);
                cur = 1 - cur;
                n = nb * p.topk;
            }
            topk_stage_kernel<<<1, kTopThreads, 0, stream>>>(g, L.cand[cur], n, p.topk, nullptr, 0, 1);
        }
    } else if (!g.last_block_fin) {
        const int64_t n_chunks = ceil_div(p.G, kFinChunk);
        fin_count_kernel<<<(uint32_t)n_chunks, kThreads, 0, stream>>>(g, L.chunk);
        fin_scan_kernel<<<1, kThreads, 0, stream>>>(L.chunk, n_chunks, o->d_n_groups);
        fin_write_kernel<<<(uint32_t)n_chunks, kThreads, 0, stream>>>(g, L.chunk);
    }
    return launch_status("tdp_groupby_probe");
}

}  // namespace

extern "C" int tdp_groupby_agg(const tdp_groupby_desc* d, const tdp_groupby_out* o, int32_t* d_status, void* ws,
                               size_t ws_bytes, hipStream_t stream) {
    Plan p;
    WsLayout L;
    int rc = prepare(d, ws, ws_bytes, p, L);
    if (rc) return rc;
    if ((rc = check_out(p, d, o))) return rc;
    if ((rc = run_build(p, L, d, d_status, stream))) return rc;
    return run_probe(p, L, d, o, d_status, stream);
}

extern "C" int tdp_groupby_build(const tdp_groupby_desc* d, int32_t* d_status, void* ws, size_t ws_bytes,
                                 hipStream_t stream) {
    Plan p;
    WsLayout L;
    int rc = prepare(d, ws, ws_bytes, p, L);
    if (rc) return rc;
    return run_build(p, L, d, d_status, stream);
}

extern "C" int tdp_groupby_probe(const tdp_groupby_desc* d, const tdp_groupby_out* o, int32_t* d_status, void* ws,
                                 size_t ws_bytes, hipStream_t stream) {
    Plan p;
    WsLayout L;
    int rc = prepare(d, ws, ws_bytes, p, L);
    if (rc) return rc;
    if ((rc = check_out(p, d, o))) return rc;
    return run_probe(p, L, d, o, d_status, stream);
}
