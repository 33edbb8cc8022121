// Hash equi-join: build an open-addressing table from the build keys, then
// stream the probe side through it.
#include "hash.hpp"

namespace tdp {

namespace {

// Resets slots [first, n_slots): every slot, or only the extra slot `cap`
// (which holds the kEmpty key's presence flag) when an LDS build writes the
// rest.
__global__ void table_clear_kernel(HashView t, int64_t first, int64_t n_slots, int32_t* d_status,
                                   unsigned long long* d_counter, unsigned int* d_done, unsigned long long* zero,
                                   int64_t n_zero) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n = (n_slots - first) > n_zero ? (n_slots - first) : n_zero;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (i < n_slots - first) {
            const int64_t j = first + i;
            const bool extra = j == n_slots - 1;
            if (t.rec) {
                AggRec r;
                r.key = extra ? 0 : kEmpty;
                r.cnt = 0;
                r.sum = 0;
                t.rec[j] = r;
            } else {
                t.keys[j] = extra ? 0 : kEmpty;
            }
            if (t.head) t.head[j] = -1;
        }
        if (i < n_zero) zero[i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (d_status) *d_status = 0;
        if (d_counter) *d_counter = 0;
        if (d_done) *d_done = 0;
    }
}

template <int KIND>
__global__ __launch_bounds__(256) void table_build_kernel(HashView t, const int32_t* __restrict__ bkey, int64_t n,
                                                          int unique, const void* __restrict__ bvals, int bdt,
                                                          int32_t* status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        if (KIND == TABLE_AGG) {
            const int64_t slot = agg_insert(t, bkey[j]);
            if (slot < 0)
                raise_flag(status, TDP_FLAG_TABLE_FULL);
            else
                agg_add(t, slot, 1u, t.with_sum ? (unsigned long long)load_int(bvals, bdt, j) : 0ull);
            continue;
        }
        bool fresh;
        const int64_t slot = ht_insert(t, bkey[j], fresh);
        if (slot < 0) {
            raise_flag(status, TDP_FLAG_TABLE_FULL);
            continue;
        }
        if (unique && !fresh) raise_flag(status, TDP_FLAG_DUP_BUILD);
        if (KIND == TABLE_ROWID) {
            if (fresh) t.rowid[slot] = (int32_t)j;
        } else if (KIND == TABLE_LIST) {
            t.next[j] = atomicExch(&t.head[slot], (int32_t)j);
        }
    }
}

// Inclusive scan of per-lane counts across the wave.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t u = __shfl_up(v, off, kWave);
        if (lane >= off) v += u;
    }
    return v;
}

template <bool PAIRS>
__global__ __launch_bounds__(256) void join_probe_kernel(HashView t, const int32_t* __restrict__ pkey,
                                                         const int32_t* __restrict__ psel, int64_t n_cand,
                                                         int32_t* __restrict__ out_p, int32_t* __restrict__ out_b,
                                                         int64_t cap, unsigned long long* d_total) {
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; c0 < n_cand; c0 += stride) {
        const int64_t c = c0 + lane;
        int32_t row = -1, first = -1;
        uint32_t count = 0;
        if (c < n_cand) {
            row = psel ? psel[c] : (int32_t)c;
            const int64_t slot = ht_find(t.keys, t.mask, t.bmask, pkey[row]);
            if (slot >= 0) {
                first = t.head[slot];
                for (int32_t j = first; j >= 0; j = t.next[j]) ++count;
            }
        }
        const uint32_t incl = wave_inclusive_scan(count);
        const uint32_t total = __shfl(incl, kWave - 1, kWave);
        if (total == 0) continue;
        unsigned long long base = 0;
        if (lane == kWave - 1) base = atomicAdd(d_total, (unsigned long long)total);
        base = __shfl(base, kWave - 1, kWave);
        if (PAIRS && count) {
            int64_t pos = (int64_t)base + incl - count;
            for (int32_t j = first; j >= 0 && pos < cap; j = t.next[j], ++pos) {
                out_p[pos] = row;
                out_b[pos] = j;
            }
        }
    }
}

// Workgroup-wide exclusive scan of one value per thread; *total receives the
// sum.  Uses s_w[blockDim.x / 64]; its barriers order LDS only.
__device__ __forceinline__ uint32_t block_scan_u32(uint32_t v, uint32_t* s_w, uint32_t* total) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const uint32_t a = wave_inclusive_scan(v);
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

// ---- LDS build: bucket the build rows by probing block, then build each
// block in LDS and write it out whole (no global atomics on the table).

// Build group of a key: its table slot >> log2(slots per group).
__device__ __forceinline__ uint32_t block_of(int32_t key, uint32_t mask, int gshift) {
    return (hash32((uint32_t)key) & mask) >> gshift;
}

// Calls f(i, key) for the build rows [lo, hi) a workgroup of T threads
// owns, four keys per thread and step when the column is 16-byte aligned (lo
// is a multiple of 4 then), so each thread keeps four loads in flight.
template <int T, class F>
__device__ __forceinline__ void for_chunk_keys(const int32_t* __restrict__ bkey, int64_t lo, int64_t hi, F f) {
    if (((uintptr_t)bkey & 15) == 0) {
        int64_t i = lo + (int64_t)threadIdx.x * 4;
        for (; i + 4 <= hi; i += T * 4) {
            const int4 q = *(const int4*)(bkey + i);
            f(i, q.x);
            f(i + 1, q.y);
            f(i + 2, q.z);
            f(i + 3, q.w);
        }
        for (; i < hi; ++i) f(i, bkey[i]);
    } else {
        for (int64_t i = lo + threadIdx.x; i < hi; i += T) f(i, bkey[i]);
    }
}

template <int T>
__global__ __launch_bounds__(T) void lb_hist_kernel(const int32_t* __restrict__ bkey, int64_t n, int64_t chunk,
                                                      uint32_t mask, int gshift, uint32_t nblk, uint32_t* mat,
                                                      uint32_t unit) {
    extern __shared__ uint32_t h[];
    for (uint32_t b = threadIdx.x; b < nblk; b += T) h[b] = 0;
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    for_chunk_keys<T>(bkey, lo, hi, [&](int64_t, int32_t key) { atomicAdd(&h[block_of(key, mask, gshift)], 1u); });
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nblk; b += T) mat[(int64_t)blockIdx.x * nblk + b] = (h[b] + unit - 1) / unit * unit;
}

// Per block b: exclusive prefix of mat[.][b] over the histogram workgroups,
// in place; tot[b] = the total.  A workgroup takes 64 blocks, its four
// waves one contiguous quarter of the rows each.
__global__ __launch_bounds__(256) void lb_colscan_kernel(uint32_t* mat, int nw, uint32_t nblk, uint32_t* tot) {
    __shared__ uint32_t s_seg[4][64];
    const int c = threadIdx.x & 63, r = threadIdx.x >> 6;
    const uint32_t b = blockIdx.x * 64 + c;
    const int seg = (nw + 3) / 4;
    const int w0 = r * seg, w1 = w0 + seg < nw ? w0 + seg : nw;
    uint32_t sum = 0;
    if (b < nblk)
        for (int w = w0; w < w1; ++w) sum += mat[(int64_t)w * nblk + b];
    s_seg[r][c] = sum;
    __syncthreads();
    uint32_t run = 0;
    for (int q = 0; q < r; ++q) run += s_seg[q][c];
    if (b < nblk) {
        for (int w = w0; w < w1; ++w) {
            const uint32_t v = mat[(int64_t)w * nblk + b];
            mat[(int64_t)w * nblk + b] = run;
            run += v;
        }
        if (r == 3) tot[b] = run;
    }
}

// base[b] = sum of tot[0..b) (in place over tot, one workgroup; each thread
// takes a contiguous run of blocks), base[nblk] = total.
__global__ __launch_bounds__(256) void lb_basescan_kernel(uint32_t* tot, uint32_t nblk) {
    __shared__ uint32_t s_w[4];
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const uint32_t per = (nblk + 255) / 256;
    const uint32_t b0 = threadIdx.x * per, b1 = b0 + per < nblk ? b0 + per : nblk;
    uint32_t sum = 0;
    for (uint32_t b = b0; b < b1; ++b) sum += tot[b];
    const uint32_t incl = wave_inclusive_scan(sum);
    if (lane == kWave - 1) s_w[wave] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int w = 0; w < wave; ++w) run += s_w[w];
    for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t v = tot[b];
        tot[b] = run;
        run += v;
    }
    if (threadIdx.x == 255) tot[nblk] = run;
}

template <int T>
__global__ __launch_bounds__(T) void lb_scatter_kernel(const int32_t* __restrict__ bkey, int64_t n, int64_t chunk,
                                                         uint32_t mask, int gshift, uint32_t nblk, const uint32_t* mat,
                                                         const uint32_t* base, int32_t* skeys, int32_t* srows,
                                                         const void* __restrict__ bvals, int bdt, AggIn* srec) {
    extern __shared__ uint32_t cur[];
    for (uint32_t b = threadIdx.x; b < nblk; b += T) cur[b] = base[b] + mat[(int64_t)blockIdx.x * nblk + b];
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    for_chunk_keys<T>(bkey, lo, hi, [&](int64_t i, int32_t key) {
        const uint32_t pos = atomicAdd(&cur[block_of(key, mask, gshift)], 1u);
        if (srec) {
            AggIn r;
            r.key = key;
            r.pad = 0;
            r.val = (unsigned long long)load_int(bvals, bdt, i);
            srec[pos] = r;
        } else {
            skeys[pos] = key;
            if (srows) srows[pos] = (int32_t)i;
        }
    });
}

// Aggregate build rows -> 16-byte records in whole 64-byte units.  Workgroup
// w takes the rows [w * chunk, (w + 1) * chunk) in sub-chunks of kAggSub
// (four consecutive rows per thread); per sub-chunk each row is ranked in its
// build group by an LDS counter, the records are ordered by group in LDS,
// every whole unit of kAggUnit records is written (the group's carried
// records first) and the rest is carried to the next sub-chunk; the last unit
// of each of the workgroup's runs is padded with records marked pad = 1.
// Each thread owns kPpt consecutive groups in the per-group steps.
constexpr int kAggMaxUnits = (kAggSub + (int)kAggUnitMaxBlk * (kAggUnit - 1)) / kAggUnit;
__global__ __launch_bounds__(kAggScatThreads) void lb_scatter_units_kernel(const int32_t* __restrict__ bkey, int64_t n,
                                                                        int64_t chunk, uint32_t mask, int gshift,
                                                                        uint32_t nblk, const uint32_t* mat,
                                                                        const uint32_t* base,
                                                                        const void* __restrict__ bvals, int bdt,
                                                                        AggIn* srec, int32_t* status) {
    constexpr int kPpt = ((int)kAggUnitMaxBlk + kAggScatThreads - 1) / kAggScatThreads;
    constexpr int kTpu = kAggUnit;  // threads per unit, one 16-byte record each
    __shared__ AggIn s_rec[kAggSub];
    __shared__ AggIn s_carry[kAggUnitMaxBlk][kAggUnit];
    __shared__ uint32_t s_cnt[kAggUnitMaxBlk];
    __shared__ uint16_t s_pref[kAggUnitMaxBlk];
    __shared__ uint16_t s_uoff[kAggUnitMaxBlk];
    __shared__ uint8_t s_cc[kAggUnitMaxBlk];
    __shared__ uint32_t s_cur[kAggUnitMaxBlk];
    __shared__ uint32_t s_end[kAggUnitMaxBlk];
    __shared__ uint16_t s_umap[kAggMaxUnits];
    __shared__ uint32_t s_w[kAggScatThreads / kWave];
    __shared__ uint32_t s_units;
    const int64_t w = blockIdx.x;
    const int tid = threadIdx.x, nw = gridDim.x;
    for (uint32_t b = tid; b < nblk; b += kAggScatThreads) {
        s_cur[b] = base[b] + mat[w * nblk + b];
        s_end[b] = base[b] + (w + 1 < nw ? mat[(w + 1) * nblk + b] : base[b + 1] - base[b]);
        s_cc[b] = 0;
        s_cnt[b] = 0;
    }
    lds_barrier();
    const int64_t lo = w * chunk, hi = lo + chunk < n ? lo + chunk : n;
    for (int64_t s0 = lo; s0 < hi; s0 += kAggSub) {
        const int64_t r0 = s0 + (int64_t)tid * 4;
        int32_t k[4];
        if (r0 + 4 <= hi && ((uintptr_t)(bkey + r0) & 15) == 0) {
            const int4 q = *(const int4*)(bkey + r0);
            k[0] = q.x; k[1] = q.y; k[2] = q.z; k[3] = q.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) k[e] = r0 + e < hi ? bkey[r0 + e] : 0;
        }
        AggIn rec[4];
        uint32_t rk[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            rec[e].key = k[e];
            rec[e].pad = 0u;
            rec[e].val = r0 + e < hi ? (unsigned long long)load_int(bvals, bdt, r0 + e) : 0ull;
            rk[e] = r0 + e < hi ? block_of(k[e], mask, gshift) : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (rk[e] != 0xFFFFFFFFu) rk[e] |= atomicAdd(&s_cnt[rk[e]], 1u) << 16;
        lds_barrier();
        {
            uint32_t cu[kPpt], sum = 0;
#pragma unroll
            for (int j = 0; j < kPpt; ++j) {
                const uint32_t b = tid * kPpt + j;
                cu[j] = 0;
                if (b < nblk) {
                    const uint32_t c = s_cnt[b];
                    cu[j] = c | (((s_cc[b] + c) / kAggUnit) << 16);
                }
                sum += cu[j];
            }
            uint32_t tot;
            uint32_t ex = block_scan_u32(sum, s_w, &tot);
#pragma unroll
            for (int j = 0; j < kPpt; ++j) {
                const uint32_t b = tid * kPpt + j;
                if (b < nblk) {
                    s_pref[b] = (uint16_t)(ex & 0xFFFFu);
                    s_uoff[b] = (uint16_t)(ex >> 16);
                }
                ex += cu[j];
            }
            if (tid == 0) s_units = tot >> 16;
        }
        lds_barrier();
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (rk[e] != 0xFFFFFFFFu) s_rec[s_pref[rk[e] & 0xFFFFu] + (rk[e] >> 16)] = rec[e];
        for (uint32_t b = tid; b < nblk; b += kAggScatThreads) {
            const uint32_t u0 = s_uoff[b], nu = (s_cc[b] + s_cnt[b]) / kAggUnit;
            for (uint32_t q = 0; q < nu; ++q) s_umap[u0 + q] = (uint16_t)b;
        }
        lds_barrier();
        const uint32_t n_units = s_units;
        for (uint32_t t = tid; t < n_units * kTpu; t += kAggScatThreads) {
            const uint32_t u = t / kTpu;
            const uint32_t b = s_umap[u];
            const uint32_t cc = s_cc[b];
            const uint32_t v = (u - s_uoff[b]) * kAggUnit + t % kTpu;
            const AggIn a = v < cc ? s_carry[b][v] : s_rec[s_pref[b] + v - cc];
            const uint32_t at = s_cur[b] + v;
            if (at < s_end[b]) srec[at] = a;
            else raise_flag(status, TDP_FLAG_TABLE_FULL);  // cannot happen: the histogram sized the run
        }
        lds_barrier();
        for (uint32_t b = tid; b < nblk; b += kAggScatThreads) {
            const uint32_t c = s_cnt[b], cc = s_cc[b], pf = s_pref[b];
            const uint32_t all = cc + c, used = all / kAggUnit * kAggUnit;
            if (used > 0) {
                for (uint32_t v = used; v < all; ++v) s_carry[b][v - used] = s_rec[pf + v - cc];
                s_cur[b] += used;
            } else {
                for (uint32_t q = 0; q < c; ++q) s_carry[b][cc + q] = s_rec[pf + q];
            }
            s_cc[b] = (uint8_t)(all - used);
            s_cnt[b] = 0;
        }
        lds_barrier();
    }
    for (uint32_t b = tid; b < nblk; b += kAggScatThreads) {
        const uint32_t cc = s_cc[b], at = s_cur[b];
        if (cc == 0) continue;
        if (at + kAggUnit <= s_end[b]) {
            for (uint32_t v = 0; v < (uint32_t)kAggUnit; ++v) {
                AggIn a;
                if (v < cc) {
                    a = s_carry[b][v];
                } else {
                    a.key = kEmpty;
                    a.pad = 1u;
                    a.val = 0ull;
                }
                srec[at + v] = a;
            }
        } else {
            raise_flag(status, TDP_FLAG_TABLE_FULL);
        }
    }
}

// One workgroup of T threads per build group (measured best: 1024 for the
// skewed 20M-row aggregate build, 0.83 -> 0.77 ms; 512 for the 15M-key
// build): insert the group's bucketed rows into an
// LDS copy of its probing blocks (linear probing wraps inside each 4096-slot
// block, as in the global table), then write the blocks out whole.
// Aggregate tables keep (count, sum) per slot in LDS.  (Folding the lanes of a wave that share
// a key before the LDS update measured slower on the skewed many-to-many
// build than letting LDS serialise the same-address atomics.)
template <int KIND, int T>
__global__ __launch_bounds__(T) void lb_build_kernel(HashView t, const int32_t* __restrict__ skeys,
                                                       const int32_t* __restrict__ srows,
                                                       const AggIn* __restrict__ srec,
                                                       const uint32_t* base, uint32_t gslots, int unique,
                                                       int32_t* status) {
    constexpr bool ROWID = KIND == TABLE_ROWID;
    constexpr bool AGG = KIND == TABLE_AGG;
    // dynamic LDS sized to the group: keys [gslots], then row ids [gslots]
    // or counts [gslots] (32 bits: n_build < 2^31) and sums [gslots]
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    int32_t* tk = (int32_t*)lds_raw;
    int32_t* tr = tk + gslots;
    uint32_t* tc = (uint32_t*)(tk + gslots);
    unsigned long long* ts = (unsigned long long*)(tc + gslots);
    __shared__ int s_full;  // the block overflowed: the result is invalid, stop inserting
    const bool with_sum = AGG && t.with_sum;
    const uint32_t b = blockIdx.x;
    for (uint32_t j = threadIdx.x; j < gslots; j += T) {
        tk[j] = kEmpty;
        if (AGG) tc[j] = ts[j] = 0;
    }
    if (threadIdx.x == 0) s_full = 0;
    __syncthreads();
    const uint32_t lo = base[b];
    // an aggregate group takes its first kBuildSegRows rows here; lb_merge_kernel the rest
    const uint32_t hi = AGG && base[b + 1] - lo > kBuildSegRows ? lo + kBuildSegRows : base[b + 1];
    // insert one row
    auto insert = [&](uint32_t i, bool act, int32_t key, unsigned long long v) {
        const unsigned long long c = 1;
        if (!act) return;
        if (key == kEmpty) {
            if (AGG) {
                agg_add(t, agg_insert(t, key), (uint32_t)c, v);
                return;
            }
            bool fresh;
            const int64_t slot = ht_insert(t, key, fresh);
            if (unique && !fresh) raise_flag(status, TDP_FLAG_DUP_BUILD);
            if (ROWID && fresh) t.rowid[slot] = srows[i];
            return;
        }
        uint32_t s = (hash32((uint32_t)key) & t.mask) & (gslots - 1);  // slot within the group
        bool placed = false;
        for (uint32_t probe = 0; probe < kTableBlock; ++probe) {
            const int32_t prev = atomicCAS(&tk[s], kEmpty, key);
            if (prev == kEmpty || prev == key) {
                if (prev == key && unique) raise_flag(status, TDP_FLAG_DUP_BUILD);
                if (ROWID && prev == kEmpty) tr[s] = srows[i];
                if (AGG) {
                    atomicAdd(&tc[s], (uint32_t)c);
                    if (with_sum) atomicAdd(&ts[s], v);
                }
                placed = true;
                break;
            }
            s = (s & ~(kTableBlock - 1)) | ((s + 1) & (kTableBlock - 1));  // wrap inside the block
        }
        if (!placed) {
            raise_flag(status, TDP_FLAG_TABLE_FULL);
            s_full = 1;
        }
    };
    // four rows per thread per step, all loaded before the first insert, so
    // a block with many rows (a skewed key) is not bound by load latency
    for (uint32_t i0 = lo; i0 < hi; i0 += 4 * T) {
        if (__builtin_amdgcn_readfirstlane(*(volatile int*)&s_full)) break;  // whole waves leave together
        int32_t kk[4];
        unsigned long long vv[4];
        bool pd[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t i = i0 + j * T + threadIdx.x;
            if (srec) {
                const AggIn r = i < hi ? srec[i] : AggIn{0, 1u, 0ull};
                kk[j] = r.key;
                vv[j] = r.val;
                pd[j] = r.pad != 0u;
            } else {
                kk[j] = i < hi ? skeys[i] : 0;
                vv[j] = 0ull;
                pd[j] = false;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t i = i0 + j * T + threadIdx.x;
            insert(i, i < hi && !pd[j], kk[j], vv[j]);
        }
    }
    __syncthreads();
    const int64_t off = (int64_t)b * gslots;
    for (uint32_t j = threadIdx.x; j < gslots; j += T) {
        if (AGG) {
            AggRec r;
            r.key = tk[j];
            r.cnt = tc[j];
            r.sum = ts[j];
            t.rec[off + j] = r;
        } else {
            t.keys[off + j] = tk[j];
            if (ROWID) t.rowid[off + j] = tr[j];
        }
    }
}

// One workgroup: xseg[b] = extra segments of the groups before b (a group
// of c rows has ceil(c / kBuildSegRows) - 1), xseg[nblk] = their total.
__global__ __launch_bounds__(256) void lb_segscan_kernel(const uint32_t* base, uint32_t nblk, uint32_t* xseg) {
    __shared__ uint32_t s_w[4];
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const uint32_t per = (nblk + 255) / 256;
    const uint32_t b0 = threadIdx.x * per, b1 = b0 + per < nblk ? b0 + per : nblk;
    auto extra = [&](uint32_t b) {
        const uint32_t c = base[b + 1] - base[b];
        return c > kBuildSegRows ? (c - 1) / kBuildSegRows : 0u;
    };
    uint32_t sum = 0;
    for (uint32_t b = b0; b < b1; ++b) sum += extra(b);
    const uint32_t incl = wave_inclusive_scan(sum);
    if (lane == kWave - 1) s_w[wave] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int w = 0; w < wave; ++w) run += s_w[w];
    for (uint32_t b = b0; b < b1; ++b) {
        xseg[b] = run;
        run += extra(b);
    }
    if (threadIdx.x == 255) xseg[nblk] = run;
}

// Extra segment w of an aggregate group: aggregate its rows in an LDS copy
// of the group's block (a skewed key collapses to one entry), then add the
// entries into the table, which lb_build_kernel has written: keys by CAS
// into the block's free slots, counts and sums by 64-bit atomics.  1024
// threads with four rows each in flight (measured: the skewed 20M-row build
// 0.76 -> 0.72 ms against 256 threads and one row).
constexpr int kMergeThreads = 1024;
__global__ __launch_bounds__(kMergeThreads) void lb_merge_kernel(HashView t, const int32_t* __restrict__ skeys,
                                                       const AggIn* __restrict__ srec,
                                                       const uint32_t* base, const uint32_t* xseg, uint32_t nblk,
                                                       int32_t* status) {
    __shared__ int32_t tk[kTableBlock];
    __shared__ uint32_t tc[kTableBlock];
    __shared__ unsigned long long ts[kTableBlock];
    __shared__ uint32_t s_b;
    const uint32_t w = blockIdx.x;
    if (w >= xseg[nblk]) return;  // uniform: fewer extra segments than launched workgroups
    if (threadIdx.x == 0) {       // the group b with xseg[b] <= w < xseg[b + 1]
        uint32_t lo = 0, hi = nblk;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) / 2;
            if (xseg[mid] <= w) lo = mid; else hi = mid;
        }
        s_b = lo;
    }
    for (uint32_t j = threadIdx.x; j < kTableBlock; j += kMergeThreads) {
        tk[j] = kEmpty;
        tc[j] = 0;
        ts[j] = 0;
    }
    __syncthreads();
    const uint32_t b = s_b;
    const uint32_t seg = w - xseg[b] + 1;
    const uint32_t lo = base[b] + seg * kBuildSegRows;
    const uint32_t hi = lo + kBuildSegRows < base[b + 1] ? lo + kBuildSegRows : base[b + 1];
    const bool with_sum = t.with_sum;
    for (uint32_t i0 = lo + threadIdx.x; i0 < hi; i0 += 4 * kMergeThreads) {
      int32_t kk[4];
      unsigned long long vv[4];
      bool pd[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t i = i0 + q * kMergeThreads;
        if (srec) {
          const AggIn r = i < hi ? srec[i] : AggIn{0, 1u, 0ull};
          kk[q] = r.key;
          vv[q] = r.val;
          pd[q] = r.pad != 0u;
        } else {
          kk[q] = i < hi ? skeys[i] : 0;
          vv[q] = 0ull;
          pd[q] = false;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (i0 + q * kMergeThreads >= hi || pd[q]) continue;  // past the segment, or a padding record
        const int32_t key = kk[q];
        const unsigned long long v = vv[q];
        if (key == kEmpty) {
            agg_add(t, agg_insert(t, key), 1u, v);
            continue;
        }
        uint32_t s = hash32((uint32_t)key) & (kTableBlock - 1);
        bool placed = false;
        for (uint32_t probe = 0; probe < kTableBlock; ++probe) {
            const int32_t prev = atomicCAS(&tk[s], kEmpty, key);
            if (prev == kEmpty || prev == key) {
                atomicAdd(&tc[s], 1u);
                if (with_sum) atomicAdd(&ts[s], v);
                placed = true;
                break;
            }
            s = (s + 1) & (kTableBlock - 1);
        }
        // a segment holds keys of one table block, so its LDS copy overflows
        // only when the block has more distinct keys than slots (a distinct-key
        // bound below the truth); the dropped key must not pass silently
        if (!placed) raise_flag(status, TDP_FLAG_TABLE_FULL);
      }
    }
    __syncthreads();
    const uint32_t g0 = b * kTableBlock;
    for (uint32_t j = threadIdx.x; j < kTableBlock; j += kMergeThreads) {
        const int32_t key = tk[j];
        if (key == kEmpty) continue;
        uint32_t s = hash32((uint32_t)key) & t.mask;
        bool placed = false;
        for (uint32_t probe = 0; probe < kTableBlock; ++probe) {
            const int32_t prev = atomicCAS(&t.rec[s].key, kEmpty, key);
            if (prev == kEmpty || prev == key) {
                agg_add(t, s, tc[j], ts[j]);
                placed = true;
                break;
            }
            s = g0 | ((s + 1) & (kTableBlock - 1));
        }
        if (!placed) raise_flag(status, TDP_FLAG_TABLE_FULL);
    }
}

int grid_for(int64_t n, int per_block_items) {
    int64_t b = ceil_div(std::max<int64_t>(n, 1), per_block_items);
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 8 * kCUs);
}

}  // namespace

int table_clear(const HashView& t, int32_t* d_status, unsigned long long* d_counter, hipStream_t s) {
    const int64_t n_slots = (int64_t)t.mask + 2;
    table_clear_kernel<<<grid_for(n_slots, 256 * 4), 256, 0, s>>>(t, 0, n_slots, d_status, d_counter, nullptr, nullptr,
                                                                  0);
    return launch_status("hash table clear");
}

int table_clear_zero(const HashView& t, bool all_slots, int32_t* d_status, unsigned int* d_done,
                     unsigned long long* zero, int64_t n_zero, hipStream_t s) {
    const int64_t n_slots = (int64_t)t.mask + 2;
    const int64_t first = all_slots ? 0 : n_slots - 1;
    table_clear_kernel<<<grid_for(std::max(n_slots - first, n_zero), 256 * 4), 256, 0, s>>>(t, first, n_slots, d_status,
                                                                                          nullptr, d_done, zero, n_zero);
    return launch_status("hash table clear");
}

int table_build(const HashView& t, const BuildScratch& bs, TableKind kind, const int32_t* build_key, int64_t n_build,
                bool unique, const void* b_vals, int b_dt, int32_t* d_status, hipStream_t s) {
    if (n_build <= 0) {
        if (bs.lds) {  // the LDS build writes every block; with no rows, clear them here
            table_clear_kernel<<<grid_for((int64_t)t.mask + 1, 256 * 4), 256, 0, s>>>(t, 0, (int64_t)t.mask + 1, nullptr,
                                                                                     nullptr, nullptr, nullptr, 0);
        }
        return launch_status("hash table build");
    }
    if (bs.lds) {
        const size_t lds = (size_t)bs.nblk * sizeof(uint32_t);
        uint32_t* tot = bs.base;
        const uint32_t unit = bs.units ? (uint32_t)kAggUnit : 1u;
        if (bs.threads == 1024)
            lb_hist_kernel<1024><<<bs.nw, 1024, lds, s>>>(build_key, n_build, bs.chunk, t.mask, bs.gshift, bs.nblk, bs.mat,
                                                          unit);
        else
            lb_hist_kernel<512><<<bs.nw, 512, lds, s>>>(build_key, n_build, bs.chunk, t.mask, bs.gshift, bs.nblk, bs.mat,
                                                        unit);
        lb_colscan_kernel<<<(unsigned)ceil_div(bs.nblk, 64), 256, 0, s>>>(bs.mat, bs.nw, bs.nblk, tot);
        lb_basescan_kernel<<<1, 256, 0, s>>>(tot, bs.nblk);
        if (bs.units)
            lb_scatter_units_kernel<<<bs.nw, kAggScatThreads, 0, s>>>(build_key, n_build, bs.chunk, t.mask, bs.gshift,
                                                                      bs.nblk, bs.mat, bs.base, b_vals, b_dt, bs.srec,
                                                                      d_status);
        else if (bs.threads == 1024)
            lb_scatter_kernel<1024><<<bs.nw, 1024, lds, s>>>(build_key, n_build, bs.chunk, t.mask, bs.gshift, bs.nblk, bs.mat,
                                                             bs.base, bs.skeys, bs.srows, b_vals, b_dt, bs.srec);
        else
            lb_scatter_kernel<512><<<bs.nw, 512, lds, s>>>(build_key, n_build, bs.chunk, t.mask, bs.gshift, bs.nblk, bs.mat,
                                                           bs.base, bs.skeys, bs.srows, b_vals, b_dt, bs.srec);
        const size_t glds = (size_t)bs.gslots * (kind == TABLE_KEYS ? 4 : kind == TABLE_ROWID ? 8 : 16);
        switch (kind) {
            case TABLE_ROWID:
                lb_build_kernel<TABLE_ROWID, 512><<<bs.nblk, 512, glds, s>>>(t, bs.skeys, bs.srows, nullptr, bs.base, bs.gslots, unique,
                                                                     d_status);
                break;
            case TABLE_AGG:
                lb_build_kernel<TABLE_AGG, 1024><<<bs.nblk, 1024, glds, s>>>(t, bs.skeys, nullptr, bs.srec, bs.base, bs.gslots, unique,
                                                                   d_status);
                lb_segscan_kernel<<<1, 256, 0, s>>>(bs.base, bs.nblk, bs.xseg);
                lb_merge_kernel<<<(unsigned)std::max<int64_t>(bs.max_xseg, 1), kMergeThreads, 0, s>>>(
                    t, bs.skeys, bs.srec, bs.base, bs.xseg, bs.nblk, d_status);
                break;
            default:
                lb_build_kernel<TABLE_KEYS, 512><<<bs.nblk, 512, glds, s>>>(t, bs.skeys, nullptr, nullptr, bs.base, bs.gslots, unique,
                                                                    d_status);
                break;
        }
        return launch_status("hash table build");
    }
    const int g = grid_for(n_build, 256 * 4);
    switch (kind) {
        case TABLE_KEYS:
            table_build_kernel<TABLE_KEYS><<<g, 256, 0, s>>>(t, build_key, n_build, unique, b_vals, b_dt, d_status);
            break;
        case TABLE_ROWID:
            table_build_kernel<TABLE_ROWID><<<g, 256, 0, s>>>(t, build_key, n_build, unique, b_vals, b_dt, d_status);
            break;
        case TABLE_AGG:
            table_build_kernel<TABLE_AGG><<<g, 256, 0, s>>>(t, build_key, n_build, unique, b_vals, b_dt, d_status);
            break;
        case TABLE_LIST:
            table_build_kernel<TABLE_LIST><<<g, 256, 0, s>>>(t, build_key, n_build, unique, b_vals, b_dt, d_status);
            break;
    }
    return launch_status("hash table build");
}

}  // namespace tdp

using namespace tdp;

static int join_check(const tdp_join_desc* d) {
    if (!d) return fail(TDP_EINVAL, "tdp_hash_join: null descriptor");
    if (d->n_build < 0 || d->n_probe < 0 || (d->probe_sel && d->n_probe_sel < 0))
        return fail(TDP_EINVAL, "tdp_hash_join: negative size");
    if (d->n_build > INT32_MAX || d->n_probe > INT32_MAX)
        return fail(TDP_EINVAL, "tdp_hash_join: tables are limited to 2^31-1 rows");
    if ((d->n_build > 0 && !d->build_key) || (d->n_probe > 0 && !d->probe_key))
        return fail(TDP_EINVAL, "tdp_hash_join: null key column");
    if (d->load_pct != 0 && (d->load_pct < 10 || d->load_pct > 90))
        return fail(TDP_EINVAL, "tdp_hash_join: load_pct %d outside 10..90", d->load_pct);
    if (d->max_distinct < 0) return fail(TDP_EINVAL, "tdp_hash_join: negative max_distinct");
    return TDP_OK;
}

extern "C" size_t tdp_hash_join_workspace_size(const tdp_join_desc* d) {
    if (!d || d->n_build < 0) return 0;
    WsAlloc wa(nullptr);
    table_alloc(wa, TABLE_LIST, d->n_build, table_cap(distinct_bound(d), d->load_pct), false);
    return wa.bytes();
}

extern "C" int tdp_hash_join(const tdp_join_desc* d, int32_t mode, int32_t* out_probe, int32_t* out_build, int64_t cap,
                             int64_t* d_n_out, int32_t* d_status, void* ws, size_t ws_bytes, hipStream_t stream) {
    int rc = join_check(d);
    if (rc) return rc;
    if (mode != TDP_JOIN_PAIRS && mode != TDP_JOIN_COUNT) return fail(TDP_EINVAL, "tdp_hash_join: mode %d", mode);
    if (!d_n_out) return fail(TDP_EINVAL, "tdp_hash_join: null count pointer");
    if (mode == TDP_JOIN_PAIRS && cap > 0 && (!out_probe || !out_build))
        return fail(TDP_EINVAL, "tdp_hash_join: null pair outputs");
    if (cap < 0) return fail(TDP_EINVAL, "tdp_hash_join: negative cap");
    const size_t need = tdp_hash_join_workspace_size(d);
    if (!ws || ws_bytes < need) return fail_need(TDP_EWORKSPACE, (int64_t)need, "tdp_hash_join: workspace %zu < %zu", ws_bytes, need);
    WsAlloc wa(ws);
    HashView t = table_alloc(wa, TABLE_LIST, d->n_build, table_cap(distinct_bound(d), d->load_pct), false);
    rc = table_clear(t, d_status, (unsigned long long*)d_n_out, stream);
    if (rc) return rc;
    rc = table_build(t, BuildScratch(), TABLE_LIST, d->build_key, d->n_build, d->build_unique != 0, nullptr, 0,
                     d_status, stream);
    if (rc) return rc;
    const int64_t n_cand = d->probe_sel ? d->n_probe_sel : d->n_probe;
    if (n_cand > 0) {
        const int g = grid_for(n_cand, 256 * 4);
        if (mode == TDP_JOIN_PAIRS)
            join_probe_kernel<true><<<g, 256, 0, stream>>>(t, d->probe_key, d->probe_sel, n_cand, out_probe, out_build,
                                                           cap, (unsigned long long*)d_n_out);
        else
            join_probe_kernel<false><<<g, 256, 0, stream>>>(t, d->probe_key, d->probe_sel, n_cand, nullptr, nullptr, 0,
                                                            (unsigned long long*)d_n_out);
    }
    return launch_status("tdp_hash_join");
}
