// Hash equi-join: build an open-addressing table from the build keys, then
// stream the probe side through it.
#include "hash.hpp"

namespace tdp {

namespace {

__global__ void table_clear_kernel(HashView t, int64_t n_slots, int32_t* d_status, unsigned long long* d_counter,
                                   unsigned int* d_done, unsigned long long* zero, int64_t n_zero) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n = n_slots > n_zero ? n_slots : n_zero;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (i < n_slots) {
            const bool extra = i == n_slots - 1;  // slot `cap` holds the kEmpty key's presence flag
            t.keys[i] = extra ? 0 : kEmpty;
            if (t.cnt) t.cnt[i] = 0;
            if (t.sum) t.sum[i] = 0;
            if (t.head) t.head[i] = -1;
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
        bool fresh;
        const int64_t slot = ht_insert(t, bkey[j], fresh);
        if (slot < 0) {
            raise_flag(status, TDP_FLAG_TABLE_FULL);
            continue;
        }
        if (unique && !fresh) raise_flag(status, TDP_FLAG_DUP_BUILD);
        if (KIND == TABLE_ROWID) {
            if (fresh) t.rowid[slot] = (int32_t)j;
        } else if (KIND == TABLE_AGG) {
            atomicAdd(&t.cnt[slot], 1ull);
            if (t.sum) atomicAdd(&t.sum[slot], (unsigned long long)load_int(bvals, bdt, j));
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
            const int64_t slot = ht_find(t.keys, t.mask, pkey[row]);
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

int grid_for(int64_t n, int per_block_items) {
    int64_t b = ceil_div(std::max<int64_t>(n, 1), per_block_items);
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 8 * kCUs);
}

}  // namespace

int table_clear(const HashView& t, int32_t* d_status, unsigned long long* d_counter, hipStream_t s) {
    const int64_t n_slots = (int64_t)t.mask + 2;
    table_clear_kernel<<<grid_for(n_slots, 256 * 4), 256, 0, s>>>(t, n_slots, d_status, d_counter, nullptr, nullptr, 0);
    return launch_status("hash table clear");
}

int table_clear_zero(const HashView& t, int32_t* d_status, unsigned int* d_done, unsigned long long* zero,
                     int64_t n_zero, hipStream_t s) {
    const int64_t n_slots = (int64_t)t.mask + 2;
    table_clear_kernel<<<grid_for(std::max(n_slots, n_zero), 256 * 4), 256, 0, s>>>(t, n_slots, d_status, nullptr,
                                                                                  d_done, zero, n_zero);
    return launch_status("hash table clear");
}

int table_build(const HashView& t, TableKind kind, const int32_t* build_key, int64_t n_build, bool unique,
                const void* b_vals, int b_dt, int32_t* d_status, hipStream_t s) {
    if (n_build <= 0) return TDP_OK;
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
    return TDP_OK;
}

extern "C" size_t tdp_hash_join_workspace_size(const tdp_join_desc* d) {
    if (!d || d->n_build < 0) return 0;
    WsAlloc wa(nullptr);
    table_alloc(wa, TABLE_LIST, d->n_build, table_cap(d->n_build, d->load_pct), false);
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
    if (!ws || ws_bytes < need) return fail(TDP_EWORKSPACE, "tdp_hash_join: workspace %zu < %zu", ws_bytes, need);
    WsAlloc wa(ws);
    HashView t = table_alloc(wa, TABLE_LIST, d->n_build, table_cap(d->n_build, d->load_pct), false);
    rc = table_clear(t, d_status, (unsigned long long*)d_n_out, stream);
    if (rc) return rc;
    rc = table_build(t, TABLE_LIST, d->build_key, d->n_build, d->build_unique != 0, nullptr, 0, d_status, stream);
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
