// Order-preserving dictionary encoding of fixed-width string columns.
//
// A string column is a zero-padded byte matrix [n][L] (L a multiple of 4,
// at most 32; strings hold no zero bytes).  Its dictionary is the sorted
// list of distinct strings, one per row of a [d][L] byte matrix, and a
// string's code is its position there, so codes compare as the strings do
// and equal strings have equal codes: the codes serve as int32 keys of the
// filter, join and group-by operators.
//
// Build (one call, asynchronous): every row inserts itself into an
// open-addressing table of row ids keyed by the string (a slot keeps the
// first row that claimed it; a later row with the same string finds it by
// comparing the words) and records its slot; the occupied slots are
// compacted to one representative row per distinct string; a bitonic sort
// orders the representatives by string; the position of each becomes the
// code of its slot and its bytes the dictionary row; finally every row
// reads its code through its slot.  Strings compare as sequences of
// big-endian 32-bit words, which is byte-wise lexicographic order with the
// zero padding sorting first.
#include "common.hpp"

namespace tdp {

namespace {

constexpr int kDictMaxWords = 8;  // 32 bytes

__device__ __forceinline__ void load_words(const uint32_t* s, int W, uint32_t w[kDictMaxWords]) {
#pragma unroll
    for (int k = 0; k < kDictMaxWords; ++k) w[k] = k < W ? __builtin_bswap32(s[k]) : 0u;
}

// -1, 0, 1 as a < b, a == b, a > b (big-endian words, lexicographic).
__device__ __forceinline__ int cmp_words(const uint32_t a[kDictMaxWords], const uint32_t b[kDictMaxWords], int W) {
#pragma unroll
    for (int k = 0; k < kDictMaxWords; ++k) {
        if (k >= W) break;
        if (a[k] != b[k]) return a[k] < b[k] ? -1 : 1;
    }
    return 0;
}

__device__ __forceinline__ uint32_t hash_words(const uint32_t w[kDictMaxWords], int W) {
    uint32_t h = 0x9E3779B9u;
#pragma unroll
    for (int k = 0; k < kDictMaxWords; ++k)
        if (k < W) h = hash32(h ^ w[k]) + (uint32_t)k;
    return h;
}

__global__ void dict_fill_kernel(int32_t* p, int64_t n, int32_t v, int64_t* d_count, int32_t* status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *d_count = 0;
        if (status) *status = 0;
    }
}

// Each row finds or claims the slot of its string; row_slot[i] = the slot.
__global__ void dict_insert_kernel(const uint32_t* __restrict__ strs, int64_t n, int W, int32_t* table, uint32_t mask,
                                   int32_t* row_slot, int32_t* status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t w[kDictMaxWords];
        load_words(strs + i * W, W, w);
        uint32_t s = hash_words(w, W) & mask;
        int32_t slot = -1;
        for (uint32_t probes = 0; probes <= mask; ++probes) {
            int32_t cur = __hip_atomic_load(&table[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (cur < 0) {
                cur = atomicCAS(&table[s], -1, (int32_t)i);
                if (cur < 0) {
                    slot = (int32_t)s;
                    break;
                }
            }
            uint32_t o[kDictMaxWords];
            load_words(strs + (int64_t)cur * W, W, o);
            if (cmp_words(w, o, W) == 0) {
                slot = (int32_t)s;
                break;
            }
            s = (s + 1) & mask;
        }
        if (slot < 0) raise_flag(status, TDP_FLAG_TABLE_FULL);
        row_slot[i] = slot;
    }
}

// One representative row per occupied slot, in any order; more than `cap`
// distinct strings raise the flag.
__global__ void dict_compact_kernel(const int32_t* table, int64_t n_slots, int32_t* reps, int64_t cap,
                                    int64_t* d_count, int32_t* status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_slots; s += stride) {
        const int32_t r = table[s];
        if (r < 0) continue;
        const unsigned long long k = atomicAdd((unsigned long long*)d_count, 1ull);
        if ((int64_t)k < cap) reps[k] = r;
        else raise_flag(status, TDP_FLAG_TABLE_FULL);
    }
}

// Representatives beyond the count (or beyond the capacity, when more
// distinct strings arrived than it holds) become the sentinel -1, sorted last.
__global__ void dict_pad_kernel(int32_t* reps, int64_t sort_n, const int64_t* d_count, int64_t cap) {
    const int64_t d = *d_count < cap ? *d_count : cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < sort_n; i += stride)
        if (i >= d) reps[i] = -1;
}

// One compare-exchange stage (k, j) of the bitonic sort of representative
// rows by their strings (ascending; the sentinel -1 is largest).
__global__ void dict_bitonic_kernel(const uint32_t* __restrict__ strs, int W, int32_t* reps, int64_t sort_n,
                                    int64_t k, int64_t j) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < sort_n; i += stride) {
        const int64_t l = i ^ j;
        if (l <= i) continue;
        const int32_t a = reps[i], b = reps[l];
        int c;
        if (a < 0 || b < 0) {
            c = (a < 0) == (b < 0) ? 0 : (a < 0 ? 1 : -1);
        } else {
            uint32_t wa[kDictMaxWords], wb[kDictMaxWords];
            load_words(strs + (int64_t)a * W, W, wa);
            load_words(strs + (int64_t)b * W, W, wb);
            c = cmp_words(wa, wb, W);
        }
        const bool up = (i & k) == 0;
        if ((up && c > 0) || (!up && c < 0)) {
            reps[i] = b;
            reps[l] = a;
        }
    }
}

// Position r of the sorted representatives: the code of its slot and the
// dictionary's row r.
__global__ void dict_rank_kernel(const uint32_t* __restrict__ strs, int W, const int32_t* reps, const int64_t* d_count,
                                 int64_t cap, const int32_t* row_slot, int32_t* slot_code, uint32_t* dict) {
    const int64_t d = *d_count < cap ? *d_count : cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < d; r += stride) {
        const int32_t row = reps[r];
        slot_code[row_slot[row]] = (int32_t)r;
        for (int k = 0; k < W; ++k) dict[r * W + k] = strs[(int64_t)row * W + k];
    }
}

__global__ void dict_codes_kernel(const int32_t* row_slot, int64_t n, const int32_t* slot_code, int32_t* codes) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t s = row_slot[i];
        codes[i] = s >= 0 ? slot_code[s] : -1;
    }
}

// Lower bound of each string in the sorted dictionary, and whether it is there.
__global__ void dict_lookup_kernel(const uint32_t* __restrict__ dict, int64_t d, int W, const uint32_t* __restrict__ strs,
                                   int64_t n, int32_t* pos, int8_t* found) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t w[kDictMaxWords];
        load_words(strs + i * W, W, w);
        int64_t lo = 0, hi = d;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            uint32_t m[kDictMaxWords];
            load_words(dict + mid * W, W, m);
            if (cmp_words(m, w, W) < 0) lo = mid + 1;
            else hi = mid;
        }
        int8_t f = 0;
        if (lo < d) {
            uint32_t m[kDictMaxWords];
            load_words(dict + lo * W, W, m);
            f = cmp_words(m, w, W) == 0 ? 1 : 0;
        }
        pos[i] = (int32_t)lo;
        if (found) found[i] = f;
    }
}

__global__ void dict_decode_kernel(const int32_t* codes, int64_t n, const uint32_t* dict, int64_t d, int W,
                                   uint32_t* out, int32_t* status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t c = codes[i];
        const bool in = c >= 0 && c < d;
        if (!in) raise_flag(status, TDP_FLAG_KEY_DOMAIN);
        for (int k = 0; k < W; ++k) out[i * W + k] = in ? dict[(int64_t)c * W + k] : 0u;
    }
}

struct DictWs {
    int32_t* table;
    int32_t* slot_code;
    int32_t* row_slot;
    int32_t* reps;
    int64_t n_slots, sort_n;
};

DictWs dict_layout(void* ws, int64_t n, int64_t max_distinct, size_t* bytes) {
    DictWs w;
    int64_t slots = 256;
    while (slots < 2 * max_distinct) slots <<= 1;
    int64_t sn = 1;
    while (sn < max_distinct) sn <<= 1;
    WsAlloc wa(ws);
    w.table = wa.take<int32_t>(slots);
    w.slot_code = wa.take<int32_t>(slots);
    w.row_slot = wa.take<int32_t>(std::max<int64_t>(n, 1));
    w.reps = wa.take<int32_t>(sn);
    w.n_slots = slots;
    w.sort_n = sn;
    if (bytes) *bytes = wa.bytes();
    return w;
}

int dict_grid(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>(ceil_div(n, 256), 1), 8192); }

int dict_check_width(int32_t L, const char* fn) {
    if (L < 4 || L > 4 * kDictMaxWords || (L & 3)) return fail(TDP_EINVAL, "%s: width %d is not a multiple of 4 in 4..32", fn, L);
    return TDP_OK;
}

}  // namespace

}  // namespace tdp

using namespace tdp;

namespace {
// The distinct-string bound a build works with: max_distinct, 0 meaning n.
int64_t dict_bound(int64_t n, int64_t max_distinct) {
    return std::max<int64_t>(max_distinct == 0 ? n : std::min(max_distinct, n), 1);
}
}  // namespace

extern "C" size_t tdp_dict_build_workspace_size(int64_t n, int64_t max_distinct) {
    size_t b;
    dict_layout(nullptr, std::max<int64_t>(n, 0), dict_bound(std::max<int64_t>(n, 0), std::max<int64_t>(max_distinct, 0)), &b);
    return b;
}

extern "C" int tdp_dict_build(const uint8_t* strs, int64_t n, int32_t L, int64_t max_distinct, uint8_t* dict,
                              int64_t* d_n_dict, int32_t* codes, int32_t* d_status, void* ws, size_t ws_bytes,
                              hipStream_t stream) {
    int rc = dict_check_width(L, "tdp_dict_build");
    if (rc) return rc;
    if (n < 0 || n > INT32_MAX || max_distinct < 0) return fail(TDP_EINVAL, "tdp_dict_build: n=%lld max_distinct=%lld", (long long)n, (long long)max_distinct);
    if (!d_n_dict || (n > 0 && (!strs || !dict || !codes))) return fail(TDP_EINVAL, "tdp_dict_build: null pointer");
    if ((uintptr_t)strs & 3 || (uintptr_t)dict & 3) return fail(TDP_EINVAL, "tdp_dict_build: strings and dictionary must be 4-byte aligned");
    const int64_t md = dict_bound(n, max_distinct);
    size_t need;
    dict_layout(nullptr, n, md, &need);
    if (!ws || ws_bytes < need) return fail_need(TDP_EWORKSPACE, (int64_t)need, "tdp_dict_build: workspace %zu < %zu", ws_bytes, need);
    DictWs w = dict_layout(ws, n, md, nullptr);
    const int W = L / 4;
    const uint32_t* s32 = (const uint32_t*)strs;
    dict_fill_kernel<<<dict_grid(w.n_slots), 256, 0, stream>>>(w.table, w.n_slots, -1, d_n_dict, d_status);
    if (n > 0) {
        dict_insert_kernel<<<dict_grid(n), 256, 0, stream>>>(s32, n, W, w.table, (uint32_t)(w.n_slots - 1), w.row_slot, d_status);
        dict_compact_kernel<<<dict_grid(w.n_slots), 256, 0, stream>>>(w.table, w.n_slots, w.reps, md, d_n_dict, d_status);
        dict_pad_kernel<<<dict_grid(w.sort_n), 256, 0, stream>>>(w.reps, w.sort_n, d_n_dict, md);
        for (int64_t k = 2; k <= w.sort_n; k <<= 1)
            for (int64_t j = k >> 1; j > 0; j >>= 1)
                dict_bitonic_kernel<<<dict_grid(w.sort_n), 256, 0, stream>>>(s32, W, w.reps, w.sort_n, k, j);
        dict_rank_kernel<<<dict_grid(md), 256, 0, stream>>>(s32, W, w.reps, d_n_dict, md, w.row_slot, w.slot_code, (uint32_t*)dict);
        dict_codes_kernel<<<dict_grid(n), 256, 0, stream>>>(w.row_slot, n, w.slot_code, codes);
    }
    return launch_status("tdp_dict_build");
}

extern "C" int tdp_dict_lookup(const uint8_t* dict, int64_t n_dict, int32_t L, const uint8_t* strs, int64_t n,
                               int32_t* pos, int8_t* found, hipStream_t stream) {
    int rc = dict_check_width(L, "tdp_dict_lookup");
    if (rc) return rc;
    if (n < 0 || n_dict < 0 || n_dict > INT32_MAX || (n > 0 && (!strs || !pos)) || (n_dict > 0 && !dict))
        return fail(TDP_EINVAL, "tdp_dict_lookup: null pointer or negative size");
    if ((uintptr_t)strs & 3 || (uintptr_t)dict & 3) return fail(TDP_EINVAL, "tdp_dict_lookup: arrays must be 4-byte aligned");
    if (n == 0) return TDP_OK;
    dict_lookup_kernel<<<dict_grid(n), 256, 0, stream>>>((const uint32_t*)dict, n_dict, L / 4, (const uint32_t*)strs, n, pos,
                                                         found);
    return launch_status("tdp_dict_lookup");
}

extern "C" int tdp_dict_decode(const int32_t* codes, int64_t n, const uint8_t* dict, int64_t n_dict, int32_t L,
                               uint8_t* out, int32_t* d_status, hipStream_t stream) {
    int rc = dict_check_width(L, "tdp_dict_decode");
    if (rc) return rc;
    if (n < 0 || n_dict < 0 || (n > 0 && (!codes || !out)) || (n_dict > 0 && !dict))
        return fail(TDP_EINVAL, "tdp_dict_decode: null pointer or negative size");
    if ((uintptr_t)out & 3 || (uintptr_t)dict & 3) return fail(TDP_EINVAL, "tdp_dict_decode: arrays must be 4-byte aligned");
    if (n == 0) return TDP_OK;
    dict_decode_kernel<<<dict_grid(n), 256, 0, stream>>>(codes, n, (const uint32_t*)dict, n_dict, L / 4, (uint32_t*)out,
                                                         d_status);
    return launch_status("tdp_dict_decode");
}
