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
// orders the representatives by string (tiles of 2048 in LDS with their
// words, only the stages whose partner lies in another tile in global
// memory); the position of each becomes the code of its slot and its bytes
// the dictionary row; finally every row reads its code through its slot.
// Lookup searches a sample of every S-th dictionary string held in LDS, then
// the one run of S strings in memory.  Strings compare as sequences of
// big-endian 32-bit words, which is byte-wise lexicographic order with the
// zero padding sorting first.
#include "common.hpp"

namespace tdp {

namespace {

constexpr int kDictMaxWords = 8;  // 32 bytes

// The W words of one string as big-endian values (zero past W): 16-byte
// loads when the string starts 16-byte aligned and W is a multiple of 4 (a
// search step is then one load instruction, not four whose lanes each touch
// another cache line), 4-byte loads otherwise.
__device__ __forceinline__ void load_words(const uint32_t* s, int W, uint32_t w[kDictMaxWords]) {
    if ((W & 3) == 0 && ((uintptr_t)s & 15) == 0) {
#pragma unroll
        for (int k = 0; k < kDictMaxWords; k += 4) {
            uint4 q = make_uint4(0u, 0u, 0u, 0u);
            if (k < W) q = *(const uint4*)(s + k);
            w[k] = __builtin_bswap32(q.x);
            w[k + 1] = __builtin_bswap32(q.y);
            w[k + 2] = __builtin_bswap32(q.z);
            w[k + 3] = __builtin_bswap32(q.w);
        }
        return;
    }
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
            // a claimed slot never changes, so a plain (cached) read that sees
            // a row is final; one that sees the slot empty may be stale, and
            // the compare-and-swap then returns the slot's current value
            int32_t cur = table[s];
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
// (A wave reserves its occupied slots' positions with one atomic add.)
__global__ void dict_compact_kernel(const int32_t* table, int64_t n_slots, int32_t* reps, int64_t cap,
                                    int64_t* d_count, int32_t* status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s0 = (int64_t)blockIdx.x * blockDim.x; s0 < n_slots; s0 += stride) {
        const int64_t s = s0 + threadIdx.x;
        const int32_t r = s < n_slots ? table[s] : -1;
        const uint64_t m = ballot(r >= 0);
        if (m == 0) continue;
        unsigned long long first = 0;
        if (lane_id() == 0) first = atomicAdd((unsigned long long*)d_count, (unsigned long long)__popcll(m));
        first = __shfl(first, 0, kWave);
        if (r < 0) continue;
        const int64_t k = (int64_t)first + lanes_below(m);
        if (k < cap) reps[k] = r;
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

// The stages of the same bitonic network whose partners lie within one tile
// of representatives, in LDS (words as [W][tile], so lanes read consecutive
// addresses).  k == 0: every stage of every merge size up to the tile (the
// tiles come out sorted, alternately ascending and descending as the network
// needs); else the stages j < tile of merge size k.  A tile is 2048
// representatives, 1024 for 32-byte strings, so that it fits 64 KiB of LDS.
constexpr int kSortThreads = 1024;
constexpr int kSortLdsBytes = 64 * 1024;

int64_t sort_tile(int64_t sort_n, int W) {
    int64_t tile = 2048;
    while (tile * (W + 1) * (int64_t)sizeof(uint32_t) > kSortLdsBytes) tile >>= 1;
    return std::min(sort_n, tile);
}

__device__ __forceinline__ int cmp_lds(const uint32_t* sw, const int32_t* si, int tile, int W, int a, int b) {
    const int32_t ia = si[a], ib = si[b];
    if (ia < 0 || ib < 0) return (ia < 0) == (ib < 0) ? 0 : (ia < 0 ? 1 : -1);
    for (int k = 0; k < W; ++k) {
        const uint32_t x = sw[k * tile + a], y = sw[k * tile + b];
        if (x != y) return x < y ? -1 : 1;
    }
    return 0;
}

__global__ __launch_bounds__(kSortThreads) void dict_sort_local_kernel(const uint32_t* __restrict__ strs, int W,
                                                                       int32_t* reps, int tile, int64_t k) {
    extern __shared__ uint32_t s_sort[];
    uint32_t* sw = s_sort;                       // [W][tile]
    int32_t* si = (int32_t*)(s_sort + W * tile);  // [tile]
    const int64_t base = (int64_t)blockIdx.x * tile;
    for (int e = threadIdx.x; e < tile; e += blockDim.x) {
        const int32_t r = reps[base + e];
        si[e] = r;
        for (int q = 0; q < W; ++q) sw[q * tile + e] = r >= 0 ? __builtin_bswap32(strs[(int64_t)r * W + q]) : 0u;
    }
    __syncthreads();
    auto stage = [&](int64_t kk, int j) {
        for (int t = threadIdx.x; t < tile / 2; t += blockDim.x) {
            const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
            const int l = i | j;
            const bool up = ((base + i) & kk) == 0;
            const int c = cmp_lds(sw, si, tile, W, i, l);
            if ((up && c > 0) || (!up && c < 0)) {
                const int32_t x = si[i];
                si[i] = si[l];
                si[l] = x;
                for (int q = 0; q < W; ++q) {
                    const uint32_t y = sw[q * tile + i];
                    sw[q * tile + i] = sw[q * tile + l];
                    sw[q * tile + l] = y;
                }
            }
        }
        __syncthreads();
    };
    if (k == 0) {
        for (int kk = 2; kk <= tile; kk <<= 1)
            for (int j = kk >> 1; j > 0; j >>= 1) stage(kk, j);
    } else {
        for (int j = tile >> 1; j > 0; j >>= 1) stage(k, j);
    }
    for (int e = threadIdx.x; e < tile; e += blockDim.x) reps[base + e] = si[e];
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

// Four rows per thread and step when `codes` is 16-byte aligned (16-byte
// loads of the workspace's row slots and stores of codes), the tail of
// fewer than four rows one by one.
__global__ void dict_codes_kernel(const int32_t* row_slot, int64_t n, const int32_t* slot_code, int32_t* codes) {
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t tail = 0;
    if (((uintptr_t)codes & 15) == 0) {
        const int64_t n4 = n / 4;
        for (int64_t q = t; q < n4; q += nthreads) {
            const int4 s = *(const int4*)&row_slot[q * 4];
            int4 c;
            c.x = s.x >= 0 ? slot_code[s.x] : -1;
            c.y = s.y >= 0 ? slot_code[s.y] : -1;
            c.z = s.z >= 0 ? slot_code[s.z] : -1;
            c.w = s.w >= 0 ? slot_code[s.w] : -1;
            *(int4*)&codes[q * 4] = c;
        }
        tail = n4 * 4;
    }
    for (int64_t j = tail + t; j < n; j += nthreads) {
        const int32_t s = row_slot[j];
        codes[j] = s >= 0 ? slot_code[s] : -1;
    }
}

// Lower bound of each string in the sorted dictionary, and whether it is
// there: first among the samples dict[0], dict[S], dict[2S], ... (held in
// LDS), which leaves one run of fewer than S strings to search in memory.
constexpr int kLookupThreads = 1024;
constexpr int kLookupLdsBytes = 48 * 1024;

__global__ __launch_bounds__(kLookupThreads) void dict_lookup_kernel(const uint32_t* __restrict__ dict, int64_t d,
                                                                     int W, const uint32_t* __restrict__ strs,
                                                                     int64_t n, int sshift, int ns, int32_t* pos,
                                                                     int8_t* found) {
    extern __shared__ uint32_t s_samp[];  // [ns][W] big-endian words
    for (int e = threadIdx.x; e < ns * W; e += blockDim.x) {
        const int q = e / W, k = e - q * W;
        s_samp[e] = __builtin_bswap32(dict[((int64_t)q << sshift) * W + k]);
    }
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t w[kDictMaxWords];
        load_words(strs + i * W, W, w);
        int slo = 0, shi = ns;  // first sample >= w
        while (slo < shi) {
            const int mid = (slo + shi) >> 1;
            uint32_t m[kDictMaxWords];
#pragma unroll
            for (int k = 0; k < kDictMaxWords; ++k) m[k] = k < W ? s_samp[mid * W + k] : 0u;
            if (cmp_words(m, w, W) < 0) slo = mid + 1;
            else shi = mid;
        }
        // the lower bound lies in ((slo - 1) * S, min(slo * S, d)]
        int64_t lo = slo == 0 ? 0 : ((int64_t)(slo - 1) << sshift) + 1;
        int64_t hi = ((int64_t)slo << sshift) < d ? ((int64_t)slo << sshift) : d;
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
    if ((uintptr_t)ws & 255) return fail(TDP_EINVAL, "tdp_dict_build: workspace not 256-byte aligned");
    DictWs w = dict_layout(ws, n, md, nullptr);
    const int W = L / 4;
    const uint32_t* s32 = (const uint32_t*)strs;
    dict_fill_kernel<<<dict_grid(w.n_slots), 256, 0, stream>>>(w.table, w.n_slots, -1, d_n_dict, d_status);
    if (n > 0) {
        dict_insert_kernel<<<dict_grid(n), 256, 0, stream>>>(s32, n, W, w.table, (uint32_t)(w.n_slots - 1), w.row_slot, d_status);
        dict_compact_kernel<<<dict_grid(w.n_slots), 256, 0, stream>>>(w.table, w.n_slots, w.reps, md, d_n_dict, d_status);
        dict_pad_kernel<<<dict_grid(w.sort_n), 256, 0, stream>>>(w.reps, w.sort_n, d_n_dict, md);
        // bitonic network: the stages within a tile in LDS, the others one launch each
        const int64_t tile = sort_tile(w.sort_n, W);
        const unsigned tiles = (unsigned)(w.sort_n / tile);
        const size_t lds = (size_t)tile * (W + 1) * sizeof(uint32_t);
        dict_sort_local_kernel<<<tiles, kSortThreads, lds, stream>>>(s32, W, w.reps, (int)tile, 0);
        for (int64_t k = 2 * tile; k <= w.sort_n; k <<= 1) {
            for (int64_t j = k >> 1; j >= tile; j >>= 1)
                dict_bitonic_kernel<<<dict_grid(w.sort_n), 256, 0, stream>>>(s32, W, w.reps, w.sort_n, k, j);
            dict_sort_local_kernel<<<tiles, kSortThreads, lds, stream>>>(s32, W, w.reps, (int)tile, k);
        }
        dict_rank_kernel<<<dict_grid(md), 256, 0, stream>>>(s32, W, w.reps, d_n_dict, md, w.row_slot, w.slot_code, (uint32_t*)dict);
        dict_codes_kernel<<<dict_grid(ceil_div(n, 4)), 256, 0, stream>>>(w.row_slot, n, w.slot_code, codes);
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
    // samples every S = 2^sshift strings, as many as fit the LDS budget
    const int W = L / 4;
    const int64_t max_samples = kLookupLdsBytes / (W * (int64_t)sizeof(uint32_t));
    int sshift = 0;
    while (ceil_div(n_dict, (int64_t)1 << sshift) > max_samples) ++sshift;
    const int ns = (int)ceil_div(n_dict, (int64_t)1 << sshift);
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(ceil_div(n, kLookupThreads), 1), 4 * kCUs);
    dict_lookup_kernel<<<grid, kLookupThreads, (size_t)ns * W * sizeof(uint32_t), stream>>>(
        (const uint32_t*)dict, n_dict, W, (const uint32_t*)strs, n, sshift, ns, pos, found);
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
