// Predicate scan with stream compaction (WHERE col <cmp> literal).
//
// One pass over the column.  Each workgroup (4 waves) takes the next tile of
// 16384 candidates from an atomic ticket, so every tile it waits on belongs
// to a workgroup that is already running.  Each lane reads 16 contiguous
// bytes per round (fully coalesced), keeps the survivors of its 64 rows as a
// bit mask in one register, and the wave counts them.  The tile's exclusive
// offset comes from a decoupled look-back over per-tile (flag, value) words;
// then each wave writes its survivors in order: a per-round exclusive prefix
// of per-lane counts (one ballot per count bit) places each survivor's row id
// in the wave's LDS stage, from which consecutive lanes store consecutive
// dwords.
#include <mutex>

#include "common.hpp"

namespace tdp {

namespace {

constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagPrefix = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;
constexpr int kSpinLimit = 1 << 24;
constexpr int kFilterThreads = 256;

template <typename T, bool SEL>
struct FilterShape {
    static constexpr int VEC = SEL ? 4 : 16 / (int)sizeof(T);
    static constexpr int ROUNDS = 64 / VEC;
    static constexpr int WAVE_ROWS = ROUNDS * kWave * VEC;
    static constexpr int TILE_ROWS = (kFilterThreads / kWave) * WAVE_ROWS;
    static constexpr int CBITS = VEC == 16 ? 5 : (VEC == 4 ? 3 : 2);
    static constexpr int UNROLL = ROUNDS <= 16 ? ROUNDS : 8;
};

__global__ void filter_init_kernel(uint64_t* state, int64_t ntiles, uint32_t* ticket, int64_t* d_n_out,
                                   int32_t* d_status) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < ntiles; i += (int64_t)gridDim.x * blockDim.x) state[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *ticket = 0;
        *d_n_out = 0;
        if (d_status) *d_status = 0;
    }
}

// Exclusive offset of `tile` from the tiles before it; publishes its own
// inclusive prefix.  Run by one thread.
__device__ uint64_t tile_lookback(uint64_t* state, uint32_t tile, uint64_t agg, int32_t* status) {
    if (tile == 0) {
        __hip_atomic_store(&state[0], kFlagPrefix | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return 0;
    }
    __hip_atomic_store(&state[tile], kFlagAgg | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    int64_t j = (int64_t)tile - 1;
    while (true) {
        uint64_t s = 0;
        int spins = 0;
        while (true) {
            s = __hip_atomic_load(&state[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (s >> 62) break;
            if (++spins >= kSpinLimit) {
                raise_flag(status, TDP_FLAG_SPIN);
                s = kFlagPrefix;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        excl += s & kValMask;
        if ((s & ~kValMask) == kFlagPrefix) break;
        --j;
    }
    __hip_atomic_store(&state[tile], kFlagPrefix | (excl + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

template <typename T, bool SEL>
__global__ __launch_bounds__(kFilterThreads) void filter_kernel(const T* __restrict__ col,
                                                               const int32_t* __restrict__ sel, int64_t n_cand,
                                                               int cmp, int64_t lit, int32_t* __restrict__ out,
                                                               int64_t* d_n_out, uint64_t* state, uint32_t* ticket,
                                                               uint32_t ntiles, int32_t* status) {
    using S = FilterShape<T, SEL>;
    constexpr int VEC = S::VEC;
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_wave[kFilterThreads / kWave];
    __shared__ uint64_t s_excl;
    __shared__ int32_t s_stage[kFilterThreads / kWave][kWave * VEC];
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t wbase = (int64_t)tile * S::TILE_ROWS + (int64_t)wave * S::WAVE_ROWS;

    // Pass 1: predicate bits of this lane's rows (all loads of up to 16
    // rounds in flight together).
    uint64_t bits = 0;
    constexpr int kUnroll = S::UNROLL;
#pragma unroll kUnroll
    for (int r = 0; r < S::ROUNDS; ++r) {
        const int64_t r0 = wbase + ((int64_t)r * kWave + lane) * VEC;
        uint32_t m = 0;
        if (r0 < n_cand) {
            if constexpr (SEL) {
                int32_t rows[4];
                if (r0 + 4 <= n_cand) {
                    int4 q = *(const int4*)(sel + r0);
                    rows[0] = q.x; rows[1] = q.y; rows[2] = q.z; rows[3] = q.w;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) rows[e] = (r0 + e < n_cand) ? sel[r0 + e] : 0;
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (r0 + e < n_cand && cmp_i64((int64_t)col[rows[e]], cmp, lit)) m |= 1u << e;
            } else {
                T v[VEC];
                if (r0 + VEC <= n_cand) {
                    uint4 q = *(const uint4*)(col + r0);
                    __builtin_memcpy(v, &q, 16);
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) v[e] = (r0 + e < n_cand) ? col[r0 + e] : T(0);
                }
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    if (r0 + e < n_cand && cmp_i64((int64_t)v[e], cmp, lit)) m |= 1u << e;
            }
        }
        bits |= (uint64_t)m << (r * VEC);
    }
    const uint32_t wtot = wave_sum<uint32_t>((uint32_t)__popcll(bits));
    if (lane == 0) s_wave[wave] = wtot;
    __syncthreads();

    // Tile offset by decoupled look-back.
    if (threadIdx.x == 0) {
        uint64_t agg = 0;
        for (int w = 0; w < kFilterThreads / kWave; ++w) agg += s_wave[w];
        uint64_t excl = tile_lookback(state, tile, agg, status);
        s_excl = excl;
        if (tile == ntiles - 1) *d_n_out = (int64_t)(excl + agg);
    }
    __syncthreads();
    uint64_t running = s_excl;
    for (int w = 0; w < wave; ++w) running += s_wave[w];
    if (wtot == 0) return;

    // Pass 2: write survivors in candidate order, one round at a time through
    // the wave's LDS stage (at most kWave * VEC ids per round).
    int32_t* stage = s_stage[wave];
    constexpr uint32_t kMask = (1u << VEC) - 1u;
    for (int r = 0; r < S::ROUNDS; ++r) {
        const uint32_t m = (uint32_t)(bits >> (r * VEC)) & kMask;
        uint32_t prefix, total;
        wave_count_scan<S::CBITS>((uint32_t)__popc(m), prefix, total);
        if (total == 0) continue;
        if (m) {
            const int64_t r0 = wbase + ((int64_t)r * kWave + lane) * VEC;
            uint32_t p = prefix;
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                if ((m >> e) & 1u) stage[p++] = SEL ? sel[r0 + e] : (int32_t)(r0 + e);
            }
        }
        wave_lds_sync();
        int32_t* dst = out + running;
        for (uint32_t j = lane; j < total; j += kWave) dst[j] = stage[j];
        wave_lds_sync();  // the stage is read before the next round fills it
        running += total;
    }
}

// Tile states and ticket: from the caller's workspace, or from the static
// scratch array of the allocation-free entry point.
struct FilterScratch {
    uint64_t* state;
    uint32_t* ticket;
};

FilterScratch filter_scratch_layout(void* ws, int64_t ntiles) {
    WsAlloc wa(ws);
    FilterScratch f;
    f.state = wa.take<uint64_t>(ntiles > 0 ? ntiles : 1);
    f.ticket = wa.take<uint32_t>(1);
    return f;
}

template <typename T, bool SEL>
int launch_filter(const void* col, const int32_t* sel, int64_t n_cand, int cmp, int64_t lit, int32_t* out,
                  int64_t* d_n_out, int32_t* d_status, void* ws, hipStream_t s) {
    using S = FilterShape<T, SEL>;
    const int64_t ntiles = ceil_div(n_cand, S::TILE_ROWS);
    const FilterScratch f = filter_scratch_layout(ws, ntiles);
    uint64_t* state = f.state;
    uint32_t* ticket = f.ticket;
    int ib = (int)std::min<int64_t>(std::max<int64_t>(ceil_div(ntiles, 256), 1), 1024);
    filter_init_kernel<<<ib, 256, 0, s>>>(state, ntiles, ticket, d_n_out, d_status);
    if (ntiles > 0) {
        filter_kernel<T, SEL><<<(uint32_t)ntiles, kFilterThreads, 0, s>>>(
            (const T*)col, sel, n_cand, cmp, lit, out, d_n_out, state, ticket, (uint32_t)ntiles, d_status);
    }
    return launch_status("tdp_filter");
}

}  // namespace

}  // namespace tdp

using namespace tdp;

extern "C" size_t tdp_filter_workspace_size(int64_t n_candidates) {
    // Smallest tile (16384 candidates) bounds the number of tiles for every dtype.
    int64_t ntiles = n_candidates > 0 ? ceil_div(n_candidates, 16384) : 1;
    WsAlloc wa(nullptr);
    wa.take<uint64_t>(ntiles);
    wa.take<uint32_t>(1);
    return wa.bytes();
}

namespace tdp {
namespace {

// Argument checks shared by both filter entry points (everything except the
// workspace); returns TDP_OK or the failure, with *n_cand set.
int filter_check(const char* fn, const tdp_col* col, int32_t cmp, const int32_t* sel_in, int64_t n_sel_in,
                 int32_t* rows_out, int64_t cap, int64_t* d_n_out, int64_t max_cand, int64_t* n_cand_out) {
    if (!col || !d_n_out) return fail(TDP_EINVAL, "%s: null column or count pointer", fn);
    if (col->n < 0 || (sel_in && n_sel_in < 0)) return fail(TDP_EINVAL, "%s: negative size", fn);
    if (!int_dtype(col->dtype)) return fail(TDP_EUNSUPPORTED, "%s: column dtype %d", fn, col->dtype);
    if (cmp < TDP_LT || cmp > TDP_NE) return fail(TDP_EINVAL, "%s: comparison %d", fn, cmp);
    const int64_t n_cand = sel_in ? n_sel_in : col->n;
    if (n_cand > max_cand)
        return fail(TDP_EINVAL, "%s: %lld candidates exceed the limit of %lld", fn, (long long)n_cand,
                    (long long)max_cand);
    if (n_cand > 0 && (!col->data || !rows_out)) return fail(TDP_EINVAL, "%s: null data or output", fn);
    if (cap < n_cand)
        return fail_need(TDP_ECAPACITY, n_cand, "%s: cap %lld < %lld candidates", fn, (long long)cap, (long long)n_cand);
    if (((uintptr_t)col->data & 15) || (sel_in && ((uintptr_t)sel_in & 15)))
        return fail(TDP_EINVAL, "%s: column and selection must be 16-byte aligned", fn);
    *n_cand_out = n_cand;
    return TDP_OK;
}

int dispatch_filter(const tdp_col* col, int32_t cmp, int64_t literal, const int32_t* sel_in, int64_t n_cand,
                    int32_t* rows_out, int64_t* d_n_out, int32_t* d_status, void* ws, hipStream_t stream) {
    switch (col->dtype) {
        case TDP_I8:
            return sel_in ? launch_filter<int8_t, true>(col->data, sel_in, n_cand, cmp, literal, rows_out, d_n_out, d_status, ws, stream)
                          : launch_filter<int8_t, false>(col->data, sel_in, n_cand, cmp, literal, rows_out, d_n_out, d_status, ws, stream);
        case TDP_I32:
            return sel_in ? launch_filter<int32_t, true>(col->data, sel_in, n_cand, cmp, literal, rows_out, d_n_out, d_status, ws, stream)
                          : launch_filter<int32_t, false>(col->data, sel_in, n_cand, cmp, literal, rows_out, d_n_out, d_status, ws, stream);
        default:
            return sel_in ? launch_filter<int64_t, true>(col->data, sel_in, n_cand, cmp, literal, rows_out, d_n_out, d_status, ws, stream)
                          : launch_filter<int64_t, false>(col->data, sel_in, n_cand, cmp, literal, rows_out, d_n_out, d_status, ws, stream);
    }
}

// ------------------------------------------------ allocation-free variant
// Scratch of tdp_filter_noalloc: the tile states and the ticket of up to
// kNoAllocMaxCand candidates (the smallest tile, 16384 candidates, bounds the
// tile count for every dtype).  Each GPU holds its own copy for the life of
// the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device.
constexpr int64_t kNoAllocMaxCand = INT32_MAX;
constexpr int64_t kNoAllocTiles = (kNoAllocMaxCand + 16383) / 16384;
constexpr size_t kNoAllocBytes = ((kNoAllocTiles * sizeof(uint64_t) + 255) & ~(size_t)255) + 256;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch, looked up once per device with
// that device current (it is the caller's current device).
int scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(TDP_EDEVICE, "tdp_filter_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(TDP_EDEVICE, "tdp_filter_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(TDP_EDEVICE, "tdp_filter_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TDP_OK;
}

}  // namespace
}  // namespace tdp

extern "C" int tdp_filter(const tdp_col* col, int32_t cmp, int64_t literal, const int32_t* sel_in, int64_t n_sel_in,
                          int32_t* rows_out, int64_t cap, int64_t* d_n_out, int32_t* d_status, void* ws,
                          size_t ws_bytes, hipStream_t stream) {
    int64_t n_cand = 0;
    int rc = filter_check("tdp_filter", col, cmp, sel_in, n_sel_in, rows_out, cap, d_n_out, INT32_MAX, &n_cand);
    if (rc != TDP_OK) return rc;
    if (!ws || ws_bytes < tdp_filter_workspace_size(n_cand))
        return fail_need(TDP_EWORKSPACE, (int64_t)tdp_filter_workspace_size(n_cand), "tdp_filter: workspace %zu < %zu",
                         ws_bytes, tdp_filter_workspace_size(n_cand));
    return dispatch_filter(col, cmp, literal, sel_in, n_cand, rows_out, d_n_out, d_status, ws, stream);
}

extern "C" int64_t tdp_filter_noalloc_max_candidates(void) { return kNoAllocMaxCand; }

extern "C" int tdp_filter_noalloc(const tdp_col* col, int32_t cmp, int64_t literal, const int32_t* sel_in,
                                  int64_t n_sel_in, int32_t* rows_out, int64_t cap, int64_t* d_n_out,
                                  int32_t* d_status, hipStream_t stream) {
    int64_t n_cand = 0;
    int rc = filter_check("tdp_filter_noalloc", col, cmp, sel_in, n_sel_in, rows_out, cap, d_n_out, kNoAllocMaxCand,
                          &n_cand);
    if (rc != TDP_OK) return rc;
    if (tdp_filter_workspace_size(n_cand) > kNoAllocBytes)
        return fail(TDP_EINVAL, "tdp_filter_noalloc: %lld candidates need %zu scratch bytes, more than %zu",
                    (long long)n_cand, tdp_filter_workspace_size(n_cand), kNoAllocBytes);
    void* ws = nullptr;
    rc = scratch_address(&ws);
    if (rc != TDP_OK) return rc;
    return dispatch_filter(col, cmp, literal, sel_in, n_cand, rows_out, d_n_out, d_status, ws, stream);
}
