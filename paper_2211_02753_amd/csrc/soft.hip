// Relaxed (differentiable) filter and grouped aggregation, forward and
// backward.
//
// The logistic w = 1 / (1 + exp(-z)), z = (c - x) / tau, is evaluated from
// t = exp(-|z|) as w = 1 / (1 + t) (z >= 0) or t / (1 + t) (z < 0), and its
// derivative factor as w (1 - w) = t / (1 + t)^2, so neither side of the
// step loses precision to cancellation.  The backward kernels recompute w
// from x instead of reading a stored mask.
//
// Scatter-adds go to an LDS copy of the group table per workgroup; each
// workgroup writes its table as one row of partial sums (plain coalesced
// stores, no global atomics), and one finishing kernel sums the rows in a
// fixed order: each workgroup takes 64 columns, adds 16 row slices in
// float64 and the slices in order, rounds S to float32 and, in the fused
// forward, evaluates its columns' squared errors and the loss gradient; the
// loss total is the workgroups' partials added in order by the workgroup
// that arrives last.  Tables too large for LDS
// add straight into a float64 accumulator with global atomics.  Scalar
// reductions (dc) write one float64 partial per workgroup, summed in
// workgroup order by a one-workgroup finishing kernel: the backward kernels
// write a value per row, and a device-wide fence at the end of each of
// their workgroups would write those lines back from the L2 early.  The
// finishing code also returns the float64 accumulator, the arrival counters
// and the flag word to zero, so a workspace prepared once by
// tdp_soft_workspace_init needs no clearing launch per call.
#include "common.hpp"

namespace tdp {

namespace {

constexpr int kSoftThreads = 256;
constexpr int kMaxLdsFloats = 16384;  // 64 KiB of LDS per workgroup
constexpr int64_t kMaxGK = 65536 * 16;
constexpr int kMaxGrid = 8 * 256;     // workgroups of a streaming soft kernel
constexpr int64_t kRowFloats = 16 << 20;  // partial-row storage (64 MiB)
constexpr int kSqMaxPreds = 4;        // conjuncts of a soft WHERE clause
constexpr int kSqScalars = 2 * kSqMaxPreds;  // dc[J] and dtau[J]
// Threads of a fused soft forward workgroup: one 1024-thread workgroup per
// CU writes a quarter of the partial rows that four 256-thread ones would
// (measured: forward plus reduction 38 -> 33 us over 10M rows, 1000 groups).
constexpr int kFwdThreads = 1024;
// Reduction of the partial rows: a 1024-thread workgroup per 64 columns, 16
// row slices per column; the loss total through one arrival counter.
constexpr int kRfCols = 64;
constexpr int kRfSlices = 16;
constexpr int kTreeTicks = 1;

struct SoftWs {
    double* acc;          // [kMaxGK] float64 group accumulator (large tables)
    float* rows;          // [grid][GK] per-workgroup partial tables (LDS-sized tables)
    double* part;         // [kMaxGrid] per-workgroup scalar partials (dc)
    double* part2;        // [kMaxGrid] second scalar partials (dtau)
    double* partq;        // [kSqScalars][kMaxGrid] scalar partials of the soft query backward
    uint32_t* tick;       // [kTreeTicks] arrival counters of the in-kernel row reduction (zero between calls)
    int32_t* flags;       // device condition bits of the running call
};

SoftWs soft_layout(void* ws, size_t* bytes) {
    WsAlloc wa(ws);
    SoftWs s;
    s.acc = wa.take<double>(kMaxGK);
    s.rows = wa.take<float>(kRowFloats);
    s.part = wa.take<double>(kMaxGrid);
    s.part2 = wa.take<double>(kMaxGrid);
    s.partq = wa.take<double>((size_t)kSqScalars * kMaxGrid);
    s.tick = wa.take<uint32_t>(kTreeTicks);
    s.flags = wa.take<int32_t>(1);
    if (bytes) *bytes = wa.bytes();
    return s;
}

// Float add into LDS by compare-and-swap on the bit pattern.  Measured on
// gfx950: the native LDS float add runs at about one lane every two cycles
// per CU, the 32-bit compare-and-swap at the integer atomic rate, so the
// soft group-by forward over 10M rows and 1000 groups takes 39 us instead of
// 71 us.  Each add still rounds once in float32, in arrival order, exactly
// as the native one; comparing bits ends the loop also when the slot holds
// a NaN.
__device__ __forceinline__ void lds_add_f32(float* p, float v) {
    unsigned* q = reinterpret_cast<unsigned*>(p);
    unsigned old = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (true) {
        const unsigned assumed = old;
        old = atomicCAS(q, assumed, __float_as_uint(__uint_as_float(assumed) + v));
        if (old == assumed) break;
    }
}

// Group j of a workgroup's LDS table kept as `copies` per-wave copies (one
// per wave when the copies fit, so that compare-and-swap adds contend only
// within a wave): the copies added in wave order in float64.
__device__ __forceinline__ float sum_copies(const float* s_tab, int G, int copies, int j) {
    if (copies == 1) return s_tab[j];
    double a = 0.0;
    for (int c = 0; c < copies; ++c) a += (double)s_tab[c * G + j];
    return (float)a;
}

// Copies of an LDS group table a 1024-thread forward keeps: one per wave
// when they fit the LDS budget, else one.
int table_copies(int64_t G) { return G * (kFwdThreads / kWave) <= kMaxLdsFloats ? kFwdThreads / kWave : 1; }

__device__ __forceinline__ float logistic_t(float z, float& wd) {
    const float t = __expf(-fabsf(z));
    const float r = __builtin_amdgcn_rcpf(1.0f + t);
    wd = t * r * r;  // w (1 - w)
    return z >= 0.0f ? r : t * r;
}

__global__ void soft_init_kernel(SoftWs s) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < kMaxGK; i += stride) s.acc[i] = 0.0;
    if (blockIdx.x == 0 && threadIdx.x < kTreeTicks) s.tick[threadIdx.x] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *s.flags = 0;
    }
}

// Run by a finishing kernel after the accumulators are consumed: report the
// call's flags and clear them for the next call.
__device__ __forceinline__ void release_scalars(const SoftWs& s, int32_t* d_status) {
    if (threadIdx.x == 0) {
        if (d_status) *d_status = __hip_atomic_load(s.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *s.flags = 0;
    }
}

constexpr int kFinishThreads = 1024;  // threads of the one-workgroup finishing kernels

// Block sum of one float64 per thread (up to 1024 threads); valid in thread 0.
__device__ __forceinline__ double block_sum_f64(double v) {
    __shared__ double s_w[kFinishThreads / kWave];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if (lane_id() == 0) s_w[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)blockDim.x / kWave; ++w) t += s_w[w];
    __syncthreads();  // s_w is read before a following call in the same kernel overwrites it
    return t;
}

// Round the float64 accumulator to S, zeroing it; optionally the MSE against
// T.  Runs in its own launch after the kernels that added into it, so plain
// loads see their sums.
__device__ void finish_groups(const SoftWs& ws, int64_t GK, float* S, const float* T, float* d_loss, float* dS) {
    double part = 0.0;
    for (int64_t j = threadIdx.x; j < GK; j += blockDim.x) {
        const double s = ws.acc[j];
        ws.acc[j] = 0.0;
        S[j] = (float)s;
        if (T) {
            const double d = s - (double)T[j];
            part += d * d;
            dS[j] = (float)(2.0 * d / (double)GK);
        }
    }
    if (T) {
        const double tot = block_sum_f64(part);
        if (threadIdx.x == 0) *d_loss = (float)(tot / (double)GK);
    }
}

// Arrival of a workgroup at one level of the in-kernel reduction: true in
// the workgroup that arrives last of `members`, which then reads what the
// others wrote before they arrived.  The counter is returned to zero.  The
// barrier completes the workgroup's stores; one thread's device-scope fences
// then publish them (and, in the last arrival, make the others' visible) --
// a fence per wave would repeat the L2 write-back and invalidation per wave.
__device__ bool tree_arrive(uint32_t* tick, int members) {
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t t = atomicAdd(tick, 1u);
        const bool last = t == (uint32_t)members - 1;
        if (last) {
            __hip_atomic_store(tick, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
        }
        s_last = last;
    }
    __syncthreads();
    return s_last;
}

// The rows [nrows][GK] summed and finished: workgroup b takes columns
// b*64 .. b*64+63; thread (slice, column) adds rows slice, slice + 16, ... in
// float64 (loads issued 16 at a time), the 16 slices are added in order.
// With T, each workgroup's squared errors go to ws.part[b] and the last
// workgroup to arrive adds those in order for the loss.
__global__ __launch_bounds__(kFinishThreads) void soft_rows_finish_kernel(SoftWs ws, int nrows, int64_t GK, float* S,
                                                                        const float* T, float* d_loss, float* dS,
                                                                        int32_t* status) {
    __shared__ double s_acc[kRfSlices][kRfCols];
    const int c = threadIdx.x % kRfCols, sl = threadIdx.x / kRfCols;
    const int64_t j = (int64_t)blockIdx.x * kRfCols + c;
    double acc = 0.0;
    if (j < GK) {
        for (int r0 = sl; r0 < nrows; r0 += 16 * kRfSlices) {
            float t[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int row = r0 + k * kRfSlices;
                t[k] = row < nrows ? ws.rows[(int64_t)row * GK + j] : 0.0f;
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) acc += (double)t[k];
        }
    }
    s_acc[sl][c] = acc;
    __syncthreads();
    double part = 0.0;
    if (threadIdx.x < kRfCols && j < GK) {
        double tot = 0.0;
#pragma unroll
        for (int k = 0; k < kRfSlices; ++k) tot += s_acc[k][c];
        S[j] = (float)tot;
        if (T) {
            const double d = tot - (double)T[j];
            part = d * d;
            dS[j] = (float)(2.0 * d / (double)GK);
        }
    }
    if (!T) {
        if (blockIdx.x == 0) release_scalars(ws, status);
        return;
    }
    const double wg_part = block_sum_f64(part);
    if (threadIdx.x == 0) ws.part[blockIdx.x] = wg_part;
    if (!tree_arrive(&ws.tick[0], gridDim.x)) return;
    double v = 0.0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) v += ws.part[i];
    const double loss = block_sum_f64(v);
    if (threadIdx.x == 0) *d_loss = (float)(loss / (double)GK);
    release_scalars(ws, status);
}

// One workgroup: the groups from the float64 accumulator, the loss when T is
// given, and the call's flags.
__global__ __launch_bounds__(kFinishThreads) void soft_groups_finish_kernel(SoftWs ws, int64_t GK, float* S,
                                                                          const float* T, float* d_loss, float* dS,
                                                                          int32_t* status) {
    finish_groups(ws, GK, S, T, d_loss, dS);
    release_scalars(ws, status);
}

// One workgroup: the scalar from the per-workgroup partials.
__global__ __launch_bounds__(kSoftThreads) void soft_scalar_finish_kernel(SoftWs ws, int n_parts, float* out,
                                                                          float* out2) {
    // all partials loaded before the first add (n_parts <= kMaxGrid), added in order
    double t[kMaxGrid / kSoftThreads];
#pragma unroll
    for (int k = 0; k < kMaxGrid / kSoftThreads; ++k) {
        const int i = threadIdx.x + k * kSoftThreads;
        t[k] = i < n_parts ? ws.part[i] : 0.0;
    }
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxGrid / kSoftThreads; ++k) v += t[k];
    const double tot = block_sum_f64(v);
    if (threadIdx.x == 0) *out = (float)tot;
    if (out2) {  // the second scalar, the same way
#pragma unroll
        for (int k = 0; k < kMaxGrid / kSoftThreads; ++k) {
            const int i = threadIdx.x + k * kSoftThreads;
            t[k] = i < n_parts ? ws.part2[i] : 0.0;
        }
        double v2 = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxGrid / kSoftThreads; ++k) v2 += t[k];
        const double tot2 = block_sum_f64(v2);
        if (threadIdx.x == 0) *out2 = (float)tot2;
    }
}

// ------------------------------------------------------------ soft filter

__global__ __launch_bounds__(kSoftThreads) void soft_filter_kernel(const float* __restrict__ x, int64_t n,
                                                                   const float* __restrict__ d_c, float inv_tau,
                                                                   float* __restrict__ w) {
    const float c = *d_c;
    const int64_t stride = (int64_t)gridDim.x * kSoftThreads * 4;
    for (int64_t i = ((int64_t)blockIdx.x * kSoftThreads + threadIdx.x) * 4; i < n; i += stride) {
        if (i + 4 <= n) {
            const float4 xv = *(const float4*)(x + i);
            float wd;
            float4 o;
            o.x = logistic_t((c - xv.x) * inv_tau, wd);
            o.y = logistic_t((c - xv.y) * inv_tau, wd);
            o.z = logistic_t((c - xv.z) * inv_tau, wd);
            o.w = logistic_t((c - xv.w) * inv_tau, wd);
            *(float4*)(w + i) = o;
        } else {
            for (int64_t j = i; j < n; ++j) {
                float wd;
                w[j] = logistic_t((c - x[j]) * inv_tau, wd);
            }
        }
    }
}

__global__ __launch_bounds__(kSoftThreads) void soft_filter_bwd_kernel(const float* __restrict__ x, int64_t n,
                                                                       const float* __restrict__ d_c, float inv_tau,
                                                                       const float* __restrict__ dw,
                                                                       float* __restrict__ dx, SoftWs ws,
                                                                       float* d_dc) {
    const float c = *d_c;
    float part = 0.0f, part_tau = 0.0f;
    const int64_t stride = (int64_t)gridDim.x * kSoftThreads;
    for (int64_t i = (int64_t)blockIdx.x * kSoftThreads + threadIdx.x; i < n; i += stride) {
        float wd;
        const float z = (c - x[i]) * inv_tau;
        logistic_t(z, wd);
        const float t = dw[i] * wd * inv_tau;
        if (dx) dx[i] = -t;
        part += t;
        part_tau -= t * z;  // dw/dtau = -w (1 - w) z / tau
    }
    const double tot = block_sum_f64((double)part);
    if (threadIdx.x == 0) ws.part[blockIdx.x] = tot;
    const double tot_tau = block_sum_f64((double)part_tau);
    if (threadIdx.x == 0) ws.part2[blockIdx.x] = tot_tau;
}

// ------------------------------------------------------- soft group-by

template <bool LDS>
__global__ __launch_bounds__(kSoftThreads) void soft_groupby_kernel(const int32_t* __restrict__ g,
                                                                    const float* __restrict__ w,
                                                                    const float* __restrict__ v, int64_t n, int K,
                                                                    int G, SoftWs ws, float* S, int32_t* status) {
    double* acc = ws.acc;
    extern __shared__ float s_tab[];
    const int64_t GK = (int64_t)G * K;
    if (LDS) {
        for (int64_t j = threadIdx.x; j < GK; j += kSoftThreads) s_tab[j] = 0.0f;
        __syncthreads();
    }
    const int64_t stride = (int64_t)gridDim.x * kSoftThreads;
    for (int64_t i = (int64_t)blockIdx.x * kSoftThreads + threadIdx.x; i < n; i += stride) {
        const int32_t gi = g[i];
        if (gi < 0 || gi >= G) {
            raise_flag(ws.flags, TDP_FLAG_GROUP_RANGE);
            continue;
        }
        const float wi = w ? w[i] : 1.0f;
        for (int k = 0; k < K; ++k) {
            const float val = wi * v[i * K + k];
            if (LDS)
                lds_add_f32(&s_tab[(int64_t)gi * K + k], val);
            else
                atomicAdd(&acc[(int64_t)gi * K + k], (double)val);
        }
    }
    if (LDS) {
        __syncthreads();
        for (int64_t j = threadIdx.x; j < GK; j += kSoftThreads) ws.rows[(int64_t)blockIdx.x * GK + j] = s_tab[j];
        return;  // the reduction kernel finishes
    }

}

__global__ __launch_bounds__(kSoftThreads) void soft_groupby_bwd_kernel(const int32_t* __restrict__ g,
                                                                        const float* __restrict__ w,
                                                                        const float* __restrict__ v,
                                                                        const float* __restrict__ dS, int64_t n, int K,
                                                                        int G, float* __restrict__ dw,
                                                                        float* __restrict__ dv) {
    const int64_t stride = (int64_t)gridDim.x * kSoftThreads;
    for (int64_t i = (int64_t)blockIdx.x * kSoftThreads + threadIdx.x; i < n; i += stride) {
        const int32_t gi = g[i];
        const bool in = gi >= 0 && gi < G;
        const float wi = w ? w[i] : 1.0f;
        float acc = 0.0f;
        for (int k = 0; k < K; ++k) {
            const float d = in ? dS[(int64_t)gi * K + k] : 0.0f;
            if (dv) dv[i * K + k] = d * wi;
            acc += d * v[i * K + k];
        }
        if (dw) dw[i] = acc;
    }
}

// ------------------------------------------- fused soft filter + group-by

// Four consecutive rows of (x, v, g) from row i0 (g = -1 past the end).
__device__ __forceinline__ void load_xvg4(const float* __restrict__ x, const float* __restrict__ v,
                                          const int32_t* __restrict__ g, int64_t i0, int64_t n, float xs[4],
                                          float vs[4], int32_t gs[4]) {
    if (i0 + 4 <= n) {
        const float4 xv = *(const float4*)(x + i0);
        const float4 vv = *(const float4*)(v + i0);
        const int4 gv = *(const int4*)(g + i0);
        xs[0] = xv.x; xs[1] = xv.y; xs[2] = xv.z; xs[3] = xv.w;
        vs[0] = vv.x; vs[1] = vv.y; vs[2] = vv.z; vs[3] = vv.w;
        gs[0] = gv.x; gs[1] = gv.y; gs[2] = gv.z; gs[3] = gv.w;
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool in = i0 + e < n;
            xs[e] = in ? x[i0 + e] : 0.0f;
            vs[e] = in ? v[i0 + e] : 0.0f;
            gs[e] = in ? g[i0 + e] : -1;
        }
    }
}

// Each thread takes two groups of four rows per step (rows i0.. and
// i0 + half-stride..), issuing all six vector loads before the first
// scatter-add, so twice the bytes are in flight per wave.
template <bool LDS>
__global__ __launch_bounds__(kFwdThreads) void soft_fg_fwd_kernel(const float* __restrict__ x,
                                                                   const float* __restrict__ v,
                                                                   const int32_t* __restrict__ g, int64_t n,
                                                                   const float* __restrict__ d_c, float inv_tau, int G,
                                                                   int copies, SoftWs ws, float* S, const float* T,
                                                                   float* d_loss, float* dS, int32_t* status) {
    extern __shared__ float s_tab[];
    double* acc = ws.acc;
    const int tab = (int)(threadIdx.x / kWave) % copies * G;  // this wave's copy of the table
    if (LDS) {
        for (int j = threadIdx.x; j < copies * G; j += kFwdThreads) s_tab[j] = 0.0f;
        __syncthreads();
    }
    const float c = *d_c;
    const int64_t half = (int64_t)gridDim.x * kFwdThreads * 4;
    for (int64_t i0 = ((int64_t)blockIdx.x * kFwdThreads + threadIdx.x) * 4; i0 < n; i0 += 2 * half) {
        float xs[8], vs[8];
        int32_t gs[8];
        load_xvg4(x, v, g, i0, n, xs, vs, gs);
        load_xvg4(x, v, g, i0 + half, n, xs + 4, vs + 4, gs + 4);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if (gs[e] == -1 && (e < 4 ? i0 + e : i0 + half + e - 4) >= n) continue;  // past the end
            if (gs[e] < 0 || gs[e] >= G) {
                raise_flag(ws.flags, TDP_FLAG_GROUP_RANGE);
                continue;
            }
            float wd;
            const float val = logistic_t((c - xs[e]) * inv_tau, wd) * vs[e];
            if (LDS)
                lds_add_f32(&s_tab[tab + gs[e]], val);
            else
                atomicAdd(&acc[gs[e]], (double)val);
        }
    }
    if (LDS) {
        __syncthreads();
        for (int j = threadIdx.x; j < G; j += kFwdThreads) ws.rows[(int64_t)blockIdx.x * G + j] = sum_copies(s_tab, G, copies, j);
    }
}

template <bool LDS>
__global__ __launch_bounds__(kSoftThreads) void soft_fg_bwd_kernel(const float* __restrict__ x,
                                                                   const float* __restrict__ v,
                                                                   const int32_t* __restrict__ g, int64_t n,
                                                                   const float* __restrict__ d_c, float inv_tau, int G,
                                                                   const float* __restrict__ dS,
                                                                   float* __restrict__ dv, float* __restrict__ dx,
                                                                   SoftWs ws, float* d_dc) {
    extern __shared__ float s_ds[];
    const float* tab = dS;
    if (LDS) {
        for (int j = threadIdx.x; j < G; j += kSoftThreads) s_ds[j] = dS[j];
        __syncthreads();
        tab = s_ds;
    }
    const float c = *d_c;
    float part = 0.0f, part_tau = 0.0f;
    const int64_t stride = (int64_t)gridDim.x * kSoftThreads * 4;
    for (int64_t i0 = ((int64_t)blockIdx.x * kSoftThreads + threadIdx.x) * 4; i0 < n; i0 += stride) {
        float xs[4], vs[4], dvs[4], dxs[4];
        int32_t gs[4];
        const bool full = i0 + 4 <= n;
        if (full) {
            const float4 xv = *(const float4*)(x + i0);
            const float4 vv = *(const float4*)(v + i0);
            const int4 gv = *(const int4*)(g + i0);
            xs[0] = xv.x; xs[1] = xv.y; xs[2] = xv.z; xs[3] = xv.w;
            vs[0] = vv.x; vs[1] = vv.y; vs[2] = vv.z; vs[3] = vv.w;
            gs[0] = gv.x; gs[1] = gv.y; gs[2] = gv.z; gs[3] = gv.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool in = i0 + e < n;
                xs[e] = in ? x[i0 + e] : 0.0f;
                vs[e] = in ? v[i0 + e] : 0.0f;
                gs[e] = in ? g[i0 + e] : -1;
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool in = gs[e] >= 0 && gs[e] < G;
            const float d = in ? tab[gs[e]] : 0.0f;
            float wd;
            const float z = (c - xs[e]) * inv_tau;
            const float w = logistic_t(z, wd);
            const float t = d * vs[e] * wd * inv_tau;
            dvs[e] = d * w;
            dxs[e] = -t;
            part += t;
            part_tau -= t * z;  // dw/dtau = -w (1 - w) z / tau
        }
        if (full) {
            *(float4*)(dv + i0) = make_float4(dvs[0], dvs[1], dvs[2], dvs[3]);
            if (dx) *(float4*)(dx + i0) = make_float4(dxs[0], dxs[1], dxs[2], dxs[3]);
        } else {
            for (int e = 0; e < 4; ++e) {
                if (i0 + e < n) {
                    dv[i0 + e] = dvs[e];
                    if (dx) dx[i0 + e] = dxs[e];
                }
            }
        }
    }
    const double tot = block_sum_f64((double)part);
    if (threadIdx.x == 0) ws.part[blockIdx.x] = tot;
    const double tot_tau = block_sum_f64((double)part_tau);
    if (threadIdx.x == 0) ws.part2[blockIdx.x] = tot_tau;
}

// One 1024-thread workgroup; eight elements per thread and step, all loads
// issued before the first use.
__global__ __launch_bounds__(kFinishThreads) void mse_kernel(const float* S, const float* T, int G, float* d_loss,
                                                             float* dS) {
    double part = 0.0;
    for (int j0 = threadIdx.x; j0 < G; j0 += 8 * kFinishThreads) {
        float s[8], t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int j = j0 + k * kFinishThreads;
            s[k] = j < G ? S[j] : 0.0f;
            t[k] = j < G ? T[j] : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int j = j0 + k * kFinishThreads;
            const double d = (double)s[k] - (double)t[k];
            part += d * d;
            if (dS && j < G) dS[j] = (float)(2.0 * d / (double)G);
        }
    }
    const double tot = block_sum_f64(part);
    if (threadIdx.x == 0) *d_loss = (float)(tot / (double)G);
}

int soft_grid(int64_t n, int rows_per_thread) {
    int64_t b = ceil_div(std::max<int64_t>(n, 1), (int64_t)kSoftThreads * rows_per_thread);
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), kMaxGrid);
}

int check_ws(void* ws, size_t ws_bytes, const char* what) {
    size_t need;
    soft_layout(nullptr, &need);
    if (!ws || ws_bytes < need) return fail_need(TDP_EWORKSPACE, (int64_t)need, "%s: workspace %zu < %zu", what, ws_bytes, need);
    if ((uintptr_t)ws & 255) return fail(TDP_EINVAL, "%s: workspace not 256-byte aligned", what);
    return TDP_OK;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

void launch_reduce(const SoftWs& s, int nrows, int64_t GK, float* S, const float* T, float* d_loss, float* dS,
                   int32_t* d_status, hipStream_t stream) {
    if (nrows > 0) {
        soft_rows_finish_kernel<<<(unsigned)ceil_div(GK, kRfCols), kFinishThreads, 0, stream>>>(s, nrows, GK, S, T,
                                                                                               d_loss, dS, d_status);
        return;
    }
    soft_groups_finish_kernel<<<1, kFinishThreads, 0, stream>>>(s, GK, S, T, d_loss, dS, d_status);
}


// --------------------------- soft COUNT grouped by two probability columns
// S[g][a][b] = sum over the rows i of segment g of p[i][a] * q[i][b]: the
// count of Section 4 on probability-encoded data (+ and * only), grouped by
// two predicted attributes as in the grid-of-images query.  A wave takes one
// work item (a segment, or without segments an equal chunk of the rows) and
// walks it in tiles of T rows: the tile's p and q rows are contiguous in
// memory, so the wave copies them to its own LDS area with 16-byte loads
// (all in flight together), then computes from LDS.  The forward maps lane
// l to cell c = l % C, (a, b) = (c / K2, c % K2), for row slot l / C; the
// backward maps lanes to rows and writes dp and dq through LDS with 16-byte
// stores.

// ------------------------------------------- soft form of a groupby query
// The relaxed counterpart of the exact grouped query: every conjunct of the
// WHERE clause is a logistic factor, the conjunction their product, and the
// grouped aggregate a scatter-add of w * e into the dense group table.

struct SqPred {
    const void* p;
    int32_t dt;
    float s;        // +1 (x below the threshold) or -1 (above)
};

struct SqDev {
    int64_t n;
    int J;
    SqPred pr[kSqMaxPreds];
    const float* c;           // [J] thresholds (device)
    const float* tau;         // [J] temperatures (device)
    int n_keys;
    const void* kp[2];
    int32_t kdt[2];
    int64_t lo[2], card[2];
    int G;
    const void* a;            // value column, or null for COUNT
    int32_t adt;
};

// Four consecutive values from row i0 (a multiple of 4) as float32 / int64;
// rows at or past n read 0.  Columns are 16-byte aligned.
__device__ __forceinline__ void sq_load4f(const void* p, int dt, int64_t i0, int64_t n, float v[4]) {
    if (i0 + 4 <= n) {
        if (dt == TDP_F32) {
            const float4 q = *(const float4*)((const float*)p + i0);
            v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else if (dt == TDP_I32) {
            const int4 q = *(const int4*)((const int32_t*)p + i0);
            v[0] = (float)q.x; v[1] = (float)q.y; v[2] = (float)q.z; v[3] = (float)q.w;
        } else if (dt == TDP_I8) {
            const char4 q = *(const char4*)((const int8_t*)p + i0);
            v[0] = (float)q.x; v[1] = (float)q.y; v[2] = (float)q.z; v[3] = (float)q.w;
        } else {
            const longlong2 a = *(const longlong2*)((const int64_t*)p + i0);
            const longlong2 b = *(const longlong2*)((const int64_t*)p + i0 + 2);
            v[0] = (float)a.x; v[1] = (float)a.y; v[2] = (float)b.x; v[3] = (float)b.y;
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float t = 0.0f;
            if (i0 + e < n) {
                if (dt == TDP_F32) t = ((const float*)p)[i0 + e];
                else if (dt == TDP_I32) t = (float)((const int32_t*)p)[i0 + e];
                else if (dt == TDP_I8) t = (float)((const int8_t*)p)[i0 + e];
                else t = (float)((const int64_t*)p)[i0 + e];
            }
            v[e] = t;
        }
    }
}

__device__ __forceinline__ void sq_load4i(const void* p, int dt, int64_t i0, int64_t n, int64_t v[4]) {
    if (i0 + 4 <= n) {
        if (dt == TDP_I32) {
            const int4 q = *(const int4*)((const int32_t*)p + i0);
            v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else if (dt == TDP_I8) {
            const char4 q = *(const char4*)((const int8_t*)p + i0);
            v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else {
            const longlong2 a = *(const longlong2*)((const int64_t*)p + i0);
            const longlong2 b = *(const longlong2*)((const int64_t*)p + i0 + 2);
            v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int64_t t = 0;
            if (i0 + e < n) {
                if (dt == TDP_I32) t = ((const int32_t*)p)[i0 + e];
                else if (dt == TDP_I8) t = ((const int8_t*)p)[i0 + e];
                else t = ((const int64_t*)p)[i0 + e];
            }
            v[e] = t;
        }
    }
}

// Dense group id of four rows; -1 for a row outside its key domain (which
// raises the flag) or past the end.
__device__ __forceinline__ void sq_gids(const SqDev& d, int64_t i0, int64_t gid[4], int32_t* flags) {
    int64_t k0[4], k1[4] = {0, 0, 0, 0};
    sq_load4i(d.kp[0], d.kdt[0], i0, d.n, k0);
    if (d.n_keys > 1) sq_load4i(d.kp[1], d.kdt[1], i0, d.n, k1);
    const int64_t c1 = d.n_keys > 1 ? d.card[1] : 1;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t u0 = k0[e] - d.lo[0];
        const int64_t u1 = d.n_keys > 1 ? k1[e] - d.lo[1] : 0;
        const bool in = u0 >= 0 && u0 < d.card[0] && u1 >= 0 && u1 < c1;
        if (i0 + e >= d.n) {
            gid[e] = -1;
        } else if (!in) {
            raise_flag(flags, TDP_FLAG_KEY_DOMAIN);
            gid[e] = -1;
        } else {
            gid[e] = u0 * c1 + u1;
        }
    }
}

// Forward: each 1024-thread workgroup adds w * e of its rows into an LDS
// table (one partial row per workgroup, reduced in fixed order afterwards),
// or into the float64 accumulator when the table exceeds LDS.
template <bool LDS>
__global__ __launch_bounds__(kFwdThreads) void soft_query_fwd_kernel(SqDev d, int copies, SoftWs ws) {
    extern __shared__ float s_tab[];
    const int tab = (int)(threadIdx.x / kWave) % copies * d.G;  // this wave's copy of the table
    if (LDS) {
        for (int j = threadIdx.x; j < copies * d.G; j += kFwdThreads) s_tab[j] = 0.0f;
        __syncthreads();
    }
    float c[kSqMaxPreds], itau[kSqMaxPreds];
#pragma unroll
    for (int j = 0; j < kSqMaxPreds; ++j) {
        c[j] = j < d.J ? d.c[j] : 0.0f;
        const float t = j < d.J ? d.tau[j] : 1.0f;
        if (!(t > 0.0f && t < INFINITY) && threadIdx.x == 0) raise_flag(ws.flags, TDP_FLAG_BAD_PARAM);
        itau[j] = 1.0f / t;
    }
    const int64_t stride = (int64_t)gridDim.x * kFwdThreads * 4;
    for (int64_t i0 = ((int64_t)blockIdx.x * kFwdThreads + threadIdx.x) * 4; i0 < d.n; i0 += stride) {
        float w[4] = {1.0f, 1.0f, 1.0f, 1.0f}, ev[4] = {1.0f, 1.0f, 1.0f, 1.0f};
        int64_t gid[4];
        sq_gids(d, i0, gid, ws.flags);
        if (d.a) sq_load4f(d.a, d.adt, i0, d.n, ev);
#pragma unroll
        for (int j = 0; j < kSqMaxPreds; ++j) {
            if (j >= d.J) break;
            float x[4];
            sq_load4f(d.pr[j].p, d.pr[j].dt, i0, d.n, x);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float wd;
                w[e] *= logistic_t(d.pr[j].s * (c[j] - x[e]) * itau[j], wd);
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (gid[e] < 0) continue;
            const float val = w[e] * ev[e];
            if (LDS)
                lds_add_f32(&s_tab[tab + gid[e]], val);
            else
                atomicAdd(&ws.acc[gid[e]], (double)val);
        }
    }
    if (LDS) {
        __syncthreads();
        for (int j = threadIdx.x; j < d.G; j += kFwdThreads)
            ws.rows[(int64_t)blockIdx.x * d.G + j] = sum_copies(s_tab, d.G, copies, j);
    }
}

// Backward: recomputes every factor; per-workgroup float64 partials of
// dc[j] and dtau[j], and optionally de per row.
template <bool LDS>
__global__ __launch_bounds__(kSoftThreads) void soft_query_bwd_kernel(SqDev d, const float* __restrict__ dS,
                                                                      float* __restrict__ de, SoftWs ws) {
    extern __shared__ float s_ds[];
    const float* tab = dS;
    if (LDS) {
        for (int j = threadIdx.x; j < d.G; j += kSoftThreads) s_ds[j] = dS[j];
        __syncthreads();
        tab = s_ds;
    }
    float c[kSqMaxPreds], itau[kSqMaxPreds], pc[kSqMaxPreds], pt[kSqMaxPreds];
#pragma unroll
    for (int j = 0; j < kSqMaxPreds; ++j) {
        c[j] = j < d.J ? d.c[j] : 0.0f;
        itau[j] = 1.0f / (j < d.J ? d.tau[j] : 1.0f);
        pc[j] = pt[j] = 0.0f;
    }
    const int64_t stride = (int64_t)gridDim.x * kSoftThreads * 4;
    for (int64_t i0 = ((int64_t)blockIdx.x * kSoftThreads + threadIdx.x) * 4; i0 < d.n; i0 += stride) {
        float ev[4] = {1.0f, 1.0f, 1.0f, 1.0f};
        int64_t gid[4];
        sq_gids(d, i0, gid, nullptr);
        if (d.a) sq_load4f(d.a, d.adt, i0, d.n, ev);
        float z[kSqMaxPreds][4], om[kSqMaxPreds][4], w[4] = {1.0f, 1.0f, 1.0f, 1.0f};
#pragma unroll
        for (int j = 0; j < kSqMaxPreds; ++j) {
            if (j >= d.J) break;
            float x[4];
            sq_load4f(d.pr[j].p, d.pr[j].dt, i0, d.n, x);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float wd;
                z[j][e] = d.pr[j].s * (c[j] - x[e]) * itau[j];
                const float sg = logistic_t(z[j][e], wd);
                // 1 - sigma(z): w (1 - w) / w where sigma >= 1/2, else 1 - sigma
                // (neither form cancels on its side)
                om[j][e] = z[j][e] >= 0.0f ? wd / sg : 1.0f - sg;
                w[e] *= sg;
            }
        }
        float dv4[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float ds = gid[e] >= 0 ? tab[gid[e]] : 0.0f;
            dv4[e] = ds * w[e];
            const float t = ds * ev[e] * w[e];
#pragma unroll
            for (int j = 0; j < kSqMaxPreds; ++j) {
                if (j >= d.J) break;
                const float u = t * om[j][e] * itau[j];
                pc[j] += u * d.pr[j].s;
                pt[j] -= u * z[j][e];
            }
        }
        if (de) {
            if (i0 + 4 <= d.n) {
                *(float4*)(de + i0) = make_float4(dv4[0], dv4[1], dv4[2], dv4[3]);
            } else {
                for (int e = 0; e < 4; ++e)
                    if (i0 + e < d.n) de[i0 + e] = dv4[e];
            }
        }
    }
    for (int j = 0; j < d.J; ++j) {
        const double a = block_sum_f64((double)pc[j]);
        if (threadIdx.x == 0) ws.partq[(int64_t)j * kMaxGrid + blockIdx.x] = a;
        const double b = block_sum_f64((double)pt[j]);
        if (threadIdx.x == 0) ws.partq[(int64_t)(kSqMaxPreds + j) * kMaxGrid + blockIdx.x] = b;
    }
}

// One workgroup: dc[j] (and dtau[j]) from the per-workgroup partials, each
// summed in workgroup order.
__global__ __launch_bounds__(kSoftThreads) void soft_query_finish_kernel(SoftWs ws, int n_parts, int J, float* d_dc,
                                                                         float* d_dtau) {
    for (int k = 0; k < 2 * J; ++k) {
        const int j = k < J ? k : kSqMaxPreds + (k - J);
        float* out = k < J ? d_dc + k : (d_dtau ? d_dtau + (k - J) : nullptr);
        if (!out) continue;  // uniform across the workgroup
        double t[kMaxGrid / kSoftThreads];
#pragma unroll
        for (int q = 0; q < kMaxGrid / kSoftThreads; ++q) {
            const int i = threadIdx.x + q * kSoftThreads;
            t[q] = i < n_parts ? ws.partq[(int64_t)j * kMaxGrid + i] : 0.0;
        }
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < kMaxGrid / kSoftThreads; ++q) v += t[q];
        const double tot = block_sum_f64(v);
        if (threadIdx.x == 0) *out = (float)tot;
    }
}

constexpr int kPeMaxK = 16;      // values of one probability attribute
constexpr int kPeMaxCells = 64;  // K1 * K2: at most one wave lane per cell
constexpr int kPeWaves = kSoftThreads / kWave;
constexpr int kPeLdsBytes = 32 * 1024;  // LDS of one workgroup, all four waves

struct PeArgs {
    const int64_t* seg;  // [G + 1] row offsets, or null: one segment of all rows
    int64_t G;
    const float* p;      // [n][K1], 16-byte aligned
    const float* q;      // [n][K2], 16-byte aligned, or null: q = 1 with K2 = 1
    int K1, K2;
    int64_t n;
    int T;               // rows per tile
};

// LDS floats of one wave's tile of T rows of a K-wide column (alignment slack included).
__host__ __device__ constexpr int pe_tile_floats(int T, int K) { return T * K + 8; }

// Rows [lo, hi) of work item `it`: segment `it`, or the it-th of `items`
// equal chunks of all rows.  False (flag raised when `flags`) for a segment
// outside [0, n] or inverted.
__device__ __forceinline__ bool pe_rows(const PeArgs& A, int64_t it, int64_t items, int64_t& lo, int64_t& hi,
                                        int32_t* flags) {
    if (A.seg) {
        lo = A.seg[it];
        hi = A.seg[it + 1];
        if (lo < 0 || hi > A.n || hi < lo) {
            if (flags) raise_flag(flags, TDP_FLAG_GROUP_RANGE);
            lo = hi = 0;
            return false;
        }
        return true;
    }
    const int64_t chunk = (A.n + items - 1) / items;
    lo = it * chunk < A.n ? it * chunk : A.n;
    hi = lo + chunk < A.n ? lo + chunk : A.n;
    return true;
}


// A lane's share of a tile's words: the 16-byte words e = (f0 & ~3) +
// 4 (lane + 64 k), k < NW, that start before f1, loaded from src (16-byte
// aligned; words reaching past nsrc are read float by float) into registers
// while the wave still computes the previous tile, then written to LDS at
// e - (f0 & ~3).
template <int NW>
__device__ __forceinline__ void pe_issue(const float* __restrict__ src, int64_t f0, int64_t f1, int64_t nsrc,
                                         float4 (&v)[NW], int lane) {
    const int64_t a0 = f0 & ~(int64_t)3;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const int64_t e = a0 + 4 * (int64_t)(lane + kWave * k);
        if (e < f1) {
            if (e + 4 <= nsrc) {
                v[k] = *(const float4*)(src + e);
            } else {
                v[k].x = e < nsrc ? src[e] : 0.0f;
                v[k].y = e + 1 < nsrc ? src[e + 1] : 0.0f;
                v[k].z = e + 2 < nsrc ? src[e + 2] : 0.0f;
                v[k].w = e + 3 < nsrc ? src[e + 3] : 0.0f;
            }
        }
    }
}

template <int NW>
__device__ __forceinline__ void pe_commit(int64_t f0, int64_t f1, const float4 (&v)[NW], float* dst, int lane) {
    const int64_t a0 = f0 & ~(int64_t)3;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const int64_t e = a0 + 4 * (int64_t)(lane + kWave * k);
        if (e < f1) *(float4*)(dst + (e - a0)) = v[k];
    }
}

// 16-byte words a tile of T rows of a K-wide column spans.
__host__ __device__ constexpr int pe_tile_words(int T, int K) { return (T * K + 3 + 3) / 4; }

// dst[f0, f1) = src[k - (f0 & ~3)]: 16-byte stores for words inside
// [f0, f1), single floats at the two ends (the rest of those words belongs to
// other rows).
__device__ __forceinline__ void pe_store_tile(float* dst, int64_t f0, int64_t f1, const float* src, int lane) {
    const int64_t a0 = f0 & ~(int64_t)3;
    for (int64_t e = a0 + 4 * (int64_t)lane; e < f1; e += 4 * kWave) {
        if (e >= f0 && e + 4 <= f1) {
            *(float4*)(dst + e) = *(const float4*)(src + (e - a0));
        } else {
            for (int k = 0; k < 4; ++k)
                if (e + k >= f0 && e + k < f1) dst[e + k] = src[e + k - a0];
        }
    }
}

// The next tile of a wave's walk: the rest of item `it`, else the first
// tile of its next item (an invalid segment is an item with no rows).
struct PeCursor {
    int64_t it, lo, hi, t0;
};

__device__ __forceinline__ PeCursor pe_start(const PeArgs& A, int64_t it, int64_t items, int32_t* flags) {
    PeCursor c{it, 0, 0, 0};
    if (it < items) {
        pe_rows(A, it, items, c.lo, c.hi, flags);
        c.t0 = c.lo;
    }
    return c;
}

__device__ __forceinline__ PeCursor pe_next(const PeArgs& A, const PeCursor& c, int64_t t1, int64_t items,
                                            int64_t waves, int32_t* flags) {
    PeCursor n = c;
    n.t0 = t1;
    if (t1 >= c.hi) n = pe_start(A, c.it + waves, items, flags);
    return n;
}

// With segments the cell sums go straight to S[it]; without, each
// workgroup writes its waves' sums as one partial row, reduced in a fixed
// order by the finishing kernels.  A lane sums its rows of one tile in
// float32 (fused multiply-adds, at most T / R products of probabilities),
// tiles and row slots in float64.  The loads of the next tile are in flight
// while the current one is summed.
template <int NWP, int NWQ>
__global__ __launch_bounds__(kSoftThreads) void pe_fwd_kernel(PeArgs A, SoftWs ws, float* S) {
    extern __shared__ __attribute__((aligned(16))) float pe_lds[];
    __shared__ double s_w[kPeWaves][kPeMaxCells];
    const int lane = lane_id(), wv = threadIdx.x / kWave;
    const int K1 = A.K1, K2 = A.K2, C = K1 * K2, R = kWave / C;
    const int r = lane / C, c = lane - r * C, a = c / K2, b = c - a * K2;
    float* sp = pe_lds + wv * (pe_tile_floats(A.T, K1) + pe_tile_floats(A.T, K2));
    float* sq = sp + pe_tile_floats(A.T, K1);
    int32_t* flags = lane == 0 ? ws.flags : nullptr;
    const int64_t waves = (int64_t)gridDim.x * kPeWaves;
    const int64_t items = A.seg ? A.G : waves;
    PeCursor cur = pe_start(A, (int64_t)blockIdx.x * kPeWaves + wv, items, flags);
    float4 rp[NWP], rq[NWQ];
    if (cur.it < items && cur.t0 < cur.hi) {
        const int64_t t1 = cur.t0 + A.T < cur.hi ? cur.t0 + A.T : cur.hi;
        pe_issue(A.p, cur.t0 * K1, t1 * K1, A.n * K1, rp, lane);
        if (A.q) pe_issue(A.q, cur.t0 * K2, t1 * K2, A.n * K2, rq, lane);
    }
    double acc = 0.0, part = 0.0;
    while (cur.it < items) {
        const bool tile = cur.t0 < cur.hi;
        const int64_t t1 = !tile ? cur.t0 : (cur.t0 + A.T < cur.hi ? cur.t0 + A.T : cur.hi);
        wave_lds_sync();  // the previous tile is consumed
        if (tile) {
            pe_commit(cur.t0 * K1, t1 * K1, rp, sp, lane);
            if (A.q) pe_commit(cur.t0 * K2, t1 * K2, rq, sq, lane);
        }
        wave_lds_sync();
        const PeCursor nxt = pe_next(A, cur, t1, items, waves, flags);
        if (nxt.it < items && nxt.t0 < nxt.hi) {
            const int64_t n1 = nxt.t0 + A.T < nxt.hi ? nxt.t0 + A.T : nxt.hi;
            pe_issue(A.p, nxt.t0 * K1, n1 * K1, A.n * K1, rp, lane);
            if (A.q) pe_issue(A.q, nxt.t0 * K2, n1 * K2, A.n * K2, rq, lane);
        }
        if (tile && r < R) {
            const float* pp = sp + (cur.t0 * K1 - ((cur.t0 * K1) & ~(int64_t)3)) + a;
            const float* qq = sq + (cur.t0 * K2 - ((cur.t0 * K2) & ~(int64_t)3)) + b;
            const int rows = (int)(t1 - cur.t0);
            // a tile's rows of this slot (at most T / R, products of probabilities) in float32, then into float64
            float fa = 0.0f;
            for (int i = r; i < rows; i += R) fa = fmaf(pp[i * K1], A.q ? qq[i * K2] : 1.0f, fa);
            acc += (double)fa;
        }
        if (t1 >= cur.hi) {  // the item is complete: its row slots of each cell, added in slot order
            double tot = 0.0;
            const int src = lane < C ? lane : 0;
            for (int k = 0; k < R; ++k) tot += __shfl(acc, k * C + src, kWave);
            if (A.seg) {
                if (lane < C) S[cur.it * C + lane] = (float)tot;
            } else {
                part = tot;
            }
            acc = 0.0;
        }
        cur = nxt;
    }
    if (!A.seg) {
        if (lane < C) s_w[wv][lane] = part;
        __syncthreads();
        if ((int)threadIdx.x < C) {
            double t = 0.0;
            for (int w = 0; w < kPeWaves; ++w) t += s_w[w][threadIdx.x];
            ws.rows[(int64_t)blockIdx.x * C + threadIdx.x] = (float)t;
        }
    }
}

// Lane = row of the tile: dp[i][a] = sum_b dS[g][a][b] q[i][b] and
// dq[i][b] = sum_a dS[g][a][b] p[i][a] from the LDS copies.  Each lane reads
// only its own row, so it writes dp and dq over that row in LDS, and the
// tile leaves with 16-byte stores.  KQ bounds K2 at compile time (2 for the
// size attribute or q = 1, else 16), so the row's q values and dq sums stay
// in few registers.  The loads of the next tile (and its item's dS) are in
// flight while the current one is computed and stored.
template <int NWP, int NWQ, int KQ>
__global__ __launch_bounds__(kSoftThreads) void pe_bwd_kernel(PeArgs A, const float* __restrict__ dS, float* dp,
                                                              float* dq) {
    extern __shared__ __attribute__((aligned(16))) float pe_lds[];
    const int lane = lane_id(), wv = threadIdx.x / kWave;
    const int K1 = A.K1, K2 = A.K2, C = K1 * K2;
    const int fp = pe_tile_floats(A.T, K1), fq = pe_tile_floats(A.T, K2);
    float* sp = pe_lds + wv * (fp + fq + kPeMaxCells);
    float* sq = sp + fp;
    float* sd = sq + fq;
    const int64_t waves = (int64_t)gridDim.x * kPeWaves;
    const int64_t items = A.seg ? A.G : waves;
    PeCursor cur = pe_start(A, (int64_t)blockIdx.x * kPeWaves + wv, items, nullptr);
    float4 rp[NWP], rq[NWQ];
    float dreg = 0.0f;  // this lane's cell of dS for the item whose first tile is in flight
    if (cur.it < items && cur.t0 < cur.hi) {
        const int64_t t1 = cur.t0 + A.T < cur.hi ? cur.t0 + A.T : cur.hi;
        pe_issue(A.p, cur.t0 * K1, t1 * K1, A.n * K1, rp, lane);
        if (A.q) pe_issue(A.q, cur.t0 * K2, t1 * K2, A.n * K2, rq, lane);
        if (lane < C) dreg = dS[(A.seg ? cur.it : 0) * C + lane];
    }
    while (cur.it < items) {
        const bool tile = cur.t0 < cur.hi;
        const int64_t t1 = !tile ? cur.t0 : (cur.t0 + A.T < cur.hi ? cur.t0 + A.T : cur.hi);
        wave_lds_sync();  // the previous tile is computed and stored
        if (tile) {
            pe_commit(cur.t0 * K1, t1 * K1, rp, sp, lane);
            if (A.q) pe_commit(cur.t0 * K2, t1 * K2, rq, sq, lane);
            if (cur.t0 == cur.lo && lane < C) sd[lane] = dreg;
        }
        wave_lds_sync();
        const PeCursor nxt = pe_next(A, cur, t1, items, waves, nullptr);
        if (nxt.it < items && nxt.t0 < nxt.hi) {
            const int64_t n1 = nxt.t0 + A.T < nxt.hi ? nxt.t0 + A.T : nxt.hi;
            pe_issue(A.p, nxt.t0 * K1, n1 * K1, A.n * K1, rp, lane);
            if (A.q) pe_issue(A.q, nxt.t0 * K2, n1 * K2, A.n * K2, rq, lane);
            if (nxt.t0 == nxt.lo && lane < C) dreg = dS[(A.seg ? nxt.it : 0) * C + lane];
        }
        if (tile) {
            const int64_t bp = cur.t0 * K1 - ((cur.t0 * K1) & ~(int64_t)3);
            const int64_t bq = cur.t0 * K2 - ((cur.t0 * K2) & ~(int64_t)3);
            const int rows = (int)(t1 - cur.t0);
            for (int i = lane; i < rows; i += kWave) {
                float* prow = sp + bp + i * K1;
                float* qrow = sq + bq + i * K2;
                float qv[KQ], aq[KQ];
#pragma unroll
                for (int b = 0; b < KQ; ++b) {
                    qv[b] = b < K2 ? (A.q ? qrow[b] : 1.0f) : 0.0f;
                    aq[b] = 0.0f;
                }
                for (int a = 0; a < K1; ++a) {
                    const float pa = prow[a];
                    float ap = 0.0f;
#pragma unroll
                    for (int b = 0; b < KQ; ++b) {
                        if (b < K2) {
                            const float d = sd[a * K2 + b];
                            ap += d * qv[b];
                            aq[b] += d * pa;
                        }
                    }
                    prow[a] = ap;  // dp over the row's own p, already read
                }
#pragma unroll
                for (int b = 0; b < KQ; ++b)
                    if (b < K2) qrow[b] = aq[b];
            }
            wave_lds_sync();
            if (dp) pe_store_tile(dp, cur.t0 * K1, t1 * K1, sp, lane);
            if (dq) pe_store_tile(dq, cur.t0 * K2, t1 * K2, sq, lane);
        }
        cur = nxt;
    }
}

// Rows per tile: 96 (a 9 x 9 grid image's 81 tiles in one pass) unless
// four waves' backward tiles would pass 32 KiB of LDS, then 64 or 32.
int pe_tile_rows(int K1, int K2) {
    for (int T = 96; T > 32; T -= 32)
        if ((size_t)kPeWaves * (pe_tile_floats(T, K1) + pe_tile_floats(T, K2) + kPeMaxCells) * sizeof(float) <=
            (size_t)kPeLdsBytes)
            return T;
    return 32;
}

size_t pe_fwd_lds(int T, int K1, int K2) {
    return (size_t)kPeWaves * (pe_tile_floats(T, K1) + pe_tile_floats(T, K2)) * sizeof(float);
}

size_t pe_bwd_lds(int T, int K1, int K2) {
    return (size_t)kPeWaves * (pe_tile_floats(T, K1) + pe_tile_floats(T, K2) + kPeMaxCells) * sizeof(float);
}

int pe_check(const int64_t* seg, int32_t G, const float* p, int32_t K1, const float* q, int32_t K2, int64_t n,
             const char* what) {
    if (n < 0 || (n > 0 && !p)) return fail(TDP_EINVAL, "%s: null p or n < 0", what);
    if (K1 < 1 || K1 > kPeMaxK || K2 < 1 || K2 > kPeMaxK || K1 * K2 > kPeMaxCells)
        return fail(TDP_EINVAL, "%s: K1=%d K2=%d (each 1..16, K1*K2 <= 64)", what, K1, K2);
    if (!q && K2 != 1) return fail(TDP_EINVAL, "%s: q == NULL requires K2 == 1", what);
    if (G < 1 || (!seg && G != 1)) return fail(TDP_EINVAL, "%s: G=%d (G must be 1 without segments)", what, G);
    if (!aligned16(p) || !aligned16(q)) return fail(TDP_EINVAL, "%s: p and q must be 16-byte aligned", what);
    const int T = pe_tile_rows(K1, K2);
    if (pe_tile_words(T, K1) > 7 * kWave || pe_tile_words(T, K2) > 7 * kWave)
        return fail(TDP_EINVAL, "%s: tile of %d rows exceeds the register words", what, T);
    return TDP_OK;
}

}  // namespace

}  // namespace tdp

using namespace tdp;

extern "C" size_t tdp_soft_workspace_size(void) {
    size_t b;
    soft_layout(nullptr, &b);
    return b;
}

extern "C" int tdp_soft_workspace_init(void* ws, size_t ws_bytes, hipStream_t stream) {
    int rc = check_ws(ws, ws_bytes, "tdp_soft_workspace_init");
    if (rc) return rc;
    soft_init_kernel<<<256, 256, 0, stream>>>(soft_layout(ws, nullptr));
    return launch_status("tdp_soft_workspace_init");
}

extern "C" int tdp_soft_filter(const float* x, int64_t n, const float* d_c, float tau, float* w, hipStream_t stream) {
    if (n < 0 || !d_c || (n > 0 && (!x || !w))) return fail(TDP_EINVAL, "tdp_soft_filter: null pointer or n < 0");
    if (!(tau > 0.0f)) return fail(TDP_EINVAL, "tdp_soft_filter: tau must be > 0");
    if (!aligned16(x) || !aligned16(w)) return fail(TDP_EINVAL, "tdp_soft_filter: x and w must be 16-byte aligned");
    if (n == 0) return TDP_OK;
    soft_filter_kernel<<<soft_grid(n, 16), kSoftThreads, 0, stream>>>(x, n, d_c, 1.0f / tau, w);
    return launch_status("tdp_soft_filter");
}

extern "C" int tdp_soft_filter_bwd(const float* x, int64_t n, const float* d_c, float tau, const float* dw, float* dx,
                                   float* d_dc, float* d_dtau, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n < 0 || !d_c || !d_dc || (n > 0 && (!x || !dw))) return fail(TDP_EINVAL, "tdp_soft_filter_bwd: null pointer");
    if (!(tau > 0.0f)) return fail(TDP_EINVAL, "tdp_soft_filter_bwd: tau must be > 0");
    int rc = check_ws(ws, ws_bytes, "tdp_soft_filter_bwd");
    if (rc) return rc;
    SoftWs s = soft_layout(ws, nullptr);
    const int grid = soft_grid(n, 16);
    soft_filter_bwd_kernel<<<grid, kSoftThreads, 0, stream>>>(x, n, d_c, 1.0f / tau, dw, dx, s, d_dc);
    soft_scalar_finish_kernel<<<1, kSoftThreads, 0, stream>>>(s, grid, d_dc, d_dtau);
    return launch_status("tdp_soft_filter_bwd");
}

extern "C" int tdp_soft_groupby(const int32_t* g, const float* w, const float* v, int64_t n, int32_t K, int32_t G,
                                float* S, int32_t* d_status, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n < 0 || !S || (n > 0 && (!g || !v))) return fail(TDP_EINVAL, "tdp_soft_groupby: null pointer or n < 0");
    if (K < 1 || K > 16 || G < 1 || G > 65536) return fail(TDP_EINVAL, "tdp_soft_groupby: K=%d G=%d out of range", K, G);
    int rc = check_ws(ws, ws_bytes, "tdp_soft_groupby");
    if (rc) return rc;
    SoftWs s = soft_layout(ws, nullptr);
    const int64_t GK = (int64_t)G * K;
    if (GK <= kMaxLdsFloats) {
        const int grid = (int)std::min<int64_t>(std::min(soft_grid(n, 16), 1024), kRowFloats / GK);
        soft_groupby_kernel<true><<<grid, kSoftThreads, GK * sizeof(float), stream>>>(g, w, v, n, K, G, s, S, d_status);
        launch_reduce(s, grid, GK, S, nullptr, nullptr, nullptr, d_status, stream);
    } else {
        soft_groupby_kernel<false><<<soft_grid(n, 16), kSoftThreads, 0, stream>>>(g, w, v, n, K, G, s, S, d_status);
        launch_reduce(s, 0, GK, S, nullptr, nullptr, nullptr, d_status, stream);
    }
    return launch_status("tdp_soft_groupby");
}

extern "C" int tdp_soft_groupby_bwd(const int32_t* g, const float* w, const float* v, const float* dS, int64_t n,
                                    int32_t K, int32_t G, float* dw, float* dv, hipStream_t stream) {
    if (n < 0 || (n > 0 && (!g || !v || !dS))) return fail(TDP_EINVAL, "tdp_soft_groupby_bwd: null pointer");
    if (K < 1 || K > 16 || G < 1 || G > 65536) return fail(TDP_EINVAL, "tdp_soft_groupby_bwd: K=%d G=%d", K, G);
    if (n == 0 || (!dw && !dv)) return TDP_OK;
    soft_groupby_bwd_kernel<<<soft_grid(n, 16), kSoftThreads, 0, stream>>>(g, w, v, dS, n, K, G, dw, dv);
    return launch_status("tdp_soft_groupby_bwd");
}

extern "C" int tdp_soft_filter_groupby(const float* x, const float* v, const int32_t* g, int64_t n, const float* d_c,
                                       float tau, int32_t G, float* S, const float* T, float* d_loss, float* dS,
                                       int32_t* d_status, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n < 0 || !d_c || !S || (n > 0 && (!x || !v || !g)))
        return fail(TDP_EINVAL, "tdp_soft_filter_groupby: null pointer or n < 0");
    if (!(tau > 0.0f)) return fail(TDP_EINVAL, "tdp_soft_filter_groupby: tau must be > 0");
    if (G < 1 || G > 65536) return fail(TDP_EINVAL, "tdp_soft_filter_groupby: G=%d", G);
    if (T && (!d_loss || !dS)) return fail(TDP_EINVAL, "tdp_soft_filter_groupby: T given without d_loss/dS");
    if (!aligned16(x) || !aligned16(v) || !aligned16(g))
        return fail(TDP_EINVAL, "tdp_soft_filter_groupby: x, v, g must be 16-byte aligned");
    int rc = check_ws(ws, ws_bytes, "tdp_soft_filter_groupby");
    if (rc) return rc;
    SoftWs s = soft_layout(ws, nullptr);
    if (G <= kMaxLdsFloats) {
        const int64_t wgs = ceil_div(std::max<int64_t>(n, 1), (int64_t)kFwdThreads * 16);
        const int grid = (int)std::min<int64_t>(std::min<int64_t>(wgs, 256), kRowFloats / G);
        const int copies = table_copies(G);
        soft_fg_fwd_kernel<true><<<grid, kFwdThreads, (size_t)copies * G * sizeof(float), stream>>>(
            x, v, g, n, d_c, 1.0f / tau, G, copies, s, S, T, d_loss, dS, d_status);
        launch_reduce(s, grid, G, S, T, d_loss, dS, d_status, stream);
    } else {
        soft_fg_fwd_kernel<false><<<(soft_grid(n, 16) + 3) / 4, kFwdThreads, 0, stream>>>(x, v, g, n, d_c, 1.0f / tau, G, 1, s, S,
                                                                                 T, d_loss, dS, d_status);
        launch_reduce(s, 0, G, S, T, d_loss, dS, d_status, stream);
    }
    return launch_status("tdp_soft_filter_groupby");
}

extern "C" int tdp_soft_filter_groupby_bwd(const float* x, const float* v, const int32_t* g, int64_t n,
                                           const float* d_c, float tau, int32_t G, const float* dS, float* dv,
                                           float* dx, float* d_dc, float* d_dtau, void* ws, size_t ws_bytes,
                                           hipStream_t stream) {
    if (n < 0 || !d_c || !dS || !d_dc || (n > 0 && (!x || !v || !g || !dv)))
        return fail(TDP_EINVAL, "tdp_soft_filter_groupby_bwd: null pointer or n < 0");
    if (!(tau > 0.0f)) return fail(TDP_EINVAL, "tdp_soft_filter_groupby_bwd: tau must be > 0");
    if (G < 1 || G > 65536) return fail(TDP_EINVAL, "tdp_soft_filter_groupby_bwd: G=%d", G);
    if (!aligned16(x) || !aligned16(v) || !aligned16(g) || !aligned16(dv) || (dx && !aligned16(dx)))
        return fail(TDP_EINVAL, "tdp_soft_filter_groupby_bwd: arrays must be 16-byte aligned");
    int rc = check_ws(ws, ws_bytes, "tdp_soft_filter_groupby_bwd");
    if (rc) return rc;
    SoftWs s = soft_layout(ws, nullptr);
    const int grid = soft_grid(n, 16);
    if (G <= kMaxLdsFloats)
        soft_fg_bwd_kernel<true><<<grid, kSoftThreads, G * sizeof(float), stream>>>(x, v, g, n, d_c, 1.0f / tau, G, dS,
                                                                                   dv, dx, s, d_dc);
    else
        soft_fg_bwd_kernel<false><<<grid, kSoftThreads, 0, stream>>>(x, v, g, n, d_c, 1.0f / tau, G, dS, dv, dx, s,
                                                                     d_dc);
    soft_scalar_finish_kernel<<<1, kSoftThreads, 0, stream>>>(s, grid, d_dc, d_dtau);
    return launch_status("tdp_soft_filter_groupby_bwd");
}

extern "C" int tdp_soft_pe_groupby(const int64_t* seg, int32_t G, const float* p, int32_t K1, const float* q,
                                   int32_t K2, int64_t n, float* S, int32_t* d_status, void* ws, size_t ws_bytes,
                                   hipStream_t stream) {
    int rc = pe_check(seg, G, p, K1, q, K2, n, "tdp_soft_pe_groupby");
    if (rc) return rc;
    if (!S) return fail(TDP_EINVAL, "tdp_soft_pe_groupby: null S");
    rc = check_ws(ws, ws_bytes, "tdp_soft_pe_groupby");
    if (rc) return rc;
    SoftWs s = soft_layout(ws, nullptr);
    const int T = pe_tile_rows(K1, K2);
    const PeArgs A{seg, G, p, q, K1, K2, n, T};
    const size_t lds = pe_fwd_lds(T, K1, K2);
    // register words of a tile: 4 x 64 of p and 1 x 64 of q cover 96 rows of
    // 10 digit and 2 size probabilities; 7 x 64 cover any K up to 16
    const bool small = pe_tile_words(T, K1) <= 4 * kWave && pe_tile_words(T, K2) <= kWave && K2 <= 2;
    auto fwd = [&](int grid) {
        if (small)
            pe_fwd_kernel<4, 1><<<grid, kSoftThreads, lds, stream>>>(A, s, S);
        else
            pe_fwd_kernel<7, 7><<<grid, kSoftThreads, lds, stream>>>(A, s, S);
    };
    if (seg) {
        const int grid = (int)std::min<int64_t>(ceil_div((int64_t)G, (int64_t)kPeWaves), 4096);
        fwd(grid);
        // no cross-workgroup sums: the finishing kernel only reports and clears the flags
        soft_groups_finish_kernel<<<1, kFinishThreads, 0, stream>>>(s, 0, nullptr, nullptr, nullptr, nullptr, d_status);
    } else {
        const int grid = (int)std::min<int64_t>(std::max<int64_t>(ceil_div(n, (int64_t)kSoftThreads * 16), 1), 1024);
        fwd(grid);
        launch_reduce(s, grid, (int64_t)K1 * K2, S, nullptr, nullptr, nullptr, d_status, stream);
    }
    return launch_status("tdp_soft_pe_groupby");
}

extern "C" int tdp_soft_pe_groupby_bwd(const int64_t* seg, int32_t G, const float* p, int32_t K1, const float* q,
                                       int32_t K2, int64_t n, const float* dS, float* dp, float* dq,
                                       hipStream_t stream) {
    int rc = pe_check(seg, G, p, K1, q, K2, n, "tdp_soft_pe_groupby_bwd");
    if (rc) return rc;
    if (!dS) return fail(TDP_EINVAL, "tdp_soft_pe_groupby_bwd: null dS");
    if (dq && !q) return fail(TDP_EINVAL, "tdp_soft_pe_groupby_bwd: dq requires q");
    if (!aligned16(dp) || !aligned16(dq)) return fail(TDP_EINVAL, "tdp_soft_pe_groupby_bwd: dp and dq must be 16-byte aligned");
    if (n == 0 || (!dp && !dq)) return TDP_OK;
    const int T = pe_tile_rows(K1, K2);
    const PeArgs A{seg, G, p, q, K1, K2, n, T};
    const int64_t want = seg ? ceil_div((int64_t)G, (int64_t)kPeWaves) : ceil_div(n, (int64_t)kSoftThreads * 16);
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(want, 1), seg ? 4096 : 2048);
    const bool small = pe_tile_words(T, K1) <= 4 * kWave && pe_tile_words(T, K2) <= kWave && K2 <= 2;
    if (small)
        pe_bwd_kernel<4, 1, 2><<<grid, kSoftThreads, pe_bwd_lds(T, K1, K2), stream>>>(A, dS, dp, dq);
    else
        pe_bwd_kernel<7, 7, kPeMaxK><<<grid, kSoftThreads, pe_bwd_lds(T, K1, K2), stream>>>(A, dS, dp, dq);
    return launch_status("tdp_soft_pe_groupby_bwd");
}

namespace {

bool sq_dtype(int dt) { return dt == TDP_I8 || dt == TDP_I32 || dt == TDP_I64 || dt == TDP_F32; }

// Checks a groupby descriptor for its relaxed run and fills the device view.
int sq_prepare(const tdp_groupby_desc* d, const float* d_c, const float* d_tau, const char* fn, SqDev& q) {
    if (!d) return fail(TDP_EINVAL, "%s: null descriptor", fn);
    if (d->n_rows < 0 || d->n_rows > INT32_MAX) return fail(TDP_EINVAL, "%s: n_rows %lld", fn, (long long)d->n_rows);
    if (d->join || d->sel || d->topk)
        return fail(TDP_EUNSUPPORTED, "%s: joins, selection vectors and top-k have no relaxed form here", fn);
    if (d->expr != TDP_EXPR_COL && d->expr != TDP_EXPR_NONE)
        return fail(TDP_EUNSUPPORTED, "%s: only SUM(a) and COUNT(*) are relaxed", fn);
    if (d->n_keys < 1 || d->n_keys > 2) return fail(TDP_EINVAL, "%s: n_keys %d", fn, d->n_keys);
    if (d->n_more_preds < 0 || d->n_more_preds > TDP_MAX_MORE_PREDS || (d->n_more_preds > 0 && !d->more_preds))
        return fail(TDP_EINVAL, "%s: more_preds", fn);
    q = SqDev{};
    q.n = d->n_rows;
    auto col_ok = [&](const tdp_col& c, bool allow_f32, const char* what) -> int {
        if (!(allow_f32 ? sq_dtype(c.dtype) : int_dtype(c.dtype)))
            return fail(TDP_EUNSUPPORTED, "%s: %s dtype %d", fn, what, c.dtype);
        if (c.side != TDP_SIDE_PROBE) return fail(TDP_EINVAL, "%s: %s must be on the probe side", fn, what);
        if (c.n < d->n_rows) return fail(TDP_EINVAL, "%s: %s shorter than n_rows", fn, what);
        if (d->n_rows > 0 && !c.data) return fail(TDP_EINVAL, "%s: %s data is null", fn, what);
        if ((uintptr_t)c.data & 15) return fail(TDP_EINVAL, "%s: %s is not 16-byte aligned", fn, what);
        return TDP_OK;
    };
    int rc;
    const tdp_col* pc[kSqMaxPreds];
    int cmp[kSqMaxPreds];
    int J = 0;
    if (d->has_pred) {
        pc[J] = &d->pred;
        cmp[J++] = d->pred_cmp;
    }
    for (int i = 0; i < d->n_more_preds; ++i) {
        pc[J] = &d->more_preds[i].col;
        cmp[J++] = d->more_preds[i].cmp;
    }
    if (J > 0 && (!d_c || !d_tau)) return fail(TDP_EINVAL, "%s: thresholds and temperatures are required", fn);
    for (int j = 0; j < J; ++j) {
        if ((rc = col_ok(*pc[j], true, "predicate column"))) return rc;
        if (cmp[j] != TDP_LT && cmp[j] != TDP_LE && cmp[j] != TDP_GT && cmp[j] != TDP_GE)
            return fail(TDP_EUNSUPPORTED, "%s: comparison %d has no logistic relaxation", fn, cmp[j]);
        q.pr[j].p = pc[j]->data;
        q.pr[j].dt = pc[j]->dtype;
        q.pr[j].s = (cmp[j] == TDP_LT || cmp[j] == TDP_LE) ? 1.0f : -1.0f;
    }
    q.J = J;
    q.c = d_c;
    q.tau = d_tau;
    int64_t G = 1;
    q.n_keys = d->n_keys;
    for (int i = 0; i < d->n_keys; ++i) {
        if ((rc = col_ok(d->key[i], false, "group key"))) return rc;
        if (d->key_card[i] < 1) return fail(TDP_EINVAL, "%s: key_card[%d] < 1", fn, i);
        G *= d->key_card[i];
        if (G > 65536) return fail(TDP_EUNSUPPORTED, "%s: more than 65536 groups", fn);
        q.kp[i] = d->key[i].data;
        q.kdt[i] = d->key[i].dtype;
        q.lo[i] = d->key_lo[i];
        q.card[i] = d->key_card[i];
    }
    q.G = (int)G;
    if (d->expr == TDP_EXPR_COL) {
        if ((rc = col_ok(d->a, true, "value column"))) return rc;
        q.a = d->a.data;
        q.adt = d->a.dtype;
    }
    return TDP_OK;
}

}  // namespace

extern "C" int tdp_soft_query(const tdp_groupby_desc* d, const float* d_c, const float* d_tau, float* S, const float* T,
                              float* d_loss, float* dS, int32_t* d_status, void* ws, size_t ws_bytes,
                              hipStream_t stream) {
    SqDev q;
    int rc = sq_prepare(d, d_c, d_tau, "tdp_soft_query", q);
    if (rc) return rc;
    if (!S) return fail(TDP_EINVAL, "tdp_soft_query: null S");
    if (T && (!d_loss || !dS)) return fail(TDP_EINVAL, "tdp_soft_query: T given without d_loss/dS");
    if ((rc = check_ws(ws, ws_bytes, "tdp_soft_query"))) return rc;
    SoftWs s = soft_layout(ws, nullptr);
    if (q.G <= kMaxLdsFloats) {
        const int64_t wgs = ceil_div(std::max<int64_t>(q.n, 1), (int64_t)kFwdThreads * 16);
        const int grid = (int)std::min<int64_t>(std::min<int64_t>(wgs, 256), kRowFloats / q.G);
        const int copies = table_copies(q.G);
        soft_query_fwd_kernel<true><<<grid, kFwdThreads, (size_t)copies * q.G * sizeof(float), stream>>>(q, copies, s);
        launch_reduce(s, grid, q.G, S, T, d_loss, dS, d_status, stream);
    } else {
        soft_query_fwd_kernel<false><<<(soft_grid(q.n, 16) + 3) / 4, kFwdThreads, 0, stream>>>(q, 1, s);
        launch_reduce(s, 0, q.G, S, T, d_loss, dS, d_status, stream);
    }
    return launch_status("tdp_soft_query");
}

extern "C" int tdp_soft_query_bwd(const tdp_groupby_desc* d, const float* d_c, const float* d_tau, const float* dS,
                                  float* d_dc, float* d_dtau, float* de, void* ws, size_t ws_bytes,
                                  hipStream_t stream) {
    SqDev q;
    int rc = sq_prepare(d, d_c, d_tau, "tdp_soft_query_bwd", q);
    if (rc) return rc;
    if (!dS || (q.J > 0 && !d_dc)) return fail(TDP_EINVAL, "tdp_soft_query_bwd: null dS or d_dc");
    if (de && !aligned16(de)) return fail(TDP_EINVAL, "tdp_soft_query_bwd: de must be 16-byte aligned");
    if ((rc = check_ws(ws, ws_bytes, "tdp_soft_query_bwd"))) return rc;
    SoftWs s = soft_layout(ws, nullptr);
    const int grid = soft_grid(q.n, 16);
    if (q.G <= kMaxLdsFloats)
        soft_query_bwd_kernel<true><<<grid, kSoftThreads, q.G * sizeof(float), stream>>>(q, dS, de, s);
    else
        soft_query_bwd_kernel<false><<<grid, kSoftThreads, 0, stream>>>(q, dS, de, s);
    if (q.J > 0) soft_query_finish_kernel<<<1, kSoftThreads, 0, stream>>>(s, grid, q.J, d_dc, d_dtau);
    return launch_status("tdp_soft_query_bwd");
}

extern "C" int tdp_mse_loss(const float* S, const float* T, int32_t G, float* d_loss, float* dS, hipStream_t stream) {
    if (!S || !T || !d_loss || G < 1) return fail(TDP_EINVAL, "tdp_mse_loss: null pointer or G < 1");
    mse_kernel<<<1, kFinishThreads, 0, stream>>>(S, T, G, d_loss, dS);
    return launch_status("tdp_mse_loss");
}
