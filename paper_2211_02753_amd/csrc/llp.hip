// Learning from label proportions with a linear classifier (the LLP and
// Label-DP use cases): the classifier labels every row of a bag, a grouped
// soft COUNT per (bag, class) of its softmax is the relaxed query answer,
// and the backward returns the classifier's weight and bias gradients.
//
// Forward: bags are consecutive runs of `bag` rows (a power of two).  For
// bag <= 64 a wave takes 64 consecutive rows, one per lane, and adds each
// bag's probabilities with a butterfly over the bag's aligned group of
// lanes; for larger bags a wave takes whole bags, lanes striding over the
// rows, then a butterfly over the wave.  Each bag's sum is formed inside one
// wave in a fixed order (float64), so results do not depend on scheduling.
// Backward: every thread recomputes its rows' probabilities, keeps the
// gradient terms in registers, the workgroup reduces them in float64 into
// one partial row, and a one-workgroup kernel adds the rows in a fixed order.
#include "common.hpp"

namespace tdp {

namespace {

constexpr int kLlpMaxF = 16;
constexpr int kLlpMaxC = 4;
constexpr int kLlpThreads = 256;
constexpr int kLlpMaxGrid = 1024;
constexpr int kLlpFinThreads = 1024;  // threads of the one-workgroup finishing kernels

struct LlpArgs {
    const float* X;
    int64_t n;
    int F;
    const float* W;  // [C][F]
    const float* b;  // [C]
    int64_t bag;
};

// Class probabilities of one row: softmax of W x + b, float32.
template <int C>
__device__ __forceinline__ void llp_probs(const float* s_w, const float* s_b, const float x[kLlpMaxF], int F,
                                          float p[C]) {
    float z[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float a = s_b[c];
#pragma unroll
        for (int f = 0; f < kLlpMaxF; ++f)
            if (f < F) a = fmaf(s_w[c * kLlpMaxF + f], x[f], a);
        z[c] = a;
    }
    float m = z[0];
#pragma unroll
    for (int c = 1; c < C; ++c) m = fmaxf(m, z[c]);
    float sum = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        z[c] = __expf(z[c] - m);
        sum += z[c];
    }
    const float inv = 1.0f / sum;
#pragma unroll
    for (int c = 0; c < C; ++c) p[c] = z[c] * inv;
}

__device__ __forceinline__ void llp_load_row(const LlpArgs& a, int64_t row, float x[kLlpMaxF]) {
#pragma unroll
    for (int f = 0; f < kLlpMaxF; ++f) x[f] = 0.0f;
    if (row >= a.n) return;
    const float* src = a.X + row * a.F;
    if ((a.F & 3) == 0) {
#pragma unroll
        for (int f = 0; f < kLlpMaxF; f += 4) {
            if (f < a.F) {
                const float4 q = *(const float4*)(src + f);
                x[f] = q.x; x[f + 1] = q.y; x[f + 2] = q.z; x[f + 3] = q.w;
            }
        }
    } else {
#pragma unroll
        for (int f = 0; f < kLlpMaxF; ++f)
            if (f < a.F) x[f] = src[f];
    }
}

__device__ __forceinline__ void llp_stage_params(const LlpArgs& a, int C, float* s_w, float* s_b) {
    for (int i = threadIdx.x; i < C * kLlpMaxF; i += blockDim.x) {
        const int c = i / kLlpMaxF, f = i % kLlpMaxF;
        s_w[i] = f < a.F ? a.W[c * a.F + f] : 0.0f;
    }
    for (int c = threadIdx.x; c < C; c += blockDim.x) s_b[c] = a.b[c];
    __syncthreads();
}

// Squared error of one bag's counts against T, its gradient written to dS
// (float64 arithmetic, as the oracle's mean squared error).
template <int C>
__device__ __forceinline__ double llp_bag_loss(int64_t j, const double acc[C], float* S, const float* T, float* dS,
                                               double inv_cells) {
    double l = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const float sv = (float)acc[c];
        S[j * C + c] = sv;
        if (T) {
            const double d = (double)sv - (double)T[j * C + c];
            l += d * d;
            dS[j * C + c] = (float)(2.0 * d * inv_cells);
        }
    }
    return l;
}

template <int C>
__global__ __launch_bounds__(kLlpThreads) void llp_fwd_kernel(LlpArgs a, float* S, const float* T, float* dS,
                                                              double* loss_part) {
    __shared__ float s_w[kLlpMaxC * kLlpMaxF], s_b[kLlpMaxC];
    __shared__ double s_l[kLlpThreads / kWave];
    llp_stage_params(a, C, s_w, s_b);
    double lsum = 0.0;  // this lane's squared errors (lanes that write bags)
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * kLlpThreads + threadIdx.x) / kWave;
    const int64_t n_waves = (int64_t)gridDim.x * kLlpThreads / kWave;
    const int64_t n_bags = (a.n + a.bag - 1) / a.bag;
    const double inv_cells = 1.0 / (double)(n_bags * C);
    if (a.bag <= kWave) {
        const int64_t units = (a.n + kWave - 1) / kWave;
        for (int64_t u = wave; u < units; u += n_waves) {
            const int64_t row = u * kWave + lane;
            float x[kLlpMaxF], p[C];
            llp_load_row(a, row, x);
            llp_probs<C>(s_w, s_b, x, a.F, p);
            double acc[C];
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] = row < a.n ? (double)p[c] : 0.0;
            for (int off = 1; off < a.bag; off <<= 1) {
#pragma unroll
                for (int c = 0; c < C; ++c) acc[c] += __shfl_xor(acc[c], off, kWave);
            }
            if ((lane & (a.bag - 1)) == 0 && row < a.n) lsum += llp_bag_loss<C>(row / a.bag, acc, S, T, dS, inv_cells);
        }
    } else {
        for (int64_t j = wave; j < n_bags; j += n_waves) {
            const int64_t r0 = j * a.bag, r1 = r0 + a.bag < a.n ? r0 + a.bag : a.n;
            double acc[C];
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] = 0.0;
            for (int64_t row = r0 + lane; row < r1; row += kWave) {
                float x[kLlpMaxF], p[C];
                llp_load_row(a, row, x);
                llp_probs<C>(s_w, s_b, x, a.F, p);
#pragma unroll
                for (int c = 0; c < C; ++c) acc[c] += (double)p[c];
            }
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
#pragma unroll
                for (int c = 0; c < C; ++c) acc[c] += __shfl_xor(acc[c], off, kWave);
            }
            if (lane == 0) lsum += llp_bag_loss<C>(j, acc, S, T, dS, inv_cells);
        }
    }
    if (T) {  // the workgroup's squared errors, in a fixed order
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, kWave);
        if (lane == 0) s_l[threadIdx.x / kWave] = lsum;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < kLlpThreads / kWave; ++w) t += s_l[w];
            loss_part[blockIdx.x] = t;
        }
    }
}

// One workgroup: the loss, the partials added in workgroup order.
__global__ __launch_bounds__(kLlpFinThreads) void llp_loss_finish_kernel(const double* part, int n_parts,
                                                                         double inv_cells, float* d_loss) {
    constexpr int kW = kLlpFinThreads / kWave;
    __shared__ double s_w[kW];
    double t = 0.0;
    for (int b = threadIdx.x; b < n_parts; b += kLlpFinThreads) t += part[b];  // each thread's strided share, in order
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, kWave);
    if (lane_id() == 0) s_w[threadIdx.x / kWave] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < kW; ++w) tot += s_w[w];
        *d_loss = (float)(tot * inv_cells);
    }
}

// Per-thread gradient terms over a grid-stride of rows, reduced to one
// float64 partial row per workgroup: [C][kLlpMaxF] weights then [C] biases.
template <int C>
__global__ __launch_bounds__(kLlpThreads) void llp_bwd_kernel(LlpArgs a, const float* __restrict__ dS, double* part) {
    __shared__ float s_w[kLlpMaxC * kLlpMaxF], s_b[kLlpMaxC];
    __shared__ double s_red[kLlpThreads / kWave];
    llp_stage_params(a, C, s_w, s_b);
    float gw[C][kLlpMaxF], gb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        gb[c] = 0.0f;
#pragma unroll
        for (int f = 0; f < kLlpMaxF; ++f) gw[c][f] = 0.0f;
    }
    const int64_t stride = (int64_t)gridDim.x * kLlpThreads;
    for (int64_t row = (int64_t)blockIdx.x * kLlpThreads + threadIdx.x; row < a.n; row += stride) {
        float x[kLlpMaxF], p[C], dp[C];
        llp_load_row(a, row, x);
        llp_probs<C>(s_w, s_b, x, a.F, p);
        const float* d = dS + (row / a.bag) * C;
        float s = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            dp[c] = d[c];
            s = fmaf(p[c], dp[c], s);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float dz = p[c] * (dp[c] - s);
            gb[c] += dz;
#pragma unroll
            for (int f = 0; f < kLlpMaxF; ++f) gw[c][f] = fmaf(dz, x[f], gw[c][f]);
        }
    }
    // workgroup sums in float64, written as this workgroup's partial row
    const int lane = lane_id(), wv = threadIdx.x / kWave;
    double* row = part + (int64_t)blockIdx.x * C * (kLlpMaxF + 1);
    for (int k = 0; k < C * (kLlpMaxF + 1); ++k) {
        const int c = k / (kLlpMaxF + 1), f = k % (kLlpMaxF + 1);
        float v = 0.0f;
#pragma unroll
        for (int cc = 0; cc < C; ++cc)
#pragma unroll
            for (int ff = 0; ff <= kLlpMaxF; ++ff)
                if (cc == c && ff == f) v = ff < kLlpMaxF ? gw[cc][ff] : gb[cc];
        double t = (double)v;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, kWave);
        if (lane == 0) s_red[wv] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            double tot = 0.0;
            for (int w = 0; w < kLlpThreads / kWave; ++w) tot += s_red[w];
            row[k] = tot;
        }
        __syncthreads();
    }
}

// One workgroup: the partial rows added in a fixed order, to float32.
// Thread (slice s, column k) adds rows s, s + slices, ... (16 loads in
// flight), then the slices are added in order: one thread per column walking
// every row one dependent load at a time took 245 us for 1024 rows.

__global__ __launch_bounds__(kLlpFinThreads) void llp_bwd_finish_kernel(const double* part, int n_parts, int C, int F,
                                                                        float* dW, float* db) {
    __shared__ double s_acc[kLlpFinThreads];
    const int cols = C * (kLlpMaxF + 1);  // <= 68
    const int slices = kLlpFinThreads / cols;
    const int k = threadIdx.x % cols, sl = threadIdx.x / cols;
    double t = 0.0;
    if (sl < slices) {
        for (int b0 = sl; b0 < n_parts; b0 += 16 * slices) {
            double v[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int b = b0 + q * slices;
                v[q] = b < n_parts ? part[(int64_t)b * cols + k] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) t += v[q];
        }
    }
    s_acc[threadIdx.x] = t;
    __syncthreads();
    if (threadIdx.x < cols) {
        double tot = 0.0;
        for (int q = 0; q < slices; ++q) tot += s_acc[q * cols + threadIdx.x];
        const int c = threadIdx.x / (kLlpMaxF + 1), f = threadIdx.x % (kLlpMaxF + 1);
        if (f < F) dW[c * F + f] = (float)tot;
        else if (f == kLlpMaxF) db[c] = (float)tot;
    }
}

// Argmax of the logits, accumulated in float64 as b, then one fused
// multiply-add per feature in feature order; ties to the smallest class.
__global__ void llp_predict_kernel(LlpArgs a, int C, int8_t* out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < a.n; row += stride) {
        int best = 0;
        double bz = 0.0;
        for (int c = 0; c < C; ++c) {
            double z = (double)a.b[c];
            for (int f = 0; f < a.F; ++f) z = fma((double)a.W[c * a.F + f], (double)a.X[row * a.F + f], z);
            if (c == 0 || z > bz) {
                best = c;
                bz = z;
            }
        }
        out[row] = (int8_t)best;
    }
}

__global__ void count_fill_kernel(float* out, int64_t cells, const float* noise) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < cells; j += stride)
        out[j] = noise ? noise[j] : 0.0f;
}

__global__ void count_place_kernel(const int64_t* k0, const int64_t* k1, const int64_t* count,
                                   const int64_t* d_n_groups, int64_t lo0, int64_t card0, int64_t lo1, int64_t card1,
                                   const float* noise, float* out, int32_t* status) {
    const int64_t m = *d_n_groups;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const int64_t u0 = k0[i] - lo0, u1 = k1 ? k1[i] - lo1 : 0;
        if (u0 < 0 || u0 >= card0 || u1 < 0 || u1 >= card1) {
            raise_flag(status, TDP_FLAG_KEY_DOMAIN);
            continue;
        }
        const int64_t j = u0 * card1 + u1;
        out[j] = (float)count[i] + (noise ? noise[j] : 0.0f);
    }
}

int llp_check(const LlpArgs& a, int C, const char* fn) {
    if (a.n < 0 || (a.n > 0 && (!a.X || !a.W || !a.b))) return fail(TDP_EINVAL, "%s: null pointer or n < 0", fn);
    if (a.F < 1 || a.F > kLlpMaxF) return fail(TDP_EINVAL, "%s: F=%d outside 1..%d", fn, a.F, kLlpMaxF);
    if (C < 2 || C > kLlpMaxC) return fail(TDP_EINVAL, "%s: C=%d outside 2..%d", fn, C, kLlpMaxC);
    if (a.bag < 1 || a.bag > (1 << 20) || (a.bag & (a.bag - 1)))
        return fail(TDP_EINVAL, "%s: bag=%lld is not a power of two in 1..2^20", fn, (long long)a.bag);
    if ((uintptr_t)a.X & 15) return fail(TDP_EINVAL, "%s: X must be 16-byte aligned", fn);
    return TDP_OK;
}

int llp_grid(int64_t n) {
    return (int)std::min<int64_t>(std::max<int64_t>(ceil_div(n, (int64_t)kLlpThreads * 16), 1), kLlpMaxGrid);
}

}  // namespace

}  // namespace tdp

using namespace tdp;

namespace {
constexpr int kLlpFwdMaxGrid = 4096;
}

extern "C" size_t tdp_llp_workspace_size(int32_t C) {
    WsAlloc wa(nullptr);
    wa.take<double>((size_t)kLlpMaxGrid * std::max(C, 1) * (kLlpMaxF + 1));
    wa.take<double>(kLlpFwdMaxGrid);
    return wa.bytes();
}

extern "C" int tdp_llp_bag_count(const float* X, int64_t n, int32_t F, const float* W, const float* b, int32_t C,
                                 int64_t bag, float* S, const float* T, float* d_loss, float* dS, void* ws,
                                 size_t ws_bytes, hipStream_t stream) {
    LlpArgs a{X, n, F, W, b, bag};
    int rc = llp_check(a, C, "tdp_llp_bag_count");
    if (rc) return rc;
    if (n > 0 && !S) return fail(TDP_EINVAL, "tdp_llp_bag_count: null S");
    if (T && (!d_loss || !dS)) return fail(TDP_EINVAL, "tdp_llp_bag_count: T given without d_loss and dS");
    if (T && (!ws || ws_bytes < tdp_llp_workspace_size(C)))
        return fail_need(TDP_EWORKSPACE, (int64_t)tdp_llp_workspace_size(C), "tdp_llp_bag_count: workspace %zu < %zu",
                         ws_bytes, tdp_llp_workspace_size(C));
    if (n == 0) return TDP_OK;
    WsAlloc wa(ws);
    wa.take<double>((size_t)kLlpMaxGrid * std::max(C, 1) * (kLlpMaxF + 1));
    double* lp = T ? wa.take<double>(kLlpFwdMaxGrid) : nullptr;
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(ceil_div(n, (int64_t)kLlpThreads * 8), 1), kLlpFwdMaxGrid);
    switch (C) {
        case 2: llp_fwd_kernel<2><<<grid, kLlpThreads, 0, stream>>>(a, S, T, dS, lp); break;
        case 3: llp_fwd_kernel<3><<<grid, kLlpThreads, 0, stream>>>(a, S, T, dS, lp); break;
        default: llp_fwd_kernel<4><<<grid, kLlpThreads, 0, stream>>>(a, S, T, dS, lp); break;
    }
    if (T) {
        const int64_t n_bags = (n + bag - 1) / bag;
        llp_loss_finish_kernel<<<1, kLlpFinThreads, 0, stream>>>(lp, grid, 1.0 / (double)(n_bags * C), d_loss);
    }
    return launch_status("tdp_llp_bag_count");
}

extern "C" int tdp_llp_bag_count_bwd(const float* X, int64_t n, int32_t F, const float* W, const float* b, int32_t C,
                                     int64_t bag, const float* dS, float* dW, float* db, void* ws, size_t ws_bytes,
                                     hipStream_t stream) {
    LlpArgs a{X, n, F, W, b, bag};
    int rc = llp_check(a, C, "tdp_llp_bag_count_bwd");
    if (rc) return rc;
    if (!dW || !db || (n > 0 && !dS)) return fail(TDP_EINVAL, "tdp_llp_bag_count_bwd: null dS, dW or db");
    if (!ws || ws_bytes < tdp_llp_workspace_size(C))
        return fail_need(TDP_EWORKSPACE, (int64_t)tdp_llp_workspace_size(C), "tdp_llp_bag_count_bwd: workspace %zu < %zu",
                         ws_bytes, tdp_llp_workspace_size(C));
    double* part = (double*)ws;
    const int grid = llp_grid(n);
    switch (C) {
        case 2: llp_bwd_kernel<2><<<grid, kLlpThreads, 0, stream>>>(a, dS, part); break;
        case 3: llp_bwd_kernel<3><<<grid, kLlpThreads, 0, stream>>>(a, dS, part); break;
        default: llp_bwd_kernel<4><<<grid, kLlpThreads, 0, stream>>>(a, dS, part); break;
    }
    llp_bwd_finish_kernel<<<1, kLlpFinThreads, 0, stream>>>(part, grid, C, F, dW, db);
    return launch_status("tdp_llp_bag_count_bwd");
}

extern "C" int tdp_llp_predict(const float* X, int64_t n, int32_t F, const float* W, const float* b, int32_t C,
                               int8_t* out, hipStream_t stream) {
    LlpArgs a{X, n, F, W, b, 1};
    int rc = llp_check(a, C, "tdp_llp_predict");
    if (rc) return rc;
    if (n > 0 && !out) return fail(TDP_EINVAL, "tdp_llp_predict: null out");
    if (n == 0) return TDP_OK;
    llp_predict_kernel<<<(int)std::min<int64_t>(ceil_div(n, 256), 4096), 256, 0, stream>>>(a, C, out);
    return launch_status("tdp_llp_predict");
}

extern "C" int tdp_count_table(const int64_t* key0, const int64_t* key1, const int64_t* count,
                               const int64_t* d_n_groups, int64_t lo0, int64_t card0, int64_t lo1, int64_t card1,
                               const float* noise, float* out, int32_t* d_status, hipStream_t stream) {
    if (!key0 || !count || !d_n_groups || !out) return fail(TDP_EINVAL, "tdp_count_table: null pointer");
    if (card0 < 1 || card1 < 1 || card0 > (1ll << 31) / card1)
        return fail(TDP_EINVAL, "tdp_count_table: table of %lld x %lld cells", (long long)card0, (long long)card1);
    if (!key1 && card1 != 1) return fail(TDP_EINVAL, "tdp_count_table: key1 == NULL requires card1 == 1");
    const int64_t cells = card0 * card1;
    count_fill_kernel<<<(int)std::min<int64_t>(ceil_div(cells, 256), 4096), 256, 0, stream>>>(out, cells, noise);
    count_place_kernel<<<(int)std::min<int64_t>(ceil_div(cells, 256), 4096), 256, 0, stream>>>(
        key0, key1, count, d_n_groups, lo0, card0, lo1, card1, noise, out, d_status);
    return launch_status("tdp_count_table");
}

namespace {
__global__ void segment_ids_kernel(int64_t n, int64_t width, int32_t* out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = (int32_t)(i / width);
}
}  // namespace

extern "C" int tdp_segment_ids(int64_t n, int64_t width, int32_t* out, hipStream_t stream) {
    if (n < 0 || width < 1 || (n > 0 && !out)) return fail(TDP_EINVAL, "tdp_segment_ids: n=%lld width=%lld", (long long)n, (long long)width);
    if ((n - 1) / width > INT32_MAX) return fail(TDP_EINVAL, "tdp_segment_ids: more than 2^31 segments");
    if (n == 0) return TDP_OK;
    segment_ids_kernel<<<(int)std::min<int64_t>(ceil_div(n, 256), 4096), 256, 0, stream>>>(n, width, out);
    return launch_status("tdp_segment_ids");
}
