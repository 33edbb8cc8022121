// The image classifier that stands in for a missing label column: bf16
// convolution / fully connected layers on MFMA with float32 accumulation,
// their input and weight gradients, 2x2 max pooling, the softmax
// expectation head, argmax and Adam.
//
// The general contraction is one tiled MFMA kernel (64x64 output tile, K
// step 64, four waves each owning a 32x32 quarter as 2x2 blocks of the
// 16x16x32 bf16 instruction).  What differs between forward, input-gradient
// and weight-gradient passes of a layer is only how a tile of A or B is
// gathered from memory (an implicit im2col for the convolutions; a load in
// natural layout transposed through LDS where the reduction index is the
// slow dimension) and what the epilogue does (bias + ReLU and a bf16 store;
// a ReLU mask; a float32 atomic add for split-K products).  Layer shapes
// that this tile fits badly have kernels of their own: a single input
// channel (nine products per output) runs on the vector ALUs, and the
// 32 -> 64 channel convolution's forward and input gradient keep the
// weights in registers and stream 16-pixel blocks through the 16x16x32
// instruction.  bf16 values are stored as uint16_t bit patterns and rounded
// from float32 to nearest even.
#include "common.hpp"

namespace tdp {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 64;   // output tile edge

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x0040u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint4 pack8(const uint16_t e[8]) {
    uint4 r;
    r.x = (uint32_t)e[0] | ((uint32_t)e[1] << 16);
    r.y = (uint32_t)e[2] | ((uint32_t)e[3] << 16);
    r.z = (uint32_t)e[4] | ((uint32_t)e[5] << 16);
    r.w = (uint32_t)e[6] | ((uint32_t)e[7] << 16);
    return r;
}

// ------------------------------------------------------------------ GEMM
//
// C[m, n] = sum_k A[m, k] B[n, k] over a 64 x 64 output tile per workgroup,
// K step 64 (two 16x16x32 MFMA sub-steps per barrier), four waves each
// owning a 32 x 32 quarter as 2 x 2 MFMA blocks.  The next step's global
// loads are issued before the current step's MFMAs.  An operand is read in
// one of two forms, fixed per operation at compile time:
//   K-contiguous (A_T / B_T false): load_a(m, k) / load_b(n, k) return 8
//     consecutive k of row m (n); each thread loads rows t/4 at k offsets
//     (t%4)*8 and +32 and stores them to LDS as 16-byte words;
//   transposed (A_T / B_T true): load_a(k, m0) / load_b(k, n0) return 8
//     consecutive m (n) at one k, the layout of activations whose reduction
//     index is the slow dimension; each thread loads two consecutive k of an
//     8-wide chunk and writes them transposed into LDS as 32-bit pairs.
// Either way the MFMA fragments read K-contiguous LDS rows.  With split-K
// (grid z) the partial tiles are added by the operation's store (float32
// atomics).  Operations with a bias gradient sum A's rows (the columns of
// dY) in the workgroups of the first column tile.

constexpr int kStep = 64;            // K step
constexpr int kLdsRow = kStep + 8;   // LDS row stride (elements), 16-byte multiple

template <bool T, class F>
__device__ __forceinline__ void stage_operand(uint16_t (*S)[kLdsRow], int t, const uint4 v[2]) {
    if (!T) {
        const int row = t >> 2, kc = (t & 3) * 8;
        *(uint4*)&S[row][kc] = v[0];
        *(uint4*)&S[row][kc + 32] = v[1];
    } else {
        const int lk = (t & 31) * 2, lc = (t >> 5) * 8;
        const uint32_t u0[4] = {v[0].x, v[0].y, v[0].z, v[0].w}, u1[4] = {v[1].x, v[1].y, v[1].z, v[1].w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            *(uint32_t*)&S[lc + 2 * h][lk] = (u0[h] & 0xFFFFu) | (u1[h] << 16);
            *(uint32_t*)&S[lc + 2 * h + 1][lk] = (u0[h] >> 16) | (u1[h] & 0xFFFF0000u);
        }
    }
}

// The row (K-contiguous form) or column chunk (transposed form) of A and B a
// thread loads: fixed for the whole K loop.
template <bool T>
__device__ __forceinline__ int64_t load_row(int t, int64_t base) { return T ? base + (t >> 5) * 8 : base + (t >> 2); }

template <class Op, class AC, class BC>
__device__ __forceinline__ void load_step(const Op& op, const AC& ac, const BC& bc, int t, int64_t k0, int64_t kend,
                                          uint4 a[2], uint4 b[2]) {
    if (!Op::A_T) {
        const int64_t k = k0 + (t & 3) * 8;
        a[0] = op.load_a(ac, k, kend);
        a[1] = op.load_a(ac, k + 32, kend);
    } else {
        const int64_t k = k0 + (t & 31) * 2;
        a[0] = op.load_a(ac, k, kend);
        a[1] = op.load_a(ac, k + 1, kend);
    }
    if (!Op::B_T) {
        const int64_t k = k0 + (t & 3) * 8;
        b[0] = op.load_b(bc, k, kend);
        b[1] = op.load_b(bc, k + 32, kend);
    } else {
        const int64_t k = k0 + (t & 31) * 2;
        b[0] = op.load_b(bc, k, kend);
        b[1] = op.load_b(bc, k + 1, kend);
    }
}

template <class Op>
__global__ __launch_bounds__(256) void mfma_gemm_kernel(Op op, float* db) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kT][kLdsRow];  // [m][k]
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kT][kLdsRow];  // [n][k]
    __shared__ float s_db[kT];
    const int64_t m0 = (int64_t)blockIdx.y * kT;
    const int n0 = blockIdx.x * kT;
    const int64_t kbeg = (int64_t)blockIdx.z * op.kchunk;
    const int64_t kend = kbeg + op.kchunk < op.K ? kbeg + op.kchunk : op.K;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    // bias gradient: only transposed A (rows of dY^T) carries it
    const bool do_bias = Op::A_T && db != nullptr && blockIdx.x == 0;
    float bsum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (t < kT) s_db[t] = 0.f;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    uint4 av[2], bv[2];
    const auto ac = op.a_ctx(load_row<Op::A_T>(t, m0));
    const auto bc = op.b_ctx(load_row<Op::B_T>(t, n0));
    load_step(op, ac, bc, t, kbeg, kend, av, bv);
    for (int64_t k0 = kbeg; k0 < kend; k0 += kStep) {
        __syncthreads();
        stage_operand<Op::A_T, Op>(As, t, av);
        stage_operand<Op::B_T, Op>(Bs, t, bv);
        if (do_bias) {
            const uint32_t u0[4] = {av[0].x, av[0].y, av[0].z, av[0].w};
            const uint32_t u1[4] = {av[1].x, av[1].y, av[1].z, av[1].w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                bsum[2 * h] += bf2f((uint16_t)(u0[h] & 0xFFFFu)) + bf2f((uint16_t)(u1[h] & 0xFFFFu));
                bsum[2 * h + 1] += bf2f((uint16_t)(u0[h] >> 16)) + bf2f((uint16_t)(u1[h] >> 16));
            }
        }
        __syncthreads();
        if (k0 + kStep < kend) load_step(op, ac, bc, t, k0 + kStep, kend, av, bv);
#pragma unroll
        for (int ks = 0; ks < kStep; ks += 32) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const bf16x8 a = *(const bf16x8*)&As[wm + i * 16 + (lane & 15)][ks + (lane >> 4) * 8];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const bf16x8 b = *(const bf16x8*)&Bs[wn + j * 16 + (lane & 15)][ks + (lane >> 4) * 8];
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t m = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
                const int n = n0 + wn + j * 16 + (lane & 15);
                if (m < op.M && n < op.N) op.store(m, n, acc[i][j][r]);
            }
    if (do_bias) {
        const int lc = (t >> 5) * 8;
#pragma unroll
        for (int q = 0; q < 8; ++q) atomicAdd(&s_db[lc + q], bsum[q]);
        __syncthreads();
        if (t < kT && m0 + t < op.M) atomicAdd(&db[m0 + t], s_db[t]);
    }
}

template <class Op>
int launch_gemm(const Op& op, hipStream_t s, const char* what, float* db = nullptr) {
    if (op.M <= 0 || op.N <= 0 || op.K <= 0) return TDP_OK;
    const int64_t splits = ceil_div(op.K, op.kchunk);
    dim3 grid((unsigned)ceil_div(op.N, kT), (unsigned)ceil_div(op.M, kT), (unsigned)splits);
    if (grid.y > 65535 * 16 || grid.z > 65535) return fail(TDP_EINVAL, "%s: problem too large", what);
    mfma_gemm_kernel<Op><<<grid, 256, 0, s>>>(op, db);
    return launch_status(what);
}

// The whole reduction in one workgroup (no split).
int64_t full_chunk(int64_t K) { return ceil_div(K, kStep) * kStep; }

// Split-K chunk: about 2 * 256 workgroups in total, at least 4 steps each.
int64_t split_chunk(int64_t K, int64_t tiles) {
    int64_t want = std::max<int64_t>(1, (2 * kCUs + tiles - 1) / tiles);
    int64_t chunk = ceil_div(K, want);
    chunk = std::max<int64_t>(kStep * 4, ceil_div(chunk, kStep) * kStep);
    return chunk;
}

// 8 bf16 from p[0..7] when all exist and the row is 16-byte aligned, else
// element by element (missing ones zero).
__device__ __forceinline__ uint4 row8(const uint16_t* p, int64_t avail, bool vec) {
    uint16_t e[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (avail <= 0) return pack8(e);
    if (vec && avail >= 8) return *(const uint4*)p;
#pragma unroll
    for (int q = 0; q < 8; ++q)
        if (q < avail) e[q] = p[q];
    return pack8(e);
}

// Operands read rows (or column chunks) that stay fixed while K advances, so
// each loader splits into a per-thread context, computed once before the K
// loop (pixel coordinates, the tap of a column), and a load per K step.
struct Ctx0 {
    int64_t i;
};

// k / c by a shift when c is a power of two (sh >= 0), else by division
__device__ __forceinline__ uint32_t div_pow2(uint32_t k, uint32_t c, int sh) { return sh >= 0 ? k >> sh : k / c; }

// y[b, oy, ox, co] = act(bias[co] + sum_{ky,kx,ci} x[b, oy+ky, ox+kx, ci] w[co][ky][kx][ci])
// A = im2col(x) [pixel][(tap, ci)], B = w [co][(tap, ci)], both K-contiguous.
struct ConvFwdOp {
    static constexpr bool A_T = false, B_T = false;
    const uint16_t* x;
    const uint16_t* w;
    const float* bias;
    uint16_t* y;
    int H, W, Cin, Ho, Wo, relu;
    int64_t M, K, kchunk;
    int N;
    int cin_shift;  // log2(Cin) when a power of two, else -1
    struct ACtx {
        int64_t pix;  // input pixel of tap (0, 0); -1 past the last output pixel
    };
    __device__ ACtx a_ctx(int64_t m) const {
        if (m >= M) return {-1};
        const uint32_t hw = (uint32_t)(Ho * Wo), mm = (uint32_t)m;  // pixel counts < 2^31
        const uint32_t b = mm / hw, r = mm - b * hw, oy = r / (uint32_t)Wo, ox = r - oy * (uint32_t)Wo;
        return {((int64_t)b * H + oy) * W + ox};
    }
    __device__ uint4 load_a(const ACtx& c, int64_t k, int64_t kend) const {
        uint16_t e[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (c.pix < 0 || k >= kend) return pack8(e);
        if ((Cin & 7) == 0 && k + 8 <= kend) {
            const uint32_t tap = div_pow2((uint32_t)k, (uint32_t)Cin, cin_shift), ci = (uint32_t)k - tap * Cin;
            const uint32_t ky = tap / 3, kx = tap - ky * 3;
            return *(const uint4*)&x[(c.pix + (int64_t)ky * W + kx) * Cin + ci];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t kk = k + q;
            if (kk < kend) {
                const uint32_t tap = div_pow2((uint32_t)kk, (uint32_t)Cin, cin_shift), ci = (uint32_t)kk - tap * Cin;
                const uint32_t ky = tap / 3, kx = tap - ky * 3;
                e[q] = x[(c.pix + (int64_t)ky * W + kx) * Cin + ci];
            }
        }
        return pack8(e);
    }
    __device__ Ctx0 b_ctx(int64_t n) const { return {n}; }
    __device__ uint4 load_b(const Ctx0& c, int64_t k, int64_t kend) const {
        return c.i < N ? row8(&w[c.i * K + k], kend - k, (K & 7) == 0) : row8(nullptr, 0, false);
    }
    __device__ void store(int64_t m, int n, float v) const {
        v += bias ? bias[n] : 0.f;
        if (relu && v < 0.f) v = 0.f;
        y[m * N + n] = f2bf(v);
    }
};

// dx[b, iy, ix, ci] = mask * sum_{ky,kx,co} dy[b, iy-ky, ix-kx, co] w[co][ky][kx][ci]
// A = gathered dy [input pixel][(tap, co)] (K-contiguous); B read transposed:
// at k = (tap, co), w[co][tap][ci0..ci0+7] holds 8 consecutive n = ci.
struct ConvDgradOp {
    static constexpr bool A_T = false, B_T = true;
    const uint16_t* dy;
    const uint16_t* w;
    const uint16_t* mask;
    uint16_t* dx;
    int H, W, Cout, Ho, Wo;
    int64_t M, K, kchunk;
    int N;  // Cin
    int cout_shift;  // log2(Cout) when a power of two, else -1
    struct ACtx {
        int64_t b;  // -1 past the last input pixel
        int iy, ix;
    };
    __device__ ACtx a_ctx(int64_t m) const {
        if (m >= M) return {-1, 0, 0};
        const uint32_t hw = (uint32_t)(H * W), mm = (uint32_t)m;
        const uint32_t b = mm / hw, r = mm - b * hw, iy = r / (uint32_t)W, ix = r - iy * (uint32_t)W;
        return {(int64_t)b, (int)iy, (int)ix};
    }
    __device__ uint4 load_a(const ACtx& c, int64_t k, int64_t kend) const {
        uint16_t e[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (c.b < 0 || k >= kend) return pack8(e);
        if ((Cout & 7) == 0 && k + 8 <= kend) {
            const uint32_t tap = div_pow2((uint32_t)k, (uint32_t)Cout, cout_shift), co = (uint32_t)k - tap * Cout;
            const int oy = c.iy - (int)(tap / 3), ox = c.ix - (int)(tap % 3);
            if (oy < 0 || oy >= Ho || ox < 0 || ox >= Wo) return pack8(e);
            return *(const uint4*)&dy[((c.b * Ho + oy) * Wo + ox) * Cout + co];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t kk = k + q;
            if (kk >= kend) continue;
            const uint32_t tap = div_pow2((uint32_t)kk, (uint32_t)Cout, cout_shift), co = (uint32_t)kk - tap * Cout;
            const int oy = c.iy - (int)(tap / 3), ox = c.ix - (int)(tap % 3);
            if (oy >= 0 && oy < Ho && ox >= 0 && ox < Wo) e[q] = dy[((c.b * Ho + oy) * Wo + ox) * Cout + co];
        }
        return pack8(e);
    }
    __device__ Ctx0 b_ctx(int64_t n0) const { return {n0}; }
    __device__ uint4 load_b(const Ctx0& c, int64_t k, int64_t kend) const {
        if (k >= kend) return row8(nullptr, 0, false);
        const uint32_t tap = div_pow2((uint32_t)k, (uint32_t)Cout, cout_shift), co = (uint32_t)k - tap * Cout;
        return row8(&w[((int64_t)co * 9 + tap) * N + c.i], N - c.i, (N & 7) == 0);
    }
    __device__ void store(int64_t m, int n, float v) const {
        if (mask && !(bf2f(mask[m * N + n]) > 0.f)) v = 0.f;
        dx[m * N + n] = f2bf(v);
    }
};

// dw[co][ky][kx][ci] += sum_{b,oy,ox} dy[b,oy,ox,co] x[b, oy+ky, ox+kx, ci]
// Both operands transposed: at output pixel k, dy[k][co0..] and
// im2col(x)[k][(tap, ci0)..] hold 8 consecutive m and n.
struct ConvWgradOp {
    static constexpr bool A_T = true, B_T = true;
    const uint16_t* x;
    const uint16_t* dy;
    float* dw;
    int H, W, Cin, Ho, Wo;
    int64_t M, K, kchunk;  // M = Cout, K = B*Ho*Wo
    int N;                 // 9*Cin
    __device__ Ctx0 a_ctx(int64_t m0) const { return {m0}; }
    __device__ uint4 load_a(const Ctx0& c, int64_t k, int64_t kend) const {
        if (k >= kend) return row8(nullptr, 0, false);
        return row8(&dy[k * M + c.i], M - c.i, (M & 7) == 0);
    }
    struct BCtx {
        int n0;
        int off;  // (ky * W + kx) * Cin + ci of column n0 when Cin is a multiple of 8
    };
    __device__ BCtx b_ctx(int64_t n0) const {
        int off = 0;
        if ((Cin & 7) == 0 && n0 < N) {  // n0..n0+7 share one tap
            const int tap = (int)(n0 / Cin), ci = (int)(n0 - (int64_t)tap * Cin);
            const int ky = tap / 3, kx = tap - ky * 3;
            off = (ky * W + kx) * Cin + ci;
        }
        return {(int)n0, off};
    }
    __device__ uint4 load_b(const BCtx& c, int64_t k, int64_t kend) const {
        uint16_t e[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (k >= kend || c.n0 >= N) return pack8(e);
        const uint32_t hw = (uint32_t)(Ho * Wo), kk = (uint32_t)k;  // pixel counts < 2^31
        const uint32_t b = kk / hw, r = kk - b * hw, oy = r / (uint32_t)Wo, ox = r - oy * (uint32_t)Wo;
        const int64_t pix = ((int64_t)b * H + oy) * W + ox;  // input pixel of tap (0, 0)
        if ((Cin & 7) == 0) return *(const uint4*)&x[pix * Cin + c.off];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int n = c.n0 + q;
            if (n < N) {
                const int tap = n / Cin, ci = n - tap * Cin;
                const int ky = tap / 3, kx = tap - ky * 3;
                e[q] = x[(pix + (int64_t)ky * W + kx) * Cin + ci];
            }
        }
        return pack8(e);
    }
    __device__ void store(int64_t m, int n, float v) const { atomicAdd(&dw[m * N + n], v); }
};

// y[m, n] = act(bias[n] + sum_k x[m, k] w[n, k])
struct LinFwdOp {
    static constexpr bool A_T = false, B_T = false;
    const uint16_t* x;
    const uint16_t* w;
    const float* bias;
    uint16_t* y;
    float* yf;
    int relu;
    int64_t M, K, kchunk;
    int N;
    __device__ Ctx0 a_ctx(int64_t m) const { return {m}; }
    __device__ Ctx0 b_ctx(int64_t n) const { return {n}; }
    __device__ uint4 load_a(const Ctx0& c, int64_t k, int64_t kend) const {
        return c.i < M ? row8(&x[c.i * K + k], kend - k, (K & 7) == 0) : row8(nullptr, 0, false);
    }
    __device__ uint4 load_b(const Ctx0& c, int64_t k, int64_t kend) const {
        return c.i < N ? row8(&w[c.i * K + k], kend - k, (K & 7) == 0) : row8(nullptr, 0, false);
    }
    __device__ void store(int64_t m, int n, float v) const {
        v += bias ? bias[n] : 0.f;
        if (relu && v < 0.f) v = 0.f;
        if (yf)
            yf[m * N + n] = v;
        else
            y[m * N + n] = f2bf(v);
    }
};

// The same product as K-parallel partial sums added into a float32 buffer;
// linear_epilogue_kernel then adds the bias and applies the activation.
struct LinFwdAccOp {
    static constexpr bool A_T = false, B_T = false;
    const uint16_t* x;
    const uint16_t* w;
    float* yf;
    int64_t M, K, kchunk;
    int N;
    __device__ Ctx0 a_ctx(int64_t m) const { return {m}; }
    __device__ Ctx0 b_ctx(int64_t n) const { return {n}; }
    __device__ uint4 load_a(const Ctx0& c, int64_t k, int64_t kend) const {
        return c.i < M ? row8(&x[c.i * K + k], kend - k, (K & 7) == 0) : row8(nullptr, 0, false);
    }
    __device__ uint4 load_b(const Ctx0& c, int64_t k, int64_t kend) const {
        return c.i < N ? row8(&w[c.i * K + k], kend - k, (K & 7) == 0) : row8(nullptr, 0, false);
    }
    __device__ void store(int64_t m, int n, float v) const { atomicAdd(&yf[m * N + n], v); }
};

// dx[m, k] = mask * sum_n dy[m, n] w[n, k]   (GEMM M x Kin, reduction over Nout)
// B read transposed: at k = nout, w[nout][kin0..kin0+7] holds 8 consecutive n.
struct LinDgradOp {
    static constexpr bool A_T = false, B_T = true;
    const uint16_t* dy;
    const uint16_t* w;
    const uint16_t* mask;
    uint16_t* dx;
    int64_t M, K, kchunk;  // K = Nout
    int N;                 // Kin
    __device__ Ctx0 a_ctx(int64_t m) const { return {m}; }
    __device__ Ctx0 b_ctx(int64_t n0) const { return {n0}; }
    __device__ uint4 load_a(const Ctx0& c, int64_t k, int64_t kend) const {
        return c.i < M ? row8(&dy[c.i * K + k], kend - k, (K & 7) == 0) : row8(nullptr, 0, false);
    }
    __device__ uint4 load_b(const Ctx0& c, int64_t k, int64_t kend) const {
        return k < kend ? row8(&w[k * N + c.i], N - c.i, (N & 7) == 0) : row8(nullptr, 0, false);
    }
    __device__ void store(int64_t m, int n, float v) const {
        if (mask && !(bf2f(mask[m * N + n]) > 0.f)) v = 0.f;
        dx[m * N + n] = f2bf(v);
    }
};

// dw[n, k] += sum_m dy[m, n] x[m, k]   (GEMM Nout x Kin, reduction over the batch)
struct LinWgradOp {
    static constexpr bool A_T = true, B_T = true;
    const uint16_t* x;
    const uint16_t* dy;
    float* dw;
    int64_t M, K, kchunk;  // M = Nout, K = batch
    int N;                 // Kin
    __device__ Ctx0 a_ctx(int64_t m0) const { return {m0}; }
    __device__ Ctx0 b_ctx(int64_t n0) const { return {n0}; }
    __device__ uint4 load_a(const Ctx0& c, int64_t k, int64_t kend) const {
        return k < kend ? row8(&dy[k * M + c.i], M - c.i, (M & 7) == 0) : row8(nullptr, 0, false);
    }
    __device__ uint4 load_b(const Ctx0& c, int64_t k, int64_t kend) const {
        return k < kend ? row8(&x[k * N + c.i], N - c.i, (N & 7) == 0) : row8(nullptr, 0, false);
    }
    __device__ void store(int64_t m, int n, float v) const { atomicAdd(&dw[m * N + n], v); }
};

// ------------------------------------------------------- elementwise kernels

__global__ void zero_f32_kernel(float* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

// Two buffers in one launch (a weight gradient and its bias gradient).
__global__ void zero2_f32_kernel(float* p, int64_t n, float* q, int64_t nq) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n + nq; i += stride) {
        if (i < n)
            p[i] = 0.f;
        else
            q[i - n] = 0.f;
    }
}

// yf = act(yf + bias), y = bf16(yf)
__global__ void linear_epilogue_kernel(float* yf, const float* bias, int64_t M, int N, int relu, uint16_t* y) {
    const int64_t n_el = M * N;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_el; i += (int64_t)gridDim.x * blockDim.x) {
        float v = yf[i] + (bias ? bias[i % N] : 0.f);
        if (relu && v < 0.f) v = 0.f;
        yf[i] = v;
        y[i] = f2bf(v);
    }
}

__global__ void image_to_bf16_kernel(const uint8_t* img, int64_t n, uint16_t* out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = f2bf((float)img[i] / 255.0f);
}

__global__ void f32_to_bf16_kernel(const float* in, int64_t n, uint16_t* out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = f2bf(in[i]);
}

__global__ void maxpool2_fwd_kernel(const uint16_t* x, int B, int H, int W, int C, uint16_t* y) {
    const int Ho = H / 2, Wo = W / 2;
    const int64_t n = (int64_t)B * Ho * Wo * C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const int64_t p = i / C;
        const int ox = (int)(p % Wo), oy = (int)((p / Wo) % Ho);
        const int64_t b = p / ((int64_t)Wo * Ho);
        const int64_t base = ((b * H + 2 * oy) * W + 2 * ox) * C + c;
        float m = bf2f(x[base]);
        m = fmaxf(m, bf2f(x[base + C]));
        m = fmaxf(m, bf2f(x[base + (int64_t)W * C]));
        m = fmaxf(m, bf2f(x[base + (int64_t)W * C + C]));
        y[i] = f2bf(m);
    }
}

// The same with eight channels per thread (C % 8 == 0, 16-byte aligned
// tensors): four 16-byte window loads and one 16-byte store per thread,
// each channel reduced in the same order as above.
__global__ void maxpool2_fwd8_kernel(const uint16_t* x, int B, int H, int W, int C, uint16_t* y) {
    const int Ho = H / 2, Wo = W / 2, C8 = C / 8;
    const int64_t n = (int64_t)B * Ho * Wo * C8;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C8) * 8;
        const int64_t p = i / C8;
        const int ox = (int)(p % Wo), oy = (int)((p / Wo) % Ho);
        const int64_t b = p / ((int64_t)Wo * Ho);
        const int64_t base = ((b * H + 2 * oy) * W + 2 * ox) * C + c;
        const int64_t off[4] = {0, C, (int64_t)W * C, (int64_t)W * C + C};
        uint4 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = *(const uint4*)(x + base + off[q]);
        uint32_t out[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {  // two channels per 32-bit word
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) w[q] = h == 0 ? v[q].x : h == 1 ? v[q].y : h == 2 ? v[q].z : v[q].w;
            float lo = bf2f((uint16_t)(w[0] & 0xFFFF)), hi = bf2f((uint16_t)(w[0] >> 16));
#pragma unroll
            for (int q = 1; q < 4; ++q) {
                lo = fmaxf(lo, bf2f((uint16_t)(w[q] & 0xFFFF)));
                hi = fmaxf(hi, bf2f((uint16_t)(w[q] >> 16)));
            }
            out[h] = (uint32_t)f2bf(lo) | ((uint32_t)f2bf(hi) << 16);
        }
        *(uint4*)(y + p * C + c) = make_uint4(out[0], out[1], out[2], out[3]);
    }
}

// Gradient of 2x2 max pooling: each output gradient goes to the first
// maximum of its window in row-major order; optionally masked by x > 0 (the
// ReLU in front of the pooling).
__global__ void maxpool2_bwd_kernel(const uint16_t* x, const uint16_t* dy, int B, int H, int W, int C, int relu_mask,
                                    uint16_t* dx) {
    const int Ho = H / 2, Wo = W / 2;
    const int64_t n = (int64_t)B * Ho * Wo * C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const int64_t p = i / C;
        const int ox = (int)(p % Wo), oy = (int)((p / Wo) % Ho);
        const int64_t b = p / ((int64_t)Wo * Ho);
        int64_t at[4];
        at[0] = ((b * H + 2 * oy) * W + 2 * ox) * C + c;
        at[1] = at[0] + C;
        at[2] = at[0] + (int64_t)W * C;
        at[3] = at[2] + C;
        int best = 0;
        float m = bf2f(x[at[0]]);
        for (int q = 1; q < 4; ++q) {
            const float v = bf2f(x[at[q]]);
            if (v > m) {
                m = v;
                best = q;
            }
        }
        const uint16_t g = dy[i];
        for (int q = 0; q < 4; ++q) {
            uint16_t o = q == best ? g : (uint16_t)0;
            if (relu_mask && !(bf2f(x[at[q]]) > 0.f)) o = 0;
            dx[at[q]] = o;
        }
    }
}

// The gradient with eight channels per thread (C % 8 == 0, 16-byte aligned):
// per channel the same first-maximum rule and optional ReLU mask.
__global__ void maxpool2_bwd8_kernel(const uint16_t* x, const uint16_t* dy, int B, int H, int W, int C, int relu_mask,
                                     uint16_t* dx) {
    const int Ho = H / 2, Wo = W / 2, C8 = C / 8;
    const int64_t n = (int64_t)B * Ho * Wo * C8;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C8) * 8;
        const int64_t p = i / C8;
        const int ox = (int)(p % Wo), oy = (int)((p / Wo) % Ho);
        const int64_t b = p / ((int64_t)Wo * Ho);
        const int64_t base = ((b * H + 2 * oy) * W + 2 * ox) * C + c;
        const int64_t off[4] = {0, C, (int64_t)W * C, (int64_t)W * C + C};
        uint16_t xv[4][8], o[4][8];
#pragma unroll
        for (int q = 0; q < 4; ++q) *(uint4*)xv[q] = *(const uint4*)(x + base + off[q]);
        uint16_t g[8];
        *(uint4*)g = *(const uint4*)(dy + p * C + c);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            int best = 0;
            float m = bf2f(xv[0][k]);
#pragma unroll
            for (int q = 1; q < 4; ++q) {
                const float v = bf2f(xv[q][k]);
                if (v > m) {
                    m = v;
                    best = q;
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint16_t r = q == best ? g[k] : (uint16_t)0;
                if (relu_mask && !(bf2f(xv[q][k]) > 0.f)) r = 0;
                o[q][k] = r;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) *(uint4*)(dx + base + off[q]) = *(const uint4*)o[q];
    }
}

// p = softmax(logits) per row, e = sum_k k p_k (the expected label).
__global__ void softmax_expect_kernel(const float* logits, int M, int K, float* p, float* e) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const float* z = logits + (int64_t)m * K;
    float mx = z[0];
    for (int k = 1; k < K; ++k) mx = fmaxf(mx, z[k]);
    float s = 0.f;
    for (int k = 0; k < K; ++k) s += __expf(z[k] - mx);
    const float inv = 1.0f / s;
    float ev = 0.f;
    for (int k = 0; k < K; ++k) {
        const float pk = __expf(z[k] - mx) * inv;
        p[(int64_t)m * K + k] = pk;
        ev += (float)k * pk;
    }
    if (e) e[m] = ev;
}

// dlogits_k = dE p_k (k - E)
__global__ void softmax_expect_bwd_kernel(const float* p, const float* dE, int M, int K, float* dz, uint16_t* dz_bf) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const float* pr = p + (int64_t)m * K;
    float ev = 0.f;
    for (int k = 0; k < K; ++k) ev += (float)k * pr[k];
    for (int k = 0; k < K; ++k) {
        const float g = dE[m] * pr[k] * ((float)k - ev);
        if (dz) dz[(int64_t)m * K + k] = g;
        if (dz_bf) dz_bf[(int64_t)m * K + k] = f2bf(g);
    }
}

// General softmax backward: dz_k = p_k (dP_k - sum_j p_j dP_j).
__global__ void softmax_bwd_kernel(const float* p, const float* dP, int M, int K, float* dz, uint16_t* dz_bf) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const float* pr = p + (int64_t)m * K;
    const float* dr = dP + (int64_t)m * K;
    float dot = 0.f;
    for (int k = 0; k < K; ++k) dot += pr[k] * dr[k];
    for (int k = 0; k < K; ++k) {
        const float g = pr[k] * (dr[k] - dot);
        if (dz) dz[(int64_t)m * K + k] = g;
        if (dz_bf) dz_bf[(int64_t)m * K + k] = f2bf(g);
    }
}

__global__ void argmax_kernel(const float* p, int M, int K, int8_t* out) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    int best = 0;
    for (int k = 1; k < K; ++k)
        if (p[(int64_t)m * K + k] > p[(int64_t)m * K + best]) best = k;
    out[m] = (int8_t)best;
}

__device__ __forceinline__ void adam_elem(float* p, const float* g, float* m, float* v, int64_t i, float lr, float b1,
                                          float b2, float eps, float c1, float c2, uint16_t* p_bf) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (p_bf) p_bf[i] = f2bf(pi);
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2, uint16_t* p_bf) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        adam_elem(p, g, m, v, i, lr, b1, b2, eps, c1, c2, p_bf);
}

// Every tensor of a model in one launch: blockIdx.y picks the tensor.
constexpr int kAdamMaxTensors = 16;
struct AdamList {
    tdp_adam_tensor t[kAdamMaxTensors];
};

__global__ void adam_multi_kernel(AdamList L, float lr, float b1, float b2, float eps, float c1, float c2) {
    const tdp_adam_tensor& a = L.t[blockIdx.y];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * blockDim.x)
        adam_elem(a.p, a.g, a.m, a.v, i, lr, b1, b2, eps, c1, c2, a.p_bf16);
}

// ------------------------------------------ one input channel (first layer)
// With a single input channel each output has only nine products, so the
// 64-deep K step of the MFMA tile would be 7/8 padding; the forward and the
// weight gradient of such a layer run on the vector ALUs.  Cout is 8, 16, 32
// or 64 (eight channels per thread).

constexpr int kC1MaxCout = 64;

// y[p][co] = act(bias[co] + sum_tap x[p + tap] w[co][tap]): one thread per
// output pixel reads its nine inputs once and writes all Cout channels, 8 at
// a time (taps summed in order with fused multiply-adds, then the bias) as
// 16-byte stores.  Weights and bias are held as float32 in LDS and read by
// every lane at the same address.
__global__ __launch_bounds__(256) void conv1_fwd_kernel(const uint16_t* __restrict__ x, const uint16_t* __restrict__ w,
                                                        const float* __restrict__ bias, int H, int W, int Cout,
                                                        int relu, int64_t M, uint16_t* __restrict__ y) {
    __shared__ float s_w[kC1MaxCout * 9];
    __shared__ float s_b[kC1MaxCout];
    for (int i = threadIdx.x; i < Cout * 9; i += blockDim.x) s_w[i] = bf2f(w[i]);
    for (int i = threadIdx.x; i < Cout; i += blockDim.x) s_b[i] = bias ? bias[i] : 0.f;
    __syncthreads();
    const uint32_t Ho = (uint32_t)(H - 2), Wo = (uint32_t)(W - 2), hw = Ho * Wo;  // pixel counts < 2^31
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < M; m += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t mm = (uint32_t)m, b = mm / hw, r = mm - b * hw, oy = r / Wo, ox = r - oy * Wo;
        const uint16_t* xp = x + ((int64_t)b * H + oy) * W + ox;
        float xv[9];
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) xv[ky * 3 + kx] = bf2f(xp[ky * W + kx]);
        for (int c0 = 0; c0 < Cout; c0 += 8) {
            uint16_t out[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float* wq = &s_w[(c0 + q) * 9];
                float acc = 0.f;
#pragma unroll
                for (int tap = 0; tap < 9; ++tap) acc = fmaf(xv[tap], wq[tap], acc);
                acc += s_b[c0 + q];
                if (relu && acc < 0.f) acc = 0.f;
                out[q] = f2bf(acc);
            }
            *(uint4*)&y[m * Cout + c0] = pack8(out);
        }
    }
}

// dw[co][tap] = sum_p dy[p][co] x[p + tap] and db[co] = sum_p dy[p][co] over
// the workgroup's pixel range: each thread keeps 8 channels x (9 taps + bias)
// in registers over its pixels (two per step, loads always issued); lanes of
// a wave that share channels are added by shuffles, the 16 waves' sums in
// LDS in wave order, then one float32 atomic add per output and workgroup
// (dw and db start at zero).  Few large workgroups: device-scope float
// atomics on the same few lines are the cost that grows with their number.
constexpr int kC1WgThreads = 1024;

__global__ __launch_bounds__(kC1WgThreads) void conv1_wgrad_kernel(const uint16_t* __restrict__ x,
                                                                   const uint16_t* __restrict__ dy, int H, int W,
                                                                   int Cout, int chunk_shift, int64_t M,
                                                                   int64_t per_wg, float* dw, float* db) {
    constexpr int kWaves = kC1WgThreads / kWave;
    __shared__ float s_part[kWaves][kC1MaxCout * 10];
    const int chunks = 1 << chunk_shift;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int c0 = (t & (chunks - 1)) * 8;
    const int pl = t >> chunk_shift, npl = kC1WgThreads >> chunk_shift;
    const uint32_t Ho = (uint32_t)(H - 2), Wo = (uint32_t)(W - 2), hw = Ho * Wo;
    float acc[8][10];
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int j = 0; j < 10; ++j) acc[q][j] = 0.f;
    const int64_t p0 = (int64_t)blockIdx.x * per_wg;
    const int64_t p1 = p0 + per_wg < M ? p0 + per_wg : M;
    for (int64_t mb = p0 + pl; mb < p1; mb += 2 * npl) {
        float xv[2][9], dv[2][8];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t m = mb + u * npl;
            const bool in = m < p1;
            const uint32_t mm = in ? (uint32_t)m : 0u, b = mm / hw, r = mm - b * hw, oy = r / Wo, ox = r - oy * Wo;
            const uint16_t* xp = x + ((int64_t)b * H + oy) * W + ox;
#pragma unroll
            for (int ky = 0; ky < 3; ++ky)
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) xv[u][ky * 3 + kx] = bf2f(xp[ky * W + kx]);
            const uint4 d = *(const uint4*)&dy[(int64_t)mm * Cout + c0];
            const uint32_t du[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
            for (int q = 0; q < 8; ++q)
                dv[u][q] = in ? bf2f((uint16_t)((q & 1) ? (du[q >> 1] >> 16) : (du[q >> 1] & 0xFFFFu))) : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
#pragma unroll
                for (int tap = 0; tap < 9; ++tap) acc[q][tap] = fmaf(dv[u][q], xv[u][tap], acc[q][tap]);
                acc[q][9] += dv[u][q];
            }
    }
    for (int off = chunks; off < kWave; off <<= 1)
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int j = 0; j < 10; ++j) acc[q][j] += __shfl_xor(acc[q][j], off, kWave);
    if (lane < chunks) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int j = 0; j < 10; ++j) s_part[wave][(c0 + q) * 10 + j] = acc[q][j];
    }
    __syncthreads();
    for (int i = t; i < Cout * 10; i += blockDim.x) {
        float v = 0.f;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) v += s_part[k][i];
        const int co = i / 10, j = i - co * 10;
        if (j < 9)
            atomicAdd(&dw[co * 9 + j], v);
        else if (db)
            atomicAdd(&db[co], v);
    }
}

// ------------------------------- 32 input channels, 16..64 output channels
// The second layer's forward as its own MFMA kernel: with Cin = 32 one tap is
// exactly one 32-deep K block, and the weight matrix (9 taps x Cout rows of
// 32) fits in registers.  The product is taken transposed, D[co][pixel] =
// sum_k W[co][k] im2col[pixel][k], so that a lane's accumulator holds four
// consecutive output channels of one pixel and leaves as one 8-byte store.
// Each wave walks a contiguous range of 16-pixel blocks (neighbouring blocks
// share input rows, which then stay in the wave's caches); each tap's pixel
// fragment (8 channels of one input pixel per lane, a 16-byte load) is
// reloaded for the next block as soon as the current block's MFMAs of that
// tap are issued, so one set of nine fragment registers serves both blocks.

// Input offset (elements) of this lane's tap-(0,0) fragment for pixel block
// `blk`, or -1 past the last output pixel.
__device__ __forceinline__ int64_t c32_base(int64_t blk, int64_t M, uint32_t hw, uint32_t Wo, int H, int W,
                                            int lane) {
    const int64_t m = blk * 16 + (lane & 15);
    if (m >= M) return -1;
    const uint32_t mm = (uint32_t)m, b = mm / hw, r = mm - b * hw, oy = r / Wo, ox = r - oy * Wo;
    return (((int64_t)b * H + oy) * W + ox) * 32 + (lane >> 4) * 8;
}

// Fragment loads go through the buffer unit: an offset past the end of the
// buffer reads zeros (its range check), so a missing fragment needs no lane
// condition.  (Loads under a lane condition make the compiler wait for every
// outstanding load at the top of the block loop, which undoes the prefetch.)
// Buffers are under 2 GiB, so byte offsets fit 31 bits.
constexpr uint32_t kNoFrag = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* p, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ uint4 buf_load16(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)byte_off, 0, 0));
}

__device__ __forceinline__ uint2 buf_load8(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    return __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, 0, 0));
}

__device__ __forceinline__ uint4 c32_frag(__amdgpu_buffer_rsrc_t xr, int64_t base, int off) {
    return buf_load16(xr, base >= 0 ? (uint32_t)((base + off) * 2) : kNoFrag);
}

template <int NB>
__global__ __launch_bounds__(256, 2) void conv_fwd_c32_kernel(const uint16_t* __restrict__ x,
                                                               const uint16_t* __restrict__ w,
                                                               const float* __restrict__ bias, int H, int W, int relu,
                                                               int64_t M, int64_t per_wave, int64_t x_bytes,
                                                               uint16_t* __restrict__ y) {
    constexpr int Cout = 16 * NB;
    const __amdgpu_buffer_rsrc_t xr = buffer_of(x, x_bytes);
    const int lane = threadIdx.x & 63;
    const int64_t wave_id = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nblk = (M + 15) / 16;
    const int64_t blk0 = wave_id * per_wave;
    const int64_t blk1 = blk0 + per_wave < nblk ? blk0 + per_wave : nblk;
    if (blk0 >= blk1) return;
    // A fragments: row co = j*16 + (lane & 15), K slice (lane >> 4) * 8 of each tap
    bf16x8 wf[9][NB];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const uint4 v = *(const uint4*)&w[((int64_t)(j * 16 + (lane & 15)) * 9 + t) * 32 + (lane >> 4) * 8];
            wf[t][j] = __builtin_bit_cast(bf16x8, v);
        }
    float bv[NB][4];
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) bv[j][r] = bias ? bias[j * 16 + (lane >> 4) * 4 + r] : 0.f;
    const uint32_t Wo = (uint32_t)(W - 2), hw = (uint32_t)(H - 2) * Wo;
    int off[9];  // element offset of tap (ky, kx) from tap (0, 0)
#pragma unroll
    for (int t = 0; t < 9; ++t) off[t] = ((t / 3) * W + t % 3) * 32;
    uint4 f[9];
    int64_t base = c32_base(blk0, M, hw, Wo, H, W, lane);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        f[t] = c32_frag(xr, base, off[t]);  // in tap order, as the loop reloads them
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int64_t blk = blk0; blk < blk1; ++blk) {
        const int64_t nbase = blk + 1 < blk1 ? c32_base(blk + 1, M, hw, Wo, H, W, lane) : -1;
        f32x4 acc[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const bf16x8 pf = __builtin_bit_cast(bf16x8, f[t]);
#pragma unroll
            for (int j = 0; j < NB; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[t][j], pf, acc[j], 0, 0, 0);
            f[t] = c32_frag(xr, nbase, off[t]);  // zero (unused) after the last block
            __builtin_amdgcn_sched_barrier(0);    // keep the reload here, not after the last tap
        }
        // lane holds channels j*16 + (lane >> 4)*4 + r of pixel blk*16 + (lane & 15)
        if (base >= 0) {
            const int64_t m = blk * 16 + (lane & 15);
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int c = j * 16 + (lane >> 4) * 4;
                uint16_t o[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float v = acc[j][r] + bv[j][r];
                    if (relu && v < 0.f) v = 0.f;
                    o[r] = f2bf(v);
                }
                const uint2 pk = make_uint2((uint32_t)o[0] | ((uint32_t)o[1] << 16),
                                            (uint32_t)o[2] | ((uint32_t)o[3] << 16));
                *(uint2*)&y[m * Cout + c] = pk;
            }
        }
        base = nbase;
    }
}

// The second layer's input gradient, the same way: with Cout = 64 a tap is
// two 32-deep K blocks, D[ci][pixel] = sum_{tap, co} W[co][tap][ci] *
// dy[pixel - tap][co] (zero outside the output), taken transposed so that a
// lane stores four consecutive input channels of one pixel (masked by the
// activation) as 8 bytes.  The workgroup copies the weights to LDS once;
// each wave owns one 16-channel block of the NJ = Cin / 16 (neighbouring
// waves take the other blocks of the same pixels, so the dy fragments they
// share come from the CU's cache), builds its 9 x 2 weight fragments (the 8
// output channels of one (tap, ci) are strided in memory) and walks a
// contiguous range of 16-pixel blocks, reloading each pixel fragment for the
// next block once the current block's MFMA on it is issued.
constexpr int kDgCout = 64;

// Zero when the tap falls outside the output (a buffer load past the end).
__device__ __forceinline__ uint4 dg_frag(__amdgpu_buffer_rsrc_t dyr, int64_t pix_b, int iy, int ix, int t, int Ho,
                                         int Wo, int co) {
    const int oy = iy - t / 3, ox = ix - t % 3;
    const bool in = pix_b >= 0 && oy >= 0 && oy < Ho && ox >= 0 && ox < Wo;
    return buf_load16(dyr, in ? (uint32_t)((((pix_b * Ho + oy) * Wo + ox) * kDgCout + co) * 2) : kNoFrag);
}

template <int NJ>
__global__ __launch_bounds__(256, 2) void conv_dgrad_c64_kernel(const uint16_t* __restrict__ dy,
                                                                 const uint16_t* __restrict__ w,
                                                                 const uint16_t* __restrict__ mask, int H, int W,
                                                                 int64_t M, int64_t per_wave, int64_t dy_bytes,
                                                                 uint16_t* __restrict__ dx) {
    constexpr int Cin = 16 * NJ;
    const __amdgpu_buffer_rsrc_t dyr = buffer_of(dy, dy_bytes);
    const __amdgpu_buffer_rsrc_t mr = buffer_of(mask, mask ? M * Cin * 2 : 0);
    constexpr int kWElems = kDgCout * 9 * Cin;
    __shared__ __attribute__((aligned(16))) uint16_t s_w[kWElems];
    for (int i = threadIdx.x * 8; i < kWElems; i += blockDim.x * 8) *(uint4*)&s_w[i] = *(const uint4*)&w[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t wave_id = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int jb = (int)(wave_id % NJ);
    const int64_t nblk = (M + 15) / 16;
    const int64_t blk0 = (wave_id / NJ) * per_wave;
    const int64_t blk1 = blk0 + per_wave < nblk ? blk0 + per_wave : nblk;
    if (blk0 >= blk1) return;
    // A fragments: row ci = jb*16 + (lane & 15); K = (tap, co), co = kb*32 + (lane >> 4)*8 + e
    bf16x8 wf[9][2];
    const int ci = jb * 16 + (lane & 15);
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            uint16_t e[8];
            const int co0 = kb * 32 + (lane >> 4) * 8;
#pragma unroll
            for (int q = 0; q < 8; ++q) e[q] = s_w[((co0 + q) * 9 + t) * Cin + ci];
            wf[t][kb] = __builtin_bit_cast(bf16x8, pack8(e));
        }
    const int Ho = H - 2, Wo = W - 2;
    const uint32_t hw = (uint32_t)(H * W);
    const int cs = (lane >> 4) * 8;  // this lane's output-channel slice within a K block
    auto pixel = [&](int64_t blk, int64_t& b, int& iy, int& ix) {
        const int64_t m = blk * 16 + (lane & 15);
        if (m >= M) {
            b = -1;
            iy = ix = 0;
            return;
        }
        const uint32_t mm = (uint32_t)m, bb = mm / hw, r = mm - bb * hw;
        b = bb;
        iy = (int)(r / (uint32_t)W);
        ix = (int)(r - (uint32_t)iy * (uint32_t)W);
    };
    int64_t b;
    int iy, ix;
    pixel(blk0, b, iy, ix);
    // the activation mask of a block is loaded one block ahead (a value used
    // in the same block would be moved after the fragment loads and make the
    // store wait for all of them)
    const int c = jb * 16 + (lane >> 4) * 4;
    uint2 mv = buf_load8(mr, b >= 0 ? (uint32_t)(((blk0 * 16 + (lane & 15)) * Cin + c) * 2) : kNoFrag);
    uint4 f[9][2];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            f[t][kb] = dg_frag(dyr, b, iy, ix, t, Ho, Wo, kb * 32 + cs);  // in the loop's reload order
            __builtin_amdgcn_sched_barrier(0);
        }
    for (int64_t blk = blk0; blk < blk1; ++blk) {
        int64_t nb = -1;
        int niy = 0, nix = 0;
        if (blk + 1 < blk1) pixel(blk + 1, nb, niy, nix);
        const int64_t m = blk * 16 + (lane & 15);
        const uint2 mv_next = buf_load8(mr, nb >= 0 ? (uint32_t)((((blk + 1) * 16 + (lane & 15)) * Cin + c) * 2) : kNoFrag);
        __builtin_amdgcn_sched_barrier(0);
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[t][kb], __builtin_bit_cast(bf16x8, f[t][kb]), acc,
                                                              0, 0, 0);
                f[t][kb] = dg_frag(dyr, nb, niy, nix, t, Ho, Wo, kb * 32 + cs);  // zero after the last block
                __builtin_amdgcn_sched_barrier(0);  // keep the reload here, not after the last tap
            }
        // lane holds input channels jb*16 + (lane >> 4)*4 + r of pixel m
        if (!mask) mv = make_uint2(0x3F803F80u, 0x3F803F80u);  // bf16 1.0 pairs: no mask
        if (b >= 0) {
            const uint16_t mk[4] = {(uint16_t)(mv.x & 0xFFFFu), (uint16_t)(mv.x >> 16), (uint16_t)(mv.y & 0xFFFFu),
                                    (uint16_t)(mv.y >> 16)};
            uint16_t o[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) o[r] = bf2f(mk[r]) > 0.f ? f2bf(acc[r]) : f2bf(0.f);
            const uint2 pk = make_uint2((uint32_t)o[0] | ((uint32_t)o[1] << 16),
                                        (uint32_t)o[2] | ((uint32_t)o[3] << 16));
            *(uint2*)&dx[m * Cin + c] = pk;
        }
        mv = mv_next;
        b = nb;
        iy = niy;
        ix = nix;
    }
}

// log2(Cout / 8) when the single-channel kernels take this layer, else -1.
int conv1_chunk_shift(int Cin, int Cout) {
    if (Cin != 1) return -1;
    switch (Cout) {
        case 8: return 0;
        case 16: return 1;
        case 32: return 2;
        case 64: return 3;
        default: return -1;
    }
}

int ew_grid(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>(ceil_div(n, 256), 1), 16 * kCUs); }

bool a16(const void* p) { return ((uintptr_t)p & 15) == 0; }

int zero_f32(float* p, int64_t n, hipStream_t s) {
    if (n > 0) zero_f32_kernel<<<ew_grid(n), 256, 0, s>>>(p, n);
    return launch_status("zero");
}

// dw (n floats) and, when db is not null, db (nb floats) in one launch.
int zero_grads(float* dw, int64_t n, float* db, int64_t nb, hipStream_t s) {
    if (!db) nb = 0;
    if (n + nb > 0) zero2_f32_kernel<<<ew_grid(n + nb), 256, 0, s>>>(dw, n, db, nb);
    return launch_status("zero");
}


}  // namespace

}  // namespace tdp

using namespace tdp;

extern "C" int tdp_image_to_bf16(const uint8_t* img, int64_t n, uint16_t* out, hipStream_t stream) {
    if (n < 0 || (n > 0 && (!img || !out))) return fail(TDP_EINVAL, "tdp_image_to_bf16: null pointer or n < 0");
    if (n == 0) return TDP_OK;
    image_to_bf16_kernel<<<ew_grid(n), 256, 0, stream>>>(img, n, out);
    return launch_status("tdp_image_to_bf16");
}

extern "C" int tdp_f32_to_bf16(const float* in, int64_t n, uint16_t* out, hipStream_t stream) {
    if (n < 0 || (n > 0 && (!in || !out))) return fail(TDP_EINVAL, "tdp_f32_to_bf16: null pointer or n < 0");
    if (n == 0) return TDP_OK;
    f32_to_bf16_kernel<<<ew_grid(n), 256, 0, stream>>>(in, n, out);
    return launch_status("tdp_f32_to_bf16");
}

// log2(c) when c is a power of two, else -1
static int log2_exact(int c) {
    int s = 0;
    while ((1 << s) < c) ++s;
    return (1 << s) == c ? s : -1;
}

static int conv_check(const char* fn, int B, int H, int W, int Cin, int Cout) {
    if (B < 0 || H < 3 || W < 3 || Cin < 1 || Cout < 1) return fail(TDP_EINVAL, "%s: bad shape", fn);
    if ((int64_t)B * H * W * std::max(Cin, Cout) >= (1ll << 40) || (int64_t)B * H * W >= (1ll << 31))
        return fail(TDP_EINVAL, "%s: tensor too large", fn);
    return TDP_OK;
}

extern "C" int tdp_conv3x3_fwd_bf16(const uint16_t* x, const uint16_t* w, const float* bias, int B, int H, int W,
                                    int Cin, int Cout, int relu, uint16_t* y, hipStream_t stream) {
    int rc = conv_check("tdp_conv3x3_fwd_bf16", B, H, W, Cin, Cout);
    if (rc) return rc;
    if (B > 0 && (!x || !w || !y)) return fail(TDP_EINVAL, "tdp_conv3x3_fwd_bf16: null pointer");
    if (!a16(x) || !a16(w)) return fail(TDP_EINVAL, "tdp_conv3x3_fwd_bf16: x and w must be 16-byte aligned");
    const int64_t M = (int64_t)B * (H - 2) * (W - 2);
    const int c1 = conv1_chunk_shift(Cin, Cout);
    if (c1 >= 0 && a16(y)) {
        if (M > 0) {
            const int grid = (int)std::min<int64_t>(ceil_div(M, 256), 64 * kCUs);
            conv1_fwd_kernel<<<grid, 256, 0, stream>>>(x, w, bias, H, W, Cout, relu, M, y);
        }
        return launch_status("tdp_conv3x3_fwd_bf16");
    }
    const int64_t x_bytes = (int64_t)B * H * W * Cin * 2;
    if (Cin == 32 && Cout % 16 == 0 && Cout <= 64 && a16(y) && x_bytes < (1ll << 31)) {
        if (M > 0) {
            // two workgroups of four waves per CU, each wave a contiguous range of 16-pixel blocks
            const int64_t nblk = ceil_div(M, 16);
            const int64_t waves = std::min<int64_t>(nblk, 2 * 4 * kCUs);
            const int64_t per_wave = ceil_div(nblk, waves);
            const unsigned grid = (unsigned)ceil_div(ceil_div(nblk, per_wave), 4);
            switch (Cout / 16) {
                case 1: conv_fwd_c32_kernel<1><<<grid, 256, 0, stream>>>(x, w, bias, H, W, relu, M, per_wave, x_bytes, y); break;
                case 2: conv_fwd_c32_kernel<2><<<grid, 256, 0, stream>>>(x, w, bias, H, W, relu, M, per_wave, x_bytes, y); break;
                case 3: conv_fwd_c32_kernel<3><<<grid, 256, 0, stream>>>(x, w, bias, H, W, relu, M, per_wave, x_bytes, y); break;
                default: conv_fwd_c32_kernel<4><<<grid, 256, 0, stream>>>(x, w, bias, H, W, relu, M, per_wave, x_bytes, y); break;
            }
        }
        return launch_status("tdp_conv3x3_fwd_bf16");
    }
    ConvFwdOp op{x, w, bias, y, H, W, Cin, H - 2, W - 2, relu, M, 9ll * Cin, 0, Cout, log2_exact(Cin)};
    op.kchunk = full_chunk(op.K);
    return launch_gemm(op, stream, "tdp_conv3x3_fwd_bf16");
}

extern "C" int tdp_conv3x3_dgrad_bf16(const uint16_t* dy, const uint16_t* w, const uint16_t* mask_act, int B, int H,
                                      int W, int Cin, int Cout, uint16_t* dx, hipStream_t stream) {
    int rc = conv_check("tdp_conv3x3_dgrad_bf16", B, H, W, Cin, Cout);
    if (rc) return rc;
    if (B > 0 && (!dy || !w || !dx)) return fail(TDP_EINVAL, "tdp_conv3x3_dgrad_bf16: null pointer");
    if (!a16(dy)) return fail(TDP_EINVAL, "tdp_conv3x3_dgrad_bf16: dy must be 16-byte aligned");
    const int64_t M = (int64_t)B * H * W;
    const int64_t dy_bytes = (int64_t)B * (H - 2) * (W - 2) * Cout * 2;
    if (Cout == kDgCout && (Cin == 16 || Cin == 32) && a16(w) && a16(dx) && (!mask_act || ((uintptr_t)mask_act & 7) == 0) &&
        dy_bytes < (1ll << 31) && M * Cin * 2 < (1ll << 31)) {
        if (M > 0) {
            // waves in groups of NJ = Cin / 16 share a contiguous range of 16-pixel blocks
            const int nj = Cin / 16;
            const int64_t nblk = ceil_div(M, 16);
            const int64_t ranges = std::min<int64_t>(nblk, 2 * 4 * kCUs / nj);
            const int64_t per_wave = ceil_div(nblk, ranges);
            const unsigned grid = (unsigned)ceil_div(ceil_div(nblk, per_wave) * nj, 4);
            if (Cin == 16)
                conv_dgrad_c64_kernel<1><<<grid, 256, 0, stream>>>(dy, w, mask_act, H, W, M, per_wave, dy_bytes, dx);
            else
                conv_dgrad_c64_kernel<2><<<grid, 256, 0, stream>>>(dy, w, mask_act, H, W, M, per_wave, dy_bytes, dx);
        }
        return launch_status("tdp_conv3x3_dgrad_bf16");
    }
    ConvDgradOp op{dy, w, mask_act, dx, H, W, Cout, H - 2, W - 2, M, 9ll * Cout, 0, Cin, log2_exact(Cout)};
    op.kchunk = full_chunk(op.K);
    return launch_gemm(op, stream, "tdp_conv3x3_dgrad_bf16");
}

extern "C" int tdp_conv3x3_wgrad_bf16(const uint16_t* x, const uint16_t* dy, int B, int H, int W, int Cin, int Cout,
                                      float* dw, float* db, hipStream_t stream) {
    int rc = conv_check("tdp_conv3x3_wgrad_bf16", B, H, W, Cin, Cout);
    if (rc) return rc;
    if (!dw || (B > 0 && (!x || !dy))) return fail(TDP_EINVAL, "tdp_conv3x3_wgrad_bf16: null pointer");
    if (!a16(dy) || ((Cin & 7) == 0 && !a16(x))) return fail(TDP_EINVAL, "tdp_conv3x3_wgrad_bf16: x, dy not 16-byte aligned");
    if ((rc = zero_grads(dw, (int64_t)Cout * 9 * Cin, db, Cout, stream))) return rc;
    const int64_t M = (int64_t)B * (H - 2) * (W - 2);
    const int c1 = conv1_chunk_shift(Cin, Cout);
    if (c1 >= 0) {
        if (M > 0) {
            // at most 96 workgroups of 1024 threads, at least 1024 pixels each
            const int64_t wgs = std::max<int64_t>(1, std::min<int64_t>(ceil_div(M, 1024), 96));
            const int64_t per_wg = ceil_div(M, wgs);
            conv1_wgrad_kernel<<<(unsigned)ceil_div(M, per_wg), kC1WgThreads, 0, stream>>>(x, dy, H, W, Cout, c1, M,
                                                                                            per_wg, dw, db);
        }
        return launch_status("tdp_conv3x3_wgrad_bf16");
    }
    ConvWgradOp op{x, dy, dw, H, W, Cin, H - 2, W - 2, Cout, M, 0, 9 * Cin};
    op.kchunk = split_chunk(op.K, ceil_div(op.M, kT) * ceil_div(op.N, kT));
    return launch_gemm(op, stream, "tdp_conv3x3_wgrad_bf16", db);
}

extern "C" int tdp_linear_fwd_bf16(const uint16_t* x, const uint16_t* w, const float* bias, int M, int N, int K,
                                   int relu, uint16_t* y_bf16, float* y_f32, hipStream_t stream) {
    if (M < 0 || N < 1 || K < 1) return fail(TDP_EINVAL, "tdp_linear_fwd_bf16: bad shape");
    if (M > 0 && (!x || !w || (!y_bf16 && !y_f32))) return fail(TDP_EINVAL, "tdp_linear_fwd_bf16: null pointer");
    if (!a16(x) || !a16(w)) return fail(TDP_EINVAL, "tdp_linear_fwd_bf16: x and w must be 16-byte aligned");
    if (y_bf16 && y_f32 && M > 0) {
        // split K so that about 2 * 256 workgroups run; y_f32 accumulates
        const int64_t tiles = ceil_div(M, kT) * ceil_div(N, kT);
        const int64_t steps = ceil_div(K, kStep);
        const int64_t splits = std::max<int64_t>(1, std::min<int64_t>(steps, ceil_div(2 * kCUs, tiles)));
        LinFwdAccOp op{x, w, y_f32, M, K, ceil_div(steps, splits) * kStep, N};
        int rc = zero_f32(y_f32, (int64_t)M * N, stream);
        if (rc) return rc;
        if ((rc = launch_gemm(op, stream, "tdp_linear_fwd_bf16"))) return rc;
        linear_epilogue_kernel<<<ew_grid((int64_t)M * N), 256, 0, stream>>>(y_f32, bias, M, N, relu, y_bf16);
        return launch_status("tdp_linear_fwd_bf16");
    }
    LinFwdOp op{x, w, bias, y_bf16, y_f32, relu, M, K, 0, N};
    op.kchunk = full_chunk(op.K);
    return launch_gemm(op, stream, "tdp_linear_fwd_bf16");
}

extern "C" int tdp_linear_dgrad_bf16(const uint16_t* dy, const uint16_t* w, const uint16_t* mask_act, int M, int N,
                                     int K, uint16_t* dx, hipStream_t stream) {
    if (M < 0 || N < 1 || K < 1) return fail(TDP_EINVAL, "tdp_linear_dgrad_bf16: bad shape");
    if (M > 0 && (!dy || !w || !dx)) return fail(TDP_EINVAL, "tdp_linear_dgrad_bf16: null pointer");
    if (!a16(dy)) return fail(TDP_EINVAL, "tdp_linear_dgrad_bf16: dy must be 16-byte aligned");
    LinDgradOp op{dy, w, mask_act, dx, M, N, 0, K};
    op.kchunk = full_chunk(op.K);
    return launch_gemm(op, stream, "tdp_linear_dgrad_bf16");
}

extern "C" int tdp_linear_wgrad_bf16(const uint16_t* x, const uint16_t* dy, int M, int N, int K, float* dw, float* db,
                                     hipStream_t stream) {
    if (M < 0 || N < 1 || K < 1) return fail(TDP_EINVAL, "tdp_linear_wgrad_bf16: bad shape");
    if (!dw || (M > 0 && (!x || !dy))) return fail(TDP_EINVAL, "tdp_linear_wgrad_bf16: null pointer");
    if (!a16(dy) || !a16(x)) return fail(TDP_EINVAL, "tdp_linear_wgrad_bf16: x, dy not 16-byte aligned");
    LinWgradOp op{x, dy, dw, N, M, 0, K};
    op.kchunk = split_chunk(op.K, ceil_div(op.M, kT) * ceil_div(op.N, kT));
    int rc = zero_grads(dw, (int64_t)N * K, db, N, stream);
    if (rc) return rc;
    return launch_gemm(op, stream, "tdp_linear_wgrad_bf16", db);
}

extern "C" int tdp_maxpool2_fwd_bf16(const uint16_t* x, int B, int H, int W, int C, uint16_t* y, hipStream_t stream) {
    if (B < 0 || H < 2 || W < 2 || C < 1 || (H & 1) || (W & 1)) return fail(TDP_EINVAL, "tdp_maxpool2_fwd_bf16: bad shape");
    if (B > 0 && (!x || !y)) return fail(TDP_EINVAL, "tdp_maxpool2_fwd_bf16: null pointer");
    const int64_t n = (int64_t)B * (H / 2) * (W / 2) * C;
    if (n > 0 && C % 8 == 0 && a16(x) && a16(y))
        maxpool2_fwd8_kernel<<<ew_grid(n / 8), 256, 0, stream>>>(x, B, H, W, C, y);
    else if (n > 0)
        maxpool2_fwd_kernel<<<ew_grid(n), 256, 0, stream>>>(x, B, H, W, C, y);
    return launch_status("tdp_maxpool2_fwd_bf16");
}

extern "C" int tdp_maxpool2_bwd_bf16(const uint16_t* x, const uint16_t* dy, int B, int H, int W, int C, int relu_mask,
                                     uint16_t* dx, hipStream_t stream) {
    if (B < 0 || H < 2 || W < 2 || C < 1 || (H & 1) || (W & 1)) return fail(TDP_EINVAL, "tdp_maxpool2_bwd_bf16: bad shape");
    if (B > 0 && (!x || !dy || !dx)) return fail(TDP_EINVAL, "tdp_maxpool2_bwd_bf16: null pointer");
    const int64_t n = (int64_t)B * (H / 2) * (W / 2) * C;
    if (n > 0 && C % 8 == 0 && a16(x) && a16(dy) && a16(dx))
        maxpool2_bwd8_kernel<<<ew_grid(n / 8), 256, 0, stream>>>(x, dy, B, H, W, C, relu_mask, dx);
    else if (n > 0)
        maxpool2_bwd_kernel<<<ew_grid(n), 256, 0, stream>>>(x, dy, B, H, W, C, relu_mask, dx);
    return launch_status("tdp_maxpool2_bwd_bf16");
}

extern "C" int tdp_softmax_expect_fwd(const float* logits, int M, int K, float* p, float* e, hipStream_t stream) {
    if (M < 0 || K < 1 || K > 64 || (M > 0 && (!logits || !p))) return fail(TDP_EINVAL, "tdp_softmax_expect_fwd: bad arguments");
    if (M > 0) softmax_expect_kernel<<<(unsigned)ceil_div(M, 256), 256, 0, stream>>>(logits, M, K, p, e);
    return launch_status("tdp_softmax_expect_fwd");
}

extern "C" int tdp_softmax_expect_bwd(const float* p, const float* dE, int M, int K, float* dlogits,
                                      uint16_t* dlogits_bf16, hipStream_t stream) {
    if (M < 0 || K < 1 || K > 64 || (M > 0 && (!p || !dE || (!dlogits && !dlogits_bf16))))
        return fail(TDP_EINVAL, "tdp_softmax_expect_bwd: bad arguments");
    if (M > 0) softmax_expect_bwd_kernel<<<(unsigned)ceil_div(M, 256), 256, 0, stream>>>(p, dE, M, K, dlogits, dlogits_bf16);
    return launch_status("tdp_softmax_expect_bwd");
}

extern "C" int tdp_softmax_bwd(const float* p, const float* dP, int M, int K, float* dlogits, uint16_t* dlogits_bf16,
                               hipStream_t stream) {
    if (M < 0 || K < 1 || K > 64 || (M > 0 && (!p || !dP || (!dlogits && !dlogits_bf16))))
        return fail(TDP_EINVAL, "tdp_softmax_bwd: bad arguments");
    if (M > 0) softmax_bwd_kernel<<<(unsigned)ceil_div(M, 256), 256, 0, stream>>>(p, dP, M, K, dlogits, dlogits_bf16);
    return launch_status("tdp_softmax_bwd");
}

extern "C" int tdp_argmax_rows(const float* p, int M, int K, int8_t* out, hipStream_t stream) {
    if (M < 0 || K < 1 || K > 127 || (M > 0 && (!p || !out))) return fail(TDP_EINVAL, "tdp_argmax_rows: bad arguments");
    if (M > 0) argmax_kernel<<<(unsigned)ceil_div(M, 256), 256, 0, stream>>>(p, M, K, out);
    return launch_status("tdp_argmax_rows");
}

extern "C" int tdp_adam_step(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                             float eps, int step, uint16_t* p_bf16, hipStream_t stream) {
    if (n < 0 || step < 1 || (n > 0 && (!p || !g || !m || !v))) return fail(TDP_EINVAL, "tdp_adam_step: bad arguments");
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    if (n > 0) adam_kernel<<<ew_grid(n), 256, 0, stream>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2, p_bf16);
    return launch_status("tdp_adam_step");
}

extern "C" int tdp_adam_step_multi(const tdp_adam_tensor* tensors, int32_t count, float lr, float b1, float b2,
                                   float eps, int step, hipStream_t stream) {
    if (count < 0 || count > kAdamMaxTensors || step < 1 || (count > 0 && !tensors))
        return fail(TDP_EINVAL, "tdp_adam_step_multi: count=%d (at most %d) or step < 1", count, kAdamMaxTensors);
    AdamList L{};
    int64_t most = 0;
    for (int k = 0; k < count; ++k) {
        const tdp_adam_tensor& a = tensors[k];
        if (a.n < 0 || (a.n > 0 && (!a.p || !a.g || !a.m || !a.v)))
            return fail(TDP_EINVAL, "tdp_adam_step_multi: tensor %d: bad arguments", k);
        L.t[k] = a;
        most = std::max(most, a.n);
    }
    if (count == 0 || most == 0) return TDP_OK;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    adam_multi_kernel<<<dim3((unsigned)ew_grid(most), (unsigned)count), 256, 0, stream>>>(L, lr, b1, b2, eps, c1, c2);
    return launch_status("tdp_adam_step_multi");
}
