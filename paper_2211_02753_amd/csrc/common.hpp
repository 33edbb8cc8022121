// Shared host and device helpers of the gfx950 operator library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/tdp.h"

namespace tdp {

// ----------------------------------------------------------------- host side

// Record an error message for tdp_last_error() and return `code`.
int fail(int code, const char* fmt, ...);
// The same for TDP_ECAPACITY / TDP_EWORKSPACE, recording the size the call
// needed (elements or bytes) for tdp_last_needed().
int fail_need(int code, int64_t needed, const char* fmt, ...);
// Records the selected stage timer's event (edge 0 before, 1 after a launch).
void stage_mark(int stage, int edge, hipStream_t s);
// Check the launch status of the kernels just enqueued.
int launch_status(const char* what);

// Bump allocator over the caller's workspace (256-byte aligned pieces).
struct WsAlloc {
    uintptr_t base;
    size_t used = 0;
    explicit WsAlloc(void* p) : base((uintptr_t)p) {}
    template <typename T>
    T* take(size_t count) {
        size_t off = (used + 255) & ~(size_t)255;
        used = off + count * sizeof(T);
        return base ? (T*)(base + off) : nullptr;
    }
    size_t bytes() const { return (used + 255) & ~(size_t)255; }
};

inline int dtype_size(int dt) {
    switch (dt) {
        case TDP_I8: return 1;
        case TDP_I32: return 4;
        case TDP_I64: return 8;
        case TDP_F32: return 4;
    }
    return 0;
}
inline bool int_dtype(int dt) { return dt == TDP_I8 || dt == TDP_I32 || dt == TDP_I64; }

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr int kCUs = 256;  // compute units of an MI355X (8 XCDs x 32)

// ---------------------------------------------------------------- device side

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Workgroup barrier ordering LDS accesses only: global loads and stores in
// flight stay in flight across it (a full __syncthreads() first waits for
// every outstanding global access of the wave, prefetches included).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Number of set bits of `mask` held by lanes below this one.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
    long long s = (long long)v;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
    return (uint64_t)s;
}

// LDS written by some lanes of a wave, then read by others of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive prefix (over lanes) and total of small per-lane counts c < 2^BITS,
// from one ballot per bit.
template <int BITS>
__device__ __forceinline__ void wave_count_scan(uint32_t c, uint32_t& prefix, uint32_t& total) {
    prefix = 0;
    total = 0;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        uint64_t m = ballot((c >> b) & 1u);
        prefix += lanes_below(m) << b;
        total += (uint32_t)__popcll(m) << b;
    }
}

__device__ __forceinline__ bool cmp_i64(int64_t a, int cmp, int64_t b) {
    switch (cmp) {
        case TDP_LT: return a < b;
        case TDP_LE: return a <= b;
        case TDP_GT: return a > b;
        case TDP_GE: return a >= b;
        case TDP_EQ: return a == b;
        default: return a != b;
    }
}

__device__ __forceinline__ int64_t load_int(const void* p, int dt, int64_t i) {
    if (dt == TDP_I32) return ((const int32_t*)p)[i];
    if (dt == TDP_I64) return ((const int64_t*)p)[i];
    return ((const int8_t*)p)[i];
}

// Four consecutive values starting at row r0 (a multiple of 4), widened to
// int64; rows at or beyond n read as 0.  Full groups use one 4-, 16- or
// 2x16-byte load.
__device__ __forceinline__ void load4_int(const void* p, int dt, int64_t r0, int64_t n, int64_t v[4]) {
    if (r0 + 4 <= n) {
        if (dt == TDP_I32) {
            int4 q = *(const int4*)((const int32_t*)p + r0);
            v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else if (dt == TDP_I64) {
            longlong2 a = *(const longlong2*)((const int64_t*)p + r0);
            longlong2 b = *(const longlong2*)((const int64_t*)p + r0 + 2);
            v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
        } else {
            char4 q = *(const char4*)((const int8_t*)p + r0);
            v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (r0 + e < n) ? load_int(p, dt, r0 + e) : 0;
    }
}

// murmur3's 32-bit finaliser: a bijection on 32 bits with full avalanche.
__device__ __forceinline__ uint32_t hash32(uint32_t k) {
    k ^= k >> 16;
    k *= 0x85EBCA6Bu;
    k ^= k >> 13;
    k *= 0xC2B2AE35u;
    k ^= k >> 16;
    return k;
}

__device__ __forceinline__ void raise_flag(int32_t* status, int flag) {
    if (status) atomicOr(status, flag);
}

__device__ __forceinline__ uint64_t load_acquire_u64(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Fill helpers (used instead of memset so that callers may capture calls
// into graphs).
__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n);
__global__ void fill_u64_kernel(uint64_t* p, uint64_t v, int64_t n);
int fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
int fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s);

}  // namespace tdp
