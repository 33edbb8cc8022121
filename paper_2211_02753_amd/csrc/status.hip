// Status codes, per-thread error text and fill kernels.
#include <stdarg.h>
#include <stdio.h>

#include "common.hpp"

namespace tdp {

static thread_local char g_last_error[512] = "";
static thread_local int64_t g_last_needed = 0;

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    g_last_needed = 0;
    return code;
}

int fail_need(int code, int64_t needed, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    g_last_needed = needed;
    return code;
}

int launch_status(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(TDP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return TDP_OK;
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; i < n; i += stride) {
        if (i + 4 <= n && ((uintptr_t)(p + i) & 15) == 0) {
            *(uint4*)(p + i) = make_uint4(v, v, v, v);
        } else {
            for (int64_t j = i; j < n && j < i + 4; ++j) p[j] = v;
        }
    }
}

__global__ void fill_u64_kernel(uint64_t* p, uint64_t v, int64_t n) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

static int fill_grid(int64_t work) {
    int64_t b = ceil_div(work, 256);
    if (b < 1) b = 1;
    if (b > 4 * kCUs * 4) b = 4 * kCUs * 4;
    return (int)b;
}

int fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return TDP_OK;
    fill_u32_kernel<<<fill_grid(ceil_div(n, 4)), 256, 0, s>>>(p, v, n);
    return launch_status("fill_u32");
}

int fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return TDP_OK;
    fill_u64_kernel<<<fill_grid(n), 256, 0, s>>>(p, v, n);
    return launch_status("fill_u64");
}

}  // namespace tdp

extern "C" const char* tdp_status_string(int status) {
    switch (status) {
        case TDP_OK: return "ok";
        case TDP_EINVAL: return "invalid argument";
        case TDP_ECAPACITY: return "output capacity too small";
        case TDP_EWORKSPACE: return "workspace too small";
        case TDP_EUNSUPPORTED: return "unsupported combination";
        case TDP_EDEVICE: return "HIP runtime error";
    }
    return "unknown status";
}

extern "C" const char* tdp_last_error(void) { return tdp::g_last_error; }

extern "C" int64_t tdp_last_needed(void) { return tdp::g_last_needed; }
