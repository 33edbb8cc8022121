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

// Stage timer: while a stage is selected, each launch of that stage records
// a pair of events around it on its own stream (at most kTimerPairs pairs
// until the next selection).
static constexpr int kTimerPairs = 256;
static int g_timer_stage = 0;
static int g_timer_used = 0;
static hipEvent_t g_timer_ev[kTimerPairs][2];
static bool g_timer_made = false;

void stage_mark(int stage, int edge, hipStream_t s) {
    if (g_timer_stage == 0 || stage != g_timer_stage || g_timer_used >= kTimerPairs) return;
    if (hipEventRecord(g_timer_ev[g_timer_used][edge], s) != hipSuccess) return;
    if (edge == 1) ++g_timer_used;
}

}  // namespace tdp

extern "C" int tdp_stage_timer(int stage) {
    using namespace tdp;
    if (stage < 0 || stage > TDP_STAGE_FUSED_PROBE) return fail(TDP_EINVAL, "tdp_stage_timer: stage %d", stage);
    if (!g_timer_made) {
        for (int i = 0; i < kTimerPairs; ++i)
            for (int j = 0; j < 2; ++j)
                if (hipEventCreate(&g_timer_ev[i][j]) != hipSuccess)
                    return fail(TDP_EDEVICE, "tdp_stage_timer: hipEventCreate failed");
        g_timer_made = true;
    }
    g_timer_stage = stage;
    g_timer_used = 0;
    return TDP_OK;
}

extern "C" int tdp_stage_time(double* total_ms, int64_t* launches) {
    using namespace tdp;
    if (!total_ms || !launches) return fail(TDP_EINVAL, "tdp_stage_time: null output");
    double t = 0.0;
    for (int i = 0; i < g_timer_used; ++i) {
        if (hipEventSynchronize(g_timer_ev[i][1]) != hipSuccess) return fail(TDP_EDEVICE, "tdp_stage_time: sync failed");
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, g_timer_ev[i][0], g_timer_ev[i][1]) != hipSuccess)
            return fail(TDP_EDEVICE, "tdp_stage_time: elapsed time failed");
        t += ms;
    }
    *total_ms = t;
    *launches = g_timer_used;
    return TDP_OK;
}

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
