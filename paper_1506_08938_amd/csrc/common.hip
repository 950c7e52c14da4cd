// Error plumbing, device queries and small utility kernels.
#include <stdarg.h>
#include <stdio.h>

#include "nmf_internal.h"

namespace nmfi {

static thread_local std::string g_last_error = "no error";

void set_error(int status, const std::string &msg) {
    (void)status;
    g_last_error = msg;
}

int fail(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    set_error(status, buf);
    return status;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? NMF_E_NOMEM : NMF_E_DEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

int device_cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
        return 256;
    return n;
}

}  // namespace nmfi

extern "C" const char *nmf_last_error(void) { return nmfi::g_last_error.c_str(); }

extern "C" void nmf_default_opts(nmf_opts *o) {
    if (!o) return;
    o->max_outer = 50;
    o->max_inner = 100;
    o->eps = 1e-3;
    o->ls_guard = 1;
    o->precision = NMF_FP32;
    o->objective_every = 0;
    o->check_finite = 0;
    o->lanes = 0;
    o->fast_break_cols = 0;
}

namespace nmfi {

// flag bit 0: a NaN/Inf was seen; bit 1: a negative value was seen.
__global__ void k_check_values(const float *__restrict__ x, int64_t n, int *flag) {
    int f = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float v = x[i];
        if (!isfinite(v)) f |= 1;
        if (v < 0.f) f |= 2;
    }
    if (f) atomicOr(flag, f);
}

int check_values(const float *x, int64_t n, int nonneg, hipStream_t s) {
    if (n <= 0) return NMF_OK;
    int *dflag = nullptr;
    NMF_HIP(hipMallocAsync((void **)&dflag, sizeof(int), s));
    int host = 0;
    hipError_t e = hipMemsetAsync(dflag, 0, sizeof(int), s);
    if (e == hipSuccess) {
        int64_t blocks = (n + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(k_check_values, dim3((unsigned)blocks), dim3(256), 0, s, x, n, dflag);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&host, dflag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFreeAsync(dflag, s);
    if (e != hipSuccess) return hip_fail(e, "check_values");
    if (host & 1) return fail(NMF_E_NONFINITE, "input holds NaN or Inf");
    if (nonneg && (host & 2)) return fail(NMF_E_NONFINITE, "input holds negative values");
    return NMF_OK;
}

}  // namespace nmfi

namespace nmfi {

// graph-safe zero fill (no memset node)
__global__ void k_zero_u64(unsigned long long *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace nmfi

namespace nmfi {

__global__ void k_zero_u32(unsigned int *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

hipError_t launch_zero_u32(unsigned int *p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace nmfi
