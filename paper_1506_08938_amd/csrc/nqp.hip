// Anti-lopsided rescale (Algorithm 3, "Re-scaling variables") and the
// nnls_solve_batch entry point (Algorithm 3 on a batch of independent NQPs).
#include <math.h>

#include "nmf_internal.h"

namespace nmfi {

// One block.  dsq_i = sqrt(Gamma_ii) (0 when Gamma_ii <= 0: frozen; 0 for the
// pad coordinates r <= i < R).  Q_ij = Gamma_ij / (dsq_i dsq_j), Q_ii = 1, and
// the row/column of a frozen or pad coordinate is zero off the diagonal.
// Also zeroes the solve kernel's work counter, so that a solve launched after
// it on the same stream starts from column 0 (no memset node is needed).
__global__ __launch_bounds__(256) void k_rescale(const float *__restrict__ gram, int r, int R,
                                                 float *__restrict__ Q, float *__restrict__ dsq,
                                                 unsigned long long *counter) {
    __shared__ float sd[NMF_MAX_RANK];
    for (int i = threadIdx.x; i < R; i += blockDim.x) {
        const float d = i < r ? gram[(size_t)i * r + i] : 0.f;
        sd[i] = d > 0.f ? sqrtf(d) : 0.f;
        dsq[i] = sd[i];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < R * R; t += blockDim.x) {
        const int i = t / R, j = t - (t / R) * R;
        float v;
        if (i == j) v = 1.f;
        else if (i >= r || j >= r || sd[i] == 0.f || sd[j] == 0.f) v = 0.f;
        else v = gram[(size_t)i * r + j] / (sd[i] * sd[j]);
        Q[t] = v;
    }
    if (threadIdx.x == 0 && counter) *counter = 0ull;
}

hipError_t launch_rescale(const float *gram, int r, int R, float *Q, float *dsq,
                          unsigned long long *counter, hipStream_t s) {
    hipLaunchKernelGGL(k_rescale, dim3(1), dim3(256), 0, s, gram, r, R, Q, dsq, counter);
    return hipGetLastError();
}

// Kernel variant per rank: one lane per column up to r = 32, two up to 64,
// four up to 128; E is the smallest instantiated size that covers r.
static const int kE1[] = {1, 2, 4, 6, 8, 12, 16, 20, 24, 28, 32};
static const int kE2[] = {20, 24, 28, 32};
static const int kE4[] = {18, 20, 22, 24, 25, 26, 28, 30, 32};

NqpVariant nqp_pick(int r) {
    if (r <= 32) {
        for (int e : kE1) if (e >= r) return {e, 1};
    } else if (r <= 64) {
        for (int e : kE2) if (2 * e >= r) return {e, 2};
    } else {
        for (int e : kE4) if (4 * e >= r) return {e, 4};
    }
    return {0, 0};
}

int nqp_padded(int r) {
    NqpVariant v = nqp_pick(r);
    return v.E * v.L;
}

hipError_t launch_nqp(const NqpVariant &v, const NqpParams &p, hipStream_t s) {
    switch (v.L) {
    case 1: return launch_nqp_l1(v.E, p, s);
    case 2: return launch_nqp_l2(v.E, p, s);
    case 4: return launch_nqp_l4(v.E, p, s);
    default: return hipErrorInvalidValue;
    }
}

int validate_opts(const nmf_opts *o) {
    if (!o) return fail(NMF_E_INVAL, "opts is NULL");
    if (o->max_inner < 1) return fail(NMF_E_INVAL, "max_inner must be >= 1 (got %d)", o->max_inner);
    if (!(o->eps >= 0.0) || !isfinite(o->eps))
        return fail(NMF_E_INVAL, "eps must be finite and >= 0");
    if (o->precision != NMF_FP32 && o->precision != NMF_BF16)
        return fail(NMF_E_INVAL, "precision must be NMF_FP32 or NMF_BF16");
    return NMF_OK;
}

}  // namespace nmfi

using namespace nmfi;

extern "C" int nnls_solve_batch(int32_t r, int64_t ncols, const float *gram, const float *h,
                                float *X, const nmf_opts *opt, int32_t *iters, void *stream) {
    if (r < 1 || r > NMF_MAX_RANK) return fail(NMF_E_INVAL, "r must be in [1, %d] (got %d)", NMF_MAX_RANK, r);
    if (ncols < 0) return fail(NMF_E_INVAL, "ncols must be >= 0");
    if (int st = validate_opts(opt)) return st;
    if (ncols == 0) return NMF_OK;
    if (!gram || !h || !X) return fail(NMF_E_INVAL, "gram, h and X must be non-NULL device pointers");
    if (ncols > (int64_t)INT32_MAX * 2) return fail(NMF_E_INVAL, "ncols too large");
    hipStream_t s = (hipStream_t)stream;
    if (opt->check_finite) {
        int st = check_values(gram, (int64_t)r * r, 0, s);
        if (!st) st = check_values(h, ncols * r, 0, s);
        if (!st) st = check_values(X, ncols * r, 1, s);
        if (st) return st;
    }
    const NqpVariant v = nqp_pick(r);
    const int R = v.E * v.L;
    // workspace (every part 256-byte aligned): counter, dsq (R), Q (R*R)
    const size_t qbytes = (size_t)R * R * sizeof(float);
    char *ws = nullptr;
    NMF_HIP(hipMallocAsync((void **)&ws, 1024 + qbytes, s));
    unsigned long long *counter = (unsigned long long *)ws;
    float *dsq = (float *)(ws + 256);
    float *Q = (float *)(ws + 1024);
    hipError_t e = launch_rescale(gram, r, R, Q, dsq, counter, s);
    if (e == hipSuccess) {
        NqpParams p{};
        p.Q = Q; p.dsq = dsq; p.P = h; p.hsign = 1.f; p.hadd = 0.f; p.X = X;
        p.ncols = ncols; p.r = r; p.ldp = r; p.ldx = r;
        p.max_inner = opt->max_inner; p.eps = opt->eps; p.ls_guard = opt->ls_guard ? 1 : 0;
        p.cold = 0; p.iters = iters; p.counter = counter; p.inner_total = nullptr;
        e = launch_nqp(v, p, s);
    }
    hipError_t e2 = hipFreeAsync(ws, s);
    if (e != hipSuccess) return hip_fail(e, "nnls_solve_batch launch");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
    return NMF_OK;
}
