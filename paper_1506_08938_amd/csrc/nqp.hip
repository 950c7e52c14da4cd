// Kernel-variant choice and the nnls_solve_batch entry point (Algorithm 3 on
// a batch of independent NQPs sharing one Hessian).
#include <math.h>

#include "nmf_internal.h"

namespace nmfi {

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
    unsigned long long *counter = nullptr;
    NMF_HIP(hipMallocAsync((void **)&counter, 256, s));
    hipError_t e = launch_zero_u64(counter, 1, s);
    if (e == hipSuccess) {
        NqpParams p{};
        p.gram = gram; p.P = h; p.hsign = 1.f; p.hadd = 0.f; p.X = X;
        p.ncols = ncols; p.r = r; p.ldp = r; p.ldx = r;
        p.max_inner = opt->max_inner; p.eps = opt->eps; p.ls_guard = opt->ls_guard ? 1 : 0;
        p.cold = 0; p.iters = iters; p.counter = counter; p.inner_total = nullptr;
        e = launch_nqp(v, p, s);
    }
    hipError_t e2 = hipFreeAsync(counter, s);
    if (e != hipSuccess) return hip_fail(e, "nnls_solve_batch launch");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
    return NMF_OK;
}
