// Kernel-variant choice and the nnls_solve_batch entry point (Algorithm 3 on
// a batch of independent NQPs sharing one Hessian).
#include <math.h>

#include "nmf_internal.h"

namespace nmfi {

// E for L lanes per column: the smallest compiled E with E * L >= r, else 0.
static int pick_e(int L, int r) {
    int n = 0;
    const int *t = nqp_e_table(L, &n);
    for (int i = 0; i < n; i++)
        if (t[i] * L >= r) return t[i];
    return 0;
}

bool nqp_lanes_ok(int r, int lanes) { return pick_e(lanes, r) != 0; }

// Lanes a launch should keep busy before widening stops paying: two waves on
// each SIMD of a 256-CU chip.  A fixed constant (not the device's CU count),
// so that the choice, and with it the rounding of every result, is the same
// on every device.
constexpr int64_t kLaneTarget = 256LL * 4 * 64 * 2;

NqpVariant nqp_pick(int r, int64_t ncols, int lanes) {
    if (lanes > 0) {
        const int e = pick_e(lanes, r);
        return {e, e ? lanes : 0};
    }
    // throughput layout: one lane per column up to r = 32, two up to 64, four
    // up to 128 (E <= 32 registers-worth of coordinates per lane)
    int L = r <= 32 ? 1 : (r <= 64 ? 2 : 4);
    // few columns: widen the lane groups (shorter per-column critical path)
    // while the launch stays under the lane target, each lane keeps more than
    // one real coordinate and the padded rank grows by at most a quarter
    while (L < 16 && ncols * L < kLaneTarget && (r + L - 1) / L > 1) {
        const int e2 = pick_e(2 * L, r);
        if (!e2 || 4 * (e2 * 2 * L) > 5 * (pick_e(L, r) * L)) break;
        L *= 2;
    }
    return {pick_e(L, r), L};
}

hipError_t launch_nqp(const NqpVariant &v, const NqpParams &p, hipStream_t s) {
    switch (v.L) {
    case 1: return launch_nqp_l1(v.E, p, s);
    case 2: return launch_nqp_l2(v.E, p, s);
    case 4: return launch_nqp_l4(v.E, p, s);
    case 8: return launch_nqp_l8(v.E, p, s);
    case 16: return launch_nqp_l16(v.E, p, s);
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
    if (o->lanes != 0 && o->lanes != 1 && o->lanes != 2 && o->lanes != 4 && o->lanes != 8 && o->lanes != 16)
        return fail(NMF_E_INVAL, "lanes must be 0, 1, 2, 4, 8 or 16 (got %d)", o->lanes);
    return NMF_OK;
}

}  // namespace nmfi

using namespace nmfi;

extern "C" int nnls_layout(int32_t r, int64_t ncols, int32_t lanes, int32_t *E, int32_t *L) {
    if (!E || !L) return fail(NMF_E_INVAL, "E and L must be non-NULL");
    if (r < 1 || r > NMF_MAX_RANK) return fail(NMF_E_INVAL, "r must be in [1, %d] (got %d)", NMF_MAX_RANK, r);
    if (ncols < 0) return fail(NMF_E_INVAL, "ncols must be >= 0");
    if (lanes != 0 && lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8 && lanes != 16)
        return fail(NMF_E_INVAL, "lanes must be 0, 1, 2, 4, 8 or 16 (got %d)", lanes);
    const NqpVariant v = nqp_pick(r, ncols, lanes);
    if (!v.E) return fail(NMF_E_INVAL, "lanes = %d cannot hold rank %d", lanes, r);
    *E = v.E;
    *L = v.L;
    return NMF_OK;
}

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
    const NqpVariant v = nqp_pick(r, ncols, opt->lanes);
    if (!v.E) return fail(NMF_E_INVAL, "lanes = %d cannot hold rank %d", opt->lanes, r);
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
