// Kernel-variant choice and the nnls_solve_batch entry point (Algorithm 3 on
// a batch of independent NQPs sharing one Hessian).
#include <math.h>

#include "nmf_internal.h"
#include "nqp_tuned.h"

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

NqpVariant nqp_pick(int r, int64_t ncols, int lanes) {
    if (lanes > 0) {
        const int e = pick_e(lanes, r);
        return {e, e ? lanes : 0};
    }
    // the autotuned table: the grid rank at or above r, the grid launch size
    // at or below ncols.  A fixed function of (r, ncols), so the layout, and
    // with it the rounding of every result, never depends on timing.
    constexpr int nr = (int)(sizeof kTunedRanks / sizeof(int));
    constexpr int nc = (int)(sizeof kTunedCols / sizeof(long long));
    int ri = 0;
    while (ri < nr - 1 && kTunedRanks[ri] < r) ri++;
    int ci = 0;
    while (ci < nc - 1 && kTunedCols[ci + 1] <= ncols) ci++;
    int L = kTunedLanes[ri][ci];
    // no more lanes than coordinates (the grid rank can be above r) ...
    while (L > 1 && L / 2 >= r) L /= 2;
    // ... and a layout that holds r
    while (L < 16 && !pick_e(L, r)) L *= 2;
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
    if (o->fast_break_cols < 0 || o->fast_break_cols > (1 << 20))
        return fail(NMF_E_INVAL, "fast_break_cols must be in [0, 2^20] (got %d)", o->fast_break_cols);
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
        p.unit = opt->fast_break_cols;
        e = launch_nqp(v, p, s);
    }
    hipError_t e2 = hipFreeAsync(counter, s);
    if (e != hipSuccess) return hip_fail(e, "nnls_solve_batch launch");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
    return NMF_OK;
}
