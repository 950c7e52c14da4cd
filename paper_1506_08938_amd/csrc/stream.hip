// Limited-internal-memory fit (Section 3.3, Algorithm 2; the memory row of
// Table 1).  V stays in host memory and every outer iteration reads it once,
// one panel of instances (columns of V) at a time.  The same single pass
// over a V already in device memory (nmf_fit_single_pass) takes each panel as
// a view of V: a panel's E-step product and its share of the M-step's product
// read the same m x panel block back to back, the second time from cache.  For a panel J the E-step
// solves the panel's columns of H against Q = W'W + 2 l2_h I, then adds the
// panel's share of the M-step's product, V_J Ht_J (the paper's sum of
// F_i V_i'), to P_W in panel order.  The M-step needs no V: its Gram
// Ht'Ht + 2 l2_w I comes from the resident Ht, and W <- NQP(Gram, -P_W +
// l1_w, W).
//
// Device memory: the caller's W (m x r) and Ht (n x r); P_W and a panel
// product (m x r each); two panel buffers (m x panel columns each: the copy
// of the next panel runs on a copy stream while the current one is worked
// on); the panel's product P_J and the Gram, product and statistics scratch.
//
// The objective, when due after iteration t, is summed panel by panel during
// the pass of iteration t + 1, before each panel's E-step changes its part of
// Ht (and its regularisation sums are taken before the pass); the one after
// the last iteration takes a pass of its own.
#include "nmf_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace nmfi {

__global__ void k_add_f32(float *__restrict__ y, const float *__restrict__ x, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += x[i];
}

__global__ void k_zero_f32(float *__restrict__ y, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = 0.f;
}

static unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

namespace {

struct Streamer {
    hipStream_t s = nullptr;   // the caller's stream: all compute
    hipStream_t cs = nullptr;  // host-to-device copies
    hipEvent_t copied[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr};
    float *buf[2] = {nullptr, nullptr};
    char *ws = nullptr;

    const float *Vh = nullptr;   // host V, or device V when resident
    bool resident = false;       // V in device memory: panels are views into it, no copies
    int64_t m = 0, n = 0, ld = 0, pc = 0, ldp = 0, np = 0;
    int64_t vld = 0;             // leading dimension of a panel as the kernels read it
    int r = 0;
    nmf_reg reg{};
    nmf_opts opt{};

    float *GW = nullptr, *GH = nullptr, *gram_scratch = nullptr, *PW = nullptr, *Ptmp = nullptr, *PJ = nullptr,
          *dense_scratch = nullptr;
    double *loss_scratch = nullptr, *loss_slots = nullptr, *kkt_slots = nullptr, *kkt_partial = nullptr;
    double *obj = nullptr;       // (max_outer + 1) x 2: loss, J after each iteration
    double *kkt_out = nullptr;   // 2: E-step (H), M-step (W) of the last iteration
    char *obj_scratch = nullptr;
    unsigned long long *counter = nullptr, *inner_total = nullptr;

    ~Streamer() {
        if (s) (void)hipStreamSynchronize(s);
        if (cs) (void)hipStreamSynchronize(cs);
        for (int b = 0; b < 2; b++) {
            if (buf[b]) (void)hipFree(buf[b]);
            if (copied[b]) (void)hipEventDestroy(copied[b]);
            if (freed[b]) (void)hipEventDestroy(freed[b]);
        }
        if (ws) (void)hipFree(ws);
        if (cs) (void)hipStreamDestroy(cs);
    }

    int64_t cols_of(int64_t p) const { return std::min(pc, n - p * pc); }

    // Runs body(p, j0, cols, V_J) for every panel on the compute stream; the
    // copy of panel p waits until the work on panel p - 2 (same buffer) is done.
    template <class F>
    int for_each_panel(F body) {
        if (resident) {
            for (int64_t p = 0; p < np; p++)
                if (int st = body(p, p * pc, cols_of(p), Vh + p * pc)) return st;
            return NMF_OK;
        }
        for (int64_t p = 0; p < np; p++) {
            const int b = (int)(p & 1);
            const int64_t j0 = p * pc, cols = cols_of(p);
            NMF_HIP(hipStreamWaitEvent(cs, freed[b], 0));
            NMF_HIP(hipMemcpy2DAsync(buf[b], (size_t)ldp * sizeof(float), Vh + j0, (size_t)ld * sizeof(float),
                                     (size_t)cols * sizeof(float), (size_t)m, hipMemcpyHostToDevice, cs));
            NMF_HIP(hipEventRecord(copied[b], cs));
            NMF_HIP(hipStreamWaitEvent(s, copied[b], 0));
            if (int st = body(p, j0, cols, (const float *)buf[b])) return st;
            NMF_HIP(hipEventRecord(freed[b], s));
        }
        return NMF_OK;
    }

    // Algorithm 3 on ncols NQPs sharing the Gram G (warm start from X);
    // the work counter must be zero (launch_gram zeroes it, or zero = true)
    hipError_t solve(const float *G, const float *P, float l1, float *X, int64_t ncols, bool zero) {
        if (zero) {
            hipError_t e = launch_zero_u64(counter, 1, s);
            if (e != hipSuccess) return e;
        }
        NqpParams q{};
        q.gram = G; q.P = P; q.hsign = -1.f; q.hadd = l1; q.X = X;
        q.ncols = ncols; q.r = r; q.ldp = r; q.ldx = r;
        q.max_inner = opt.max_inner; q.eps = opt.eps; q.ls_guard = opt.ls_guard ? 1 : 0;
        q.cold = 0; q.iters = nullptr; q.counter = counter; q.inner_total = inner_total;
        q.unit = opt.fast_break_cols;
        return launch_nqp(nqp_pick(r, ncols, opt.lanes), q, s);
    }
};

}  // namespace

}  // namespace nmfi

namespace nmfi {
namespace {
int run_panels(Streamer &S, float *W, float *Ht, double *trace, nmf_stats *stats);
}  // namespace
}  // namespace nmfi

using namespace nmfi;

extern "C" int nmf_fit_streamed(const float *V_host, int64_t m, int64_t n, int64_t ld, int32_t r,
                                const nmf_reg *reg, const nmf_opts *opt, int64_t panel_cols, float *W,
                                float *Ht, double *trace, nmf_stats *stats, void *stream) {
    if (!V_host) return fail(NMF_E_INVAL, "V_host is NULL");
    if (m < 1 || n < 1) return fail(NMF_E_INVAL, "V must be non-empty (m = %lld, n = %lld)", (long long)m, (long long)n);
    if (ld < n) return fail(NMF_E_INVAL, "ld (%lld) must be >= n (%lld)", (long long)ld, (long long)n);
    if (r < 1 || r > NMF_MAX_RANK) return fail(NMF_E_INVAL, "r must be in [1, %d] (got %d)", NMF_MAX_RANK, r);
    if (!reg) return fail(NMF_E_INVAL, "reg is NULL");
    if (int st = validate_opts(opt)) return st;
    if (opt->precision != NMF_FP32)
        return fail(NMF_E_UNSUPPORTED, "the streamed fit computes its products in FP32 only");
    const float regs[4] = {reg->l1_w, reg->l2_w, reg->l1_h, reg->l2_h};
    for (float v : regs)
        if (!(v >= 0.f) || !std::isfinite(v)) return fail(NMF_E_INVAL, "regularisation weights must be finite and >= 0");
    if (opt->max_outer < 0) return fail(NMF_E_INVAL, "max_outer must be >= 0");
    if (panel_cols < 1) return fail(NMF_E_INVAL, "panel_cols must be >= 1 (got %lld)", (long long)panel_cols);
    if (!W || !Ht) return fail(NMF_E_INVAL, "W and Ht must be non-NULL");
    if (!nqp_pick(r, 1, opt->lanes).E) return fail(NMF_E_INVAL, "lanes = %d cannot hold rank %d", opt->lanes, r);

    Streamer S;
    S.s = (hipStream_t)stream;
    S.Vh = V_host; S.m = m; S.n = n; S.ld = ld; S.r = r; S.reg = *reg; S.opt = *opt;
    S.pc = std::min(panel_cols, n);
    S.ldp = (S.pc + 3) / 4 * 4;  // 16-byte rows for the product's vector loads
    S.vld = S.ldp;
    S.np = (n + S.pc - 1) / S.pc;
    return run_panels(S, W, Ht, trace, stats);
}

namespace nmfi {
namespace {
// The outer iterations over the panels of S (set up by the caller), shared
// by the host-memory and the resident single-pass fits.
int run_panels(Streamer &S, float *W, float *Ht, double *trace, nmf_stats *stats) {
    const int64_t m = S.m, n = S.n;
    const int r = S.r;
    const nmf_opts *opt = &S.opt;
    const nmf_reg *reg = &S.reg;
    const int T = opt->max_outer;
    if (opt->check_finite) {
        if (int st = check_values(W, m * r, 1, S.s)) return st;
        if (int st = check_values(Ht, n * r, 1, S.s)) return st;
    }

    // ---------------------------------------------------------------- workspace
    const int64_t last = S.cols_of(S.np - 1);
    const size_t dsb = std::max(dense_scratch_bytes(m, S.pc, r), dense_scratch_bytes(m, last, r));
    size_t off = 0;
    auto place = [&](size_t bytes) { const size_t o = off; off += al256(bytes); return o; };
    const size_t o_gw = place((size_t)r * r * 4), o_gh = place((size_t)r * r * 4);
    const size_t o_gs = place(gram_scratch_bytes(r, std::max(m, n)));
    const size_t o_pw = place((size_t)m * r * 4), o_pt = place((size_t)m * r * 4);
    const size_t o_pj = place((size_t)S.pc * r * 4);
    const size_t o_ds = place(dsb);
    const size_t o_ls = place(loss_panel_scratch_bytes(m, S.pc));
    const size_t o_lsl = place((size_t)S.np * 8), o_ksl = place((size_t)S.np * 4 * 8);
    const size_t o_kp = place(kkt_partial_bytes(std::max(m, S.pc)));
    const size_t o_obj = place((size_t)(T + 1) * 2 * 8), o_ko = place(8 * 8);
    const size_t o_os = place(objective_slots_scratch_bytes());
    const size_t o_ctr = place(2 * 8);
    NMF_HIP(hipMalloc((void **)&S.ws, off));
    char *w = S.ws;
    S.GW = (float *)(w + o_gw); S.GH = (float *)(w + o_gh); S.gram_scratch = (float *)(w + o_gs);
    S.PW = (float *)(w + o_pw); S.Ptmp = (float *)(w + o_pt); S.PJ = (float *)(w + o_pj);
    S.dense_scratch = (float *)(w + o_ds); S.loss_scratch = (double *)(w + o_ls);
    S.loss_slots = (double *)(w + o_lsl); S.kkt_slots = (double *)(w + o_ksl); S.kkt_partial = (double *)(w + o_kp);
    S.obj = (double *)(w + o_obj); S.kkt_out = (double *)(w + o_ko); S.obj_scratch = w + o_os;
    S.counter = (unsigned long long *)(w + o_ctr); S.inner_total = S.counter + 1;
    if (!S.resident) {
        // panel buffers: the padding columns stay zero (copies write cols of ldp)
        for (int b = 0; b < 2; b++) {
            NMF_HIP(hipMalloc((void **)&S.buf[b], (size_t)m * S.ldp * sizeof(float)));
            NMF_HIP(hipMemsetAsync(S.buf[b], 0, (size_t)m * S.ldp * sizeof(float), S.s));
        }
        NMF_HIP(hipStreamCreateWithFlags(&S.cs, hipStreamNonBlocking));
        for (int b = 0; b < 2; b++) {
            NMF_HIP(hipEventCreateWithFlags(&S.copied[b], hipEventDisableTiming));
            NMF_HIP(hipEventCreateWithFlags(&S.freed[b], hipEventDisableTiming));
            NMF_HIP(hipEventRecord(S.freed[b], S.s));
        }
    }
    NMF_HIP(launch_zero_u64(S.inner_total, 1, S.s));

    const bool want_obj = trace || stats;
    const int every = opt->objective_every > 0 ? opt->objective_every : 1;
    // objective after iteration t (t = 0: the start point)
    auto due = [&](int t) {
        if (trace && (t == 0 || t % every == 0 || t == T)) return true;
        return stats != nullptr && t == T;
    };
    auto panel_loss = [&](int64_t p, int64_t j0, int64_t cols, const float *VJ) {
        return launch_loss_panel(VJ, S.vld, m, cols, W, Ht + j0 * r, r, S.loss_scratch, S.loss_slots + p, S.s);
    };

    // ---------------------------------------------------------------- outer iterations
    for (int t = 1; t <= T; t++) {
        const bool last = t == T;
        const bool obj_prev = want_obj && due(t - 1);
        NMF_HIP(launch_gram(W, m, r, reg->l2_h, NMF_FP32, S.GW, S.gram_scratch, S.s, nullptr));
        if (obj_prev) NMF_HIP(launch_objective_regs(W, m, Ht, n, r, S.obj_scratch, S.s));
        hipLaunchKernelGGL(k_zero_f32, dim3(grid_for(m * r)), dim3(256), 0, S.s, S.PW, m * r);
        NMF_HIP(hipGetLastError());
        int st = S.for_each_panel([&](int64_t p, int64_t j0, int64_t cols, const float *VJ) -> int {
            float *HJ = Ht + j0 * r;
            if (t == 1 && opt->check_finite && !S.resident) {
                if (int st = check_values(VJ, m * S.ldp, 1, S.s)) return st;
            }
            if (obj_prev) NMF_HIP(panel_loss(p, j0, cols, VJ));
            // E-step: P_J = (W' V_J)', then the panel's NQPs
            NMF_HIP(launch_dense_product(VJ, 0, m, cols, S.vld, nullptr, 0, W, r, S.PJ, S.dense_scratch, S.s));
            NMF_HIP(S.solve(S.GW, S.PJ, reg->l1_h, HJ, cols, true));
            if (stats && last)
                NMF_HIP(launch_kkt(S.GW, r, S.PJ, -1.f, reg->l1_h, HJ, cols, S.kkt_partial, S.kkt_slots + p,
                                   S.np, S.s));
            // the M-step's product: P_W += V_J Ht_J
            NMF_HIP(launch_dense_product(VJ, 0, m, cols, S.vld, nullptr, 1, HJ, r, S.Ptmp, S.dense_scratch, S.s));
            hipLaunchKernelGGL(k_add_f32, dim3(grid_for(m * r)), dim3(256), 0, S.s, S.PW, S.Ptmp, m * r);
            NMF_HIP(hipGetLastError());
            return NMF_OK;
        });
        if (st) return st;
        if (obj_prev)
            NMF_HIP(launch_objective_slots(S.loss_slots, S.np, reg, S.obj_scratch, S.obj + 2 * (t - 1), S.s));
        if (stats && last)
            for (int q = 0; q < 4; q++)
                NMF_HIP(launch_max_ordered(S.kkt_slots + q * S.np, S.np, S.kkt_out + q, S.s));
        // M-step (no V): Gram of the new H, then every row of W
        NMF_HIP(launch_gram(Ht, n, r, reg->l2_w, NMF_FP32, S.GH, S.gram_scratch, S.s, S.counter));
        NMF_HIP(S.solve(S.GH, S.PW, reg->l1_w, W, m, false));
        if (stats && last)
            NMF_HIP(launch_kkt(S.GH, r, S.PW, -1.f, reg->l1_w, W, m, S.kkt_partial, S.kkt_out + 4, 1, S.s));
    }
    // the objective after the last iteration (or of the start point when T = 0)
    if (want_obj && due(T)) {
        NMF_HIP(launch_objective_regs(W, m, Ht, n, r, S.obj_scratch, S.s));
        int st = S.for_each_panel([&](int64_t p, int64_t j0, int64_t cols, const float *VJ) -> int {
            NMF_HIP(panel_loss(p, j0, cols, VJ));
            return NMF_OK;
        });
        if (st) return st;
        NMF_HIP(launch_objective_slots(S.loss_slots, S.np, reg, S.obj_scratch, S.obj + 2 * T, S.s));
    }

    // ---------------------------------------------------------------- host outputs
    std::vector<double> ob((size_t)(T + 1) * 2, 0.0);
    double kk[8];
    for (double &v : kk) v = NAN;
    unsigned long long inner = 0;
    if (want_obj) NMF_HIP(hipMemcpyAsync(ob.data(), S.obj, ob.size() * 8, hipMemcpyDeviceToHost, S.s));
    if (stats && T > 0) NMF_HIP(hipMemcpyAsync(kk, S.kkt_out, 8 * 8, hipMemcpyDeviceToHost, S.s));
    NMF_HIP(hipMemcpyAsync(&inner, S.inner_total, 8, hipMemcpyDeviceToHost, S.s));
    NMF_HIP(hipStreamSynchronize(S.s));
    if (trace)
        for (int t = 0; t <= T; t++) trace[t] = due(t) ? ob[2 * t] : NAN;
    if (stats) {
        stats->loss = ob[2 * T];
        stats->objective = ob[2 * T + 1];
        set_kkt_stats(stats, kk, kk + 4);
        stats->inner_total = (int64_t)inner;
        stats->outer_done = T;
        stats->kbar = T > 0 ? (double)inner / ((double)T * (double)(m + n)) : 0.0;
    }
    return NMF_OK;
}
}  // namespace
}  // namespace nmfi


extern "C" int nmf_fit_single_pass(const nmf_matrix *V, int32_t r, const nmf_reg *reg, const nmf_opts *opt,
                                   int64_t panel_cols, float *W, float *Ht, double *trace, nmf_stats *stats,
                                   void *stream) {
    if (!V) return fail(NMF_E_INVAL, "V is NULL");
    if (V->kind != NMF_DENSE) return fail(NMF_E_UNSUPPORTED, "the single-pass fit takes dense V");
    if (!V->dense) return fail(NMF_E_INVAL, "V->dense is NULL");
    const int64_t m = V->rows, n = V->cols, ld = V->ld;
    if (m < 1 || n < 1) return fail(NMF_E_INVAL, "V must be non-empty (m = %lld, n = %lld)", (long long)m, (long long)n);
    if (ld < n) return fail(NMF_E_INVAL, "ld (%lld) must be >= n (%lld)", (long long)ld, (long long)n);
    if (r < 1 || r > NMF_MAX_RANK) return fail(NMF_E_INVAL, "r must be in [1, %d] (got %d)", NMF_MAX_RANK, r);
    if (!reg) return fail(NMF_E_INVAL, "reg is NULL");
    if (int st = validate_opts(opt)) return st;
    if (opt->precision != NMF_FP32)
        return fail(NMF_E_UNSUPPORTED, "the single-pass fit computes its products in FP32 only");
    const float regs[4] = {reg->l1_w, reg->l2_w, reg->l1_h, reg->l2_h};
    for (float v : regs)
        if (!(v >= 0.f) || !std::isfinite(v)) return fail(NMF_E_INVAL, "regularisation weights must be finite and >= 0");
    if (opt->max_outer < 0) return fail(NMF_E_INVAL, "max_outer must be >= 0");
    if (panel_cols < 1) return fail(NMF_E_INVAL, "panel_cols must be >= 1 (got %lld)", (long long)panel_cols);
    if (!W || !Ht) return fail(NMF_E_INVAL, "W and Ht must be non-NULL");
    if (!nqp_pick(r, 1, opt->lanes).E) return fail(NMF_E_INVAL, "lanes = %d cannot hold rank %d", opt->lanes, r);
    hipStream_t s = (hipStream_t)stream;
    if (opt->check_finite) {
        int st = NMF_OK;
        if (ld != n) {
            for (int64_t i = 0; i < m && !st; i++) st = check_values(V->dense + i * ld, n, 1, s);
        } else {
            st = check_values(V->dense, m * n, 1, s);
        }
        if (st) return st;
    }
    Streamer S;
    S.s = s;
    S.resident = true;
    S.Vh = V->dense; S.m = m; S.n = n; S.ld = ld; S.r = r; S.reg = *reg; S.opt = *opt;
    S.pc = std::min(panel_cols, n);
    S.ldp = (S.pc + 3) / 4 * 4;
    S.vld = ld;  // panels are column ranges of V itself
    S.np = (n + S.pc - 1) / S.pc;
    return run_panels(S, W, Ht, trace, stats);
}
