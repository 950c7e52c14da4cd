// Batched fit of many independent, unevenly sized dense NMF problems
// (Algorithm 2 on each, with the regularised NQPs of Section 3.5).
//
// Every phase of a half-iteration is one launch across all problems: the
// Gram partials (work item = problem x 512 rows), the Gram finish (one block
// per problem), the data product (work item = problem x 128 output rows x k
// slice; in BF16 mode preceded by the factor's BF16 copy), and
// one persistent solve per kernel variant whose blocks take (problem, column
// range) chunks from a queue.  All max_outer outer iterations are captured
// into one hipGraph and launched once.  Problems only ever read their own
// buffers, so a problem's result does not depend on the batch it runs in.
//
// The same set-up serves the server's batches of fit requests
// (batched_fit_start): memory stream-ordered on the slot's stream, the
// phases launched straight onto it, and each problem's solve layout chosen
// from its own column counts as nmf_fit chooses it, so that every request's
// result equals its nmf_fit bitwise.
#include <math.h>

#include <map>
#include <vector>

#include "nmf_internal.h"

using namespace nmfi;

namespace {

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Relative cost of a column of an NQP whose Gram matrix sums K products in
// rank r: coordinate descent needs more iterations the worse the Gram's
// conditioning, which worsens as K / r falls towards 1.  Measured on 1024
// uneven problems (30 outer iterations): the mean inner iterations per column
// grow from 7 at K / r >= 10 to 8.5 at 4..10, 14 at 2..4 and 29..31 below 2;
// 1 + 20 / x^1.5 follows that rise.  Only the order in which chunks are taken
// depends on it, never a column's arithmetic.
double column_cost_weight(double x) { return 1.0 + 20.0 / (x * sqrt(x)); }

struct HalfLists {
    std::vector<BItem> gram_items, prod_items, red_items, f16_items;
    std::vector<BGramProb> gram;
    std::vector<BProdProb> prod;
    std::vector<BSolveProb> solve;
    std::map<std::pair<int, int>, std::vector<BSolveChunk>> chunks;  // per (E, L)
};

struct DevHalf {
    BItem *gram_items = nullptr, *prod_items = nullptr, *red_items = nullptr, *f16_items = nullptr;
    BGramProb *gram = nullptr;
    BProdProb *prod = nullptr;
    BSolveProb *solve = nullptr;
    std::vector<std::pair<NqpVariant, std::pair<BSolveChunk *, int>>> groups;
    int64_t n_gram_items = 0, n_prod_items = 0, n_red_items = 0, n_f16_items = 0;
};

template <class T>
int upload(const std::vector<T> &v, T **dst, char *&cursor, hipStream_t s) {
    *dst = (T *)cursor;
    cursor += al256(v.size() * sizeof(T) + 1);
    if (!v.empty()) NMF_HIP(hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return NMF_OK;
}

}  // namespace


namespace nmfi {

// A batched fit: its device buffers, its work lists (host copies kept while
// their uploads may be in flight) and how to launch them.
struct BatchedFit {
    int count = 0;
    nmf_opts opt{};
    bool bf16 = false, async_mem = false;
    hipStream_t s = nullptr;
    int ntmax = 1;
    char *base = nullptr, *lists = nullptr;
    HalfLists hl[2];
    DevHalf dh[2];
    unsigned int *queues = nullptr;
    struct Slot {
        size_t G, part, P, V16, V16t, A16, inner, kpart[2];
    };
    std::vector<Slot> slot;
    std::vector<nmf_problem> probs;

    void *dptr(size_t o) const { return (void *)(base + o); }

    hipError_t dmalloc(void **p, size_t bytes) {
        return async_mem ? hipMallocAsync(p, bytes, s) : hipMalloc(p, bytes);
    }
    void dfree(void *p) {
        if (!p) return;
        if (async_mem) (void)hipFreeAsync(p, s);
        else (void)hipFree(p);
    }
    void release() {
        dfree(lists);
        dfree(base);
        lists = base = nullptr;
    }

    // Validates the problems, allocates, builds and uploads the work lists.
    // solo_layout: each problem's solve layout from its own column counts
    // (as nmf_fit), else from the whole launch's.
    int prepare(int32_t count_, const nmf_problem *pr, const nmf_opts *o, hipStream_t s_, bool async,
                bool solo_layout);
    // Every outer iteration's phases straight onto the stream.
    int launch_direct();
    // Every outer iteration captured into one graph (the variants' solves as
    // parallel branches) and launched on the stream; synchronises it.
    int launch_graph();
};

int BatchedFit::prepare(int32_t count_, const nmf_problem *pr, const nmf_opts *o, hipStream_t s_, bool async,
                        bool solo_layout) {
    count = count_;
    opt = *o;
    s = s_;
    async_mem = async;
    bf16 = opt.precision == NMF_BF16;
    probs.assign(pr, pr + count);
    for (int p = 0; p < count; p++) {
        const nmf_problem &q = probs[p];
        if (q.V.kind != NMF_DENSE)
            return fail(NMF_E_UNSUPPORTED, "problem %d: the batched fit takes dense V", p);
        if (q.V.rows < 1 || q.V.cols < 1 || !q.V.dense || q.V.ld < q.V.cols)
            return fail(NMF_E_INVAL, "problem %d: bad dense V", p);
        if (q.r < 1 || q.r > NMF_MAX_RANK) return fail(NMF_E_INVAL, "problem %d: r out of range", p);
        if (opt.lanes && !nqp_lanes_ok(q.r, opt.lanes))
            return fail(NMF_E_INVAL, "problem %d: lanes = %d cannot hold rank %d", p, opt.lanes, q.r);
        if (!q.W || !q.Ht) return fail(NMF_E_INVAL, "problem %d: W and Ht must be non-NULL", p);
        const float rg[4] = {q.reg.l1_w, q.reg.l2_w, q.reg.l1_h, q.reg.l2_h};
        for (float v : rg)
            if (!(v >= 0.f) || !isfinite(v)) return fail(NMF_E_INVAL, "problem %d: bad regularisation", p);
        const int nt = (q.r + 31) / 32;
        if (nt > ntmax) ntmax = nt;
    }

    // ---------------------------------------------------------------- buffers
    slot.resize(count);
    size_t off = 0;
    auto place = [&](size_t bytes) { size_t o2 = off; off += al256(bytes); return o2; };
    for (int p = 0; p < count; p++) {
        const nmf_problem &q = probs[p];
        const int64_t m = q.V.rows, n = q.V.cols, r = q.r;
        slot[p].G = place((size_t)r * r * 4);
        slot[p].part = place(std::max(bgram_partial_floats(q.r, m), bgram_partial_floats(q.r, n)) * 4);
        slot[p].P = place((size_t)std::max(m, n) * r * 4);
        slot[p].V16 = bf16 ? place((size_t)m * n * 2) : 0;
        slot[p].V16t = bf16 ? place((size_t)m * n * 2) : 0;
        slot[p].A16 = bf16 ? place((size_t)((r + 31) / 32 * 32) * ((std::max(m, n) + 63) / 64 * 64) * 2) : 0;
        slot[p].inner = place(8);
        for (int h = 0; h < 2; h++) {  // split-K partials of each half's product
            const int64_t C = h == 0 ? n : m, K = h == 0 ? m : n;
            const int64_t kc = dense_kchunk(C, K, q.r, bf16, h == 0 && !bf16);
            const int64_t ns = (K + kc - 1) / kc;
            slot[p].kpart[h] = ns > 1 ? place((size_t)ns * C * r * 4) : 0;
        }
    }
    const size_t data_bytes = off;

    // ---------------------------------------------------------------- work lists
    {
        const hipError_t e0 = dmalloc((void **)&base, data_bytes + 256);
        if (e0 != hipSuccess) {
            base = nullptr;
            return fail(NMF_E_DEVICE, "batched buffers (%zu bytes): %s", data_bytes + 256, hipGetErrorString(e0));
        }
    }
    int64_t ctot[2] = {0, 0};  // columns solved per half-iteration, all problems
    for (int p = 0; p < count; p++) {
        ctot[0] += probs[p].V.cols;
        ctot[1] += probs[p].V.rows;
    }
    for (int h = 0; h < 2; h++) {
        for (int p = 0; p < count; p++) {
            const nmf_problem &q = probs[p];
            const int64_t m = q.V.rows, n = q.V.cols;
            const int r = q.r;
            const bool H = h == 0;
            const int64_t k = H ? m : n, C = H ? n : m;
            const float *A = H ? q.W : q.Ht;
            const int64_t grows = gram_rows(k);
            BGramProb g{A, k, r, H ? q.reg.l2_h : q.reg.l2_w, (float *)dptr(slot[p].part),
                        (float *)dptr(slot[p].G), (int)((k + grows - 1) / grows), grows};
            hl[h].gram.push_back(g);
            for (int c = 0; c < g.nchunks; c++) hl[h].gram_items.push_back({p, c});
            // BF16 reads the copy along k: V16t (n x m) for the H-update, V16 for the W-update
            const void *V = bf16 ? dptr(H ? slot[p].V16t : slot[p].V16) : (const void *)q.V.dense;
            const int64_t kc = dense_kchunk(C, k, r, bf16, H && !bf16);
            const int ns = (int)((k + kc - 1) / kc);
            const int64_t lda16 = (std::max(m, n) + 63) / 64 * 64;
            BProdProb prd{V, bf16 ? k : q.V.ld, C, k, A, r, (float *)dptr(slot[p].P),
                          ns > 1 ? (float *)dptr(slot[p].kpart[h]) : nullptr, kc, ns,
                          bf16 ? (__bf16 *)dptr(slot[p].A16) : nullptr, bf16 ? lda16 : 0};
            hl[h].prod.push_back(prd);
            if (bf16)
                for (int64_t kb = 0; kb < (k + 63) / 64; kb++) hl[h].f16_items.push_back({p, (int32_t)kb});
            for (int64_t cb = 0; cb < (C + DENSE_BM - 1) / DENSE_BM; cb++)
                for (int sl = 0; sl < ns; sl++) hl[h].prod_items.push_back({p, (int32_t)(cb * ns + sl)});
            if (ns > 1)
                for (int64_t eb = 0; eb < (C * r + 4095) / 4096; eb++) hl[h].red_items.push_back({p, (int32_t)eb});
            BSolveProb sv{(const float *)dptr(slot[p].G), (const float *)dptr(slot[p].P), H ? q.Ht : q.W,
                          r, H ? q.reg.l1_h : q.reg.l1_w, (unsigned long long *)dptr(slot[p].inner),
                          nullptr, 0};
            hl[h].solve.push_back(sv);
            // the layout is chosen for the whole launch's column count, or (solo
            // layout) for the problem's own, as nmf_fit chooses it
            const NqpVariant v = nqp_pick(r, solo_layout ? C : ctot[h], opt.lanes);
            const int chunk = bnqp_chunk_cols(v.L, opt.fast_break_cols);
            auto &lst = hl[h].chunks[{v.E, v.L}];
            for (int64_t c0 = 0; c0 < C; c0 += chunk)
                lst.push_back({p, (int32_t)c0, (int32_t)std::min<int64_t>(C, c0 + chunk)});
        }
    }
    // costliest chunks first (columns x r^2 x the conditioning weight), so that
    // the long ones do not start at the tail of the launch; order only, never a
    // column's arithmetic (measured on 1024 uneven problems, BF16: 0.93 s in
    // problem order, 0.87 s by columns x r^2, 0.79 s with the weight)
    for (int h = 0; h < 2; h++)
        for (auto &kv : hl[h].chunks) {
            auto cost = [&](const BSolveChunk &c) {
                const nmf_problem &q = probs[c.prob];
                const double x = (double)(h == 0 ? q.V.rows : q.V.cols) / q.r;  // Gram rows per rank
                return (double)(c.c1 - c.c0) * q.r * q.r * column_cost_weight(x);
            };
            std::stable_sort(kv.second.begin(), kv.second.end(),
                             [&](const BSolveChunk &x, const BSolveChunk &y) { return cost(x) > cost(y); });
        }
    // device copies of the lists (one allocation)
    size_t list_bytes = 0;
    for (int h = 0; h < 2; h++) {
        list_bytes += al256(hl[h].gram_items.size() * sizeof(BItem) + 1) + al256(hl[h].prod_items.size() * sizeof(BItem) + 1);
        list_bytes += al256(hl[h].red_items.size() * sizeof(BItem) + 1) + al256(hl[h].f16_items.size() * sizeof(BItem) + 1);
        list_bytes += al256(hl[h].gram.size() * sizeof(BGramProb) + 1) + al256(hl[h].prod.size() * sizeof(BProdProb) + 1);
        list_bytes += al256(hl[h].solve.size() * sizeof(BSolveProb) + 1);
        for (auto &kv : hl[h].chunks) list_bytes += al256(kv.second.size() * sizeof(BSolveChunk) + 1);
    }
    const int ngroups = (int)(hl[0].chunks.size() + hl[1].chunks.size());
    list_bytes += al256((size_t)(ngroups + 1) * sizeof(unsigned int));
    hipError_t e = dmalloc((void **)&lists, list_bytes + 256);
    if (e != hipSuccess) { lists = nullptr; return hip_fail(e, "batched work lists"); }
    int st = NMF_OK;
    char *cur = lists;
    for (int h = 0; h < 2 && !st; h++) {
        st = upload(hl[h].gram_items, &dh[h].gram_items, cur, s);
        if (!st) st = upload(hl[h].prod_items, &dh[h].prod_items, cur, s);
        if (!st) st = upload(hl[h].red_items, &dh[h].red_items, cur, s);
        if (!st) st = upload(hl[h].f16_items, &dh[h].f16_items, cur, s);
        if (!st) st = upload(hl[h].gram, &dh[h].gram, cur, s);
        if (!st) st = upload(hl[h].prod, &dh[h].prod, cur, s);
        if (!st) st = upload(hl[h].solve, &dh[h].solve, cur, s);
        dh[h].n_gram_items = (int64_t)hl[h].gram_items.size();
        dh[h].n_prod_items = (int64_t)hl[h].prod_items.size();
        dh[h].n_red_items = (int64_t)hl[h].red_items.size();
        dh[h].n_f16_items = (int64_t)hl[h].f16_items.size();
        for (auto &kv : hl[h].chunks) {
            BSolveChunk *d = nullptr;
            if (!st) st = upload(kv.second, &d, cur, s);
            dh[h].groups.push_back({NqpVariant{kv.first.first, kv.first.second}, {d, (int)kv.second.size()}});
        }
    }
    queues = (unsigned int *)cur;
    // BF16 copies of V and zeroed iteration counters
    for (int p = 0; p < count && !st; p++) {
        const nmf_problem &q = probs[p];
        if (bf16) {
            e = launch_to_bf16(q.V.dense, q.V.rows, q.V.cols, q.V.ld, (__bf16 *)dptr(slot[p].V16), s);
            if (e == hipSuccess)
                e = launch_to_bf16_t(q.V.dense, q.V.rows, q.V.cols, q.V.ld, (__bf16 *)dptr(slot[p].V16t), s);
            if (e != hipSuccess) st = hip_fail(e, "BF16 copies");
        }
        if (!st) {
            e = launch_zero_u64((unsigned long long *)dptr(slot[p].inner), 1, s);
            if (e != hipSuccess) st = hip_fail(e, "zero counters");
        }
    }
    if (!st && !async_mem) {
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "batched set-up");
    }
    return st;
}

int BatchedFit::launch_direct() {
    hipError_t e = hipSuccess;
    for (int t = 0; t < opt.max_outer && e == hipSuccess; t++) {
        for (int h = 0; h < 2 && e == hipSuccess; h++) {
            const int gi = h * (int)hl[0].chunks.size();
            e = launch_zero_u32(queues + gi, (int)dh[h].groups.size(), s);
            if (e == hipSuccess) e = launch_bgram(dh[h].gram_items, dh[h].n_gram_items, dh[h].gram, count, ntmax,
                                                  opt.precision, s);
            if (e == hipSuccess)
                e = launch_bdense(dh[h].prod_items, dh[h].n_prod_items, dh[h].prod, ntmax, h == 0, bf16,
                                  dh[h].red_items, dh[h].n_red_items, dh[h].f16_items, dh[h].n_f16_items, s);
            for (size_t g = 0; g < dh[h].groups.size() && e == hipSuccess; g++)
                e = launch_bnqp(dh[h].groups[g].first, dh[h].groups[g].second.first, dh[h].groups[g].second.second,
                                queues + gi + (int)g, dh[h].solve, opt.max_inner, opt.eps, opt.ls_guard ? 1 : 0,
                                opt.fast_break_cols, s);
        }
    }
    if (e != hipSuccess) return hip_fail(e, "batched launches");
    return NMF_OK;
}

int BatchedFit::launch_graph() {
    int st = NMF_OK;
    hipError_t e = hipSuccess;
    // The solve launches of a half (one per kernel variant) are independent:
    // they are captured as parallel branches (fork/join through events on
    // side streams), so one variant's tail overlaps the others' work.
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    size_t maxg = 0;
    for (int h = 0; h < 2; h++) maxg = std::max(maxg, dh[h].groups.size());
    std::vector<hipStream_t> side(maxg > 1 ? maxg - 1 : 0, nullptr);
    std::vector<hipEvent_t> evs;
    if (opt.max_outer > 0) {
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        for (size_t i = 0; i < side.size() && e == hipSuccess; i++)
            e = hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking);
        // one fork event and one join event per side stream and half-iteration
        const size_t nev = (size_t)opt.max_outer * 2 * (1 + side.size());
        for (size_t i = 0; i < nev && e == hipSuccess; i++) {
            hipEvent_t ev = nullptr;
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) evs.push_back(ev);
        }
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        for (int t = 0; t < opt.max_outer && e == hipSuccess; t++) {
            for (int h = 0; h < 2 && e == hipSuccess; h++) {
                int gi = h * (int)hl[0].chunks.size();
                e = launch_zero_u32(queues + gi, (int)dh[h].groups.size(), cs);
                if (e == hipSuccess)
                    e = launch_bgram(dh[h].gram_items, dh[h].n_gram_items, dh[h].gram, count, ntmax,
                                     opt.precision, cs);
                if (e == hipSuccess)
                    e = launch_bdense(dh[h].prod_items, dh[h].n_prod_items, dh[h].prod, ntmax, h == 0,
                                      bf16, dh[h].red_items, dh[h].n_red_items, dh[h].f16_items,
                                      dh[h].n_f16_items, cs);
                const size_t ng = dh[h].groups.size();
                const size_t ev0 = ((size_t)t * 2 + h) * (1 + side.size());
                if (e == hipSuccess && ng > 1) e = hipEventRecord(evs[ev0], cs);  // fork
                for (size_t g = 0; g < ng && e == hipSuccess; g++) {
                    hipStream_t gs = g == 0 ? cs : side[g - 1];
                    if (g > 0) e = hipStreamWaitEvent(gs, evs[ev0], 0);
                    if (e == hipSuccess)
                        e = launch_bnqp(dh[h].groups[g].first, dh[h].groups[g].second.first,
                                        dh[h].groups[g].second.second, queues + gi + (int)g,
                                        dh[h].solve, opt.max_inner, opt.eps, opt.ls_guard ? 1 : 0,
                                        opt.fast_break_cols, gs);
                    if (e == hipSuccess && g > 0) e = hipEventRecord(evs[ev0 + g], gs);
                }
                for (size_t g = 1; g < ng && e == hipSuccess; g++) e = hipStreamWaitEvent(cs, evs[ev0 + g], 0);  // join
            }
        }
        hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e == hipSuccess) e = hipGraphLaunch(exec, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "batched graph");
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cs) (void)hipStreamDestroy(cs);
    for (hipStream_t x : side)
        if (x) (void)hipStreamDestroy(x);
    for (hipEvent_t ev : evs) (void)hipEventDestroy(ev);
    return st;
}

// The server's batches of fit requests: prepared and launched on `stream`
// without waiting for the device; *out is released (batched_fit_end) once
// the stream has passed the launches.
int batched_fit_start(int32_t count, const nmf_problem *probs, const nmf_opts *opt, hipStream_t stream,
                      BatchedFit **out) {
    *out = nullptr;
    auto *b = new BatchedFit();
    int st = b->prepare(count, probs, opt, stream, true, true);
    if (!st) st = b->launch_direct();
    b->release();  // stream-ordered: after the launches
    if (st) {
        delete b;
        return st;
    }
    *out = b;
    return NMF_OK;
}

void batched_fit_end(BatchedFit *b) { delete b; }

}  // namespace nmfi

extern "C" int nmf_fit_batched(int32_t count, const nmf_problem *probs, const nmf_opts *opt,
                               nmf_stats *per_problem, void *stream) {
    if (count < 0) return fail(NMF_E_INVAL, "count must be >= 0");
    if (count == 0) return NMF_OK;
    if (!probs) return fail(NMF_E_INVAL, "probs is NULL");
    if (int st = validate_opts(opt)) return st;
    if (opt->max_outer < 0) return fail(NMF_E_INVAL, "max_outer must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    BatchedFit b;
    int st = b.prepare(count, probs, opt, s, false, false);
    if (!st) st = b.launch_graph();

    // ---------------------------------------------------------------- statistics
    if (!st && per_problem) {
        for (int p = 0; p < count && !st; p++) {
            const nmf_problem &q = probs[p];
            double loss = NAN, obj = NAN;
            st = nmf_objective(&q.V, q.r, &q.reg, q.W, q.Ht, &loss, &obj, stream);
            unsigned long long inner = 0;
            if (!st) {
                hipError_t e = hipMemcpy(&inner, b.dptr(b.slot[p].inner), sizeof inner, hipMemcpyDeviceToHost);
                if (e != hipSuccess) st = hip_fail(e, "batched stats");
            }
            nmf_stats &o = per_problem[p];
            o.loss = loss;
            o.objective = obj;
            o.kkt_w = NAN;
            o.kkt_h = NAN;
            for (int q2 = 0; q2 < 3; q2++) o.kkt_w_cond[q2] = o.kkt_h_cond[q2] = NAN;
            o.inner_total = (int64_t)inner;
            o.outer_done = opt->max_outer;
            o.kbar = opt->max_outer > 0
                         ? (double)inner / ((double)opt->max_outer * (double)(q.V.rows + q.V.cols))
                         : 0.0;
        }
    }
    (void)hipStreamSynchronize(s);
    b.release();
    return st;
}

namespace nmfi {
hipError_t launch_bnqp(const NqpVariant &v, const BSolveChunk *chunks, int nchunks,
                       unsigned int *queue, const BSolveProb *probs, int max_inner, double eps,
                       int ls_guard, int unit, hipStream_t s) {
    switch (v.L) {
    case 1: return launch_bnqp_l1(v.E, chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 2: return launch_bnqp_l2(v.E, chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 4: return launch_bnqp_l4(v.E, chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 8: return launch_bnqp_l8(v.E, chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    case 16: return launch_bnqp_l16(v.E, chunks, nchunks, queue, probs, max_inner, eps, ls_guard, unit, s);
    default: return hipErrorInvalidValue;
    }
}
}  // namespace nmfi
