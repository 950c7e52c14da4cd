// Serving: fold-in requests (the E-step alone against a resident basis,
// Section 3.1) and small full fits (Algorithm 2), continuously batched.
//
// Each of `max_slots` worker threads owns a HIP stream (default priority).
// Requests queue in arrival order; a free worker admits from the head of the
// queue (fit requests hold at most max_slots - 1 slots: one stays free for
// fold-ins, which pass a fit that has to wait) while the HBM footprint of the
// admitted work stays within the budget:
// consecutive fold-in requests (up to max_batch_cols columns) become one
// batch -- one product launch per request, then ONE solve launch over all of
// the batch's columns -- and a full-fit request runs alone on its slot.
// Requests arriving while batches run are picked up by the next free slot,
// so work from different batches overlaps on the device.  A column's
// arithmetic does not depend on the batch it lands in: results are the same
// alone and in the mix.
#include <math.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "nmf_internal.h"

using namespace nmfi;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Req {
    uint64_t ticket = 0;
    nmf_request q{};
    size_t footprint = 0;
    double t_submit = 0.0, t_done = 0.0;
    int state = 0;  // 0 queued, 1 running, 2 done
    int status = NMF_OK;
};

int64_t req_cols(const nmf_request &q) { return q.V.cols; }

}  // namespace

struct nmf_server {
    const nmf_basis *B = nullptr;
    size_t budget = 0, in_use = 0;
    int64_t max_cols = 0;
    int max_fits = 1;      // fit requests running at once: one slot stays free for fold-ins
    int fits_running = 0;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Req>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Req>> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> workers;
    int64_t batches = 0, completed = 0, columns = 0, submitted = 0;
};

namespace {

size_t foldin_footprint(const nmf_basis *B, const nmf_request &q) {
    size_t b = al256((size_t)q.V.cols * B->r * 4) + 4096;
    if (q.V.kind == NMF_DENSE) b += al256(dense_scratch_bytes(B->m, q.V.cols, B->r));
    return b;
}

// one batch of fold-in requests on stream s
int run_foldin_batch(nmf_server *S, std::vector<std::shared_ptr<Req>> &batch, hipStream_t s) {
    const nmf_basis *B = S->B;
    const int r = B->r;
    int64_t ctot = 0;
    size_t dense_scr = 0;
    for (auto &q : batch) {
        ctot += req_cols(q->q);
        if (q->q.V.kind == NMF_DENSE) dense_scr = std::max(dense_scr, dense_scratch_bytes(B->m, q->q.V.cols, r));
    }
    std::vector<BSolveProb> probs;
    std::vector<BSolveChunk> chunks;
    const int chunk = bnqp_chunk_cols(B->var.L, B->opt.fast_break_cols);
    int64_t off = 0;
    for (size_t j = 0; j < batch.size(); j++) {
        const nmf_request &q = batch[j]->q;
        probs.push_back(BSolveProb{B->G, nullptr, q.out, r, B->l1, nullptr, q.iters, 1});
        for (int64_t c0 = 0; c0 < q.V.cols; c0 += chunk)
            chunks.push_back({(int32_t)j, (int32_t)c0, (int32_t)std::min<int64_t>(q.V.cols, c0 + chunk)});
        off += q.V.cols;
    }
    const size_t pbytes = al256((size_t)ctot * r * 4), dbytes = al256(dense_scr);
    const size_t lbytes = al256(probs.size() * sizeof(BSolveProb)) + al256(chunks.size() * sizeof(BSolveChunk));
    char *ws = nullptr;
    NMF_HIP(hipMallocAsync((void **)&ws, 256 + pbytes + dbytes + lbytes, s));
    unsigned int *queue = (unsigned int *)ws;
    float *P = (float *)(ws + 256);
    float *dscr = (float *)(ws + 256 + pbytes);
    BSolveProb *dprobs = (BSolveProb *)(ws + 256 + pbytes + dbytes);
    BSolveChunk *dchunks = (BSolveChunk *)((char *)dprobs + al256(probs.size() * sizeof(BSolveProb)));
    hipError_t e = hipSuccess;
    off = 0;
    for (size_t j = 0; j < batch.size() && e == hipSuccess; j++) {
        const nmf_request &q = batch[j]->q;
        float *Pj = P + off * r;
        probs[j].P = Pj;
        if (q.V.kind == NMF_DENSE)
            e = launch_dense_product(q.V.dense, 0, B->m, q.V.cols, q.V.ld, nullptr, 0, B->W, r, Pj, dscr, s);
        else if (B->W16)
            e = launch_spmm_rows16(q.V.t_rowptr, q.V.cols, q.V.t_colidx, q.V.t_vals, B->W16, B->lda16, r, Pj, s);
        else
            e = launch_spmm_rows(q.V.t_rowptr, q.V.cols, q.V.t_colidx, q.V.t_vals, B->W, r, Pj, s);
        off += q.V.cols;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(dprobs, probs.data(), probs.size() * sizeof(BSolveProb), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dchunks, chunks.data(), chunks.size() * sizeof(BSolveChunk), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_zero_u32(queue, 1, s);
    if (e == hipSuccess)
        e = launch_bnqp(B->var, dchunks, (int)chunks.size(), queue, dprobs, B->opt.max_inner,
                        B->opt.eps, B->opt.ls_guard ? 1 : 0, B->opt.fast_break_cols, s);
    (void)hipFreeAsync(ws, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host vectors live until here
    if (e != hipSuccess) return hip_fail(e, "server fold-in batch");
    return NMF_OK;
}

int run_fit_request(nmf_server *S, Req &R, hipStream_t s) {
    (void)S;
    nmf_opts o = R.q.fit_opts;
    return nmf_fit(&R.q.V, R.q.r, &R.q.reg, &o, R.q.W, R.q.Ht, nullptr, nullptr, s);
}

void worker(nmf_server *S) {
    (void)hipSetDevice(S->device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    for (;;) {
        std::vector<std::shared_ptr<Req>> batch;
        size_t fp = 0;
        bool is_fit = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // The first request this worker may start: the head of the queue,
            // except that a fit request waits while max_fits fits run, and the
            // fold-in requests queued behind it go ahead meanwhile.
            auto first = [&]() -> std::deque<std::shared_ptr<Req>>::iterator {
                for (auto it = S->queue.begin(); it != S->queue.end(); ++it) {
                    if ((*it)->q.kind == NMF_REQ_FIT && S->fits_running >= S->max_fits) continue;
                    return it;
                }
                return S->queue.end();
            };
            S->cv_work.wait(lk, [&] {
                if (S->stop && S->queue.empty()) return true;
                auto it = first();
                return it != S->queue.end() && S->in_use + (*it)->footprint <= S->budget;
            });
            if (S->queue.empty()) break;  // stopping
            auto it = first();
            if ((*it)->q.kind == NMF_REQ_FIT) {
                batch.push_back(*it);
                fp = (*it)->footprint;
                S->queue.erase(it);
                is_fit = true;
                S->fits_running++;
            } else {
                // consecutive fold-in requests from there, in arrival order
                int64_t cols = 0;
                while (it != S->queue.end()) {
                    auto &q = *it;
                    if (q->q.kind != NMF_REQ_FOLDIN) break;
                    if (!batch.empty() && cols + req_cols(q->q) > S->max_cols) break;
                    if (S->in_use + fp + q->footprint > S->budget) break;
                    cols += req_cols(q->q);
                    fp += q->footprint;
                    batch.push_back(q);
                    it = S->queue.erase(it);
                }
            }
            S->in_use += fp;
            for (auto &q : batch) q->state = 1;
        }
        int st;
        if (batch.size() == 1 && batch[0]->q.kind == NMF_REQ_FIT) st = run_fit_request(S, *batch[0], s);
        else st = run_foldin_batch(S, batch, s);
        const double t = now_s();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->in_use -= fp;
            if (is_fit) S->fits_running--;
            S->batches++;
            for (auto &q : batch) {
                q->state = 2;
                q->status = st;
                q->t_done = t;
                S->completed++;
                S->columns += req_cols(q->q);
            }
        }
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
    (void)hipStreamDestroy(s);
}

}  // namespace

extern "C" int nmf_server_create(const nmf_basis *B, size_t hbm_budget, int32_t max_slots,
                                 int64_t max_batch_cols, nmf_server **out) {
    if (!out) return fail(NMF_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!B) return fail(NMF_E_INVAL, "basis is NULL");
    if (max_slots < 1 || max_slots > 16) return fail(NMF_E_INVAL, "max_slots must be in [1, 16]");
    if (max_batch_cols < 1) return fail(NMF_E_INVAL, "max_batch_cols must be >= 1");
    if (hbm_budget < 4096) return fail(NMF_E_INVAL, "hbm_budget too small");
    nmf_server *S = new nmf_server();
    S->B = B;
    S->budget = hbm_budget;
    S->max_cols = max_batch_cols;
    S->max_fits = max_slots > 1 ? max_slots - 1 : 1;
    if (hipGetDevice(&S->device) != hipSuccess) S->device = 0;
    for (int i = 0; i < max_slots; i++) S->workers.emplace_back(worker, S);
    *out = S;
    return NMF_OK;
}

extern "C" int nmf_server_submit(nmf_server *S, const nmf_request *q, uint64_t *ticket) {
    if (!S || !q || !ticket) return fail(NMF_E_INVAL, "server, request and ticket must be non-NULL");
    auto R = std::make_shared<Req>();
    R->q = *q;
    if (q->kind == NMF_REQ_FOLDIN) {
        if (q->V.rows != S->B->m) return fail(NMF_E_INVAL, "fold-in request must have m = %lld rows", (long long)S->B->m);
        if (q->V.cols < 1 || !q->out) return fail(NMF_E_INVAL, "fold-in request needs >= 1 column and an output");
        if (q->V.kind == NMF_CSR && !(q->V.t_rowptr && q->V.t_colidx && q->V.t_vals))
            return fail(NMF_E_INVAL, "sparse fold-in requests give CSR(V') in the t_* arrays");
        if (q->V.kind == NMF_DENSE && (!q->V.dense || q->V.ld < q->V.cols))
            return fail(NMF_E_INVAL, "dense fold-in request needs V and ld >= cols");
        R->footprint = foldin_footprint(S->B, *q);
    } else if (q->kind == NMF_REQ_FIT) {
        if (q->V.kind != NMF_DENSE || !q->W || !q->Ht || q->r < 1 || q->r > NMF_MAX_RANK)
            return fail(NMF_E_INVAL, "fit request needs dense V, W, Ht and r in [1, %d]", NMF_MAX_RANK);
        if (int st = validate_opts(&q->fit_opts)) return st;
        R->footprint = plan_footprint(&q->V, q->r, &q->fit_opts);
    } else {
        return fail(NMF_E_INVAL, "unknown request kind %d", q->kind);
    }
    if (R->footprint > S->budget)
        return fail(NMF_E_BUSY, "request needs %zu bytes of HBM; the budget is %zu", R->footprint, S->budget);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return fail(NMF_E_INVAL, "server is shutting down");
        R->ticket = S->next_ticket++;
        R->t_submit = now_s();
        S->queue.push_back(R);
        S->reqs[R->ticket] = R;
        S->submitted++;
        *ticket = R->ticket;
    }
    S->cv_work.notify_all();
    return NMF_OK;
}

extern "C" int nmf_server_poll(nmf_server *S, uint64_t ticket, int32_t *done, double *latency_ms) {
    if (!S || !done) return fail(NMF_E_INVAL, "server and done must be non-NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(NMF_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
    const Req &R = *it->second;
    *done = R.state == 2;
    if (latency_ms) *latency_ms = R.state == 2 ? (R.t_done - R.t_submit) * 1e3 : NAN;
    if (R.state != 2) return NMF_OK;
    const int st = R.status;
    S->reqs.erase(it);  // reported done: the record is released
    return st;
}

extern "C" int nmf_server_wait(nmf_server *S, uint64_t ticket, double *latency_ms) {
    if (!S) return fail(NMF_E_INVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    if (ticket == 0) {  // every submitted request
        S->cv_done.wait(lk, [&] { return S->completed == S->submitted; });
        return NMF_OK;
    }
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(NMF_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
    auto R = it->second;
    S->cv_done.wait(lk, [&] { return R->state == 2; });
    if (latency_ms) *latency_ms = (R->t_done - R->t_submit) * 1e3;
    S->reqs.erase(ticket);  // reported done: the record is released
    return R->status;
}

extern "C" int nmf_server_stats(nmf_server *S, int64_t *completed, int64_t *columns, int64_t *batches) {
    if (!S) return fail(NMF_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    if (completed) *completed = S->completed;
    if (columns) *columns = S->columns;
    if (batches) *batches = S->batches;
    return NMF_OK;
}

extern "C" void nmf_server_destroy(nmf_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto &t : S->workers) t.join();
    delete S;
}
