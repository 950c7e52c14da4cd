// Serving: fold-in requests (the E-step alone against a resident basis,
// Section 3.1) and small full fits (Algorithm 2), continuously batched.
//
// Each of `max_slots` slots owns a HIP stream (default priority), a launcher
// thread and a completion thread.  Requests queue in arrival order; a
// launcher admits the oldest fold-in request when one waits, else the oldest
// fit request (fits hold at most max_slots - 1 slots, and one that has waited
// 50 ms goes ahead of fold-ins), while the HBM footprint of the admitted work
// stays within the budget:
// queued fold-in requests (up to max_batch_cols columns) become one
// batch -- one product launch over all of its sparse requests' columns, then
// ONE solve launch over all of the batch's columns -- and a full-fit request
// runs on its slot, its memory stream-ordered on the slot's stream (no
// device-wide synchronisation); fit requests with the same options that are
// waiting in the queue go with it (up to kMaxFitBatch), through the batched
// fit's kernels -- a fit is latency-bound (its solves wait for their slowest
// column), so a batch of them takes about as long as one.  The launcher never waits for the
// device: it hands the batch, with an event recorded after its last launch,
// to the slot's completion thread and may admit the next one.  A fold-in
// batch runs in one of its slot's kMaxInFlight reused workspaces (device
// and page-locked host memory, grown to the largest batch they have held and
// kept until the server is destroyed, beside the budgeted footprints).  A slot with
// work in flight takes more (at most kMaxInFlight batches) only behind a
// fold-in batch and only while no slot is idle: work queued on a stream waits
// for the work ahead of it, and a fit keeps its stream busy for long.  The
// completion thread waits for the events in order and releases the batch's
// footprint.
// Requests arriving while batches run are picked up by the next free slot,
// so work from different batches overlaps on the device.  A column's
// arithmetic does not depend on the batch it lands in: results are the same
// alone and in the mix.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
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

constexpr size_t kMaxInFlight = 2;  // batches launched and not yet complete, per slot
constexpr size_t kMaxFitBatch = 32; // fit requests launched together
constexpr double kFitMaxWait = 0.05; // s a fit waits behind fold-in requests at most

struct Req {
    uint64_t ticket = 0;
    nmf_request q{};
    size_t footprint = 0;
    double t_submit = 0.0, t_admit = 0.0, t_launch = 0.0, t_done = 0.0;
    int state = 0;  // 0 queued, 1 running, 2 done
    int status = NMF_OK;
    std::string msg;  // the failure's message (the status is reported on another thread)
};

int64_t req_cols(const nmf_request &q) { return q.V.cols; }

// A batch whose launches are on its slot's stream; the host arrays it
// copied from live here until the batch completes.
struct InFlight {
    std::vector<std::shared_ptr<Req>> batch;
    size_t fp = 0;
    bool is_fit = false;
    int status = NMF_OK;
    std::string msg;
    hipEvent_t ev = nullptr;
    BatchedFit *fits = nullptr;  // several fit requests run together
    std::vector<BSolveProb> probs;
    std::vector<BSolveChunk> chunks;
    std::vector<SpRowsReq> rows;
    int work = -1;  // the slot's workspace this fold-in batch uses
};

// A fold-in batch's workspace, kept by its slot and reused: device memory
// (the work counter, the product rows P, dense scratch, the descriptors) and
// page-locked host memory the descriptors are copied up from in one copy.
// Allocating and freeing per batch cost ~0.2 ms of the launcher's time
// (hipMallocAsync ~65 us, hipFreeAsync ~130 us on average, in a HIP API
// trace of the serving loop), and a copy from pageable memory returns only
// once the stream reaches it.
struct Work {
    char *dev = nullptr, *host = nullptr;
    size_t dev_bytes = 0, host_bytes = 0;
    bool busy = false;  // under the slot's mutex
};

struct Slot {
    hipStream_t s = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::unique_ptr<InFlight>> inflight;
    bool closing = false;  // the launcher has finished; drain and stop
    std::thread launcher, completer;
    // under the server's mutex: batches in flight, and whether one is a fit
    int busy = 0;
    bool has_fit = false;
    Work work[kMaxInFlight];  // one per fold-in batch in flight
};

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
    std::vector<std::unique_ptr<Slot>> slots;
    int idle = 0;  // slots with nothing in flight
    int64_t batches = 0, completed = 0, columns = 0, submitted = 0;
};

namespace {

size_t foldin_footprint(const nmf_basis *B, const nmf_request &q) {
    size_t b = al256((size_t)q.V.cols * B->r * 4) + 4096;
    if (q.V.kind == NMF_DENSE) b += al256(dense_scratch_bytes(B->m, q.V.cols, B->r));
    return b;
}

// A free workspace of the slot with at least the given sizes, grown when
// needed (a workspace that is not busy has no work left on the stream that
// uses it, and the stream orders its replacement after that work); -1 if
// none is free or an allocation fails.
int take_work(Slot *sl, size_t dev_bytes, size_t host_bytes) {
    std::lock_guard<std::mutex> lk(sl->mu);
    for (int i = 0; i < (int)kMaxInFlight; i++) {
        Work &w = sl->work[i];
        if (w.busy) continue;
        if (w.dev_bytes < dev_bytes) {
            if (w.dev) (void)hipFreeAsync(w.dev, sl->s);
            w.dev = nullptr;
            w.dev_bytes = 0;
            const size_t want = std::max<size_t>(dev_bytes + dev_bytes / 4, 1 << 20);
            if (hipMallocAsync((void **)&w.dev, want, sl->s) != hipSuccess) {
                w.dev = nullptr;
                return -1;
            }
            w.dev_bytes = want;
        }
        if (w.host_bytes < host_bytes) {
            if (w.host) (void)hipHostFree(w.host);
            w.host = nullptr;
            w.host_bytes = 0;
            const size_t want = std::max<size_t>(host_bytes + host_bytes / 4, 64 << 10);
            if (hipHostMalloc((void **)&w.host, want, hipHostMallocDefault) != hipSuccess) {
                w.host = nullptr;
                return -1;
            }
            w.host_bytes = want;
        }
        w.busy = true;
        return i;
    }
    return -1;
}

// Launches one batch of fold-in requests on its slot's stream (no waiting).
int launch_foldin_batch(nmf_server *S, InFlight &F, Slot *sl) {
    const hipStream_t s = sl->s;
    const nmf_basis *B = S->B;
    const int r = B->r;
    int64_t ctot = 0, sparse_rows = 0;
    size_t dense_scr = 0;
    for (auto &q : F.batch) {
        ctot += req_cols(q->q);
        if (q->q.V.kind == NMF_DENSE) dense_scr = std::max(dense_scr, dense_scratch_bytes(B->m, q->q.V.cols, r));
    }
    // Chunks of the solve: a block takes one at a time, so a batch of fewer
    // columns than the chip has lane groups is cut finer (about two chunks
    // per CU, whole waves' worth of lane groups) to run on every CU instead
    // of a few; with the fast-break, whole units as always.  Only which block
    // solves a column depends on it, never the column's arithmetic.
    int chunk = bnqp_chunk_cols(B->var.L, B->opt.fast_break_cols);
    if (B->opt.fast_break_cols <= 1) {
        const int64_t gw = 64 / B->var.L;  // lane groups of a wave
        const int64_t want = (ctot + 2 * (int64_t)device_cu_count() - 1) / (2 * (int64_t)device_cu_count());
        chunk = (int)std::min<int64_t>(chunk, std::max<int64_t>(gw, (want + gw - 1) / gw * gw));
    }
    int64_t off = 0;
    for (size_t j = 0; j < F.batch.size(); j++) {
        const nmf_request &q = F.batch[j]->q;
        F.probs.push_back(BSolveProb{B->G, nullptr, q.out, r, B->l1, nullptr, q.iters, 1});
        for (int64_t c0 = 0; c0 < q.V.cols; c0 += chunk)
            F.chunks.push_back({(int32_t)j, (int32_t)c0, (int32_t)std::min<int64_t>(q.V.cols, c0 + chunk)});
        if (q.V.kind == NMF_CSR) {
            F.rows.push_back(SpRowsReq{q.V.t_rowptr, q.V.t_colidx, q.V.t_vals, sparse_rows, off});
            sparse_rows += q.V.cols;
        }
        off += q.V.cols;
    }
    const size_t pbytes = al256((size_t)ctot * r * 4), dbytes = al256(dense_scr);
    const size_t bp = al256(F.probs.size() * sizeof(BSolveProb)), bc = al256(F.chunks.size() * sizeof(BSolveChunk));
    const size_t br = al256(F.rows.size() * sizeof(SpRowsReq));
    const size_t ws_bytes = 256 + pbytes + dbytes + bp + bc + br;
    F.work = take_work(sl, ws_bytes, bp + bc + br);
    if (F.work < 0) return fail(NMF_E_DEVICE, "server fold-in workspace (%zu bytes)", ws_bytes);
    char *ws = sl->work[F.work].dev;
    unsigned int *queue = (unsigned int *)ws;
    float *P = (float *)(ws + 256);
    float *dscr = (float *)(ws + 256 + pbytes);
    BSolveProb *dprobs = (BSolveProb *)(ws + 256 + pbytes + dbytes);
    BSolveChunk *dchunks = (BSolveChunk *)((char *)dprobs + bp);
    SpRowsReq *drows = (SpRowsReq *)((char *)dchunks + bc);
    off = 0;
    for (size_t j = 0; j < F.batch.size(); j++) {
        F.probs[j].P = P + off * r;
        off += F.batch[j]->q.V.cols;
    }
    // the descriptors (probs, chunks, rows: contiguous in the workspace) in one copy
    char *h = sl->work[F.work].host;
    memcpy(h, F.probs.data(), F.probs.size() * sizeof(BSolveProb));
    memcpy(h + bp, F.chunks.data(), F.chunks.size() * sizeof(BSolveChunk));
    if (!F.rows.empty()) memcpy(h + bp + bc, F.rows.data(), F.rows.size() * sizeof(SpRowsReq));
    hipError_t e = hipMemcpyAsync(dprobs, h, bp + bc + br, hipMemcpyHostToDevice, s);
    off = 0;
    for (size_t j = 0; j < F.batch.size() && e == hipSuccess; j++) {
        const nmf_request &q = F.batch[j]->q;
        if (q.V.kind == NMF_DENSE)
            e = launch_dense_product(q.V.dense, 0, B->m, q.V.cols, q.V.ld, nullptr, 0, B->W, r, P + off * r, dscr, s);
        off += q.V.cols;
    }
    if (e == hipSuccess && !F.rows.empty())
        e = launch_spmm_rows_multi(drows, (int)F.rows.size(), sparse_rows, B->W, B->W16, B->lda16, r, P, s);
    if (e == hipSuccess) e = launch_zero_u32(queue, 1, s);
    if (e == hipSuccess)
        e = launch_bnqp(B->var, dchunks, (int)F.chunks.size(), queue, dprobs, B->opt.max_inner,
                        B->opt.eps, B->opt.ls_guard ? 1 : 0, B->opt.fast_break_cols, s);
    if (e != hipSuccess) return hip_fail(e, "server fold-in batch");
    return NMF_OK;
}

// A batch of fit requests (same options): alone through nmf_fit's plan
// (stream-ordered), together through the batched kernels with each
// problem's nmf_fit layout -- the results equal nmf_fit's bitwise either way.
int launch_fit_request(InFlight &F, hipStream_t s) {
    nmf_opts o = F.batch[0]->q.fit_opts;
    if (F.batch.size() == 1) {
        Req &R = *F.batch[0];
        return fit_stream_ordered(&R.q.V, R.q.r, &R.q.reg, &o, R.q.W, R.q.Ht, s);
    }
    std::vector<nmf_problem> pr;
    for (auto &q : F.batch) pr.push_back(nmf_problem{q->q.V, q->q.r, q->q.reg, q->q.W, q->q.Ht});
    return batched_fit_start((int32_t)pr.size(), pr.data(), &o, s, &F.fits);
}

// Fit requests that may run in one batch: same options, no input scan (the
// batched fit does not check its inputs), at least one outer iteration.
bool fit_batchable(const nmf_request &a, const nmf_request &b) {
    return !a.fit_opts.check_finite && a.fit_opts.max_outer > 0 &&
           memcmp(&a.fit_opts, &b.fit_opts, sizeof(nmf_opts)) == 0;
}

// Whether a slot may take more work now: always when idle; a second batch
// behind a fold-in batch (never behind a fit, whose stream stays busy for
// long) only when no slot is idle, since work queued on a busy stream waits
// for the work ahead of it.
bool slot_can_take(const nmf_server *S, const Slot *sl) {
    if (sl->busy == 0) return true;
    return sl->busy < (int)kMaxInFlight && !sl->has_fit && S->idle == 0;
}

// Takes admissible work off the queue, launches it, hands it to the
// completion thread; never waits for the device.
void launcher(nmf_server *S, Slot *sl) {
    (void)hipSetDevice(S->device);
    const hipStream_t s = sl->s;
    for (;;) {
        auto F = std::make_unique<InFlight>();
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // The first request this slot may start: the oldest fold-in
            // request when one waits (a fold-in batch takes a fraction of a
            // millisecond, a batch of fits tens of them), else the oldest fit
            // -- a fit may start only while fewer than max_fits fits run, and
            // one that has waited kFitMaxWait goes ahead of fold-ins.
            auto first = [&]() -> std::deque<std::shared_ptr<Req>>::iterator {
                auto fold = S->queue.end(), fit = S->queue.end();
                for (auto it = S->queue.begin(); it != S->queue.end(); ++it) {
                    if ((*it)->q.kind == NMF_REQ_FIT) {
                        if (fit == S->queue.end() && S->fits_running < S->max_fits) fit = it;
                    } else if (fold == S->queue.end()) {
                        fold = it;
                    }
                    if (fold != S->queue.end() && fit != S->queue.end()) break;
                }
                if (fit != S->queue.end() && (fold == S->queue.end() || now_s() - (*fit)->t_submit > kFitMaxWait))
                    return fit;
                return fold;
            };
            S->cv_work.wait(lk, [&] {
                if (S->stop && S->queue.empty()) return true;
                if (!slot_can_take(S, sl)) return false;
                auto it = first();
                return it != S->queue.end() && S->in_use + (*it)->footprint <= S->budget;
            });
            if (S->queue.empty()) break;  // stopping
            auto it = first();
            if ((*it)->q.kind == NMF_REQ_FIT) {
                F->batch.push_back(*it);
                F->fp = (*it)->footprint;
                it = S->queue.erase(it);
                F->is_fit = true;
                S->fits_running++;
                // queued fit requests that can run with it, in arrival order
                const nmf_request &head = F->batch[0]->q;
                while (it != S->queue.end() && F->batch.size() < kMaxFitBatch) {
                    auto &q = *it;
                    if (q->q.kind == NMF_REQ_FIT && fit_batchable(head, q->q) &&
                        S->in_use + F->fp + q->footprint <= S->budget) {
                        F->fp += q->footprint;
                        F->batch.push_back(q);
                        it = S->queue.erase(it);
                    } else {
                        ++it;
                    }
                }
            } else {
                // fold-in requests from there, in arrival order (fits stay queued)
                int64_t cols = 0;
                while (it != S->queue.end()) {
                    auto &q = *it;
                    if (q->q.kind != NMF_REQ_FOLDIN) {
                        ++it;
                        continue;
                    }
                    if (!F->batch.empty() && cols + req_cols(q->q) > S->max_cols) break;
                    if (S->in_use + F->fp + q->footprint > S->budget) break;
                    cols += req_cols(q->q);
                    F->fp += q->footprint;
                    F->batch.push_back(q);
                    it = S->queue.erase(it);
                }
            }
            S->in_use += F->fp;
            if (sl->busy++ == 0) S->idle--;
            if (F->is_fit) sl->has_fit = true;
            const double t = now_s();
            for (auto &q : F->batch) {
                q->state = 1;
                q->t_admit = t;
            }
        }
        F->status = F->is_fit ? launch_fit_request(*F, s) : launch_foldin_batch(S, *F, sl);
        if (F->status) F->msg = nmf_last_error();
        if (hipEventCreateWithFlags(&F->ev, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(F->ev, s) != hipSuccess) {
            if (F->ev) (void)hipEventDestroy(F->ev);
            F->ev = nullptr;  // the completion thread drains the stream instead
        }
        const double t = now_s();
        for (auto &q : F->batch) q->t_launch = t;
        {
            std::lock_guard<std::mutex> lk(sl->mu);
            sl->inflight.push_back(std::move(F));
        }
        sl->cv.notify_all();
    }
    {
        std::lock_guard<std::mutex> lk(sl->mu);
        sl->closing = true;
    }
    sl->cv.notify_all();
}

// Waits for the slot's batches in launch order and reports them done.
void completer(nmf_server *S, Slot *sl) {
    (void)hipSetDevice(S->device);
    for (;;) {
        InFlight *F = nullptr;
        {
            std::unique_lock<std::mutex> lk(sl->mu);
            sl->cv.wait(lk, [&] { return !sl->inflight.empty() || sl->closing; });
            if (sl->inflight.empty()) break;  // closing, drained
            F = sl->inflight.front().get();
        }
        hipError_t e = F->ev ? hipEventSynchronize(F->ev) : hipStreamSynchronize(sl->s);
        if (F->ev) (void)hipEventDestroy(F->ev);
        // the batch's workspace is free before the slot counts the batch as
        // done, so the launcher never finds a slot with room and no workspace
        if (F->work >= 0) {
            std::lock_guard<std::mutex> lk(sl->mu);
            sl->work[F->work].busy = false;
        }
        if (F->fits) batched_fit_end(F->fits);
        int st = F->status;
        std::string msg = F->msg;
        if (!st && e != hipSuccess) {
            st = hip_fail(e, "server batch");
            msg = nmf_last_error();
        }
        const double t = now_s();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->in_use -= F->fp;
            if (F->is_fit) {
                S->fits_running--;
                sl->has_fit = false;
            }
            if (--sl->busy == 0) S->idle++;
            S->batches++;
            for (auto &q : F->batch) {
                q->state = 2;
                q->status = st;
                q->msg = msg;
                q->t_done = t;
                S->completed++;
                S->columns += req_cols(q->q);
            }
        }
        {
            std::lock_guard<std::mutex> lk(sl->mu);
            sl->inflight.pop_front();  // releases the batch's host arrays
        }
        sl->cv.notify_all();
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
}

}  // namespace

namespace {
// Streams the server may use without two of them sharing a hardware queue:
// the HIP runtime gives a process GPU_MAX_HW_QUEUES hardware queues (4 unless
// set) and assigns streams to them in turn, and the work of streams on one
// queue runs in order -- a fold-in batch would wait behind a fit on another
// slot.  One queue is left to the default stream.
int hw_queue_slots() {
    int q = 4;
    if (const char *e = getenv("GPU_MAX_HW_QUEUES")) {
        const int v = atoi(e);
        if (v >= 1) q = v;
    }
    return q > 1 ? q - 1 : 1;
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
    max_slots = std::min(max_slots, hw_queue_slots());
    nmf_server *S = new nmf_server();
    S->B = B;
    S->budget = hbm_budget;
    S->max_cols = max_batch_cols;
    S->max_fits = max_slots > 1 ? max_slots - 1 : 1;
    if (hipGetDevice(&S->device) != hipSuccess) S->device = 0;
    {
        // Batches allocate their workspace stream-ordered from the device's
        // default pool; keep what the pool holds instead of returning it to
        // the system at every synchronisation (the next batch's allocation
        // would then wait for a fresh one).
        hipMemPool_t pool = nullptr;
        if (hipDeviceGetDefaultMemPool(&pool, S->device) == hipSuccess && pool) {
            uint64_t keep = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
    }
    for (int i = 0; i < max_slots; i++) {
        auto sl = std::make_unique<Slot>();
        hipError_t e = hipStreamCreateWithFlags(&sl->s, hipStreamNonBlocking);
        if (e != hipSuccess) {
            nmf_server_destroy(S);
            return hip_fail(e, "server stream");
        }
        S->slots.push_back(std::move(sl));
    }
    S->idle = max_slots;
    for (auto &sl : S->slots) {
        sl->completer = std::thread(completer, S, sl.get());
        sl->launcher = std::thread(launcher, S, sl.get());
    }
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
    const std::string msg = R.msg;
    S->reqs.erase(it);  // reported done: the record is released
    return st ? fail(st, "%s", msg.c_str()) : NMF_OK;
}

extern "C" int nmf_server_poll_times(nmf_server *S, uint64_t ticket, int32_t *done, double *times_ms) {
    if (!S || !done || !times_ms) return fail(NMF_E_INVAL, "server, done and times_ms must be non-NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(NMF_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
    const Req &R = *it->second;
    *done = R.state == 2;
    if (R.state != 2) {
        for (int i = 0; i < 4; i++) times_ms[i] = NAN;
        return NMF_OK;
    }
    times_ms[0] = (R.t_admit - R.t_submit) * 1e3;
    times_ms[1] = (R.t_launch - R.t_admit) * 1e3;
    times_ms[2] = (R.t_done - R.t_launch) * 1e3;
    times_ms[3] = (R.t_done - R.t_submit) * 1e3;
    const int st = R.status;
    const std::string msg = R.msg;
    S->reqs.erase(it);  // reported done: the record is released
    return st ? fail(st, "%s", msg.c_str()) : NMF_OK;
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
    return R->status ? fail(R->status, "%s", R->msg.c_str()) : NMF_OK;
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
    for (auto &sl : S->slots) {
        if (sl->launcher.joinable()) sl->launcher.join();
        if (sl->completer.joinable()) sl->completer.join();
        // every batch has completed
        for (Work &w : sl->work) {
            if (w.dev && sl->s) (void)hipFreeAsync(w.dev, sl->s);
            if (w.host) (void)hipHostFree(w.host);
        }
        if (sl->s) {
            (void)hipStreamSynchronize(sl->s);
            (void)hipStreamDestroy(sl->s);
        }
    }
    delete S;
}
