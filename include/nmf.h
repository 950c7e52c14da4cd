/*
 * nmf.h -- C ABI of the MI355X (gfx950) library for the alternating
 * anti-lopsided NNLS method of L1/L2-regularised NMF, after Nguyen & Ho,
 * arXiv:1506.08938.
 *
 * Notation.  The paper factors an n x m matrix of column instances as G F.
 * This library factors V (m x n) = W (m x r) * H (r x n) and stores H as
 * Ht = H' (n x r), so that every NNLS solution is one contiguous row:
 *   H-update (the paper's E-step, Algorithm 1): W fixed, one NQP per column
 *            j of V, solution = row j of Ht;
 *   W-update (the paper's M-step): H fixed, one NQP per row i of V, solution
 *            = row i of W.
 * Each NQP (Section 3.2, Eq. QP; regularised form Section 3.5, Eq. L1L2NMF)
 * is   min_x 0.5 x' Gamma x + h' x,  x >= 0,  with Gamma = A'A + 2 l2 I and
 * h = -A'b + l1 1, A the fixed factor and b the data column.  It is solved by
 * Algorithm 3: anti-lopsided rescale to unit diagonal, then iterations of an
 * exact line search on the projected gradient followed by r greedy
 * coordinate-descent steps, stopped by ||pg_k||^2 <= eps ||pg_0||^2
 * (Section 3.4) or max_inner.
 *
 * Conventions for every call:
 *  - Matrix pointers are DEVICE pointers owned by the caller; the library
 *    never frees or reallocates them.  Matrices are row-major, indices int32
 *    (nnz < 2^31), values float32.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are stream-ordered and asynchronous, except those that return
 *    host-side results (trace, stats, *_host arguments), which synchronise
 *    `stream` before returning.
 *  - Argument errors are found on the host before any launch and return
 *    NMF_E_INVAL; HIP runtime errors return NMF_E_DEVICE; allocation failures
 *    NMF_E_NOMEM.  nmf_last_error() gives a message for the calling thread.
 *    Reaching max_inner is not an error.
 *  - r must lie in [1, NMF_MAX_RANK].
 */
#ifndef NMF_MI355X_H
#define NMF_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NMF_MAX_RANK 128

#if defined(NMF_BUILDING_LIBRARY)
#define NMF_API __attribute__((visibility("default")))
#else
#define NMF_API
#endif

typedef enum {
    NMF_OK = 0,
    NMF_E_INVAL = -1,
    NMF_E_NOMEM = -2,
    NMF_E_DEVICE = -3,
    NMF_E_UNSUPPORTED = -4,
    NMF_E_BUSY = -5,
    NMF_E_NONFINITE = -6
} nmf_status;

enum { NMF_DENSE = 0, NMF_CSR = 1 };
enum { NMF_FP32 = 0, NMF_BF16 = 1 };

/* The data matrix V (Definition 1: V >= 0).  kind = NMF_DENSE: `dense` is
 * rows x cols with leading dimension ld >= cols.  kind = NMF_CSR: rowptr
 * (rows+1), colidx and vals (nnz) hold CSR(V), column indices ascending in
 * each row.  t_rowptr/t_colidx/t_vals optionally hold CSR(V') (cols+1 row
 * pointers); when NULL the library builds it on the device. */
typedef struct {
    int32_t kind;
    int64_t rows, cols;
    const float *dense;
    int64_t ld;
    const int32_t *rowptr;
    const int32_t *colidx;
    const float *vals;
    int64_t nnz;
    const int32_t *t_rowptr;
    const int32_t *t_colidx;
    const float *t_vals;
} nmf_matrix;

/* Regularisation weights of Section 3.5: J = 0.5||V - WH||^2 + l1_h sum(H)
 * + l2_h ||H||^2 + l1_w sum(W) + l2_w ||W||^2 (the paper's mu1, mu2 on the
 * coefficients and beta1, beta2 on the components). */
typedef struct {
    float l1_w, l2_w, l1_h, l2_h;
} nmf_reg;

/* Solver options.  max_inner: iteration cap of Algorithm 3 (>= 1).  eps: the
 * accelerated stopping condition ||pg_k||^2 <= eps ||pg_0||^2, evaluated in
 * double precision; eps = 0 stops only when the projected gradient is exactly
 * zero, so in practice it runs max_inner iterations.  ls_guard:
 * 1 rejects a line-search step that would raise the objective (the literal
 * projected step of Algorithm 3 can), 0 keeps the literal step.  precision:
 * NMF_FP32 or NMF_BF16 for the Gram and data products (the solve is always
 * float32, products are accumulated in float32).  BF16 with dense V: V and
 * the fixed factor in BF16 on the matrix cores (BF16 copies of V made once
 * per plan).  BF16 with CSR V: the row gathers read a BF16 copy of the fixed
 * factor (values stay float32), and the dense product of the hot columns
 * runs on the matrix cores from BF16 copies.  objective_every: compute the
 * loss every s outer iterations (0 = only when a trace or stats are
 * requested, at the end).  check_finite:
 * scan inputs for NaN/Inf (and V for negatives) before running.  lanes:
 * lanes of a wavefront that cooperate on one column in the solve kernel
 * (1, 2, 4, 8 or 16; 0 = chosen from r and the launch's column count: few
 * columns get wider groups).  It is a layout choice: results for different
 * lanes agree to rounding, and are bitwise reproducible for a fixed choice.
 * fast_break_cols: Algorithm 3's fast-break (maxStop) with each thread of
 * computation a fixed run of this many consecutive columns, solved in order:
 * within a run a column also stops once ||f~_k||^2 falls to the largest final
 * ||f~||^2 of the run's earlier columns (the first column of every run, and
 * every run of each half-iteration, start from 0).  0 (default) or 1: off.
 * The runs are a fixed partition, so results stay reproducible. */
typedef struct {
    int32_t max_outer;
    int32_t max_inner;
    double eps;
    int32_t ls_guard;
    int32_t precision;
    int32_t objective_every;
    int32_t check_finite;
    int32_t lanes;
    int32_t fast_break_cols;
} nmf_opts;

/* Statistics of a fit.  loss = 0.5||V - W H||^2, objective = J above (both
 * accumulated in double precision), kkt_* = max |min(x, grad)| over the last
 * half-iteration's NQPs (zero exactly at a KKT point of Eq. QP, Section 3.2),
 * kbar = inner iterations / (outer iterations x (m+n)) (Section 5.3).
 * kkt_*_cond: the three KKT conditions of the same NQPs separately, each 0
 * when it holds: [0] max(0, -min x) (nonnegativity), [1] max x_i |grad_i|
 * (complementarity), [2] max(0, -min grad_i over x_i = 0) (gradient >= 0 on
 * the zero entries).  grad = Gamma x + h in the original scale, in double. */
typedef struct {
    double loss, objective, kkt_w, kkt_h, kbar;
    int64_t inner_total;
    int32_t outer_done;
    double kkt_w_cond[3], kkt_h_cond[3];
} nmf_stats;

/* Fills *o with the defaults: max_outer 50, max_inner 100, eps 1e-3,
 * ls_guard 1, NMF_FP32, objective_every 0, check_finite 0, lanes 0,
 * fast_break_cols 0. */
NMF_API void nmf_default_opts(nmf_opts *o);

/* Message describing the calling thread's last non-OK status. */
NMF_API const char *nmf_last_error(void);

/* ---------------------------------------------------------------- NQP batch
 * Algorithm 3 on ncols independent NQPs sharing one Hessian (the per-column
 * units of Section 3.2, Algorithm 2):
 *   gram  r x r, = A'A + 2 l2 I (symmetric positive semidefinite; a
 *         coordinate with gram_ii <= 0 is held at 0);
 *   h     ncols x r, row j = -A'b_j + l1;
 *   X     ncols x r, in: x0 >= 0 (warm start), out: solution;
 *   iters optional device int32[ncols]: iterations run per column.
 * All device pointers; X must not alias gram or h. */
NMF_API int nnls_solve_batch(int32_t r, int64_t ncols, const float *gram, const float *h, float *X,
                     const nmf_opts *opt, int32_t *iters, void *stream);

/* The solve kernel's layout for rank r and a launch of ncols columns: *L
 * lanes per column, *E coordinates per lane (E * L >= r, the padded rank).
 * lanes as in nmf_opts.  Host-only; NMF_E_INVAL when lanes cannot hold r.
 * nmf_fit uses (r, n, lanes) for its H-update and (r, m, lanes) for its
 * W-update; nmf_fit_batched the total columns of all problems of a half-
 * iteration; a fold-in basis (r, 8192, lanes). */
NMF_API int nnls_layout(int32_t r, int64_t ncols, int32_t lanes, int32_t *E, int32_t *L);

/* ---------------------------------------------------------------- building blocks
 * One step of a half-iteration each (Algorithm 2; Section 4.2 costs them at
 * O(k r^2) and O(r S(mn)) / O(mnr)).  Device pointers throughout.
 * nmf_gram:    G (r x r) = A'A + 2 l2 I for A (k x r).
 * nmf_product: trans = 0: P (n x r) = (W'V)' with A = W (m x r);
 *              trans = 1: P (m x r) = V Ht   with A = Ht (n x r).
 * precision as in nmf_opts (BF16 makes temporary BF16 copies of what it
 * reads).  Sparse V with trans = 0 reads CSR(V') (the t_* arrays) when
 * given, else builds a temporary one; the CSR form plans its work on the
 * host and synchronises the stream, the dense form is stream-ordered. */
NMF_API int nmf_gram(const float *A, int64_t k, int32_t r, float l2, int32_t precision, float *G,
             void *stream);
NMF_API int nmf_product(const nmf_matrix *V, int32_t trans, int32_t r, const float *A, int32_t precision,
                float *P, void *stream);

/* ---------------------------------------------------------------- fit
 * Algorithm 2 with the regularised NQPs of Section 3.5: opt->max_outer outer
 * iterations, each an H-update followed by a W-update whose Gram is built
 * from the new H.
 *   W  m x r (device), in: start point >= 0, out: result.
 *   Ht n x r (device), in: start point >= 0, out: result.
 *   trace optional HOST double[max_outer + 1]: 0.5||V - WH||^2 before the
 *         first and after each outer iteration (NaN where not computed when
 *         objective_every > 0 skips it).
 *   stats optional HOST nmf_stats.
 * A plan keeps the device workspace and any derived copy of V (CSR(V'),
 * the BF16 copy) so that repeated runs pay set-up once; nmf_fit is
 * nmf_plan_create + nmf_plan_run + nmf_plan_destroy. */
typedef struct nmf_plan nmf_plan;

NMF_API int nmf_plan_create(const nmf_matrix *V, int32_t r, const nmf_reg *reg, const nmf_opts *opt,
                    nmf_plan **out, void *stream);
/* Runs `outer` outer iterations on (W, Ht); trace (host, [outer + 1]) and
 * stats (host) are optional. */
NMF_API int nmf_plan_run(nmf_plan *p, float *W, float *Ht, int32_t outer, double *trace, nmf_stats *stats,
                 void *stream);
NMF_API void nmf_plan_destroy(nmf_plan *p);

/* Per-phase device time of nmf_plan_run.  nmf_plan_profile(p, mode) clears
 * the totals and sets the mode: 0 stops; 1 records HIP events on the run's
 * stream around each phase's launches (a phase covers all of its kernels in
 * one half-iteration); 2 times the solve phase only, with the event pair
 * attached to the solve kernel's own dispatch, so nothing is added to the
 * stream between kernels.  nmf_plan_timers fills ms[NMF_PHASES]
 * (accumulated milliseconds) and calls[NMF_PHASES] (number of timed
 * phases) for the phases below. */
#define NMF_PHASES 4
enum { NMF_PHASE_GRAM = 0, NMF_PHASE_RESCALE = 1, NMF_PHASE_PRODUCT = 2, NMF_PHASE_SOLVE = 3 };
NMF_API int nmf_plan_profile(nmf_plan *p, int32_t mode);
NMF_API int nmf_plan_timers(const nmf_plan *p, double *ms, int64_t *calls);

NMF_API int nmf_fit(const nmf_matrix *V, int32_t r, const nmf_reg *reg, const nmf_opts *opt, float *W,
            float *Ht, double *trace, nmf_stats *stats, void *stream);

/* ---------------------------------------------------------------- limited internal memory
 * Algorithm 2 in the limited-internal-memory form of Section 3.3 (the
 * memory row of Table 1): V stays in HOST memory and each outer iteration
 * reads it once, a panel of panel_cols instances (columns of V) at a time.
 * Per panel J: the E-step's product (W'V_J)' and the NQPs of its columns of
 * Ht against W'W + 2 l2_h I, then the panel's share V_J Ht_J of the M-step's
 * product (the paper's sum of F_i V_i'), added in panel order.  The M-step
 * reads no V: W <- NQP(Ht'Ht + 2 l2_w I, -V Ht + l1_w, W).  Same iteration as
 * nmf_fit (H-update, then W-update from the new H); the products' sums are
 * grouped by panel, so results agree with nmf_fit to FP32 rounding.
 *   V_host   m x n row-major FP32 in host memory, leading dimension ld >= n.
 *            Page-locked memory (hipHostMalloc, torch pin_memory) lets the
 *            copy of the next panel overlap the work on the current one;
 *            pageable memory works, with copies that block the host.
 *   panel_cols >= 1 (capped at n); device memory beyond W and Ht is about
 *            4 * (2 * m * panel_cols + 2 * m * r + panel_cols * r) bytes plus
 *            scratch, whatever n is.
 *   W, Ht    device, as in nmf_fit; trace, stats as in nmf_fit.
 * opt->precision must be NMF_FP32 (NMF_E_UNSUPPORTED otherwise);
 * fast_break_cols runs are formed within each panel; check_finite also scans
 * each panel of V (for NaN/Inf and negatives) during the first pass.  The call
 * synchronises `stream` before returning (it frees its buffers). */
NMF_API int nmf_fit_streamed(const float *V_host, int64_t m, int64_t n, int64_t ld, int32_t r,
                             const nmf_reg *reg, const nmf_opts *opt, int64_t panel_cols, float *W,
                             float *Ht, double *trace, nmf_stats *stats, void *stream);

/* Algorithm 2's single pass over a V resident in device memory (dense,
 * float32, any leading dimension): the loop of Section 3.3 that forms the
 * M-step's data term as the sum over instance panels J of V_J Ht_J while the
 * E-step solves those panels, so that each outer iteration reads V from
 * memory once (the panel's second read, for its share of V Ht right after
 * its E-step product, comes from cache) instead of once per half.  Same
 * iteration as nmf_fit and nmf_fit_streamed (H-update, then the W-update
 * from the new H; results agree with nmf_fit to float32 rounding, the
 * products' sums being grouped by panel); the panels' E-step solves are
 * launches of panel_cols columns.  Arguments and outputs as nmf_fit_streamed,
 * V given as an nmf_matrix (kind NMF_DENSE, device pointer).  opt->precision
 * must be NMF_FP32.  Synchronises `stream` before returning. */
NMF_API int nmf_fit_single_pass(const nmf_matrix *V, int32_t r, const nmf_reg *reg, const nmf_opts *opt,
                                int64_t panel_cols, float *W, float *Ht, double *trace, nmf_stats *stats,
                                void *stream);

/* Loss and objective of (V, W, Ht) in double precision (host outputs). */
NMF_API int nmf_objective(const nmf_matrix *V, int32_t r, const nmf_reg *reg, const float *W,
                  const float *Ht, double *loss_host, double *objective_host, void *stream);

/* ---------------------------------------------------------------- batched
 * Many independent NMF problems of uneven sizes, each fitted as nmf_fit does
 * (Algorithm 2 with the regularised NQPs of Section 3.5), run together: each
 * phase of a half-iteration is one launch across all problems, and all
 * opt->max_outer outer iterations are captured in one hipGraph launched once.
 * A problem's result does not depend on the other problems in the batch.
 *   probs       HOST array of `count` problems; V dense (m x n) on the device,
 *               r in [1, NMF_MAX_RANK], W (m x r) and Ht (n x r) device
 *               start points, overwritten with the results.
 *   per_problem optional HOST array of `count` statistics (loss, objective,
 *               kbar, inner_total; KKT fields are NaN).
 * Synchronises `stream`. */
typedef struct {
    nmf_matrix V;
    int32_t r;
    nmf_reg reg;
    float *W;
    float *Ht;
} nmf_problem;

NMF_API int nmf_fit_batched(int32_t count, const nmf_problem *probs, const nmf_opts *opt,
                            nmf_stats *per_problem, void *stream);

/* ---------------------------------------------------------------- fold-in
 * The E-step alone against a resident basis (Section 3.1: the new columns'
 * coefficients F+ in the space of the learned components): for every column
 * v of Vnew (m x c), x = argmin_{x>=0} 0.5||v - W x||^2 + l1 1'x + l2||x||^2,
 * started from x0 = 0.
 * nmf_basis_create copies W (m x r, device) and computes Gamma = W'W + 2 l2 I
 * and its rescale once; with opt->precision = NMF_BF16 the Gram is formed in
 * BF16 and sparse requests gather from a BF16 copy of W (dense requests'
 * products stay float32).  nmf_foldin takes Vnew dense (m x c) or sparse given
 * as CSR(Vnew') (the t_* arrays, c rows over m columns) and writes
 * Ht_new (c x r, device); iters optional device int32[c]. */
typedef struct nmf_basis nmf_basis;

NMF_API int nmf_basis_create(const float *W, int64_t m, int32_t r, float l1, float l2, const nmf_opts *opt,
                     nmf_basis **out, void *stream);
NMF_API int nmf_foldin(const nmf_basis *B, const nmf_matrix *Vnew, float *Ht_new, int32_t *iters,
               void *stream);
NMF_API void nmf_basis_destroy(nmf_basis *B);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): nmf_foldin for
 * sparse Vnew (CSR(Vnew') in the t_* arrays) with no allocation.  Its scratch
 * (the solve's work counter and the c x r data-product rows) is a fixed
 * device array of NMF_FOLDIN_NOALLOC_BYTES, held on every GPU the library
 * runs on until the process ends; so c may be at most
 * (NMF_FOLDIN_NOALLOC_BYTES - 256) / (4 r) columns (32767 at r = 128), and
 * larger requests return NMF_E_INVAL before any launch.  Dense Vnew returns
 * NMF_E_UNSUPPORTED.  Results equal nmf_foldin's bitwise.  Every call on a
 * GPU shares that GPU's scratch and leaves its contents behind: calls that
 * overlap on one GPU (different streams or host threads) race; serialise
 * them. */
#define NMF_FOLDIN_NOALLOC_BYTES (16 << 20)
NMF_API int nmf_foldin_noalloc(const nmf_basis *B, const nmf_matrix *Vnew, float *Ht_new, int32_t *iters,
                               void *stream);

/* ---------------------------------------------------------------- serving
 * A request loop over a resident basis: fold-in requests (the E-step of
 * nmf_foldin for new columns) and small full fits (nmf_fit), continuously
 * batched.  max_slots slots each own a stream, a launcher thread and a
 * completion thread; a launcher admits the oldest waiting fold-in request,
 * else the oldest fit request (a fit that has waited 50 ms goes ahead of
 * fold-ins), while the HBM footprint of the admitted work stays within
 * hbm_budget bytes, packing queued fold-in requests (up to max_batch_cols
 * columns, in arrival order) into one batch with one product launch over its
 * sparse requests and a single solve launch; fit requests run on a slot with
 * stream-ordered memory, those waiting with the same options (and no
 * check_finite) together as one batch of up to 32 through the batched fit's
 * kernels, each result equal to its nmf_fit bitwise; fits hold at most
 * max_slots - 1 slots.  Launchers do not wait for the device (up to two
 * batches per slot are in flight); the completion thread reports a batch
 * done when its stream has passed it.  The slots are capped at the process's
 * hardware queues minus one (GPU_MAX_HW_QUEUES, 4 unless set, so 3 slots by
 * default): streams beyond that would share hardware queues, whose work runs
 * in order.  Requests arriving while others run are picked up by the next
 * free slot, so batches overlap on the device.  A request's result does not
 * depend on what it is batched with.  A fold-in batch runs in one of its
 * slot's two reused workspaces (device memory and page-locked host memory
 * for its descriptors, grown to the largest batch they have held and kept,
 * beside the budgeted footprints, until nmf_server_destroy); fit batches
 * allocate theirs stream-ordered from the device's default memory pool, and
 * nmf_server_create sets that pool's release threshold to keep what it
 * holds (a process-wide setting of the pool).
 * Request memory is the caller's (device pointers): its inputs must be
 * written before submission (workers run on their own streams, unordered with
 * the caller's) and it must stay valid until the request is done.  Fold-in requests use the basis' options; fit requests
 * carry their own (max_outer, ...). */
enum { NMF_REQ_FOLDIN = 0, NMF_REQ_FIT = 1 };

typedef struct {
    int32_t kind;
    nmf_matrix V;    /* fold-in: Vnew (m x c), dense or CSR(Vnew') in t_*; fit: dense V */
    float *out;      /* fold-in: c x r result (device) */
    int32_t *iters;  /* fold-in: optional device int32[c] */
    int32_t r;       /* fit: rank */
    nmf_reg reg;     /* fit */
    nmf_opts fit_opts; /* fit */
    float *W, *Ht;   /* fit: start points, overwritten with the results */
} nmf_request;

typedef struct nmf_server nmf_server;

NMF_API int nmf_server_create(const nmf_basis *B, size_t hbm_budget, int32_t max_slots,
                              int64_t max_batch_cols, nmf_server **out);
/* Queues a request; NMF_E_BUSY iff its footprint exceeds the whole budget. */
NMF_API int nmf_server_submit(nmf_server *s, const nmf_request *req, uint64_t *ticket);
/* *done = 1 once finished; latency_ms (optional) = completion - submission
 * (host clock; completion is when the request's stream has drained).
 * Returns the request's status once done.  A request reported done by poll
 * or by wait(ticket) is forgotten: its ticket is unknown afterwards. */
NMF_API int nmf_server_poll(nmf_server *s, uint64_t ticket, int32_t *done, double *latency_ms);
/* As nmf_server_poll, with the request's timeline (host clock, ms): once done,
 * times_ms[0] = submission -> admission (waiting in the queue), [1] =
 * admission -> its batch's last launch returned, [2] = that -> completion,
 * [3] = the whole latency; NaN while not done.  A request reported done is
 * forgotten, as with nmf_server_poll. */
NMF_API int nmf_server_poll_times(nmf_server *s, uint64_t ticket, int32_t *done, double *times_ms);
/* Blocks until the request (ticket 0: every request submitted so far; those
 * records stay until polled) is done. */
NMF_API int nmf_server_wait(nmf_server *s, uint64_t ticket, double *latency_ms);
NMF_API int nmf_server_stats(nmf_server *s, int64_t *completed, int64_t *columns, int64_t *batches);
/* Finishes the queued work, stops the workers and frees the server. */
NMF_API void nmf_server_destroy(nmf_server *s);

/* ---------------------------------------------------------------- measurement aid
 * nmf_probe_gather is not a step of the method: it reads the rows of `table`
 * (rows x row_bytes, device, row-major, row_bytes a multiple of 16) named by
 * idx[0..n) (device int32, NULL when n = 0; an index outside [0, rows) reads
 * the nearest row)
 * in that order, as the row gathers of the sparse data products do (Section
 * 4.2, one factor row per stored entry), with no other work, and writes
 * NMF_PROBE_GATHER_OUT_FLOATS floats of running sums to `out` (device) so
 * that no load is dead.  Its rate (n * row_bytes / its time) is the gather
 * ceiling the products are measured against.  Stream-ordered, allocates
 * nothing; NMF_E_INVAL for bad arguments or n * row_bytes / 16 >= 2^32 less
 * one launch's worth of work. */
#define NMF_PROBE_GATHER_OUT_FLOATS (2048 * 256 * 4)
/* nmf_dense_product_time (measurement aid for the autotuner): the dense
 * product of nmf_product (V m x n FP32 row-major with leading dimension ld,
 * device; A the fixed factor, device, (trans ? n : m) x r) with its split-K
 * slice count forced to nsplit (0: the library's own choice, the tuned table
 * or its rule), timed with HIP events over reps launches after one warm-up
 * (BF16: V converted once beforehand, untimed; the factor's BF16 copy and
 * the slices' sum are part of each launch).  *ms: milliseconds per launch.
 * Allocates stream-ordered and synchronises the stream. */
NMF_API int nmf_probe_gather(const void *table, int64_t rows, int32_t row_bytes, const int32_t *idx, int64_t n,
                             float *out, void *stream);
NMF_API int nmf_dense_product_time(const float *V, int64_t m, int64_t n, int64_t ld, int32_t trans, int32_t r,
                                   const float *A, int32_t precision, int32_t nsplit, int32_t reps, double *ms,
                                   void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NMF_MI355X_H */
