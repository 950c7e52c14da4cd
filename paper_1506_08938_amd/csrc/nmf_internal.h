// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "nmf.h"
#include "nqp_variants.h"

namespace nmfi {

// ------------------------------------------------------------------ errors
void set_error(int status, const std::string &msg);
int fail(int status, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);

#define NMF_HIP(call)                                    \
    do {                                                 \
        hipError_t _e = (call);                          \
        if (_e != hipSuccess) return nmfi::hip_fail(_e, #call); \
    } while (0)

// ------------------------------------------------------------------ NQP solve
struct NqpParams {
    const float *gram;   // r x r Hessian Gamma (rescaled while staging)
    const float *P;      // ncols x ldp: product rows (or h rows)
    float hsign, hadd;   // h = hsign * P + hadd
    float *X;            // ncols x ldx, in: x0 (ignored when cold), out: x
    int64_t ncols;
    int r, ldp, ldx;
    int max_inner;
    double eps;
    int ls_guard;
    int cold;
    int32_t *iters;                    // optional, per column
    unsigned long long *counter;       // work counter; must be zero at launch
    unsigned long long *inner_total;   // optional accumulator of iterations
    int unit;  // columns per fast-break thread of computation (<= 1: off)
    // host side (unused by the kernel): when set, the launch records these
    // events with its own dispatch (start and end of the kernel)
    hipEvent_t ev_start, ev_stop;
};

// Kernel variant (entries per lane E, lanes per column L).
struct NqpVariant {
    int E, L;
};
// Lanes per column for rank r and a launch of ncols columns: `lanes` > 0
// forces L (E = 0 when L cannot hold r); 0 picks the throughput layout for r
// and widens it while the launch would leave the chip short of lanes.
NqpVariant nqp_pick(int r, int64_t ncols, int lanes);
// Lanes-per-column values a launch can use for rank r (nonzero E).
bool nqp_lanes_ok(int r, int lanes);

// Launches the persistent solve kernel for the given variant.
hipError_t launch_nqp(const NqpVariant &v, const NqpParams &p, hipStream_t s);

// ------------------------------------------------------------------ products
constexpr int SPMM_CHUNK = 512;  // stored entries per SpMM work item
constexpr int DENSE_BM = 128;    // rows of P per dense-product block

struct SpChunk {
    int32_t row, start, end, dest;  // dest < 0: write P[row]; else partial slot
};
struct SpSplit {
    int32_t row, first, count;  // a split row's partial slots
};
struct SpmmPlan {
    SpChunk *chunks;
    SpSplit *splits;
    int64_t nrows, nchunks, nsplits;
    int32_t nslots;
};
// skip (optional, one flag per row): rows that get no chunk (written elsewhere)
int build_spmm_plan(const std::vector<int32_t> &rowptr, SpmmPlan *pl, hipStream_t s,
                    const std::vector<char> *skip = nullptr);
hipError_t launch_hot_scatter_v(const int32_t *rowptr, int64_t m, const int32_t *colidx,
                                const float *vals, const int32_t *slot, int T, float *Vhot,
                                hipStream_t s);
hipError_t launch_hot_rows_out(const float *Phot, const int32_t *idx, int T, int r, float *P,
                               hipStream_t s);
void free_spmm_plan(SpmmPlan *pl);
hipError_t launch_spmm(const SpmmPlan &pl, const int32_t *colidx, const float *vals, const float *A,
                       int r, float *P, float *partial, hipStream_t s);
// one wave per row straight from the row pointers (no split); for short rows
hipError_t launch_spmm_rows(const int32_t *rowptr, int64_t nrows, const int32_t *colidx,
                            const float *vals, const float *A, int r, float *P, hipStream_t s);
// BF16 mode: the same products gathering from A16 (k x lda16 BF16, rows of r
// values padded with zeros to spmm_lda16(r)), accumulated in float32
#ifndef NMF_SPMM_VEC16
#define NMF_SPMM_VEC16 8  // BF16 values per lane and piece (8: 16-byte loads, 4: 8-byte)
#endif
inline int spmm_lda16(int r) { return (r + NMF_SPMM_VEC16 - 1) / NMF_SPMM_VEC16 * NMF_SPMM_VEC16; }
hipError_t launch_rows_to_bf16(const float *A, int64_t k, int r, int lda16, __bf16 *A16, hipStream_t s);
hipError_t launch_spmm16(const SpmmPlan &pl, const int32_t *colidx, const float *vals,
                         const __bf16 *A16, int lda16, int r, float *P, float *partial, hipStream_t s);
hipError_t launch_spmm_rows16(const int32_t *rowptr, int64_t nrows, const int32_t *colidx,
                              const float *vals, const __bf16 *A16, int lda16, int r, float *P,
                              hipStream_t s);
// One request of a multi-request row product: its CSR (rows of the
// request's transpose) and the global index of its first row.
struct SpRowsReq {
    const int32_t *rowptr;
    const int32_t *colidx;
    const float *vals;
    int64_t row0;  // index of its first row among the launch's rows
    int64_t p0;    // row of P its first row is written to
};
// The launch's nrows rows are those of nreq requests (reqs: device array
// sorted by row0, row0[0] = 0, every request non-empty); request q's row i
// times A (FP32), or A16 (BF16 copy with leading dimension lda16) when A16 is
// non-null, goes to row q.p0 + i of P (ld r).
hipError_t launch_spmm_rows_multi(const SpRowsReq *reqs, int nreq, int64_t nrows, const float *A,
                                  const __bf16 *A16, int lda16, int r, float *P, hipStream_t s);

size_t gram_scratch_bytes(int r, int64_t k);
// Also zeroes *counter (when non-NULL) so that a solve can follow on the stream.
hipError_t launch_gram(const float *A, int64_t k, int r, float l2, int precision, float *G,
                       float *scratch, hipStream_t s, unsigned long long *counter = nullptr);

size_t dense_scratch_bytes(int64_t m, int64_t n, int r);
// scratch for a product with its slices forced (the autotuner's timing)
size_t dense_forced_partial_bytes(int64_t m, int64_t n, int r, int force_nsplit);
size_t dense_scratch_bytes_forced(int64_t m, int64_t n, int r, int force_nsplit);
// split-K decomposition of P (C x r) = X (C x K) A shared by the single and
// batched products: nsplit slices of kchunk (a multiple of 64) each, from the
// autotuned table (dense_tuned.h) for the kernel -- bf16, or FP32 reading X
// k-major (xt: V' in the H-update) or not -- and the rank's column tiles
int dense_nsplit(int64_t C, int64_t K, int r, int bf16, int xt);
int64_t dense_kchunk(int64_t C, int64_t K, int r, int bf16, int xt);
// force_nsplit > 0 (the autotuner): that many slices instead (scratch:
// dense_scratch_bytes_forced)
hipError_t launch_dense_product(const void *V, int bf16, int64_t m, int64_t n, int64_t ld,
                                const __bf16 *V16t, int trans, const float *A, int r, float *P,
                                float *scratch, hipStream_t s, int force_nsplit = 0);
hipError_t launch_to_bf16_t(const float *x, int64_t rows, int64_t cols, int64_t ld, __bf16 *y,
                            hipStream_t s);
hipError_t launch_to_bf16(const float *x, int64_t rows, int64_t cols, int64_t ld, __bf16 *y,
                          hipStream_t s);

// ------------------------------------------------------------------ batched
// one block's work item: (problem index, chunk / row-block index)
struct BItem {
    int32_t prob, idx;
};
constexpr int BGRAM_ROWS = 512;  // rows of A per Gram work item (at least; solo and batched)
int64_t gram_rows(int64_t k);     // rows per Gram work item for k rows of A
struct BGramProb {
    const float *A;
    int64_t k;
    int r;
    float l2;
    float *partial;  // ceil(k / rows) partials of NTILE * 1024 floats
    float *G;        // r x r
    int nchunks;
    int64_t rows;    // rows of A per work item: gram_rows(k)
};
struct BProdProb {
    const void *V;  // FP32: V (m x n, ld); BF16: the copy read along k (V16 for
                    // the W-update, V16t for the H-update; ld = K)
    int64_t ld;
    int64_t C, K;   // P is C x r, summed over K
    const float *A; // K x r
    int r;
    float *P;
    float *part;    // nsplit x C x r split-K partials (when nsplit > 1)
    int64_t kchunk;
    int nsplit;
    __bf16 *A16;    // BF16: the factor converted and transposed, R32 x lda16
    int64_t lda16;
};
struct BSolveProb {
    const float *G;  // r x r
    const float *P;  // C x r data products
    float *X;        // C x r solutions (warm start unless cold)
    int r;
    float l1;
    unsigned long long *inner;  // iterations of this problem's columns
    int32_t *iters;             // optional per-column iteration counts
    int cold;                   // 1: start from x0 = 0 (X is not read)
};
struct BSolveChunk {
    int32_t prob, c0, c1;
};
size_t bgram_partial_floats(int r, int64_t k);
hipError_t launch_bgram(const BItem *items, int64_t nitems, const BGramProb *probs, int nprobs,
                        int ntmax, int precision, hipStream_t s);
// items: (problem, row block * nsplit + slice); reduce items: (problem,
// block of 4096 entries of P) for problems with nsplit > 1
// f16_items (BF16): (problem, block of 64 rows of A) for the factor conversion
hipError_t launch_bdense(const BItem *items, int64_t nitems, const BProdProb *probs, int ntmax,
                         bool xt, bool bf16, const BItem *red_items, int64_t nred,
                         const BItem *f16_items, int64_t nf16, hipStream_t s);
// unit: columns per fast-break thread of computation (<= 1: no fast-break)
hipError_t launch_bnqp(const NqpVariant &v, const BSolveChunk *chunks, int nchunks,
                       unsigned int *queue, const BSolveProb *probs, int max_inner, double eps,
                       int ls_guard, int unit, hipStream_t s);
// columns per chunk of a batched solve launch: four trips of every lane
// group of a block
inline int bnqp_chunk_cols(int L) { return 4 * (64 / L) * 4; }
// ... with the fast-break: one unit for every lane group of a 512-thread
// block (whole units, so a chunk's units are the units a single launch over
// the same columns would form)
inline int bnqp_chunk_cols(int L, int unit) {
    return unit > 1 ? (512 / L) * unit : bnqp_chunk_cols(L);
}

// A batched fit of dense problems launched on a stream without waiting
// (the server's batches of fit requests): each problem's solve layout is its
// nmf_fit layout, so results equal nmf_fit's bitwise; memory is
// stream-ordered.  batched_fit_end releases the host side once the stream
// has passed the launches.
struct BatchedFit;
int batched_fit_start(int32_t count, const nmf_problem *probs, const nmf_opts *opt, hipStream_t stream,
                      BatchedFit **out);
void batched_fit_end(BatchedFit *b);

hipError_t launch_zero_u32(unsigned int *p, int n, hipStream_t s);

// ------------------------------------------------------------------ objective
size_t objective_scratch_bytes(const nmf_matrix *V, int r);
hipError_t launch_objective(const nmf_matrix *V, int r, const nmf_reg *reg, const float *W,
                            const float *Ht, char *scratch, double *dev_out, hipStream_t s);
size_t kkt_partial_bytes(int64_t c);
// Fills the KKT fields of *st from the four residuals of each half (h: the
// H-update's, w: the W-update's; minmap, nonnegativity, complementarity,
// gradient on zero entries).
inline void set_kkt_stats(nmf_stats *st, const double *h, const double *w) {
    st->kkt_h = h[0];
    st->kkt_w = w[0];
    for (int q = 0; q < 3; q++) {
        st->kkt_h_cond[q] = h[q + 1];
        st->kkt_w_cond[q] = w[q + 1];
    }
}
hipError_t launch_kkt(const float *G, int r, const float *P, float hsign, float hadd,
                      const float *X, int64_t c, double *partial, double *dev_out, int64_t stride,
                      hipStream_t s);
// V seen one panel at a time: a panel's sum of squared errors (rows x cols
// block of V at V with leading dimension ld, against W's rows and Ht's rows
// of the panel) into *slot; scratch of loss_panel_scratch_bytes(rows, cols)
size_t loss_panel_scratch_bytes(int64_t rows, int64_t cols);
hipError_t launch_loss_panel(const float *V, int64_t ld, int64_t rows, int64_t cols, const float *W,
                             const float *Ht, int r, double *scratch, double *slot, hipStream_t s);
// Objective from panel sums, in two steps on one scratch (of
// objective_slots_scratch_bytes()): launch_objective_regs takes the
// regularisation sums of (W, Ht) as they are when it runs;
// launch_objective_slots later adds the nslots panel sums in slot order and
// writes loss and J (dev_out[0..1]).
size_t objective_slots_scratch_bytes();
hipError_t launch_objective_regs(const float *W, int64_t m, const float *Ht, int64_t n, int r, char *scratch,
                                 hipStream_t s);
hipError_t launch_objective_slots(const double *slots, int64_t nslots, const nmf_reg *reg, char *scratch,
                                  double *dev_out, hipStream_t s);
// *out = max of in[0..n) (single block)
hipError_t launch_max_ordered(const double *in, int64_t n, double *out, hipStream_t s);

// ------------------------------------------------------------------ fold-in basis
}  // namespace nmfi
struct nmf_basis {
    float *W = nullptr;  // m x r copy
    __bf16 *W16 = nullptr;  // BF16 mode: m x lda16 copy for the sparse fold-in gathers
    int lda16 = 0;
    int64_t m = 0;
    int r = 0;
    float l1 = 0.f, l2 = 0.f;
    nmf_opts opt{};
    nmfi::NqpVariant var{};
    char *ws = nullptr;  // G, Gram scratch
    float *G = nullptr;
};
namespace nmfi {
size_t plan_footprint(const nmf_matrix *V, int r, const nmf_opts *opt);
// The fold-in's solve of c columns whose data-product rows P (c x r) are on
// the stream: zeroes *counter (a kernel, no memset) and launches Algorithm 3
// from x0 = 0 against the basis' Gram.
int basis_solve(const nmf_basis *B, const float *P, int64_t c, float *Ht_new, int32_t *iters,
                unsigned long long *counter, hipStream_t s);
// nmf_fit with stream-ordered plan memory and no host synchronisation (dense
// V): complete once `stream` drains.
int fit_stream_ordered(const nmf_matrix *V, int32_t r, const nmf_reg *reg, const nmf_opts *opt, float *W,
                       float *Ht, hipStream_t stream);

// ------------------------------------------------------------------ misc
hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s);
int device_cu_count();
int validate_opts(const nmf_opts *o);
// Scans n floats for NaN/Inf (and, when nonneg != 0, negative values);
// synchronises the stream.  Returns NMF_OK or NMF_E_NONFINITE.
int check_values(const float *x, int64_t n, int nonneg, hipStream_t s);

}  // namespace nmfi
