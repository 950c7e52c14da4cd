// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "nmf.h"

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
// Rescaled problem of Algorithm 3 as the solve kernel reads it.
struct RescaledHessian {
    float *Q;    // R x R, row-major, symmetric, unit diagonal (pads and frozen
                 // coordinates: identity rows/columns)
    float *dsq;  // R: sqrt(Gamma_ii); 0 marks a frozen or pad coordinate
    int R;       // padded size (>= r) the solve kernel was built for
};

struct NqpParams {
    const float *Q;      // R x R rescaled Hessian
    const float *dsq;    // R
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
    unsigned long long *counter;       // work counter; zeroed by the rescale kernel
    unsigned long long *inner_total;   // optional accumulator of iterations
};

// Kernel variant (entries per lane E, lanes per column L) for rank r.
struct NqpVariant {
    int E, L;
};
NqpVariant nqp_pick(int r);
int nqp_padded(int r);

// Launches the rescale (Gamma -> Q, dsq; also zeroes the work counter).
hipError_t launch_rescale(const float *gram, int r, int R, float *Q, float *dsq,
                          unsigned long long *counter, hipStream_t s);
// Launches the persistent solve kernel for the given variant.
hipError_t launch_nqp(const NqpVariant &v, const NqpParams &p, hipStream_t s);
hipError_t launch_nqp_l1(int E, const NqpParams &p, hipStream_t s);
hipError_t launch_nqp_l2(int E, const NqpParams &p, hipStream_t s);
hipError_t launch_nqp_l4(int E, const NqpParams &p, hipStream_t s);

// ------------------------------------------------------------------ products
constexpr int SPMM_CHUNK = 512;  // stored entries per SpMM work item

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
int build_spmm_plan(const std::vector<int32_t> &rowptr, SpmmPlan *pl, hipStream_t s);
void free_spmm_plan(SpmmPlan *pl);
hipError_t launch_spmm(const SpmmPlan &pl, const int32_t *colidx, const float *vals, const float *A,
                       int r, float *P, float *partial, hipStream_t s);
// one wave per row straight from the row pointers (no split); for short rows
hipError_t launch_spmm_rows(const int32_t *rowptr, int64_t nrows, const int32_t *colidx,
                            const float *vals, const float *A, int r, float *P, hipStream_t s);

size_t gram_scratch_bytes(int r);
hipError_t launch_gram(const float *A, int64_t k, int r, float l2, int precision, float *G,
                       float *scratch, hipStream_t s);

size_t dense_scratch_bytes(int64_t m, int64_t n, int r);
hipError_t launch_dense_product(const void *V, int bf16, int64_t m, int64_t n, int64_t ld,
                                int trans, const float *A, int r, float *P, float *scratch,
                                hipStream_t s);
hipError_t launch_to_bf16(const float *x, int64_t rows, int64_t cols, int64_t ld, __bf16 *y,
                          hipStream_t s);

// ------------------------------------------------------------------ objective
size_t objective_scratch_bytes(const nmf_matrix *V, int r);
hipError_t launch_objective(const nmf_matrix *V, int r, const nmf_reg *reg, const float *W,
                            const float *Ht, char *scratch, double *dev_out, hipStream_t s);
hipError_t launch_kkt(const float *G, int r, const float *P, float hsign, float hadd,
                      const float *X, int64_t c, double *partial, double *dev_out, hipStream_t s);

// ------------------------------------------------------------------ misc
hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s);
int device_cu_count();
int validate_opts(const nmf_opts *o);
// Scans n floats for NaN/Inf (and, when nonneg != 0, negative values);
// synchronises the stream.  Returns NMF_OK or NMF_E_NONFINITE.
int check_values(const float *x, int64_t n, int nonneg, hipStream_t s);

}  // namespace nmfi
