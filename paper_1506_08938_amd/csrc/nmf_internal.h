// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

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

// ------------------------------------------------------------------ misc
int device_cu_count();
int validate_opts(const nmf_opts *o);
// Scans n floats for NaN/Inf (and, when nonneg != 0, negative values);
// synchronises the stream.  Returns NMF_OK or NMF_E_NONFINITE.
int check_values(const float *x, int64_t n, int nonneg, hipStream_t s);

}  // namespace nmfi
