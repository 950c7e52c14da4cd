// nmf_foldin_noalloc: the fold-in of sparse columns (the E-step alone against
// a resident basis) with no device allocation, for callers that cannot
// allocate (code under stream capture, tight serving loops).  Its scratch --
// the solve's work counter and the data-product rows P (c x r) -- is one
// file-scope device array, held by every GPU the library runs on until the
// process ends.  Every call on a GPU uses that GPU's array: calls that
// overlap on one GPU race (serialise them, e.g. on one stream).
#include <mutex>

#include "nmf_internal.h"

using namespace nmfi;

static_assert(NMF_FOLDIN_NOALLOC_BYTES % 256 == 0, "scratch size must be a multiple of 256 bytes");
static __device__ __align__(256) char scratch[NMF_FOLDIN_NOALLOC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
constexpr size_t kCounterBytes = 256;  // the work counter, then P

std::mutex g_mu;
char *g_ptr[kMaxDevices] = {};  // scratch's device address on each GPU (host code uses only these)

// The scratch array's address on the current device, looked up once per
// device with that device current.
int scratch_ptr(char **out) {
    int dev = 0;
    NMF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(NMF_E_UNSUPPORTED, "device %d is beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(NMF_E_DEVICE, "hipGetSymbolAddress(scratch) gave a null address");
        g_ptr[dev] = (char *)p;
    }
    *out = g_ptr[dev];
    return NMF_OK;
}

}  // namespace

extern "C" int nmf_foldin_noalloc(const nmf_basis *B, const nmf_matrix *Vnew, float *Ht_new, int32_t *iters,
                                  void *stream) {
    if (!B) return fail(NMF_E_INVAL, "basis is NULL");
    if (!Vnew || !Ht_new) return fail(NMF_E_INVAL, "Vnew and Ht_new must be non-NULL");
    if (Vnew->rows != B->m) return fail(NMF_E_INVAL, "Vnew must have m = %lld rows", (long long)B->m);
    if (Vnew->cols < 0) return fail(NMF_E_INVAL, "Vnew must have >= 0 columns");
    if (Vnew->kind != NMF_CSR)
        return fail(NMF_E_UNSUPPORTED, "nmf_foldin_noalloc takes sparse columns only (CSR(Vnew') in t_*)");
    if (!Vnew->t_rowptr || !Vnew->t_colidx || !Vnew->t_vals)
        return fail(NMF_E_INVAL, "sparse Vnew must be given as CSR(Vnew') (t_* arrays)");
    if (Vnew->cols == 0) return NMF_OK;
    const int64_t c = Vnew->cols;
    const int r = B->r;
    const int64_t max_cols = (int64_t)((NMF_FOLDIN_NOALLOC_BYTES - kCounterBytes) / ((size_t)r * sizeof(float)));
    if (c > max_cols)
        return fail(NMF_E_INVAL,
                    "nmf_foldin_noalloc holds at most %lld columns at r = %d (its scratch is %d bytes); got %lld",
                    (long long)max_cols, r, NMF_FOLDIN_NOALLOC_BYTES, (long long)c);
    char *base = nullptr;
    if (int st = scratch_ptr(&base)) return st;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *counter = (unsigned long long *)base;
    float *P = (float *)(base + kCounterBytes);
    hipError_t e = B->W16 ? launch_spmm_rows16(Vnew->t_rowptr, c, Vnew->t_colidx, Vnew->t_vals, B->W16, B->lda16,
                                               r, P, s)
                          : launch_spmm_rows(Vnew->t_rowptr, c, Vnew->t_colidx, Vnew->t_vals, B->W, r, P, s);
    if (e != hipSuccess) return hip_fail(e, "fold-in product");
    return basis_solve(B, P, c, Ht_new, iters, counter, s);
}
