// Host orchestration: the building-block entry points, the fit plan
// (Algorithm 2 with the regularised NQPs of Section 3.5), the objective, and
// fold-in against a resident basis (the E-step alone).
#include <math.h>

#include <vector>

#include <algorithm>

#include "nmf_internal.h"

using namespace nmfi;

namespace nmfi {

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

int validate_matrix(const nmf_matrix *V, bool need_transpose_ok) {
    (void)need_transpose_ok;
    if (!V) return fail(NMF_E_INVAL, "matrix descriptor is NULL");
    if (V->rows < 1 || V->cols < 1) return fail(NMF_E_INVAL, "V must have at least one row and column");
    if (V->rows > INT32_MAX || V->cols > INT32_MAX) return fail(NMF_E_INVAL, "V dimensions exceed int32");
    if (V->kind == NMF_DENSE) {
        if (!V->dense) return fail(NMF_E_INVAL, "dense V pointer is NULL");
        if (V->ld < V->cols) return fail(NMF_E_INVAL, "ld (%lld) < cols (%lld)", (long long)V->ld, (long long)V->cols);
    } else if (V->kind == NMF_CSR) {
        if (!V->rowptr || !V->colidx || !V->vals) return fail(NMF_E_INVAL, "CSR arrays must be non-NULL");
        if (V->nnz < 0 || V->nnz > INT32_MAX) return fail(NMF_E_INVAL, "nnz must be in [0, 2^31)");
        const bool any_t = V->t_rowptr || V->t_colidx || V->t_vals;
        const bool all_t = V->t_rowptr && V->t_colidx && V->t_vals;
        if (any_t && !all_t) return fail(NMF_E_INVAL, "give all three CSR(V') arrays or none");
    } else {
        return fail(NMF_E_INVAL, "unknown matrix kind %d", V->kind);
    }
    return NMF_OK;
}

// ------------------------------------------------------------------ CSR transpose
// CSR(V') from CSR(V) by a counting sort on the column index that keeps the
// rows ascending inside each column (what the products' fixed summation order
// relies on).  The rows are cut into B contiguous blocks; block b counts its
// entries per column, an exclusive scan over the blocks and the columns gives
// every (block, column) its first output position, and then block b places
// its rows one after another (a barrier between rows), each column's cursor
// advanced by atomics: within a column, lower blocks come first and inside a
// block lower rows come first.

__global__ void k_zero_i32(int32_t *__restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// cnt[b * n + j] = entries of column j in rows [b * rows_per, (b + 1) * rows_per)
__global__ __launch_bounds__(256) void k_tr_count(const int32_t *__restrict__ rowptr, int64_t m,
                                                  const int32_t *__restrict__ colidx, int64_t rows_per, int64_t n,
                                                  int32_t *__restrict__ cnt) {
    const int64_t i0 = (int64_t)blockIdx.x * rows_per, i1 = min(m, i0 + rows_per);
    int32_t *c = cnt + (int64_t)blockIdx.x * n;
    if (i0 >= i1) return;
    for (int64_t t = rowptr[i0] + threadIdx.x; t < rowptr[i1]; t += blockDim.x) atomicAdd(&c[colidx[t]], 1);
}

// Per column j: cnt[b][j] <- sum over earlier blocks (the block's offset
// inside column j), colcnt[j] <- the column's total.
__global__ void k_tr_block_offsets(int32_t *__restrict__ cnt, int64_t nb, int64_t n, int32_t *__restrict__ colcnt) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        int32_t run = 0;
        for (int64_t b = 0; b < nb; b++) {
            const int32_t v = cnt[b * n + j];
            cnt[b * n + j] = run;
            run += v;
        }
        colcnt[j] = run;
    }
}

// out[0] = 0, out[j + 1] = in[0] + ... + in[j]: one block walks the array in
// chunks of 1024, scanning each in LDS and carrying the running total.
__global__ __launch_bounds__(1024) void k_tr_exclusive_scan(const int32_t *__restrict__ in, int64_t n,
                                                            int32_t *__restrict__ out) {
    __shared__ int32_t buf[1024];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) { carry = 0; out[0] = 0; }
    __syncthreads();
    for (int64_t base = 0; base < n; base += 1024) {
        const int64_t j = base + threadIdx.x;
        buf[threadIdx.x] = j < n ? in[j] : 0;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan (Hillis-Steele)
            const int32_t v = threadIdx.x >= (unsigned)off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += v;
            __syncthreads();
        }
        if (j < n) out[j + 1] = carry + buf[threadIdx.x];
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
}

// Block b places the entries of its rows, row after row.
__global__ __launch_bounds__(256) void k_tr_scatter(const int32_t *__restrict__ rowptr, int64_t m,
                                                    const int32_t *__restrict__ colidx, const float *__restrict__ vals,
                                                    int64_t rows_per, int64_t n, const int32_t *__restrict__ trp,
                                                    int32_t *__restrict__ cur, int32_t *__restrict__ tci,
                                                    float *__restrict__ tv) {
    const int64_t i0 = (int64_t)blockIdx.x * rows_per, i1 = min(m, i0 + rows_per);
    int32_t *c = cur + (int64_t)blockIdx.x * n;
    for (int64_t i = i0; i < i1; i++) {
        for (int32_t t = rowptr[i] + (int32_t)threadIdx.x; t < rowptr[i + 1]; t += (int32_t)blockDim.x) {
            const int32_t j = colidx[t];
            const int32_t pos = trp[j] + atomicAdd(&c[j], 1);
            tci[pos] = (int32_t)i;
            tv[pos] = vals[t];
        }
        __syncthreads();  // this row's cursor advances before the next row reads them
    }
}

// Row blocks for the counting sort: as many as keep the (block x column)
// cursors within about 64 MB, at most 256, at least one.
static int64_t transpose_blocks(int64_t m, int64_t n) {
    int64_t nb = (int64_t)(16 << 20) / std::max<int64_t>(n, 1);
    nb = std::min<int64_t>(std::min<int64_t>(nb, 256), m);
    return std::max<int64_t>(nb, 1);
}

// CSR(V') from CSR(V) (counting sort, rows ascending inside each column).
// Outputs are hipMalloc'd and owned by the caller.
int csr_transpose(const nmf_matrix *V, int32_t **trp, int32_t **tci, float **tv, hipStream_t s) {
    const int64_t m = V->rows, n = V->cols, nnz = V->nnz;
    *trp = nullptr; *tci = nullptr; *tv = nullptr;
    NMF_HIP(hipMalloc((void **)trp, (n + 1) * sizeof(int32_t)));
    NMF_HIP(hipMalloc((void **)tci, (nnz > 0 ? nnz : 1) * sizeof(int32_t)));
    NMF_HIP(hipMalloc((void **)tv, (nnz > 0 ? nnz : 1) * sizeof(float)));
    const int64_t nb = transpose_blocks(m, n), rows_per = (m + nb - 1) / nb;
    int32_t *cnt = nullptr, *colcnt = nullptr;
    NMF_HIP(hipMalloc((void **)&cnt, (size_t)nb * n * sizeof(int32_t)));
    NMF_HIP(hipMalloc((void **)&colcnt, (size_t)n * sizeof(int32_t)));
    const unsigned gcols = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero_i32, dim3(4096), dim3(256), 0, s, cnt, nb * n);
    hipLaunchKernelGGL(k_tr_count, dim3((unsigned)nb), dim3(256), 0, s, V->rowptr, m, V->colidx, rows_per, n, cnt);
    hipLaunchKernelGGL(k_tr_block_offsets, dim3(gcols), dim3(256), 0, s, cnt, nb, n, colcnt);
    hipLaunchKernelGGL(k_tr_exclusive_scan, dim3(1), dim3(1024), 0, s, colcnt, n, *trp);
    hipLaunchKernelGGL(k_tr_scatter, dim3((unsigned)nb), dim3(256), 0, s, V->rowptr, m, V->colidx, V->vals, rows_per,
                       n, *trp, cnt, *tci, *tv);
    NMF_HIP(hipGetLastError());
    NMF_HIP(hipStreamSynchronize(s));
    (void)hipFree(cnt); (void)hipFree(colcnt);
    return NMF_OK;
}

static int host_rowptr(const int32_t *d, int64_t nrows, std::vector<int32_t> &h, hipStream_t s) {
    h.resize(nrows + 1);
    NMF_HIP(hipMemcpyAsync(h.data(), d, (nrows + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    NMF_HIP(hipStreamSynchronize(s));
    if (h[0] != 0) return fail(NMF_E_INVAL, "rowptr[0] must be 0");
    for (int64_t i = 0; i < nrows; i++)
        if (h[i + 1] < h[i]) return fail(NMF_E_INVAL, "rowptr must be non-decreasing");
    return NMF_OK;
}

}  // namespace nmfi

// ============================================================ building blocks
extern "C" int nmf_gram(const float *A, int64_t k, int32_t r, float l2, int32_t precision, float *G,
                        void *stream) {
    if (r < 1 || r > NMF_MAX_RANK) return fail(NMF_E_INVAL, "r must be in [1, %d]", NMF_MAX_RANK);
    if (k < 1) return fail(NMF_E_INVAL, "k must be >= 1");
    if (!A || !G) return fail(NMF_E_INVAL, "A and G must be non-NULL");
    if (precision != NMF_FP32 && precision != NMF_BF16) return fail(NMF_E_INVAL, "bad precision");
    hipStream_t s = (hipStream_t)stream;
    float *scratch = nullptr;
    NMF_HIP(hipMallocAsync((void **)&scratch, gram_scratch_bytes(r, k), s));
    hipError_t e = launch_gram(A, k, r, l2, precision, G, scratch, s);
    hipError_t e2 = hipFreeAsync(scratch, s);
    if (e != hipSuccess) return hip_fail(e, "nmf_gram");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
    return NMF_OK;
}

extern "C" int nmf_dense_product_time(const float *V, int64_t m, int64_t n, int64_t ld, int32_t trans, int32_t r,
                                      const float *A, int32_t precision, int32_t nsplit, int32_t reps, double *ms,
                                      void *stream) {
    if (!V || !A || !ms) return fail(NMF_E_INVAL, "V, A and ms must be non-NULL");
    if (m < 1 || n < 1 || ld < n) return fail(NMF_E_INVAL, "bad dense V (m, n >= 1, ld >= n)");
    if (r < 1 || r > NMF_MAX_RANK) return fail(NMF_E_INVAL, "r must be in [1, %d]", NMF_MAX_RANK);
    if (trans != 0 && trans != 1) return fail(NMF_E_INVAL, "trans must be 0 or 1");
    if (precision != NMF_FP32 && precision != NMF_BF16) return fail(NMF_E_INVAL, "bad precision");
    if (nsplit < 0 || nsplit > 512) return fail(NMF_E_INVAL, "nsplit must be in [0, 512]");
    if (reps < 1) return fail(NMF_E_INVAL, "reps must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    const bool bf16 = precision == NMF_BF16;
    const int64_t C = trans ? m : n;
    char *buf = nullptr;
    const size_t pb = ((size_t)C * r * 4 + 255) & ~(size_t)255;
    const size_t vb = bf16 ? (((size_t)m * n * 2 + 255) & ~(size_t)255) : 0;
    const size_t sb = dense_scratch_bytes_forced(m, n, r, nsplit);
    NMF_HIP(hipMallocAsync((void **)&buf, pb + vb + sb, s));
    float *P = (float *)buf;
    __bf16 *v16 = bf16 ? (__bf16 *)(buf + pb) : nullptr;
    float *scratch = (float *)(buf + pb + vb);
    hipError_t e = hipSuccess;
    if (bf16) e = trans ? launch_to_bf16(V, m, n, ld, v16, s) : launch_to_bf16_t(V, m, n, ld, v16, s);
    const void *src = bf16 ? (const void *)v16 : (const void *)V;
    auto once = [&]() {
        return launch_dense_product(src, bf16, m, n, bf16 ? n : ld, (bf16 && !trans) ? v16 : nullptr, trans, A, r,
                                    P, scratch, s, nsplit);
    };
    if (e == hipSuccess) e = once();  // warm-up
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e == hipSuccess) e = hipEventRecord(ev[0], s);
    for (int i = 0; i < reps && e == hipSuccess; i++) e = once();
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float el = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&el, ev[0], ev[1]);
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    (void)hipFreeAsync(buf, s);
    if (e != hipSuccess) return hip_fail(e, "nmf_dense_product_time");
    *ms = (double)el / reps;
    return NMF_OK;
}

extern "C" int nmf_product(const nmf_matrix *V, int32_t trans, int32_t r, const float *A,
                           int32_t precision, float *P, void *stream) {
    if (int st = validate_matrix(V, true)) return st;
    if (r < 1 || r > NMF_MAX_RANK) return fail(NMF_E_INVAL, "r must be in [1, %d]", NMF_MAX_RANK);
    if (!A || !P) return fail(NMF_E_INVAL, "A and P must be non-NULL");
    if (trans != 0 && trans != 1) return fail(NMF_E_INVAL, "trans must be 0 or 1");
    if (precision != NMF_FP32 && precision != NMF_BF16) return fail(NMF_E_INVAL, "bad precision");
    hipStream_t s = (hipStream_t)stream;
    const int64_t m = V->rows, n = V->cols;
    if (V->kind == NMF_DENSE) {
        const void *src = V->dense;
        __bf16 *v16 = nullptr;
        if (precision == NMF_BF16) {  // the BF16 copy the product reads along k
            NMF_HIP(hipMallocAsync((void **)&v16, (size_t)m * n * sizeof(__bf16), s));
            if (trans) NMF_HIP(launch_to_bf16(V->dense, m, n, V->ld, v16, s));
            else NMF_HIP(launch_to_bf16_t(V->dense, m, n, V->ld, v16, s));
            src = v16;
        }
        float *scratch = nullptr;
        NMF_HIP(hipMallocAsync((void **)&scratch, dense_scratch_bytes(m, n, r), s));
        hipError_t e = launch_dense_product(src, precision == NMF_BF16, m, n,
                                            precision == NMF_BF16 ? n : V->ld,
                                            (precision == NMF_BF16 && !trans) ? v16 : nullptr, trans,
                                            A, r, P, scratch, s);
        (void)hipFreeAsync(scratch, s);
        if (v16) (void)hipFreeAsync(v16, s);
        if (e != hipSuccess) return hip_fail(e, "nmf_product");
        return NMF_OK;
    }
    // CSR: trans = 1 runs over CSR(V) with A = Ht; trans = 0 over CSR(V')
    const int32_t *rp = trans ? V->rowptr : V->t_rowptr;
    const int32_t *ci = trans ? V->colidx : V->t_colidx;
    const float *vv = trans ? V->vals : V->t_vals;
    int32_t *trp = nullptr, *tci = nullptr;
    float *tvv = nullptr;
    if (!rp) {
        if (int st = csr_transpose(V, &trp, &tci, &tvv, s)) return st;
        rp = trp; ci = tci; vv = tvv;
    }
    const int64_t nrows = trans ? m : n;
    std::vector<int32_t> h;
    int st = host_rowptr(rp, nrows, h, s);
    SpmmPlan pl{};
    if (!st) st = build_spmm_plan(h, &pl, s);
    float *partial = nullptr;
    __bf16 *a16 = nullptr;  // BF16: the factor's BF16 copy the gathers read
    const int lda16 = spmm_lda16(r);
    if (!st && pl.nslots > 0) {
        hipError_t e = hipMalloc((void **)&partial, (size_t)pl.nslots * r * sizeof(float));
        if (e != hipSuccess) st = hip_fail(e, "hipMalloc");
    }
    if (!st && precision == NMF_BF16) {
        const int64_t k = trans ? n : m;
        hipError_t e = hipMalloc((void **)&a16, (size_t)(k > 0 ? k : 1) * lda16 * sizeof(__bf16));
        if (e == hipSuccess) e = launch_rows_to_bf16(A, k, r, lda16, a16, s);
        if (e != hipSuccess) st = hip_fail(e, "BF16 copy of the factor");
    }
    if (!st) {
        hipError_t e = a16 ? launch_spmm16(pl, ci, vv, a16, lda16, r, P, partial, s)
                           : launch_spmm(pl, ci, vv, A, r, P, partial, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "nmf_product");
    }
    free_spmm_plan(&pl);
    if (partial) (void)hipFree(partial);
    if (a16) (void)hipFree(a16);
    if (trp) { (void)hipFree(trp); (void)hipFree(tci); (void)hipFree(tvv); }
    return st;
}

// ============================================================ plan / fit
struct nmf_plan {
    // stream-ordered memory (hipMallocAsync / hipFreeAsync on mem_stream): no
    // device-wide synchronisation when the plan comes and goes (the server's
    // fit requests; dense V only)
    bool async_mem = false;
    hipStream_t mem_stream = nullptr;
    nmf_matrix V{};
    int64_t m = 0, n = 0;
    int r = 0;
    nmf_reg reg{};
    nmf_opts opt{};
    NqpVariant var_h{}, var_w{};  // solve layouts of the H-update (n columns) and W-update (m)
    // CSR
    int32_t *t_rowptr = nullptr, *t_colidx = nullptr;
    float *t_vals = nullptr;
    bool own_t = false;
    SpmmPlan sp_h{}, sp_w{};
    float *sp_partial = nullptr;
    // hot columns of V (the H-update's longest rows of CSR(V')): their products
    // come from a dense m x T copy through the dense product instead of row gathers
    int T_hot = 0, ld_hot = 0;    // ld_hot: T rounded up to 4 (16-byte rows)
    int32_t *hot_idx = nullptr;   // T column indices (device)
    float *V_hot = nullptr;       // m x ld_hot
    __bf16 *V_hot16t = nullptr;   // BF16 mode: T x m, V_hot' in BF16 (the product reads it along k)
    float *P_hot = nullptr;       // T x r
    float *hot_scratch = nullptr; // dense_scratch_bytes(m, T, r)
    // BF16 mode: the fixed factor's BF16 copy (max(m, n) x lda16) that the
    // row gathers read
    __bf16 *A16 = nullptr;
    int lda16 = 0;
    // dense
    __bf16 *V16 = nullptr, *V16t = nullptr;  // BF16 copies of V and V'
    float *dense_scratch = nullptr;
    // workspace
    char *ws = nullptr;
    float *G = nullptr, *gram_scratch = nullptr, *P = nullptr;
    unsigned long long *counter = nullptr, *inner_total = nullptr;
    char *obj_scratch = nullptr;
    double *obj_out = nullptr, *kkt_partial = nullptr, *kkt_out = nullptr;
    // per-phase HIP-event timers
    int prof = 0;  // 0 off; 1 events around every phase; 2 the solve's dispatch only
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    size_t ev_used = 0;
    double ms[NMF_PHASES] = {0, 0, 0, 0};
    int64_t calls[NMF_PHASES] = {0, 0, 0, 0};
};

static void plan_free(nmf_plan *p) {
    if (!p) return;
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    if (p->own_t) { (void)hipFree(p->t_rowptr); (void)hipFree(p->t_colidx); (void)hipFree(p->t_vals); }
    free_spmm_plan(&p->sp_h);
    free_spmm_plan(&p->sp_w);
    if (p->sp_partial) (void)hipFree(p->sp_partial);
    if (p->hot_idx) (void)hipFree(p->hot_idx);
    if (p->V_hot) (void)hipFree(p->V_hot);
    if (p->V_hot16t) (void)hipFree(p->V_hot16t);
    if (p->P_hot) (void)hipFree(p->P_hot);
    if (p->hot_scratch) (void)hipFree(p->hot_scratch);
    if (p->A16) (void)hipFree(p->A16);
    auto rel = [p](void *x) {
        if (!x) return;
        if (p->async_mem) (void)hipFreeAsync(x, p->mem_stream);
        else (void)hipFree(x);
    };
    rel(p->V16);
    rel(p->V16t);
    rel(p->dense_scratch);
    rel(p->ws);
    delete p;
}

static hipError_t plan_malloc(const nmf_plan *p, void **ptr, size_t bytes) {
    return p->async_mem ? hipMallocAsync(ptr, bytes, p->mem_stream) : hipMalloc(ptr, bytes);
}

// Hot columns of a CSR V: a column j with c_j stored entries costs the
// H-update c_j gathered rows of W (4r bytes each, from cache), and costs the
// dense product about m (4 bytes + 2r flop).  At the gather and MFMA rates
// measured on MI355X the dense side wins from about c_j ~ m/32 on (a second
// slab of 128 columns adds about 0.4 us per column to the dense product, a
// column's gathers cost c_j x 400 bytes at 5.8 TB/s); columns with
// c_j >= max(m/24, 256) are taken, the longest first (ties: lower index):
// all of them up to 127, else 128 or 256 (whole 128-row slabs of the dense
// product), and only when there are at least 4.
static int choose_hot_columns(nmf_plan *p, const std::vector<int32_t> &t_rowptr,
                              std::vector<char> &hot, hipStream_t s) {
    const int64_t n = p->n, m = p->m;
    const int64_t thr = std::max<int64_t>((m + 23) / 24, 256);
    std::vector<int32_t> cand;
    for (int64_t j = 0; j < n; j++)
        if (t_rowptr[j + 1] - t_rowptr[j] >= thr) cand.push_back((int32_t)j);
    std::stable_sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) {
        return t_rowptr[a + 1] - t_rowptr[a] > t_rowptr[b + 1] - t_rowptr[b];
    });
    // whole 128-row slabs of the dense product once there are enough
    if (cand.size() >= 128) cand.resize(std::min<size_t>(cand.size(), 256) / 128 * 128);
    if (cand.size() < 4) return NMF_OK;
    std::sort(cand.begin(), cand.end());  // slots in column order
    const int T = (int)cand.size(), ldT = (T + 3) / 4 * 4;
    hot.assign(n, 0);
    std::vector<int32_t> slot(n, -1);
    for (int t = 0; t < T; t++) {
        hot[cand[t]] = 1;
        slot[cand[t]] = t;
    }
    int32_t *dslot = nullptr;
    hipError_t e = hipMalloc((void **)&p->hot_idx, T * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&dslot, n * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&p->V_hot, (size_t)m * ldT * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&p->P_hot, (size_t)T * p->r * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&p->hot_scratch, dense_scratch_bytes(m, T, p->r));
    if (e == hipSuccess) e = hipMemcpyAsync(p->hot_idx, cand.data(), T * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dslot, slot.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_hot_scatter_v(p->V.rowptr, m, p->V.colidx, p->V.vals, dslot, ldT, p->V_hot, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (dslot) (void)hipFree(dslot);
    if (e != hipSuccess) return hip_fail(e, "hot columns");
    p->T_hot = T;
    p->ld_hot = ldT;
    return NMF_OK;
}

static int plan_create(const nmf_matrix *V, int32_t r, const nmf_reg *reg, const nmf_opts *opt,
                       nmf_plan **out, void *stream, bool async_mem);

extern "C" int nmf_plan_create(const nmf_matrix *V, int32_t r, const nmf_reg *reg, const nmf_opts *opt,
                               nmf_plan **out, void *stream) {
    return plan_create(V, r, reg, opt, out, stream, false);
}

static int plan_create(const nmf_matrix *V, int32_t r, const nmf_reg *reg, const nmf_opts *opt,
                       nmf_plan **out, void *stream, bool async_mem) {
    if (!out) return fail(NMF_E_INVAL, "out is NULL");
    *out = nullptr;
    if (int st = validate_matrix(V, true)) return st;
    if (r < 1 || r > NMF_MAX_RANK) return fail(NMF_E_INVAL, "r must be in [1, %d] (got %d)", NMF_MAX_RANK, r);
    if (!reg) return fail(NMF_E_INVAL, "reg is NULL");
    if (int st = validate_opts(opt)) return st;
    const float regs[4] = {reg->l1_w, reg->l2_w, reg->l1_h, reg->l2_h};
    for (float v : regs)
        if (!(v >= 0.f) || !isfinite(v)) return fail(NMF_E_INVAL, "regularisation weights must be finite and >= 0");
    if (opt->max_outer < 0) return fail(NMF_E_INVAL, "max_outer must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    if (opt->check_finite) {
        int st = V->kind == NMF_DENSE ? NMF_OK : check_values(V->vals, V->nnz, 1, s);
        if (V->kind == NMF_DENSE) {
            if (V->ld != V->cols) {
                for (int64_t i = 0; i < V->rows && !st; i++) st = check_values(V->dense + i * V->ld, V->cols, 1, s);
            } else {
                st = check_values(V->dense, V->rows * V->cols, 1, s);
            }
        }
        if (st) return st;
    }
    nmf_plan *p = new nmf_plan();
    p->async_mem = async_mem && V->kind == NMF_DENSE;
    p->mem_stream = s;
    p->V = *V; p->m = V->rows; p->n = V->cols; p->r = r; p->reg = *reg; p->opt = *opt;
    p->var_h = nqp_pick(r, p->n, opt->lanes);
    p->var_w = nqp_pick(r, p->m, opt->lanes);
    if (!p->var_h.E || !p->var_w.E) {
        delete p;
        return fail(NMF_E_INVAL, "lanes = %d cannot hold rank %d", opt->lanes, r);
    }
    int st = NMF_OK;
    if (V->kind == NMF_CSR) {
        if (!V->t_rowptr) {
            st = csr_transpose(V, &p->t_rowptr, &p->t_colidx, &p->t_vals, s);
            p->own_t = true;
        } else {
            p->t_rowptr = (int32_t *)V->t_rowptr; p->t_colidx = (int32_t *)V->t_colidx; p->t_vals = (float *)V->t_vals;
        }
        std::vector<int32_t> h;
        if (!st) st = host_rowptr(p->t_rowptr, p->n, h, s);
        std::vector<char> hot;
        if (!st) st = choose_hot_columns(p, h, hot, s);
        if (!st) st = build_spmm_plan(h, &p->sp_h, s, p->T_hot ? &hot : nullptr);
        if (!st) st = host_rowptr(V->rowptr, p->m, h, s);
        if (!st) st = build_spmm_plan(h, &p->sp_w, s);
        if (!st) {
            const int32_t slots = p->sp_h.nslots > p->sp_w.nslots ? p->sp_h.nslots : p->sp_w.nslots;
            if (slots > 0) {
                hipError_t e = hipMalloc((void **)&p->sp_partial, (size_t)slots * r * sizeof(float));
                if (e != hipSuccess) st = hip_fail(e, "hipMalloc");
            }
        }
        if (!st && opt->precision == NMF_BF16) {
            const int64_t kmax = std::max<int64_t>(std::max(p->m, p->n), 1);
            p->lda16 = spmm_lda16(r);
            hipError_t e = hipMalloc((void **)&p->A16, (size_t)kmax * p->lda16 * sizeof(__bf16));
            if (e == hipSuccess && p->T_hot) {  // the hot columns' product on BF16 MFMA
                e = hipMalloc((void **)&p->V_hot16t, (size_t)p->T_hot * p->m * sizeof(__bf16));
                if (e == hipSuccess) e = launch_to_bf16_t(p->V_hot, p->m, p->T_hot, p->ld_hot, p->V_hot16t, s);
            }
            if (e != hipSuccess) st = hip_fail(e, "BF16 copies");
        }
    } else {
        if (opt->precision == NMF_BF16) {
            hipError_t e = plan_malloc(p, (void **)&p->V16, (size_t)p->m * p->n * sizeof(__bf16));
            if (e == hipSuccess) e = plan_malloc(p, (void **)&p->V16t, (size_t)p->m * p->n * sizeof(__bf16));
            if (e == hipSuccess) e = launch_to_bf16(V->dense, p->m, p->n, V->ld, p->V16, s);
            if (e == hipSuccess) e = launch_to_bf16_t(V->dense, p->m, p->n, V->ld, p->V16t, s);
            if (e != hipSuccess) st = hip_fail(e, "BF16 copy of V");
        }
        if (!st) {
            hipError_t e = plan_malloc(p, (void **)&p->dense_scratch, dense_scratch_bytes(p->m, p->n, r));
            if (e != hipSuccess) st = hip_fail(e, "hipMalloc");
        }
    }
    if (!st) {
        const int64_t cmax = p->m > p->n ? p->m : p->n;
        size_t off = 0;
        auto place = [&](size_t bytes) { size_t o = off; off += al256(bytes); return o; };
        const size_t o_cnt = place(2 * sizeof(unsigned long long));
        const size_t o_G = place((size_t)r * r * sizeof(float));
        const size_t o_gs = place(gram_scratch_bytes(r, cmax));
        const size_t o_P = place((size_t)cmax * r * sizeof(float));
        const size_t o_oo = place(4 * sizeof(double));
        const size_t o_ko = place(8 * sizeof(double));
        const size_t o_kp = place(kkt_partial_bytes(cmax));
        const size_t o_os = place(objective_scratch_bytes(V, r));
        hipError_t e = plan_malloc(p, (void **)&p->ws, off);
        if (e != hipSuccess) {
            st = hip_fail(e, "plan workspace");
        } else {
            p->counter = (unsigned long long *)(p->ws + o_cnt);
            p->inner_total = p->counter + 1;
            p->G = (float *)(p->ws + o_G);
            p->gram_scratch = (float *)(p->ws + o_gs);
            p->P = (float *)(p->ws + o_P);
            p->obj_out = (double *)(p->ws + o_oo);
            p->kkt_out = (double *)(p->ws + o_ko);
            p->kkt_partial = (double *)(p->ws + o_kp);
            p->obj_scratch = p->ws + o_os;
        }
    }
    if (!st && !p->async_mem) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "plan set-up");
    }
    if (st) {
        if (p->async_mem) (void)hipStreamSynchronize(s);
        plan_free(p);
        return st;
    }
    *out = p;
    return NMF_OK;
}

namespace nmfi {
// Device bytes nmf_plan_create + nmf_plan_run need for V (the server's
// admission estimate of a full-fit request).
size_t plan_footprint(const nmf_matrix *V, int r, const nmf_opts *opt) {
    const int64_t m = V->rows, n = V->cols, cmax = m > n ? m : n;
    size_t b = 0;
    b += al256(64) + al256((size_t)r * r * 4) + al256(gram_scratch_bytes(r, cmax));
    b += al256((size_t)cmax * r * 4) + 2 * al256(32) + al256((size_t)cmax * 8);
    b += al256(objective_scratch_bytes(V, r));
    if (V->kind == NMF_DENSE) {
        b += al256(dense_scratch_bytes(m, n, r));
        if (opt->precision == NMF_BF16) b += 2 * al256((size_t)m * n * 2);  // V16 and V16t
    } else {
        b += 3 * al256((size_t)(V->nnz + n + 1) * 4);  // CSR(V') when built here
        b += al256((size_t)m * 256 * 4) + al256(dense_scratch_bytes(m, 256, r));  // hot columns, at most
        b += al256((size_t)(V->nnz / SPMM_CHUNK + m + n + 2) * (sizeof(SpChunk) + sizeof(SpSplit)));
        if (opt->precision == NMF_BF16)  // A16 and the hot columns' BF16 copy
            b += al256((size_t)cmax * spmm_lda16(r) * 2) + al256((size_t)m * 256 * 2);
    }
    return b + 65536;
}
}  // namespace nmfi

extern "C" void nmf_plan_destroy(nmf_plan *p) {
    if (!p) return;
    (void)hipDeviceSynchronize();
    plan_free(p);
}

namespace nmfi {

static hipEvent_t next_event(nmf_plan *p) {
    if (p->ev_used == p->ev_pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        p->ev_pool.push_back(e);
    }
    return p->ev_pool[p->ev_used++];
}

// records an event pair around a phase when profiling is on
struct PhaseMark {
    nmf_plan *p;
    int phase;
    hipStream_t s;
    hipEvent_t a = nullptr;
    PhaseMark(nmf_plan *p_, int ph, hipStream_t s_) : p(p_), phase(ph), s(s_) {
        if (p->prof == 1 && (a = next_event(p))) (void)hipEventRecord(a, s);
    }
    ~PhaseMark() {
        if (!a) return;
        hipEvent_t b = next_event(p);
        if (!b) return;
        (void)hipEventRecord(b, s);
        p->pending.push_back({phase, {a, b}});
    }
};

static int collect_timers(nmf_plan *p, hipStream_t s) {
    if (p->pending.empty()) { p->ev_used = 0; return NMF_OK; }
    NMF_HIP(hipStreamSynchronize(s));
    for (auto &q : p->pending) {
        float t = 0.f;
        NMF_HIP(hipEventElapsedTime(&t, q.second.first, q.second.second));
        p->ms[q.first] += t;
        p->calls[q.first] += 1;
    }
    p->pending.clear();
    p->ev_used = 0;
    return NMF_OK;
}

// One half-iteration: X (c x r) <- NQP(A'A + 2 l2 I, -(data product) + l1, X)
static hipError_t half_update(nmf_plan *p, bool h_update, const float *A, float *X, hipStream_t s) {
    const int64_t k = h_update ? p->m : p->n;   // rows of the fixed factor
    const int64_t c = h_update ? p->n : p->m;   // NQPs to solve
    const float l1 = h_update ? p->reg.l1_h : p->reg.l1_w;
    const float l2 = h_update ? p->reg.l2_h : p->reg.l2_w;
    hipError_t e;
    {
        // the Gram also zeroes the solve's work counter; the anti-lopsided
        // rescale happens inside the solve kernel while it stages Gamma
        PhaseMark pm(p, NMF_PHASE_GRAM, s);
        e = launch_gram(A, k, p->r, l2, p->opt.precision, p->G, p->gram_scratch, s, p->counter);
    }
    if (e != hipSuccess) return e;
    {
        PhaseMark pm(p, NMF_PHASE_PRODUCT, s);
        if (p->V.kind == NMF_CSR) {
            const SpmmPlan &pl = h_update ? p->sp_h : p->sp_w;
            const int32_t *ci = h_update ? p->t_colidx : p->V.colidx;
            const float *vv = h_update ? p->t_vals : p->V.vals;
            if (p->A16) {
                e = launch_rows_to_bf16(A, k, p->r, p->lda16, p->A16, s);
                if (e == hipSuccess) e = launch_spmm16(pl, ci, vv, p->A16, p->lda16, p->r, p->P, p->sp_partial, s);
            } else {
                e = launch_spmm(pl, ci, vv, A, p->r, p->P, p->sp_partial, s);
            }
            if (e == hipSuccess && h_update && p->T_hot) {  // the hot rows: (V_hot' W), then into P
                const bool bf = p->V_hot16t != nullptr;
                e = launch_dense_product(p->V_hot, bf, p->m, p->T_hot, p->ld_hot, p->V_hot16t, 0, A, p->r,
                                         p->P_hot, p->hot_scratch, s);
                if (e == hipSuccess) e = launch_hot_rows_out(p->P_hot, p->hot_idx, p->T_hot, p->r, p->P, s);
            }
        } else {
            const bool bf = p->V16 != nullptr;
            e = launch_dense_product(bf ? (const void *)p->V16 : (const void *)p->V.dense, bf, p->m, p->n,
                                     bf ? p->n : p->V.ld, p->V16t, h_update ? 0 : 1, A, p->r, p->P,
                                     p->dense_scratch, s);
        }
    }
    if (e != hipSuccess) return e;
    NqpParams q{};
    q.gram = p->G; q.P = p->P; q.hsign = -1.f; q.hadd = l1; q.X = X;
    q.ncols = c; q.r = p->r; q.ldp = p->r; q.ldx = p->r;
    q.max_inner = p->opt.max_inner; q.eps = p->opt.eps; q.ls_guard = p->opt.ls_guard ? 1 : 0;
    q.cold = 0; q.iters = nullptr; q.counter = p->counter; q.inner_total = p->inner_total;
    q.unit = p->opt.fast_break_cols;
    if (p->prof == 2) {  // the solve's own dispatch records the pair
        hipEvent_t a = next_event(p), b = a ? next_event(p) : nullptr;
        if (a && b) {
            q.ev_start = a;
            q.ev_stop = b;
            p->pending.push_back({NMF_PHASE_SOLVE, {a, b}});
        }
    }
    PhaseMark pm(p, NMF_PHASE_SOLVE, s);
    return launch_nqp(h_update ? p->var_h : p->var_w, q, s);
}

static int objective_now(nmf_plan *p, const float *W, const float *Ht, double out[2], hipStream_t s) {
    NMF_HIP(launch_objective(&p->V, p->r, &p->reg, W, Ht, p->obj_scratch, p->obj_out, s));
    NMF_HIP(hipMemcpyAsync(out, p->obj_out, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    NMF_HIP(hipStreamSynchronize(s));
    return NMF_OK;
}

}  // namespace nmfi

extern "C" int nmf_plan_run(nmf_plan *p, float *W, float *Ht, int32_t outer, double *trace,
                            nmf_stats *stats, void *stream) {
    if (!p) return fail(NMF_E_INVAL, "plan is NULL");
    if (!W || !Ht) return fail(NMF_E_INVAL, "W and Ht must be non-NULL");
    if (outer < 0) return fail(NMF_E_INVAL, "outer must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    if (p->opt.check_finite) {
        int st = check_values(W, p->m * p->r, 1, s);
        if (!st) st = check_values(Ht, p->n * p->r, 1, s);
        if (st) return st;
    }
    NMF_HIP(launch_zero_u64(p->inner_total, 1, s));
    double ob[2] = {NAN, NAN};
    const int every = p->opt.objective_every > 0 ? p->opt.objective_every : 1;
    if (trace) {
        for (int t = 0; t <= outer; t++) trace[t] = NAN;
        if (int st = objective_now(p, W, Ht, ob, s)) return st;
        trace[0] = ob[0];
    }
    for (int t = 0; t < outer; t++) {
        const bool last = t == outer - 1;
        hipError_t e = half_update(p, true, W, Ht, s);
        if (e == hipSuccess && stats && last)
            e = launch_kkt(p->G, p->r, p->P, -1.f, p->reg.l1_h, Ht, p->n, p->kkt_partial, p->kkt_out, 1, s);
        if (e == hipSuccess) e = half_update(p, false, Ht, W, s);
        if (e == hipSuccess && stats && last)
            e = launch_kkt(p->G, p->r, p->P, -1.f, p->reg.l1_w, W, p->m, p->kkt_partial, p->kkt_out + 4, 1, s);
        if (e != hipSuccess) return hip_fail(e, "outer iteration");
        if (trace && ((t + 1) % every == 0 || last)) {
            if (int st = objective_now(p, W, Ht, ob, s)) return st;
            trace[t + 1] = ob[0];
        }
    }
    if (int st = collect_timers(p, s)) return st;
    if (stats) {
        if (!trace || outer == 0) {
            if (int st = objective_now(p, W, Ht, ob, s)) return st;
        }
        unsigned long long inner = 0;
        double kk[8];
        for (double &v : kk) v = NAN;
        NMF_HIP(hipMemcpyAsync(&inner, p->inner_total, sizeof inner, hipMemcpyDeviceToHost, s));
        if (outer > 0) NMF_HIP(hipMemcpyAsync(kk, p->kkt_out, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
        NMF_HIP(hipStreamSynchronize(s));
        stats->loss = ob[0];
        stats->objective = ob[1];
        set_kkt_stats(stats, kk, kk + 4);
        stats->inner_total = (int64_t)inner;
        stats->outer_done = outer;
        stats->kbar = outer > 0 ? (double)inner / ((double)outer * (double)(p->m + p->n)) : 0.0;
    }
    return NMF_OK;
}

namespace nmfi {
// nmf_fit without host synchronisation: the plan's memory comes and goes
// stream-ordered on `stream` (dense V), so nothing waits for the device and
// no other stream is held up; the results are complete once `stream` drains.
int fit_stream_ordered(const nmf_matrix *V, int32_t r, const nmf_reg *reg, const nmf_opts *opt, float *W,
                       float *Ht, hipStream_t stream) {
    nmf_plan *p = nullptr;
    if (int st = plan_create(V, r, reg, opt, &p, stream, true)) return st;
    int st = nmf_plan_run(p, W, Ht, opt->max_outer, nullptr, nullptr, stream);
    if (!p->async_mem) (void)hipStreamSynchronize(stream);
    plan_free(p);
    return st;
}
}  // namespace nmfi

extern "C" int nmf_fit(const nmf_matrix *V, int32_t r, const nmf_reg *reg, const nmf_opts *opt, float *W,
                       float *Ht, double *trace, nmf_stats *stats, void *stream) {
    nmf_plan *p = nullptr;
    if (int st = nmf_plan_create(V, r, reg, opt, &p, stream)) return st;
    int st = nmf_plan_run(p, W, Ht, opt->max_outer, trace, stats, stream);
    (void)hipStreamSynchronize((hipStream_t)stream);
    plan_free(p);
    return st;
}

extern "C" int nmf_objective(const nmf_matrix *V, int32_t r, const nmf_reg *reg, const float *W,
                             const float *Ht, double *loss_host, double *objective_host, void *stream) {
    if (int st = validate_matrix(V, false)) return st;
    if (r < 1 || r > NMF_MAX_RANK) return fail(NMF_E_INVAL, "r must be in [1, %d]", NMF_MAX_RANK);
    if (!reg || !W || !Ht) return fail(NMF_E_INVAL, "reg, W and Ht must be non-NULL");
    hipStream_t s = (hipStream_t)stream;
    char *scratch = nullptr;
    const size_t bytes = objective_scratch_bytes(V, r) + 256;
    NMF_HIP(hipMallocAsync((void **)&scratch, bytes, s));
    double *dout = (double *)scratch;
    hipError_t e = launch_objective(V, r, reg, W, Ht, scratch + 256, dout, s);
    double h[2] = {NAN, NAN};
    if (e == hipSuccess) e = hipMemcpyAsync(h, dout, sizeof h, hipMemcpyDeviceToHost, s);
    (void)hipFreeAsync(scratch, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "nmf_objective");
    if (loss_host) *loss_host = h[0];
    if (objective_host) *objective_host = h[1];
    return NMF_OK;
}

// ============================================================ fold-in
// Column count the fold-in solve layout is chosen for.
constexpr int64_t kFoldinLayoutCols = 8192;

extern "C" int nmf_basis_create(const float *W, int64_t m, int32_t r, float l1, float l2,
                                const nmf_opts *opt, nmf_basis **out, void *stream) {
    if (!out) return fail(NMF_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!W) return fail(NMF_E_INVAL, "W is NULL");
    if (m < 1) return fail(NMF_E_INVAL, "m must be >= 1");
    if (r < 1 || r > NMF_MAX_RANK) return fail(NMF_E_INVAL, "r must be in [1, %d]", NMF_MAX_RANK);
    if (!(l1 >= 0.f) || !(l2 >= 0.f) || !isfinite(l1) || !isfinite(l2))
        return fail(NMF_E_INVAL, "l1 and l2 must be finite and >= 0");
    if (int st = validate_opts(opt)) return st;
    hipStream_t s = (hipStream_t)stream;
    // One solve layout for every fold-in of this basis (so a column's result
    // never depends on the request or batch it arrives in), chosen for
    // batches of a few thousand columns unless opt->lanes forces it.
    const NqpVariant var = nqp_pick(r, kFoldinLayoutCols, opt->lanes);
    if (!var.E) return fail(NMF_E_INVAL, "lanes = %d cannot hold rank %d", opt->lanes, r);
    nmf_basis *b = new nmf_basis();
    b->m = m; b->r = r; b->l1 = l1; b->l2 = l2; b->opt = *opt;
    b->var = var;
    const size_t oG = 0, oS = al256((size_t)r * r * 4), total = oS + al256(gram_scratch_bytes(r, m));
    hipError_t e = hipMalloc((void **)&b->W, (size_t)m * r * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&b->ws, total);
    if (e == hipSuccess) {
        b->G = (float *)(b->ws + oG);
        e = hipMemcpyAsync(b->W, W, (size_t)m * r * sizeof(float), hipMemcpyDeviceToDevice, s);
    }
    if (e == hipSuccess) e = launch_gram(b->W, m, r, l2, opt->precision, b->G, (float *)(b->ws + oS), s);
    if (e == hipSuccess && opt->precision == NMF_BF16) {
        b->lda16 = spmm_lda16(r);
        e = hipMalloc((void **)&b->W16, (size_t)m * b->lda16 * sizeof(__bf16));
        if (e == hipSuccess) e = launch_rows_to_bf16(b->W, m, r, b->lda16, b->W16, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        if (b->W) (void)hipFree(b->W);
        if (b->W16) (void)hipFree(b->W16);
        if (b->ws) (void)hipFree(b->ws);
        delete b;
        return hip_fail(e, "nmf_basis_create");
    }
    *out = b;
    return NMF_OK;
}

extern "C" void nmf_basis_destroy(nmf_basis *b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    (void)hipFree(b->W);
    if (b->W16) (void)hipFree(b->W16);
    (void)hipFree(b->ws);
    delete b;
}

namespace nmfi {
// Fold-in of c columns whose product rows P (c x r) the caller's stream will
// produce: launches the solve.
int basis_solve(const nmf_basis *B, const float *P, int64_t c, float *Ht_new, int32_t *iters,
                unsigned long long *counter, hipStream_t s) {
    NMF_HIP(launch_zero_u64(counter, 1, s));
    NqpParams q{};
    q.gram = B->G; q.P = P; q.hsign = -1.f; q.hadd = B->l1; q.X = Ht_new;
    q.ncols = c; q.r = B->r; q.ldp = B->r; q.ldx = B->r;
    q.max_inner = B->opt.max_inner; q.eps = B->opt.eps; q.ls_guard = B->opt.ls_guard ? 1 : 0;
    q.cold = 1; q.iters = iters; q.counter = counter; q.inner_total = nullptr;
    q.unit = B->opt.fast_break_cols;
    NMF_HIP(launch_nqp(B->var, q, s));
    return NMF_OK;
}
}  // namespace nmfi

extern "C" int nmf_foldin(const nmf_basis *B, const nmf_matrix *Vnew, float *Ht_new, int32_t *iters,
                          void *stream) {
    if (!B) return fail(NMF_E_INVAL, "basis is NULL");
    if (!Vnew || !Ht_new) return fail(NMF_E_INVAL, "Vnew and Ht_new must be non-NULL");
    if (Vnew->rows != B->m) return fail(NMF_E_INVAL, "Vnew must have m = %lld rows", (long long)B->m);
    if (Vnew->cols < 0) return fail(NMF_E_INVAL, "Vnew must have >= 0 columns");
    if (Vnew->cols == 0) return NMF_OK;
    const int64_t c = Vnew->cols;
    const int r = B->r;
    hipStream_t s = (hipStream_t)stream;
    if (Vnew->kind == NMF_DENSE) {
        if (!Vnew->dense || Vnew->ld < c) return fail(NMF_E_INVAL, "dense Vnew needs a pointer and ld >= cols");
    } else if (Vnew->kind == NMF_CSR) {
        if (!Vnew->t_rowptr || !Vnew->t_colidx || !Vnew->t_vals)
            return fail(NMF_E_INVAL, "sparse Vnew must be given as CSR(Vnew') (t_* arrays)");
    } else {
        return fail(NMF_E_INVAL, "unknown matrix kind");
    }
    // per-call workspace: counter, P (c x r), dense scratch
    const size_t pbytes = al256((size_t)c * r * sizeof(float));
    const size_t dbytes = Vnew->kind == NMF_DENSE ? dense_scratch_bytes(B->m, c, r) : 0;
    char *ws = nullptr;
    NMF_HIP(hipMallocAsync((void **)&ws, 256 + pbytes + dbytes, s));
    unsigned long long *counter = (unsigned long long *)ws;
    float *P = (float *)(ws + 256);
    hipError_t e;
    if (Vnew->kind == NMF_DENSE)
        e = launch_dense_product(Vnew->dense, 0, B->m, c, Vnew->ld, nullptr, 0, B->W, r, P,
                                 (float *)(ws + 256 + pbytes), s);
    else if (B->W16)
        e = launch_spmm_rows16(Vnew->t_rowptr, c, Vnew->t_colidx, Vnew->t_vals, B->W16, B->lda16, r, P, s);
    else
        e = launch_spmm_rows(Vnew->t_rowptr, c, Vnew->t_colidx, Vnew->t_vals, B->W, r, P, s);
    int st = NMF_OK;
    if (e != hipSuccess) st = hip_fail(e, "fold-in product");
    if (!st) st = basis_solve(B, P, c, Ht_new, iters, counter, s);
    (void)hipFreeAsync(ws, s);
    return st;
}

extern "C" int nmf_plan_profile(nmf_plan *p, int32_t mode) {
    if (!p) return fail(NMF_E_INVAL, "plan is NULL");
    if (mode < 0 || mode > 2) return fail(NMF_E_INVAL, "profile mode must be 0, 1 or 2 (got %d)", mode);
    p->prof = mode;
    for (int i = 0; i < NMF_PHASES; i++) { p->ms[i] = 0.0; p->calls[i] = 0; }
    p->pending.clear();
    p->ev_used = 0;
    return NMF_OK;
}

extern "C" int nmf_plan_timers(const nmf_plan *p, double *ms, int64_t *calls) {
    if (!p || !ms || !calls) return fail(NMF_E_INVAL, "plan, ms and calls must be non-NULL");
    for (int i = 0; i < NMF_PHASES; i++) { ms[i] = p->ms[i]; calls[i] = p->calls[i]; }
    return NMF_OK;
}
