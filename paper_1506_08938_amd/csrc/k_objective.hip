// Double-precision objective and optimality reductions.
//
// Loss 0.5 ||V - W H||_F^2 (the quantity Section 5 reports) and the
// regularised objective J of Section 3.5 (Eq. L1L2NMF with the 1/2 on the
// loss).  Dense V: summed entry by entry, (V_ij - sum_a W_ia H_ja)^2 with the
// inner product in double.  CSR V: the exact expansion ||V||^2 - 2 <V, WH>
// + <W'W, HH'>, which needs only the stored entries.  KKT residual of one
// half's NQPs: max over entries of |min(x, g)| with g = Gamma x + h in the
// original scale (zero exactly at a KKT point).
//
// Every reduction writes per-block partials that a single block then sums in
// index order, so results are bitwise reproducible.
#include "nmf_internal.h"

namespace nmfi {

constexpr int LD_T = 64;  // dense loss tile

// ------------------------------------------------------------ dense loss
__global__ __launch_bounds__(256) void k_loss_dense(const float *__restrict__ V, int64_t ld,
                                                    int64_t m, int64_t n,
                                                    const float *__restrict__ W,
                                                    const float *__restrict__ Ht, int r,
                                                    double *__restrict__ partial) {
    extern __shared__ float sm[];
    float *Ws = sm;               // LD_T x r
    float *Hs = sm + LD_T * r;    // LD_T x r
    __shared__ double red[256];
    const int tid = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.y * LD_T, j0 = (int64_t)blockIdx.x * LD_T;
    for (int e = tid; e < LD_T * r; e += 256) {
        const int row = e / r, a = e - row * r;
        Ws[e] = (i0 + row < m) ? W[(i0 + row) * r + a] : 0.f;
        Hs[e] = (j0 + row < n) ? Ht[(j0 + row) * r + a] : 0.f;
    }
    __syncthreads();
    const int ty = tid >> 4, tx = tid & 15;
    double acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; p++)
#pragma unroll
        for (int q = 0; q < 4; q++) acc[p][q] = 0.0;
    for (int a = 0; a < r; a++) {
        double wv[4], hv[4];
#pragma unroll
        for (int p = 0; p < 4; p++) wv[p] = (double)Ws[(4 * ty + p) * r + a];
#pragma unroll
        for (int q = 0; q < 4; q++) hv[q] = (double)Hs[(4 * tx + q) * r + a];
#pragma unroll
        for (int p = 0; p < 4; p++)
#pragma unroll
            for (int q = 0; q < 4; q++) acc[p][q] = fma(wv[p], hv[q], acc[p][q]);
    }
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < 4; p++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int64_t i = i0 + 4 * ty + p, j = j0 + 4 * tx + q;
            if (i < m && j < n) {
                const double e = (double)V[i * ld + j] - acc[p][q];
                s = fma(e, e, s);
            }
        }
    red[tid] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// ------------------------------------------------------------ CSR cross term
// one wave per row i: sum over stored (i, j) of V_ij * <W_i, H_j> and V_ij^2
__global__ __launch_bounds__(256) void k_loss_csr(const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ colidx,
                                                  const float *__restrict__ vals, int64_t m,
                                                  const float *__restrict__ W,
                                                  const float *__restrict__ Ht, int r,
                                                  double *__restrict__ partial) {
    __shared__ float wrow[4][NMF_MAX_RANK];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + wave;
    double cross = 0.0, vv = 0.0;
    if (i < m) {
        for (int a = lane; a < r; a += 64) wrow[wave][a] = W[i * r + a];
    }
    __syncthreads();
    if (i < m) {
        for (int t = rowptr[i] + lane; t < rowptr[i + 1]; t += 64) {
            const float *h = Ht + (int64_t)colidx[t] * r;
            double d = 0.0;
            for (int a = 0; a < r; a++) d = fma((double)wrow[wave][a], (double)h[a], d);
            const double v = vals[t];
            cross = fma(v, d, cross);
            vv = fma(v, v, vv);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        cross += __shfl_xor(cross, off);
        vv += __shfl_xor(vv, off);
    }
    if (lane == 0 && i < m) {
        partial[2 * i] = cross;
        partial[2 * i + 1] = vv;
    }
}

// ------------------------------------------------------------ double Gram
// block b sums rows [b*rpb, ...) of A'A in double, entries e = tid + 256 q
constexpr int G64_MAXQ = (NMF_MAX_RANK * NMF_MAX_RANK + 255) / 256;

__global__ __launch_bounds__(256) void k_gram64(const float *__restrict__ A, int64_t k, int r,
                                                int64_t rpb, double *__restrict__ partial) {
    __shared__ float rows[16][NMF_MAX_RANK];
    const int tid = threadIdx.x;
    const int nq = (r * r + 255) / 256;
    double acc[G64_MAXQ];
#pragma unroll
    for (int q = 0; q < G64_MAXQ; q++) acc[q] = 0.0;
    const int64_t b0 = (int64_t)blockIdx.x * rpb, b1 = min(k, b0 + rpb);
    for (int64_t t0 = b0; t0 < b1; t0 += 16) {
        for (int e = tid; e < 16 * r; e += 256) {
            const int rr = e / r, a = e - rr * r;
            rows[rr][a] = (t0 + rr < b1) ? A[(t0 + rr) * r + a] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < G64_MAXQ; q++) {
            if (q < nq) {
                const int e = tid + 256 * q;
                if (e < r * r) {
                    const int a = e / r, b = e - (e / r) * r;
#pragma unroll 4
                    for (int rr = 0; rr < 16; rr++)
                        acc[q] = fma((double)rows[rr][a], (double)rows[rr][b], acc[q]);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < G64_MAXQ; q++) {
        const int e = tid + 256 * q;
        if (q < nq && e < r * r) partial[(int64_t)blockIdx.x * r * r + e] = acc[q];
    }
}

// ------------------------------------------------------------ sums
// per block: sum x and sum x^2 over a flat array
__global__ __launch_bounds__(256) void k_sums(const float *__restrict__ x, int64_t n,
                                              double *__restrict__ partial) {
    __shared__ double r1[256], r2[256];
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double v = x[i];
        s1 += v;
        s2 = fma(v, v, s2);
    }
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            r1[threadIdx.x] += r1[threadIdx.x + w];
            r2[threadIdx.x] += r2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = r1[0];
        partial[2 * blockIdx.x + 1] = r2[0];
    }
}

// ------------------------------------------------------------ fixed-order reductions
// out[o] = sum_i in[i * stride + o] for o < width (single block, ordered)
__global__ __launch_bounds__(256) void k_reduce_ordered(const double *__restrict__ in, int64_t count,
                                                        int width, double *__restrict__ out) {
    for (int o = blockIdx.x * 256 + threadIdx.x; o < width; o += gridDim.x * 256) {
        double s = 0.0;
        for (int64_t i = 0; i < count; i++) s += in[i * width + o];
        out[o] = s;
    }
}

// sum over a long array in a fixed order: 256 strided partials, then a tree
__global__ __launch_bounds__(256) void k_sum_ordered(const double *__restrict__ in, int64_t n,
                                                     int64_t stride, int64_t offset,
                                                     double *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += in[i * stride + offset];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// <G1, G2> over r*r doubles
__global__ __launch_bounds__(256) void k_dot_ordered(const double *__restrict__ a,
                                                     const double *__restrict__ b, int64_t n,
                                                     double *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s = fma(a[i], b[i], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// terms: [0] dense sum e^2 | [1] ||V||^2 [2] cross [3] <W'W, HH'> (CSR)
//        [4] sum W [5] sum W^2 [6] sum H [7] sum H^2 ; out: loss, J
__global__ void k_finish(const double *__restrict__ t, int csr, double l1w, double l2w, double l1h,
                         double l2h, double *__restrict__ out) {
    const double loss = csr ? 0.5 * (t[1] - 2.0 * t[2] + t[3]) : 0.5 * t[0];
    out[0] = loss;
    out[1] = loss + l1h * t[6] + l2h * t[7] + l1w * t[4] + l2w * t[5];
}

// ------------------------------------------------------------ KKT residual
// one wave per row j: g = G x_j + hsign P_j + hadd (double); partial[j] =
// max_a |min(x_a, g_a)|
__global__ __launch_bounds__(256) void k_kkt(const float *__restrict__ G, int r,
                                             const float *__restrict__ P, float hsign, float hadd,
                                             const float *__restrict__ X, int64_t c,
                                             double *__restrict__ partial) {
    __shared__ float xs[4][NMF_MAX_RANK];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + wave;
    if (j < c)
        for (int a = lane; a < r; a += 64) xs[wave][a] = X[j * r + a];
    __syncthreads();
    if (j >= c) return;
    double mx = 0.0;
    for (int a = lane; a < r; a += 64) {
        double g = (double)hsign * (double)P[j * r + a] + (double)hadd;
        for (int b = 0; b < r; b++) g = fma((double)G[(int64_t)a * r + b], (double)xs[wave][b], g);
        const double x = xs[wave][a];
        const double v = fabs(x < g ? x : g);
        mx = v > mx ? v : mx;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_xor(mx, off);
        mx = o > mx ? o : mx;
    }
    if (lane == 0) partial[j] = mx;
}

__global__ __launch_bounds__(256) void k_max_ordered(const double *__restrict__ in, int64_t n,
                                                     double *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s = in[i] > s ? in[i] : s;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x + w] > red[threadIdx.x] ? red[threadIdx.x + w] : red[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// ------------------------------------------------------------ host side
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t objective_scratch_bytes(const nmf_matrix *V, int r) {
    const int64_t m = V->rows, n = V->cols;
    size_t b = 0;
    if (V->kind == NMF_DENSE) {
        b += align256((size_t)((n + LD_T - 1) / LD_T) * ((m + LD_T - 1) / LD_T) * sizeof(double));
    } else {
        b += align256((size_t)2 * m * sizeof(double));
        b += 2 * align256((size_t)256 * r * r * sizeof(double));  // Gram partials (reused)
        b += 2 * align256((size_t)r * r * sizeof(double));        // GW, GH
    }
    b += align256(2 * 4096 * sizeof(double)) * 2;  // sums of W and H
    b += align256(16 * sizeof(double));           // terms
    b += align256(2 * sizeof(double));            // out
    return b + 1024;
}

static hipError_t gram64(const float *A, int64_t k, int r, double *partial, double *G,
                         hipStream_t s) {
    int64_t nb = (k + 255) / 256;
    if (nb > 256) nb = 256;
    if (nb < 1) nb = 1;
    int64_t rpb = (k + nb - 1) / nb;
    nb = (k + rpb - 1) / rpb;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_gram64, dim3((unsigned)nb), dim3(256), 0, s, A, k, r, rpb, partial);
    hipLaunchKernelGGL(k_reduce_ordered, dim3((unsigned)((r * r + 255) / 256)), dim3(256), 0, s,
                       partial, nb, r * r, G);
    return hipGetLastError();
}

// Loss and J into dev_out[0..1] (device doubles); scratch of
// objective_scratch_bytes().
hipError_t launch_objective(const nmf_matrix *V, int r, const nmf_reg *reg, const float *W,
                            const float *Ht, char *scratch, double *dev_out, hipStream_t s) {
    const int64_t m = V->rows, n = V->cols;
    char *p = scratch;
    auto take = [&](size_t bytes) { char *q = p; p += align256(bytes); return q; };
    double *terms = (double *)take(16 * sizeof(double));
    hipLaunchKernelGGL(k_reduce_ordered, dim3(1), dim3(256), 0, s, (const double *)nullptr,
                       (int64_t)0, 16, terms);  // zero the terms
    if (V->kind == NMF_DENSE) {
        const unsigned gx = (unsigned)((n + LD_T - 1) / LD_T), gy = (unsigned)((m + LD_T - 1) / LD_T);
        double *part = (double *)take((size_t)gx * gy * sizeof(double));
        const size_t lds = (size_t)2 * LD_T * r * sizeof(float);
        hipLaunchKernelGGL(k_loss_dense, dim3(gx, gy), dim3(256), lds, s, V->dense, V->ld, m, n, W,
                           Ht, r, part);
        hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(256), 0, s, part, (int64_t)gx * gy,
                           (int64_t)1, (int64_t)0, terms + 0);
    } else {
        double *part = (double *)take((size_t)2 * m * sizeof(double));
        hipLaunchKernelGGL(k_loss_csr, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, V->rowptr,
                           V->colidx, V->vals, m, W, Ht, r, part);
        hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(256), 0, s, part, m, (int64_t)2,
                           (int64_t)1, terms + 1);
        hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(256), 0, s, part, m, (int64_t)2,
                           (int64_t)0, terms + 2);
        double *gp = (double *)take((size_t)256 * r * r * sizeof(double));
        double *gw = (double *)take((size_t)r * r * sizeof(double));
        double *gh = (double *)take((size_t)r * r * sizeof(double));
        hipError_t e = gram64(W, m, r, gp, gw, s);
        if (e == hipSuccess) e = gram64(Ht, n, r, gp, gh, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_dot_ordered, dim3(1), dim3(256), 0, s, gw, gh, (int64_t)r * r,
                           terms + 3);
    }
    double *sw = (double *)take(2 * 4096 * sizeof(double));
    double *sh = (double *)take(2 * 4096 * sizeof(double));
    int64_t bw = (m * r + 255) / 256, bh = (n * r + 255) / 256;
    bw = bw > 4096 ? 4096 : (bw < 1 ? 1 : bw);
    bh = bh > 4096 ? 4096 : (bh < 1 ? 1 : bh);
    hipLaunchKernelGGL(k_sums, dim3((unsigned)bw), dim3(256), 0, s, W, m * r, sw);
    hipLaunchKernelGGL(k_sums, dim3((unsigned)bh), dim3(256), 0, s, Ht, n * r, sh);
    hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(256), 0, s, sw, bw, (int64_t)2, (int64_t)0, terms + 4);
    hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(256), 0, s, sw, bw, (int64_t)2, (int64_t)1, terms + 5);
    hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(256), 0, s, sh, bh, (int64_t)2, (int64_t)0, terms + 6);
    hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(256), 0, s, sh, bh, (int64_t)2, (int64_t)1, terms + 7);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1), 0, s, terms, V->kind == NMF_CSR ? 1 : 0,
                       (double)reg->l1_w, (double)reg->l2_w, (double)reg->l1_h, (double)reg->l2_h,
                       dev_out);
    return hipGetLastError();
}

// KKT residual of one half into *dev_out; partial needs c doubles.
hipError_t launch_kkt(const float *G, int r, const float *P, float hsign, float hadd,
                      const float *X, int64_t c, double *partial, double *dev_out, hipStream_t s) {
    if (c <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_kkt, dim3((unsigned)((c + 3) / 4)), dim3(256), 0, s, G, r, P, hsign, hadd,
                       X, c, partial);
    hipLaunchKernelGGL(k_max_ordered, dim3(1), dim3(256), 0, s, partial, c, dev_out);
    return hipGetLastError();
}

}  // namespace nmfi
