// Dense data product (Algorithm 2's Y = F V' and G'V_i; Section 4.2: O(mnr)).
// P (c x r) = X (c x k) * A (k x r), with X = V' (trans = 0: the H-update,
// A = W) or X = V (trans = 1: the W-update, A = Ht).  V is m x n row-major
// with leading dimension ld.
//
// Each block of four waves computes a 64 x R32 slab of P over one slice of
// k (split-K), staging a 64 x 32 tile of X and a 32 x R32 tile of A in LDS
// per step and accumulating 32x32 MFMA tiles (FP32 32x32x2, or BF16 32x32x16
// with FP32 accumulation on the BF16 copies).  Split-K partials are summed in
// slice order by a second kernel, so the result is deterministic.
#include "kernels_common.h"
#include "nmf_internal.h"

namespace nmfi {

constexpr int DP_BC = 64;  // rows of P per block
constexpr int DP_KT = 32;  // k per LDS stage

// LDS a block needs for the FP32 product body
template <int NT>
constexpr int dense_fp32_lds_floats() {
    return DP_BC * (DP_KT + 1) + DP_KT * NT * 32;
}

// 64 rows of P = X A starting at row c0, summed over k in [kb, ke), written
// to o (C x r).  lds: dense_fp32_lds_floats<NT>() floats.
template <int NT, bool XT>
__device__ __forceinline__ void dense_fp32_body(const float *__restrict__ V, int64_t ld, int64_t C,
                                                const float *__restrict__ A, int r, int64_t c0,
                                                int64_t kb, int64_t ke, float *lds,
                                                float *__restrict__ o) {
    constexpr int R32 = NT * 32;
    constexpr int NTILES = 2 * NT;
    constexpr int TPW = (NTILES + 3) / 4;
    float(*Xs)[DP_KT + 1] = (float(*)[DP_KT + 1])lds;
    float(*As)[R32] = (float(*)[R32])(lds + DP_BC * (DP_KT + 1));
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    f32x16 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; q++) acc[q] = f32x16{};

    for (int64_t k0 = kb; k0 < ke; k0 += DP_KT) {
        if constexpr (XT) {  // X[c][k] = V[k][c]: rows of V, 64 contiguous columns
            for (int e = tid; e < DP_KT * DP_BC; e += 256) {
                const int kk = e / DP_BC, c = e % DP_BC;
                const int64_t gk = k0 + kk, gc = c0 + c;
                Xs[c][kk] = (gk < ke && gc < C) ? V[gk * ld + gc] : 0.f;
            }
        } else {  // X[c][k] = V[c][k]: rows of V, 32 contiguous columns
            for (int e = tid; e < DP_KT * DP_BC; e += 256) {
                const int c = e / DP_KT, kk = e % DP_KT;
                const int64_t gk = k0 + kk, gc = c0 + c;
                Xs[c][kk] = (gk < ke && gc < C) ? V[gc * ld + gk] : 0.f;
            }
        }
        for (int e = tid; e < DP_KT * R32; e += 256) {
            const int kk = e / R32, a = e % R32;
            const int64_t gk = k0 + kk;
            As[kk][a] = (gk < ke && a < r) ? A[gk * r + a] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < TPW; q++) {
            const int tile = wave + 4 * q;
            if (tile < NTILES) {
                const int rt = tile / NT, ct = tile % NT;
#pragma unroll
                for (int kp = 0; kp < DP_KT / 2; kp++) {
                    const float a_op = Xs[32 * rt + (lane & 31)][2 * kp + (lane >> 5)];
                    const float b_op = As[2 * kp + (lane >> 5)][32 * ct + (lane & 31)];
                    acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a_op, b_op, acc[q], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < TPW; q++) {
        const int tile = wave + 4 * q;
        if (tile < NTILES) {
            const int rt = tile / NT, ct = tile % NT;
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3), j = lane & 31;
                const int64_t c = c0 + 32 * rt + i;
                const int a = 32 * ct + j;
                if (c < C && a < r) o[c * r + a] = acc[q][v];
            }
        }
    }
}

template <int NT, bool XT>
__global__ __launch_bounds__(256) void k_dense_fp32(const float *__restrict__ V, int64_t ld,
                                                    int64_t C, int64_t K,
                                                    const float *__restrict__ A, int r,
                                                    int64_t kchunk, float *__restrict__ out) {
    __shared__ float lds[dense_fp32_lds_floats<NT>()];
    const int64_t kb = (int64_t)blockIdx.y * kchunk;
    dense_fp32_body<NT, XT>(V, ld, C, A, r, (int64_t)blockIdx.x * DP_BC, kb, min(K, kb + kchunk),
                            lds, out + (int64_t)blockIdx.y * C * r);
}

// BF16 operands (V16: the BF16 copy of V; A converted while staging)
template <int NT>
constexpr int dense_bf16_lds_bytes() {
    return (DP_BC + NT * 32) * (DP_KT + 8) * 2;
}

template <int NT, bool XT>
__device__ __forceinline__ void dense_bf16_body(const __bf16 *__restrict__ V16, int64_t ld,
                                                int64_t C, const float *__restrict__ A, int r,
                                                int64_t c0, int64_t kb, int64_t ke, void *lds,
                                                float *__restrict__ o) {
    constexpr int R32 = NT * 32;
    constexpr int NTILES = 2 * NT;
    constexpr int TPW = (NTILES + 3) / 4;
    // k-major staging so that a lane's eight consecutive k are contiguous
    __bf16(*Xs)[DP_KT + 8] = (__bf16(*)[DP_KT + 8])lds;
    __bf16(*As)[DP_KT + 8] = (__bf16(*)[DP_KT + 8])((char *)lds + DP_BC * (DP_KT + 8) * 2);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    f32x16 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; q++) acc[q] = f32x16{};
    const __bf16 zero = (__bf16)0.f;

    for (int64_t k0 = kb; k0 < ke; k0 += DP_KT) {
        if constexpr (XT) {
            for (int e = tid; e < DP_KT * DP_BC; e += 256) {
                const int kk = e / DP_BC, c = e % DP_BC;
                const int64_t gk = k0 + kk, gc = c0 + c;
                Xs[c][kk] = (gk < ke && gc < C) ? V16[gk * ld + gc] : zero;
            }
        } else {
            for (int e = tid; e < DP_KT * DP_BC; e += 256) {
                const int c = e / DP_KT, kk = e % DP_KT;
                const int64_t gk = k0 + kk, gc = c0 + c;
                Xs[c][kk] = (gk < ke && gc < C) ? V16[gc * ld + gk] : zero;
            }
        }
        for (int e = tid; e < DP_KT * R32; e += 256) {
            const int kk = e / R32, a = e % R32;
            const int64_t gk = k0 + kk;
            As[a][kk] = (gk < ke && a < r) ? (__bf16)A[gk * r + a] : zero;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < TPW; q++) {
            const int tile = wave + 4 * q;
            if (tile < NTILES) {
                const int rt = tile / NT, ct = tile % NT;
#pragma unroll
                for (int ks = 0; ks < DP_KT / 16; ks++) {
                    bf16x8 a_op, b_op;
                    const int kq = 16 * ks + 8 * (lane >> 5);
#pragma unroll
                    for (int t = 0; t < 8; t++) {
                        a_op[t] = Xs[32 * rt + (lane & 31)][kq + t];
                        b_op[t] = As[32 * ct + (lane & 31)][kq + t];
                    }
                    acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_op, b_op, acc[q], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < TPW; q++) {
        const int tile = wave + 4 * q;
        if (tile < NTILES) {
            const int rt = tile / NT, ct = tile % NT;
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3), j = lane & 31;
                const int64_t c = c0 + 32 * rt + i;
                const int a = 32 * ct + j;
                if (c < C && a < r) o[c * r + a] = acc[q][v];
            }
        }
    }
}

template <int NT, bool XT>
__global__ __launch_bounds__(256) void k_dense_bf16(const __bf16 *__restrict__ V16, int64_t ld,
                                                    int64_t C, int64_t K,
                                                    const float *__restrict__ A, int r,
                                                    int64_t kchunk, float *__restrict__ out) {
    __shared__ __attribute__((aligned(16))) char lds[dense_bf16_lds_bytes<NT>()];
    const int64_t kb = (int64_t)blockIdx.y * kchunk;
    dense_bf16_body<NT, XT>(V16, ld, C, A, r, (int64_t)blockIdx.x * DP_BC, kb, min(K, kb + kchunk),
                            lds, out + (int64_t)blockIdx.y * C * r);
}

// P = sum over split-K slices in slice order
__global__ void k_split_reduce(const float *__restrict__ part, int nsplit, int64_t n,
                               float *__restrict__ P) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int k = 0; k < nsplit; k++) s += part[(int64_t)k * n + i];
        P[i] = s;
    }
}

__global__ void k_to_bf16(const float *__restrict__ x, int64_t rows, int64_t cols, int64_t ld,
                          __bf16 *__restrict__ y) {
    const int64_t n = rows * cols;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rr = i / cols, cc = i - rr * cols;
        y[i] = (__bf16)x[rr * ld + cc];
    }
}

hipError_t launch_to_bf16(const float *x, int64_t rows, int64_t cols, int64_t ld, __bf16 *y,
                          hipStream_t s) {
    int64_t blocks = (rows * cols + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) return hipSuccess;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)blocks), dim3(256), 0, s, x, rows, cols, ld, y);
    return hipGetLastError();
}

// split-K factor: enough blocks to fill the chip, at least 256 k per slice
int dense_nsplit(int64_t C, int64_t K) {
    const int64_t rb = (C + DP_BC - 1) / DP_BC;
    int64_t ns = (2048 + rb - 1) / rb;
    const int64_t maxs = (K + 255) / 256;
    if (ns > maxs) ns = maxs;
    if (ns < 1) ns = 1;
    if (ns > 64) ns = 64;
    return (int)ns;
}

int64_t dense_kchunk(int64_t C, int64_t K) {
    const int ns = dense_nsplit(C, K);
    int64_t kchunk = (K + ns - 1) / ns;
    kchunk = ((kchunk + DP_KT - 1) / DP_KT) * DP_KT;
    return kchunk < DP_KT ? DP_KT : kchunk;
}

size_t dense_scratch_bytes(int64_t m, int64_t n, int r) {
    const int64_t a = (int64_t)dense_nsplit(n, m) * n, b = (int64_t)dense_nsplit(m, n) * m;
    return (size_t)(a > b ? a : b) * r * sizeof(float) + 256;
}

template <int NT>
static void dense_launch_nt(bool bf16, bool xt, const void *V, int64_t ld, int64_t C, int64_t K,
                            const float *A, int r, int64_t kchunk, float *out, dim3 grid,
                            hipStream_t s) {
    if (bf16) {
        if (xt)
            hipLaunchKernelGGL((k_dense_bf16<NT, true>), grid, dim3(256), 0, s,
                               (const __bf16 *)V, ld, C, K, A, r, kchunk, out);
        else
            hipLaunchKernelGGL((k_dense_bf16<NT, false>), grid, dim3(256), 0, s,
                               (const __bf16 *)V, ld, C, K, A, r, kchunk, out);
    } else {
        if (xt)
            hipLaunchKernelGGL((k_dense_fp32<NT, true>), grid, dim3(256), 0, s, (const float *)V,
                               ld, C, K, A, r, kchunk, out);
        else
            hipLaunchKernelGGL((k_dense_fp32<NT, false>), grid, dim3(256), 0, s,
                               (const float *)V, ld, C, K, A, r, kchunk, out);
    }
}

// V (m x n, ld): float32, or its BF16 copy when bf16 != 0.
hipError_t launch_dense_product(const void *V, int bf16, int64_t m, int64_t n, int64_t ld,
                                int trans, const float *A, int r, float *P, float *scratch,
                                hipStream_t s) {
    const bool xt = trans == 0;
    const int64_t C = xt ? n : m, K = xt ? m : n;
    if (C == 0) return hipSuccess;
    const int64_t kchunk = dense_kchunk(C, K);
    const int nsplit = (int)((K + kchunk - 1) / kchunk);
    float *out = nsplit > 1 ? scratch : P;
    dim3 grid((unsigned)((C + DP_BC - 1) / DP_BC), (unsigned)(nsplit > 0 ? nsplit : 1));
    if (K == 0) return hipErrorInvalidValue;  // callers reject empty V
    const int NT = (r + 31) / 32;
    switch (NT) {
    case 1: dense_launch_nt<1>(bf16, xt, V, ld, C, K, A, r, kchunk, out, grid, s); break;
    case 2: dense_launch_nt<2>(bf16, xt, V, ld, C, K, A, r, kchunk, out, grid, s); break;
    case 3: dense_launch_nt<3>(bf16, xt, V, ld, C, K, A, r, kchunk, out, grid, s); break;
    default: dense_launch_nt<4>(bf16, xt, V, ld, C, K, A, r, kchunk, out, grid, s); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nsplit <= 1) return e;
    const int64_t nel = C * r;
    int64_t blocks = (nel + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_split_reduce, dim3((unsigned)blocks), dim3(256), 0, s, scratch, nsplit,
                       nel, P);
    return hipGetLastError();
}

}  // namespace nmfi

// ------------------------------------------------------------------ batched
namespace nmfi {

// Many problems at once: block b computes 64 rows of one problem's P over
// one k slice (items[b].idx = row block * nsplit + slice), exactly as the
// single-problem product does, so the result is bitwise the same.
template <int NTMAX, bool XT, bool BF16>
__global__ __launch_bounds__(256) void k_bdense(const BItem *__restrict__ items,
                                                const BProdProb *__restrict__ probs) {
    constexpr int FP32_BYTES = dense_fp32_lds_floats<NTMAX>() * 4;
    constexpr int BF16_BYTES = dense_bf16_lds_bytes<NTMAX>();
    __shared__ __attribute__((aligned(16))) char lds[BF16 ? BF16_BYTES : FP32_BYTES];
    const BItem it = items[blockIdx.x];
    const BProdProb P = probs[it.prob];
    const int NT = (P.r + 31) / 32;
    const int slice = it.idx % P.nsplit;
    const int64_t c0 = (int64_t)(it.idx / P.nsplit) * DP_BC;
    const int64_t kb = (int64_t)slice * P.kchunk;
    const int64_t ke = min(P.K, kb + P.kchunk);
    float *o = P.nsplit > 1 ? P.part + (int64_t)slice * P.C * P.r : P.P;
#define NMF_BDENSE_CASE(N)                                                                     \
    if constexpr (BF16)                                                                        \
        dense_bf16_body<N, XT>((const __bf16 *)P.V, P.ld, P.C, P.A, P.r, c0, kb, ke, lds, o);  \
    else                                                                                       \
        dense_fp32_body<N, XT>((const float *)P.V, P.ld, P.C, P.A, P.r, c0, kb, ke,            \
                               (float *)lds, o);
    switch (NT) {
    case 1: { NMF_BDENSE_CASE(1) } break;
    case 2: if constexpr (NTMAX >= 2) { NMF_BDENSE_CASE(2) } break;
    case 3: if constexpr (NTMAX >= 3) { NMF_BDENSE_CASE(3) } break;
    default: if constexpr (NTMAX >= 4) { NMF_BDENSE_CASE(4) } break;
    }
#undef NMF_BDENSE_CASE
}

// split-K sums of many problems, the same loop as k_split_reduce
__global__ void k_bsplit_reduce(const BItem *__restrict__ items, const BProdProb *__restrict__ probs) {
    const BItem it = items[blockIdx.x];
    const BProdProb P = probs[it.prob];
    const int64_t n = P.C * P.r;
    const int64_t e0 = (int64_t)it.idx * 4096;
    for (int64_t i = e0 + threadIdx.x; i < min(n, e0 + 4096); i += blockDim.x) {
        float s = 0.f;
        for (int k = 0; k < P.nsplit; k++) s += P.part[(int64_t)k * n + i];
        P.P[i] = s;
    }
}

hipError_t launch_bdense(const BItem *items, int64_t nitems, const BProdProb *probs, int ntmax,
                         bool xt, bool bf16, const BItem *red_items, int64_t nred, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    const dim3 g((unsigned)nitems), b(256);
#define NMF_BD(NTM, X, B) hipLaunchKernelGGL((k_bdense<NTM, X, B>), g, b, 0, s, items, probs)
    if (ntmax <= 2) {
        if (xt) { if (bf16) NMF_BD(2, true, true); else NMF_BD(2, true, false); }
        else { if (bf16) NMF_BD(2, false, true); else NMF_BD(2, false, false); }
    } else {
        if (xt) { if (bf16) NMF_BD(4, true, true); else NMF_BD(4, true, false); }
        else { if (bf16) NMF_BD(4, false, true); else NMF_BD(4, false, false); }
    }
#undef NMF_BD
    if (nred > 0)
        hipLaunchKernelGGL(k_bsplit_reduce, dim3((unsigned)nred), dim3(256), 0, s, red_items, probs);
    return hipGetLastError();
}

}  // namespace nmfi
