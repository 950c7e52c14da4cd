// Gram matrix Gamma = A'A + 2 l2 I of the fixed factor (Algorithm 2 forms it
// once per half-iteration; Section 4.2 costs it at O(k r^2)).
//
// A is k x r row-major (k up to a few 10^5, r <= 128).  Phase 1: each block
// of four waves owns a contiguous range of rows; each wave accumulates the
// upper-triangle 32x32 tiles of A_rows' A_rows with MFMA (FP32: 32x32x2 on
// two rows per step; BF16: 32x32x16 on sixteen rows per step, FP32
// accumulation), the four waves are summed in LDS, and the block writes one
// partial.  Phase 2 sums the partials in block order (deterministic) and
// writes the symmetric r x r result with 2 l2 on the diagonal.
//
// Operand layout of the 32x32 MFMAs: lane l supplies row (l % 32) of the A
// operand / column (l % 32) of the B operand for k-slice l / 32.  For the
// Gram both operands are A[t][c*32 + l%32] from the same rows t, so one load
// per column block feeds every tile of that block row and column.
#include <algorithm>

#include "nmf_internal.h"
#include "kernels_common.h"

namespace nmfi {

constexpr int GRAM_BLOCK = 256;

// tile index of (ta <= tb) in row-major upper-triangle order
template <int NT>
__device__ __forceinline__ void tile_of(int ti, int &ta, int &tb) {
    int t = ti;
    ta = 0;
    while (t >= NT - ta) { t -= NT - ta; ta++; }
    tb = ta + t;
}

// One block's partial Gram over rows [b0, b1) of A (k x r), written to out
// (NTILE * 1024 floats in MFMA accumulator order).  red: LDS of NTILE * 1024.
template <int NT, int PREC>
__device__ __forceinline__ void gram_partial_rows(const float *__restrict__ A, int r, int64_t b0,
                                                  int64_t b1, float *red,
                                                  float *__restrict__ out) {
    constexpr int NTILE = NT * (NT + 1) / 2;
    constexpr int RSTEP = PREC == NMF_BF16 ? 16 : 2;  // rows per MFMA
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, col = lane & 31;

    // the block's rows split over its four waves in RSTEP-aligned pieces
    const int64_t nsteps = (b1 - b0 + RSTEP - 1) / RSTEP;
    const int64_t s0 = b0 + (nsteps * wave / 4) * RSTEP;
    const int64_t s1 = min(b1, b0 + (nsteps * (wave + 1) / 4) * RSTEP);

    f32x16 acc[NTILE];
#pragma unroll
    for (int i = 0; i < NTILE; i++) acc[i] = f32x16{};

    // Every load is from a valid (clamped) address and is zeroed only when
    // its trip runs, so the next trip's loads are issued before this trip's
    // MFMAs and arrive while they run.
    if constexpr (PREC == NMF_BF16) {
        if (s0 < s1) {
            float f[NT][8];
            auto load = [&](int64_t t, float (&w)[NT][8]) {
#pragma unroll
                for (int c = 0; c < NT; c++) {
                    const int a = c * 32 + col;
#pragma unroll
                    for (int q = 0; q < 8; q++) {
                        const int64_t row = t + half * 8 + q;
                        w[c][q] = A[(row < s1 ? row : s0) * r + (a < r ? a : 0)];
                    }
                }
            };
            load(s0, f);
            for (int64_t t = s0; t < s1; t += 16) {
                bf16x8 v[NT];
#pragma unroll
                for (int c = 0; c < NT; c++) {
                    const int a = c * 32 + col;
#pragma unroll
                    for (int q = 0; q < 8; q++) {
                        const int64_t row = t + half * 8 + q;
                        if (!(row < s1 && a < r)) f[c][q] = 0.f;
                    }
                    v[c] = pack_bf16x8(f[c]);
                }
                load(t + 16, f);
                int ti = 0;
#pragma unroll
                for (int ta = 0; ta < NT; ta++)
#pragma unroll
                    for (int tb = ta; tb < NT; tb++, ti++)
                        acc[ti] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(v[ta], v[tb], acc[ti], 0, 0, 0);
            }
        }
    } else {
        constexpr int U = 4;  // row pairs per trip
        if (s0 < s1) {
            float v[U][NT], w[U][NT];
            auto load = [&](int64_t t, float (&x)[U][NT]) {
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const int64_t row = t + 2 * u + half;
#pragma unroll
                    for (int c = 0; c < NT; c++) {
                        const int a = c * 32 + col;
                        x[u][c] = A[(row < s1 ? row : s0) * r + (a < r ? a : 0)];
                    }
                }
            };
            load(s0, w);
            for (int64_t t = s0; t < s1; t += 2 * U) {
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const int64_t row = t + 2 * u + half;
#pragma unroll
                    for (int c = 0; c < NT; c++) v[u][c] = (row < s1 && c * 32 + col < r) ? w[u][c] : 0.f;
                }
                load(t + 2 * U, w);
#pragma unroll
                for (int u = 0; u < U; u++) {
                    int ti = 0;
#pragma unroll
                    for (int ta = 0; ta < NT; ta++)
#pragma unroll
                        for (int tb = ta; tb < NT; tb++, ti++)
                            acc[ti] = __builtin_amdgcn_mfma_f32_32x32x2f32(v[u][ta], v[u][tb], acc[ti],
                                                                           0, 0, 0);
                }
            }
        }
    }
    // sum the four waves in LDS (fixed order), then one partial per block
    for (int w = 0; w < 4; w++) {
        if (wave == w) {
#pragma unroll
            for (int ti = 0; ti < NTILE; ti++)
#pragma unroll
                for (int q = 0; q < 16; q++) {
                    float *p = &red[(ti * 16 + q) * 64 + lane];
                    *p = (w == 0) ? acc[ti][q] : *p + acc[ti][q];
                }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < NTILE * 1024; e += GRAM_BLOCK) out[e] = red[e];
}

template <int NT, int PREC>
__global__ __launch_bounds__(GRAM_BLOCK) void k_gram_partial(const float *__restrict__ A, int64_t k,
                                                             int r, int64_t rows_per_block,
                                                             float *__restrict__ partial) {
    constexpr int NTILE = NT * (NT + 1) / 2;
    __shared__ float red[NTILE * 1024];
    const int64_t b0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t b1 = min(k, b0 + rows_per_block);
    gram_partial_rows<NT, PREC>(A, r, b0, b1, red, partial + (size_t)blockIdx.x * NTILE * 1024);
}

// Gram entry e (of NTILE * 1024, accumulator order) summed over nblocks
// partials (eight interleaved sums, combined in a fixed order), written to
// the symmetric r x r G with 2 l2 on the diagonal.
template <int NT>
__device__ __forceinline__ void gram_reduce_entry(const float *__restrict__ partial, int nblocks,
                                                  int r, float l2, float *__restrict__ G, int e) {
    constexpr int NTILE = NT * (NT + 1) / 2;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int pb = 0;
    for (; pb + 8 <= nblocks; pb += 8)
#pragma unroll
        for (int q = 0; q < 8; q++) acc[q] += partial[(size_t)(pb + q) * NTILE * 1024 + e];
    for (int q = 0; pb < nblocks; pb++, q++) acc[q] += partial[(size_t)pb * NTILE * 1024 + e];
    float s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    const int ti = e >> 10, rem = e & 1023, q = rem >> 6, lane = rem & 63;
    int ta, tb;
    tile_of<NT>(ti, ta, tb);
    const int i = 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3), j = lane & 31;
    const int a = ta * 32 + i, b = tb * 32 + j;
    if (a >= r || b >= r) return;
    if (ta == tb && a > b) return;  // the diagonal tile writes its upper half only
    if (a == b) s += 2.f * l2;
    G[(size_t)a * r + b] = s;
    G[(size_t)b * r + a] = s;
}

// The same sums as gram_reduce_entry, eight threads per entry: thread q of
// an entry forms that entry's interleaved sum acc[q] (partials q, q + 8, ...
// in order, then its tail partial), and the eight are combined in the same
// fixed order.  32 entries per block, consecutive entries on consecutive
// lanes (coalesced reads of each partial).
template <int NT>
__global__ __launch_bounds__(256) void k_gram_reduce(const float *__restrict__ partial, int nblocks,
                                                     int r, float l2, float *__restrict__ G,
                                                     unsigned long long *counter) {
    constexpr int NTILE = NT * (NT + 1) / 2;
    constexpr int N = NTILE * 1024;
    __shared__ float sm[8][32];
    const int el = threadIdx.x & 31, q = threadIdx.x >> 5;
    const int e = blockIdx.x * 32 + el;
    if (blockIdx.x == 0 && threadIdx.x == 0 && counter) *counter = 0ull;
    float a = 0.f;
    if (e < N) {
        const int full = nblocks / 8 * 8;
        // partials q, q + 8, ... added in order, their loads issued eight at a time
        for (int pb0 = q; pb0 < full; pb0 += 64) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; u++) v[u] = pb0 + 8 * u < full ? partial[(size_t)(pb0 + 8 * u) * N + e] : 0.f;
#pragma unroll
            for (int u = 0; u < 8; u++)
                if (pb0 + 8 * u < full) a += v[u];
        }
        if (full + q < nblocks) a += partial[(size_t)(full + q) * N + e];
    }
    sm[q][el] = a;
    __syncthreads();
    if (q != 0 || e >= N) return;
    float s = ((sm[0][el] + sm[1][el]) + (sm[2][el] + sm[3][el])) +
              ((sm[4][el] + sm[5][el]) + (sm[6][el] + sm[7][el]));
    const int ti = e >> 10, rem = e & 1023, qq = rem >> 6, lane = rem & 63;
    int ta, tb;
    tile_of<NT>(ti, ta, tb);
    const int i = 8 * (qq >> 2) + 4 * (lane >> 5) + (qq & 3), j = lane & 31;
    const int ra = ta * 32 + i, cb = tb * 32 + j;
    if (ra >= r || cb >= r) return;
    if (ta == tb && ra > cb) return;  // the diagonal tile writes its upper half only
    if (ra == cb) s += 2.f * l2;
    G[(size_t)ra * r + cb] = s;
    G[(size_t)cb * r + ra] = s;
}

// Rows of A per block: BGRAM_ROWS, or about k / 256 (a multiple of 16) for
// tall A, so that a large Gram runs as one round of blocks (measured: the
// 200000 x 100 and 100000 x 100 Grams of one outer iteration take 119 us
// against 143 us with 512-row blocks; half as many rows per block, 156 us).
// The batched fit uses the same rule, so a problem's Gram is bitwise the same
// alone or in a batch.
int64_t gram_rows(int64_t k) {
    const int64_t per = ((k + 255) / 256 + 15) / 16 * 16;
    return per > BGRAM_ROWS ? per : BGRAM_ROWS;
}

template <int NT, int PREC>
static hipError_t gram_t(const float *A, int64_t k, int r, float l2, float *G, float *scratch,
                         hipStream_t s, unsigned long long *counter) {
    constexpr int NTILE = NT * (NT + 1) / 2;
    const int64_t rows = gram_rows(k);
    const int64_t nb = k > 0 ? (k + rows - 1) / rows : 1;
    hipLaunchKernelGGL((k_gram_partial<NT, PREC>), dim3((unsigned)nb), dim3(GRAM_BLOCK), 0, s, A, k,
                       r, rows, scratch);
    hipLaunchKernelGGL((k_gram_reduce<NT>), dim3((NTILE * 1024 + 31) / 32), dim3(256), 0, s,
                       scratch, (int)nb, r, l2, G, counter);
    return hipGetLastError();
}

// Enough for the Gram of any A with at most k rows: the block count is
// ceil(k' / 512) <= 256 below 131073 rows and at most 256 above.
size_t gram_scratch_bytes(int r, int64_t k) {
    const int NT = (r + 31) / 32;
    int64_t nb = k > 0 ? (k + BGRAM_ROWS - 1) / BGRAM_ROWS : 1;
    if (nb > 256) nb = 256;
    return (size_t)nb * (NT * (NT + 1) / 2) * 1024 * sizeof(float);
}

hipError_t launch_gram(const float *A, int64_t k, int r, float l2, int precision, float *G,
                       float *scratch, hipStream_t s, unsigned long long *counter) {
    const int NT = (r + 31) / 32;
    if (precision == NMF_BF16) {
        switch (NT) {
        case 1: return gram_t<1, NMF_BF16>(A, k, r, l2, G, scratch, s, counter);
        case 2: return gram_t<2, NMF_BF16>(A, k, r, l2, G, scratch, s, counter);
        case 3: return gram_t<3, NMF_BF16>(A, k, r, l2, G, scratch, s, counter);
        case 4: return gram_t<4, NMF_BF16>(A, k, r, l2, G, scratch, s, counter);
        }
    } else {
        switch (NT) {
        case 1: return gram_t<1, NMF_FP32>(A, k, r, l2, G, scratch, s, counter);
        case 2: return gram_t<2, NMF_FP32>(A, k, r, l2, G, scratch, s, counter);
        case 3: return gram_t<3, NMF_FP32>(A, k, r, l2, G, scratch, s, counter);
        case 4: return gram_t<4, NMF_FP32>(A, k, r, l2, G, scratch, s, counter);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace nmfi

// ------------------------------------------------------------------ batched
namespace nmfi {

// Phase 1 for many problems at once: block b computes items[b] = (problem,
// chunk), the partial Gram of rows [chunk * P.rows, ...) of that problem's A.
template <int NTMAX, int PREC>
__global__ __launch_bounds__(GRAM_BLOCK) void k_bgram_partial(const BItem *__restrict__ items,
                                                              const BGramProb *__restrict__ probs) {
    __shared__ float red[NTMAX * (NTMAX + 1) / 2 * 1024];
    const BItem it = items[blockIdx.x];
    const BGramProb P = probs[it.prob];
    const int64_t b0 = (int64_t)it.idx * P.rows;
    const int64_t b1 = min(P.k, b0 + P.rows);
    const int NT = (P.r + 31) / 32;
    float *out = P.partial + (size_t)it.idx * (NT * (NT + 1) / 2) * 1024;
    switch (NT) {
    case 1: gram_partial_rows<1, PREC>(P.A, P.r, b0, b1, red, out); break;
    case 2: if constexpr (NTMAX >= 2) gram_partial_rows<2, PREC>(P.A, P.r, b0, b1, red, out); break;
    case 3: if constexpr (NTMAX >= 3) gram_partial_rows<3, PREC>(P.A, P.r, b0, b1, red, out); break;
    default: if constexpr (NTMAX >= 4) gram_partial_rows<4, PREC>(P.A, P.r, b0, b1, red, out); break;
    }
}

// Phase 2: one block per problem sums its partials into Gamma.
template <int NTMAX>
__global__ __launch_bounds__(256) void k_bgram_finish(const BGramProb *__restrict__ probs) {
    const BGramProb P = probs[blockIdx.x];
    const int NT = (P.r + 31) / 32;
    const int n = NT * (NT + 1) / 2 * 1024;
    for (int e = threadIdx.x; e < n; e += 256) {
        switch (NT) {
        case 1: gram_reduce_entry<1>(P.partial, P.nchunks, P.r, P.l2, P.G, e); break;
        case 2: if constexpr (NTMAX >= 2) gram_reduce_entry<2>(P.partial, P.nchunks, P.r, P.l2, P.G, e); break;
        case 3: if constexpr (NTMAX >= 3) gram_reduce_entry<3>(P.partial, P.nchunks, P.r, P.l2, P.G, e); break;
        default: if constexpr (NTMAX >= 4) gram_reduce_entry<4>(P.partial, P.nchunks, P.r, P.l2, P.G, e); break;
        }
    }
}

size_t bgram_partial_floats(int r, int64_t k) {
    const int NT = (r + 31) / 32;
    const int64_t rows = gram_rows(k);
    return (size_t)((k + rows - 1) / rows) * (NT * (NT + 1) / 2) * 1024;
}

hipError_t launch_bgram(const BItem *items, int64_t nitems, const BGramProb *probs, int nprobs,
                        int ntmax, int precision, hipStream_t s) {
    if (nitems > 0) {
        const dim3 g((unsigned)nitems), b(GRAM_BLOCK);
        if (ntmax <= 2) {
            if (precision == NMF_BF16) hipLaunchKernelGGL((k_bgram_partial<2, NMF_BF16>), g, b, 0, s, items, probs);
            else hipLaunchKernelGGL((k_bgram_partial<2, NMF_FP32>), g, b, 0, s, items, probs);
        } else {
            if (precision == NMF_BF16) hipLaunchKernelGGL((k_bgram_partial<4, NMF_BF16>), g, b, 0, s, items, probs);
            else hipLaunchKernelGGL((k_bgram_partial<4, NMF_FP32>), g, b, 0, s, items, probs);
        }
    }
    if (nprobs > 0) {
        if (ntmax <= 2) hipLaunchKernelGGL((k_bgram_finish<2>), dim3(nprobs), dim3(256), 0, s, probs);
        else hipLaunchKernelGGL((k_bgram_finish<4>), dim3(nprobs), dim3(256), 0, s, probs);
    }
    return hipGetLastError();
}

}  // namespace nmfi
