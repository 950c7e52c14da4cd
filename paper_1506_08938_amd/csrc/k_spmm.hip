// Sparse data product (Section 4.2: O(r S(mn)) for sparse data): for CSR B,
// P[row] = sum_t vals[t] * A[colidx[t]] -- one gathered row of the fixed
// factor A (k x r) per stored entry.  The H-update uses CSR(V') with A = W,
// the W-update CSR(V) with A = Ht.
//
// Work is a list of chunks (row, [start, end)) of at most SPMM_CHUNK entries;
// one wave per chunk.  A chunk of a row that was split writes its sum to a
// partial slot and a fix-up kernel adds a split row's slots in chunk order,
// so results never depend on scheduling.  Lanes are grouped LPN per entry,
// each lane covering VEC consecutive columns (NV such pieces), so one wave
// step gathers 64 / LPN entries with full-row contiguous loads.
//
// The gathered factor is float32 (row stride r), or in BF16 mode a BF16
// copy with rows padded to a multiple of eight (16-byte pieces of eight
// values): half the gathered bytes, each product still accumulated in
// float32.  Measured on the 200000 x 100000 text-like workload at r = 100:
// both products with their BF16 conversions take 1.04 ms per outer iteration
// against 1.48 ms in float32 (8-byte pieces: 1.08 ms).
#include <algorithm>
#include <vector>

#include "kernels_common.h"
#include "nmf_internal.h"

namespace nmfi {

// Gathers of one chunk: the chunk's (column, value) pairs are loaded 64 at a
// time with one coalesced load per lane and handed to the lane groups with
// ds_bpermute, so every gather's address is known up front and U row
// gathers per lane are in flight at once.
// VEC consecutive entries of a factor row as floats (BF16: VEC = 8 or 4, one
// 16- or 8-byte load; a BF16 value is the high half of its float)
template <typename TA, int VEC>
__device__ __forceinline__ void load_piece(const TA *p, float (&out)[VEC]) {
    if constexpr (sizeof(TA) == 2 && VEC == 8) {
        const uint4 u = *(const uint4 *)p;
        const unsigned w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int h = 0; h < 4; h++) {
            out[2 * h] = __uint_as_float(w[h] << 16);
            out[2 * h + 1] = __uint_as_float(w[h] & 0xffff0000u);
        }
    } else if constexpr (sizeof(TA) == 2) {
        static_assert(VEC == 4, "BF16 pieces are four or eight values");
        const uint2 u = *(const uint2 *)p;
        out[0] = __uint_as_float(u.x << 16);
        out[1] = __uint_as_float(u.x & 0xffff0000u);
        out[2] = __uint_as_float(u.y << 16);
        out[3] = __uint_as_float(u.y & 0xffff0000u);
    } else if constexpr (VEC == 4) {
        const f32x4 a4 = *(const f32x4 *)p;
#pragma unroll
        for (int v = 0; v < 4; v++) out[v] = a4[v];
    } else if constexpr (VEC == 2) {
        const f32x2 a2 = *(const f32x2 *)p;
        out[0] = a2[0];
        out[1] = a2[1];
    } else {
        out[0] = p[0];
    }
}

// lda: row stride of A in elements (r for float32, r rounded up to 4 for BF16)
template <typename TA, int VEC, int LPN, int NV>
__device__ __forceinline__ void spmm_range(int start, int end, const int32_t *__restrict__ colidx,
                                           const float *__restrict__ vals,
                                           const TA *__restrict__ A, int r, int lda,
                                           float (&acc)[NV][VEC]) {
    const int lane = threadIdx.x & 63;
    constexpr int NPW = 64 / LPN;
#ifndef NMF_SPMM_TRIP
#define NMF_SPMM_TRIP 16
#endif
    constexpr int U = NPW >= NMF_SPMM_TRIP ? 1 : NMF_SPMM_TRIP / NPW;  // entries per slot per trip
    const int slot = lane / LPN, part = lane % LPN;
    for (int b = start; b < end; b += 64) {
        const int nb = min(64, end - b);
        const int my_ci = lane < nb ? colidx[b + lane] : 0;
        const float my_cv = lane < nb ? vals[b + lane] : 0.f;
        for (int j0 = 0; j0 < nb; j0 += NPW * U) {
            int ci[U];
            float cv[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int j = j0 + u * NPW + slot;  // entry of this slot (< 64)
                ci[u] = __builtin_amdgcn_ds_bpermute(j << 2, my_ci);
                cv[u] = __builtin_bit_cast(
                    float, __builtin_amdgcn_ds_bpermute(j << 2, __builtin_bit_cast(int, my_cv)));
                if (j >= nb) cv[u] = 0.f, ci[u] = -1;
            }
            // every gather of the trip is issued before the first FMA: entries
            // past the chunk's end read row 0 with weight 0, and lanes past r
            // read column 0 into sums that are never written (they add
            // exactly nothing to the written ones)
            float av[U][NV][VEC];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const TA *arow = A + (int64_t)(ci[u] < 0 ? 0 : ci[u]) * lda;
#pragma unroll
                for (int q = 0; q < NV; q++) {
                    const int col0 = (q * LPN + part) * VEC;
                    load_piece<TA, VEC>(arow + (col0 < r ? col0 : 0), av[u][q]);
                }
            }
#pragma unroll
            for (int u = 0; u < U; u++)
#pragma unroll
                for (int q = 0; q < NV; q++)
#pragma unroll
                    for (int v = 0; v < VEC; v++) acc[q][v] = fmaf(cv[u], av[u][q][v], acc[q][v]);
        }
    }
}

// sum the NPW slots' partial rows (fixed butterfly) and write slot 0's
template <int VEC, int LPN, int NV>
__device__ __forceinline__ void spmm_finish(float (&acc)[NV][VEC], int r, float *dst) {
    const int lane = threadIdx.x & 63;
    const int slot = lane / LPN, part = lane % LPN;
#pragma unroll
    for (int off = LPN; off < 64; off <<= 1)
#pragma unroll
        for (int q = 0; q < NV; q++)
#pragma unroll
            for (int v = 0; v < VEC; v++) acc[q][v] += __shfl_xor(acc[q][v], off);
    if (slot != 0) return;
#pragma unroll
    for (int q = 0; q < NV; q++) {
        const int col0 = (q * LPN + part) * VEC;
#pragma unroll
        for (int v = 0; v < VEC; v++)
            if (col0 + v < r) dst[col0 + v] = acc[q][v];
    }
}

template <typename TA, int VEC, int LPN, int NV>
__global__ __launch_bounds__(256) void k_spmm(const SpChunk *__restrict__ chunks, int64_t nchunks,
                                              const int32_t *__restrict__ colidx,
                                              const float *__restrict__ vals,
                                              const TA *__restrict__ A, int r, int lda,
                                              float *__restrict__ P, float *__restrict__ partial) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= nchunks) return;
    const SpChunk c = chunks[w];
    float acc[NV][VEC];
#pragma unroll
    for (int q = 0; q < NV; q++)
#pragma unroll
        for (int v = 0; v < VEC; v++) acc[q][v] = 0.f;
    spmm_range<TA, VEC, LPN, NV>(c.start, c.end, colidx, vals, A, r, lda, acc);
    spmm_finish<VEC, LPN, NV>(acc, r,
                              c.dest < 0 ? P + (int64_t)c.row * r : partial + (int64_t)c.dest * r);
}

// P[row] = sum of the row's partial slots in chunk order
__global__ __launch_bounds__(128) void k_spmm_fixup(const SpSplit *__restrict__ splits,
                                                    const float *__restrict__ partial, int r,
                                                    float *__restrict__ P) {
    const SpSplit s = splits[blockIdx.x];
    for (int a = threadIdx.x; a < r; a += 128) {
        // eight interleaved sums (loads in flight), combined in a fixed order
        float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        const float *p = partial + (int64_t)s.first * r + a;
        int c = 0;
        for (; c + 8 <= s.count; c += 8)
#pragma unroll
            for (int q = 0; q < 8; q++) acc[q] += p[(int64_t)(c + q) * r];
        for (int q = 0; c < s.count; c++, q++) acc[q] += p[(int64_t)c * r];
        P[(int64_t)s.row * r + a] =
            ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    }
}

template <int VEC, int LPN, int NV, typename TA = float>
static void launch_spmm_t(const SpmmPlan &pl, const int32_t *colidx, const float *vals,
                          const TA *A, int r, float *P, float *partial, hipStream_t s, int lda = -1) {
    const unsigned blocks = (unsigned)((pl.nchunks + 3) / 4);
    hipLaunchKernelGGL((k_spmm<TA, VEC, LPN, NV>), dim3(blocks), dim3(256), 0, s, pl.chunks,
                       pl.nchunks, colidx, vals, A, r, lda < 0 ? r : lda, P, partial);
}

static int pow2_at_least(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

static hipError_t launch_spmm_fixup(const SpmmPlan &pl, float *partial, int r, float *P, hipStream_t s) {
    if (pl.nsplits > 0) {
        hipLaunchKernelGGL(k_spmm_fixup, dim3((unsigned)pl.nsplits), dim3(128), 0, s, pl.splits,
                           partial, r, P);
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_spmm(const SpmmPlan &pl, const int32_t *colidx, const float *vals, const float *A,
                       int r, float *P, float *partial, hipStream_t s) {
    if (pl.nrows == 0) return hipSuccess;
    if (pl.nchunks > 0) {
        if (r % 4 == 0) {
            switch (pow2_at_least(r / 4)) {
            case 1: launch_spmm_t<4, 1, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            case 2: launch_spmm_t<4, 2, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            case 4: launch_spmm_t<4, 4, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            case 8: launch_spmm_t<4, 8, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            case 16: launch_spmm_t<4, 16, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            default: launch_spmm_t<4, 32, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            }
        } else if (r % 2 == 0) {
            switch (pow2_at_least(r / 2)) {
            case 1: launch_spmm_t<2, 1, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            case 2: launch_spmm_t<2, 2, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            case 4: launch_spmm_t<2, 4, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            case 8: launch_spmm_t<2, 8, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            case 16: launch_spmm_t<2, 16, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            case 32: launch_spmm_t<2, 32, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            default: launch_spmm_t<2, 64, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            }
        } else if (r <= 64) {
            switch (pow2_at_least(r)) {
            case 1: launch_spmm_t<1, 1, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            case 2: launch_spmm_t<1, 2, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            case 4: launch_spmm_t<1, 4, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            case 8: launch_spmm_t<1, 8, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            case 16: launch_spmm_t<1, 16, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            case 32: launch_spmm_t<1, 32, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            default: launch_spmm_t<1, 64, 1>(pl, colidx, vals, A, r, P, partial, s); break;
            }
        } else {
            launch_spmm_t<1, 64, 2>(pl, colidx, vals, A, r, P, partial, s);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_spmm_fixup(pl, partial, r, P, s);
}

// BF16 gathers: A16 is k x lda16 (lda16 = r rounded up to NMF_SPMM_VEC16),
// NMF_SPMM_VEC16 values per lane and piece
hipError_t launch_spmm16(const SpmmPlan &pl, const int32_t *colidx, const float *vals,
                         const __bf16 *A16, int lda16, int r, float *P, float *partial, hipStream_t s) {
    if (pl.nrows == 0) return hipSuccess;
    if (pl.nchunks > 0) {
        constexpr int V16 = NMF_SPMM_VEC16;
        switch (pow2_at_least((r + V16 - 1) / V16)) {
        case 1: launch_spmm_t<V16, 1, 1>(pl, colidx, vals, A16, r, P, partial, s, lda16); break;
        case 2: launch_spmm_t<V16, 2, 1>(pl, colidx, vals, A16, r, P, partial, s, lda16); break;
        case 4: launch_spmm_t<V16, 4, 1>(pl, colidx, vals, A16, r, P, partial, s, lda16); break;
        case 8: launch_spmm_t<V16, 8, 1>(pl, colidx, vals, A16, r, P, partial, s, lda16); break;
        case 16: launch_spmm_t<V16, 16, 1>(pl, colidx, vals, A16, r, P, partial, s, lda16); break;
        default: launch_spmm_t<V16, 32, 1>(pl, colidx, vals, A16, r, P, partial, s, lda16); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_spmm_fixup(pl, partial, r, P, s);
}

// A16[i][j] = bf16(A[i][j]) (round to nearest even) for j < r, 0 for
// r <= j < lda16
__global__ void k_rows_to_bf16(const float *__restrict__ A, int64_t k, int r, int lda16,
                               __bf16 *__restrict__ A16) {
    const int64_t n = k * lda16;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = i / lda16;
        const int j = (int)(i - row * lda16);
        A16[i] = (__bf16)(j < r ? A[row * r + j] : 0.f);
    }
}

hipError_t launch_rows_to_bf16(const float *A, int64_t k, int r, int lda16, __bf16 *A16, hipStream_t s) {
    if (k <= 0) return hipSuccess;
    int64_t blocks = (k * lda16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_rows_to_bf16, dim3((unsigned)blocks), dim3(256), 0, s, A, k, r, lda16, A16);
    return hipGetLastError();
}

// Chunk list of a CSR matrix from its host row pointers.
int build_spmm_plan(const std::vector<int32_t> &rowptr, SpmmPlan *pl, hipStream_t s,
                    const std::vector<char> *skip) {
    const int64_t nrows = (int64_t)rowptr.size() - 1;
    std::vector<SpChunk> ch;
    std::vector<SpSplit> sp;
    ch.reserve(nrows + 16);
    int32_t slots = 0;
    for (int64_t i = 0; i < nrows; i++) {
        if (skip && (*skip)[i]) continue;  // written by someone else
        const int32_t b = rowptr[i], e = rowptr[i + 1];
        const int32_t len = e - b;
        if (len <= SPMM_CHUNK) {
            ch.push_back({(int32_t)i, b, e, -1});
        } else {
            const int32_t n = (len + SPMM_CHUNK - 1) / SPMM_CHUNK;
            sp.push_back({(int32_t)i, slots, n});
            for (int32_t c = 0; c < n; c++) {
                const int32_t cb = b + c * SPMM_CHUNK;
                ch.push_back({(int32_t)i, cb, std::min(e, cb + SPMM_CHUNK), slots++});
            }
        }
    }
    // long rows' chunks first: they are the stragglers
    std::stable_partition(ch.begin(), ch.end(), [](const SpChunk &c) { return c.dest >= 0; });
    pl->nrows = nrows;
    pl->nchunks = (int64_t)ch.size();
    pl->nsplits = (int64_t)sp.size();
    pl->nslots = slots;
    pl->chunks = nullptr;
    pl->splits = nullptr;
    if (!ch.empty()) {
        NMF_HIP(hipMalloc((void **)&pl->chunks, ch.size() * sizeof(SpChunk)));
        NMF_HIP(hipMemcpyAsync(pl->chunks, ch.data(), ch.size() * sizeof(SpChunk),
                               hipMemcpyHostToDevice, s));
    }
    if (!sp.empty()) {
        NMF_HIP(hipMalloc((void **)&pl->splits, sp.size() * sizeof(SpSplit)));
        NMF_HIP(hipMemcpyAsync(pl->splits, sp.data(), sp.size() * sizeof(SpSplit),
                               hipMemcpyHostToDevice, s));
    }
    NMF_HIP(hipStreamSynchronize(s));
    return NMF_OK;
}

void free_spmm_plan(SpmmPlan *pl) {
    if (pl->chunks) (void)hipFree(pl->chunks);
    if (pl->splits) (void)hipFree(pl->splits);
    pl->chunks = nullptr;
    pl->splits = nullptr;
}

}  // namespace nmfi

namespace nmfi {

// one wave per row, rows read straight from the row pointers
template <typename TA, int VEC, int LPN, int NV>
__global__ __launch_bounds__(256) void k_spmm_rows(const int32_t *__restrict__ rowptr, int64_t nrows,
                                                   const int32_t *__restrict__ colidx,
                                                   const float *__restrict__ vals,
                                                   const TA *__restrict__ A, int r, int lda,
                                                   float *__restrict__ P) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= nrows) return;
    float acc[NV][VEC];
#pragma unroll
    for (int q = 0; q < NV; q++)
#pragma unroll
        for (int v = 0; v < VEC; v++) acc[q][v] = 0.f;
    spmm_range<TA, VEC, LPN, NV>(rowptr[w], rowptr[w + 1], colidx, vals, A, r, lda, acc);
    spmm_finish<VEC, LPN, NV>(acc, r, P + w * r);
}

// The rows of several matrices in one launch (a fold-in batch of several
// requests): launch row w belongs to the last request with row0 <= w and is
// written to row p0 + (w - row0) of P; each row's arithmetic is that of
// k_spmm_rows.
template <typename TA, int VEC, int LPN, int NV>
__global__ __launch_bounds__(256) void k_spmm_rows_multi(const SpRowsReq *__restrict__ reqs, int nreq,
                                                         int64_t nrows, const TA *__restrict__ A, int r,
                                                         int lda, float *__restrict__ P) {
    const int64_t w = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= nrows) return;
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (reqs[mid].row0 <= w) lo = mid;
        else hi = mid - 1;
    }
    const SpRowsReq q = reqs[lo];
    const int64_t i = w - q.row0;
    float acc[NV][VEC];
#pragma unroll
    for (int t = 0; t < NV; t++)
#pragma unroll
        for (int v = 0; v < VEC; v++) acc[t][v] = 0.f;
    spmm_range<TA, VEC, LPN, NV>(q.rowptr[i], q.rowptr[i + 1], q.colidx, q.vals, A, r, lda, acc);
    spmm_finish<VEC, LPN, NV>(acc, r, P + (q.p0 + i) * r);
}

hipError_t launch_spmm_rows_multi(const SpRowsReq *reqs, int nreq, int64_t nrows, const float *A,
                                  const __bf16 *A16, int lda16, int r, float *P, hipStream_t s) {
    if (nrows <= 0 || nreq <= 0) return hipSuccess;
    const dim3 grid((unsigned)((nrows + 3) / 4)), blk(256);
    if (A16)
        hipLaunchKernelGGL((k_spmm_rows_multi<__bf16, NMF_SPMM_VEC16, 128 / NMF_SPMM_VEC16, 1>), grid, blk, 0, s,
                           reqs, nreq, nrows, A16, r, lda16, P);
    else if (r % 4 == 0 && r <= 128)
        hipLaunchKernelGGL((k_spmm_rows_multi<float, 4, 32, 1>), grid, blk, 0, s, reqs, nreq, nrows, A, r, r, P);
    else if (r <= 64)
        hipLaunchKernelGGL((k_spmm_rows_multi<float, 1, 64, 1>), grid, blk, 0, s, reqs, nreq, nrows, A, r, r, P);
    else
        hipLaunchKernelGGL((k_spmm_rows_multi<float, 1, 64, 2>), grid, blk, 0, s, reqs, nreq, nrows, A, r, r, P);
    return hipGetLastError();
}

hipError_t launch_spmm_rows(const int32_t *rowptr, int64_t nrows, const int32_t *colidx,
                            const float *vals, const float *A, int r, float *P, hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    const dim3 grid((unsigned)((nrows + 3) / 4)), blk(256);
    if (r % 4 == 0 && r <= 128)
        hipLaunchKernelGGL((k_spmm_rows<float, 4, 32, 1>), grid, blk, 0, s, rowptr, nrows, colidx, vals, A, r, r, P);
    else if (r <= 64)
        hipLaunchKernelGGL((k_spmm_rows<float, 1, 64, 1>), grid, blk, 0, s, rowptr, nrows, colidx, vals, A, r, r, P);
    else
        hipLaunchKernelGGL((k_spmm_rows<float, 1, 64, 2>), grid, blk, 0, s, rowptr, nrows, colidx, vals, A, r, r, P);
    return hipGetLastError();
}

hipError_t launch_spmm_rows16(const int32_t *rowptr, int64_t nrows, const int32_t *colidx,
                              const float *vals, const __bf16 *A16, int lda16, int r, float *P,
                              hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    const dim3 grid((unsigned)((nrows + 3) / 4)), blk(256);
    hipLaunchKernelGGL((k_spmm_rows<__bf16, NMF_SPMM_VEC16, 128 / NMF_SPMM_VEC16, 1>), grid, blk, 0, s, rowptr,
                       nrows, colidx, vals, A16, r, lda16, P);
    return hipGetLastError();
}

}  // namespace nmfi

// ------------------------------------------------------------------ hot columns
namespace nmfi {

// V_hot (m x T with row stride T, T >= the number of hot columns; zero
// elsewhere): V_hot[i][slot[j]] = V[i][j] for the stored entries of the hot
// columns (slot[j] >= 0).
__global__ void k_hot_scatter_v(const int32_t *__restrict__ rowptr, int64_t m,
                                const int32_t *__restrict__ colidx, const float *__restrict__ vals,
                                const int32_t *__restrict__ slot, int T, float *__restrict__ Vhot) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        float *row = Vhot + i * T;
        for (int t = 0; t < T; t++) row[t] = 0.f;
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
            const int32_t sl = slot[colidx[e]];
            if (sl >= 0) row[sl] = vals[e];
        }
    }
}

hipError_t launch_hot_scatter_v(const int32_t *rowptr, int64_t m, const int32_t *colidx,
                                const float *vals, const int32_t *slot, int T, float *Vhot,
                                hipStream_t s) {
    if (m <= 0 || T <= 0) return hipSuccess;
    int64_t blocks = (m + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_hot_scatter_v, dim3((unsigned)blocks), dim3(256), 0, s, rowptr, m, colidx,
                       vals, slot, T, Vhot);
    return hipGetLastError();
}

// P[idx[t]] = Phot[t] for the T hot rows (r floats each)
__global__ void k_hot_rows_out(const float *__restrict__ Phot, const int32_t *__restrict__ idx,
                               int T, int r, float *__restrict__ P) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)T * r;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = e / r, a = e - t * r;
        P[(int64_t)idx[t] * r + a] = Phot[e];
    }
}

hipError_t launch_hot_rows_out(const float *Phot, const int32_t *idx, int T, int r, float *P,
                               hipStream_t s) {
    if (T <= 0) return hipSuccess;
    int64_t blocks = ((int64_t)T * r + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_hot_rows_out, dim3((unsigned)blocks), dim3(256), 0, s, Phot, idx, T, r, P);
    return hipGetLastError();
}

}  // namespace nmfi
