// Dense data product (Algorithm 2's Y = F V' and G'V_i; Section 4.2: O(mnr)).
// P (c x r) = X (c x k) * A (k x r), with X = V' (trans = 0: the H-update,
// A = W) or X = V (trans = 1: the W-update, A = Ht).  V is m x n row-major
// with leading dimension ld.
//
// Each block of four waves computes a 128 x R32 slab of P (R32 = r rounded
// up to 32) over one slice of k (split-K).  Per stage it streams a 128 x BK
// tile of X (16 KB: BK = 32 floats or 64 BF16 values) and a BK x R32 tile of
// A with 16-byte loads into registers, one stage ahead of the MFMAs, and
// stores them into the block's one LDS stage buffer once every wave has
// read the previous stage (two barriers per stage; one buffer instead of
// two lets four blocks share a CU, twice the loads in flight).
// Wave w owns rows [32w, 32w + 32) of the slab and accumulates NT 32x32
// tiles: FP32 32x32x2 MFMAs on float operands, or BF16 32x32x16 MFMAs with
// FP32 accumulation.  In BF16 mode X is always read along k (V for the
// W-update, a transposed BF16 copy of V for the H-update) and A arrives as a
// BF16 copy transposed to R32 x K, so every tile moves with 16-byte loads and
// stores and no lane-by-lane transposition.
// Split-K partials are summed in slice order by a second kernel, so the
// result is deterministic; a P entry's arithmetic depends only on its
// slice's k range, never on the block that computes it.
#include "kernels_common.h"
#include <math.h>

#include <algorithm>

#include "dense_tuned.h"
#include "nmf_internal.h"

namespace nmfi {

typedef float f32x4a __attribute__((ext_vector_type(4)));

template <bool BF16>
struct DenseCfg;
template <>
struct DenseCfg<false> {
    using T = float;
    static constexpr int BK = 32;    // k per stage
    static constexpr int VEC = 4;    // elements per 16-byte load
};
template <>
struct DenseCfg<true> {
    using T = __bf16;
    static constexpr int BK = 64;
    static constexpr int VEC = 8;
};

// LDS layout of the stage buffer: one row per row of P (Xs) and per column of
// P (As), k along the row.
//   FP32: Xs[BM][BK + 4], As[R32][BK + 4], the 32 k of a stage stored
//         even k first, then odd k (position perm(k) = (k % 2) * 16 + k / 2):
//         the 32x32x2 MFMA's lanes 0-31 take the even k and lanes 32-63 the
//         odd k of each pair, so a lane's sixteen operands of a stage are 16
//         consecutive floats -- four 128-bit reads; the 144-byte pitch spreads
//         16 lanes' rows over all banks.
//   BF16: Xs[BM][BK + 8], As[R32][BK + 8] (a lane's operand is eight
//         consecutive k, one 16-byte read; the 144-byte pitch spreads the 32
//         rows of a half-wave over all banks).
//   FP32 with X = V' (XT): Xs[BK][BM + 4] instead (k-major, as V's rows
//         arrive: 16-byte stores; a lane reads its one-float operands per k).
template <bool BF16, bool XT, int NT>
struct DenseLds {
    static constexpr int BK = DenseCfg<BF16>::BK;
    static constexpr int R32 = 32 * NT;
    static constexpr bool XKMAJOR = XT && !BF16;
    static constexpr int XP = BF16 ? BK + 8 : (XKMAJOR ? DENSE_BM + 4 : BK + 4);  // pitch (elements)
    static constexpr int AP = BF16 ? BK + 8 : BK + 4;
    static constexpr int X_ELEMS = XKMAJOR ? BK * XP : DENSE_BM * XP;
    static constexpr int A_ELEMS = R32 * AP;
    static constexpr int ESZ = BF16 ? 2 : 4;
    static constexpr int STAGE_BYTES = ((X_ELEMS + A_ELEMS) * ESZ + 15) & ~15;
    static constexpr int BYTES = STAGE_BYTES;
};


// 128 rows of P = X A starting at row c0, summed over k in [kb, ke), written
// to o (C x r).  lds: DenseLds<BF16, XT, NT>::BYTES bytes, 16-byte aligned.
// vec_ok: V's rows and base are 16-byte aligned (ld * sizeof(T) % 16 == 0).
// A16 (BF16 mode): the factor as BF16, transposed, R32 x lda16 (row j holds
// A[., j]); unused in FP32 mode, where A (k x r float32) is read directly.
template <bool BF16, bool XT, int NT>
__device__ __forceinline__ void dense_body(const void *__restrict__ Vv, int64_t ld, int64_t C,
                                           const float *__restrict__ A, int r,
                                           const __bf16 *__restrict__ A16, int64_t lda16,
                                           int64_t c0, int64_t kb, int64_t ke, bool vec_ok,
                                           char *lds, float *__restrict__ o) {
    static_assert(!(BF16 && XT), "BF16 products read X along k");
    using Cfg = DenseCfg<BF16>;
    using T = typename Cfg::T;
    using L = DenseLds<BF16, XT, NT>;
    constexpr int BK = Cfg::BK, VEC = Cfg::VEC, R32 = 32 * NT, BM = DENSE_BM;
    // X tile: 1024 16-byte chunks, four per thread
    constexpr int XCH = BM * BK * (int)sizeof(T) / 16 / 256;
    static_assert(XCH == 4, "a 16 KB X tile per stage");
    // A tile in chunks (BK * R32 / 4 of four floats, or R32 * BK / 8 of eight
    // BF16 values of one row j of A16).  FP32 takes a float4 of four j of one
    // k, stored as four 4-byte writes into four rows; or, for the widest tile
    // with X = V' (the hot columns' product), four consecutive k of one
    // column j, stored as two 8-byte pairs -- the faster of the two there,
    // the slower everywhere else (measured).
    constexpr bool A_KPAIRS = !BF16 && XT && NT == 4;
    // FP32 float4 chunk q of the A tile: row kk of the stage, columns j..j+3.
    // A wave's 64 chunks are eight rows (every other k of one half of the
    // stage, so their even/odd positions are eight consecutive floats) by
    // eight column groups: each row is one 128-byte read, and the four
    // 4-byte stores of a chunk meet at most two lanes per bank.
    auto a_chunk = [](int q, int &kk, int &j) {
        constexpr int CPR = R32 / 4;  // column groups (a multiple of 8)
        const int kl = q & 7, j4 = (q >> 3) % CPR, g = (q >> 3) / CPR;  // g < BK / 8
        kk = 16 * (g >> 1) + 2 * kl + (g & 1);
        j = 4 * j4;
    };
    constexpr int ACH = BK * R32 / 4 / 256 / (BF16 ? 2 : 1);
    static_assert(ACH >= 1, "A tile smaller than one chunk per thread");
    const T *__restrict__ V = (const T *)Vv;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool a_vec = (r % 4) == 0 && ((uintptr_t)A % 16) == 0;

    typedef T tvec __attribute__((ext_vector_type(VEC)));
    tvec xr[XCH];
    f32x4a ar[BF16 ? 1 : ACH];
    bf16x8 ar16[BF16 ? ACH : 1];

    auto load_stage = [&](int64_t k0) {
#pragma unroll
        for (int u = 0; u < XCH; u++) {
            const int q = tid + 256 * u;
            int64_t row, col;  // element (row, col) of V where the chunk starts
            int64_t lim;       // elements of the chunk inside the tile's bounds
            if constexpr (XT) {  // V rows are k, 128 contiguous c per row
                constexpr int CPR = BM / VEC;  // chunks per row
                const int kk = q / CPR, cc = (q % CPR) * VEC;
                row = k0 + kk;
                col = c0 + cc;
                lim = (row < ke) ? min<int64_t>(VEC, C - col) : 0;
            } else {  // V rows are c, BK contiguous k per row
                constexpr int CPR = BK / VEC;
                const int rr = q / CPR, kk = (q % CPR) * VEC;
                row = c0 + rr;
                col = k0 + kk;
                lim = (row < C) ? min<int64_t>(VEC, ke - col) : 0;
            }
            if (vec_ok && lim == VEC) {
                xr[u] = *(const tvec *)(V + row * ld + col);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; e++) xr[u][e] = e < lim ? V[row * ld + col + e] : (T)0.f;
            }
        }
#pragma unroll
        for (int u = 0; u < ACH; u++) {
            const int q = tid + 256 * u;
            if constexpr (BF16) {  // row j of A16, eight k
                constexpr int CPR = BK / 8;
                const int j = q / CPR, kk = (q % CPR) * 8;
                const int64_t gk = k0 + kk;
                if (gk + 8 <= ke) {
                    ar16[u] = *(const bf16x8 *)(A16 + j * lda16 + gk);
                } else {
#pragma unroll
                    for (int e = 0; e < 8; e++) ar16[u][e] = gk + e < ke ? A16[j * lda16 + gk + e] : (__bf16)0.f;
                }
            } else if constexpr (A_KPAIRS) {  // four consecutive k of one column j
                const int j = q % R32, kq = (q / R32) * 4;
                const float *Ab = A + k0 * r;  // the stage's first row (uniform)
                const int kn = (int)min<int64_t>(ke - k0, BK);
#pragma unroll
                for (int e = 0; e < 4; e++) ar[u][e] = (kq + e < kn && j < r) ? Ab[(kq + e) * r + j] : 0.f;
            } else {  // four consecutive j of one row k of A (a float4)
                int kk, j;
                a_chunk(q, kk, j);
                const int64_t gk = k0 + kk;
                if (gk < ke && a_vec && j + 4 <= r) {
                    ar[u] = *(const f32x4a *)(A + gk * r + j);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; e++) ar[u][e] = (gk < ke && j + e < r) ? A[gk * r + j + e] : 0.f;
                }
            }
        }
    };

    auto store_stage = [&](char *buf) {
        T *Xs = (T *)buf;
        T *As = (T *)(buf + L::X_ELEMS * L::ESZ);
#pragma unroll
        for (int u = 0; u < XCH; u++) {
            const int q = tid + 256 * u;
            if constexpr (XT) {  // FP32 only: Xs[k][c]
                constexpr int CPR = BM / VEC;
                const int kk = q / CPR, cc = (q % CPR) * VEC;
                *(tvec *)(Xs + kk * L::XP + cc) = xr[u];
            } else {
                constexpr int CPR = BK / VEC;
                const int rr = q / CPR, kk = (q % CPR) * VEC;
                if constexpr (BF16) {  // Xs[c][k]
                    *(tvec *)(Xs + rr * L::XP + kk) = xr[u];
                } else {  // k .. k+3 of one c (k % 4 == 0): evens and odds are pairs
                    f32x2 ev, od;
                    ev[0] = xr[u][0]; ev[1] = xr[u][2];
                    od[0] = xr[u][1]; od[1] = xr[u][3];
                    *(f32x2 *)(Xs + rr * L::XP + (kk >> 1)) = ev;
                    *(f32x2 *)(Xs + rr * L::XP + 16 + (kk >> 1)) = od;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < ACH; u++) {
            const int q = tid + 256 * u;
            if constexpr (BF16) {  // As[j][k]
                constexpr int CPR = BK / 8;
                const int j = q / CPR, kk = (q % CPR) * 8;
                *(bf16x8 *)(As + j * L::AP + kk) = ar16[u];
            } else if constexpr (A_KPAIRS) {  // k .. k+3 of one j (k % 4 == 0): pairs, as for X
                const int j = q % R32, kq = (q / R32) * 4;
                f32x2 ev, od;
                ev[0] = ar[u][0]; ev[1] = ar[u][2];
                od[0] = ar[u][1]; od[1] = ar[u][3];
                *(f32x2 *)(As + j * L::AP + (kq >> 1)) = ev;
                *(f32x2 *)(As + j * L::AP + 16 + (kq >> 1)) = od;
            } else {  // the four j of one k, into four rows
                int kk, j;
                a_chunk(q, kk, j);
                const int pk = (kk & 1) * 16 + (kk >> 1);
#pragma unroll
                for (int e = 0; e < 4; e++) As[(j + e) * L::AP + pk] = ar[u][e];
            }
        }
    };

    f32x16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) acc[t] = f32x16{};

    auto compute_stage = [&](const char *buf) {
        const T *Xs = (const T *)buf;
        const T *As = (const T *)(buf + L::X_ELEMS * L::ESZ);
        if constexpr (BF16) {
#pragma unroll
            for (int ks = 0; ks < BK / 16; ks++) {
                const int kq = 16 * ks + 8 * (lane >> 5);
                const bf16x8 a_op = *(const bf16x8 *)(Xs + (32 * wave + (lane & 31)) * L::XP + kq);
#pragma unroll
                for (int t = 0; t < NT; t++) {
                    const bf16x8 b_op = *(const bf16x8 *)(As + (32 * t + (lane & 31)) * L::AP + kq);
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_op, b_op, acc[t], 0, 0, 0);
                }
            }
        } else {
            // lane half h takes k = 2 kp + h: the sixteen floats at h * 16 of its row
            const int h16 = 16 * (lane >> 5);
#pragma unroll
            for (int half = 0; half < 2; half++) {  // kp in [8 half, 8 half + 8)
                float a_op[8];
                if constexpr (L::XKMAJOR) {
#pragma unroll
                    for (int e = 0; e < 8; e++)
                        a_op[e] = Xs[(2 * (8 * half + e) + (lane >> 5)) * L::XP + 32 * wave + (lane & 31)];
                } else {
                    const f32x4a *pa = (const f32x4a *)(Xs + (32 * wave + (lane & 31)) * L::XP + h16 + 8 * half);
                    const f32x4a a0 = pa[0], a1 = pa[1];
#pragma unroll
                    for (int e = 0; e < 4; e++) { a_op[e] = a0[e]; a_op[4 + e] = a1[e]; }
                }
#pragma unroll
                for (int t = 0; t < NT; t++) {
                    const f32x4a *pb = (const f32x4a *)(As + (32 * t + (lane & 31)) * L::AP + h16 + 8 * half);
                    const f32x4a b0 = pb[0], b1 = pb[1];
                    float b_op[8];
#pragma unroll
                    for (int e = 0; e < 4; e++) { b_op[e] = b0[e]; b_op[4 + e] = b1[e]; }
#pragma unroll
                    for (int kp = 0; kp < 8; kp++)
                        acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a_op[kp], b_op[kp], acc[t], 0, 0, 0);
                }
            }
        }
    };

    const int64_t nstage = (ke - kb + BK - 1) / BK;
    if (nstage > 0) {
        load_stage(kb);
        store_stage(lds);
        __syncthreads();
        for (int64_t st = 0; st < nstage; st++) {
            const bool more = st + 1 < nstage;
            if (more) load_stage(kb + (st + 1) * BK);
            compute_stage(lds);
            // every wave's reads of this stage end before the next stage
            // overwrites it (more is uniform in the block)
            if (more) {
                __syncthreads();
                store_stage(lds);
                __syncthreads();
            }
        }
    }
    // acc[t][v]: row 8 (v / 4) + 4 (lane / 32) + v % 4 of the wave's 32, column lane % 32
#pragma unroll
    for (int t = 0; t < NT; t++) {
#pragma unroll
        for (int v = 0; v < 16; v++) {
            const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3), j = lane & 31;
            const int64_t c = c0 + 32 * wave + i;
            const int a = 32 * t + j;
            if (c < C && a < r) o[c * r + a] = acc[t][v];
        }
    }
}

template <bool BF16, bool XT, int NT>
__global__ __launch_bounds__(256) void k_dense(const void *__restrict__ V, int64_t ld, int64_t C,
                                               int64_t K, const float *__restrict__ A, int r,
                                               const __bf16 *__restrict__ A16, int64_t lda16,
                                               int64_t kchunk, int vec_ok, float *__restrict__ out) {
    __shared__ __attribute__((aligned(16))) char lds[DenseLds<BF16, XT, NT>::BYTES];
    const int64_t kb = (int64_t)blockIdx.y * kchunk;
    dense_body<BF16, XT, NT>(V, ld, C, A, r, A16, lda16, (int64_t)blockIdx.x * DENSE_BM, kb,
                             min(K, kb + kchunk), vec_ok != 0, lds, out + (int64_t)blockIdx.y * C * r);
}

// A16[j][k] = bf16(A[k][j]) for j < r, 0 for r <= j < R32 (rows of lda16 >= K
// entries; columns K..lda16 are left alone).  A tile of 64 rows of A (64 r <=
// 8192 contiguous floats) moves through LDS: every thread issues all of its
// (coalesced) loads of the tile at once, and then packs eight consecutive k of
// one row j into one 16-byte store.  LDS rows are S = r or r + 1 (the odd
// one) floats apart, so the eight lanes of one j and the eight k that a lane
// reads fall in 64 distinct banks.
constexpr int FT16_U = 32;  // loads per thread: 256 * 32 = 64 rows of r <= 128

__device__ __forceinline__ void ft16_load(const float *__restrict__ A, int64_t K, int r, int64_t k0,
                                          float (&v)[FT16_U]) {
    const int nflat = (int)min<int64_t>(64, K - k0) * r;
    const float *src = A + k0 * r;
#pragma unroll
    for (int u = 0; u < FT16_U; ++u) {
        const int f = u * 256 + (int)threadIdx.x;
        if (f < nflat) v[u] = src[f];
    }
}

// element f = u * 256 + thread of the tile is A[k0 + f / r][f % r]; the row
// and column advance by 256 / r and 256 % r from one u to the next
__device__ __forceinline__ void ft16_to_lds(int64_t K, int r, int64_t k0, const float (&v)[FT16_U],
                                            float *tile) {
    const int S = r | 1;
    const int nflat = (int)min<int64_t>(64, K - k0) * r;
    const int dq = 256 / r, dr = 256 - dq * r;
    int kk = (int)threadIdx.x / r, j = (int)threadIdx.x - kk * r;
#pragma unroll
    for (int u = 0; u < FT16_U; ++u) {
        if (u * 256 + (int)threadIdx.x < nflat) tile[kk * S + j] = v[u];
        kk += dq;
        j += dr;
        if (j >= r) { j -= r; ++kk; }
    }
}

__device__ __forceinline__ void ft16_store(int64_t K, int r, int R32, __bf16 *__restrict__ A16,
                                           int64_t lda16, int64_t k0, const float *tile) {
    const int S = r | 1;
    const int nk = (int)min<int64_t>(64, K - k0);
    const bool vst = (((uintptr_t)A16 | (uintptr_t)(lda16 * 2)) & 15) == 0;
    for (int e = threadIdx.x; e < R32 * 8; e += blockDim.x) {
        const int j = e >> 3, kk0 = (e & 7) * 8;
        if (kk0 >= nk) continue;
        float x[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) x[t] = j < r && kk0 + t < nk ? tile[(kk0 + t) * S + j] : 0.f;
        __bf16 *dst = A16 + j * lda16 + k0 + kk0;
        if (vst && kk0 + 8 <= nk) {
            uint32_t w[4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                w[t] = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)x[2 * t]) |
                       (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)x[2 * t + 1]) << 16;
            *reinterpret_cast<uint4 *>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
        } else {
            for (int t = 0; t < 8 && kk0 + t < nk; ++t) dst[t] = (__bf16)x[t];
        }
    }
}

// one tile (k0 = first row of A)
__device__ __forceinline__ void factor_t16_body(const float *__restrict__ A, int64_t K, int r,
                                                int R32, __bf16 *__restrict__ A16, int64_t lda16,
                                                int64_t k0, float *tile /* 64 x 129 */) {
    float v[FT16_U];
    ft16_load(A, K, r, k0, v);
    ft16_to_lds(K, r, k0, v, tile);
    __syncthreads();
    ft16_store(K, r, R32, A16, lda16, k0, tile);
}

// every tile of one factor: a block takes tiles blockIdx.x, + gridDim.x, ...
// and loads the next while it stores the current
__global__ __launch_bounds__(256) void k_factor_t16(const float *__restrict__ A, int64_t K, int r,
                                                    int R32, __bf16 *__restrict__ A16, int64_t lda16) {
    __shared__ float tile[64 * 129];
    const int64_t ntiles = (K + 63) / 64;
    float v[FT16_U];
    int64_t t = blockIdx.x;
    if (t < ntiles) ft16_load(A, K, r, t * 64, v);
    for (; t < ntiles; t += gridDim.x) {
        ft16_to_lds(K, r, t * 64, v, tile);
        __syncthreads();
        if (t + gridDim.x < ntiles) ft16_load(A, K, r, (t + gridDim.x) * 64, v);
        ft16_store(K, r, R32, A16, lda16, t * 64, tile);
        __syncthreads();
    }
}

// y (cols x rows) = x' in BF16: 64 x 64 tiles through LDS
__global__ __launch_bounds__(256) void k_to_bf16_t(const float *__restrict__ x, int64_t rows,
                                                   int64_t cols, int64_t ld, __bf16 *__restrict__ y) {
    __shared__ float tile[64 * 65];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int i = e / 64, j = e % 64;
        tile[i * 65 + j] = (r0 + i < rows && c0 + j < cols) ? x[(r0 + i) * ld + c0 + j] : 0.f;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int j = e / 64, i = e % 64;
        if (c0 + j < cols && r0 + i < rows) y[(c0 + j) * rows + r0 + i] = (__bf16)tile[i * 65 + j];
    }
}

hipError_t launch_to_bf16_t(const float *x, int64_t rows, int64_t cols, int64_t ld, __bf16 *y,
                            hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const int64_t gy = (rows + 63) / 64, gx = (cols + 63) / 64;
    if (gy > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_to_bf16_t, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, x, rows, cols,
                       ld, y);
    return hipGetLastError();
}

// P = sum over split-K slices in slice order
// The split-K sum of one entry, in a fixed order: slices in groups of
// SPLIT_GROUP, each group summed in slice order, the group sums added in
// group order.  (Up to SPLIT_GROUP slices this is the plain slice-order sum.)
constexpr int SPLIT_GROUP = 8;

// Sum of slices g0 .. g1 - 1 (at most SPLIT_GROUP of them) of entry i, in
// slice order; all loads are issued before the adds.
__device__ __forceinline__ float group_sum(const float *__restrict__ part, int g0, int g1, int64_t n,
                                           int64_t i) {
    float v[SPLIT_GROUP];
#pragma unroll
    for (int k = 0; k < SPLIT_GROUP; k++) v[k] = g0 + k < g1 ? part[(int64_t)(g0 + k) * n + i] : 0.f;
    float gs = 0.f;
#pragma unroll
    for (int k = 0; k < SPLIT_GROUP; k++)
        if (g0 + k < g1) gs += v[k];
    return gs;
}

__device__ __forceinline__ float split_sum(const float *__restrict__ part, int nsplit, int64_t n,
                                           int64_t i) {
    float s = 0.f;
    for (int g0 = 0; g0 < nsplit; g0 += SPLIT_GROUP)
        s += group_sum(part, g0, min(nsplit, g0 + SPLIT_GROUP), n, i);
    return s;
}

__global__ void k_split_reduce(const float *__restrict__ part, int nsplit, int64_t n,
                               float *__restrict__ P) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        P[i] = split_sum(part, nsplit, n, i);
}

// Many slices: the same sum in two parallel passes.  Pass 1 writes each
// group's sum over the group's first slice (in place: a group is read and
// written by one thread per entry), pass 2 adds the group sums in order.
__global__ void k_split_groups(float *__restrict__ part, int nsplit, int64_t n) {
    const int ng = (nsplit + SPLIT_GROUP - 1) / SPLIT_GROUP;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * ng;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int g = (int)(e / n);
        const int64_t i = e - (int64_t)g * n;
        const int g0 = g * SPLIT_GROUP;
        part[(int64_t)g0 * n + i] = group_sum(part, g0, min(nsplit, g0 + SPLIT_GROUP), n, i);
    }
}

__global__ void k_split_final(const float *__restrict__ part, int nsplit, int64_t n,
                              float *__restrict__ P) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        // the group sums (at slices 0, SPLIT_GROUP, ...) added in order, eight
        // loads at a time
        float s = 0.f;
        for (int g0 = 0; g0 < nsplit; g0 += SPLIT_GROUP * SPLIT_GROUP) {
            float v[SPLIT_GROUP];
#pragma unroll
            for (int k = 0; k < SPLIT_GROUP; k++) {
                const int sl = g0 + k * SPLIT_GROUP;
                v[k] = sl < nsplit ? part[(int64_t)sl * n + i] : 0.f;
            }
#pragma unroll
            for (int k = 0; k < SPLIT_GROUP; k++)
                if (g0 + k * SPLIT_GROUP < nsplit) s += v[k];
        }
        P[i] = s;
    }
}

static hipError_t launch_split_reduce(float *part, int nsplit, int64_t n, float *P, hipStream_t s) {
    if (nsplit <= 4 * SPLIT_GROUP) {
        int64_t blocks = (n + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(k_split_reduce, dim3((unsigned)blocks), dim3(256), 0, s, part, nsplit, n, P);
        return hipGetLastError();
    }
    const int64_t ng = (nsplit + SPLIT_GROUP - 1) / SPLIT_GROUP;
    int64_t b1 = (n * ng + 255) / 256;
    if (b1 > 16384) b1 = 16384;
    hipLaunchKernelGGL(k_split_groups, dim3((unsigned)b1), dim3(256), 0, s, part, nsplit, n);
    int64_t b2 = (n + 255) / 256;
    if (b2 > 4096) b2 = 4096;
    hipLaunchKernelGGL(k_split_final, dim3((unsigned)b2), dim3(256), 0, s, part, nsplit, n, P);
    return hipGetLastError();
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

// split-K factor without a measurement: as many slices as keep the grid
// within one round of resident blocks (a block uses one stage buffer of LDS,
// so four fit per CU: 1024 on the chip), at least 256 k per slice.
// Measured at 20000 x 10000, r = 64: 5-8% faster than double-buffered LDS
// with a 2048 (FP32) or 1024 (BF16) block target rounded up.
constexpr int64_t DENSE_SPLIT_BLOCKS = 1024;
static int dense_rule_nsplit(int64_t C, int64_t K) {
    const int64_t rb = (C + DENSE_BM - 1) / DENSE_BM;
    int64_t ns = DENSE_SPLIT_BLOCKS / rb;
    const int64_t maxs = (K + 255) / 256;
    if (ns > maxs) ns = maxs;
    if (ns < 1) ns = 1;
    return (int)ns;
}

// index of the grid value nearest v in log scale
static int nearest_log(const long long *grid, int n, int64_t v) {
    int best = 0;
    double bd = 1e300;
    for (int i = 0; i < n; i++) {
        const double d = fabs(log((double)(v > 0 ? v : 1)) - log((double)grid[i]));
        if (d < bd) { bd = d; best = i; }
    }
    return best;
}

// slices of the split-K: from the autotuned table at the grid point nearest
// (C, K) in log scale, for the kernel instantiation and the column tiles --
// read as the block count it gave there (slices x the grid point's 128-row
// blocks) and divided by this product's row blocks, rounded down (the slices
// a product needs to fill the chip fall as its rows grow, and one block past
// a round of resident blocks costs a whole extra round: measured at 20000 x
// 10000, r = 64, 13 slices of the H-update's 79 row blocks, 1027 blocks,
// took 352 us against 300 us for 12) -- else the rule; at least 64 k per
// slice, at most 512 slices
int dense_nsplit(int64_t C, int64_t K, int r, int bf16, int xt) {
    const int nt = std::min(4, std::max(1, (r + 31) / 32));
    const int kern = bf16 ? 2 : (xt ? 1 : 0);
    constexpr int nC = (int)(sizeof kDenseTunedC / sizeof(long long));
    constexpr int nK = (int)(sizeof kDenseTunedK / sizeof(long long));
    const int ci = nearest_log(kDenseTunedC, nC, C);
    const int64_t tuned = kDenseTunedSplit[kern][nt - 1][ci][nearest_log(kDenseTunedK, nK, K)];
    int64_t ns;
    if (tuned > 0) {
        const int64_t blocks = tuned * ((kDenseTunedC[ci] + DENSE_BM - 1) / DENSE_BM);
        const int64_t rb = (C + DENSE_BM - 1) / DENSE_BM;
        ns = blocks / rb;
    } else {
        ns = dense_rule_nsplit(C, K);
    }
    const int64_t maxs = (K + 63) / 64;
    if (ns > maxs) ns = maxs;
    if (ns > 512) ns = 512;
    if (ns < 1) ns = 1;
    return (int)ns;
}

// slice length for ns slices: a multiple of 64 (both stage depths)
static int64_t kchunk_for(int64_t K, int64_t ns) {
    int64_t kchunk = (K + ns - 1) / ns;
    kchunk = ((kchunk + 63) / 64) * 64;
    return kchunk < 64 ? 64 : kchunk;
}
int64_t dense_kchunk(int64_t C, int64_t K, int r, int bf16, int xt) {
    return kchunk_for(K, dense_nsplit(C, K, r, bf16, xt));
}

// Split-K partials of the larger half (either precision), then the BF16
// factor copy (R32 x lda16 with lda16 = max(m, n) rounded up to 64).
static size_t dense_partial_bytes(int64_t m, int64_t n, int r) {
    // slices actually used (a single slice writes P directly)
    auto used = [&](int64_t C, int64_t K, int bf16, int xt) {
        const int64_t kc = dense_kchunk(C, K, r, bf16, xt);
        const int64_t ns = K > 0 ? (K + kc - 1) / kc : 0;
        return ns > 1 ? ns * C : 0;
    };
    // H-update: C = n, K = m (FP32 reads V' k-major); W-update: C = m, K = n
    const int64_t most = std::max(std::max(used(n, m, 0, 1), used(m, n, 0, 0)),
                                  std::max(used(n, m, 1, 0), used(m, n, 1, 0)));
    return (((size_t)most * r * sizeof(float)) + 255) & ~(size_t)255;
}
static int64_t dense_lda16(int64_t m, int64_t n) {
    const int64_t k = m > n ? m : n;
    return (k + 63) / 64 * 64;
}
size_t dense_scratch_bytes(int64_t m, int64_t n, int r) {
    const int R32 = (r + 31) / 32 * 32;
    return dense_partial_bytes(m, n, r) + (size_t)R32 * dense_lda16(m, n) * 2 + 256;
}
// ... with the slices forced (force_nsplit > 0, either half): the partials
// region grows to hold them
size_t dense_forced_partial_bytes(int64_t m, int64_t n, int r, int force_nsplit) {
    size_t b = dense_partial_bytes(m, n, r);
    if (force_nsplit > 0)
        for (int h = 0; h < 2; h++) {
            const int64_t C = h ? m : n, K = h ? n : m;
            const int64_t kc = kchunk_for(K, std::min<int64_t>(force_nsplit, (K + 63) / 64));
            const int64_t ns = (K + kc - 1) / kc;
            if (ns > 1) b = std::max(b, (((size_t)ns * C * r * sizeof(float)) + 255) & ~(size_t)255);
        }
    return b;
}
size_t dense_scratch_bytes_forced(int64_t m, int64_t n, int r, int force_nsplit) {
    const int R32 = (r + 31) / 32 * 32;
    return dense_forced_partial_bytes(m, n, r, force_nsplit) + (size_t)R32 * dense_lda16(m, n) * 2 + 256;
}

template <int NT>
static void dense_launch_nt(bool bf16, bool xt, const void *X, int64_t ld, int64_t C, int64_t K,
                            const float *A, int r, const __bf16 *A16, int64_t lda16, int64_t kchunk,
                            int vec_ok, float *out, dim3 grid, hipStream_t s) {
#define NMF_DL(B, XTT) hipLaunchKernelGGL((k_dense<B, XTT, NT>), grid, dim3(256), 0, s, X, ld, C, K, A, \
                                          r, A16, lda16, kchunk, vec_ok, out)
    if (bf16) NMF_DL(true, false);
    else if (xt) NMF_DL(false, true);
    else NMF_DL(false, false);
#undef NMF_DL
}

// 16-byte vector loads of V are used when its base and rows are 16-byte aligned
int dense_vec_ok(const void *V, int64_t ld, int bf16) {
    return ((uintptr_t)V % 16) == 0 && ((ld * (bf16 ? 2 : 4)) % 16) == 0;
}

// V (m x n, ld): float32, or its BF16 copy when bf16 != 0, in which case
// V16t (n x m) is the transposed BF16 copy (the H-update reads it; the
// W-update reads V).  trans = 0: P (n x r) = V' A; trans = 1: P (m x r) = V A.
// scratch: dense_scratch_bytes(m, n, r) bytes.
hipError_t launch_dense_product(const void *V, int bf16, int64_t m, int64_t n, int64_t ld,
                                const __bf16 *V16t, int trans, const float *A, int r, float *P,
                                float *scratch, hipStream_t s, int force_nsplit) {
    const bool h_update = trans == 0;
    const int64_t C = h_update ? n : m, K = h_update ? m : n;
    if (C == 0) return hipSuccess;
    if (K == 0) return hipErrorInvalidValue;  // callers reject empty V
    const int64_t kchunk = force_nsplit > 0 ? kchunk_for(K, std::min<int64_t>(force_nsplit, (K + 63) / 64))
                                            : dense_kchunk(C, K, r, bf16, h_update && !bf16);
    const int nsplit = (int)((K + kchunk - 1) / kchunk);
    float *out = nsplit > 1 ? scratch : P;
    const int NT = (r + 31) / 32;
    const void *X = V;
    int64_t ldx = ld;
    bool xt = h_update;
    __bf16 *A16 = nullptr;
    int64_t lda16 = 0;
    if (bf16) {
        if (h_update) {
            if (!V16t) return hipErrorInvalidValue;
            X = V16t;
            ldx = m;
        }
        xt = false;
        lda16 = dense_lda16(m, n);
        A16 = (__bf16 *)((char *)scratch + dense_forced_partial_bytes(m, n, r, force_nsplit));
        // four blocks fit a CU (33 KB of LDS each); tiles are shared out evenly
        const int64_t ntiles = (K + 63) / 64;
        const int64_t per = (ntiles + 4 * device_cu_count() - 1) / (4 * device_cu_count());
        hipLaunchKernelGGL(k_factor_t16, dim3((unsigned)((ntiles + per - 1) / per)), dim3(256), 0, s, A,
                           K, r, 32 * NT, A16, lda16);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    dim3 grid((unsigned)((C + DENSE_BM - 1) / DENSE_BM), (unsigned)(nsplit > 0 ? nsplit : 1));
    const int vec = dense_vec_ok(X, ldx, bf16);
    switch (NT) {
    case 1: dense_launch_nt<1>(bf16, xt, X, ldx, C, K, A, r, A16, lda16, kchunk, vec, out, grid, s); break;
    case 2: dense_launch_nt<2>(bf16, xt, X, ldx, C, K, A, r, A16, lda16, kchunk, vec, out, grid, s); break;
    case 3: dense_launch_nt<3>(bf16, xt, X, ldx, C, K, A, r, A16, lda16, kchunk, vec, out, grid, s); break;
    default: dense_launch_nt<4>(bf16, xt, X, ldx, C, K, A, r, A16, lda16, kchunk, vec, out, grid, s); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nsplit <= 1) return e;
    return launch_split_reduce(scratch, nsplit, C * r, P, s);
}

}  // namespace nmfi

// ------------------------------------------------------------------ batched
namespace nmfi {

// Many problems at once: block b computes 128 rows of one problem's P over
// one k slice (items[b].idx = row block * nsplit + slice) with the same body
// as the single-problem product, so the result is bitwise the same.
template <int NTMAX, bool XT, bool BF16>
__global__ __launch_bounds__(256) void k_bdense(const BItem *__restrict__ items,
                                                const BProdProb *__restrict__ probs) {
    __shared__ __attribute__((aligned(16))) char lds[DenseLds<BF16, XT, NTMAX>::BYTES];
    const BItem it = items[blockIdx.x];
    const BProdProb P = probs[it.prob];
    const int NT = (P.r + 31) / 32;
    const int slice = it.idx % P.nsplit;
    const int64_t c0 = (int64_t)(it.idx / P.nsplit) * DENSE_BM;
    const int64_t kb = (int64_t)slice * P.kchunk;
    const int64_t ke = min(P.K, kb + P.kchunk);
    float *o = P.nsplit > 1 ? P.part + (int64_t)slice * P.C * P.r : P.P;
    const bool vec = ((uintptr_t)P.V % 16) == 0 && ((P.ld * (BF16 ? 2 : 4)) % 16) == 0;
#define NMF_BD_BODY(N) \
    dense_body<BF16, XT, N>(P.V, P.ld, P.C, P.A, P.r, P.A16, P.lda16, c0, kb, ke, vec, lds, o)
    switch (NT) {
    case 1: NMF_BD_BODY(1); break;
    case 2: if constexpr (NTMAX >= 2) NMF_BD_BODY(2); break;
    case 3: if constexpr (NTMAX >= 3) NMF_BD_BODY(3); break;
    default: if constexpr (NTMAX >= 4) NMF_BD_BODY(4); break;
    }
#undef NMF_BD_BODY
}

// BF16 factor copies of many problems: item = (problem, block of 64 rows of A)
__global__ __launch_bounds__(256) void k_bfactor_t16(const BItem *__restrict__ items,
                                                     const BProdProb *__restrict__ probs) {
    __shared__ float tile[64 * 129];
    const BItem it = items[blockIdx.x];
    const BProdProb P = probs[it.prob];
    factor_t16_body(P.A, P.K, P.r, (P.r + 31) / 32 * 32, P.A16, P.lda16, (int64_t)it.idx * 64, tile);
}

// split-K sums of many problems, in the same order as the single-problem sum
__global__ void k_bsplit_reduce(const BItem *__restrict__ items, const BProdProb *__restrict__ probs) {
    const BItem it = items[blockIdx.x];
    const BProdProb P = probs[it.prob];
    const int64_t n = P.C * P.r;
    const int64_t e0 = (int64_t)it.idx * 4096;
    for (int64_t i = e0 + threadIdx.x; i < min(n, e0 + 4096); i += blockDim.x)
        P.P[i] = split_sum(P.part, P.nsplit, n, i);
}

hipError_t launch_bdense(const BItem *items, int64_t nitems, const BProdProb *probs, int ntmax,
                         bool xt, bool bf16, const BItem *red_items, int64_t nred,
                         const BItem *f16_items, int64_t nf16, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (bf16 && nf16 > 0)
        hipLaunchKernelGGL(k_bfactor_t16, dim3((unsigned)nf16), dim3(256), 0, s, f16_items, probs);
    const dim3 g((unsigned)nitems), b(256);
#define NMF_BD(NTM, X, B) hipLaunchKernelGGL((k_bdense<NTM, X, B>), g, b, 0, s, items, probs)
    if (ntmax <= 2) {
        if (bf16) NMF_BD(2, false, true);
        else if (xt) NMF_BD(2, true, false);
        else NMF_BD(2, false, false);
    } else {
        if (bf16) NMF_BD(4, false, true);
        else if (xt) NMF_BD(4, true, false);
        else NMF_BD(4, false, false);
    }
#undef NMF_BD
    if (nred > 0)
        hipLaunchKernelGGL(k_bsplit_reduce, dim3((unsigned)nred), dim3(256), 0, s, red_items, probs);
    return hipGetLastError();
}

}  // namespace nmfi
