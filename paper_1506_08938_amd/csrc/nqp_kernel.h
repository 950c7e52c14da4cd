// Algorithm 3 (Fast Combinational Algorithm for NQP, Section 3.4) as a
// persistent gfx950 kernel.
//
// Mapping.  L lanes (1, 2, 4, 8 or 16: a DPP quad, half-row or row)
// cooperate on one column; lane `sub` of the group owns the E contiguous
// coordinates [sub*E, sub*E + E) of the padded rank R = E*L.  The rescaled
// Hessian Q (unit diagonal) sits in LDS (QLayout: row stride SQ, each lane's
// segment of a row padded to a multiple of four floats); because Q is
// symmetric, both the matrix-vector products and the coordinate-descent
// gradient update read one row segment per lane: Q[j][sub*E .. sub*E+E).
// Group reductions (sums, the greedy argmax) are DPP butterflies, so every
// lane of a group holds bitwise-identical results.
//
// Persistence.  Each wave keeps 64/L columns in flight.  When a column meets
// its stopping rule the group writes the result and takes the next column
// index from a global counter (one atomic per wave per refill), so waves do
// not idle while a few of their columns need extra iterations.  A column's
// arithmetic never depends on which group or wave solves it, or when.
//
// Pad coordinates (r <= i < R) and frozen ones (Gamma_ii <= 0) have dsq = 0,
// an identity row/column in Q, y = 0 and q = 1: their gradient stays 1, their
// projected gradient and best step are 0, so they never move and never touch
// the other coordinates.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "nmf_internal.h"

namespace nmfi {

constexpr int NQP_BLOCK_SMALL = 256;  // threads per block of a small launch

__device__ __forceinline__ int f2i(float v) { return __builtin_bit_cast(int, v); }
__device__ __forceinline__ float i2f(int v) { return __builtin_bit_cast(float, v); }

template <int CTRL>
__device__ __forceinline__ float dppf(float v) {
    return i2f(__builtin_amdgcn_mov_dpp(f2i(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ int dppi(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dppd(double v) {
    long long b = __builtin_bit_cast(long long, v);
    int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    long long r = ((long long)hi << 32) | (unsigned int)lo;
    return __builtin_bit_cast(double, r);
}

// quad_perm selectors: xor 1 = [1,0,3,2], xor 2 = [2,3,0,1]
constexpr int DPP_XOR1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);
constexpr int DPP_XOR2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);
// lane i of each 8-lane half-row reads lane 7 - i; of each 16-lane row, 15 - i.
// Once every quad (half-row) agrees on a value these pair it with the other
// quad (half-row) of the group, so each stage is a butterfly step.
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_MIRROR = 0x140;
// lane S of each 16-lane row, broadcast to the row
constexpr int DPP_ROW_BCAST0 = 0x150;

// broadcast the value of group member S to every lane of its group
template <int L, int S>
__device__ __forceinline__ float grp_bcast(float v) {
    if constexpr (L == 1) {
        return v;
    } else if constexpr (L == 2) {
        return dppf<S | (S << 2) | ((2 + S) << 4) | ((2 + S) << 6)>(v);
    } else if constexpr (L == 4) {
        return dppf<S * 0x55>(v);
    } else if constexpr (L == 8) {
        // member S of the lower and of the upper half-row; keep the own half's
        const float lo = dppf<DPP_ROW_BCAST0 + S>(v);
        const float hi = dppf<DPP_ROW_BCAST0 + 8 + S>(v);
        return (threadIdx.x & 8) ? hi : lo;
    } else {
        static_assert(L == 16, "lanes per column: 1, 2, 4, 8 or 16");
        return dppf<DPP_ROW_BCAST0 + S>(v);
    }
}

template <int L>
__device__ __forceinline__ float grp_sum(float v) {
    if constexpr (L >= 2) v += dppf<DPP_XOR1>(v);
    if constexpr (L >= 4) v += dppf<DPP_XOR2>(v);
    if constexpr (L >= 8) v += dppf<DPP_HALF_MIRROR>(v);
    if constexpr (L >= 16) v += dppf<DPP_MIRROR>(v);
    return v;
}
template <int L>
__device__ __forceinline__ double grp_sum_d(double v) {
    if constexpr (L >= 2) v += dppd<DPP_XOR1>(v);
    if constexpr (L >= 4) v += dppd<DPP_XOR2>(v);
    if constexpr (L >= 8) v += dppd<DPP_HALF_MIRROR>(v);
    if constexpr (L >= 16) v += dppd<DPP_MIRROR>(v);
    return v;
}

#ifndef NMF_NQP_ARGMAX64
#define NMF_NQP_ARGMAX64 1  // 1: one 64-bit key compare per step (no branches)
#endif

// (best, idx, m) <- the entry with the largest best; lowest idx on ties.
// best >= 0 (a decrease), so its bit pattern orders like its value (after
// clearing the sign of a -0); the key (bits(best), ~idx) compares as one
// 64-bit unsigned integer: larger best first, then the lower index.
template <int CTRL>
__device__ __forceinline__ void argmax_step(float &best, int &idx, float &m) {
#if NMF_NQP_ARGMAX64
    const unsigned hi = (unsigned)f2i(best) & 0x7fffffffu, lo = ~(unsigned)idx;
    const unsigned ohi = (unsigned)dppi<CTRL>((int)hi), olo = (unsigned)dppi<CTRL>((int)lo);
    const float om = dppf<CTRL>(m);
    const unsigned long long k = ((unsigned long long)hi << 32) | lo;
    const unsigned long long ok = ((unsigned long long)ohi << 32) | olo;
    const bool take = ok > k;
    best = i2f((int)(take ? ohi : hi));
    idx = (int)~(take ? olo : lo);
    m = take ? om : m;
#else
    float ob = dppf<CTRL>(best);
    int oi = dppi<CTRL>(idx);
    float om = dppf<CTRL>(m);
    bool take = (ob > best) || (ob == best && oi < idx);
    best = take ? ob : best;
    idx = take ? oi : idx;
    m = take ? om : m;
#endif
}
#if NMF_NQP_ARGMAX64
// one butterfly step on the key halves (hi = bits of the decrease, lo = ~index)
template <int CTRL>
__device__ __forceinline__ void argmax_key_step(unsigned &hi, unsigned &lo, float &m) {
    const unsigned ohi = (unsigned)dppi<CTRL>((int)hi), olo = (unsigned)dppi<CTRL>((int)lo);
    const float om = dppf<CTRL>(m);
    const bool take = (((unsigned long long)ohi << 32) | olo) > (((unsigned long long)hi << 32) | lo);
    hi = take ? ohi : hi;
    lo = take ? olo : lo;
    m = take ? om : m;
}
#endif

template <int L>
__device__ __forceinline__ void grp_argmax(float &best, int &idx, float &m) {
#if NMF_NQP_ARGMAX64
    if constexpr (L >= 2) {
        // the key is formed once, carried through every step, and unpacked once
        unsigned hi = (unsigned)f2i(best) & 0x7fffffffu, lo = ~(unsigned)idx;
        argmax_key_step<DPP_XOR1>(hi, lo, m);
        if constexpr (L >= 4) argmax_key_step<DPP_XOR2>(hi, lo, m);
        if constexpr (L >= 8) argmax_key_step<DPP_HALF_MIRROR>(hi, lo, m);
        if constexpr (L >= 16) argmax_key_step<DPP_MIRROR>(hi, lo, m);
        best = i2f((int)hi);
        idx = (int)~lo;
    }
#else
    if constexpr (L >= 2) argmax_step<DPP_XOR1>(best, idx, m);
    if constexpr (L >= 4) argmax_step<DPP_XOR2>(best, idx, m);
    if constexpr (L >= 8) argmax_step<DPP_HALF_MIRROR>(best, idx, m);
    if constexpr (L >= 16) argmax_step<DPP_MIRROR>(best, idx, m);
#endif
}

#ifndef NMF_NQP_PADSEG
#define NMF_NQP_PADSEG 1  // 1: lane segments of Q rows padded to 16 bytes (b128 reads)
#endif

// LDS layout of Q: row j (of R) at j * SQ.  Padded form: group member sub's
// E entries, padded to ES (a multiple of four), are stored as ES/4 float4
// blocks interleaved across the group -- block q of member sub at
// (q * L + sub) * 4 -- so one 128-bit load per block q reads a contiguous
// run of the row across the group's lanes (no bank conflicts) at an
// immediate offset from one base address.  Plain form: member sub's entries
// contiguous at sub * E.
template <int E, int L>
struct QLayout {
    static constexpr int R = E * L;
    static constexpr int ES = NMF_NQP_PADSEG ? ((E + 3) & ~3) : E;
    static constexpr int SQ = NMF_NQP_PADSEG ? L * ES + 4 : ((R + 3) & ~3) + 4;
    // this member's first entry in row 0
    __device__ static constexpr int seg(int sub) { return NMF_NQP_PADSEG ? sub * 4 : sub * E; }
    // position of entry j within a row
    __device__ static constexpr int col(int j) {
        return NMF_NQP_PADSEG ? ((j % E) / 4 * L + j / E) * 4 + (j % E) % 4 : j;
    }
};

// the E entries of one lane's row segment, starting at p = row + seg(sub)
template <int E, int L>
__device__ __forceinline__ void load_seg(const float *__restrict__ p, float (&x)[E]) {
    if constexpr (NMF_NQP_PADSEG) {
        constexpr int ES = QLayout<E, L>::ES;
        float t[ES];
#pragma unroll
        for (int q = 0; q < ES / 4; q++) {
            const float4 v = *(const float4 *)(p + q * L * 4);
            t[4 * q] = v.x; t[4 * q + 1] = v.y; t[4 * q + 2] = v.z; t[4 * q + 3] = v.w;
        }
#pragma unroll
        for (int e = 0; e < E; e++) x[e] = t[e];
    } else {
#pragma unroll
        for (int e = 0; e < E; e++) x[e] = p[e];
    }
}

// out[e] = sum_j Q[sub*E + e][j] v_j for this lane's E rows; v is spread over
// the group (entry j lives in member j / E).  qseg = this lane's segment of
// row 0.
template <int E, int L, int S = 0>
__device__ __forceinline__ void matvec_acc(const float *__restrict__ qseg, const float (&v)[E],
                                           float (&out)[E]) {
    using QL = QLayout<E, L>;
    if constexpr (S < L) {
#pragma unroll
        for (int e2 = 0; e2 < E; e2++) {
            const float w = grp_bcast<L, S>(v[e2]);
            float row[E];
            load_seg<E, L>(qseg + (S * E + e2) * QL::SQ, row);  // Q symmetric: row j = column j
#pragma unroll
            for (int e = 0; e < E; e++) out[e] = fmaf(row[e], w, out[e]);
        }
        matvec_acc<E, L, S + 1>(qseg, v, out);
    }
}
// The rescaled Hessian in LDS never changes inside the kernel, so without a
// fence the compiler hoists its loads out of the persistent loop and tries to
// keep R*E of them in registers.  The fence makes every use reload it.
__device__ __forceinline__ void lds_reload_fence() { asm volatile("" ::: "memory"); }

template <int E, int L>
__device__ __forceinline__ void matvec(const float *__restrict__ qseg, const float (&v)[E],
                                       float (&out)[E]) {
    lds_reload_fence();
#pragma unroll
    for (int e = 0; e < E; e++) out[e] = 0.f;
    matvec_acc<E, L>(qseg, v, out);
}

__device__ __forceinline__ bool passive(float y, float g) { return y > 0.f || g < 0.f; }

// min and max(., 0) as one v_med3_f32 each (no NaN canonicalisation: every
// operand here is finite)
__device__ __forceinline__ float min2(float a, float b) {
    return __builtin_amdgcn_fmed3f(a, b, -__builtin_huge_valf());
}
__device__ __forceinline__ float relu(float a) {
    return __builtin_amdgcn_fmed3f(a, 0.f, __builtin_huge_valf());
}

// Occupancy target: about 4E live registers per lane (y, g, the search
// direction and the product), so ask for as many waves per SIMD as fit.
#ifndef NMF_NQP_WPE
#define NMF_NQP_WPE 0  // 0: occupancy from the table below
#endif
// The y update of a CD step changes one entry, y_p -= m.  Either a compare
// and select per entry (0), or an FMA per entry with the lane's segment of
// the unit vector e_p read from LDS (1): fma(-m, 1, y) = y - m at p, and
// fma(-m, 0, y) = y elsewhere, bitwise the same result.  The LDS form costs
// one FMA instead of three instructions per entry plus a few for the address
// and 128-bit reads; measured faster from E = 12 on, slower below.
#ifndef NMF_NQP_ONEHOT_LDS
#define NMF_NQP_ONEHOT_LDS -1  // -1: by E as measured; 0 or 1 forces a form
#endif
template <int E>
constexpr int nqp_oh_mode() {
    return NMF_NQP_ONEHOT_LDS >= 0 ? NMF_NQP_ONEHOT_LDS : (E >= 12 ? 1 : 0);
}

// Unit-vector windows (form 1): four copies of nqp_oh_lw() floats, copy k
// with its 1 at index R + k.  The lane's segment of e_p starts at offset
// R + k + base - p of copy k = (p - base - R) mod 4, a multiple of 4, so it
// is read with 16-byte-aligned loads.
template <int E, int L>
constexpr int nqp_oh_lw() {
    return (2 * E * L + 8 + 3) / 4 * 4;
}
template <int E, int L>
constexpr int nqp_oh_floats() {
    return nqp_oh_mode<E>() == 1 ? 4 * nqp_oh_lw<E, L>() : 4;
}

// LDS of one block: Q (R x SQ), sqrt-diagonal (R), unit-vector windows,
// and a few counters
template <int E, int L>
constexpr int nqp_lds_bytes() {
    return (E * L * QLayout<E, L>::SQ + E * L + nqp_oh_floats<E, L>()) * 4 + 64;
}

template <int E>
constexpr int nqp_regs_waves() {
    return NMF_NQP_WPE ? NMF_NQP_WPE : (E <= 12 ? 6 : (E <= 20 ? 4 : (E <= 28 ? 3 : 2)));
}

// Threads per block of a large launch.  The block's waves share one staged
// Q, so eight waves per block halve the LDS per wave; used when registers
// allow at least four waves per SIMD (two such blocks per CU), measured up to
// 25% faster than four-wave blocks at r = 100..128.
template <int E, int L>
constexpr int nqp_block() {
    return nqp_regs_waves<E>() >= 4 ? 512 : 256;
}

// Waves per SIMD: the register table, capped by how many blocks the 160 KB
// of LDS of a CU holds (a block puts block/256 waves on each of the 4 SIMDs).
// Asking for more than LDS allows makes the compiler drop the register cap.
template <int E, int L>
constexpr int nqp_waves_per_eu() {
    constexpr int by_regs = nqp_regs_waves<E>();
    constexpr int by_lds = (160 * 1024) / nqp_lds_bytes<E, L>() * (nqp_block<E, L>() / 256);
    return by_regs < by_lds ? by_regs : (by_lds > 0 ? by_lds : 1);
}

// Where one solve's columns come from and go to.
struct ColumnIO {
    const float *P;    // column j's data row: P + j * ldp (h = hsign * P + hadd)
    float hsign, hadd;
    float *X;          // column j's start point / solution: X + j * ldx
    int ldp, ldx;
    int32_t *iters;    // optional, per column
    int r;
    int max_inner;
    double eps;
    int ls_guard;
    int cold;
    int64_t ncols;     // columns of this launch (or chunk)
    int unit;          // columns per work unit; > 1: the fast-break's thread of computation
};

// Work counters over [0, n) work units: a global 64-bit counter, or a
// 32-bit LDS counter over the units of one chunk.
struct GlobalFetch {
    unsigned long long *ctr;
    int64_t n;
    __device__ __forceinline__ unsigned long long take(int cnt) {
        return atomicAdd(ctr, (unsigned long long)cnt);
    }
};
struct LdsFetch {
    unsigned int *ctr;
    int64_t n;
    __device__ __forceinline__ unsigned long long take(int cnt) {
        return (unsigned long long)atomicAdd(ctr, (unsigned int)cnt);
    }
};

// One wave's share of a batch of NQPs sharing the rescaled Hessian sQ (LDS,
// R x SQ) and its sqrt-diagonal sD (LDS): every group of L lanes solves
// columns taken from `fetch` until none are left.  Adds the iterations of the
// columns it finished (counted once per group) to my_inner.
// sZ (LDS) holds the unit-vector windows of the y update (nqp_oh_mode).
template <int E, int L, class Fetch>
__device__ __forceinline__ void nqp_columns(const float *__restrict__ sQ,
                                            const float *__restrict__ sD,
                                            const float *__restrict__ sZ, const ColumnIO &a,
                                            Fetch &fetch, unsigned long long &my_inner) {
    const int lane = threadIdx.x & 63;
    const int sub = lane & (L - 1);
    const int base = sub * E;
    using QL = QLayout<E, L>;
    const float *qseg = sQ + QL::seg(sub);
    const int r = a.r;

    float y[E], g[E];
#pragma unroll
    for (int e = 0; e < E; e++) { y[e] = 0.f; g[e] = 1.f; }
    bool active = false;
    bool exhausted = false;  // wave-uniform
    int64_t col = 0, cend = 0;  // current column; end of the group's work unit
    // fast-break threshold of the unit's thread of computation (Algorithm 3):
    // reset to 0 per unit, raised to each finished column's ||f~||^2;
    // negative when the fast-break is off
    double mstop = -1.0;
    double n0 = 0.0;
    int k = 0;

    for (;;) {
        // ------------------------------------------------ refill finished groups
        // the next column of the group's own unit, in order; else a new unit
        bool fresh = false;
        if (!active && col + 1 < cend) {
            col++;
            fresh = true;
        }
        if (!exhausted) {
            const unsigned long long needmask = __ballot(!active && !fresh && sub == 0);
            if (needmask) {
                const int cnt = __popcll(needmask);
                unsigned long long b0 = 0;
                if (lane == 0) b0 = fetch.take(cnt);
                const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(b0 & 0xffffffffull));
                const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b0 >> 32));
                b0 = ((unsigned long long)hi << 32) | lo;
                if (b0 + (unsigned long long)cnt >= (unsigned long long)fetch.n) exhausted = true;
                const int leader = lane - sub;
                const int rank = __popcll(needmask & ((1ull << leader) - 1ull));
                if (!active && !fresh) {
                    const unsigned long long u = b0 + (unsigned long long)rank;
                    if (u < (unsigned long long)fetch.n) {
                        col = (int64_t)u * a.unit;
                        cend = min(a.ncols, col + a.unit);
                        mstop = a.unit > 1 ? 0.0 : -1.0;
                        fresh = true;
                    }
                }
            }
        }
        {
            {
                if (fresh) {
                    // y0 = x0 * sqrt(diag), q = h / sqrt(diag), g0 = Q y0 + q
                    float q[E];
                    const float *prow = a.P + col * (int64_t)a.ldp;
                    const float *xrow = a.X + col * (int64_t)a.ldx;
                    // The loads of the P row are issued together (a pad
                    // coordinate reads entry 0, then takes 0); those of the X
                    // row one after another: issued together, they raised the
                    // kernel's HBM reads and writes of X rows (measured: 2.3x
                    // the fetched and 3x the written bytes), at the same speed.
                    float pv[E];
#pragma unroll
                    for (int e = 0; e < E; e++) {
                        const int i = base + e;
                        pv[e] = prow[i < r ? i : 0];
                    }
#pragma unroll
                    for (int e = 0; e < E; e++) {
                        const int i = base + e;
                        const float ds = sD[i];
                        float xv = 0.f;
                        if (i < r && !a.cold) xv = xrow[i];
                        const float hv = i < r ? fmaf(a.hsign, pv[e], a.hadd) : 0.f;
                        y[e] = ds > 0.f ? xv * ds : 0.f;
                        q[e] = ds > 0.f ? hv / ds : 1.f;
                    }
                    float u[E];
                    matvec<E, L>(qseg, y, u);
                    double nl = 0.0;
#pragma unroll
                    for (int e = 0; e < E; e++) {
                        g[e] = u[e] + q[e];
                        const float p = passive(y[e], g[e]) ? g[e] : 0.f;
                        nl = fma((double)p, (double)p, nl);
                    }
                    n0 = grp_sum_d<L>(nl);
                    k = 0;
                    active = true;
                }
            }
        }
        if (!__ballot(active)) break;

        if (active) {
            // ------------------------------------------------ exact line search
            float gb[E], u[E];
            float sl = 0.f;
#pragma unroll
            for (int e = 0; e < E; e++) {
                gb[e] = passive(y[e], g[e]) ? g[e] : 0.f;
                sl = fmaf(gb[e], gb[e], sl);
            }
            const float s = grp_sum<L>(sl);
            if (s > 0.f) {
                matvec<E, L>(qseg, gb, u);
                float dl = 0.f;
#pragma unroll
                for (int e = 0; e < E; e++) dl = fmaf(gb[e], u[e], dl);
                const float den = grp_sum<L>(dl);
                if (den > 0.f) {
                    const float alpha = s / den;
#pragma unroll
                    for (int e = 0; e < E; e++) gb[e] = relu(fmaf(-alpha, gb[e], y[e])) - y[e];
                    matvec<E, L>(qseg, gb, u);
                    bool accept = true;
                    if (a.ls_guard) {
                        float gl = 0.f;
#pragma unroll
                        for (int e = 0; e < E; e++) gl = fmaf(gb[e], fmaf(0.5f, u[e], g[e]), gl);
                        accept = !(grp_sum<L>(gl) > 0.f);
                    }
                    if (accept) {
#pragma unroll
                        for (int e = 0; e < E; e++) { y[e] += gb[e]; g[e] += u[e]; }
                    }
                }
            }
            // ------------------------------------------------ r greedy CD steps
            for (int t = 0; t < r; t++) {
                // best step and decrease of every own coordinate (independent)
                float Dv[E], mv[E];
                int iv[E];
#pragma unroll
                for (int e = 0; e < E; e++) {
                    const float m = min2(y[e], g[e]);              // -(best step)
                    mv[e] = m;
                    Dv[e] = m * fmaf(2.f, g[e], -m);               // 2 x decrease
                    iv[e] = e;
                }
                // argmax as a tree (depth log2 E instead of a chain of E): the
                // right operand holds higher indices and wins only when
                // strictly larger, so ties keep the lowest index
#pragma unroll
                for (int w = 1; w < E; w <<= 1) {
#pragma unroll
                    for (int e = 0; e + w < E; e += 2 * w) {
                        const bool c = Dv[e + w] > Dv[e];
                        Dv[e] = c ? Dv[e + w] : Dv[e];
                        mv[e] = c ? mv[e + w] : mv[e];
                        iv[e] = c ? iv[e + w] : iv[e];
                    }
                }
                float best = Dv[0], bm = mv[0];
                int bi = iv[0];
                bi += base;
                grp_argmax<L>(best, bi, bm);
                const bool go = best > 0.f;
                if (!__ballot(go)) break;
                lds_reload_fence();
                if (go) {
                    float row[E];
                    load_seg<E, L>(qseg + bi * QL::SQ, row);
                    if constexpr (nqp_oh_mode<E>() == 1) {
                        constexpr int R = E * L, E4 = (E + 3) / 4;
                        const int k4 = (bi - base - R) & 3;
                        const float *oh = sZ + k4 * nqp_oh_lw<E, L>() + (R + k4 + base - bi);
                        float ohv[4 * E4];
#pragma unroll
                        for (int q = 0; q < E4; q++) {
                            const float4 v = *(const float4 *)(oh + 4 * q);
                            ohv[4 * q] = v.x; ohv[4 * q + 1] = v.y; ohv[4 * q + 2] = v.z; ohv[4 * q + 3] = v.w;
                        }
#pragma unroll
                        for (int e = 0; e < E; e++) g[e] = fmaf(-bm, row[e], g[e]);
#pragma unroll
                        for (int e = 0; e < E; e++) y[e] = fmaf(-bm, ohv[e], y[e]);
                    } else {
#pragma unroll
                        for (int e = 0; e < E; e++) g[e] = fmaf(-bm, row[e], g[e]);
                        const int el = bi - base;  // the step's coordinate in this lane's segment, if any
#pragma unroll
                        for (int e = 0; e < E; e++) y[e] = (el == e) ? y[e] - bm : y[e];
                    }
                }
            }
            // ------------------------------------------------ stopping rule
            k++;
            double nl = 0.0;
#pragma unroll
            for (int e = 0; e < E; e++) {
                const float p = passive(y[e], g[e]) ? g[e] : 0.f;
                nl = fma((double)p, (double)p, nl);
            }
            const double nk = grp_sum_d<L>(nl);
            if (nk <= a.eps * n0 || nk <= mstop || k >= a.max_inner) {
                if (mstop >= 0.0 && nk > mstop) mstop = nk;
                float *xrow = a.X + col * (int64_t)a.ldx;
#pragma unroll
                for (int e = 0; e < E; e++) {
                    const int i = base + e;
                    if (i < r) {
                        const float ds = sD[i];
                        xrow[i] = ds > 0.f ? y[e] / ds : 0.f;
                    }
                }
                if (sub == 0) {
                    if (a.iters) a.iters[col] = k;
                    my_inner += (unsigned long long)k;
                }
                active = false;
            }
        }
    }
}

// Anti-lopsided rescale (Algorithm 3, "Re-scaling variables") while staging
// into LDS: sD[i] = sqrt(Gamma_ii) (0 when Gamma_ii <= 0, a frozen coordinate,
// and for the pads r <= i < R); sQ[i][j] = Gamma_ij / (sD[i] sD[j]) with a
// unit diagonal, zero rows/columns off the diagonal for frozen or pad
// coordinates.  Every block forms the same Q from the same Gamma.
template <int E, int L>
__device__ __forceinline__ void stage_q(const float *__restrict__ gram, int r, float *sQ,
                                        float *sD, float *sZ) {
    using QL = QLayout<E, L>;
    constexpr int R = E * L;
    if constexpr (nqp_oh_mode<E>() == 1) {
        constexpr int LW = nqp_oh_lw<E, L>();
        for (int t = threadIdx.x; t < 4 * LW; t += blockDim.x) sZ[t] = (t % LW) == R + t / LW ? 1.f : 0.f;
    }
    for (int i = threadIdx.x; i < R; i += blockDim.x) {
        const float d = i < r ? gram[(size_t)i * r + i] : 0.f;
        sD[i] = d > 0.f ? sqrtf(d) : 0.f;
    }
    __syncthreads();
    // four entries per thread per trip, their loads (from clamped, valid
    // addresses) issued together
    constexpr int UN = 4;
    for (int t0 = threadIdx.x; t0 < R * R; t0 += UN * blockDim.x) {
        float gv[UN];
#pragma unroll
        for (int u = 0; u < UN; u++) {
            const int t = t0 + u * blockDim.x;
            const int i = t / R, j = t - (t / R) * R;
            const bool ok = t < R * R && i < r && j < r;
            gv[u] = gram[ok ? (size_t)i * r + j : 0];
        }
#pragma unroll
        for (int u = 0; u < UN; u++) {
            const int t = t0 + u * blockDim.x;
            if (t >= R * R) break;
            const int i = t / R, j = t - (t / R) * R;
            float v;
            if (i == j) v = 1.f;
            else if (i >= r || j >= r || sD[i] == 0.f || sD[j] == 0.f) v = 0.f;
            else v = gv[u] / (sD[i] * sD[j]);
            sQ[i * QL::SQ + QL::col(j)] = v;
        }
    }
}

__device__ __forceinline__ void flush_inner(unsigned long long v, unsigned long long *total) {
    if (!total) return;
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(total, v);
}

template <int E, int L>
__global__ __launch_bounds__((nqp_block<E, L>()))
__attribute__((amdgpu_waves_per_eu(nqp_waves_per_eu<E, L>(), 8))) void k_nqp(const NqpParams a) {
    constexpr int R = E * L;
    __shared__ __attribute__((aligned(16))) float sQ[R * QLayout<E, L>::SQ];
    __shared__ float sD[R];
    __shared__ __attribute__((aligned(16))) float sZ[nqp_oh_floats<E, L>()];
    stage_q<E, L>(a.gram, a.r, sQ, sD, sZ);
    __syncthreads();
    const int unit = a.unit > 1 ? a.unit : 1;
    ColumnIO io{a.P, a.hsign, a.hadd, a.X, a.ldp, a.ldx, a.iters, a.r, a.max_inner, a.eps,
                a.ls_guard, a.cold, a.ncols, unit};
    GlobalFetch f{a.counter, (a.ncols + unit - 1) / unit};
    unsigned long long my_inner = 0;
    nqp_columns<E, L>(sQ, sD, sZ, io, f, my_inner);
    flush_inner(my_inner, a.inner_total);
}

// Many problems at once (the batched fit): a block takes chunks (problem,
// columns [c0, c1)) from a queue, stages that problem's rescaled Hessian and
// solves the chunk's columns; its lane groups refill from an LDS counter.
// All problems of one launch share the kernel variant (E, L).
template <int E, int L>
__global__ __launch_bounds__((nqp_block<E, L>()))
__attribute__((amdgpu_waves_per_eu(nqp_waves_per_eu<E, L>(), 8))) void k_bnqp(
    const BSolveChunk *__restrict__ chunks, int nchunks, unsigned int *queue,
    const BSolveProb *__restrict__ probs, int max_inner, double eps, int ls_guard, int unit) {
    constexpr int R = E * L;
    __shared__ __attribute__((aligned(16))) float sQ[R * QLayout<E, L>::SQ];
    __shared__ float sD[R];
    __shared__ __attribute__((aligned(16))) float sZ[nqp_oh_floats<E, L>()];
    __shared__ unsigned int s_task, s_ctr;
    for (;;) {
        if (threadIdx.x == 0) {
            s_task = atomicAdd(queue, 1u);
            s_ctr = 0u;
        }
        __syncthreads();
        const unsigned int t = s_task;
        if (t >= (unsigned int)nchunks) break;
        const BSolveChunk ch = chunks[t];
        const BSolveProb P = probs[ch.prob];
        stage_q<E, L>(P.G, P.r, sQ, sD, sZ);
        __syncthreads();
        const int64_t nc = ch.c1 - ch.c0;
        const int u = unit > 1 ? unit : 1;
        ColumnIO io{P.P + (int64_t)ch.c0 * P.r, -1.f, P.l1, P.X + (int64_t)ch.c0 * P.r, P.r, P.r,
                    P.iters ? P.iters + ch.c0 : nullptr, P.r, max_inner, eps, ls_guard, P.cold, nc, u};
        LdsFetch f{&s_ctr, (nc + u - 1) / u};
        unsigned long long my_inner = 0;
        nqp_columns<E, L>(sQ, sD, sZ, io, f, my_inner);
        flush_inner(my_inner, P.inner);
        __syncthreads();
    }
}

// Blocks of one kernel per CU at the given block size (cached per size; the
// cache is shared by every host thread that launches the kernel, and each one
// that finds it empty stores the same value).
template <class K>
int nqp_blocks_per_cu(K kernel, int block, std::atomic<int> (&cache)[2]) {
    std::atomic<int> &c = cache[block == NQP_BLOCK_SMALL ? 0 : 1];
    int v = c.load(std::memory_order_relaxed);
    if (v < 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, block, 0) != hipSuccess || nb < 1) nb = 1;
        c.store(nb, std::memory_order_relaxed);
        v = nb;
    }
    return v;
}

template <int E, int L>
hipError_t launch_bnqp_t(const BSolveChunk *chunks, int nchunks, unsigned int *queue,
                         const BSolveProb *probs, int max_inner, double eps, int ls_guard, int unit,
                         hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    static std::atomic<int> cache[2] = {{-1}, {-1}};
    // small launches spread four-wave blocks over more CUs
    const int block = nchunks >= 2 * device_cu_count() ? nqp_block<E, L>() : NQP_BLOCK_SMALL;
    const int64_t cap = (int64_t)nqp_blocks_per_cu(k_bnqp<E, L>, block, cache) * device_cu_count();
    const int grid = (int)(nchunks < cap ? nchunks : cap);
    hipLaunchKernelGGL((k_bnqp<E, L>), dim3(grid), dim3(block), 0, s, chunks, nchunks, queue,
                       probs, max_inner, eps, ls_guard, unit);
    return hipGetLastError();
}

template <int E, int L>
hipError_t launch_nqp_t(const NqpParams &p, hipStream_t s) {
    if (p.ncols <= 0) return hipSuccess;
    static std::atomic<int> cache[2] = {{-1}, {-1}};
    // a launch that cannot give every CU two large blocks uses four-wave blocks
    const int big = nqp_block<E, L>();
    const int64_t big_cols = (int64_t)2 * device_cu_count() * (big / 64) * (64 / L);
    const int block = p.ncols >= big_cols ? big : NQP_BLOCK_SMALL;
    const int64_t cols_per_block = (block / 64) * (64 / L);
    const int64_t want = (p.ncols + cols_per_block - 1) / cols_per_block;
    const int64_t cap = (int64_t)nqp_blocks_per_cu(k_nqp<E, L>, block, cache) * device_cu_count();
    const int grid = (int)(want < cap ? want : cap);
    if (p.ev_start || p.ev_stop)
        hipExtLaunchKernelGGL((k_nqp<E, L>), dim3(grid), dim3(block), 0, s, p.ev_start, p.ev_stop, 0u, p);
    else
        hipLaunchKernelGGL((k_nqp<E, L>), dim3(grid), dim3(block), 0, s, p);
    return hipGetLastError();
}

}  // namespace nmfi
