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
// Work is dealt to a grid whose size depends only on the problem's shape,
// and every reduction sums per-block partials in a fixed order (in fixed
// groups first where there are many), so results are bitwise reproducible.
#include "kernels_common.h"
#include "nmf_internal.h"

namespace nmfi {

constexpr int LD_T = 64;  // dense loss tile

// LDS pitch of a factor tile (floats per rank index): LD_T + 4 spreads the
// staging stores over the banks; past r = 120 that would exceed 64 KB, and
// the pitch is LD_T (the compute reads are conflict-free either way)
__host__ __device__ inline int loss_dense_pitch(int r) { return r <= 120 ? LD_T + 4 : LD_T; }
static size_t loss_dense_lds(int r) { return (size_t)2 * loss_dense_pitch(r) * r * sizeof(float); }

// ------------------------------------------------------------ dense loss
// The tiles of W and Ht sit in LDS rank-major (Ws[a][row]): a thread's four
// rows of one rank index are one 16-byte read and the sixteen column threads
// of a wave read 256 consecutive bytes (no bank conflicts); with pitch
// LD_T + 4 the coalesced row-major staging stores hit banks 4a + row (4-way).
// (Row-major tiles had put the sixteen column threads' reads in one bank.)
__global__ __launch_bounds__(256) void k_loss_dense(const float *__restrict__ V, int64_t ld,
                                                    int64_t m, int64_t n,
                                                    const float *__restrict__ W,
                                                    const float *__restrict__ Ht, int r,
                                                    double *__restrict__ partial) {
    extern __shared__ __attribute__((aligned(16))) float sm[];
    const int lp = loss_dense_pitch(r);
    float *Ws = sm;             // r x lp
    float *Hs = sm + lp * r;    // r x lp
    __shared__ double red[256];
    const int tid = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.y * LD_T, j0 = (int64_t)blockIdx.x * LD_T;
    // loads from clamped (valid) rows, zeroed after, so that they overlap
#pragma unroll 4
    for (int e = tid; e < LD_T * r; e += 256) {
        const int row = e / r, a = e - row * r;
        const float w = W[(i0 + row < m ? i0 + row : i0) * r + a];
        const float h = Ht[(j0 + row < n ? j0 + row : j0) * r + a];
        Ws[a * lp + row] = (i0 + row < m) ? w : 0.f;
        Hs[a * lp + row] = (j0 + row < n) ? h : 0.f;
    }
    __syncthreads();
    const int ty = tid >> 4, tx = tid & 15;
    double acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; p++)
#pragma unroll
        for (int q = 0; q < 4; q++) acc[p][q] = 0.0;
    for (int a = 0; a < r; a++) {
        const f32x4 w4 = *(const f32x4 *)(Ws + a * lp + 4 * ty);
        const f32x4 h4 = *(const f32x4 *)(Hs + a * lp + 4 * tx);
        double wv[4], hv[4];
#pragma unroll
        for (int p = 0; p < 4; p++) wv[p] = (double)w4[p];
#pragma unroll
        for (int q = 0; q < 4; q++) hv[q] = (double)h4[q];
#pragma unroll
        for (int p = 0; p < 4; p++)
#pragma unroll
            for (int q = 0; q < 4; q++) acc[p][q] = fma(wv[p], hv[q], acc[p][q]);
    }
    // the sixteen loads of V first (clamped rows and columns), then the sums
    float vv[4][4];
#pragma unroll
    for (int p = 0; p < 4; p++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int64_t i = i0 + 4 * ty + p, j = j0 + 4 * tx + q;
            vv[p][q] = V[(i < m ? i : i0) * ld + (j < n ? j : j0)];
        }
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < 4; p++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int64_t i = i0 + 4 * ty + p, j = j0 + 4 * tx + q;
            if (i < m && j < n) {
                const double e = (double)vv[p][q] - acc[p][q];
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
// Rows are dealt to the waves of a fixed grid (row i to wave i mod 4 * grid).
// For row i the wave forms acc_a = sum over the stored (i, j) of V_ij H_ja in
// double (a product of two floats is exact in double), then adds W_ia acc_a:
// the cross term <V, W H'> taken as sum_i W_i . (V H')_i.  The squares of the
// stored values give ||V||^2.  One (cross, ||V||^2) pair per block, summed in
// a fixed order.
//
// VEC floats of a factor row per lane: with VEC = 4 a half-wave covers a row
// (r <= 128) and one 128-bit load per lane fetches two stored entries' rows;
// VEC = 2 and 1 serve ranks that are not multiples of 4 (one entry per load,
// a second load for r > 64 when VEC = 1).
constexpr int LOSS_CSR_GRID = 2048;
constexpr int LOSS_CSR_UNROLL = 8;  // loads in flight per lane

// sum over the 64 lanes; every lane gets the same value (each butterfly step
// adds the same two numbers in both lanes)
__device__ inline double wave_sum_d(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ inline float lane_f(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

template <int VEC> struct LossVec;
template <> struct LossVec<4> { using T = float4; static constexpr int EPL = 2, NA = 4; };
template <> struct LossVec<2> { using T = float2; static constexpr int EPL = 1, NA = 2; };
template <> struct LossVec<1> { using T = float; static constexpr int EPL = 1, NA = 2; };

template <int VEC>
__global__ __launch_bounds__(256) void k_loss_csr(const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ colidx,
                                                  const float *__restrict__ vals, int64_t m,
                                                  const float *__restrict__ W,
                                                  const float *__restrict__ Ht, int r,
                                                  double *__restrict__ partial) {
    using LV = LossVec<VEC>;
    constexpr int EPL = LV::EPL;  // stored entries per load instruction
    constexpr int NA = LV::NA;    // rank coordinates per lane
    __shared__ double red[2][4];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    // the lane's part of an entry's row: coordinates ca[k], valid when < r
    const int half = EPL == 2 ? lane >> 5 : 0;
    const int sl = EPL == 2 ? lane & 31 : lane;
    int ca[NA];
#pragma unroll
    for (int k = 0; k < NA; k++) ca[k] = VEC == 1 ? lane + 64 * k : VEC * sl + k;
    const bool ok = VEC == 1 ? true : ca[0] < r;  // whole vector in range (r % VEC == 0)
    double cross = 0.0, vv = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 4 + wave; i < m; i += (int64_t)gridDim.x * 4) {
        const int t0 = rowptr[i], t1 = rowptr[i + 1];
        double acc[NA];
#pragma unroll
        for (int k = 0; k < NA; k++) acc[k] = 0.0;
        for (int tb = t0; tb < t1; tb += 64) {
            const int cnt = min(64, t1 - tb);
            int jl = 0;
            float vl = 0.f;
            if (lane < cnt) {
                jl = colidx[tb + lane];
                vl = vals[tb + lane];
                vv = fma((double)vl, (double)vl, vv);
            }
            // entry q + EPL u + half
            for (int q = 0; q < cnt; q += EPL * LOSS_CSR_UNROLL) {
                float hv[LOSS_CSR_UNROLL][NA];
                float w[LOSS_CSR_UNROLL];
#pragma unroll
                for (int u = 0; u < LOSS_CSR_UNROLL; u++) {
                    const int t = q + EPL * u + half;
                    const bool in = t < cnt;
                    const int src = in ? t : 0;
                    int j;
                    if (EPL == 2) {
                        j = __shfl(jl, src);
                        w[u] = __shfl(vl, src);
                    } else {
                        j = __builtin_amdgcn_readlane(jl, src);
                        w[u] = lane_f(vl, src);
                    }
                    w[u] = in ? w[u] : 0.f;
                    // unconditional loads, so that all of the trip's are in
                    // flight at once: past the row's end the weight is 0 (on a
                    // valid row), and lanes past r read column 0 into sums
                    // that are never used
                    const float *hr = Ht + (int64_t)j * r;
                    if (VEC == 4) {
                        const float4 x = *(const float4 *)(hr + (ok ? ca[0] : 0));
                        hv[u][0] = x.x; hv[u][1] = x.y; hv[u][2 % NA] = x.z; hv[u][3 % NA] = x.w;
                    } else if (VEC == 2) {
                        const float2 x = *(const float2 *)(hr + (ok ? ca[0] : 0));
                        hv[u][0] = x.x; hv[u][1] = x.y;
                    } else {
                        hv[u][0] = hr[ca[0] < r ? ca[0] : 0];
                        hv[u][1 % NA] = hr[ca[1 % NA] < r ? ca[1 % NA] : 0];
                    }
                }
#pragma unroll
                for (int u = 0; u < LOSS_CSR_UNROLL; u++) {
                    const double v = (double)w[u];
#pragma unroll
                    for (int k = 0; k < NA; k++) acc[k] = fma(v, (double)hv[u][k], acc[k]);
                }
            }
        }
        // both half-waves hold partial sums over their entries for the same
        // coordinates: each adds its own W_ia acc_a, the wave sum adds both
        const float *wr = W + i * r;
#pragma unroll
        for (int k = 0; k < NA; k++)
            if (ca[k] < r && (VEC == 1 || ok)) cross = fma((double)wr[ca[k]], acc[k], cross);
    }
    cross = wave_sum_d(cross);
    vv = wave_sum_d(vv);
    if (lane == 0) {
        red[0][wave] = cross;
        red[1][wave] = vv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
        partial[2 * blockIdx.x + 1] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    }
}

// ------------------------------------------------------------ double Gram
// Block b sums rows [b * rpb, min(k, (b + 1) * rpb)) of A'A in double.
// Thread (ta, tb) = (tid / 16, tid % 16) holds the 8 x 8 output tile at rows
// [8 ta, 8 ta + 8) and columns [8 tb, 8 tb + 8) (a 16 x 16 grid of tiles
// covers r <= 128); the staged rows are converted to double once.
constexpr int G64_ROWS = 32;   // rows of A staged per pass
constexpr int G64_MAXB = 512;  // blocks (and partial Grams) at most
constexpr int G64_GROUP = 16;  // partials summed per group in the first reduce pass

__global__ __launch_bounds__(256) void k_gram64(const float *__restrict__ A, int64_t k, int r,
                                                int64_t rpb, double *__restrict__ partial) {
    __shared__ __attribute__((aligned(16))) double rows[G64_ROWS][NMF_MAX_RANK];
    const int tid = threadIdx.x, ta = tid >> 4, tb = tid & 15;
    const int nt = (r + 7) >> 3, rp = nt * 8;
    const bool act = ta < nt && tb < nt;
    double acc[8][8];
#pragma unroll
    for (int p = 0; p < 8; p++)
#pragma unroll
        for (int q = 0; q < 8; q++) acc[p][q] = 0.0;
    const int64_t b0 = (int64_t)blockIdx.x * rpb, b1 = min(k, b0 + rpb);
    for (int64_t t0 = b0; t0 < b1; t0 += G64_ROWS) {
        for (int e = tid; e < G64_ROWS * rp; e += 256) {
            const int rr = e / rp, a = e - rr * rp;
            rows[rr][a] = (t0 + rr < b1 && a < r) ? (double)A[(t0 + rr) * r + a] : 0.0;
        }
        __syncthreads();
        if (act) {
            for (int rr = 0; rr < G64_ROWS; rr++) {
                double x[8], y[8];
#pragma unroll
                for (int p = 0; p < 8; p++) {
                    x[p] = rows[rr][8 * ta + p];
                    y[p] = rows[rr][8 * tb + p];
                }
#pragma unroll
                for (int p = 0; p < 8; p++)
#pragma unroll
                    for (int q = 0; q < 8; q++) acc[p][q] = fma(x[p], y[q], acc[p][q]);
            }
        }
        __syncthreads();
    }
    if (act) {
        double *out = partial + (int64_t)blockIdx.x * r * r;
#pragma unroll
        for (int p = 0; p < 8; p++)
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int a = 8 * ta + p, b = 8 * tb + q;
                if (a < r && b < r) out[a * r + b] = acc[p][q];
            }
    }
}

// out[g * width + o] = sum of in[i * width + o] over i in group g
// ([g * G, min(count, (g + 1) * G)), in order); grid (width / 256, groups)
__global__ __launch_bounds__(256) void k_reduce_groups(const double *__restrict__ in, int64_t count,
                                                       int width, int G, double *__restrict__ out) {
    const int o = blockIdx.x * 256 + threadIdx.x;
    if (o >= width) return;
    const int64_t i0 = (int64_t)blockIdx.y * G, i1 = min(count, i0 + G);
    double s = 0.0;
    for (int64_t i = i0; i < i1; i++) s += in[i * width + o];
    out[(int64_t)blockIdx.y * width + o] = s;
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
// Groups of KKT_ROWS rows j are dealt to the waves of a fixed grid; lanes run
// over the coordinate a.  Gamma sits in LDS (float, transposed so that a wave
// reads a row of it without bank conflicts) and each entry read serves the
// group's rows; x_j reaches every lane through lane reads.  g = Gamma x_j +
// hsign P_j + hadd in double.  Per block four maxima (the optimality
// conditions of Eq. QP, Section 3.2): |min(x_a, g_a)| (zero exactly at a KKT
// point), max(0, -x_a) (nonnegativity), x_a |g_a| (complementarity) and
// max(0, -g_a) over x_a = 0 (gradient >= 0 on the zero entries); partial[q *
// gridDim.x + block] for q = 0..3.
constexpr int KKT_GRID = 2048;
constexpr int KKT_ROWS = 4;

__global__ __launch_bounds__(256) void k_kkt(const float *__restrict__ G, int r,
                                             const float *__restrict__ P, float hsign, float hadd,
                                             const float *__restrict__ X, int64_t c,
                                             double *__restrict__ partial) {
    extern __shared__ float gt[];  // gt[b * r + a] = Gamma[a][b]
    __shared__ double red[16];
    for (int e = threadIdx.x; e < r * r; e += 256) {
        const int a = e / r, b = e - a * r;
        gt[b * r + a] = G[e];
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const bool has0 = lane < r, has1 = lane + 64 < r;
    // LDS columns read by this lane (clamped into the matrix; unused when the
    // lane has no coordinate)
    const int c0 = has0 ? lane : r - 1, c1 = has1 ? lane + 64 : r - 1;
    const int r0 = r < 64 ? r : 64;
    double mx = 0.0, mneg = 0.0, mcompl = 0.0, mgrad = 0.0;
    const int64_t step = (int64_t)gridDim.x * 4 * KKT_ROWS;
    for (int64_t j0 = ((int64_t)blockIdx.x * 4 + wave) * KKT_ROWS; j0 < c; j0 += step) {
        float x0[KKT_ROWS], x1[KKT_ROWS];
        double g0[KKT_ROWS], g1[KKT_ROWS];
        // the group's loads from clamped (valid) rows and columns first
        float xa[KKT_ROWS], xb[KKT_ROWS], pa[KKT_ROWS], pb[KKT_ROWS];
#pragma unroll
        for (int k = 0; k < KKT_ROWS; k++) {
            const int64_t j = j0 + k < c ? j0 + k : j0;
            const float *xr = X + j * r, *pr = P + j * r;
            xa[k] = xr[c0]; xb[k] = xr[c1]; pa[k] = pr[c0]; pb[k] = pr[c1];
        }
#pragma unroll
        for (int k = 0; k < KKT_ROWS; k++) {
            const bool in = j0 + k < c;
            x0[k] = (in && has0) ? xa[k] : 0.f;
            x1[k] = (in && has1) ? xb[k] : 0.f;
            g0[k] = (in && has0) ? (double)hsign * (double)pa[k] + (double)hadd : 0.0;
            g1[k] = (in && has1) ? (double)hsign * (double)pb[k] + (double)hadd : 0.0;
        }
        for (int b = 0; b < r0; b++) {
            const double ga = (double)gt[b * r + c0];
            const double gb = r > 64 ? (double)gt[b * r + c1] : 0.0;
#pragma unroll
            for (int k = 0; k < KKT_ROWS; k++) {
                const double xb = (double)lane_f(x0[k], b);
                g0[k] = fma(ga, xb, g0[k]);
                g1[k] = fma(gb, xb, g1[k]);
            }
        }
        for (int b = 64; b < r; b++) {
            const double ga = (double)gt[b * r + c0], gb = (double)gt[b * r + c1];
#pragma unroll
            for (int k = 0; k < KKT_ROWS; k++) {
                const double xb = (double)lane_f(x1[k], b - 64);
                g0[k] = fma(ga, xb, g0[k]);
                g1[k] = fma(gb, xb, g1[k]);
            }
        }
        auto account = [&](double x, double g) {
            const double v = fabs(x < g ? x : g);
            mx = v > mx ? v : mx;
            mneg = -x > mneg ? -x : mneg;
            const double cv = x * fabs(g);
            mcompl = cv > mcompl ? cv : mcompl;
            if (x == 0.0 && -g > mgrad) mgrad = -g;
        };
#pragma unroll
        for (int k = 0; k < KKT_ROWS; k++) {
            if (j0 + k >= c) break;
            if (has0) account(x0[k], g0[k]);
            if (has1) account(x1[k], g1[k]);
        }
    }
    double vals[4] = {mx, mneg, mcompl, mgrad};
#pragma unroll
    for (int q = 0; q < 4; q++) {
        double v = vals[q];
        for (int off = 32; off >= 1; off >>= 1) {
            const double o = __shfl_xor(v, off);
            v = o > v ? o : v;
        }
        if (lane == 0) red[q * 4 + wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int q = threadIdx.x;
        double v = red[q * 4];
        for (int w = 1; w < 4; w++) v = red[q * 4 + w] > v ? red[q * 4 + w] : v;
        partial[(size_t)q * gridDim.x + blockIdx.x] = v;
    }
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
static size_t finish_scratch_bytes() { return 2 * align256(2 * 4096 * sizeof(double)); }

size_t objective_scratch_bytes(const nmf_matrix *V, int r) {
    const int64_t m = V->rows, n = V->cols;
    size_t b = 0;
    if (V->kind == NMF_DENSE) {
        b += align256((size_t)((n + LD_T - 1) / LD_T) * ((m + LD_T - 1) / LD_T) * sizeof(double));
    } else {
        b += align256((size_t)2 * LOSS_CSR_GRID * sizeof(double));
        b += align256((size_t)G64_MAXB * r * r * sizeof(double));  // Gram partials (reused)
        b += align256((size_t)(G64_MAXB / G64_GROUP) * r * r * sizeof(double));  // group sums
        b += 2 * align256((size_t)r * r * sizeof(double));         // GW, GH
    }
    b += finish_scratch_bytes();                  // sums of W and H
    b += align256(16 * sizeof(double));           // terms
    b += align256(2 * sizeof(double));            // out
    return b + 1024;
}

static hipError_t gram64(const float *A, int64_t k, int r, double *partial, double *groups,
                         double *G, hipStream_t s) {
    // about 64 rows per block at least, G64_MAXB blocks at most
    int64_t nb = (k + 63) / 64;
    if (nb > G64_MAXB) nb = G64_MAXB;
    if (nb < 1) nb = 1;
    const int64_t rpb = (k + nb - 1) / nb;
    nb = k > 0 ? (k + rpb - 1) / rpb : 1;
    hipLaunchKernelGGL(k_gram64, dim3((unsigned)nb), dim3(256), 0, s, A, k, r, rpb, partial);
    const int width = r * r;
    const int ng = (int)((nb + G64_GROUP - 1) / G64_GROUP);
    hipLaunchKernelGGL(k_reduce_groups, dim3((unsigned)((width + 255) / 256), (unsigned)ng), dim3(256), 0,
                       s, partial, nb, width, G64_GROUP, groups);
    hipLaunchKernelGGL(k_reduce_ordered, dim3((unsigned)((width + 255) / 256)), dim3(256), 0, s,
                       groups, (int64_t)ng, width, G);
    return hipGetLastError();
}

static hipError_t finish_objective(double *terms, int csr, const nmf_reg *reg, const float *W, int64_t m,
                                   const float *Ht, int64_t n, int r, char *p, double *dev_out,
                                   hipStream_t s);

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
        const size_t lds = loss_dense_lds(r);
        hipLaunchKernelGGL(k_loss_dense, dim3(gx, gy), dim3(256), lds, s, V->dense, V->ld, m, n, W,
                           Ht, r, part);
        hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(256), 0, s, part, (int64_t)gx * gy,
                           (int64_t)1, (int64_t)0, terms + 0);
    } else {
        double *part = (double *)take((size_t)2 * LOSS_CSR_GRID * sizeof(double));
        int64_t nb = (m + 3) / 4;
        nb = nb > LOSS_CSR_GRID ? LOSS_CSR_GRID : (nb < 1 ? 1 : nb);
        if (r % 4 == 0)
            hipLaunchKernelGGL(k_loss_csr<4>, dim3((unsigned)nb), dim3(256), 0, s, V->rowptr, V->colidx,
                               V->vals, m, W, Ht, r, part);
        else if (r % 2 == 0)
            hipLaunchKernelGGL(k_loss_csr<2>, dim3((unsigned)nb), dim3(256), 0, s, V->rowptr, V->colidx,
                               V->vals, m, W, Ht, r, part);
        else
            hipLaunchKernelGGL(k_loss_csr<1>, dim3((unsigned)nb), dim3(256), 0, s, V->rowptr, V->colidx,
                               V->vals, m, W, Ht, r, part);
        hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(256), 0, s, part, nb, (int64_t)2,
                           (int64_t)1, terms + 1);
        hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(256), 0, s, part, nb, (int64_t)2,
                           (int64_t)0, terms + 2);
        double *gp = (double *)take((size_t)G64_MAXB * r * r * sizeof(double));
        double *gg = (double *)take((size_t)(G64_MAXB / G64_GROUP) * r * r * sizeof(double));
        double *gw = (double *)take((size_t)r * r * sizeof(double));
        double *gh = (double *)take((size_t)r * r * sizeof(double));
        hipError_t e = gram64(W, m, r, gp, gg, gw, s);
        if (e == hipSuccess) e = gram64(Ht, n, r, gp, gg, gh, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_dot_ordered, dim3(1), dim3(256), 0, s, gw, gh, (int64_t)r * r,
                           terms + 3);
    }
    return finish_objective(terms, V->kind == NMF_CSR ? 1 : 0, reg, W, m, Ht, n, r, p, dev_out, s);
}

// The regularisation sums of W and Ht into terms[4..7]; scratch of
// finish_scratch_bytes().
static hipError_t objective_sums(double *terms, const float *W, int64_t m, const float *Ht, int64_t n, int r,
                                 char *p, hipStream_t s) {
    auto take = [&](size_t bytes) { char *q = p; p += align256(bytes); return q; };
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
    return hipGetLastError();
}

static hipError_t launch_finish(const double *terms, int csr, const nmf_reg *reg, double *dev_out,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1), 0, s, terms, csr, (double)reg->l1_w,
                       (double)reg->l2_w, (double)reg->l1_h, (double)reg->l2_h, dev_out);
    return hipGetLastError();
}

// The regularisation sums, then loss and J from terms[] (the loss terms
// already in place); scratch of finish_scratch_bytes().
static hipError_t finish_objective(double *terms, int csr, const nmf_reg *reg, const float *W, int64_t m,
                                   const float *Ht, int64_t n, int r, char *p, double *dev_out,
                                   hipStream_t s) {
    hipError_t e = objective_sums(terms, W, m, Ht, n, r, p, s);
    return e == hipSuccess ? launch_finish(terms, csr, reg, dev_out, s) : e;
}

// ------------------------------------------------------------ V in row or column panels
// Streamed fits see V one panel at a time: each panel's sum of squared
// errors goes to a slot, and the slots are summed in panel order.
size_t loss_panel_scratch_bytes(int64_t rows, int64_t cols) {
    return align256((size_t)((cols + LD_T - 1) / LD_T) * ((rows + LD_T - 1) / LD_T) * sizeof(double));
}

hipError_t launch_loss_panel(const float *V, int64_t ld, int64_t rows, int64_t cols, const float *W,
                             const float *Ht, int r, double *scratch, double *slot, hipStream_t s) {
    if (rows <= 0 || cols <= 0) {
        hipLaunchKernelGGL(k_reduce_ordered, dim3(1), dim3(256), 0, s, (const double *)nullptr,
                           (int64_t)0, 1, slot);  // an empty panel adds zero
        return hipGetLastError();
    }
    const unsigned gx = (unsigned)((cols + LD_T - 1) / LD_T), gy = (unsigned)((rows + LD_T - 1) / LD_T);
    const size_t lds = loss_dense_lds(r);
    hipLaunchKernelGGL(k_loss_dense, dim3(gx, gy), dim3(256), lds, s, V, ld, rows, cols, W, Ht, r, scratch);
    hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(256), 0, s, scratch, (int64_t)gx * gy, (int64_t)1,
                       (int64_t)0, slot);
    return hipGetLastError();
}

size_t objective_slots_scratch_bytes() { return align256(16 * sizeof(double)) + finish_scratch_bytes(); }

hipError_t launch_objective_regs(const float *W, int64_t m, const float *Ht, int64_t n, int r, char *scratch,
                                 hipStream_t s) {
    double *terms = (double *)scratch;
    hipLaunchKernelGGL(k_reduce_ordered, dim3(1), dim3(256), 0, s, (const double *)nullptr, (int64_t)0, 16,
                       terms);  // zero the terms
    return objective_sums(terms, W, m, Ht, n, r, scratch + align256(16 * sizeof(double)), s);
}

hipError_t launch_objective_slots(const double *slots, int64_t nslots, const nmf_reg *reg, char *scratch,
                                  double *dev_out, hipStream_t s) {
    double *terms = (double *)scratch;
    hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(256), 0, s, slots, nslots, (int64_t)1, (int64_t)0,
                       terms + 0);
    return launch_finish(terms, 0, reg, dev_out, s);
}

hipError_t launch_max_ordered(const double *in, int64_t n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_max_ordered, dim3(1), dim3(256), 0, s, in, n, out);
    return hipGetLastError();
}

static int64_t kkt_blocks(int64_t c) {
    const int64_t nb = (c + 4 * KKT_ROWS - 1) / (4 * KKT_ROWS);
    return nb > KKT_GRID ? KKT_GRID : nb;
}

size_t kkt_partial_bytes(int64_t c) { return (size_t)(4 * (c > 0 ? kkt_blocks(c) : 1)) * sizeof(double); }

// The four KKT residuals of one half (minmap, nonnegativity, complementarity,
// gradient on zero entries) into dev_out[0], dev_out[stride], dev_out[2 *
// stride], dev_out[3 * stride]; partial holds kkt_partial_bytes(c).
hipError_t launch_kkt(const float *G, int r, const float *P, float hsign, float hadd,
                      const float *X, int64_t c, double *partial, double *dev_out, int64_t stride,
                      hipStream_t s) {
    if (c <= 0) return hipSuccess;
    const int64_t nb = kkt_blocks(c);
    hipLaunchKernelGGL(k_kkt, dim3((unsigned)nb), dim3(256), (size_t)r * r * sizeof(float), s, G, r, P,
                       hsign, hadd, X, c, partial);
    for (int q = 0; q < 4; q++)
        hipLaunchKernelGGL(k_max_ordered, dim3(1), dim3(256), 0, s, partial + q * nb, nb, dev_out + q * stride);
    return hipGetLastError();
}

}  // namespace nmfi
