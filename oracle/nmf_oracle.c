/*
 * nmf_oracle.c -- plain FP64 CPU oracle for the alternating NNLS method of
 * Nguyen & Ho, "Accelerated Parallel and Distributed Algorithm using Limited
 * Internal Memory for Nonnegative Matrix Factorization" (arXiv:1506.08938).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or helper with the GPU library, and the GPU library
 * never calls it.
 *
 * Conventions (the paper stores instances as columns of an n x m matrix; this
 * file uses V = W * H with V m x n):
 *   V   m x n, row-major (dense) or CSR of V.
 *   W   m x r, row-major; row i is the solution of one W-update NNLS.
 *   Ht  n x r, row-major (= H transposed); row j is one H-update solution.
 * Every floating-point quantity is double; sums run in ascending index order.
 *
 * Parity status per function is listed at each definition; every function
 * here is pinned by a CPU test against an independent check (closed forms,
 * brute force, Lawson-Hanson NNLS, the paper's worked example, or scipy).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Debug switches that strip parts of the NQP solver, so that tests can pin
 * the remaining part against numbers the paper prints for its 2-D example
 * (Section 3.4, the function of Eq. NQP and its rescaled form Eq. NQPI). */
#define ORACLE_NO_RESCALE 1 /* solve in x directly: Q = H, q = h, y = x  */
#define ORACLE_NO_CD      2 /* skip the greedy coordinate-descent sweep  */
#define ORACLE_NO_LS      4 /* skip the exact line search                 */

/* Doubles recorded per coordinate-descent step by oracle_nqp_cdtrace. */
#define CD_TRACE_FIELDS 6

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Anti-lopsided rescale (Section 3.4, Algorithm 3 "Re-scaling variables").
 * Q = H / sqrt(diag(H) diag(H)^T), so that Q_ii = 1.  A coordinate whose
 * diagonal is <= 0 (a zero column of A with no L2 term) cannot be rescaled;
 * it is frozen: its row and column of Q are zero except Q_ii = 1, and its
 * variable stays 0.  d[i] = sqrt(H_ii) (0 when frozen). */
void oracle_rescale(int r, const double *H, double *Q, double *d, int *frozen) {
    for (int i = 0; i < r; i++) {
        frozen[i] = !(H[(size_t)i * r + i] > 0.0);
        d[i] = frozen[i] ? 0.0 : sqrt(H[(size_t)i * r + i]);
    }
    for (int i = 0; i < r; i++)
        for (int j = 0; j < r; j++) {
            double v;
            if (i == j) v = 1.0;
            else if (frozen[i] || frozen[j]) v = 0.0;
            else v = H[(size_t)i * r + j] / (d[i] * d[j]);
            Q[(size_t)i * r + j] = v;
        }
}

/* Projected gradient (Section 3.4): the gradient restricted to the passive
 * set P = { i : y_i > 0 or grad_i < 0 }, zero elsewhere. */
static double pg_entry(double y, double g) { return (y > 0.0 || g < 0.0) ? g : 0.0; }

static double pg_norm2(int r, const double *y, const double *g, const int *frozen) {
    double s = 0.0;
    for (int i = 0; i < r; i++)
        if (!frozen[i]) { double p = pg_entry(y[i], g[i]); s += p * p; }
    return s;
}

static double quad_form_value(int r, const double *Q, const double *q, const double *y) {
    /* 0.5 y'Qy + q'y */
    double f = 0.0;
    for (int i = 0; i < r; i++) {
        double t = 0.0;
        for (int j = 0; j < r; j++) t += Q[(size_t)i * r + j] * y[j];
        f += y[i] * (0.5 * t + q[i]);
    }
    return f;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 3 (Fast Combinational Algorithm for NQP): minimise
 * f(x) = 0.5 x'Hx + h'x subject to x >= 0, from the start point x0.
 *
 *   H, h    : r x r (row-major, symmetric) and r.
 *   x       : in = x0 (>= 0), out = solution.
 *   max_inner, eps : stop when ||pg_k||^2 <= eps ||pg_0||^2 (the accelerated
 *             condition) or after max_inner iterations; at least one
 *             iteration always runs (repeat-until).  eps = 0 stops only on
 *             an exactly zero projected gradient (further iterations would
 *             not move), otherwise it runs max_inner iterations.
 *   ls_guard: 1 = reject a line-search step that would raise f.  The paper's
 *             projected step is not monotone; 0 keeps the literal step.
 *   flags   : ORACLE_NO_* debug switches (0 for the method itself).
 *   fk      : optional, fk[k] = rescaled objective after iteration k
 *             (fk[0] at the start); length max_inner + 1.
 * Returns the number of iterations run.
 *
 * Each iteration: (1) exact line search on the projected gradient with
 * alpha = |pg|^2 / pg'Q pg, projection onto x >= 0 and the incremental
 * gradient update g += Q (y_new - y); (2) r greedy coordinate-descent steps,
 * each computing the best step delta_i = max(0, y_i - g_i/Q_ii) - y_i for
 * every i, taking the coordinate with the largest decrease |f(y) - f(y +
 * delta_i e_i)| (lowest index on ties) and updating y_p and g.  Finally the
 * solution is unscaled, x = y / sqrt(diag H).
 * The fast-break test against a per-thread maxStop is not part of this
 * oracle: columns are solved independently. */
/* Algorithm 3 with its optional fast-break: besides ||f~_k||^2 <= eps
 * ||f~_0||^2 the loop also ends once ||f~_k||^2 <= max_stop (max_stop < 0:
 * no fast-break).  nk_out (optional) gets the final ||f~_k||^2; nk_trace
 * (optional, max_inner + 1 entries) gets ||f~_k||^2 for k = 0..iters. */
static int nqp_core(int r, const double *H, const double *h, double *x, int max_inner, double eps,
                    int ls_guard, int flags, double *fk, double max_stop, double *nk_out,
                    double *nk_trace, double *cd_trace, int trace_iters);

int oracle_nqp_flags(int r, const double *H, const double *h, double *x, int max_inner, double eps,
                     int ls_guard, int flags, double *fk) {
    return nqp_core(r, H, h, x, max_inner, eps, ls_guard, flags, fk, -1.0, NULL, NULL, NULL, 0);
}

static int nqp_core(int r, const double *H, const double *h, double *x, int max_inner, double eps,
                    int ls_guard, int flags, double *fk, double max_stop, double *nk_out,
                    double *nk_trace, double *cd_trace, int trace_iters) {
    double *Q = (double *)malloc(sizeof(double) * (size_t)r * r);
    double *buf = (double *)malloc(sizeof(double) * (size_t)r * 8);
    int *frozen = (int *)malloc(sizeof(int) * (size_t)r);
    double *d = buf, *q = buf + r, *y = buf + 2 * r, *g = buf + 3 * r;
    double *gb = buf + 4 * r, *u = buf + 5 * r, *yn = buf + 6 * r, *w = buf + 7 * r;

    if (flags & ORACLE_NO_RESCALE) {
        for (int i = 0; i < r; i++) frozen[i] = 0;
        for (size_t t = 0; t < (size_t)r * r; t++) Q[t] = H[t];
        for (int i = 0; i < r; i++) { d[i] = 1.0; q[i] = h[i]; y[i] = x[i]; }
    } else {
        oracle_rescale(r, H, Q, d, frozen);
        for (int i = 0; i < r; i++) {
            q[i] = frozen[i] ? 0.0 : h[i] / d[i];
            y[i] = frozen[i] ? 0.0 : x[i] * d[i];
        }
    }
    /* gradient of the rescaled problem */
    for (int i = 0; i < r; i++) {
        double t = 0.0;
        for (int j = 0; j < r; j++) t += Q[(size_t)i * r + j] * y[j];
        g[i] = t + q[i];
    }
    if (fk) fk[0] = quad_form_value(r, Q, q, y);
    double n0 = pg_norm2(r, y, g, frozen);
    double nk = n0;
    if (nk_trace) nk_trace[0] = n0;

    int k = 0;
    for (;;) {
        k++;
        /* (1) exact line search on the projected gradient */
        if (!(flags & ORACLE_NO_LS)) {
            double s = 0.0;
            for (int i = 0; i < r; i++) {
                gb[i] = frozen[i] ? 0.0 : pg_entry(y[i], g[i]);
                s += gb[i] * gb[i];
            }
            if (s > 0.0) {
                double den = 0.0;
                for (int i = 0; i < r; i++) {
                    double t = 0.0;
                    for (int j = 0; j < r; j++) t += Q[(size_t)i * r + j] * gb[j];
                    u[i] = t;
                    den += gb[i] * t;
                }
                if (den > 0.0) {
                    double alpha = s / den;
                    for (int i = 0; i < r; i++) {
                        double v = y[i] - alpha * gb[i];
                        yn[i] = v > 0.0 ? v : 0.0;
                        yn[i] -= y[i]; /* yn now holds the step y_new - y */
                    }
                    double gd = 0.0, dqd = 0.0;
                    for (int i = 0; i < r; i++) {
                        double t = 0.0;
                        for (int j = 0; j < r; j++) t += Q[(size_t)i * r + j] * yn[j];
                        w[i] = t;
                    }
                    for (int i = 0; i < r; i++) { gd += g[i] * yn[i]; dqd += yn[i] * w[i]; }
                    int accept = !(ls_guard && (gd + 0.5 * dqd > 0.0));
                    if (accept)
                        for (int i = 0; i < r; i++) { y[i] += yn[i]; g[i] += w[i]; }
                }
            }
        }
        /* (2) r greedy coordinate-descent steps */
        if (!(flags & ORACLE_NO_CD)) {
            for (int t = 0; t < r; t++) {
                int p = -1;
                double best = 0.0, dp = 0.0, second = -1.0, dsec = 0.0;
                for (int i = 0; i < r; i++) {
                    if (frozen[i]) continue;
                    double qii = Q[(size_t)i * r + i];
                    double v = y[i] - g[i] / qii;
                    double delta = (v > 0.0 ? v : 0.0) - y[i];
                    double dec = fabs(g[i] * delta + 0.5 * qii * delta * delta);
                    if (p < 0 || dec > best) {
                        if (p >= 0) { second = best; dsec = dp; }
                        p = i; best = dec; dp = delta;
                    } else if (dec > second) {
                        second = dec; dsec = delta;
                    }
                }
                if (cd_trace && k <= trace_iters) { /* record only: the step is unchanged */
                    double *e = cd_trace + CD_TRACE_FIELDS * ((size_t)(k - 1) * r + t);
                    double gs = 0.0; /* magnitude of the terms that make up g */
                    for (int i = 0; i < r; i++) {
                        if (frozen[i]) continue;
                        double a = fabs(q[i]);
                        for (int j = 0; j < r; j++) a += fabs(Q[(size_t)i * r + j] * y[j]);
                        if (a > gs) gs = a;
                    }
                    e[0] = (p < 0 || !(best > 0.0)) ? -1.0 : (double)p;
                    e[1] = best;
                    e[2] = second;
                    e[3] = fabs(dp);
                    e[4] = fabs(dsec);
                    e[5] = gs;
                }
                if (p < 0 || !(best > 0.0)) break; /* every remaining step is a no-op */
                for (int i = 0; i < r; i++) g[i] += Q[(size_t)i * r + p] * dp;
                y[p] += dp;
            }
        }
        if (fk) fk[k] = quad_form_value(r, Q, q, y);
        nk = pg_norm2(r, y, g, frozen);
        if (nk_trace) nk_trace[k] = nk;
        if (nk <= eps * n0 || nk <= max_stop || k >= max_inner) break;
    }
    if (nk_out) *nk_out = nk;
    for (int i = 0; i < r; i++) x[i] = frozen[i] ? 0.0 : y[i] / d[i];
    free(Q); free(buf); free(frozen);
    return k;
}

int oracle_nqp(int r, const double *H, const double *h, double *x, int max_inner, double eps,
               int ls_guard) {
    return oracle_nqp_flags(r, H, h, x, max_inner, eps, ls_guard, 0, NULL);
}

/* Independent NQPs sharing one H (Algorithm 2: every column solved alone).
 * h and x are ncols x r row-major; iters (optional) gets each column's
 * iteration count.  Returns the total number of iterations. */
long oracle_nqp_batch(int r, long ncols, const double *H, const double *h, double *x,
                      int max_inner, double eps, int ls_guard, int *iters) {
    long total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
    for (long j = 0; j < ncols; j++) {
        int k = oracle_nqp(r, H, h + (size_t)j * r, x + (size_t)j * r, max_inner, eps, ls_guard);
        if (iters) iters[j] = k;
        total += k;
    }
    return total;
}

/* One NQP with the per-iteration projected-gradient norms ||f~_k||^2
 * (k = 0..iters) written to nk_trace; no fast-break. */
int oracle_nqp_trace(int r, const double *H, const double *h, double *x, int max_inner, double eps,
                     int ls_guard, double *nk_trace) {
    return nqp_core(r, H, h, x, max_inner, eps, ls_guard, 0, NULL, -1.0, NULL, nk_trace, NULL, 0);
}

/* Independent NQPs sharing H (h, x: ncols x r; iters optional), with a
 * record of every greedy coordinate-descent choice of the first trace_iters
 * iterations, for telling rounding-sensitive columns apart: column j's block
 * of cd_trace has trace_iters * r entries of CD_TRACE_FIELDS doubles, entry
 * (k, t) for CD step t of iteration k + 1: the chosen coordinate p (-1 for the step at which the
 * sweep ended because no coordinate decreases f), the decrease
 * |f(y) - f(y + delta_p e_p)| of that choice, the largest decrease among the
 * other coordinates (-1 when there is none), |delta| of the choice and of
 * that runner-up, and max_i (|q_i| + sum_j |Q_ij y_j|), the size of the
 * terms the gradient is made of (its rounding error in a lower precision
 * scales with it).  A gap between the two decreases that is small against
 * the rounding error of the decreases marks a near-tie, which a computation
 * in lower precision may resolve the other way.  Steps after the end of a
 * sweep and iterations not run are not written (the caller initialises
 * them).  The arithmetic of the solve is that of oracle_nqp. */


long oracle_nqp_batch_cdtrace(int r, long ncols, const double *H, const double *h, double *x,
                              int max_inner, double eps, int ls_guard, int trace_iters, int *iters,
                              double *cd_trace) {
    long total = 0;
    const size_t blk = (size_t)trace_iters * r * CD_TRACE_FIELDS;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
    for (long j = 0; j < ncols; j++) {
        int k = nqp_core(r, H, h + (size_t)j * r, x + (size_t)j * r, max_inner, eps, ls_guard, 0,
                         NULL, -1.0, NULL, NULL, cd_trace + (size_t)j * blk, trace_iters);
        if (iters) iters[j] = k;
        total += k;
    }
    return total;
}

/* Independent NQPs with the fast-break of Algorithm 3: the columns are cut
 * into "threads of computation" of `chunk` consecutive columns (a fixed
 * partition, so the result never depends on scheduling); within one, the
 * columns are solved in order with maxStop starting at 0 (Algorithm 2 resets
 * it before each half) and raised to the final ||f~||^2 of every solved
 * column; a column also stops once ||f~_k||^2 <= maxStop.  nk (optional) gets
 * each column's final ||f~||^2.  Returns the total number of iterations. */
long oracle_nqp_batch_faststop(int r, long ncols, const double *H, const double *h, double *x,
                               int max_inner, double eps, int ls_guard, long chunk, int *iters,
                               double *nk) {
    long total = 0;
    if (chunk < 1) chunk = 1;
    const long nch = (ncols + chunk - 1) / chunk;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : total)
    for (long c = 0; c < nch; c++) {
        double max_stop = 0.0;
        const long j1 = (c + 1) * chunk < ncols ? (c + 1) * chunk : ncols;
        for (long j = c * chunk; j < j1; j++) {
            double fin = 0.0;
            int k = nqp_core(r, H, h + (size_t)j * r, x + (size_t)j * r, max_inner, eps, ls_guard, 0,
                             NULL, max_stop, &fin, NULL, NULL, 0);
            if (fin > max_stop) max_stop = fin;
            if (iters) iters[j] = k;
            if (nk) nk[j] = fin;
            total += k;
        }
    }
    return total;
}

/* ------------------------------------------------------------------------ */
/* Building blocks of one half-iteration (Section 3.2, Eq. QP; Section 3.5,
 * Eq. L1L2NMF): with A fixed (k x r) and data B (k x c), column j solves
 *   min_x 0.5||B_j - A x||^2 + l1 1'x + l2 ||x||^2,
 * an NQP with H = A'A + 2 l2 I and h = -A'B_j + l1 1. */

/* G = A'A + 2 l2 I   (A k x r row-major, G r x r).  Each entry is summed in
 * ascending t; the t loop sits outside the (a, b) loops only so that rows of
 * A are read contiguously (the same additions in the same order). */
void oracle_gram(long k, int r, const double *A, double l2, double *G) {
#pragma omp parallel for schedule(static)
    for (int a = 0; a < r; a++) {
        double *row = G + (size_t)a * r;
        for (int b = 0; b < r; b++) row[b] = 0.0;
        for (long t = 0; t < k; t++) {
            const double at = A[(size_t)t * r + a];
            const double *At = A + (size_t)t * r;
            for (int b = 0; b < r; b++) row[b] += at * At[b];
        }
        row[a] += 2.0 * l2;
    }
}

/* P = (A'B)' : c x r, P[j][a] = sum_t A[t][a] B[t][j].
 * B is the dense m x n data V (trans = 0: B = V, k = m, c = n) or its
 * transpose (trans = 1: B = V', k = n, c = m). */
void oracle_product_dense(long m, long n, const double *V, int trans, int r, const double *A,
                          double *P) {
    long c = trans ? m : n, k = trans ? n : m;
#pragma omp parallel for schedule(static)
    for (long j = 0; j < c; j++)
        for (int a = 0; a < r; a++) {
            double s = 0.0;
            for (long t = 0; t < k; t++) {
                double b = trans ? V[(size_t)j * n + t] : V[(size_t)t * n + j];
                s += A[(size_t)t * r + a] * b;
            }
            P[(size_t)j * r + a] = s;
        }
}

/* The same products for V given as CSR (rowptr m+1, colidx/vals nnz).
 * trans = 1 (P = V A, m x r, A = Ht n x r) runs over the rows of V.
 * trans = 0 (P = V' A, n x r, A = W m x r) first transposes the CSR with a
 * counting sort (entries of each column keep ascending row order). */
void oracle_product_csr(long m, long n, const int *rowptr, const int *colidx, const double *vals,
                        int trans, int r, const double *A, double *P) {
    if (trans) {
#pragma omp parallel for schedule(dynamic, 256)
        for (long i = 0; i < m; i++)
            for (int a = 0; a < r; a++) {
                double s = 0.0;
                for (long t = rowptr[i]; t < rowptr[i + 1]; t++)
                    s += vals[t] * A[(size_t)colidx[t] * r + a];
                P[(size_t)i * r + a] = s;
            }
        return;
    }
    long nnz = rowptr[m];
    long *cp = (long *)calloc((size_t)n + 1, sizeof(long));
    long *fill = (long *)malloc(sizeof(long) * (size_t)(n + 1));
    int *ri = (int *)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    double *rv = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    for (long t = 0; t < nnz; t++) cp[colidx[t] + 1]++;
    for (long j = 0; j < n; j++) cp[j + 1] += cp[j];
    memcpy(fill, cp, sizeof(long) * (size_t)(n + 1));
    for (long i = 0; i < m; i++)
        for (long t = rowptr[i]; t < rowptr[i + 1]; t++) {
            long pos = fill[colidx[t]]++;
            ri[pos] = (int)i;
            rv[pos] = vals[t];
        }
#pragma omp parallel for schedule(dynamic, 256)
    for (long j = 0; j < n; j++)
        for (int a = 0; a < r; a++) {
            double s = 0.0;
            for (long t = cp[j]; t < cp[j + 1]; t++) s += rv[t] * A[(size_t)ri[t] * r + a];
            P[(size_t)j * r + a] = s;
        }
    free(cp); free(fill); free(ri); free(rv);
}

/* One half-iteration: x_j <- NQP(A'A + 2 l2 I, -P_j + l1, x_j) for every
 * row j of X (c x r), warm-started from X.  Returns the total iterations. */
long oracle_half_update(long c, int r, const double *G, const double *P, double l1, double *X,
                        int max_inner, double eps, int ls_guard, int *iters) {
    double *h = (double *)malloc(sizeof(double) * (size_t)(c > 0 ? c : 1) * r);
    for (long j = 0; j < c; j++)
        for (int a = 0; a < r; a++) h[(size_t)j * r + a] = -P[(size_t)j * r + a] + l1;
    long tot = oracle_nqp_batch(r, c, G, h, X, max_inner, eps, ls_guard, iters);
    free(h);
    return tot;
}

/* ------------------------------------------------------------------------ */
/* Objectives (Section 5.1 reports 0.5||V - GF||^2; Section 3.5, Eq.
 * L1L2NMF, adds the regularisers with the 1/2 on the loss). */

/* 0.5 ||V - W Ht'||_F^2, dense V, summed directly entry by entry. */
double oracle_loss_dense(long m, long n, const double *V, int r, const double *W,
                         const double *Ht) {
    double *row = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
#pragma omp parallel for schedule(static)
    for (long i = 0; i < m; i++) {
        double si = 0.0;
        for (long j = 0; j < n; j++) {
            double wh = 0.0;
            for (int a = 0; a < r; a++) wh += W[(size_t)i * r + a] * Ht[(size_t)j * r + a];
            double e = V[(size_t)i * n + j] - wh;
            si += e * e;
        }
        row[i] = si;
    }
    double s = 0.0;
    for (long i = 0; i < m; i++) s += row[i];
    free(row);
    return 0.5 * s;
}

/* 0.5 ||V - W Ht'||_F^2 for CSR V via the exact expansion
 * ||V||^2 - 2 <V, W Ht'> + <W'W, Ht'Ht>, which needs only the stored
 * entries of V. */
double oracle_loss_csr(long m, long n, const int *rowptr, const int *colidx, const double *vals,
                       int r, const double *W, const double *Ht) {
    double *rv = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? 2 * m : 1));
#pragma omp parallel for schedule(dynamic, 256)
    for (long i = 0; i < m; i++) {
        double v2 = 0.0, cr = 0.0;
        for (long t = rowptr[i]; t < rowptr[i + 1]; t++) {
            double wh = 0.0;
            for (int a = 0; a < r; a++) wh += W[(size_t)i * r + a] * Ht[(size_t)colidx[t] * r + a];
            v2 += vals[t] * vals[t];
            cr += vals[t] * wh;
        }
        rv[2 * i] = v2;
        rv[2 * i + 1] = cr;
    }
    double vv = 0.0, cross = 0.0;
    for (long i = 0; i < m; i++) { vv += rv[2 * i]; cross += rv[2 * i + 1]; }
    free(rv);
    double *GW = (double *)malloc(sizeof(double) * (size_t)r * r);
    double *GH = (double *)malloc(sizeof(double) * (size_t)r * r);
    oracle_gram(m, r, W, 0.0, GW);
    oracle_gram(n, r, Ht, 0.0, GH);
    double tr = 0.0;
    for (size_t t = 0; t < (size_t)r * r; t++) tr += GW[t] * GH[t];
    free(GW); free(GH);
    (void)n;
    return 0.5 * (vv - 2.0 * cross + tr);
}

/* Regulariser sum  l1 sum(X) + l2 ||X||_F^2  over a c x r factor. */
double oracle_reg_term(long c, int r, const double *X, double l1, double l2) {
    double s1 = 0.0, s2 = 0.0;
    for (size_t t = 0; t < (size_t)c * r; t++) { s1 += X[t]; s2 += X[t] * X[t]; }
    return l1 * s1 + l2 * s2;
}

/* KKT residuals of one half's NQPs at X (c x r): g = G x + h in the original
 * scale.  out[0] = max_i |min(x_i, g_i)| (0 exactly at a KKT point),
 * out[1] = max(0, -min x) (nonnegativity), out[2] = max x_i |g_i|
 * (complementarity), out[3] = max(0, -min over x_i == 0 of g_i)
 * (gradient >= 0 on zero entries). */
void oracle_kkt(long c, int r, const double *G, const double *P, double l1, const double *X,
                double *out) {
    double o0 = 0.0, o1 = 0.0, o2 = 0.0, o3 = 0.0;
    for (long j = 0; j < c; j++)
        for (int a = 0; a < r; a++) {
            double gv = -P[(size_t)j * r + a] + l1;
            for (int b = 0; b < r; b++) gv += G[(size_t)a * r + b] * X[(size_t)j * r + b];
            double xv = X[(size_t)j * r + a];
            double mm = fabs(xv < gv ? xv : gv);
            if (mm > o0) o0 = mm;
            if (-xv > o1) o1 = -xv;
            if (xv * fabs(gv) > o2) o2 = xv * fabs(gv);
            if (xv == 0.0 && -gv > o3) o3 = -gv;
        }
    out[0] = o0; out[1] = o1; out[2] = o2; out[3] = o3;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2 (with the regularised NQPs of Section 3.5): T outer
 * iterations, each an H-update (E-step: W fixed, one NQP per column of V)
 * followed by a W-update (M-step: H fixed, one NQP per row of V) whose Gram
 * is built from the freshly updated H.
 *
 *   kind     : 0 dense V (m x n row-major in V), 1 CSR V (rowptr/colidx/vals).
 *   reg      : {l1_w, l2_w, l1_h, l2_h}.
 *   W, Ht    : in = start point, out = result.
 *   loss     : optional [T+1], 0.5||V - W H||^2 before and after each outer
 *              iteration.
 *   jhalf    : optional [2T+1], the regularised objective J before and after
 *              every half-iteration.
 *   inner    : optional [2T], total inner iterations of each half.
 */
int oracle_nmf_fit(int kind, long m, long n, const double *V, const int *rowptr, const int *colidx,
                   const double *vals, int r, const double *reg, double *W, double *Ht, int T,
                   int max_inner, double eps, int ls_guard, double *loss, double *jhalf,
                   long *inner) {
    double l1w = reg[0], l2w = reg[1], l1h = reg[2], l2h = reg[3];
    double *G = (double *)malloc(sizeof(double) * (size_t)r * r);
    double *PH = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * r);
    double *PW = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * r);
#define LOSS() (kind == 0 ? oracle_loss_dense(m, n, V, r, W, Ht) \
                          : oracle_loss_csr(m, n, rowptr, colidx, vals, r, W, Ht))
#define JOBJ(l) ((l) + oracle_reg_term(n, r, Ht, l1h, l2h) + oracle_reg_term(m, r, W, l1w, l2w))
    if (loss || jhalf) {
        double l = LOSS();
        if (loss) loss[0] = l;
        if (jhalf) jhalf[0] = JOBJ(l);
    }
    for (int t = 0; t < T; t++) {
        /* E-step: H-update with W fixed */
        oracle_gram(m, r, W, l2h, G);
        if (kind == 0) oracle_product_dense(m, n, V, 0, r, W, PH);
        else oracle_product_csr(m, n, rowptr, colidx, vals, 0, r, W, PH);
        long kh = oracle_half_update(n, r, G, PH, l1h, Ht, max_inner, eps, ls_guard, NULL);
        if (inner) inner[2 * t] = kh;
        if (jhalf) jhalf[2 * t + 1] = JOBJ(LOSS());
        /* M-step: W-update with the new H fixed */
        oracle_gram(n, r, Ht, l2w, G);
        if (kind == 0) oracle_product_dense(m, n, V, 1, r, Ht, PW);
        else oracle_product_csr(m, n, rowptr, colidx, vals, 1, r, Ht, PW);
        long kw = oracle_half_update(m, r, G, PW, l1w, W, max_inner, eps, ls_guard, NULL);
        if (inner) inner[2 * t + 1] = kw;
        if (loss || jhalf) {
            double l = LOSS();
            if (loss) loss[t + 1] = l;
            if (jhalf) jhalf[2 * t + 2] = JOBJ(l);
        }
    }
#undef LOSS
#undef JOBJ
    free(G); free(PH); free(PW);
    return 0;
}
