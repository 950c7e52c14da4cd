"""Seeded synthetic inputs shaped like the paper's NMF workloads.

This module only draws random numbers and assembles matrices.  It holds none
of the method's arithmetic (no Gram, no product, no solve), so both the GPU
library's tests and the FP64 oracle can be fed from it.

All streams are numpy PCG64.  Data of workload ``c`` uses seed ``1000 + c``
and the start point of the fit uses ``1100 + c``, so the start point never
depends on how the data were drawn.  Every start point is drawn in float32
and handed identically to the GPU (float32) and to the oracle (the same
values widened to float64).

Workloads (V is m x n; W m x r and Ht n x r are the factors):
  1 dense, small    V(200x150) = W0 H0 + |N(0, 0.01)|, W0, H0 ~ U[0,1],
                    inner dimension 10; r = 10, no regularisation.
  2 dense, large    V(20000x10000) = W0 H0 + |N(0, 0.05)|, W0, H0 ~
                    Gamma(shape 2, scale 0.5), inner dimension 64; r = 64,
                    L2 = 0.01 on both factors.
  3 sparse, text    CSR V(200000x100000): each row holds 100 distinct
                    columns, the first 100 distinct values of an i.i.d.
                    truncated-Zipf(1.1) rank sequence over 1..100000 mapped
                    through a seeded permutation; values log(1 + K), K ~
                    Poisson(3) conditioned on K >= 1; r = 100, L1 = 0.1 on H,
                    L2 = 0.01 on W.
  4 batched         many small dense problems, m ~ logU[64, 4096], n ~
                    logU[64, 2048], r ~ U{4..64}, V = W0 H0 + |N(0, 0.01)|,
                    W0, H0 ~ U[0,1] with inner dimension r.
  5 serving         a resident basis (100000 x 128) fitted to V = W0 H0 +
                    |N(0, 0.05)| with Gamma(2, 0.5) factors; fold-in requests
                    of c ~ logU[1, 8192] sparse columns over its 100000 rows,
                    0.5% density (500 uniform rows per column, duplicates
                    dropped), values as workload 3; 5% of the requests are
                    small full fits (m, n ~ logU[64, 2048], r ~ U{4..32}).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

DATA_SEED = 1000
INIT_SEED = 1100


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def start_point(m: int, n: int, r: int, seed: int):
    """W0 (m x r) and Ht0 (n x r) ~ U[0,1) in float32 (the random start of
    the alternating fit)."""
    g = rng(seed)
    W = g.random((m, r), dtype=np.float32)
    Ht = g.random((n, r), dtype=np.float32)
    return W, Ht


# ----------------------------------------------------------------------------- dense
def dense_lowrank(m, n, k, seed, dist="uniform", noise=0.01):
    """V = W0 H0 + |N(0, noise)| in float32 (float64 accumulation of W0 H0)."""
    g = rng(seed)
    if dist == "uniform":
        W0 = g.random((m, k)); H0 = g.random((k, n))
    elif dist == "gamma":
        W0 = g.gamma(2.0, 0.5, (m, k)); H0 = g.gamma(2.0, 0.5, (k, n))
    else:
        raise ValueError(dist)
    V = W0 @ H0
    V += np.abs(g.normal(0.0, noise, (m, n)))
    return np.ascontiguousarray(V, dtype=np.float32)


def workload1():
    V = dense_lowrank(200, 150, 10, DATA_SEED + 1, "uniform", 0.01)
    W, Ht = start_point(200, 150, 10, INIT_SEED + 1)
    return dict(name="dense 200x150 r=10", V=V, r=10, reg=(0.0, 0.0, 0.0, 0.0), T=50, W0=W, Ht0=Ht)


def workload2(m=20000, n=10000):
    """The large dense workload; m, n may be reduced for a same-recipe slice."""
    V = dense_lowrank(m, n, 64, DATA_SEED + 2, "gamma", 0.05)
    W, Ht = start_point(m, n, 64, INIT_SEED + 2)
    return dict(name=f"dense {m}x{n} r=64", V=V, r=64, reg=(0.0, 0.01, 0.0, 0.01), T=100, W0=W,
                Ht0=Ht)


def workload2_slice():
    """V[:2000, :1000] of workload 2, run as a problem of its own (same data)."""
    full = workload2()
    V = np.ascontiguousarray(full["V"][:2000, :1000])
    W = np.ascontiguousarray(full["W0"][:2000]); Ht = np.ascontiguousarray(full["Ht0"][:1000])
    return dict(name="dense 2000x1000 slice r=64", V=V, r=64, reg=full["reg"], T=100, W0=W, Ht0=Ht)


# ----------------------------------------------------------------------------- sparse
def _positive_poisson(g, lam, size):
    k = g.poisson(lam, size)
    bad = np.nonzero(k == 0)[0]
    while bad.size:
        k[bad] = g.poisson(lam, bad.size)
        bad = bad[k[bad] == 0]
    return k


def zipf_rows(m, ncols, per_row, s, seed, batch=20000):
    """CSR (indptr, indices) of an m x ncols pattern with exactly ``per_row``
    distinct columns per row: the first distinct values of an i.i.d.
    truncated-Zipf(s) rank sequence, mapped through a seeded permutation."""
    g = rng(seed)
    pk = np.arange(1, ncols + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(pk); cdf /= cdf[-1]
    perm = g.permutation(ncols).astype(np.int32)
    out = np.empty((m, per_row), dtype=np.int32)
    for r0 in range(0, m, batch):
        rows = np.arange(r0, min(m, r0 + batch))
        todo = rows
        draws = max(2 * per_row, per_row + 64)
        while todo.size:
            u = g.random((todo.size, draws))
            d = np.searchsorted(cdf, u, side="right").astype(np.int32)
            np.minimum(d, ncols - 1, out=d)
            order = np.argsort(d, axis=1, kind="stable")
            sd = np.take_along_axis(d, order, axis=1)
            first_sorted = np.ones_like(sd, dtype=bool)
            first_sorted[:, 1:] = sd[:, 1:] != sd[:, :-1]
            first = np.zeros_like(first_sorted)
            np.put_along_axis(first, order, first_sorted, axis=1)
            cnt = first.sum(axis=1)
            ok = cnt >= per_row
            keep = first & (np.cumsum(first, axis=1) <= per_row)
            sel = d[ok][keep[ok]].reshape(-1, per_row)
            out[todo[ok]] = perm[sel]
            todo = todo[~ok]
            draws *= 2
    out.sort(axis=1)
    indptr = np.arange(0, (m + 1) * per_row, per_row, dtype=np.int64)
    return indptr, out.reshape(-1)


def log_poisson_values(nnz, seed, lam=3.0):
    g = rng(seed)
    return np.log1p(_positive_poisson(g, lam, nnz).astype(np.float64)).astype(np.float32)


def sparse_text(m, n, per_row, seed, s=1.1):
    indptr, indices = zipf_rows(m, n, per_row, s, seed)
    vals = log_poisson_values(indices.size, seed + 7)
    V = sp.csr_matrix((vals, indices, indptr.astype(np.int32)), shape=(m, n))
    V.has_sorted_indices = True
    return V


def workload3(m=200000, n=100000, per_row=100):
    """Sparse text-like workload; smaller m, n, per_row give a same-recipe
    instance for tests."""
    V = sparse_text(m, n, per_row, DATA_SEED + 3)
    W, Ht = start_point(m, n, 100, INIT_SEED + 3)
    return dict(name=f"sparse {m}x{n} nnz/row={per_row} r=100", V=V, r=100,
                reg=(0.0, 0.01, 0.1, 0.0), T=50, W0=W, Ht0=Ht)


def csr_transpose(V: sp.csr_matrix) -> sp.csr_matrix:
    """CSR of V' (columns of V as rows, ascending row order within each)."""
    T = V.T.tocsr()
    T.sort_indices()
    return T


# ----------------------------------------------------------------------------- batched
def workload4(count=1024, seed=DATA_SEED + 4, first=None):
    """``count`` uneven dense problems; ``first`` keeps only the first few
    (the shapes of problem i never depend on ``first``)."""
    g = rng(seed)
    ms = np.rint(np.exp(g.uniform(np.log(64), np.log(4096), count))).astype(int)
    ns = np.rint(np.exp(g.uniform(np.log(64), np.log(2048), count))).astype(int)
    rs = g.integers(4, 65, count)
    probs = []
    for i in range(count if first is None else min(first, count)):
        V = dense_lowrank(int(ms[i]), int(ns[i]), int(rs[i]), seed * 10007 + i, "uniform", 0.01)
        W, Ht = start_point(int(ms[i]), int(ns[i]), int(rs[i]), INIT_SEED + 4 + 7919 * (i + 1))
        probs.append(dict(V=V, r=int(rs[i]), reg=(0.0, 0.0, 0.0, 0.0), W0=W, Ht0=Ht))
    return probs


# ----------------------------------------------------------------------------- serving
def request_sizes(count, seed, cmax=8192):
    g = rng(seed)
    return np.rint(np.exp(g.uniform(0.0, np.log(cmax), count))).astype(int)


def foldin_columns(m, c, per_col, seed):
    """A request of c sparse columns over m rows: CSR of the request's
    transpose (c x m), per_col distinct uniform rows per column."""
    g = rng(seed)
    idx = np.empty((c, per_col), dtype=np.int32)
    for j in range(c):
        idx[j] = np.sort(g.choice(m, per_col, replace=False))
    vals = log_poisson_values(c * per_col, seed + 13)
    indptr = np.arange(0, (c + 1) * per_col, per_col, dtype=np.int32)
    return sp.csr_matrix((vals, idx.reshape(-1), indptr), shape=(c, m))


def foldin_columns_many(m, c, per_col, seed):
    """Large requests quickly: per_col rows per column drawn uniformly with
    replacement and de-duplicated (a column keeps per_col minus its few
    collisions), values as workload 3.  CSR of the request's transpose."""
    g = rng(seed)
    idx = np.sort(g.integers(0, m, (c, per_col), dtype=np.int32), axis=1)
    keep = np.ones((c, per_col), dtype=bool)
    keep[:, 1:] = idx[:, 1:] != idx[:, :-1]
    counts = keep.sum(axis=1)
    indptr = np.zeros(c + 1, dtype=np.int32)
    np.cumsum(counts, out=indptr[1:])
    cols = idx[keep]
    vals = log_poisson_values(cols.size, seed + 13)
    return sp.csr_matrix((vals, cols, indptr), shape=(c, m))


def workload5_basis(m=100000, nb=2048, r=128):
    """Data and start point of the prior fit that yields the resident basis:
    V (m x nb) = W0 H0 + |N(0, 0.05)|, Gamma(2, 0.5) factors of inner
    dimension r."""
    V = dense_lowrank(m, nb, r, DATA_SEED + 5, "gamma", 0.05)
    W, Ht = start_point(m, nb, r, INIT_SEED + 5)
    return dict(V=V, r=r, W0=W, Ht0=Ht)


def workload5_fits(count, seed=DATA_SEED + 55):
    """Small full-fit requests mixed into the serving stream: m, n ~
    logU[64, 2048], r ~ U{4..32}, V = W0 H0 + |N(0, 0.01)|, U[0,1] factors."""
    g = rng(seed)
    ms = np.rint(np.exp(g.uniform(np.log(64), np.log(2048), count))).astype(int)
    ns = np.rint(np.exp(g.uniform(np.log(64), np.log(2048), count))).astype(int)
    rs = g.integers(4, 33, count)
    out = []
    for i in range(count):
        V = dense_lowrank(int(ms[i]), int(ns[i]), int(rs[i]), seed * 10007 + i, "uniform", 0.01)
        W, Ht = start_point(int(ms[i]), int(ns[i]), int(rs[i]), INIT_SEED + 55 + 7919 * (i + 1))
        out.append(dict(V=V, r=int(rs[i]), W0=W, Ht0=Ht))
    return out


def poisson_arrivals(count, rate, seed):
    """Arrival times (s) of a Poisson process of the given rate."""
    return np.cumsum(rng(seed).exponential(1.0 / rate, count))


def nqp_instance(r, ncols, seed, k=None, l1=0.0, l2=0.0, kind="random"):
    """Random NNLS data (A k x r, B k x ncols, x0 ncols x r), nonnegative like
    the NMF subproblems.  ``kind`` shapes A: "random" U[0,1); "orthogonal"
    (disjoint row supports, so A'A is diagonal); "dupcol" (column 1 repeats
    column 0, a singular A'A); "zerocol" (column 0 is zero)."""
    g = rng(seed)
    k = k or max(2 * r, 16)
    A = g.random((k, r))
    if kind == "orthogonal":
        A = np.zeros((k, r))
        owner = np.arange(k) % r
        A[np.arange(k), owner] = g.random(k) + 0.5
    elif kind == "dupcol" and r > 1:
        A[:, 1] = A[:, 0]
    elif kind == "zerocol":
        A[:, 0] = 0.0
    B = g.random((k, ncols)) * r * 0.25
    x0 = g.random((ncols, r)).astype(np.float32)
    return dict(A=A.astype(np.float32), B=B.astype(np.float32), x0=x0, l1=l1, l2=l2)
