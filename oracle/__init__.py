"""FP64 CPU oracle for the alternating anti-lopsided NNLS method (arXiv:1506.08938).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the GPU
library never does, and the two share no code.

Everything here is a thin ctypes wrapper over ``nmf_oracle.c`` (plain C,
double precision, sums in ascending index order, OpenMP only across
independent columns).  Citations of the paper sit in that file, next to each
function.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nmf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NO_RESCALE = 1
NO_CD = 2
NO_LS = 4

_d = ctypes.POINTER(ctypes.c_double)
_i = ctypes.POINTER(ctypes.c_int)
_l = ctypes.POINTER(ctypes.c_long)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, IEEE double, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_rescale.argtypes = [ctypes.c_int, _d, _d, _d, _i]
        L.oracle_nqp_flags.argtypes = [ctypes.c_int, _d, _d, _d, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_int, _d]
        L.oracle_nqp_flags.restype = ctypes.c_int
        L.oracle_nqp_batch.argtypes = [ctypes.c_int, ctypes.c_long, _d, _d, _d, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_int, _i]
        L.oracle_nqp_batch.restype = ctypes.c_long
        L.oracle_nqp_trace.argtypes = [ctypes.c_int, _d, _d, _d, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_int, _d]
        L.oracle_nqp_trace.restype = ctypes.c_int
        L.oracle_nqp_batch_cdtrace.argtypes = [ctypes.c_int, ctypes.c_long, _d, _d, _d, ctypes.c_int,
                                               ctypes.c_double, ctypes.c_int, ctypes.c_int, _i, _d]
        L.oracle_nqp_batch_cdtrace.restype = ctypes.c_long
        L.oracle_nqp_batch_faststop.argtypes = [ctypes.c_int, ctypes.c_long, _d, _d, _d, ctypes.c_int,
                                                ctypes.c_double, ctypes.c_int, ctypes.c_long, _i, _d]
        L.oracle_nqp_batch_faststop.restype = ctypes.c_long
        L.oracle_gram.argtypes = [ctypes.c_long, ctypes.c_int, _d, ctypes.c_double, _d]
        L.oracle_product_dense.argtypes = [ctypes.c_long, ctypes.c_long, _d, ctypes.c_int,
                                           ctypes.c_int, _d, _d]
        L.oracle_product_csr.argtypes = [ctypes.c_long, ctypes.c_long, _i, _i, _d, ctypes.c_int,
                                         ctypes.c_int, _d, _d]
        L.oracle_half_update.argtypes = [ctypes.c_long, ctypes.c_int, _d, _d, ctypes.c_double, _d,
                                         ctypes.c_int, ctypes.c_double, ctypes.c_int, _i]
        L.oracle_half_update.restype = ctypes.c_long
        L.oracle_loss_dense.argtypes = [ctypes.c_long, ctypes.c_long, _d, ctypes.c_int, _d, _d]
        L.oracle_loss_dense.restype = ctypes.c_double
        L.oracle_loss_csr.argtypes = [ctypes.c_long, ctypes.c_long, _i, _i, _d, ctypes.c_int, _d,
                                      _d]
        L.oracle_loss_csr.restype = ctypes.c_double
        L.oracle_reg_term.argtypes = [ctypes.c_long, ctypes.c_int, _d, ctypes.c_double,
                                      ctypes.c_double]
        L.oracle_reg_term.restype = ctypes.c_double
        L.oracle_kkt.argtypes = [ctypes.c_long, ctypes.c_int, _d, _d, ctypes.c_double, _d, _d]
        L.oracle_nmf_fit.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_long, _d, _i, _i, _d,
                                     ctypes.c_int, _d, _d, _d, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_int, _d, _d, _l]
        L.oracle_nmf_fit.restype = ctypes.c_int
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=_d):
    return None if a is None else a.ctypes.data_as(t)


def num_threads() -> int:
    return lib().oracle_num_threads()


def rescale(H):
    """Anti-lopsided rescale of H: returns (Q, d, frozen) with Q_ii = 1."""
    H = _f64(H)
    r = H.shape[0]
    Q = np.empty((r, r)); d = np.empty(r); fr = np.empty(r, dtype=np.int32)
    lib().oracle_rescale(r, _p(H), _p(Q), _p(d), _p(fr, _i))
    return Q, d, fr.astype(bool)


def nqp(H, h, x0, max_inner=100, eps=1e-3, ls_guard=1, flags=0, trace=False):
    """Algorithm 3 on one problem.  Returns (x, iters) or (x, iters, fk)."""
    H = _f64(H); h = _f64(h); x = _f64(x0).copy()
    r = H.shape[0]
    fk = np.full(max_inner + 1, np.nan) if trace else None
    k = lib().oracle_nqp_flags(r, _p(H), _p(h), _p(x), int(max_inner), float(eps), int(ls_guard),
                               int(flags), _p(fk))
    return (x, k, fk[:k + 1]) if trace else (x, k)


def nqp_batch(H, h, x0, max_inner=100, eps=1e-3, ls_guard=1):
    """Independent NQPs sharing H; h, x0 are (ncols, r).  Returns (x, iters)."""
    H = _f64(H); h = _f64(h); x = _f64(x0).copy()
    ncols, r = h.shape
    it = np.zeros(ncols, dtype=np.int32)
    lib().oracle_nqp_batch(r, ncols, _p(H), _p(h), _p(x), int(max_inner), float(eps),
                           int(ls_guard), _p(it, _i))
    return x, it


def nqp_trace(H, h, x0, max_inner=100, eps=1e-3, ls_guard=1):
    """Algorithm 3 on one problem, returning (x, iters, nk) with nk[k] =
    ||f~_k||^2 for k = 0..iters (no fast-break)."""
    H = _f64(H); h = _f64(h); x = _f64(x0).copy()
    r = H.shape[0]
    nk = np.full(max_inner + 1, np.nan)
    k = lib().oracle_nqp_trace(r, _p(H), _p(h), _p(x), int(max_inner), float(eps), int(ls_guard),
                               _p(nk))
    return x, k, nk[:k + 1]


def nqp_batch_cdtrace(H, h, x0, max_inner=100, eps=1e-3, ls_guard=1, trace_iters=None):
    """Independent NQPs sharing H (the results of nqp_batch) with a record of
    every greedy CD choice of the first trace_iters (default max_inner)
    iterations.  Returns (x, iters, cd) with cd of shape (ncols, trace_iters,
    r, 6): per CD step the chosen coordinate (-1: the sweep ended there; -2:
    not reached), the decrease of that choice, the largest decrease among the
    other coordinates (-1: none), |delta| of both, and the size of the terms
    of the gradient, max_i (|q_i| + sum_j |Q_ij y_j|)."""
    H = _f64(H); h = _f64(h); x = _f64(x0).copy()
    ncols, r = h.shape
    ti = int(max_inner if trace_iters is None else min(trace_iters, max_inner))
    it = np.zeros(ncols, dtype=np.int32)
    cd = np.full((ncols, ti, r, 6), -2.0)
    lib().oracle_nqp_batch_cdtrace(r, ncols, _p(H), _p(h), _p(x), int(max_inner), float(eps),
                                   int(ls_guard), ti, _p(it, _i), _p(cd))
    return x, it, cd


def nqp_batch_faststop(H, h, x0, chunk, max_inner=100, eps=1e-3, ls_guard=1):
    """Independent NQPs with Algorithm 3's fast-break over fixed chunks of
    `chunk` consecutive columns.  Returns (x, iters, final ||f~||^2)."""
    H = _f64(H); h = _f64(h); x = _f64(x0).copy()
    ncols, r = h.shape
    it = np.zeros(ncols, dtype=np.int32)
    nk = np.zeros(ncols)
    lib().oracle_nqp_batch_faststop(r, ncols, _p(H), _p(h), _p(x), int(max_inner), float(eps),
                                    int(ls_guard), int(chunk), _p(it, _i), _p(nk))
    return x, it, nk


def gram(A, l2=0.0):
    A = _f64(A)
    k, r = A.shape
    G = np.empty((r, r))
    lib().oracle_gram(k, r, _p(A), float(l2), _p(G))
    return G


def product_dense(V, A, trans):
    """trans=0: (W'V)' (n x r) with A = W; trans=1: V Ht (m x r) with A = Ht."""
    V = _f64(V); A = _f64(A)
    m, n = V.shape
    r = A.shape[1]
    P = np.empty(((m if trans else n), r))
    lib().oracle_product_dense(m, n, _p(V), int(trans), r, _p(A), _p(P))
    return P


def _csr_parts(csr):
    rowptr = np.ascontiguousarray(csr.indptr, dtype=np.int32)
    colidx = np.ascontiguousarray(csr.indices, dtype=np.int32)
    vals = _f64(csr.data)
    return rowptr, colidx, vals


def product_csr(csr, A, trans):
    m, n = csr.shape
    rp, ci, va = _csr_parts(csr)
    A = _f64(A)
    r = A.shape[1]
    P = np.empty(((m if trans else n), r))
    lib().oracle_product_csr(m, n, _p(rp, _i), _p(ci, _i), _p(va), int(trans), r, _p(A), _p(P))
    return P


def half_update(G, P, l1, X, max_inner=100, eps=1e-3, ls_guard=1):
    G = _f64(G); P = _f64(P); X = _f64(X).copy()
    c, r = X.shape
    it = np.zeros(c, dtype=np.int32)
    lib().oracle_half_update(c, r, _p(G), _p(P), float(l1), _p(X), int(max_inner), float(eps),
                             int(ls_guard), _p(it, _i))
    return X, it


def loss(V, W, Ht):
    """0.5||V - W Ht'||^2 for dense ndarray V or scipy CSR V."""
    W = _f64(W); Ht = _f64(Ht)
    r = W.shape[1]
    if isinstance(V, np.ndarray):
        V = _f64(V)
        m, n = V.shape
        return lib().oracle_loss_dense(m, n, _p(V), r, _p(W), _p(Ht))
    m, n = V.shape
    rp, ci, va = _csr_parts(V)
    return lib().oracle_loss_csr(m, n, _p(rp, _i), _p(ci, _i), _p(va), r, _p(W), _p(Ht))


def objective(V, W, Ht, reg):
    """J = 0.5||V - WH||^2 + l1_h sum H + l2_h ||H||^2 + l1_w sum W + l2_w ||W||^2."""
    l1w, l2w, l1h, l2h = reg
    W = _f64(W); Ht = _f64(Ht)
    L = lib()
    return (loss(V, W, Ht) + L.oracle_reg_term(Ht.shape[0], Ht.shape[1], _p(Ht), l1h, l2h)
            + L.oracle_reg_term(W.shape[0], W.shape[1], _p(W), l1w, l2w))


def kkt(G, P, l1, X):
    """KKT residuals of one half's NQPs: (minmap, neg, compl, gradneg)."""
    G = _f64(G); P = _f64(P); X = _f64(X)
    c, r = X.shape
    out = np.empty(4)
    lib().oracle_kkt(c, r, _p(G), _p(P), float(l1), _p(X), _p(out))
    return out


def nmf_fit(V, r, reg, W0, Ht0, T, max_inner=100, eps=1e-3, ls_guard=1, want_trace=True):
    """Algorithm 2 with regularised NQPs.  V is a dense ndarray or a scipy CSR
    matrix; reg = (l1_w, l2_w, l1_h, l2_h).  Returns a dict with W, Ht, loss
    [T+1], jhalf [2T+1] and inner [2T]."""
    W = _f64(W0).copy(); Ht = _f64(Ht0).copy()
    m, n = V.shape
    regv = _f64(reg)
    loss_tr = np.full(T + 1, np.nan) if want_trace else None
    jh = np.full(2 * T + 1, np.nan) if want_trace else None
    inner = np.zeros(2 * T, dtype=np.int64)
    if isinstance(V, np.ndarray):
        Vd = _f64(V)
        lib().oracle_nmf_fit(0, m, n, _p(Vd), None, None, None, r, _p(regv), _p(W), _p(Ht), T,
                             max_inner, eps, ls_guard, _p(loss_tr), _p(jh), _p(inner, _l))
    else:
        rp, ci, va = _csr_parts(V)
        lib().oracle_nmf_fit(1, m, n, None, _p(rp, _i), _p(ci, _i), _p(va), r, _p(regv), _p(W),
                             _p(Ht), T, max_inner, eps, ls_guard, _p(loss_tr), _p(jh),
                             _p(inner, _l))
    return {"W": W, "Ht": Ht, "loss": loss_tr, "jhalf": jh, "inner": inner}
