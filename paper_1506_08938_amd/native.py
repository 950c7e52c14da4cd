"""ctypes binding of ``libnmf_mi355x.so`` (the C ABI in ``include/nmf.h``).

Argument marshalling only: torch supplies device memory and the current
stream; every step of the method runs in the library's HIP kernels.  If the
library has not been built this module raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libnmf_mi355x.so")

NMF_OK, NMF_E_INVAL, NMF_E_NOMEM, NMF_E_DEVICE, NMF_E_UNSUPPORTED, NMF_E_BUSY, NMF_E_NONFINITE = (
    0, -1, -2, -3, -4, -5, -6)
NMF_DENSE, NMF_CSR = 0, 1
NMF_FP32, NMF_BF16 = 0, 1
MAX_RANK = 128

# every entry point include/nmf.h declares
EXPORTS = [
    "nmf_default_opts", "nmf_last_error", "nnls_solve_batch", "nnls_layout", "nmf_gram",
    "nmf_product",
    "nmf_plan_create", "nmf_plan_run", "nmf_plan_destroy", "nmf_plan_profile", "nmf_plan_timers",
    "nmf_fit", "nmf_fit_streamed", "nmf_fit_single_pass", "nmf_objective", "nmf_fit_batched",
    "nmf_server_create", "nmf_server_submit", "nmf_server_poll", "nmf_server_poll_times", "nmf_server_wait",
    "nmf_server_stats", "nmf_server_destroy",
    "nmf_basis_create", "nmf_foldin", "nmf_basis_destroy", "nmf_foldin_noalloc",
    "nmf_probe_gather", "nmf_dense_product_time",
]


class NmfMatrix(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("dense", ctypes.c_void_p), ("ld", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("colidx", ctypes.c_void_p),
                ("vals", ctypes.c_void_p), ("nnz", ctypes.c_int64),
                ("t_rowptr", ctypes.c_void_p), ("t_colidx", ctypes.c_void_p),
                ("t_vals", ctypes.c_void_p)]


class NmfReg(ctypes.Structure):
    _fields_ = [("l1_w", ctypes.c_float), ("l2_w", ctypes.c_float), ("l1_h", ctypes.c_float),
                ("l2_h", ctypes.c_float)]


class NmfOpts(ctypes.Structure):
    _fields_ = [("max_outer", ctypes.c_int32), ("max_inner", ctypes.c_int32),
                ("eps", ctypes.c_double), ("ls_guard", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("objective_every", ctypes.c_int32),
                ("check_finite", ctypes.c_int32), ("lanes", ctypes.c_int32),
                ("fast_break_cols", ctypes.c_int32)]


class NmfStats(ctypes.Structure):
    _fields_ = [("loss", ctypes.c_double), ("objective", ctypes.c_double),
                ("kkt_w", ctypes.c_double), ("kkt_h", ctypes.c_double), ("kbar", ctypes.c_double),
                ("inner_total", ctypes.c_int64), ("outer_done", ctypes.c_int32),
                ("kkt_w_cond", ctypes.c_double * 3), ("kkt_h_cond", ctypes.c_double * 3)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        for k in ("kkt_w_cond", "kkt_h_cond"):
            d[k] = tuple(d[k])
        return d


class NmfProblem(ctypes.Structure):
    _fields_ = [("V", NmfMatrix), ("r", ctypes.c_int32), ("reg", NmfReg),
                ("W", ctypes.c_void_p), ("Ht", ctypes.c_void_p)]


NMF_REQ_FOLDIN, NMF_REQ_FIT = 0, 1


class NmfRequest(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("V", NmfMatrix), ("out", ctypes.c_void_p),
                ("iters", ctypes.c_void_p), ("r", ctypes.c_int32), ("reg", NmfReg),
                ("fit_opts", NmfOpts), ("W", ctypes.c_void_p), ("Ht", ctypes.c_void_p)]


class NmfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"nmf status {status}: {msg}")
        self.status = status


_lib = None
_vp = ctypes.c_void_p


def lib():
    """Loads the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1506_08938_amd.build` (hipcc, gfx950)")
        # torch loads its own copy of the HIP runtime (by an unversioned
        # name).  Importing it first lets this library's libamdhip64.so.7
        # dependency resolve to that same copy: one runtime per process, so
        # device pointers and streams are shared.  Loaded the other way round,
        # the process would hold two runtimes and one of them sees no GPU.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        L.nmf_last_error.restype = ctypes.c_char_p
        L.nmf_default_opts.argtypes = [ctypes.POINTER(NmfOpts)]
        L.nmf_default_opts.restype = None
        L.nnls_solve_batch.argtypes = [ctypes.c_int32, ctypes.c_int64, _vp, _vp, _vp,
                                       ctypes.POINTER(NmfOpts), _vp, _vp]
        L.nnls_layout.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.nmf_gram.argtypes = [_vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_int32,
                               _vp, _vp]
        L.nmf_product.argtypes = [ctypes.POINTER(NmfMatrix), ctypes.c_int32, ctypes.c_int32, _vp,
                                  ctypes.c_int32, _vp, _vp]
        L.nmf_plan_create.argtypes = [ctypes.POINTER(NmfMatrix), ctypes.c_int32,
                                      ctypes.POINTER(NmfReg), ctypes.POINTER(NmfOpts),
                                      ctypes.POINTER(_vp), _vp]
        L.nmf_plan_run.argtypes = [_vp, _vp, _vp, ctypes.c_int32, _vp, ctypes.POINTER(NmfStats),
                                   _vp]
        L.nmf_plan_profile.argtypes = [_vp, ctypes.c_int32]
        L.nmf_plan_timers.argtypes = [_vp, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64)]
        L.nmf_plan_destroy.argtypes = [_vp]
        L.nmf_plan_destroy.restype = None
        L.nmf_fit.argtypes = [ctypes.POINTER(NmfMatrix), ctypes.c_int32, ctypes.POINTER(NmfReg),
                              ctypes.POINTER(NmfOpts), _vp, _vp, _vp, ctypes.POINTER(NmfStats),
                              _vp]
        L.nmf_fit_streamed.argtypes = [_vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                       ctypes.POINTER(NmfReg), ctypes.POINTER(NmfOpts), ctypes.c_int64,
                                       _vp, _vp, _vp, ctypes.POINTER(NmfStats), _vp]
        L.nmf_fit_single_pass.argtypes = [ctypes.POINTER(NmfMatrix), ctypes.c_int32, ctypes.POINTER(NmfReg),
                                          ctypes.POINTER(NmfOpts), ctypes.c_int64, _vp, _vp, _vp,
                                          ctypes.POINTER(NmfStats), _vp]
        L.nmf_objective.argtypes = [ctypes.POINTER(NmfMatrix), ctypes.c_int32,
                                    ctypes.POINTER(NmfReg), _vp, _vp, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double), _vp]
        L.nmf_fit_batched.argtypes = [ctypes.c_int32, ctypes.POINTER(NmfProblem),
                                      ctypes.POINTER(NmfOpts), ctypes.POINTER(NmfStats), _vp]
        L.nmf_server_create.argtypes = [_vp, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64,
                                        ctypes.POINTER(_vp)]
        L.nmf_server_submit.argtypes = [_vp, ctypes.POINTER(NmfRequest),
                                        ctypes.POINTER(ctypes.c_uint64)]
        L.nmf_server_poll.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_double)]
        L.nmf_server_poll_times.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_double)]
        L.nmf_server_wait.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
        L.nmf_server_stats.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.nmf_server_destroy.argtypes = [_vp]
        L.nmf_server_destroy.restype = None
        L.nmf_basis_create.argtypes = [_vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_float,
                                       ctypes.c_float, ctypes.POINTER(NmfOpts),
                                       ctypes.POINTER(_vp), _vp]
        L.nmf_foldin.argtypes = [_vp, ctypes.POINTER(NmfMatrix), _vp, _vp, _vp]
        L.nmf_foldin_noalloc.argtypes = [_vp, ctypes.POINTER(NmfMatrix), _vp, _vp, _vp]
        L.nmf_basis_destroy.argtypes = [_vp]
        L.nmf_basis_destroy.restype = None
        L.nmf_probe_gather.argtypes = [_vp, ctypes.c_int64, ctypes.c_int32, _vp, ctypes.c_int64, _vp, _vp]
        L.nmf_dense_product_time.argtypes = [_vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                             ctypes.c_int32, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_double), _vp]
        _lib = L
    return _lib


def last_error() -> str:
    return lib().nmf_last_error().decode()


def check(status: int):
    if status != NMF_OK:
        raise NmfError(status, last_error())


def opts(**kw) -> NmfOpts:
    o = NmfOpts()
    lib().nmf_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


# --------------------------------------------------------------------------- torch plumbing
def _torch():
    import torch
    return torch


def stream_ptr():
    return _torch().cuda.current_stream().cuda_stream


def _dev(t, dtype, name, shape=None):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _ptr(t):
    return None if t is None else t.data_ptr()


def nnls_solve_batch(gram, h, X, opt: NmfOpts | None = None, iters=None):
    """Algorithm 3 on every row of h/X (in place on X).  gram (r, r), h and X
    (ncols, r) float32 device tensors; iters optional int32 (ncols,)."""
    torch = _torch()
    r = gram.shape[0]
    ncols = h.shape[0]
    _dev(gram, torch.float32, "gram", (r, r))
    _dev(h, torch.float32, "h", (ncols, r))
    _dev(X, torch.float32, "X", (ncols, r))
    _dev(iters, torch.int32, "iters", (ncols,))
    opt = opt or opts()
    check(lib().nnls_solve_batch(r, ncols, _ptr(gram), _ptr(h), _ptr(X), ctypes.byref(opt),
                                 _ptr(iters), stream_ptr()))
    return X


def layout(r, ncols, lanes=0):
    """nnls_layout: (E, L) of the solve kernel for rank r and ncols columns."""
    E = ctypes.c_int32(); L = ctypes.c_int32()
    check(lib().nnls_layout(int(r), int(ncols), int(lanes), ctypes.byref(E), ctypes.byref(L)))
    return E.value, L.value


class DeviceMatrix:
    """Keeps the device arrays of V alive and exposes its nmf_matrix struct."""

    def __init__(self, V, with_transpose=True):
        torch = _torch()
        self.keep = []
        m = NmfMatrix()
        if isinstance(V, torch.Tensor):
            # row-major rows with a leading dimension >= cols (a column slice
            # of a wider matrix is fine)
            if not V.is_cuda or V.dtype != torch.float32:
                raise TypeError("dense V must be a float32 CUDA (HIP) tensor")
            if V.dim() != 2 or (V.shape[0] > 1 and V.stride(0) < V.shape[1]) or (V.shape[1] > 1 and V.stride(1) != 1):
                raise ValueError("dense V must be 2-D with unit column stride and row stride >= its columns")
            m.kind = NMF_DENSE
            m.rows, m.cols = V.shape
            m.dense = V.data_ptr()
            m.ld = max(V.stride(0), V.shape[1]) if V.shape[0] > 1 else V.shape[1]
            self.keep.append(V)
        else:  # scipy CSR on the host, or a dict of device arrays
            import numpy as np
            csr = V
            m.kind = NMF_CSR
            m.rows, m.cols = csr.shape

            def up(a, dt):
                t = torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()
                self.keep.append(t)
                return t.data_ptr()

            m.rowptr = up(csr.indptr.astype(np.int32), torch.int32)
            m.colidx = up(csr.indices.astype(np.int32), torch.int32)
            m.vals = up(csr.data.astype(np.float32), torch.float32)
            m.nnz = csr.nnz
            if with_transpose:
                t = csr.T.tocsr()
                t.sort_indices()
                m.t_rowptr = up(t.indptr.astype(np.int32), torch.int32)
                m.t_colidx = up(t.indices.astype(np.int32), torch.int32)
                m.t_vals = up(t.data.astype(np.float32), torch.float32)
        self.m = m

    @property
    def shape(self):
        return (self.m.rows, self.m.cols)


def gram(A, l2=0.0, precision=NMF_FP32):
    torch = _torch()
    _dev(A, torch.float32, "A")
    k, r = A.shape
    G = torch.empty((r, r), dtype=torch.float32, device=A.device)
    check(lib().nmf_gram(_ptr(A), k, r, float(l2), precision, _ptr(G), stream_ptr()))
    return G


def product(V: DeviceMatrix, A, trans, precision=NMF_FP32):
    torch = _torch()
    _dev(A, torch.float32, "A")
    r = A.shape[1]
    m, n = V.shape
    P = torch.empty(((m if trans else n), r), dtype=torch.float32, device=A.device)
    check(lib().nmf_product(ctypes.byref(V.m), int(trans), r, _ptr(A), precision, _ptr(P),
                            stream_ptr()))
    return P


PROBE_GATHER_OUT_FLOATS = 2048 * 256 * 4


def probe_gather(table, idx, out=None):
    """Measurement aid (not a step of the method): reads the rows of `table`
    (2-D device tensor, rows of a multiple of 16 bytes) named by `idx` (int32
    device tensor) in that order; returns the float32 output buffer of
    running sums."""
    torch = _torch()
    if not isinstance(table, torch.Tensor) or not table.is_cuda or not table.is_contiguous() or table.dim() != 2:
        raise TypeError("table must be a contiguous 2-D CUDA (HIP) tensor")
    _dev(idx, torch.int32, "idx")
    if out is None:
        out = torch.empty(PROBE_GATHER_OUT_FLOATS, dtype=torch.float32, device=table.device)
    _dev(out, torch.float32, "out", (PROBE_GATHER_OUT_FLOATS,))
    row_bytes = table.shape[1] * table.element_size()
    check(lib().nmf_probe_gather(_ptr(table), table.shape[0], row_bytes, _ptr(idx), idx.numel(), _ptr(out),
                                 stream_ptr()))
    return out


def dense_product_time(V, A, trans, precision=NMF_FP32, nsplit=0, reps=5):
    """Measurement aid for the autotuner: ms per launch of the dense product
    with its split-K slice count forced (0: the library's choice)."""
    torch = _torch()
    _dev(V, torch.float32, "V")
    _dev(A, torch.float32, "A")
    m, n = V.shape
    ms = ctypes.c_double()
    check(lib().nmf_dense_product_time(_ptr(V), m, n, n, int(trans), A.shape[1], _ptr(A), precision, nsplit,
                                       reps, ctypes.byref(ms), stream_ptr()))
    return ms.value


def reg(l1_w=0.0, l2_w=0.0, l1_h=0.0, l2_h=0.0) -> NmfReg:
    return NmfReg(l1_w, l2_w, l1_h, l2_h)


class Plan:
    """nmf_plan_create / nmf_plan_run / nmf_plan_destroy."""

    def __init__(self, V: DeviceMatrix, r: int, regw: NmfReg, opt: NmfOpts):
        self.V = V
        self.r = r
        self.h = _vp()
        self.opt = opt
        self.regw = regw
        check(lib().nmf_plan_create(ctypes.byref(V.m), r, ctypes.byref(regw), ctypes.byref(opt),
                                    ctypes.byref(self.h), stream_ptr()))

    def run(self, W, Ht, outer, want_trace=False, want_stats=False):
        import numpy as np
        torch = _torch()
        m, n = self.V.shape
        _dev(W, torch.float32, "W", (m, self.r))
        _dev(Ht, torch.float32, "Ht", (n, self.r))
        trace = np.full(outer + 1, np.nan) if want_trace else None
        st = NmfStats() if want_stats else None
        check(lib().nmf_plan_run(self.h, _ptr(W), _ptr(Ht), int(outer),
                                 None if trace is None else trace.ctypes.data,
                                 None if st is None else ctypes.byref(st), stream_ptr()))
        return trace, (st.as_dict() if st is not None else None)

    PHASES = ("gram", "rescale", "product", "solve")

    def profile(self, enable=True):
        """True/1: events around every phase; 2: the solve kernel's own
        dispatch only (nothing added between kernels); False/0: off."""
        mode = 1 if enable is True else (0 if enable is False else int(enable))
        check(lib().nmf_plan_profile(self.h, mode))

    def timers(self):
        ms = (ctypes.c_double * 4)(); calls = (ctypes.c_int64 * 4)()
        check(lib().nmf_plan_timers(self.h, ms, calls))
        return {k: (ms[i], calls[i]) for i, k in enumerate(self.PHASES)}

    def close(self):
        if self.h:
            lib().nmf_plan_destroy(self.h)
            self.h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fit(V: DeviceMatrix, r, regw: NmfReg, opt: NmfOpts, W, Ht, want_trace=True):
    """nmf_fit on device tensors W (m, r) and Ht (n, r), updated in place."""
    import numpy as np
    torch = _torch()
    m, n = V.shape
    _dev(W, torch.float32, "W", (m, r))
    _dev(Ht, torch.float32, "Ht", (n, r))
    trace = np.full(opt.max_outer + 1, np.nan) if want_trace else None
    st = NmfStats()
    check(lib().nmf_fit(ctypes.byref(V.m), r, ctypes.byref(regw), ctypes.byref(opt), _ptr(W),
                        _ptr(Ht), None if trace is None else trace.ctypes.data, ctypes.byref(st),
                        stream_ptr()))
    return trace, st.as_dict()


def fit_single_pass(V: DeviceMatrix, r, regw: NmfReg, opt: NmfOpts, W, Ht, panel_cols, want_trace=True):
    """nmf_fit_single_pass: dense V on the device (a DeviceMatrix), W (m, r)
    and Ht (n, r) device tensors, updated in place."""
    import numpy as np
    torch = _torch()
    m, n = V.shape
    _dev(W, torch.float32, "W", (m, r))
    _dev(Ht, torch.float32, "Ht", (n, r))
    trace = np.full(opt.max_outer + 1, np.nan) if want_trace else None
    st = NmfStats()
    check(lib().nmf_fit_single_pass(ctypes.byref(V.m), r, ctypes.byref(regw), ctypes.byref(opt), int(panel_cols),
                                    _ptr(W), _ptr(Ht), None if trace is None else trace.ctypes.data,
                                    ctypes.byref(st), stream_ptr()))
    return trace, st.as_dict()


def fit_streamed(V_host, r, regw: NmfReg, opt: NmfOpts, W, Ht, panel_cols, want_trace=True):
    """nmf_fit_streamed: V_host a CPU float32 tensor (m, n) with unit column
    stride (pinned memory lets copies overlap compute); W (m, r) and Ht (n, r)
    device tensors, updated in place."""
    import numpy as np
    torch = _torch()
    if not isinstance(V_host, torch.Tensor) or V_host.is_cuda or V_host.dtype != torch.float32:
        raise TypeError("V_host must be a CPU float32 tensor")
    if V_host.dim() != 2 or V_host.stride(1) != 1:
        raise ValueError("V_host must be 2-D with unit column stride")
    m, n = V_host.shape
    _dev(W, torch.float32, "W", (m, r))
    _dev(Ht, torch.float32, "Ht", (n, r))
    trace = np.full(opt.max_outer + 1, np.nan) if want_trace else None
    st = NmfStats()
    check(lib().nmf_fit_streamed(V_host.data_ptr(), m, n, V_host.stride(0), r, ctypes.byref(regw),
                                 ctypes.byref(opt), int(panel_cols), _ptr(W), _ptr(Ht),
                                 None if trace is None else trace.ctypes.data, ctypes.byref(st),
                                 stream_ptr()))
    return trace, st.as_dict()


def objective(V: DeviceMatrix, r, regw: NmfReg, W, Ht):
    loss = ctypes.c_double(); obj = ctypes.c_double()
    check(lib().nmf_objective(ctypes.byref(V.m), r, ctypes.byref(regw), _ptr(W), _ptr(Ht),
                              ctypes.byref(loss), ctypes.byref(obj), stream_ptr()))
    return loss.value, obj.value


class Basis:
    """nmf_basis_create / nmf_foldin / nmf_basis_destroy."""

    def __init__(self, W, l1=0.0, l2=0.0, opt: NmfOpts | None = None):
        torch = _torch()
        _dev(W, torch.float32, "W")
        self.m, self.r = W.shape
        self.h = _vp()
        self.opt = opt or opts()
        check(lib().nmf_basis_create(_ptr(W), self.m, self.r, float(l1), float(l2),
                                     ctypes.byref(self.opt), ctypes.byref(self.h), stream_ptr()))

    def foldin(self, Vnew: DeviceMatrix, out=None, iters=None):
        torch = _torch()
        c = Vnew.m.cols
        if out is None:
            out = torch.empty((c, self.r), dtype=torch.float32, device="cuda")
        _dev(out, torch.float32, "Ht_new", (c, self.r))
        _dev(iters, torch.int32, "iters", (c,))
        check(lib().nmf_foldin(self.h, ctypes.byref(Vnew.m), _ptr(out), _ptr(iters),
                               stream_ptr()))
        return out

    def foldin_noalloc(self, Vnew: DeviceMatrix, out, iters=None):
        """nmf_foldin_noalloc: sparse Vnew, no device allocation by the
        library (out, and iters if given, are the caller's)."""
        torch = _torch()
        c = Vnew.m.cols
        _dev(out, torch.float32, "Ht_new", (c, self.r))
        _dev(iters, torch.int32, "iters", (c,))
        check(lib().nmf_foldin_noalloc(self.h, ctypes.byref(Vnew.m), _ptr(out), _ptr(iters),
                                       stream_ptr()))
        return out

    def close(self):
        if self.h:
            lib().nmf_basis_destroy(self.h)
            self.h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fit_batched(problems, opt: NmfOpts, want_stats=True):
    """nmf_fit_batched.  problems: list of dicts with V (device float32 m x n),
    r, reg (NmfReg), W (m x r) and Ht (n x r) device tensors, updated in place.
    Returns the per-problem statistics."""
    torch = _torch()
    arr = (NmfProblem * len(problems))()
    keep = []
    for i, pb in enumerate(problems):
        V = pb["V"]
        _dev(V, torch.float32, "V")
        m, n = V.shape
        r = pb["r"]
        _dev(pb["W"], torch.float32, "W", (m, r))
        _dev(pb["Ht"], torch.float32, "Ht", (n, r))
        d = DeviceMatrix(V)
        keep.append(d)
        arr[i].V = d.m
        arr[i].r = r
        arr[i].reg = pb["reg"]
        arr[i].W = pb["W"].data_ptr()
        arr[i].Ht = pb["Ht"].data_ptr()
    st = (NmfStats * len(problems))() if want_stats else None
    check(lib().nmf_fit_batched(len(problems), arr, ctypes.byref(opt), st, stream_ptr()))
    return [x.as_dict() for x in st] if want_stats else None


def sparse_request(csr_t, m):
    """DeviceMatrix for new columns given as CSR of their transpose (c x m):
    the t_* arrays of an m x c matrix."""
    c = csr_t.shape[0]
    d = DeviceMatrix(csr_t, with_transpose=False)
    mm = d.m
    mm.t_rowptr, mm.t_colidx, mm.t_vals = mm.rowptr, mm.colidx, mm.vals
    mm.rows, mm.cols = m, c
    return d


class Server:
    """nmf_server_*: continuously batched fold-in requests and small fits."""

    def __init__(self, basis: Basis, hbm_budget=1 << 30, max_slots=2, max_batch_cols=16384):
        self.basis = basis
        self.h = _vp()
        self.refs = {}
        check(lib().nmf_server_create(basis.h, int(hbm_budget), int(max_slots),
                                      int(max_batch_cols), ctypes.byref(self.h)))

    def _submit(self, req, refs):
        t = ctypes.c_uint64()
        check(lib().nmf_server_submit(self.h, ctypes.byref(req), ctypes.byref(t)))
        self.refs[t.value] = refs
        return t.value

    def submit_foldin(self, Vnew: DeviceMatrix, out, iters=None):
        torch = _torch()
        _dev(out, torch.float32, "out", (Vnew.m.cols, self.basis.r))
        _dev(iters, torch.int32, "iters", (Vnew.m.cols,))
        q = NmfRequest()
        q.kind = NMF_REQ_FOLDIN
        q.V = Vnew.m
        q.out = out.data_ptr()
        q.iters = _ptr(iters)
        return self._submit(q, (Vnew, out, iters))

    def submit_fit(self, V, r, regw: NmfReg, opt: NmfOpts, W, Ht):
        torch = _torch()
        d = DeviceMatrix(V)
        m, n = V.shape
        _dev(W, torch.float32, "W", (m, r))
        _dev(Ht, torch.float32, "Ht", (n, r))
        q = NmfRequest()
        q.kind = NMF_REQ_FIT
        q.V = d.m
        q.r = r
        q.reg = regw
        q.fit_opts = opt
        q.W = W.data_ptr()
        q.Ht = Ht.data_ptr()
        return self._submit(q, (d, W, Ht))

    def poll(self, ticket):
        done = ctypes.c_int32(); lat = ctypes.c_double()
        check(lib().nmf_server_poll(self.h, ticket, ctypes.byref(done), ctypes.byref(lat)))
        if done.value:
            self.refs.pop(ticket, None)
        return bool(done.value), lat.value

    def poll_times(self, ticket):
        """(done, (queued_ms, launch_ms, device_ms, latency_ms)) -- the
        request's timeline once done."""
        done = ctypes.c_int32(); t = (ctypes.c_double * 4)()
        check(lib().nmf_server_poll_times(self.h, ticket, ctypes.byref(done), t))
        if done.value:
            self.refs.pop(ticket, None)
        return bool(done.value), tuple(t)

    def wait(self, ticket=0):
        lat = ctypes.c_double()
        check(lib().nmf_server_wait(self.h, ticket, ctypes.byref(lat)))
        if ticket:
            self.refs.pop(ticket, None)
            return lat.value
        self.refs.clear()
        return None

    def stats(self):
        a = ctypes.c_int64(); b = ctypes.c_int64(); c = ctypes.c_int64()
        check(lib().nmf_server_stats(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"completed": a.value, "columns": b.value, "batches": c.value}

    def close(self):
        if self.h:
            lib().nmf_server_destroy(self.h)
            self.h = _vp()
            self.refs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
