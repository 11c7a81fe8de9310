"""ctypes binding of libccm (argument marshalling only).

Each function carries the name of the C entry point it calls (include/ccm.h)
and forwards device pointers of torch tensors plus sizes; every step of the
computation runs in the library's HIP kernels.  The library must be built
(paper_2501_15964_amd/_build.py); nothing here falls back to another
implementation when it is missing.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

__all__ = [
    "CCM_SSNAL", "CCM_ADMM", "CCM_AMA", "CCM_HPR",
    "CCM_CONVERGED", "CCM_MAX_ITER", "CCM_TIMEOUT", "CCM_NUMERICAL",
    "CcmError", "CcmOptions", "CcmStats", "lib", "library_path",
    "ccm_version", "ccm_default_options", "ccm_build_knn_graph", "ccm_solve_path",
    "ccm_canonical_edge_count", "ccm_op_gather", "ccm_op_project", "ccm_op_prox",
    "ccm_op_scatter", "ccm_op_hess_matvec", "ccm_kkt", "ccm_labels", "ccm_stream_copy",
    "ccm_path_vjp", "CCMSolve", "ccm_solve_path_batched", "CcmInstance", "EXPORTED_SYMBOLS",
    "ccm_build_knn_graph_u8", "ccm_release_workspace", "ccm_labels_noalloc",
    "ccm_weights_from_log", "CCM_OK", "CCM_E_INVALID", "CCM_E_UNSUPPORTED", "CCM_E_HIP",
    "CCM_E_NOMEM", "CCM_E_CAPACITY", "CCM_E_NOT_CONVERGED",
]

(CCM_OK, CCM_E_INVALID, CCM_E_UNSUPPORTED, CCM_E_HIP, CCM_E_NOMEM, CCM_E_CAPACITY,
 CCM_E_NOT_CONVERGED) = range(7)

CCM_SSNAL, CCM_ADMM, CCM_AMA, CCM_HPR = 0, 1, 2, 3
CCM_CONVERGED, CCM_MAX_ITER, CCM_TIMEOUT, CCM_NUMERICAL = 0, 1, 2, 3
CCM_NK = 5

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libccm.so")

EXPORTED_SYMBOLS = [
    "ccm_status_string", "ccm_last_error", "ccm_version", "ccm_default_options",
    "ccm_build_knn_graph", "ccm_solve_path", "ccm_canonical_edge_count",
    "ccm_op_gather", "ccm_op_project", "ccm_op_prox", "ccm_op_scatter",
    "ccm_op_hess_matvec", "ccm_kkt", "ccm_labels", "ccm_stream_copy", "ccm_path_vjp",
    "ccm_solve_path_batched", "ccm_build_knn_graph_u8", "ccm_release_workspace",
    "ccm_labels_noalloc", "ccm_weights_from_log",
]


class CcmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libccm status {status}: {msg}")
        self.status = status


class CcmOptions(ctypes.Structure):
    _fields_ = [
        ("method", ctypes.c_int32), ("max_outer", ctypes.c_int32),
        ("max_newton", ctypes.c_int32), ("cg_max_iter", ctypes.c_int32),
        ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("cg_chunk", ctypes.c_int32), ("profile", ctypes.c_int32),
        ("sigma0", ctypes.c_double), ("sigma_max", ctypes.c_double),
        ("tau", ctypes.c_double), ("time_budget_s", ctypes.c_double),
        ("locality", ctypes.c_int32), ("window_chunk", ctypes.c_int32),
        ("dual_scale", ctypes.c_int32),
    ]


class CcmStats(ctypes.Structure):
    _fields_ = [
        ("outer", ctypes.c_int32), ("newton", ctypes.c_int32),
        ("cg", ctypes.c_int32), ("linesearch", ctypes.c_int32),
        ("seconds", ctypes.c_double), ("f_p", ctypes.c_double), ("f_d", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("kern_ms", ctypes.c_double * CCM_NK), ("kern_calls", ctypes.c_int64 * CCM_NK),
        ("matvec_bytes", ctypes.c_double), ("matvec_launches", ctypes.c_int64),
    ]

    def as_dict(self):
        return dict(outer=self.outer, newton=self.newton, cg=self.cg,
                    linesearch=self.linesearch, seconds=self.seconds, f_p=self.f_p,
                    f_d=self.f_d, sigma=self.sigma, kern_ms=list(self.kern_ms),
                    kern_calls=list(self.kern_calls), matvec_bytes=self.matvec_bytes,
                    matvec_launches=self.matvec_launches)


class CcmInstance(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("d", ctypes.c_int64), ("m", ctypes.c_int64),
        ("a_offset", ctypes.c_int64), ("e_offset", ctypes.c_int64),
        ("x_offset", ctypes.c_int64), ("l_offset", ctypes.c_int64), ("q", ctypes.c_double),
    ]


_lib = None
P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int32
F64 = ctypes.c_double


def lib():
    """Load libccm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(library_path):
        raise RuntimeError(f"{library_path} is missing: build it with "
                           "python paper_2501_15964_amd/_build.py")
    L = ctypes.CDLL(library_path)
    L.ccm_status_string.restype = ctypes.c_char_p
    L.ccm_status_string.argtypes = [I32]
    L.ccm_last_error.restype = ctypes.c_char_p
    L.ccm_version.restype = ctypes.c_char_p
    L.ccm_default_options.restype = CcmOptions
    sigs = {
        "ccm_build_knn_graph": [P, I64, I64, I32, F64, P, P, P, I64, P, P, P],
        "ccm_solve_path": [P, I64, I64, P, P, P, I64, P, I32, F64, F64, P, P, P, P, P, P, P, P,
                           P, P, P],
        "ccm_canonical_edge_count": [P, P, P, I64, I64, P, P],
        "ccm_op_gather": [P, I64, I64, P, P, I64, P, P],
        "ccm_op_project": [P, I64, I64, P, F64, F64, P, P],
        "ccm_op_prox": [P, I64, I64, P, F64, F64, P, P],
        "ccm_op_scatter": [P, I64, I64, P, P, I64, P, P],
        "ccm_op_hess_matvec": [P, P, I64, I64, P, P, P, I64, F64, F64, F64, P, P, I32, P, P],
        "ccm_kkt": [P, P, P, I64, I64, P, P, P, I64, F64, F64, P, P],
        "ccm_labels": [P, P, I64, I64, P, P, I64, P, P, P],
        "ccm_labels_noalloc": [P, P, I64, I64, P, P, I64, P, P, P],
        "ccm_weights_from_log": [P, I64, P, P],
        "ccm_stream_copy": [P, P, I64, I32, P, P],
        "ccm_path_vjp": [P, I64, I64, P, P, P, I64, F64, F64, P, P, P, P, P, P, F64, I32, P, P],
        "ccm_solve_path_batched": [P, I32, P, P, P, P, P, I32, F64, P, P, P, P, P, P, P],
        "ccm_build_knn_graph_u8": [P, I64, I64, F64, I32, F64, P, P, P, I64, P, P, P],
        "ccm_release_workspace": [],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = I32
    _lib = L
    return L


def _check(status):
    if status != 0:
        L = lib()
        raise CcmError(status, f"{L.ccm_status_string(status).decode()}: "
                               f"{L.ccm_last_error().decode()}")


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return P(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return P(t.data_ptr())


def _f64(t):
    torch = _torch()
    if t.dtype != torch.float64:
        raise ValueError("float64 tensor expected")
    return t


def _i32(t):
    torch = _torch()
    if t.dtype != torch.int32:
        raise ValueError("int32 tensor expected")
    return t


def _graph_args(A, src, dst, w):
    """dtype and shape checks of a point set and its edge list (before any
    device call): A float64 [n, d]; src, dst int32 [m]; w float64 [m]."""
    _f64(A)
    if A.dim() != 2:
        raise ValueError("A must be a 2-D [n, d] tensor")
    _i32(src)
    _i32(dst)
    _f64(w)
    if src.dim() != 1 or dst.dim() != 1 or w.dim() != 1:
        raise ValueError("src, dst and w must be 1-D")
    if not (src.numel() == dst.numel() == w.numel()):
        raise ValueError("src, dst and w must have the same length")


def ccm_weights_from_log(log_w, stream=None):
    """w = exp(log_w) computed by the library (device float64 [m])."""
    torch = _torch()
    _f64(log_w)
    w = torch.empty_like(log_w)
    if log_w.numel():
        _check(lib().ccm_weights_from_log(_ptr(log_w.contiguous()), log_w.numel(), _ptr(w),
                                          _stream(stream)))
    return w


def ccm_version():
    return lib().ccm_version().decode()


def ccm_release_workspace():
    """Return the device memory the library keeps in reserve to the driver."""
    _check(lib().ccm_release_workspace())


def ccm_default_options(**kw):
    o = lib().ccm_default_options()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def ccm_build_knn_graph(A, k, phi=0.0, m_cap=None, stream=None):
    """k-NN Gaussian weight graph of the rows of A (device float64 [n, d]).
    Returns (src int32 [m], dst int32 [m], w float64 [m], phi)."""
    torch = _torch()
    _f64(A)
    n, d = A.shape
    m_cap = int(m_cap if m_cap is not None else n * k)
    src = torch.empty(max(m_cap, 1), dtype=torch.int32, device=A.device)
    dst = torch.empty_like(src)
    w = torch.empty(max(m_cap, 1), dtype=torch.float64, device=A.device)
    m_out = ctypes.c_int64(0)
    phi_out = ctypes.c_double(0.0)
    _check(lib().ccm_build_knn_graph(_ptr(A), n, d, int(k), float(phi), _ptr(src), _ptr(dst),
                                     _ptr(w), m_cap, ctypes.byref(m_out), ctypes.byref(phi_out),
                                     _stream(stream)))
    m = m_out.value
    return src[:m], dst[:m], w[:m], phi_out.value


def ccm_build_knn_graph_u8(K, scale, k, phi=0.0, m_cap=None, stream=None):
    """k-NN Gaussian weight graph of quantised points scale * K (K: device
    uint8 [n, d]) with exact integer distances.  Returns (src, dst, w, phi)."""
    torch = _torch()
    if K.dtype != torch.uint8:
        raise ValueError("uint8 tensor expected")
    n, d = K.shape
    m_cap = int(m_cap if m_cap is not None else n * k)
    src = torch.empty(max(m_cap, 1), dtype=torch.int32, device=K.device)
    dst = torch.empty_like(src)
    w = torch.empty(max(m_cap, 1), dtype=torch.float64, device=K.device)
    m_out = ctypes.c_int64(0)
    phi_out = ctypes.c_double(0.0)
    _check(lib().ccm_build_knn_graph_u8(_ptr(K), n, d, float(scale), int(k), float(phi),
                                        _ptr(src), _ptr(dst), _ptr(w), m_cap,
                                        ctypes.byref(m_out), ctypes.byref(phi_out),
                                        _stream(stream)))
    m = m_out.value
    return src[:m], dst[:m], w[:m], phi_out.value


def ccm_canonical_edge_count(src, dst, w, n, stream=None):
    out = ctypes.c_int64(0)
    _check(lib().ccm_canonical_edge_count(_ptr(_i32(src)), _ptr(_i32(dst)), _ptr(_f64(w)),
                                          src.numel(), int(n), ctypes.byref(out), _stream(stream)))
    return out.value


def ccm_solve_path(A, src, dst, w, gammas, q, tol, opts=None, want_U=False, want_labels=True,
                   X_warm=None, U_warm=None, stream=None):
    """Solve the clustering path.  A: device float64 [n, d]; src/dst int32
    [m]; w float64 [m]; gammas: sequence of floats; q in {1, 2, inf}.
    Returns a dict with X [T, n, d], U [T, m_canon, d] (if want_U), labels
    [T, n], n_clusters, kkt [T, 4] (R_D, R_C, R_U, eta), status, stats."""
    torch = _torch()
    _graph_args(A, src, dst, w)
    n, d = A.shape
    m = int(src.numel())
    if X_warm is not None and (_f64(X_warm).shape != (n, d)):
        raise ValueError("X_warm must be float64 [n, d]")
    if U_warm is not None and (_f64(U_warm).dim() != 2 or U_warm.shape[1] != d):
        raise ValueError("U_warm must be float64 [m_canon, d]")
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64))
    T = int(g.size)
    if U_warm is not None:
        mc = ccm_canonical_edge_count(src, dst, w, n, stream) if m else 0
        if U_warm.shape[0] != mc:
            raise ValueError(f"U_warm has {U_warm.shape[0]} rows, the canonical edges are {mc}")
    X = torch.empty((T, n, d), dtype=torch.float64, device=A.device)
    U = None
    if want_U:
        mc = ccm_canonical_edge_count(src, dst, w, n, stream) if m else 0
        U = torch.empty((T, max(mc, 1), d), dtype=torch.float64, device=A.device)[:, :mc]
    labels = torch.empty((T, n), dtype=torch.int32, device=A.device) if want_labels else None
    ncl = np.zeros(T, dtype=np.int32)
    kkt = np.zeros((T, 4), dtype=np.float64)
    status = np.zeros(T, dtype=np.int32)
    stats = (CcmStats * max(T, 1))()
    o = opts if opts is not None else lib().ccm_default_options()
    _check(lib().ccm_solve_path(
        _ptr(A), n, d, _ptr(src) if m else None, _ptr(dst) if m else None,
        _ptr(w) if m else None, m,
        g.ctypes.data_as(P), T, float(q), float(tol), ctypes.byref(o),
        _ptr(X), P(U.data_ptr()) if U is not None else None,
        _ptr(labels) if labels is not None else None,
        ncl.ctypes.data_as(P), kkt.ctypes.data_as(P), status.ctypes.data_as(P),
        ctypes.cast(stats, P), _ptr(X_warm), _ptr(U_warm), _stream(stream)))
    return dict(X=X, U=U, labels=labels, n_clusters=ncl, kkt=kkt, status=status,
                stats=[stats[t].as_dict() for t in range(T)])


def ccm_op_gather(X, src, dst, stream=None):
    torch = _torch()
    n, d = X.shape
    m = src.numel()
    Y = torch.empty((m, d), dtype=torch.float64, device=X.device)
    _check(lib().ccm_op_gather(_ptr(_f64(X)), n, d, _ptr(_i32(src)), _ptr(_i32(dst)), m,
                               _ptr(Y), _stream(stream)))
    return Y


def ccm_op_project(Y, w, gamma, q, stream=None):
    torch = _torch()
    m, d = Y.shape
    out = torch.empty_like(Y)
    _check(lib().ccm_op_project(_ptr(_f64(Y)), m, d, _ptr(_f64(w)), float(gamma), float(q),
                                _ptr(out), _stream(stream)))
    return out


def ccm_op_prox(Y, w, gamma, q, stream=None):
    torch = _torch()
    m, d = Y.shape
    out = torch.empty_like(Y)
    _check(lib().ccm_op_prox(_ptr(_f64(Y)), m, d, _ptr(_f64(w)), float(gamma), float(q),
                             _ptr(out), _stream(stream)))
    return out


def ccm_op_scatter(Z, src, dst, n, stream=None):
    torch = _torch()
    m, d = Z.shape
    out = torch.empty((n, d), dtype=torch.float64, device=Z.device)
    _check(lib().ccm_op_scatter(_ptr(_f64(Z)), m, d, _ptr(_i32(src)), _ptr(_i32(dst)), int(n),
                                _ptr(out), _stream(stream)))
    return out


def ccm_op_hess_matvec(X, U, src, dst, w, gamma, sigma, q, V, repeats=1, stream=None):
    """out = V + sigma B^T P B V at Y = U + sigma B X.  Returns (out, ms)."""
    torch = _torch()
    n, d = X.shape
    m = src.numel()
    out = torch.empty_like(V)
    ms = ctypes.c_double(0.0)
    _check(lib().ccm_op_hess_matvec(_ptr(_f64(X)), _ptr(_f64(U)), n, d, _ptr(_i32(src)),
                                    _ptr(_i32(dst)), _ptr(_f64(w)), m, float(gamma),
                                    float(sigma), float(q), _ptr(_f64(V)), _ptr(out),
                                    int(repeats), ctypes.byref(ms), _stream(stream)))
    return out, ms.value


def ccm_kkt(A, X, U, src, dst, w, gamma, q, stream=None):
    """Returns dict R_D, R_C, R_U, eta, f_p, f_d, kkt."""
    n, d = A.shape
    m = src.numel()
    out = np.zeros(7, dtype=np.float64)
    _check(lib().ccm_kkt(_ptr(_f64(A)), _ptr(_f64(X)), _ptr(_f64(U)), n, d, _ptr(_i32(src)),
                         _ptr(_i32(dst)), _ptr(_f64(w)), m, float(gamma), float(q),
                         out.ctypes.data_as(P), _stream(stream)))
    return dict(zip(["R_D", "R_C", "R_U", "eta", "f_p", "f_d", "kkt"], out.tolist()))


def ccm_labels(A, X, src, dst, stream=None):
    torch = _torch()
    n, d = A.shape
    m = src.numel()
    lab = torch.empty(n, dtype=torch.int32, device=A.device)
    nc = ctypes.c_int32(0)
    _check(lib().ccm_labels(_ptr(_f64(A)), _ptr(_f64(X)), n, d, _ptr(_i32(src)),
                            _ptr(_i32(dst)), m, _ptr(lab), ctypes.byref(nc), _stream(stream)))
    return lab, nc.value


def ccm_labels_noalloc(A, X, src, dst, labels=None, stream=None):
    """ccm_labels with the library's fixed work space (no device allocation
    inside the call); `labels` (device int32 [n]) may be given by the caller."""
    torch = _torch()
    n, d = A.shape
    m = src.numel()
    lab = labels if labels is not None else torch.empty(n, dtype=torch.int32, device=A.device)
    if lab.dtype != torch.int32 or lab.numel() != n or not lab.is_contiguous():
        raise ValueError("labels must be a contiguous int32 tensor of n values")
    nc = ctypes.c_int32(0)
    _check(lib().ccm_labels_noalloc(_ptr(_f64(A)), _ptr(_f64(X)), n, d, _ptr(_i32(src)),
                                    _ptr(_i32(dst)), m, _ptr(lab), ctypes.byref(nc),
                                    _stream(stream)))
    return lab, nc.value


def ccm_stream_copy(src, dst, nbytes, repeats=1, stream=None):
    """Device copy with the library's streaming kernel; returns ms per launch."""
    ms = ctypes.c_double(0.0)
    _check(lib().ccm_stream_copy(P(src.data_ptr()), P(dst.data_ptr()), int(nbytes), int(repeats),
                                 ctypes.byref(ms), _stream(stream)))
    return ms.value


def ccm_path_vjp(A, src, dst, w, gamma, X, labels, dLdX, tol=1e-12, max_iter=5000, q=2.0,
                 stream=None):
    """VJP of X*(A, w, gamma) at one gamma (q = 2).  Returns (dL/dA, dL/dlog w,
    dL/dgamma, CG iterations)."""
    torch = _torch()
    n, d = A.shape
    m = src.numel()
    dA = torch.empty_like(A)
    dlw = torch.empty(max(m, 1), dtype=torch.float64, device=A.device)
    dg = ctypes.c_double(0.0)
    it = ctypes.c_int32(0)
    _check(lib().ccm_path_vjp(_ptr(_f64(A)), n, d, _ptr(_i32(src)) if m else None,
                              _ptr(_i32(dst)) if m else None, _ptr(_f64(w)) if m else None, m,
                              float(gamma), float(q), _ptr(_f64(X)), _ptr(_i32(labels)),
                              _ptr(_f64(dLdX.contiguous())), _ptr(dA), _ptr(dlw),
                              ctypes.byref(dg), float(tol), int(max_iter), ctypes.byref(it),
                              _stream(stream)))
    return dA, dlw[:m], dg.value, it.value


def _make_ccm_solve():
    torch = _torch()

    class CCMSolve(torch.autograd.Function):
        """X = CCMSolve.apply(A, log_w, gamma, src, dst, tol): the minimiser of
        (CCM) at one gamma with q = 2 and weights exp(log_w) on the canonical
        edges (src, dst).  The forward pass runs ccm_solve_path to relative
        KKT <= tol; the backward pass runs ccm_path_vjp.  Gradients flow to A,
        log_w and gamma (a 0-d tensor)."""

        @staticmethod
        def forward(ctx, A, log_w, gamma, src, dst, tol=1e-11):
            w = ccm_weights_from_log(log_w.contiguous())
            g = float(gamma)
            out = ccm_solve_path(A.contiguous(), src, dst, w, [g], 2.0, tol)
            if int(out["status"][0]) != CCM_CONVERGED:
                raise CcmError(CCM_E_NOT_CONVERGED,
                               f"forward solve stopped with status {int(out['status'][0])} at "
                               f"KKT {float(np.max(out['kkt'][0][:3])):.3g} (tol {tol})")
            X = out["X"][0]
            labels = out["labels"][0]
            ctx.save_for_backward(A, w, X, labels, src, dst)
            ctx.gamma = g
            return X

        @staticmethod
        def backward(ctx, gX):
            A, w, X, labels, src, dst = ctx.saved_tensors
            dA, dlw, dg, _ = ccm_path_vjp(A, src, dst, w, ctx.gamma, X, labels, gX)
            gam = torch.tensor(dg, dtype=torch.float64, device=A.device)
            return dA, dlw, gam, None, None, None

    return CCMSolve


class _LazySolve:
    _cls = None

    def __getattr__(self, name):
        if _LazySolve._cls is None:
            _LazySolve._cls = _make_ccm_solve()
        return getattr(_LazySolve._cls, name)


CCMSolve = _LazySolve()


def ccm_solve_path_batched(instances, gammas, tol, opts=None, stream=None):
    """Solve many independent instances along the same gamma sequence.
    instances: list of dicts with device tensors A (n x d float64), src, dst
    (int32, canonical, local endpoints), w (float64) and a float q.  Returns a
    list of dicts (one per instance) with X [T, n, d], labels [T, n],
    n_clusters [T], kkt [T, 4], status [T]."""
    torch = _torch()
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64))
    T = int(g.size)
    N = len(instances)
    desc = (CcmInstance * max(N, 1))()
    a_off = e_off = x_off = l_off = 0
    for inst in instances:
        _graph_args(inst["A"], inst["src"], inst["dst"], inst["w"])
    for i, inst in enumerate(instances):
        n, d = inst["A"].shape
        m = int(inst["src"].numel())
        desc[i] = CcmInstance(n, d, m, a_off, e_off, x_off, l_off, float(inst["q"]))
        a_off += n * d
        e_off += m
        x_off += T * n * d
        l_off += T * n
    dev = instances[0]["A"].device
    A_all = torch.cat([inst["A"].reshape(-1) for inst in instances]).contiguous()
    if e_off:
        src_all = torch.cat([inst["src"] for inst in instances]).contiguous()
        dst_all = torch.cat([inst["dst"] for inst in instances]).contiguous()
        w_all = torch.cat([inst["w"] for inst in instances]).contiguous()
    else:
        src_all = dst_all = torch.zeros(1, dtype=torch.int32, device=dev)
        w_all = torch.zeros(1, dtype=torch.float64, device=dev)
    X_all = torch.empty(max(x_off, 1), dtype=torch.float64, device=dev)
    L_all = torch.empty(max(l_off, 1), dtype=torch.int32, device=dev)
    ncl = np.zeros(N * T, dtype=np.int32)
    kkt = np.zeros(N * T * 4, dtype=np.float64)
    st = np.zeros(N * T, dtype=np.int32)
    o = opts if opts is not None else lib().ccm_default_options()
    _check(lib().ccm_solve_path_batched(
        ctypes.cast(desc, P), N, _ptr(A_all), _ptr(src_all), _ptr(dst_all), _ptr(w_all),
        g.ctypes.data_as(P), T, float(tol), ctypes.byref(o), _ptr(X_all), _ptr(L_all),
        ncl.ctypes.data_as(P), kkt.ctypes.data_as(P), st.ctypes.data_as(P), _stream(stream)))
    out = []
    for i, inst in enumerate(instances):
        n, d = inst["A"].shape
        D = desc[i]
        out.append(dict(
            X=X_all[D.x_offset:D.x_offset + T * n * d].view(T, n, d),
            labels=L_all[D.l_offset:D.l_offset + T * n].view(T, n),
            n_clusters=ncl[i * T:(i + 1) * T].copy(),
            kkt=kkt[i * T * 4:(i + 1) * T * 4].reshape(T, 4).copy(),
            status=st[i * T:(i + 1) * T].copy()))
    return out
