"""ctypes binding of libcoxmi.so, the C ABI declared in include/coxmi.h.

Argument marshalling only: every step of the path runs in the HIP library.
Function names match the C entry points.  Errors raise CoxError carrying the
status code and the library's message.  If the library has not been built the
first call raises RuntimeError; there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

COX_OK = 0
COX_NOT_CONVERGED = 1
COX_EINVAL = -1
COX_ENOMEM = -2
COX_EDEVICE = -3
COX_ENUMERIC = -4
COX_EUNSUPPORTED = -5

COX_CCD = 0
COX_NEWTON_REFINE = 1
COX_F64 = 0
COX_F32 = 1
COX_BF16 = 2
COX_FP8_E4M3 = 3
COX_BRESLOW = 0
COX_EFRON = 1

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcoxmi.so")


class CoxError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"[{code}] {message}")
        self.code = code
        self.message = message


class cox_data(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("p", ctypes.c_int64),
                ("x", ctypes.POINTER(ctypes.c_double)), ("ldx", ctypes.c_int64),
                ("time", ctypes.POINTER(ctypes.c_double)),
                ("event", ctypes.POINTER(ctypes.c_uint8)),
                ("stratum", ctypes.POINTER(ctypes.c_int32)), ("on_device", ctypes.c_int)]


class cox_intervals(ctypes.Structure):
    _fields_ = [("data", cox_data), ("intervals", ctypes.c_int),
                ("row_subject", ctypes.POINTER(ctypes.c_int64)), ("row_interval", ctypes.POINTER(ctypes.c_int32)),
                ("col_source", ctypes.POINTER(ctypes.c_int32)), ("col_interval", ctypes.POINTER(ctypes.c_int32))]


class cox_options(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("penalize", ctypes.POINTER(ctypes.c_uint8)),
                ("mode", ctypes.c_int), ("x_precision", ctypes.c_int), ("ties", ctypes.c_int),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("stream", ctypes.c_void_p)]


class cox_fit_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("coord_evals", ctypes.c_int64),
                ("objective", ctypes.c_double), ("kkt_inf", ctypes.c_double),
                ("last_step", ctypes.c_double), ("n_pinned", ctypes.c_int), ("fallback", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class cox_profile(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double), ("evaluations", ctypes.c_int), ("evaluation_ms", ctypes.c_double),
                ("contractions", ctypes.c_int), ("contraction_ms", ctypes.c_double), ("solves", ctypes.c_int),
                ("solve_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class cox_server_options(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("staging_bytes", ctypes.c_size_t),
                ("max_resident", ctypes.c_int), ("prep_threads", ctypes.c_int),
                ("x_precision", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("device", ctypes.c_int), ("fused_rounds", ctypes.c_int)]


class cox_request_times(ctypes.Structure):
    _fields_ = [("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class cox_fit_request(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("penalize", ctypes.POINTER(ctypes.c_uint8)),
                ("beta0", ctypes.POINTER(ctypes.c_double))]


class cox_server_counters(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("iterations", ctypes.c_int64),
                ("resident_now", ctypes.c_int64), ("resident_peak", ctypes.c_int64),
                ("mean_resident", ctypes.c_double), ("arena_bytes", ctypes.c_size_t),
                ("arena_peak", ctypes.c_size_t), ("gpu_busy_s", ctypes.c_double), ("now_s", ctypes.c_double),
                ("launches", ctypes.c_int64), ("phase_s", ctypes.c_double * 6)]

    def as_dict(self) -> dict:
        return {k: (list(getattr(self, k)) if k == "phase_s" else getattr(self, k)) for k, _ in self._fields_}


COX_SUBMIT_BORROW = 1
COX_SUBMIT_DEVICE = 2

_lib = None

# Handles and servers still open when the interpreter exits are released before its
# teardown starts, while the HIP runtime is whole (a release from a finalizer during
# teardown can run after the runtime's own exit handlers).
_live = weakref.WeakSet()


@atexit.register
def _release_all():
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass

# (name, restype, argtypes) of every entry point in include/coxmi.h
_VP = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
SIGNATURES = [
    ("cox_default_options", None, [ctypes.POINTER(cox_options)]),
    ("cox_init", ctypes.c_int, [ctypes.POINTER(_VP), ctypes.POINTER(cox_data), ctypes.POINTER(cox_options)]),
    ("cox_fit", ctypes.c_int, [_VP, _DP, _DP, ctypes.POINTER(cox_fit_info)]),
    ("cox_evaluate", ctypes.c_int, [_VP, _DP, _DP, _DP, _DP]),
    ("cox_evaluate_full", ctypes.c_int, [_VP, _DP, _DP, _DP, _DP, _DP]),
    ("cox_coordinate", ctypes.c_int, [_VP, _DP, ctypes.c_int64, _DP]),
    ("cox_layout", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint32)]),
    ("cox_split_intervals", ctypes.c_int, [ctypes.POINTER(cox_data), ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.POINTER(cox_intervals))]),
    ("cox_intervals_release", None, [ctypes.POINTER(cox_intervals)]),
    ("cox_baseline_hazard", ctypes.c_int, [_VP, _DP, _DP]),
    ("cox_init_indicator", ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int64, ctypes.c_int64,
                                          ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32), _DP,
                                          ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(cox_options)]),
    ("cox_init_sparse", ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int64, ctypes.c_int64,
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32), _DP, _DP,
                                       ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(cox_options)]),
    ("cox_init_resample", ctypes.c_int, [ctypes.POINTER(_VP), _VP, ctypes.POINTER(ctypes.c_uint32),
                                         ctypes.POINTER(cox_options)]),
    ("cox_init_intervals", ctypes.c_int, [ctypes.POINTER(_VP), _VP, _DP, ctypes.POINTER(ctypes.c_uint8),
                                          ctypes.POINTER(ctypes.c_int32), ctypes.c_int, _DP,
                                          ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(cox_options)]),
    ("cox_set_penalty", ctypes.c_int, [_VP, ctypes.c_double, ctypes.POINTER(ctypes.c_uint8)]),
    ("cox_cross_validate", ctypes.c_int, [_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_int32), ctypes.c_int, _DP,
                                          ctypes.POINTER(ctypes.c_uint8), _DP, _DP, ctypes.POINTER(ctypes.c_int)]),
    ("cox_cross_validate_served", ctypes.c_int, [_VP, _VP, ctypes.POINTER(cox_data), ctypes.c_int,
                                                 ctypes.POINTER(ctypes.c_int32), ctypes.c_int, _DP,
                                                 ctypes.POINTER(ctypes.c_uint8), _DP, _DP, ctypes.POINTER(ctypes.c_int)]),
    ("cox_bootstrap", ctypes.c_int, [_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_uint32), _DP, _DP,
                                     ctypes.POINTER(ctypes.c_int)]),
    ("cox_canonical_order", ctypes.c_int, [ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint32)]),
    ("cox_last_kernel_ms", ctypes.c_int, [_VP, _DP]),
    ("cox_last_profile", ctypes.c_int, [_VP, ctypes.POINTER(cox_profile)]),
    ("cox_shape", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int64)]),
    ("cox_segscan_f64", ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, _VP]),
    ("cox_segscan_f64_noalloc", ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, _VP]),
    ("cox_release", None, [_VP]),
    ("cox_last_error", ctypes.c_char_p, [_VP]),
    ("cox_server_default_options", None, [ctypes.POINTER(cox_server_options)]),
    ("cox_server_create", ctypes.c_int, [ctypes.POINTER(_VP), ctypes.POINTER(cox_server_options)]),
    ("cox_server_submit", ctypes.c_int, [_VP, ctypes.POINTER(cox_data), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_uint64)]),
    ("cox_server_submit_fit", ctypes.c_int, [_VP, ctypes.POINTER(cox_data), ctypes.c_int,
                                             ctypes.POINTER(cox_fit_request), ctypes.POINTER(ctypes.c_uint64)]),
    ("cox_server_poll", ctypes.c_int, [_VP, ctypes.c_uint64, _DP, ctypes.POINTER(cox_fit_info),
                                       ctypes.POINTER(cox_request_times)]),
    ("cox_server_wait", ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.c_double]),
    ("cox_server_drain", ctypes.c_int, [_VP, ctypes.c_double]),
    ("cox_server_stats", ctypes.c_int, [_VP, ctypes.POINTER(cox_server_counters)]),
    ("cox_server_last_error", ctypes.c_char_p, [_VP]),
    ("cox_server_destroy", None, [_VP]),
]


def lib():
    """Load libcoxmi.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(_DP)


def _check(h, rc, ok=(COX_OK,)):
    if rc not in ok:
        msg = lib().cox_last_error(h)
        raise CoxError(rc, msg.decode() if msg else "")
    return rc


def cox_default_options() -> cox_options:
    o = cox_options()
    lib().cox_default_options(ctypes.byref(o))
    return o


def cox_init(X, time, event, stratum=None, *, gamma=0.0, penalize=None, tol=1e-12, max_iter=1000,
             stream=None, mode=COX_CCD, x_precision=COX_F64, ties=COX_BRESLOW):
    """Create a handle.  X: (n, p) float64 (any order), time float64[n], event 0/1[n],
    stratum int32[n] or None.  Returns an opaque handle (int)."""
    X = np.asfortranarray(X, dtype=np.float64)
    n, p = X.shape
    time = np.ascontiguousarray(time, dtype=np.float64)
    event = np.ascontiguousarray(event, dtype=np.uint8)
    d = cox_data(n=n, p=p, x=_dptr(X), ldx=n, time=_dptr(time),
                 event=event.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    keep = [X, time, event]
    if stratum is not None:
        st = np.ascontiguousarray(stratum, dtype=np.int32)
        keep.append(st)
        d.stratum = st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    o = cox_default_options()
    o.gamma = float(gamma)
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.mode = int(mode)
    o.x_precision = int(x_precision)
    o.ties = int(ties)
    if penalize is not None:
        pen = np.ascontiguousarray(penalize, dtype=np.uint8)
        keep.append(pen)
        o.penalize = pen.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    if stream is not None:
        o.stream = ctypes.c_void_p(int(stream))
    h = ctypes.c_void_p()
    rc = lib().cox_init(ctypes.byref(h), ctypes.byref(d), ctypes.byref(o))
    _check(None, rc)
    return h.value


def _device_data(X, time, event, stratum):
    """cox_data over device-resident torch tensors (checked here for shape and dtype only;
    the library checks that every array lies in device memory)."""
    import torch
    n, p = X.shape
    if X.dtype != torch.float64 or not X.is_cuda or X.stride(0) != 1 or X.stride(1) < n:
        raise ValueError("X must be a float64 CUDA tensor with unit row stride (column-major)")
    checks = [(time, torch.float64), (event, torch.uint8)] + ([(stratum, torch.int32)] if stratum is not None else [])
    for t, dt in checks:
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
            raise ValueError("time / event / stratum must be contiguous CUDA tensors of n float64 / uint8 / int32")
    d = cox_data(n=n, p=p, x=ctypes.cast(X.data_ptr(), _DP), ldx=X.stride(1),
                 time=ctypes.cast(time.data_ptr(), _DP),
                 event=ctypes.cast(event.data_ptr(), ctypes.POINTER(ctypes.c_uint8)), on_device=1)
    if stratum is not None:
        d.stratum = ctypes.cast(stratum.data_ptr(), ctypes.POINTER(ctypes.c_int32))
    return d


def cox_init_device(X, time, event, stratum=None, *, gamma=0.0, penalize=None, tol=1e-12, max_iter=1000,
                    stream=None, mode=COX_CCD, x_precision=COX_F64, ties=COX_BRESLOW):
    """cox_init on device-resident data: X a float64 CUDA tensor with unit row stride
    (column-major, e.g. the transpose of a contiguous p x n tensor), time float64, event
    uint8, stratum int32 or None (contiguous CUDA tensors).  The library reads them after
    the work queued on `stream` (default: the default stream); order other producers first."""
    d = _device_data(X, time, event, stratum)
    keep = []
    o = _options(gamma, penalize, tol, max_iter, stream, mode, x_precision, keep, ties)
    h = ctypes.c_void_p()
    rc = lib().cox_init(ctypes.byref(h), ctypes.byref(d), ctypes.byref(o))
    _check(None, rc)
    return h.value


def _options(gamma, penalize, tol, max_iter, stream, mode, x_precision, keep, ties=COX_BRESLOW):
    o = cox_default_options()
    o.gamma = float(gamma)
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.mode = int(mode)
    o.x_precision = int(x_precision)
    o.ties = int(ties)
    if penalize is not None:
        pen = np.ascontiguousarray(penalize, dtype=np.uint8)
        keep.append(pen)
        o.penalize = pen.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    if stream is not None:
        o.stream = ctypes.c_void_p(int(stream))
    return o


def cox_baseline_hazard(h, beta):
    """Breslow cumulative baseline hazard at each row's time, in its stratum (cox_baseline_hazard)."""
    n, _, _ = cox_shape(h)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    out = np.zeros(n)
    _check(h, lib().cox_baseline_hazard(h, _dptr(b), _dptr(out)))
    return out


def cox_init_indicator(n, col_ptr, row_idx, time, event, stratum=None, *, gamma=0.0, penalize=None, tol=1e-12,
                       max_iter=1000, stream=None, ties=COX_BRESLOW):
    """A handle on indicator X given as compressed sparse columns: column j holds 1 at rows
    row_idx[col_ptr[j]:col_ptr[j + 1]] and 0 elsewhere (cox_init_indicator)."""
    cp = np.ascontiguousarray(col_ptr, dtype=np.int64)
    ri = np.ascontiguousarray(row_idx, dtype=np.int32)
    p = cp.shape[0] - 1
    time = np.ascontiguousarray(time, dtype=np.float64)
    event = np.ascontiguousarray(event, dtype=np.uint8)
    if time.shape != (n,) or event.shape != (n,):
        raise ValueError(f"time and event need {n} entries")
    keep = [cp, ri, time, event]
    st = None
    if stratum is not None:
        st = np.ascontiguousarray(stratum, dtype=np.int32)
        keep.append(st)
    o = _options(gamma, penalize, tol, max_iter, stream, COX_CCD, COX_F64, keep, ties)
    h = ctypes.c_void_p()
    rc = lib().cox_init_indicator(ctypes.byref(h), int(n), int(p), cp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  ri.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dptr(time),
                                  event.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                  None if st is None else st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  ctypes.byref(o))
    _check(None, rc)
    return h.value


def cox_init_sparse(n, col_ptr, row_idx, values, time, event, stratum=None, *, gamma=0.0, penalize=None,
                    tol=1e-12, max_iter=1000, stream=None, ties=COX_BRESLOW):
    """A handle on sparse X given as compressed sparse columns with values: column j holds
    values[col_ptr[j]:col_ptr[j + 1]] at rows row_idx[col_ptr[j]:col_ptr[j + 1]] and 0
    elsewhere (cox_init_sparse)."""
    cp = np.ascontiguousarray(col_ptr, dtype=np.int64)
    ri = np.ascontiguousarray(row_idx, dtype=np.int32)
    va = np.ascontiguousarray(values, dtype=np.float64)
    p = cp.shape[0] - 1
    if ri.shape != va.shape:
        raise ValueError("row_idx and values need the same length")
    time = np.ascontiguousarray(time, dtype=np.float64)
    event = np.ascontiguousarray(event, dtype=np.uint8)
    if time.shape != (n,) or event.shape != (n,):
        raise ValueError(f"time and event need {n} entries")
    keep = [cp, ri, va, time, event]
    st = None
    if stratum is not None:
        st = np.ascontiguousarray(stratum, dtype=np.int32)
        keep.append(st)
    o = _options(gamma, penalize, tol, max_iter, stream, COX_CCD, COX_F64, keep, ties)
    h = ctypes.c_void_p()
    rc = lib().cox_init_sparse(ctypes.byref(h), int(n), int(p), cp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               ri.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dptr(va), _dptr(time),
                               event.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                               None if st is None else st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               ctypes.byref(o))
    _check(None, rc)
    return h.value


def cox_init_resample(parent, count, *, inherit=True, gamma=0.0, penalize=None, tol=1e-12, max_iter=1000,
                      stream=None, mode=COX_CCD, x_precision=COX_F64, ties=COX_BRESLOW):
    """A handle on the data set in which row i of the parent's data appears count[i] times,
    gathered on the device from the parent's X.  inherit=True keeps the parent's options
    and l1 weights (the keyword options are then ignored)."""
    n, _, _ = cox_shape(parent)
    cnt = np.ascontiguousarray(count, dtype=np.uint32)
    if cnt.shape != (n,):
        raise ValueError(f"count needs {n} entries")
    keep = [cnt]
    o = None if inherit else _options(gamma, penalize, tol, max_iter, stream, mode, x_precision, keep, ties)
    h = ctypes.c_void_p()
    rc = lib().cox_init_resample(ctypes.byref(h), parent, cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                 None if o is None else ctypes.byref(o))
    _check(None, rc)
    return h.value


def cox_init_intervals(parent, time, event, stratum=None, cuts=(), tv_coef=None, *, inherit=True, gamma=0.0,
                       penalize=None, tol=1e-12, max_iter=1000, stream=None, mode=COX_CCD, x_precision=COX_F64,
                       ties=COX_BRESLOW):
    """The interval-stratified model (cox_init_intervals) built on the device from the parent's
    X; time, event, stratum are the data the parent was built from."""
    n, p, _ = cox_shape(parent)
    time = np.ascontiguousarray(time, dtype=np.float64)
    event = np.ascontiguousarray(event, dtype=np.uint8)
    if time.shape != (n,) or event.shape != (n,):
        raise ValueError(f"time and event need {n} entries")
    keep = [time, event]
    st = None
    if stratum is not None:
        st = np.ascontiguousarray(stratum, dtype=np.int32)
        keep.append(st)
    cuts = np.ascontiguousarray(cuts, dtype=np.float64)
    tv = None
    if tv_coef is not None:
        tv = np.ascontiguousarray(tv_coef, dtype=np.uint8)
        if tv.shape != (p,):
            raise ValueError(f"tv_coef needs {p} entries")
    o = None if inherit else _options(gamma, penalize, tol, max_iter, stream, mode, x_precision, keep, ties)
    h = ctypes.c_void_p()
    rc = lib().cox_init_intervals(ctypes.byref(h), parent, _dptr(time),
                                  event.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                  None if st is None else st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  cuts.shape[0], _dptr(cuts) if cuts.shape[0] else None,
                                  None if tv is None else tv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                  None if o is None else ctypes.byref(o))
    _check(None, rc)
    return h.value


def cox_set_penalty(h, gamma, penalize=None):
    pen = None if penalize is None else np.ascontiguousarray(penalize, dtype=np.uint8)
    rc = lib().cox_set_penalty(h, float(gamma), None if pen is None else pen.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    _check(h, rc)


def cox_cross_validate(h, fold, gammas, penalize=None, nfolds=None):
    """Cross-validated log partial likelihood along `gammas` (cox_cross_validate).
    Returns (cvl[ngamma], betas[nfolds, ngamma, p], status[nfolds, ngamma])."""
    n, p, _ = cox_shape(h)
    fold = np.ascontiguousarray(fold, dtype=np.int32)
    if fold.shape != (n,):
        raise ValueError(f"fold needs {n} entries")
    K = int(fold.max()) + 1 if nfolds is None else int(nfolds)
    gam = np.ascontiguousarray(gammas, dtype=np.float64)
    pen = None if penalize is None else np.ascontiguousarray(penalize, dtype=np.uint8)
    cvl = np.zeros(gam.shape[0])
    betas = np.zeros((K, gam.shape[0], p))
    status = np.zeros((K, gam.shape[0]), dtype=np.int32)
    rc = lib().cox_cross_validate(h, K, fold.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), gam.shape[0], _dptr(gam),
                                  None if pen is None else pen.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                  _dptr(cvl), _dptr(betas), status.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    _check(h, rc, ok=(COX_OK, COX_NOT_CONVERGED))
    return cvl, betas, status


def cox_cross_validate_served(h, server, X, time, event, stratum, fold, gammas, penalize=None, nfolds=None):
    """cox_cross_validate with the fold fits batched through `server` (a CoxServer); X, time,
    event, stratum: the host data h was made from (cox_cross_validate_served)."""
    n, p, _ = cox_shape(h)
    X = np.asfortranarray(X, dtype=np.float64)
    time = np.ascontiguousarray(time, dtype=np.float64)
    event = np.ascontiguousarray(event, dtype=np.uint8)
    d = cox_data(n=X.shape[0], p=X.shape[1], x=_dptr(X), ldx=X.shape[0], time=_dptr(time),
                 event=event.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    st = None
    if stratum is not None:
        st = np.ascontiguousarray(stratum, dtype=np.int32)
        d.stratum = st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    fold = np.ascontiguousarray(fold, dtype=np.int32)
    if fold.shape != (n,):
        raise ValueError(f"fold needs {n} entries")
    K = int(fold.max()) + 1 if nfolds is None else int(nfolds)
    gam = np.ascontiguousarray(gammas, dtype=np.float64)
    pen = None if penalize is None else np.ascontiguousarray(penalize, dtype=np.uint8)
    cvl = np.zeros(gam.shape[0])
    betas = np.zeros((K, gam.shape[0], p))
    status = np.zeros((K, gam.shape[0]), dtype=np.int32)
    rc = lib().cox_cross_validate_served(h, server.h, ctypes.byref(d), K,
                                         fold.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), gam.shape[0],
                                         _dptr(gam), None if pen is None else pen.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                         _dptr(cvl), _dptr(betas), status.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    _check(h, rc, ok=(COX_OK, COX_NOT_CONVERGED))
    return cvl, betas, status


def cox_bootstrap(h, counts, beta0=None):
    """Refits on the row multiplicities counts[b] (cox_bootstrap).  Returns (betas[B, p], status[B])."""
    n, p, _ = cox_shape(h)
    cnt = np.ascontiguousarray(counts, dtype=np.uint32)
    if cnt.ndim != 2 or cnt.shape[1] != n:
        raise ValueError(f"counts needs shape (B, {n})")
    B = cnt.shape[0]
    b0 = None if beta0 is None else np.ascontiguousarray(beta0, dtype=np.float64)
    betas = np.zeros((B, p))
    status = np.zeros(B, dtype=np.int32)
    rc = lib().cox_bootstrap(h, B, cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                             None if b0 is None else _dptr(b0), _dptr(betas),
                             status.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    _check(h, rc, ok=(COX_OK, COX_NOT_CONVERGED))
    return betas, status


def cox_fit(h, beta0=None, p=None):
    """Returns (beta, info_dict).  Raises CoxError unless the status is OK or NOT_CONVERGED."""
    n_, p_, _ = cox_shape(h)
    beta = np.zeros(p_)
    b0 = None if beta0 is None else np.ascontiguousarray(beta0, dtype=np.float64)
    info = cox_fit_info()
    rc = lib().cox_fit(h, None if b0 is None else _dptr(b0), _dptr(beta), ctypes.byref(info))
    _check(h, rc, ok=(COX_OK, COX_NOT_CONVERGED))
    return beta, info.as_dict()


def cox_evaluate(h, beta):
    """Returns (objective, grad[p], hess_diag[p])."""
    b = np.ascontiguousarray(beta, dtype=np.float64)
    g = np.zeros(b.shape[0])
    hd = np.zeros(b.shape[0])
    obj = ctypes.c_double()
    _check(h, lib().cox_evaluate(h, _dptr(b), ctypes.byref(obj), _dptr(g), _dptr(hd)))
    return obj.value, g, hd


def cox_evaluate_full(h, beta, want_info=True):
    """Returns (objective, grad[p], hess_diag[p], info[p, p] or None)."""
    b = np.ascontiguousarray(beta, dtype=np.float64)
    p = b.shape[0]
    g = np.zeros(p)
    hd = np.zeros(p)
    info = np.zeros((p, p)) if want_info else None
    obj = ctypes.c_double()
    _check(h, lib().cox_evaluate_full(h, _dptr(b), ctypes.byref(obj), _dptr(g), _dptr(hd),
                                      None if info is None else _dptr(info)))
    return obj.value, g, hd, info


def cox_coordinate(h, beta, j):
    """Returns [g', g'', -log L, delta'(S[N2]/S[D])] for column j at beta."""
    b = np.ascontiguousarray(beta, dtype=np.float64)
    out = np.zeros(4)
    _check(h, lib().cox_coordinate(h, _dptr(b), int(j), _dptr(out)))
    return out


def cox_layout(h):
    n, _, _ = cox_shape(h)
    perm = np.zeros(n, dtype=np.int64)
    meta = np.zeros(n, dtype=np.uint32)
    _check(h, lib().cox_layout(h, perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               meta.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
    return perm, meta


def cox_canonical_order(time, event, stratum=None):
    """Host canonical order (no device): (perm int64[n], meta uint32[n])."""
    time = np.ascontiguousarray(time, dtype=np.float64)
    event = np.ascontiguousarray(event, dtype=np.uint8)
    n = time.shape[0]
    st = None if stratum is None else np.ascontiguousarray(stratum, dtype=np.int32)
    perm = np.zeros(n, dtype=np.int64)
    meta = np.zeros(n, dtype=np.uint32)
    rc = lib().cox_canonical_order(n, _dptr(time), event.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                   None if st is None else st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   meta.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    if rc != COX_OK:
        raise CoxError(rc, "cox_canonical_order")
    return perm, meta


def split_intervals(X, time, event, stratum=None, cuts=(), tv_coef=None, X_by_interval=None):
    """Secs. 2.2-2.3 augmentation (cox_split_intervals): returns a dict with the augmented
    X (n_aug, p_aug, column-major), time, event, stratum, and the maps row_subject,
    row_interval, col_source, col_interval.  The arrays are views of the library's result,
    which is released once none of them is referenced."""
    X = np.asfortranarray(X, dtype=np.float64)
    n, p = X.shape
    time = np.ascontiguousarray(time, dtype=np.float64)
    event = np.ascontiguousarray(event, dtype=np.uint8)
    d = cox_data(n=n, p=p, x=_dptr(X), ldx=n, time=_dptr(time),
                 event=event.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    keep = [X, time, event]
    if stratum is not None:
        st = np.ascontiguousarray(stratum, dtype=np.int32)
        keep.append(st)
        d.stratum = st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    cuts = np.ascontiguousarray(cuts, dtype=np.float64)
    tv = None if tv_coef is None else np.ascontiguousarray(tv_coef, dtype=np.uint8)
    xk = None
    if X_by_interval is not None:
        xk = np.ascontiguousarray(np.stack([np.asfortranarray(b, dtype=np.float64).T for b in X_by_interval]))
        if xk.shape != (len(cuts) + 1, p, n):
            raise ValueError("X_by_interval needs one n x p block per interval")
    out = ctypes.POINTER(cox_intervals)()
    rc = lib().cox_split_intervals(ctypes.byref(d), len(cuts), _dptr(cuts) if len(cuts) else None,
                                   None if tv is None else tv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                   None if xk is None else _dptr(xk), ctypes.byref(out))
    if rc != COX_OK:
        raise CoxError(rc, "cox_split_intervals")
    owner = _IntervalsOwner(out)
    r = out.contents
    na, pa = r.data.n, r.data.p
    return {
        "X": owner.view(r.data.x, ctypes.c_double, pa * na).reshape(pa, na).T,
        "time": owner.view(r.data.time, ctypes.c_double, na),
        "event": owner.view(r.data.event, ctypes.c_uint8, na),
        "stratum": owner.view(r.data.stratum, ctypes.c_int32, na),
        "row_subject": owner.view(r.row_subject, ctypes.c_int64, na),
        "row_interval": owner.view(r.row_interval, ctypes.c_int32, na),
        "col_source": owner.view(r.col_source, ctypes.c_int32, pa),
        "col_interval": owner.view(r.col_interval, ctypes.c_int32, pa),
        "intervals": int(r.intervals),
    }


class _IntervalsOwner:
    """Holds a cox_intervals result; the numpy views made by view() keep it alive, and it is
    released (cox_intervals_release) when the last of them goes."""

    def __init__(self, ptr):
        self.ptr = ptr
        self.lib = lib()   # held, so that the release works during interpreter shutdown too

    def view(self, p, ctype, count):
        buf = (ctype * count).from_address(ctypes.cast(p, ctypes.c_void_p).value)
        buf._owner = self
        return np.frombuffer(buf, dtype=np.dtype(ctype))

    def __del__(self):
        if self.ptr:
            self.lib.cox_intervals_release(self.ptr)
        self.ptr = None


def cox_shape(h):
    n, p, ld = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(h, lib().cox_shape(h, ctypes.byref(n), ctypes.byref(p), ctypes.byref(ld)))
    return n.value, p.value, ld.value


def cox_last_kernel_ms(h) -> float:
    ms = ctypes.c_double()
    _check(h, lib().cox_last_kernel_ms(h, ctypes.byref(ms)))
    return ms.value


def cox_last_profile(h) -> dict:
    prof = cox_profile()
    _check(h, lib().cox_last_profile(h, ctypes.byref(prof)))
    return prof.as_dict()


def cox_segscan_f64(a_ptr: int, head_ptr: int, b_ptr: int, n: int, stream=None) -> int:
    """Device-pointer segmented scan; returns the status code (raises on error)."""
    rc = lib().cox_segscan_f64(ctypes.c_void_p(a_ptr), ctypes.c_void_p(head_ptr), ctypes.c_void_p(b_ptr),
                               int(n), None if stream is None else ctypes.c_void_p(int(stream)))
    if rc != COX_OK:
        raise CoxError(rc, "cox_segscan_f64 failed")
    return rc


def cox_segscan_f64_noalloc(a_ptr: int, head_ptr: int, b_ptr: int, n: int, stream=None) -> int:
    """cox_segscan_f64 without device allocation (library-owned scratch); raises on error."""
    rc = lib().cox_segscan_f64_noalloc(ctypes.c_void_p(a_ptr), ctypes.c_void_p(head_ptr), ctypes.c_void_p(b_ptr),
                                       int(n), None if stream is None else ctypes.c_void_p(int(stream)))
    if rc != COX_OK:
        raise CoxError(rc, "cox_segscan_f64_noalloc failed")
    return rc


def cox_release(h) -> None:
    if h:
        lib().cox_release(h)


def cox_last_error(h=None) -> str:
    m = lib().cox_last_error(h)
    return m.decode() if m else ""


class CoxModel:
    """Owns one handle; a thin convenience over the functions above."""

    def __init__(self, X, time, event, stratum=None, **opts):
        self.h = cox_init(X, time, event, stratum, **opts)
        _live.add(self)

    @classmethod
    def from_device(cls, X, time, event, stratum=None, **opts):
        """A CoxModel on device-resident torch tensors (see cox_init_device)."""
        m = cls.__new__(cls)
        m.h = cox_init_device(X, time, event, stratum, **opts)
        _live.add(m)
        return m

    @classmethod
    def sparse(cls, n, col_ptr, row_idx, values, time, event, stratum=None, **opts):
        """A CoxModel on sparse X in compressed sparse columns with values (see cox_init_sparse)."""
        m = cls.__new__(cls)
        m.h = cox_init_sparse(n, col_ptr, row_idx, values, time, event, stratum, **opts)
        _live.add(m)
        return m

    @classmethod
    def indicator(cls, n, col_ptr, row_idx, time, event, stratum=None, **opts):
        """A CoxModel on indicator X in compressed sparse columns (see cox_init_indicator)."""
        m = cls.__new__(cls)
        m.h = cox_init_indicator(n, col_ptr, row_idx, time, event, stratum, **opts)
        _live.add(m)
        return m

    def fit(self, beta0=None):
        return cox_fit(self.h, beta0)

    def evaluate(self, beta):
        return cox_evaluate(self.h, beta)

    def coordinate(self, beta, j):
        return cox_coordinate(self.h, beta, j)

    def evaluate_full(self, beta, want_info=True):
        return cox_evaluate_full(self.h, beta, want_info)

    def layout(self):
        return cox_layout(self.h)

    def resample(self, count, **opts):
        """A CoxModel on the data set with row multiplicities `count` (see cox_init_resample)."""
        m = CoxModel.__new__(CoxModel)
        m.h = cox_init_resample(self.h, count, inherit=not opts, **opts)
        _live.add(m)
        return m

    def intervals(self, time, event, stratum=None, cuts=(), tv_coef=None, **opts):
        """A CoxModel on the interval-stratified data (see cox_init_intervals)."""
        m = CoxModel.__new__(CoxModel)
        m.h = cox_init_intervals(self.h, time, event, stratum, cuts, tv_coef, inherit=not opts, **opts)
        _live.add(m)
        return m

    def baseline_hazard(self, beta):
        return cox_baseline_hazard(self.h, beta)

    def set_penalty(self, gamma, penalize=None):
        cox_set_penalty(self.h, gamma, penalize)

    def cross_validate(self, fold, gammas, penalize=None, nfolds=None):
        return cox_cross_validate(self.h, fold, gammas, penalize, nfolds)

    def cross_validate_served(self, server, X, time, event, stratum, fold, gammas, penalize=None, nfolds=None):
        return cox_cross_validate_served(self.h, server, X, time, event, stratum, fold, gammas, penalize, nfolds)

    def bootstrap(self, counts, beta0=None):
        return cox_bootstrap(self.h, counts, beta0)

    def kernel_ms(self):
        return cox_last_kernel_ms(self.h)

    def profile(self):
        return cox_last_profile(self.h)

    def close(self):
        if self.h:
            cox_release(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ fit server

def cox_server_default_options() -> cox_server_options:
    o = cox_server_options()
    lib().cox_server_default_options(ctypes.byref(o))
    return o


class CoxServer:
    """Continuous-batching server of independent unpenalised fits (cox_server_* in the C ABI).

    submit() returns a ticket at once; poll() returns None while the fit is
    pending, else (beta, info, times).  Inputs are borrowed by default (the
    arrays are kept referenced here until their result is collected).
    """

    def __init__(self, hbm_budget=None, staging_bytes=None, max_resident=None, prep_threads=None,
                 tol=None, max_iter=None, device=None, fused_rounds=None):
        o = cox_server_default_options()
        if fused_rounds is not None:
            o.fused_rounds = int(fused_rounds)
        if hbm_budget is not None:
            o.hbm_budget = int(hbm_budget)
        if staging_bytes is not None:
            o.staging_bytes = int(staging_bytes)
        if max_resident is not None:
            o.max_resident = int(max_resident)
        if prep_threads is not None:
            o.prep_threads = int(prep_threads)
        if tol is not None:
            o.tol = float(tol)
        if max_iter is not None:
            o.max_iter = int(max_iter)
        if device is not None:
            o.device = int(device)
        h = ctypes.c_void_p()
        rc = lib().cox_server_create(ctypes.byref(h), ctypes.byref(o))
        if rc != COX_OK:
            msg = lib().cox_server_last_error(None)
            raise CoxError(rc, msg.decode() if msg else "")
        self.h = h.value
        self._keep = {}
        self._p = {}
        _live.add(self)

    def _check(self, rc, ok=(COX_OK,)):
        if rc not in ok:
            msg = lib().cox_server_last_error(self.h)
            raise CoxError(rc, msg.decode() if msg else "")
        return rc

    @staticmethod
    def _request(p, gamma, penalize, beta0):
        """(cox_fit_request or None, arrays to keep alive) for the per-request options."""
        if gamma == 0.0 and penalize is None and beta0 is None:
            return None, []
        r = cox_fit_request(gamma=float(gamma))
        keep = []
        if penalize is not None:
            pen = np.ascontiguousarray(penalize, dtype=np.uint8)
            if pen.shape != (p,):
                raise ValueError(f"penalize needs {p} entries")
            r.penalize = pen.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
            keep.append(pen)
        if beta0 is not None:
            b0 = np.ascontiguousarray(beta0, dtype=np.float64)
            if b0.shape != (p,):
                raise ValueError(f"beta0 needs {p} entries")
            r.beta0 = _dptr(b0)
            keep.append(b0)
        return r, keep

    def _submit(self, d, flags, p, gamma, penalize, beta0):
        r, keep = self._request(p, gamma, penalize, beta0)
        t = ctypes.c_uint64()
        if r is None:
            self._check(lib().cox_server_submit(self.h, ctypes.byref(d), flags, ctypes.byref(t)))
        else:
            self._check(lib().cox_server_submit_fit(self.h, ctypes.byref(d), flags, ctypes.byref(r), ctypes.byref(t)))
        del keep   # the request options are copied by the call
        return t.value

    def submit_device(self, X, time, event, stratum=None, gamma=0.0, penalize=None, beta0=None) -> int:
        """Submit device-resident data (torch tensors on the server's device):
        X float64 n x p with unit row stride (column-major, e.g. a transposed
        contiguous p x n tensor), time float64, event uint8, stratum int32 or
        None.  The tensors are read in place and kept referenced until the
        result is collected; the caller synchronises the stream that wrote them.
        gamma, penalize, beta0: l1 weight, penalised columns and start point
        (cox_server_submit_fit)."""
        n, p = X.shape
        d = _device_data(X, time, event, stratum)
        t = self._submit(d, COX_SUBMIT_DEVICE, p, gamma, penalize, beta0)
        self._keep[t] = [X, time, event, stratum]
        self._p[t] = p
        return t

    def submit(self, X, time, event, stratum=None, borrow=True, gamma=0.0, penalize=None, beta0=None) -> int:
        X = np.asfortranarray(X, dtype=np.float64)
        n, p = X.shape
        time = np.ascontiguousarray(time, dtype=np.float64)
        event = np.ascontiguousarray(event, dtype=np.uint8)
        keep = [X, time, event]
        d = cox_data(n=n, p=p, x=_dptr(X), ldx=n, time=_dptr(time),
                     event=event.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        if stratum is not None:
            st = np.ascontiguousarray(stratum, dtype=np.int32)
            keep.append(st)
            d.stratum = st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        t = self._submit(d, COX_SUBMIT_BORROW if borrow else 0, p, gamma, penalize, beta0)
        if borrow:
            self._keep[t] = keep
        self._p[t] = p
        return t

    def poll(self, ticket):
        p = self._p[ticket]
        beta = np.zeros(p)
        info = cox_fit_info()
        times = cox_request_times()
        rc = self._check(lib().cox_server_poll(self.h, ticket, _dptr(beta), ctypes.byref(info), ctypes.byref(times)),
                         ok=(COX_OK, 1))
        if rc == 1:
            return None
        self._keep.pop(ticket, None)
        self._p.pop(ticket, None)
        return beta, info.as_dict(), times.as_dict()

    def wait(self, ticket, timeout=None) -> bool:
        rc = self._check(lib().cox_server_wait(self.h, ticket, -1.0 if timeout is None else float(timeout)),
                         ok=(COX_OK, 1))
        return rc == COX_OK

    def drain(self, timeout=None) -> bool:
        rc = self._check(lib().cox_server_drain(self.h, -1.0 if timeout is None else float(timeout)),
                         ok=(COX_OK, 1))
        return rc == COX_OK

    def stats(self) -> dict:
        c = cox_server_counters()
        self._check(lib().cox_server_stats(self.h, ctypes.byref(c)))
        return c.as_dict()

    def close(self):
        if self.h:
            lib().cox_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
