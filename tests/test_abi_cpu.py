"""Host-only checks of the C ABI: the library loads, exports every symbol that
include/coxmi.h declares, and rejects bad inputs before touching a device."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2310_16238_amd import coxmi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "coxmi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\**\s*(cox_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_expected_entry_points():
    names = _declared()
    for must in ["cox_init", "cox_fit", "cox_evaluate", "cox_release", "cox_coordinate",
                 "cox_layout", "cox_segscan_f64", "cox_last_error", "cox_default_options"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(coxmi.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    bound = {name for name, _, _ in coxmi.SIGNATURES}
    assert bound == set(_declared())


def test_default_options():
    o = coxmi.cox_default_options()
    assert o.gamma == 0.0 and o.tol == 1e-12 and o.max_iter == 1000
    assert o.mode == coxmi.COX_CCD and o.x_precision == coxmi.COX_F64 and o.ties == coxmi.COX_BRESLOW


def _data(n=20, p=3):
    rng = np.random.default_rng(0)
    return rng.standard_normal((n, p)), rng.exponential(1.0, n), (rng.random(n) < 0.5).astype(np.uint8)


@pytest.mark.parametrize("case", ["nan_time", "inf_time", "event2", "gamma_neg", "tol_neg", "maxit0", "ties"])
def test_init_rejects_bad_inputs(case):
    X, t, e = _data()
    kw = {}
    if case == "nan_time":
        t[3] = math.nan
    elif case == "inf_time":
        t[0] = math.inf
    elif case == "event2":
        e[5] = 2
    elif case == "gamma_neg":
        kw["gamma"] = -1.0
    elif case == "tol_neg":
        kw["tol"] = -1e-3
    elif case == "maxit0":
        kw["max_iter"] = 0
    elif case == "ties":
        kw["ties"] = 7            # neither COX_BRESLOW nor COX_EFRON
    with pytest.raises(coxmi.CoxError) as ei:
        coxmi.cox_init(X, t, e, **kw)
    assert ei.value.code == coxmi.COX_EINVAL
    assert coxmi.cox_last_error(None)


def test_init_rejects_bad_shapes():
    lib = coxmi.lib()
    X, t, e = _data()
    dp = ctypes.POINTER(ctypes.c_double)
    Xf = np.asfortranarray(X)
    base = dict(x=Xf.ctypes.data_as(dp), time=t.ctypes.data_as(dp),
                event=e.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    h = ctypes.c_void_p()
    for n, p, ldx in [(0, 3, 20), (20, 0, 20), (20, 3, 19)]:
        d = coxmi.cox_data(n=n, p=p, ldx=ldx, **base)
        assert lib.cox_init(ctypes.byref(h), ctypes.byref(d), None) == coxmi.COX_EINVAL
        assert not h.value
    d = coxmi.cox_data(n=20, p=3, ldx=20, time=base["time"], event=base["event"])
    assert lib.cox_init(ctypes.byref(h), ctypes.byref(d), None) == coxmi.COX_EINVAL
    assert lib.cox_init(None, ctypes.byref(d), None) == coxmi.COX_EINVAL


def test_init_on_device_rejects_host_arrays():
    """on_device = 1 with host arrays: rejected by the pointer checks, before any copy."""
    lib = coxmi.lib()
    X, t, e = _data()
    dp = ctypes.POINTER(ctypes.c_double)
    Xf = np.asfortranarray(X)
    d = coxmi.cox_data(n=20, p=3, ldx=20, x=Xf.ctypes.data_as(dp), time=t.ctypes.data_as(dp),
                       event=e.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), on_device=1)
    h = ctypes.c_void_p()
    assert lib.cox_init(ctypes.byref(h), ctypes.byref(d), None) == coxmi.COX_EINVAL
    assert not h.value
    assert coxmi.cox_last_error(None)


def test_null_handle_calls_are_errors():
    lib = coxmi.lib()
    b = np.zeros(3)
    dp = ctypes.POINTER(ctypes.c_double)
    assert lib.cox_fit(None, None, b.ctypes.data_as(dp), None) == coxmi.COX_EINVAL
    assert lib.cox_evaluate(None, b.ctypes.data_as(dp), None, None, None) == coxmi.COX_EINVAL
    assert lib.cox_layout(None, None, None) == coxmi.COX_EINVAL
    lib.cox_release(None)


def test_server_rejects_bad_options_before_the_device():
    lib = coxmi.lib()
    h = ctypes.c_void_p()
    for field, value, code in [("x_precision", coxmi.COX_F64, coxmi.COX_EUNSUPPORTED),
                               ("max_iter", 0, coxmi.COX_EINVAL), ("tol", -1.0, coxmi.COX_EINVAL),
                               ("prep_threads", 0, coxmi.COX_EINVAL), ("hbm_budget", 1024, coxmi.COX_EINVAL)]:
        o = coxmi.cox_server_default_options()
        setattr(o, field, value)
        assert lib.cox_server_create(ctypes.byref(h), ctypes.byref(o)) == code, field
        assert h.value is None
        assert lib.cox_server_last_error(None)


def test_server_default_options():
    o = coxmi.cox_server_default_options()
    assert o.x_precision == coxmi.COX_F32 and o.tol == 1e-12 and o.max_iter == 100
    assert o.hbm_budget == 8 << 30 and o.staging_bytes == 1 << 30 and o.device == -1


def test_new_entry_points_reject_bad_inputs_before_the_device():
    L = coxmi.lib()
    out = ctypes.c_void_p()
    cnt = np.ones(4, np.uint32)
    # resampling, intervals, penalties, CV, bootstrap, baseline hazard: NULL handles and outputs
    assert L.cox_init_resample(None, None, cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), None) == coxmi.COX_EINVAL
    assert L.cox_init_resample(ctypes.byref(out), None, None, None) == coxmi.COX_EINVAL and out.value is None
    t = np.array([1.0, 2.0]); e = np.array([1, 0], np.uint8)
    assert L.cox_init_intervals(ctypes.byref(out), None, coxmi._dptr(t), e.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                None, 0, None, None, None) == coxmi.COX_EINVAL
    assert L.cox_set_penalty(None, 1.0, None) == coxmi.COX_EINVAL
    assert L.cox_cross_validate(None, 2, None, 1, None, None, None, None, None) == coxmi.COX_EINVAL
    assert L.cox_bootstrap(None, 1, None, None, None, None) == coxmi.COX_EINVAL
    b = np.zeros(1)
    assert L.cox_baseline_hazard(None, coxmi._dptr(b), coxmi._dptr(b)) == coxmi.COX_EINVAL


@pytest.mark.parametrize("case", ["col_ptr_start", "col_ptr_decreasing", "row_out_of_range", "nan_time",
                                  "event_2", "p_too_large", "newton_mode"])
def test_indicator_init_rejects_bad_inputs(case):
    n, p = 5, 2
    ptr = np.array([0, 2, 3], np.int64)
    idx = np.array([0, 3, 4], np.int32)
    time = np.linspace(1.0, 2.0, n)
    event = np.array([1, 0, 1, 1, 0], np.uint8)
    kw = {}
    code = coxmi.COX_EINVAL
    if case == "col_ptr_start":
        ptr = np.array([1, 2, 3], np.int64)
    elif case == "col_ptr_decreasing":
        ptr = np.array([0, 3, 2], np.int64)
    elif case == "row_out_of_range":
        idx = np.array([0, 3, 5], np.int32)
    elif case == "nan_time":
        time[2] = math.nan
    elif case == "event_2":
        event[1] = 2
    elif case == "p_too_large":
        ptr = np.zeros(12290, np.int64)
        code = coxmi.COX_EUNSUPPORTED
    elif case == "newton_mode":
        code = coxmi.COX_EUNSUPPORTED
    o = coxmi.cox_default_options()
    if case == "newton_mode":
        o.mode = coxmi.COX_NEWTON_REFINE
    out = ctypes.c_void_p()
    rc = coxmi.lib().cox_init_indicator(ctypes.byref(out), n, ptr.shape[0] - 1,
                                        ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), coxmi._dptr(time),
                                        event.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), None, ctypes.byref(o))
    assert rc == code and out.value is None
    assert coxmi.lib().cox_last_error(None)
