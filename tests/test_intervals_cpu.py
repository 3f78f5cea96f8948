"""Time intervals (Secs. 2.2-2.3): the oracle's augmentation pinned to the
paper's likelihoods, and the library's cox_split_intervals bit-exact against it.

Pins of the oracle (none retypes its construction):
* splitting at cut points with time-fixed covariates and coefficients leaves
  Eq. strat_l, its gradient and its information unchanged (every risk set of
  the original data reappears whole in one interval stratum);
* step-function coefficients (Sec. 2.3) and piecewise-constant covariates
  (Sec. 2.2): the augmented stratified likelihood equals Eq. time_coef_l /
  Eq. time_cov_l evaluated by brute force, which reads x_r(t) and beta(t) at
  each event time without any augmentation;
* tying the K coefficients of a step column reproduces the time-fixed fit;
* the paper's K N-row matrix (rows outside their interval kept, with no event)
  gives the same likelihood as the reduced one;
* structural invariants: every augmented time lies in its interval (closed at
  the right end), events are conserved one for one, and the Sec. 2.3 example
  rows read (x_i1, 0, x_i2, ...) before the cut and (0, x_i1, x_i2, ...) after.
Planted mistakes in a copy of the oracle's split must each break one of them.
"""
import inspect

import numpy as np
import pytest

from oracle import cox_oracle as o
from paper_2310_16238_amd import coxmi, synth


def _data(n=90, p=4, K=3, seed=5):
    d = synth.make("iid", n, p, K, seed, beta_sd=0.6, tie_round=10.0)
    return d.X, d.time, d.event, d.stratum


def _cuts(time, m):
    """m cut points placed on observed times (so that some subjects end exactly at a cut)."""
    u = np.unique(time)
    return u[np.linspace(1, len(u) - 2, m).round().astype(int)]


def _aug_obj(a, beta):
    return o.neg_loglik_brute(a["X"], a["time"], a["event"], a["stratum"], beta)


# ---------------------------------------------------------------- pins of the oracle

def _pin_invariance(split):
    X, t, e, s = _data()
    cuts = _cuts(t, 3)
    a = split(X, t, e, s, cuts)
    ok = True
    for seed in range(3):
        beta = np.random.default_rng(seed).normal(0, 0.5, X.shape[1])
        ref = o.neg_loglik_brute(X, t, e, s, beta)
        ok &= abs(_aug_obj(a, beta) - ref) <= 1e-12 * abs(ref)
        ok &= np.allclose(o.grad_brute(a["X"], a["time"], a["event"], a["stratum"], beta),
                          o.grad_brute(X, t, e, s, beta), rtol=0, atol=1e-12 * e.sum())
        ok &= np.allclose(o.info_brute(a["X"], a["time"], a["event"], a["stratum"], beta),
                          o.info_brute(X, t, e, s, beta), rtol=0, atol=1e-12 * e.sum())
    return bool(ok)


def _pin_step_coefficients(split):
    X, t, e, s = _data(seed=7)
    cuts = _cuts(t, 2)
    K = len(cuts) + 1
    tv = np.array([1, 0, 1, 0], np.uint8)
    a = split(X, t, e, s, cuts, tv_coef=tv)
    rng = np.random.default_rng(3)
    beta_k = rng.normal(0, 0.6, (K, X.shape[1]))        # beta(t) on each interval
    beta_k[:, ~tv.astype(bool)] = beta_k[0, ~tv.astype(bool)]
    beta_aug = np.array([beta_k[max(k, 0), j] for j, k in zip(a["col_source"], a["col_interval"])])
    ref = o.neg_loglik_time_varying_brute([X] * K, t, e, s, cuts, beta_k)
    return abs(_aug_obj(a, beta_aug) - ref) <= 1e-12 * abs(ref)


def _pin_time_varying_covariates(split):
    X, t, e, s = _data(seed=9)
    cuts = _cuts(t, 3)
    K = len(cuts) + 1
    rng = np.random.default_rng(4)
    XK = [X + rng.normal(0, 0.4, X.shape) for _ in range(K)]   # x_i(t) piecewise constant
    tv = np.array([0, 1, 0, 0], np.uint8)
    a = split(X, t, e, s, cuts, tv_coef=tv, X_by_interval=XK)
    beta_k = np.tile(rng.normal(0, 0.5, X.shape[1]), (K, 1))
    beta_k[:, 1] = rng.normal(0, 0.5, K)
    beta_aug = np.array([beta_k[max(k, 0), j] for j, k in zip(a["col_source"], a["col_interval"])])
    ref = o.neg_loglik_time_varying_brute(XK, t, e, s, cuts, beta_k)
    return abs(_aug_obj(a, beta_aug) - ref) <= 1e-12 * abs(ref)


def _pin_tied_coefficients(split):
    X, t, e, s = _data(seed=11)
    cuts = _cuts(t, 2)
    a = split(X, t, e, s, cuts, tv_coef=np.array([0, 1, 1, 0], np.uint8))
    beta = np.array([0.3, -0.7, 0.5, 0.2])
    beta_aug = beta[a["col_source"]]
    ref = o.neg_loglik_brute(X, t, e, s, beta)
    return abs(_aug_obj(a, beta_aug) - ref) <= 1e-12 * abs(ref)


def _pin_all_rows_form(split):
    X, t, e, s = _data(seed=13)
    cuts = _cuts(t, 3)
    full = split(X, t, e, s, cuts, keep_all_rows=True)
    red = split(X, t, e, s, cuts)
    beta = np.array([0.4, -0.2, 0.1, 0.8])
    K = len(cuts) + 1
    ok = full["X"].shape[0] == K * X.shape[0]
    return ok and abs(_aug_obj(full, beta) - _aug_obj(red, beta)) <= 1e-12 * abs(_aug_obj(red, beta))


def _pin_structure(split):
    X, t, e, s = _data(seed=15)
    cuts = _cuts(t, 3)
    a = split(X, t, e, s, cuts)
    bounds = np.concatenate([[-np.inf], cuts, [np.inf]])
    k = a["row_interval"]
    ok = np.all(a["time"] >= bounds[k]) and np.all(a["time"] <= bounds[k + 1])
    ok &= int(a["event"].sum()) == int(e.sum())
    ev = a["event"] == 1
    ok &= np.array_equal(a["time"][ev], t[a["row_subject"][ev]])       # an event keeps its own time
    ok &= np.array_equal(np.sort(a["row_subject"][ev]), np.flatnonzero(e))
    # Sec. 2.3 example: one cut t_s, a step coefficient on the first column
    ts = cuts[1]
    b = split(X, t, e, s, [ts], tv_coef=np.array([1, 0, 0, 0], np.uint8))
    i = b["row_subject"]
    before = b["row_interval"] == 0
    ok &= np.array_equal(b["X"][before], np.column_stack([X[i[before], 0], np.zeros(before.sum()), X[i[before], 1:]]))
    ok &= np.array_equal(b["X"][~before], np.column_stack([np.zeros((~before).sum()), X[i[~before], 0], X[i[~before], 1:]]))
    return bool(ok)


PINS = {
    "invariance": _pin_invariance,
    "step_coefficients": _pin_step_coefficients,
    "time_varying_covariates": _pin_time_varying_covariates,
    "tied_coefficients": _pin_tied_coefficients,
    "all_rows_form": _pin_all_rows_form,
    "structure": _pin_structure,
}


@pytest.mark.parametrize("name", sorted(PINS))
def test_oracle_split_pin(name):
    assert PINS[name](o.split_intervals)


# Planted mistakes in a copy of the oracle's split: each must break a pin.
MUTANTS = {
    "event_everywhere": ("event=np.where(in_k, d[rows], 0)", "event=d[rows]"),
    "time_not_clipped": ("time=np.minimum(Y[rows], hi)", "time=Y[rows]"),
    "strata_merged": ("stratum=srank[rows] * K + k", "stratum=srank[rows]"),
    "strata_collide": ("stratum=srank[rows] * K + k", "stratum=srank[rows] + k"),
    "step_column_wrong_interval": ("if kc < 0 or kc == k:", "if kc < 0 or kc != k:"),
    "interval_covariates_ignored": ("xk = X if X_by_interval is None else", "xk = X if True else"),
    "left_end_open": ("in_k = (Y[rows] >= lo) & (Y[rows] < hi)", "in_k = (Y[rows] > lo) & (Y[rows] < hi)"),
    "right_end_closed": ("in_k = (Y[rows] >= lo) & (Y[rows] < hi)", "in_k = (Y[rows] >= lo) & (Y[rows] <= hi)"),
    "rows_not_dropped": ("rows = np.arange(n) if keep_all_rows else np.flatnonzero(Y >= lo)",
                         "rows = np.arange(n)"),
}


def _mutant(name):
    src = inspect.getsource(o.split_intervals)
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    ns = {"np": np, "augmented_columns": o.augmented_columns}
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return ns["split_intervals"]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_split_mutant_is_caught(name):
    split = _mutant(name)
    failed = []
    for pin, fn in PINS.items():
        try:
            with np.errstate(all="ignore"):
                ok = fn(split)
        except Exception:
            ok = False
        if not ok:
            failed.append(pin)
    assert failed, f"mutant {name} passes every pin"


# ---------------------------------------------------------------- library vs oracle

def _compare(X, t, e, s, cuts, tv=None, XK=None):
    a = o.split_intervals(X, t, e, s, cuts, tv_coef=tv, X_by_interval=XK)
    b = coxmi.split_intervals(X, t, e, s, cuts, tv_coef=tv, X_by_interval=XK)
    assert b["intervals"] == a["intervals"]
    for key in ("X", "time", "event", "stratum", "row_subject", "row_interval", "col_source", "col_interval"):
        assert b[key].shape == a[key].shape, key
        assert np.array_equal(b[key], a[key]), key
    return b


@pytest.mark.parametrize("ncuts", [0, 1, 3, 7])
@pytest.mark.parametrize("strata", [False, True])
def test_split_matches_oracle(ncuts, strata):
    X, t, e, s = _data(n=300, p=5, K=4, seed=21 + ncuts)
    cuts = _cuts(t, ncuts) if ncuts else []
    tv = np.array([1, 0, 0, 1, 0], np.uint8)
    _compare(X, t, e, s if strata else None, cuts, tv)
    _compare(X, t, e, s if strata else None, cuts)


def test_split_interval_covariates_match_oracle():
    X, t, e, s = _data(n=200, p=3, K=2, seed=31)
    cuts = _cuts(t, 2)
    rng = np.random.default_rng(2)
    XK = [rng.normal(size=X.shape) for _ in range(3)]
    _compare(X, t, e, s, cuts, np.array([0, 1, 0], np.uint8), XK)


def test_split_edge_cases():
    X, t, e, s = _data(n=50, p=2, K=2, seed=41)
    # cuts outside the observed range: an empty first interval boundary, a last interval with no rows but
    # subjects still carried (every Y >= the low cut)
    _compare(X, t, e, s, [t.min() - 1.0, t.max() + 1.0], np.array([1, 0], np.uint8))
    # a cut at the largest time: subjects ending there belong to the last interval
    b = _compare(X, t, e, s, [t.max()])
    assert np.all(b["row_interval"][b["time"] == t.max()] >= 0)
    # one subject
    _compare(np.array([[1.5, -2.0]]), np.array([3.0]), np.array([1], np.uint8), None, [1.0, 5.0],
             np.array([0, 1], np.uint8))
    # labels that are not 0..S-1 map to their ranks
    _compare(X, t, e, s * 7 - 100, _cuts(t, 2))


@pytest.mark.parametrize("cuts", [[1.0, 1.0], [2.0, 1.0], [np.nan], [np.inf], [-np.inf, 0.0]])
def test_split_rejects_bad_cuts(cuts):
    X, t, e, s = _data(n=20, p=2, K=1, seed=51)
    with pytest.raises(coxmi.CoxError) as err:
        coxmi.split_intervals(X, t, e, s, cuts)
    assert err.value.code == coxmi.COX_EINVAL


def test_split_rejects_bad_data():
    X, t, e, s = _data(n=20, p=2, K=1, seed=52)
    e2 = e.copy()
    e2[0] = 2
    with pytest.raises(coxmi.CoxError):
        coxmi.split_intervals(X, t, e2, s, [0.5])
    t2 = t.copy()
    t2[3] = np.nan
    with pytest.raises(coxmi.CoxError):
        coxmi.split_intervals(X, t2, e, s, [0.5])
    with pytest.raises(ValueError):
        coxmi.split_intervals(X, t, e, s, [0.5], X_by_interval=[X])
