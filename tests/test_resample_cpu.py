"""Resampling, cross-validation and bootstrap in the oracle (Secs. 2.1, 3.2), pinned.

Pins (none retypes the oracle's own construction):
* duplicating every row doubles -log L and adds 2 E log 2 (Breslow: each tie group's
  event count and risk-set sum both double), so the unpenalised optimum is unchanged and
  an l1 fit with weight gamma on the doubled data equals the fit with gamma / 2 on the
  original;
* with folds that are whole strata, l(beta) - l_{-k}(beta) is fold k's own stratum
  likelihood (strata are independent factors of Eq. strat_l), evaluated by brute force;
* with a penalty large enough to hold every coefficient at 0, the criterion is
  sum_k [l(0) - l_{-k}(0)] by brute force;
* every fold's coefficients satisfy the l1 optimality conditions on that fold's
  training rows (brute-force gradient of Eq. strat_g);
* the percentile interval of 0..100 at level 0.9 is [5, 95].
Planted mistakes in a copy of cross_validate must each break one of them.
"""
import inspect
import math

import numpy as np
import pytest

from oracle import cox_oracle as o
from paper_2310_16238_amd import synth


def _data(n=160, p=3, K=4, seed=3):
    d = synth.make("iid", n, p, K, seed, beta_sd=0.6, tie_round=20.0)
    return d.X, d.time, d.event, d.stratum


def test_duplication_closed_form():
    X, t, e, s = _data()
    Xd, td, ed, sd = o.resample(X, t, e, s, np.full(t.shape[0], 2))
    E = int(e.sum())
    for seed in range(3):
        beta = np.random.default_rng(seed).normal(0, 0.5, X.shape[1])
        ref = o.neg_loglik_brute(X, t, e, s, beta)
        dup = o.neg_loglik(Xd, td, ed, sd, beta)
        assert abs(dup - (2.0 * ref + 2.0 * E * math.log(2.0))) <= 1e-11 * abs(dup)
    b1 = o.fit_ccd(X, t, e, s, tol=1e-14).beta
    b2 = o.fit_ccd(Xd, td, ed, sd, tol=1e-14).beta
    assert np.max(np.abs(b1 - b2)) <= 1e-10 * np.max(np.abs(b1))
    g1 = o.fit_ccd(X, t, e, s, gamma=1.5, tol=1e-14).beta
    g2 = o.fit_ccd(Xd, td, ed, sd, gamma=3.0, tol=1e-14).beta
    assert np.array_equal(g1 == 0, g2 == 0) and np.max(np.abs(g1 - g2)) <= 1e-10 * np.max(np.abs(g1))


def test_bootstrap_counts_one_and_two():
    X, t, e, s = _data(seed=5)
    n = t.shape[0]
    counts = np.stack([np.ones(n, np.int64), np.full(n, 2)])
    betas, conv = o.bootstrap(X, t, e, s, counts, gamma=1.0)
    assert conv.all()
    ref = o.fit_ccd(X, t, e, s, gamma=1.0, tol=1e-13).beta
    half = o.fit_ccd(X, t, e, s, gamma=0.5, tol=1e-13).beta
    assert np.max(np.abs(betas[0] - ref)) <= 1e-10 * np.max(np.abs(ref))
    assert np.max(np.abs(betas[1] - half)) <= 1e-10 * np.max(np.abs(half))


def test_percentile_interval():
    lo, hi = o.percentile_interval(np.arange(101.0), 0.9)
    assert abs(lo - 5.0) <= 1e-12 and abs(hi - 95.0) <= 1e-12


# ---------------------------------------------------------------- CV pins (also run on mutants)

def _pin_strata_folds(cv):
    X, t, e, s = _data(seed=7)
    fold = s.astype(np.int64)          # fold k = stratum k
    gammas = [4.0, 1.0, 0.0]
    cvl, betas, conv = cv(X, t, e, s, fold, gammas)
    ok = bool(conv.all())
    for g in range(len(gammas)):
        ref = 0.0
        for k in range(4):
            r = fold == k
            ref += -o.neg_loglik_brute(X[r], t[r], e[r], s[r], betas[k, g])
        ok &= abs(cvl[g] - ref) <= 1e-10 * abs(ref)
    return ok


def _pin_zero_path(cv):
    X, t, e, s = _data(seed=9)
    fold = np.arange(t.shape[0]) % 5
    cvl, betas, _ = cv(X, t, e, s, fold, [1e6])
    z = np.zeros(X.shape[1])
    ref = 0.0
    for k in range(5):
        r = fold != k
        ref += -o.neg_loglik_brute(X, t, e, s, z) + o.neg_loglik_brute(X[r], t[r], e[r], s[r], z)
    return bool(np.all(betas == 0.0)) and abs(cvl[0] - ref) <= 1e-10 * abs(ref)


def _pin_fold_optimality(cv):
    X, t, e, s = _data(seed=11)
    fold = np.random.default_rng(1).integers(0, 4, t.shape[0])
    gammas = [3.0, 0.7]
    _, betas, _ = cv(X, t, e, s, fold, gammas)
    ok = True
    for k in range(4):
        r = fold != k
        E = float(e[r].sum())
        for g, gam in enumerate(gammas):
            b = betas[k, g]
            gr = o.grad_brute(X[r], t[r], e[r], s[r], b)
            res = np.where(b != 0.0, np.abs(gr + gam * np.sign(b)), np.maximum(np.abs(gr) - gam, 0.0))
            ok &= float(res.max()) <= 1e-9 * E
    return ok


PINS = {"strata_folds": _pin_strata_folds, "zero_path": _pin_zero_path, "fold_optimality": _pin_fold_optimality}


@pytest.mark.parametrize("name", sorted(PINS))
def test_cross_validation_pin(name):
    assert PINS[name](o.cross_validate)


MUTANTS = {
    "trains_on_fold": ("(fold != k).astype(np.int64)", "(fold == k).astype(np.int64)"),
    "criterion_sign": ("cvl[g] += l_all - l_train", "cvl[g] += l_train - l_all"),
    "held_out_alone": ("l_all = -neg_loglik(X, time, event, stratum, beta)", "l_all = 0.0"),
    "gamma_ignored": ("fit_ccd(Xt, tt, et, st, gamma=gam,", "fit_ccd(Xt, tt, et, st, gamma=0.0,"),
    "path_reuses_first": ("betas[k, g] = beta", "betas[k, g] = betas[k, 0] if g else beta"),
}


def _mutant(name):
    src = inspect.getsource(o.cross_validate)
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    ns = dict(vars(o))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return ns["cross_validate"]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_cross_validation_mutant_is_caught(name):
    cv = _mutant(name)
    failed = []
    for pin, fn in PINS.items():
        try:
            with np.errstate(all="ignore"):
                ok = fn(cv)
        except Exception:
            ok = False
        if not ok:
            failed.append(pin)
    assert failed, f"mutant {name} passes every pin"
