"""Pins of the oracle's Efron tie correction (Efron, JASA 72, 1977).

The paper's risk sets (Eq. strat_l) are Breslow's; Efron's correction is a variant it
does not discuss.  What fixes the oracle's Efron functions independently of themselves:
* the hand-derived closed forms of toy 3 (tests/golden/toy_closed_forms.txt): values at
  beta = 0 and the optimum as the root of a cubic, solved here by numpy.roots;
* with no tied events Efron's and Breslow's likelihoods are the same function;
* the scan form (C) against the definition written as loops over tie groups and their
  events, for objective, gradient, diagonal and full Hessian;
* central finite differences of the brute-force objective and gradient;
* the optimum: zero brute-force score, CCD and Newton agreeing, and input order, stratum
  labels and monotone time transforms leaving everything unchanged.
"""
import math

import numpy as np
import pytest

from conftest import read_golden
from oracle import cox_oracle as o
from paper_2310_16238_amd import synth


def _toy3():
    g = read_golden("toy_closed_forms.txt")
    X = np.array(g["toy3.x"])[:, None]
    return g, X, np.array(g["toy3.time"]), np.array(g["toy3.event"], dtype=np.uint8)


def _tied(n, p, K, seed, round_to=5.0):
    return synth.make("iid", n, p, K, seed, beta_sd=0.6, tie_round=round_to)


def test_toy3_closed_forms_efron_and_breslow():
    g, X, t, e = _toy3()
    for order in [[0, 1, 2, 3], [2, 1, 3, 0], [3, 2, 0, 1]]:
        Xo, to, eo = X[order], t[order], e[order]
        L = o.canonical_layout(to, eo)
        Xc = o.to_canonical(Xo, L)
        for ties in ("breslow", "efron"):
            c = o.coord_terms(Xc, L, 0, np.zeros(4), ties)
            fe = o.full_eval(Xc, L, [0.0], ties=ties)
            for val, key in [(c["grad"], "grad0"), (fe.grad[0], "grad0"), (c["hess"], "hess0"),
                             (fe.hess_diag[0], "hess0"), (fe.info[0, 0], "hess0"), (c["obj"], "negloglik0"),
                             (fe.objective, "negloglik0")]:
                assert val == pytest.approx(g[f"toy3.{ties}.{key}"][0], rel=1e-15, abs=1e-15), (ties, key)
        assert o.neg_loglik_efron_brute(Xo, to, eo, None, [0.0]) == pytest.approx(g["toy3.efron.negloglik0"][0],
                                                                                   rel=1e-15)
        assert o.grad_efron_brute(Xo, to, eo, None, [0.0])[0] == pytest.approx(g["toy3.efron.grad0"][0], rel=1e-15)
        assert o.info_efron_brute(Xo, to, eo, None, [0.0])[0, 0] == pytest.approx(g["toy3.efron.hess0"][0],
                                                                                   rel=1e-15)
    # optima: Breslow in closed form, Efron the positive root of the stored cubic
    r = np.roots(g["toy3.efron.cubic"])
    u = float(r[(np.abs(r.imag) < 1e-12) & (r.real > 0)].real[0])
    for fit in (o.fit_newton(X, t, e, ties="efron"), o.fit_ccd(X, t, e, ties="efron", tol=1e-15)):
        assert fit.beta[0] == pytest.approx(math.log(u), abs=1e-13)
    for fit in (o.fit_newton(X, t, e), o.fit_ccd(X, t, e, tol=1e-15)):
        assert fit.beta[0] == pytest.approx(g["toy3.breslow.betahat"][0], abs=1e-13)


def test_no_ties_efron_equals_breslow():
    d = synth.make("iid", 300, 4, 5, 31, beta_sd=0.6)      # continuous times: every group has one row
    beta = np.array([0.3, -0.4, 0.2, 0.6])
    L = o.canonical_layout(d.time, d.event, d.stratum)
    assert L.dcount.max() == 1
    Xc = o.to_canonical(d.X, L)
    eta = Xc @ beta
    for j in range(4):
        a, b = o.coord_terms(Xc, L, j, eta), o.coord_terms(Xc, L, j, eta, "efron")
        for k in ("grad", "hess", "obj", "m2"):
            assert a[k] == pytest.approx(b[k], rel=1e-14, abs=1e-14)
    fb, fe = o.full_eval(Xc, L, beta), o.full_eval(Xc, L, beta, ties="efron")
    np.testing.assert_allclose(fe.info, fb.info, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(fe.grad, fb.grad, rtol=1e-13, atol=1e-13)
    assert o.neg_loglik_efron_brute(d.X, d.time, d.event, d.stratum, beta) == pytest.approx(
        o.neg_loglik_brute(d.X, d.time, d.event, d.stratum, beta), rel=1e-14)


@pytest.mark.parametrize("K,round_to", [(1, 5.0), (4, 10.0), (30, 2.0)])
def test_efron_scan_form_equals_definition(K, round_to):
    d = _tied(180, 4, K, 40 + K, round_to)
    beta = np.array([0.5, -0.8, 0.2, 1.1])
    L = o.canonical_layout(d.time, d.event, d.stratum)
    assert L.dcount.max() >= 3                      # real ties
    Xc = o.to_canonical(d.X, L)
    ref_obj = o.neg_loglik_efron_brute(d.X, d.time, d.event, d.stratum, beta)
    ref_g = o.grad_efron_brute(d.X, d.time, d.event, d.stratum, beta)
    ref_I = o.info_efron_brute(d.X, d.time, d.event, d.stratum, beta)
    eta = Xc @ beta
    scale = max(1.0, float(d.event.sum()))
    for j in range(4):
        c = o.coord_terms(Xc, L, j, eta, "efron")
        assert abs(c["grad"] - ref_g[j]) <= 1e-13 * scale
        assert abs(c["hess"] - ref_I[j, j]) <= 1e-13 * scale
        assert abs(c["obj"] - ref_obj) <= 1e-13 * scale
    fe = o.full_eval(Xc, L, beta, ties="efron")
    assert abs(fe.objective - ref_obj) <= 1e-13 * scale
    np.testing.assert_allclose(fe.grad, ref_g, rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(fe.hess_diag, np.diag(ref_I), rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(fe.info, ref_I, rtol=0, atol=1e-13 * scale)
    # and it is a different function from Breslow's when events tie
    assert abs(o.neg_loglik_brute(d.X, d.time, d.event, d.stratum, beta) - ref_obj) > 1e-6


def test_efron_finite_differences_of_the_definition():
    d = _tied(120, 3, 3, 77)
    beta = np.array([0.4, -0.2, 0.3])
    g = o.grad_efron_brute(d.X, d.time, d.event, d.stratum, beta)
    H = o.info_efron_brute(d.X, d.time, d.event, d.stratum, beta)
    h = 1e-5
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        fp = o.neg_loglik_efron_brute(d.X, d.time, d.event, d.stratum, beta + e)
        fm = o.neg_loglik_efron_brute(d.X, d.time, d.event, d.stratum, beta - e)
        assert (fp - fm) / (2 * h) == pytest.approx(g[j], rel=1e-7, abs=1e-7)
        gp = o.grad_efron_brute(d.X, d.time, d.event, d.stratum, beta + e)
        gm = o.grad_efron_brute(d.X, d.time, d.event, d.stratum, beta - e)
        np.testing.assert_allclose((gp - gm) / (2 * h), H[:, j], rtol=1e-6, atol=1e-6)
    assert np.linalg.eigvalsh(H).min() > 0


def test_efron_optimum_and_invariances():
    d = _tied(400, 4, 6, 91, round_to=4.0)
    X = np.asfortranarray(d.X)
    nt = o.fit_newton(X, d.time, d.event, d.stratum, ties="efron")
    cd = o.fit_ccd(X, d.time, d.event, d.stratum, ties="efron", tol=1e-14)
    assert nt.converged and cd.converged
    assert np.max(np.abs(cd.beta - nt.beta)) <= 1e-12 * np.max(np.abs(nt.beta))
    g = o.grad_efron_brute(X, d.time, d.event, d.stratum, nt.beta)
    assert np.max(np.abs(g)) <= 1e-10 * d.event.sum()
    # differs from the Breslow optimum on tied data
    assert np.max(np.abs(o.fit_newton(X, d.time, d.event, d.stratum).beta - nt.beta)) > 1e-4
    # row order, stratum labels and a monotone transform of time do not matter
    perm = np.random.default_rng(5).permutation(d.n)
    st2 = (d.stratum * 3 + 11).astype(np.int32)
    nt2 = o.fit_newton(X[perm], np.exp(d.time[perm]), d.event[perm], st2[perm], ties="efron")
    np.testing.assert_allclose(nt2.beta, nt.beta, rtol=1e-12, atol=1e-13)
    # l1: optimality conditions of the penalised Efron objective
    gam = 3.0
    c1 = o.fit_ccd(X, d.time, d.event, d.stratum, ties="efron", gamma=gam, tol=1e-14)
    g1 = o.grad_efron_brute(X, d.time, d.event, d.stratum, c1.beta)
    nz = c1.beta != 0
    np.testing.assert_allclose(g1[nz] + gam * np.sign(c1.beta[nz]), 0.0, atol=1e-9)
    assert np.all(np.abs(g1[~nz]) <= gam + 1e-9)
