"""Pins for the CPU oracle: each test ties it to something other than itself.

What fixes the values here (never the oracle's own formulas retyped):
* the worked segmented-scan example of Sec. 2.6 (tests/golden/segscan_example.txt);
* hand-derived closed forms from Eq. strat_l (tests/golden/toy_closed_forms.txt);
* textbook reductions: the two-group log-rank statistic at beta = 0 (counts),
  and conditional logistic regression for strata of two rows;
* brute force from the definitions (Eqs. strat_l / strat_g / strat_h);
* exact invariances and special cases (K = N, stratum additivity, monotone
  time transforms, shifts and rescaling of a column);
* calculus: finite differences, a zero score / KKT at the optimum, a general
  purpose optimiser (scipy) on the brute-force objective.
"""
import math

import numpy as np
import pytest

from conftest import read_golden
from oracle import cox_oracle as o
from paper_2310_16238_amd import synth


def _layout_py(time, event, stratum):
    """Independent reference for the canonical order: Python's sorted() on tuples."""
    n = len(time)
    order = sorted(range(n), key=lambda i: (int(stratum[i]), -float(time[i]), i))
    head, gend, dcount = [], [0] * n, [0] * n
    for pos, i in enumerate(order):
        head.append(1 if pos == 0 or stratum[order[pos - 1]] != stratum[i] else 0)
    pos = 0
    while pos < n:
        end = pos
        while end + 1 < n and stratum[order[end + 1]] == stratum[order[pos]] and \
                time[order[end + 1]] == time[order[pos]]:
            end += 1
        for q in range(pos, end + 1):
            gend[q] = end
        dcount[end] = sum(int(event[order[q]]) for q in range(pos, end + 1))
        pos = end + 1
    return order, head, gend, dcount


def _small(n=120, p=4, K=3, seed=11, ties=True):
    return synth.make("iid", n, p, K, seed, beta_sd=0.7, tie_round=10.0 if ties else 0.0)


# ------------------------------------------------------------------ scan (Sec. 2.6)

def test_paper_segmented_scan_example():
    g = read_golden("segscan_example.txt")
    a, f, b = [int(v) for v in g["a"]], [int(v) for v in g["f"]], [int(v) for v in g["b"]]
    assert o.segmented_scan(a, f) == b
    np.testing.assert_array_equal(o.segmented_scan_c(np.array(a, float), np.array(f)), np.array(b, float))


def test_seg_op_associative_and_equals_separate_scans():
    rng = np.random.default_rng(3)
    for _ in range(200):
        x, y, z = [(int(rng.integers(0, 2)), int(rng.integers(-50, 50))) for _ in range(3)]
        assert o.seg_op(o.seg_op(x, y), z) == o.seg_op(x, o.seg_op(y, z))
    # one segmented scan == K separate ordinary scans (the naive method the paper rejects)
    for n in [1, 2, 17, 300]:
        a = rng.integers(-1000, 1000, size=n)
        f = (rng.random(n) < 0.2).astype(np.uint8)
        f[0] = 1
        starts = list(np.flatnonzero(f)) + [n]
        sep = np.concatenate([np.cumsum(a[s:e]) for s, e in zip(starts[:-1], starts[1:])])
        assert o.segmented_scan(list(a), list(f)) == list(sep)
        np.testing.assert_array_equal(o.segmented_scan_c(a.astype(float), f), sep.astype(float))


# ------------------------------------------------------------------ layout (Sec. 2.7)

@pytest.mark.parametrize("ties,K", [(False, 1), (True, 1), (True, 7), (True, 60)])
def test_canonical_layout_matches_python_sort(ties, K):
    d = _small(n=240, K=K, ties=ties, seed=5)
    L = o.canonical_layout(d.time, d.event, d.stratum)
    order, head, gend, dcount = _layout_py(d.time, d.event, d.stratum)
    np.testing.assert_array_equal(L.perm, order)
    np.testing.assert_array_equal(L.head, head)
    np.testing.assert_array_equal(L.gend, gend)
    np.testing.assert_array_equal(L.dcount, dcount)
    assert int(L.dcount.sum()) == int(d.event.sum())
    exp_meta = [(h << 31) | (int(d.event[i]) << 30) | c for h, i, c in zip(head, order, dcount)]
    np.testing.assert_array_equal(L.meta, np.array(exp_meta, dtype=np.uint32))


def test_layout_invariant_to_monotone_time_transform():
    d = _small(n=200, K=4, ties=True)
    L1 = o.canonical_layout(d.time, d.event, d.stratum)
    L2 = o.canonical_layout(np.exp(3.0 * d.time) + 7.0, d.event, d.stratum)
    np.testing.assert_array_equal(L1.perm, L2.perm)
    np.testing.assert_array_equal(L1.meta, L2.meta)


# ------------------------------------------------------------------ closed forms

def _toy(prefix):
    g = read_golden("toy_closed_forms.txt")
    X = np.array(g[prefix + ".x"])[:, None]
    return g, X, np.array(g[prefix + ".time"]), np.array(g[prefix + ".event"], dtype=np.uint8)


def test_toy1_closed_forms():
    g, X, t, e = _toy("toy1")
    L = o.canonical_layout(t, e)
    Xc = o.to_canonical(X, L)
    for val in [o.neg_loglik_brute(X, t, e, None, [0.0]), o.coord_terms(Xc, L, 0, np.zeros(3))["obj"],
                o.full_eval(Xc, L, [0.0]).objective]:
        assert val == pytest.approx(g["toy1.negloglik0"][0], rel=1e-15, abs=1e-15)
    assert o.coord_terms(Xc, L, 0, np.zeros(3))["grad"] == pytest.approx(g["toy1.grad0"][0], rel=1e-15)
    assert o.coord_terms(Xc, L, 0, np.zeros(3))["hess"] == pytest.approx(g["toy1.hess0"][0], rel=1e-15)
    assert o.grad_brute(X, t, e, None, [0.0])[0] == pytest.approx(g["toy1.grad0"][0], rel=1e-15)
    assert o.hess_diag_brute(X, t, e, None, [0.0])[0] == pytest.approx(g["toy1.hess0"][0], rel=1e-15)
    bh = g["toy1.betahat"][0]
    assert o.fit_ccd(X, t, e, tol=1e-15).beta[0] == pytest.approx(bh, abs=1e-14)
    assert o.fit_newton(X, t, e).beta[0] == pytest.approx(bh, abs=1e-14)


def test_toy2_breslow_ties():
    g, X, t, e = _toy("toy2")
    for order in [[0, 1, 2], [1, 0, 2], [2, 1, 0]]:   # input order must not matter
        Xo, to, eo = X[order], t[order], e[order]
        L = o.canonical_layout(to, eo)
        Xc = o.to_canonical(Xo, L)
        c = o.coord_terms(Xc, L, 0, np.zeros(3))
        assert c["grad"] == pytest.approx(g["toy2.grad0"][0], rel=1e-15)
        assert c["hess"] == pytest.approx(g["toy2.hess0"][0], rel=1e-15)
        assert c["obj"] == pytest.approx(g["toy2.negloglik0"][0], rel=1e-15)
        assert o.grad_brute(Xo, to, eo, None, [0.0])[0] == pytest.approx(g["toy2.grad0"][0], rel=1e-15)
        fe = o.full_eval(Xc, L, [0.0])
        assert fe.grad[0] == pytest.approx(g["toy2.grad0"][0], rel=1e-15)
        assert fe.hess_diag[0] == pytest.approx(g["toy2.hess0"][0], rel=1e-15)


def test_logrank_at_zero_binary_covariate():
    """At beta = 0 with a 0/1 covariate, g' = -(O - E) and g'' = V of the log-rank test.

    Textbook counting form: at each distinct event time t of a stratum, n_t at
    risk, n1_t of them with x = 1, d_t events; E = sum d_t n1_t / n_t and
    V = sum d_t (n1_t / n_t)(1 - n1_t / n_t) (the Breslow-type variance).
    """
    rng = np.random.default_rng(8)
    n, K = 400, 5
    x = (rng.random(n) < 0.4).astype(float)
    time = np.floor(rng.exponential(1.0, n) * 8) / 8      # many ties
    event = (rng.random(n) < 0.6).astype(np.uint8)
    stratum = rng.integers(0, K, n)
    O = E = V = 0.0
    for k in range(K):
        ins = stratum == k
        for t in np.unique(time[ins & (event == 1)]):
            at_risk = ins & (time >= t)
            died = ins & (time == t) & (event == 1)
            nt, n1 = at_risk.sum(), (at_risk & (x == 1)).sum()
            dt = died.sum()
            O += (died & (x == 1)).sum()
            E += dt * n1 / nt
            V += dt * (n1 / nt) * (1 - n1 / nt)
    L = o.canonical_layout(time, event, stratum)
    Xc = o.to_canonical(x[:, None], L)
    c = o.coord_terms(Xc, L, 0, np.zeros(n))
    assert c["grad"] == pytest.approx(-(O - E), rel=1e-12, abs=1e-12)
    assert c["hess"] == pytest.approx(V, rel=1e-12)


def _logistic_fit(Z):
    """Plain Newton for logistic regression without intercept, all labels 1."""
    b = np.zeros(Z.shape[1])
    for _ in range(100):
        pr = 1.0 / (1.0 + np.exp(Z @ b))           # 1 - sigmoid(z'b)
        grad = -(Z.T @ pr)
        W = pr * (1 - pr)
        H = (Z.T * W) @ Z
        step = np.linalg.solve(H, grad)
        b -= step
        if np.max(np.abs(step)) < 1e-15 * max(1.0, np.max(np.abs(b))):
            break
    return b


def test_pairs_equal_conditional_logistic():
    """K = N/2 strata of two rows: -log L = sum_{pairs, earlier row an event} log(1 + exp(-(x_a - x_b)'b))."""
    rng = np.random.default_rng(21)
    npair, p = 1500, 3
    X = rng.standard_normal((2 * npair, p))
    time = rng.exponential(1.0, 2 * npair)
    event = (rng.random(2 * npair) < 0.7).astype(np.uint8)
    stratum = np.repeat(np.arange(npair), 2)
    Z = []
    for k in range(npair):
        a, b = 2 * k, 2 * k + 1
        if time[a] > time[b]:
            a, b = b, a                         # a is the earlier (shorter) time
        if event[a]:
            Z.append(X[a] - X[b])
    Z = np.array(Z)
    beta = np.array([0.3, -0.2, 0.5])
    ll_logit = np.sum(np.log1p(np.exp(-(Z @ beta))))
    L = o.canonical_layout(time, event, stratum)
    Xc = o.to_canonical(X, L)
    assert o.full_eval(Xc, L, beta).objective == pytest.approx(ll_logit, rel=1e-12)
    b_logit = _logistic_fit(Z)
    b_newton = o.fit_newton(X, time, event, stratum, layout=L, Xc=Xc).beta
    b_ccd = o.fit_ccd(X, time, event, stratum, layout=L, Xc=Xc, tol=1e-14).beta
    assert np.max(np.abs(b_newton - b_logit)) <= 1e-12 * np.max(np.abs(b_logit))
    assert np.max(np.abs(b_ccd - b_logit)) <= 1e-11 * np.max(np.abs(b_logit))


def test_singleton_strata_give_zero():
    """Every risk set is a single row: each ratio is 1 (or x_i), so all terms vanish (to rounding)."""
    d = _small(n=50, K=50)
    L = o.canonical_layout(d.time, d.event, d.stratum)
    Xc = o.to_canonical(d.X, L)
    beta = np.array([0.4, -1.0, 2.0, 0.1])
    fe = o.full_eval(Xc, L, beta)
    tol = 1e-14 * 50 * (1 + np.abs(d.X).max()) ** 2
    assert abs(fe.objective) <= tol
    assert np.all(np.abs(fe.grad) <= tol) and np.all(np.abs(fe.hess_diag) <= tol)
    eta = Xc @ beta
    for j in range(4):
        c = o.coord_terms(Xc, L, j, eta)
        assert abs(c["grad"]) <= tol and abs(c["hess"]) <= tol and abs(c["obj"]) <= tol


def test_intercept_column_is_exactly_degenerate():
    d = synth.config_small(n=500, K=4, ties=True)
    L = o.canonical_layout(d.time, d.event, d.stratum)
    Xc = o.to_canonical(d.X, L)
    eta = Xc @ (0.3 * d.beta_true)
    c = o.coord_terms(Xc, L, 0, eta)
    assert c["grad"] == 0.0 and c["hess"] == 0.0
    assert o.degenerate_columns(Xc, L)[0] and not o.degenerate_columns(Xc, L)[1:].any()


# ------------------------------------------------------------------ brute force vs scan form

@pytest.mark.parametrize("K,ties", [(1, False), (1, True), (6, True), (40, True)])
def test_scan_form_equals_definition(K, ties):
    d = _small(n=160, p=4, K=K, ties=ties, seed=K)
    beta = np.array([0.5, -0.8, 0.2, 1.1])
    L = o.canonical_layout(d.time, d.event, d.stratum)
    Xc = o.to_canonical(d.X, L)
    ref_obj = o.neg_loglik_brute(d.X, d.time, d.event, d.stratum, beta)
    ref_g = o.grad_brute(d.X, d.time, d.event, d.stratum, beta)
    ref_h = o.hess_diag_brute(d.X, d.time, d.event, d.stratum, beta)
    ref_I = o.info_brute(d.X, d.time, d.event, d.stratum, beta)
    eta = Xc @ beta
    scale = max(1.0, float(d.event.sum()))
    for j in range(4):
        c = o.coord_terms(Xc, L, j, eta)
        assert abs(c["grad"] - ref_g[j]) <= 1e-13 * scale
        assert abs(c["hess"] - ref_h[j]) <= 1e-13 * scale
        assert abs(c["obj"] - ref_obj) <= 1e-13 * scale
    fe = o.full_eval(Xc, L, beta)
    assert abs(fe.objective - ref_obj) <= 1e-13 * scale
    np.testing.assert_allclose(fe.grad, ref_g, rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(fe.hess_diag, ref_h, rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(fe.info, ref_I, rtol=0, atol=1e-13 * scale)


def test_extreme_linear_predictor_is_finite():
    """A per-stratum shift keeps exp() in range where exp(x'b) itself overflows."""
    d = _small(n=80, p=2, K=2, ties=False)
    X = np.asfortranarray(d.X * 400.0)
    beta = np.array([2.0, -1.5])                      # |x'b| reaches thousands
    L = o.canonical_layout(d.time, d.event, d.stratum)
    Xc = o.to_canonical(X, L)
    fe = o.full_eval(Xc, L, beta)
    assert np.isfinite(fe.objective) and np.all(np.isfinite(fe.grad))
    # same values as the definition evaluated with the shift done by hand per event
    eta = X @ beta
    ref = 0.0
    for i in range(80):
        if d.event[i]:
            R = (d.stratum == d.stratum[i]) & (d.time >= d.time[i])
            mx = eta[R].max()
            ref -= eta[i] - (mx + np.log(np.sum(np.exp(eta[R] - mx))))
    assert fe.objective == pytest.approx(ref, rel=1e-12)


# ------------------------------------------------------------------ structure

def test_stratum_additivity():
    d = _small(n=300, K=5, ties=True)
    beta = np.array([0.2, 0.7, -0.4, 0.0])
    whole = o.neg_loglik_brute(d.X, d.time, d.event, d.stratum, beta)
    L = o.canonical_layout(d.time, d.event, d.stratum)
    fe = o.full_eval(o.to_canonical(d.X, L), L, beta)
    parts, gparts = 0.0, np.zeros(4)
    for k in range(5):
        m = d.stratum == k
        Lk = o.canonical_layout(d.time[m], d.event[m])
        fk = o.full_eval(o.to_canonical(d.X[m], Lk), Lk, beta)
        parts += fk.objective
        gparts += fk.grad
    assert fe.objective == pytest.approx(parts, rel=1e-13)
    assert whole == pytest.approx(parts, rel=1e-12)
    np.testing.assert_allclose(fe.grad, gparts, rtol=1e-12, atol=1e-12)


def test_invariances():
    d = _small(n=200, K=4, ties=True, seed=2)
    beta = np.array([0.3, -0.6, 0.9, 0.15])
    L = o.canonical_layout(d.time, d.event, d.stratum)
    base = o.full_eval(o.to_canonical(d.X, L), L, beta)
    tol = dict(rtol=1e-12, atol=1e-12)
    # row permutation
    rng = np.random.default_rng(0)
    q = rng.permutation(200)
    Lq = o.canonical_layout(d.time[q], d.event[q], d.stratum[q])
    fq = o.full_eval(o.to_canonical(d.X[q], Lq), Lq, beta)
    np.testing.assert_allclose(fq.grad, base.grad, **tol)
    assert fq.objective == pytest.approx(base.objective, rel=1e-13)
    # stratum relabelling (order of strata changes)
    relab = np.array([17, -3, 5, 2])[d.stratum]
    Lr = o.canonical_layout(d.time, d.event, relab)
    fr = o.full_eval(o.to_canonical(d.X, Lr), Lr, beta)
    np.testing.assert_allclose(fr.grad, base.grad, **tol)
    np.testing.assert_allclose(fr.info, base.info, **tol)
    # strictly increasing transform of time
    Lt = o.canonical_layout(np.log1p(d.time) * 5 - 2, d.event, d.stratum)
    ft = o.full_eval(o.to_canonical(d.X, Lt), Lt, beta)
    np.testing.assert_allclose(ft.grad, base.grad, **tol)
    # shifting a column by a constant leaves gradient and Hessian unchanged
    Xs = d.X.copy(order="F")
    Xs[:, 2] += 3.0
    fs = o.full_eval(o.to_canonical(Xs, L), L, beta)
    np.testing.assert_allclose(fs.grad, base.grad, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(fs.hess_diag, base.hess_diag, rtol=1e-10, atol=1e-10)
    # rescaling a column by s with beta_j / s: same objective, gradient scaled by s
    Xm = d.X.copy(order="F")
    Xm[:, 1] *= 4.0
    bm = beta.copy()
    bm[1] /= 4.0
    fm = o.full_eval(o.to_canonical(Xm, L), L, bm)
    assert fm.objective == pytest.approx(base.objective, rel=1e-13)
    assert fm.grad[1] == pytest.approx(4.0 * base.grad[1], rel=1e-12)


def test_information_symmetric_psd_and_diag():
    d = _small(n=250, p=5, K=3, ties=True, seed=9)
    beta = np.array([0.2, -0.3, 0.5, 0.8, -0.1])
    L = o.canonical_layout(d.time, d.event, d.stratum)
    fe = o.full_eval(o.to_canonical(d.X, L), L, beta)
    I = fe.info
    np.testing.assert_allclose(I, I.T, rtol=0, atol=1e-12 * np.abs(I).max())
    assert np.linalg.eigvalsh(I).min() >= -1e-12 * np.abs(I).max()
    np.testing.assert_allclose(np.diag(I), fe.hess_diag, rtol=1e-12)


def test_finite_differences():
    d = _small(n=150, p=3, K=3, ties=True, seed=4)
    beta = np.array([0.4, -0.2, 0.3])
    L = o.canonical_layout(d.time, d.event, d.stratum)
    Xc = o.to_canonical(d.X, L)
    fe = o.full_eval(Xc, L, beta)
    h = 1e-5
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        fp, fm = o.full_eval(Xc, L, beta + e), o.full_eval(Xc, L, beta - e)
        assert (fp.objective - fm.objective) / (2 * h) == pytest.approx(fe.grad[j], rel=1e-7, abs=1e-7)
        np.testing.assert_allclose((fp.grad - fm.grad) / (2 * h), fe.info[:, j], rtol=1e-6, atol=1e-6)


# ------------------------------------------------------------------ optimum

def test_unpenalised_optimum_zero_score_and_scipy_agree():
    from scipy.optimize import minimize
    d = synth.config_small(n=400, K=3, ties=True)
    X = d.X[:, 1:5]          # drop the ones column: brute force on an identifiable design
    Xf = np.asfortranarray(X)
    res_ccd = o.fit_ccd(Xf, d.time, d.event, d.stratum, tol=1e-14)
    res_nt = o.fit_newton(Xf, d.time, d.event, d.stratum)
    g = o.grad_brute(X, d.time, d.event, d.stratum, res_nt.beta)
    assert np.max(np.abs(g)) <= 1e-10 * d.event.sum()
    assert np.max(np.abs(res_ccd.beta - res_nt.beta)) <= 1e-12 * np.max(np.abs(res_nt.beta))
    sp = minimize(lambda b: o.neg_loglik_brute(X, d.time, d.event, d.stratum, b), np.zeros(4),
                  jac=lambda b: o.grad_brute(X, d.time, d.event, d.stratum, b), method="BFGS",
                  options={"gtol": 1e-10})
    np.testing.assert_allclose(sp.x, res_nt.beta, rtol=1e-6, atol=1e-6)


def test_l1_optimum_satisfies_kkt():
    d = synth.config_small(n=600, K=5, ties=True)
    gamma = math.sqrt(2.0)
    X = np.asfortranarray(d.X[:, 1:])
    # a weak column so that the l1 solution has an exact zero
    X[:, 0] = np.random.default_rng(1).standard_normal(X.shape[0]) * 0.01
    res = o.fit_ccd(X, d.time, d.event, d.stratum, gamma=gamma, tol=1e-14)
    assert res.converged
    g = o.grad_brute(X, d.time, d.event, d.stratum, res.beta)
    nz = res.beta != 0
    assert (~nz).any() and nz.any()
    np.testing.assert_allclose(g[nz] + gamma * np.sign(res.beta[nz]), 0.0, atol=1e-9)
    assert np.all(np.abs(g[~nz]) <= gamma + 1e-9)
    # objective at the estimate is not beaten by small moves along each coordinate
    F = lambda b: o.neg_loglik_brute(X, d.time, d.event, d.stratum, b) + gamma * np.abs(b).sum()
    f0 = F(res.beta)
    for j in range(X.shape[1]):
        for s in (1e-4, -1e-4):
            b = res.beta.copy()
            b[j] += s
            assert F(b) >= f0 - 1e-10


def test_penalize_mask_and_ccd_step_rules():
    # beta = 0 and |g'| <= gamma: no move; directional derivative g'+gamma < 0: move up
    assert o.ccd_step(0.0, 0.5, 2.0, 3.0, 1.0, 1.0)[0] == 0.0
    s, t = o.ccd_step(0.0, -3.0, 2.0, 3.0, 1.0, 10.0)
    assert s == pytest.approx(1.0) and t == pytest.approx(5.0)
    s, _ = o.ccd_step(0.0, 3.0, 2.0, 3.0, 1.0, 10.0)
    assert s == pytest.approx(-1.0)
    # a step that would cross zero stops at zero
    s, _ = o.ccd_step(0.1, 5.0, 1.0, 3.0, 1.0, 10.0)
    assert s == pytest.approx(-0.1)
    # trust region clips, then halves when the applied step is small
    s, t = o.ccd_step(0.0, -100.0, 1.0, 3.0, 0.0, 0.25)
    assert s == 0.25 and t == 0.5
    s, t = o.ccd_step(0.0, -1e-3, 1.0, 3.0, 0.0, 1.0)
    assert s == pytest.approx(1e-3) and t == 0.5
    # degenerate curvature: no move
    assert o.ccd_step(0.0, -1.0, 0.0, 3.0, 0.0, 1.0)[0] == 0.0
