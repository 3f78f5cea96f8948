"""Resampled handles, cross-validation and bootstrap on the GPU (Secs. 2.1, 3.2) against
the oracle on the explicitly repeated data.

* layout of a resampled handle: bit-exact against the oracle's canonical order of the
  data with row i repeated count[i] times (folds, bootstrap counts, dropped strata and
  dropped tie groups with events);
* fits and evaluations on it: FP64 tolerances as for every fit (max|gpu - oracle| /
  max|oracle| <= 1e-10, l1 zero pattern exact, objective 1e-11 relative);
* cross-validated log likelihood: |gpu - oracle| <= 1e-11 sum_k (|l| + |l_{-k}|): each term
  is a difference of two FP64 log likelihoods (rounding ~1e-13 of their size), and the fold
  estimates, equal to 1e-10 relative, enter l(beta) to first order through the held-out
  rows' score, whose size is a small fraction of |l|.
"""
import numpy as np
import pytest

from oracle import cox_oracle as orc
from paper_2310_16238_amd import coxmi, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    coxmi.lib()


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b))))


def _counts(kind, d, seed=0):
    n = d.time.shape[0]
    rng = np.random.default_rng(seed)
    if kind == "fold":
        return (rng.integers(0, 10, n) != 3).astype(np.uint32)
    if kind == "bootstrap":
        return rng.multinomial(n, np.full(n, 1.0 / n)).astype(np.uint32)
    if kind == "drop_stratum":
        c = np.ones(n, np.uint32)
        c[d.stratum == d.stratum[0]] = 0
        return c
    if kind == "drop_event_groups":
        # remove every row of the tie groups holding events at a set of times
        c = np.ones(n, np.uint32)
        ev_t = np.unique(d.time[d.event == 1])
        gone = np.isin(d.time, ev_t[::3])
        c[gone] = 0
        c[::17] = 3
        return c
    raise ValueError(kind)


KINDS = ["fold", "bootstrap", "drop_stratum", "drop_event_groups"]


@pytest.mark.parametrize("kind", KINDS)
def test_resampled_layout_and_fit(kind):
    d = synth.make("ar1", 30_000, 6, 40, 21, beta_sd=0.5, tie_round=100.0)
    cnt = _counts(kind, d)
    Xr, tr, er, sr = orc.resample(d.X, d.time, d.event, d.stratum, cnt)
    L = orc.canonical_layout(tr, er, sr)
    _say(f"resample {kind}: n={len(tr)}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, gamma=2.0, tol=1e-13) as m:
        with m.resample(cnt) as c:
            perm, meta = c.layout()
            np.testing.assert_array_equal(perm, L.perm)
            np.testing.assert_array_equal(meta, L.meta)
            beta, info = c.fit()
    ref = orc.fit_ccd(Xr, tr, er, sr, gamma=2.0, tol=1e-13)
    assert ref.converged and info["status"] == coxmi.COX_OK
    assert np.array_equal(beta == 0.0, ref.beta == 0.0)
    err = _rel(beta, ref.beta)
    _say(f"  sweeps={info['iters']} rel err {err:.3e}")
    assert err <= 1e-10


def test_resample_options_newton_and_penalty():
    d = synth.make("iid", 20_000, 5, 20, 23, beta_sd=0.5, tie_round=50.0)
    cnt = _counts("bootstrap", d, seed=4)
    Xr, tr, er, sr = orc.resample(d.X, d.time, d.event, d.stratum, cnt)
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum) as m:
        with m.resample(cnt, mode=coxmi.COX_NEWTON_REFINE, tol=1e-13, max_iter=100) as c:
            beta, info = c.fit()
            obj, g, _, _ = c.evaluate_full(beta, want_info=False)
        ref = orc.fit_newton(Xr, tr, er, sr, tol=1e-14)
        assert info["status"] == coxmi.COX_OK and _rel(beta, ref.beta) <= 1e-10
        assert abs(obj - ref.objective) <= 1e-11 * abs(ref.objective)
        pen = np.array([0, 1, 1, 1, 1], np.uint8)
        with m.resample(cnt, gamma=5.0, penalize=pen, tol=1e-13) as c:
            b5, _ = c.fit()
            c.set_penalty(1.0, pen)
            b1, _ = c.fit(beta0=b5)
        for gam, b in ((5.0, b5), (1.0, b1)):
            r = orc.fit_ccd(Xr, tr, er, sr, gamma=gam, penalize=pen, tol=1e-13)
            assert np.array_equal(b == 0.0, r.beta == 0.0) and _rel(b, r.beta) <= 1e-10


def test_cross_validation_matches_oracle():
    d = synth.make("binary", 40_000, 30, 20, 25, beta_sd=1.0, beta_nonzero=0.3, density=0.1, tie_round=50.0)
    fold = np.random.default_rng(9).integers(0, 5, d.time.shape[0]).astype(np.int32)
    gammas = np.array([60.0, 20.0, 6.0, 2.0, 0.5])
    pen = np.ones(30, np.uint8)
    pen[0] = 0
    _say("cross-validation: 5 folds x 5 gammas, n=40000 p=30")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, tol=1e-13) as m:
        cvl, betas, status = m.cross_validate(fold, gammas, pen)
    rcvl, rbetas, rconv = orc.cross_validate(d.X, d.time, d.event, d.stratum, fold, gammas, pen, tol=1e-13)
    assert rconv.all() and np.all(status == coxmi.COX_OK)
    for k in range(5):
        for g in range(len(gammas)):
            assert np.array_equal(betas[k, g] == 0.0, rbetas[k, g] == 0.0), (k, g)
            assert _rel(betas[k, g], rbetas[k, g]) <= 1e-10, (k, g)
    nll_all = orc.neg_loglik(d.X, d.time, d.event, d.stratum, np.zeros(30))
    scale = 2.0 * 5 * abs(nll_all)
    err = float(np.max(np.abs(cvl - rcvl)))
    _say(f"  cvl {np.round(cvl, 3)}; max |gpu - oracle| {err:.3e} (bound {1e-11 * scale:.3e})")
    assert err <= 1e-11 * scale
    assert int(np.argmax(cvl)) == int(np.argmax(rcvl))


def test_cross_validation_through_the_server():
    """The same l1 path with the fold fits batched through a fit server (every fold of one weight
    in one batch, warm-started from the previous weight): fold estimates at the oracle's to 1e-10
    with the same zero patterns, and the criterion within the same bound as above."""
    d = synth.make("binary", 40_000, 30, 20, 25, beta_sd=1.0, beta_nonzero=0.3, density=0.1, tie_round=50.0)
    fold = np.random.default_rng(9).integers(0, 5, d.time.shape[0]).astype(np.int32)
    gammas = np.array([60.0, 20.0, 6.0, 2.0, 0.5])
    pen = np.ones(30, np.uint8)
    pen[0] = 0
    _say("cross-validation through the server: 5 folds x 5 gammas, n=40000 p=30")
    with coxmi.CoxServer(hbm_budget=1 << 30, staging_bytes=256 << 20, prep_threads=4) as srv:
        with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, tol=1e-13) as m:
            cvl, betas, status = m.cross_validate_served(srv, d.X, d.time, d.event, d.stratum, fold, gammas, pen)
            with pytest.raises(coxmi.CoxError) as e:   # data of another shape than the handle's
                m.cross_validate_served(srv, d.X[:, :5], d.time, d.event, d.stratum, fold, gammas, pen[:5])
            assert e.value.code == coxmi.COX_EINVAL
    rcvl, rbetas, rconv = orc.cross_validate(d.X, d.time, d.event, d.stratum, fold, gammas, pen, tol=1e-13)
    assert rconv.all() and np.all(status == coxmi.COX_OK)
    worst = 0.0
    for k in range(5):
        for g in range(len(gammas)):
            assert np.array_equal(betas[k, g] == 0.0, rbetas[k, g] == 0.0), (k, g)
            err = _rel(betas[k, g], rbetas[k, g])
            assert err <= 1e-10, (k, g, err)
            worst = max(worst, err)
    nll_all = orc.neg_loglik(d.X, d.time, d.event, d.stratum, np.zeros(30))
    scale = 2.0 * 5 * abs(nll_all)
    err = float(np.max(np.abs(cvl - rcvl)))
    _say(f"  worst fold rel err {worst:.2e}; max |cvl - oracle| {err:.3e} (bound {1e-11 * scale:.3e})")
    assert err <= 1e-11 * scale
    assert int(np.argmax(cvl)) == int(np.argmax(rcvl))


def test_bootstrap_matches_oracle():
    d = synth.make("iid", 15_000, 8, 15, 27, beta_sd=0.5, tie_round=100.0)
    n = d.time.shape[0]
    rng = np.random.default_rng(11)
    counts = np.stack([rng.multinomial(n, np.full(n, 1.0 / n)) for _ in range(6)]).astype(np.uint32)
    _say("bootstrap: 6 replicates, n=15000 p=8, gamma=3")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, gamma=3.0, tol=1e-13) as m:
        betas, status = m.bootstrap(counts)
    rb, rconv = orc.bootstrap(d.X, d.time, d.event, d.stratum, counts, gamma=3.0, tol=1e-13)
    assert rconv.all() and np.all(status == coxmi.COX_OK)
    for b in range(6):
        assert np.array_equal(betas[b] == 0.0, rb[b] == 0.0) and _rel(betas[b], rb[b]) <= 1e-10
    lo, hi = orc.percentile_interval(np.exp(betas), 0.95)
    rlo, rhi = orc.percentile_interval(np.exp(rb), 0.95)
    assert np.allclose(lo, rlo, rtol=1e-9, atol=0) and np.allclose(hi, rhi, rtol=1e-9, atol=0)


def test_resample_and_cv_errors():
    d = synth.make("iid", 2000, 3, 2, 29)
    n = d.time.shape[0]
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum) as m:
        with pytest.raises(coxmi.CoxError) as e:
            m.resample(np.zeros(n, np.uint32))
        assert e.value.code == coxmi.COX_EINVAL
        with pytest.raises(ValueError):
            m.resample(np.ones(n - 1, np.uint32))
        bad = np.zeros(n, np.int32)
        bad[0] = 7
        with pytest.raises(coxmi.CoxError) as e:
            m.cross_validate(bad, [1.0], nfolds=3)
        assert e.value.code == coxmi.COX_EINVAL
        with pytest.raises(coxmi.CoxError) as e:
            m.cross_validate(np.zeros(n, np.int32), [1.0], nfolds=2)    # fold 1 empty
        assert e.value.code == coxmi.COX_EINVAL
        with pytest.raises(coxmi.CoxError) as e:
            m.set_penalty(-1.0)
        assert e.value.code == coxmi.COX_EINVAL


def test_cross_validation_newton_bf16_matches_oracle():
    """The same cross-validation with proximal Newton fits and a BF16 information matrix: the
    fold optima are the same, so the criterion and the estimates match the oracle's CCD path."""
    d = synth.make("binary", 30_000, 20, 10, 31, beta_sd=1.0, beta_nonzero=0.3, density=0.1, tie_round=50.0)
    fold = np.random.default_rng(13).integers(0, 4, d.time.shape[0]).astype(np.int32)
    gammas = np.array([40.0, 10.0, 2.0])
    pen = np.ones(20, np.uint8)
    pen[0] = 0
    _say("cross-validation by proximal Newton (BF16): 4 folds x 3 gammas, n=30000 p=20")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE,
                        x_precision=coxmi.COX_BF16, tol=1e-13, max_iter=300) as m:
        cvl, betas, status = m.cross_validate(fold, gammas, pen)
    rcvl, rbetas, rconv = orc.cross_validate(d.X, d.time, d.event, d.stratum, fold, gammas, pen, tol=1e-14)
    assert rconv.all() and np.all(status == coxmi.COX_OK)
    for k in range(4):
        for g in range(len(gammas)):
            assert np.array_equal(betas[k, g] == 0.0, rbetas[k, g] == 0.0), (k, g)
            assert _rel(betas[k, g], rbetas[k, g]) <= 1e-10, (k, g)
    nll_all = orc.neg_loglik(d.X, d.time, d.event, d.stratum, np.zeros(20))
    err = float(np.max(np.abs(cvl - rcvl)))
    _say(f"  max |gpu - oracle| {err:.3e}")
    assert err <= 1e-11 * 2.0 * 4 * abs(nll_all)
