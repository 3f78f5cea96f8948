"""GPU fits of models with step-function coefficients and piecewise-constant
covariates (Secs. 2.2-2.3), on the interval-stratified augmented data that
cox_split_intervals builds, against the oracle's fits of the oracle's own
augmentation.

Workload: the Sec. 3.3 setting in miniature -- one covariate whose coefficient
changes at a cut (two intervals), the rest time-fixed -- and a K = 4 version
with a time-varying covariate; times with ties, several original strata.
Tolerance as for every FP64 fit: max|gpu - oracle| / max|oracle| <= 1e-10 with
the oracle's Newton / CCD fit run to 1e-14 / 1e-13.
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


def _case(kind):
    if kind == "step_coef_2":
        d = synth.make("binary", 6000, 12, 6, 101, beta_sd=0.5, density=0.2, tie_round=50.0)
        cuts = [float(np.quantile(d.time, 0.5))]
        tv = np.zeros(12, np.uint8)
        tv[0] = 1
        return d, cuts, tv, None
    d = synth.make("iid", 4000, 6, 3, 103, beta_sd=0.4, tie_round=20.0)
    cuts = [float(q) for q in np.quantile(d.time, [0.25, 0.5, 0.75])]
    rng = np.random.default_rng(7)
    XK = [d.X.copy() for _ in range(4)]
    for k in range(4):
        XK[k][:, 2] += 0.3 * k + rng.normal(0, 0.2, d.X.shape[0])   # a covariate measured again each interval
    tv = np.array([0, 1, 0, 0, 0, 0], np.uint8)
    return d, cuts, tv, XK


@pytest.mark.parametrize("kind", ["step_coef_2", "tv_cov_4"])
@pytest.mark.parametrize("mode", ["newton", "ccd"])
def test_interval_fit_matches_oracle(kind, mode):
    d, cuts, tv, XK = _case(kind)
    a = coxmi.split_intervals(d.X, d.time, d.event, d.stratum, cuts, tv_coef=tv, X_by_interval=XK)
    r = orc.split_intervals(d.X, d.time, d.event, d.stratum, cuts, tv_coef=tv, X_by_interval=XK)
    assert np.array_equal(a["X"], r["X"]) and np.array_equal(a["stratum"], r["stratum"])
    _say(f"interval fit {kind} {mode}: n_aug={a['X'].shape[0]} p_aug={a['X'].shape[1]} "
         f"strata={len(np.unique(a['stratum']))}")
    if mode == "newton":
        with coxmi.CoxModel(a["X"], a["time"], a["event"], a["stratum"], mode=coxmi.COX_NEWTON_REFINE,
                            tol=1e-13, max_iter=200) as m:
            beta, info = m.fit()
        ref = orc.fit_newton(r["X"], r["time"], r["event"], r["stratum"], tol=1e-14)
    else:
        with coxmi.CoxModel(a["X"], a["time"], a["event"], a["stratum"], tol=1e-13) as m:
            beta, info = m.fit()
        ref = orc.fit_ccd(r["X"], r["time"], r["event"], r["stratum"], tol=1e-13)
    assert ref.converged
    assert info["status"] == coxmi.COX_OK, info
    err = _rel(beta, ref.beta)
    _say(f"  iters={info['iters']} rel err {err:.3e}")
    assert err <= 1e-10


def test_step_effect_l1_fit_matches_oracle():
    """The Sec. 3.3 model in miniature: a treatment coefficient that steps at 10 days, l1 on
    every column but the two treatment columns, CCD to convergence on the two interval strata."""
    d = synth.config_step_effect(n=30_000, p=40)
    tv = np.zeros(40, np.uint8)
    tv[0] = 1
    a = coxmi.split_intervals(d.X, d.time, d.event, None, [10.0], tv_coef=tv)
    r = orc.split_intervals(d.X, d.time, d.event, None, [10.0], tv_coef=tv)
    assert np.array_equal(a["X"], r["X"]) and np.array_equal(a["time"], r["time"])
    pen = np.ones(a["X"].shape[1], np.uint8)
    pen[a["col_source"] == 0] = 0
    _say(f"step-effect l1 fit: n_aug={a['X'].shape[0]} p_aug={a['X'].shape[1]}")
    with coxmi.CoxModel(a["X"], a["time"], a["event"], a["stratum"], gamma=d.gamma, penalize=pen, tol=1e-13) as m:
        beta, info = m.fit()
    ref = orc.fit_ccd(r["X"], r["time"], r["event"], r["stratum"], gamma=d.gamma, penalize=pen, tol=1e-13)
    assert ref.converged and info["status"] == coxmi.COX_OK
    assert np.array_equal(beta == 0.0, ref.beta == 0.0)
    err = _rel(beta, ref.beta)
    _say(f"  iters={info['iters']} nonzero={int(np.count_nonzero(beta))} rel err {err:.3e}")
    assert err <= 1e-10


@pytest.mark.parametrize("strata", [False, True])
def test_device_mapping_matches_split(strata):
    """cox_init_intervals (augmented X gathered on the device from the parent's columns) against
    the host split: identical canonical layout, fits equal to the oracle's on its own split."""
    d = synth.make("ar1", 20_000, 7, 12, 105, beta_sd=0.4, tie_round=50.0)
    st = d.stratum if strata else None
    cuts = [float(q) for q in np.quantile(d.time, [0.3, 0.6])]
    tv = np.array([1, 0, 0, 1, 0, 0, 0], np.uint8)
    r = orc.split_intervals(d.X, d.time, d.event, st, cuts, tv_coef=tv)
    L = orc.canonical_layout(r["time"], r["event"], r["stratum"])
    pa = r["X"].shape[1]
    pen = np.ones(pa, np.uint8)
    pen[r["col_source"] == 0] = 0
    _say(f"device interval mapping strata={strata}: n_aug={r['X'].shape[0]} p_aug={pa}")
    with coxmi.CoxModel(d.X, d.time, d.event, st) as m:
        with m.intervals(d.time, d.event, st, cuts, tv, gamma=1.5, penalize=pen, tol=1e-13) as c:
            perm, meta = c.layout()
            np.testing.assert_array_equal(perm, L.perm)
            np.testing.assert_array_equal(meta, L.meta)
            beta, info = c.fit()
            obj, _, _ = c.evaluate(beta)
        with m.intervals(d.time, d.event, st, cuts, tv, mode=coxmi.COX_NEWTON_REFINE, tol=1e-13) as c:
            bn, infon = c.fit()
    ref = orc.fit_ccd(r["X"], r["time"], r["event"], r["stratum"], gamma=1.5, penalize=pen, tol=1e-13)
    assert ref.converged and info["status"] == coxmi.COX_OK
    assert np.array_equal(beta == 0.0, ref.beta == 0.0) and _rel(beta, ref.beta) <= 1e-10
    refn = orc.fit_newton(r["X"], r["time"], r["event"], r["stratum"], tol=1e-14)
    assert infon["status"] == coxmi.COX_OK and _rel(bn, refn.beta) <= 1e-10
    _say(f"  ccd rel err {_rel(beta, ref.beta):.3e}, newton rel err {_rel(bn, refn.beta):.3e}")


def test_device_mapping_errors():
    d = synth.make("iid", 3000, 3, 3, 107)
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum) as m:
        ev = d.event.copy()
        ev[np.flatnonzero(ev)[0]] = 0
        with pytest.raises(coxmi.CoxError) as e:
            m.intervals(d.time, ev, d.stratum, [0.5])
        assert e.value.code == coxmi.COX_EINVAL
        with pytest.raises(coxmi.CoxError) as e:
            m.intervals(d.time, d.event, d.stratum, [2.0, 1.0])
        assert e.value.code == coxmi.COX_EINVAL
        # keys other than the parent's: permuted times, a merged tie group, other strata
        rng = np.random.default_rng(3)
        bad_time = [rng.permutation(d.time), d.time.copy()]
        perm, meta = m.layout()
        c = next(c for c in range(d.n - 1) if d.event[perm[c]] and d.event[perm[c + 1]] and not meta[c + 1] >> 31)
        bad_time[1][perm[c + 1]] = d.time[perm[c]]     # two events of one stratum merged into a tie group
        for t in bad_time:
            with pytest.raises(coxmi.CoxError) as e:
                m.intervals(t, d.event, d.stratum, [0.5])
            assert e.value.code == coxmi.COX_EINVAL
        for st in [None, (d.stratum + 1) % 3, np.where(np.arange(d.n) == 5, d.stratum + 7, d.stratum)]:
            with pytest.raises(coxmi.CoxError) as e:
                m.intervals(d.time, d.event, None if st is None else st.astype(np.int32), [0.5])
            assert e.value.code == coxmi.COX_EINVAL
        # relabelled strata in the same order are the same strata
        with m.intervals(d.time, d.event, (d.stratum * 5 + 2).astype(np.int32), [0.5]) as c:
            assert coxmi.cox_shape(c.h)[0] >= d.n
        # cross-validation folds on interval rows: a subject split across folds is refused,
        # per-subject folds are accepted
        cuts = [float(np.quantile(d.time, 0.5))]
        r = orc.split_intervals(d.X, d.time, d.event, d.stratum, cuts)
        fold_subj = np.arange(d.n, dtype=np.int32) % 3
        with m.intervals(d.time, d.event, d.stratum, cuts, tol=1e-10) as c:
            naug = coxmi.cox_shape(c.h)[0]
            assert naug == r["X"].shape[0] > d.n
            split = fold_subj[r["row_subject"]].copy()
            a = int(np.flatnonzero(r["row_interval"] == 1)[0])
            split[a] = (split[a] + 1) % 3
            with pytest.raises(coxmi.CoxError) as e:
                c.cross_validate(split, [0.0], nfolds=3)
            assert e.value.code == coxmi.COX_EINVAL
            cvl, _, status = c.cross_validate(fold_subj[r["row_subject"]], [0.0], nfolds=3)
            assert np.isfinite(cvl[0]) and np.all(status == coxmi.COX_OK)
        with pytest.raises(ValueError):
            m.intervals(d.time, d.event, d.stratum, [0.5], tv_coef=np.ones(2, np.uint8))
