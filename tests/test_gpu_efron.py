"""GPU parity of Efron's tie correction on the CCD path, through the C ABI, against the
oracle's Efron functions (orc.coord_terms / fit_ccd / fit_newton with ties="efron"; the
oracle's Efron definition is pinned in test_oracle_efron_cpu.py).

Tolerances as for the plain risk sets (test_gpu_parity.py): per-coordinate sums within
1e-11 * max(1, E), -log L within 1e-11 * max(E, |-log L|), fitted beta within 1e-10
relative with the same l1 zero pattern.  Efron's term of a group with one event is the
plain term, so on data without tied events the two tie rules give the same fit.
"""
import math

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
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(float(np.max(np.abs(b))), 1e-300))


def _max_tie(d):
    L = orc.canonical_layout(d.time, d.event, d.stratum)
    return int(np.max(L.meta & 0x1FFFFFFF))


@pytest.mark.parametrize("n,K,tie_round", [(5000, 1, 100.0), (5000, 250, 100.0), (150_000, 7500, 100.0),
                                           (600_000, 1, 100.0), (600_000, 30_000, 100.0), (40_000, 1, 2.0)])
def test_efron_coordinate_parity(n, K, tie_round):
    d = synth.make("ar1", n, 6, K, seed=200 + K, beta_sd=0.5, tie_round=tie_round)
    beta = np.array([0.3, -0.4, 0.25, 0.0, 0.6, -0.2])
    _say(f"efron coordinate parity n={n} K={K} round={tie_round} largest tie group={_max_tie(d)}")
    L = orc.canonical_layout(d.time, d.event, d.stratum)
    Xc = orc.to_canonical(d.X, L)
    eta = Xc @ beta
    E = float(d.event.sum())
    tol = 1e-11 * max(1.0, E)
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, ties=coxmi.COX_EFRON) as m:
        for j in range(6):
            got = m.coordinate(beta, j)
            ref = orc.coord_terms(Xc, L, j, eta, ties="efron")
            assert abs(got[0] - ref["grad"]) <= tol, (j, got[0], ref["grad"])
            assert abs(got[1] - ref["hess"]) <= tol, (j, got[1], ref["hess"])
            assert abs(got[2] - ref["obj"]) <= 1e-11 * max(E, abs(ref["obj"])), (j, got[2], ref["obj"])
            assert abs(got[3] - ref["m2"]) <= tol
            # the tie rule matters on these data
            br = orc.coord_terms(Xc, L, j, eta)
            if j == 0:
                assert abs(br["grad"] - ref["grad"]) > 100 * tol


@pytest.mark.parametrize("K", [1, 10, 500])
@pytest.mark.parametrize("gamma", [math.sqrt(2.0), 0.0])
def test_efron_fit_small(K, gamma):
    d = synth.config_small(K=K, ties=True, gamma=gamma)
    _say(f"efron fit small K={K} gamma={gamma:.3f} largest tie group={_max_tie(d)}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, gamma=gamma, tol=1e-13, ties=coxmi.COX_EFRON) as m:
        beta, info = m.fit()
    ref = orc.fit_ccd(d.X, d.time, d.event, d.stratum, gamma=gamma, tol=1e-13, ties="efron")
    assert info["status"] == coxmi.COX_OK and ref.converged
    assert beta[0] == 0.0
    assert np.array_equal(beta == 0.0, ref.beta == 0.0)
    assert _rel(beta, ref.beta) <= 1e-10
    if gamma == 0.0:
        nw = orc.fit_newton(d.X, d.time, d.event, d.stratum, ties="efron")
        assert _rel(beta, nw.beta) <= 1e-10
        br = orc.fit_newton(d.X, d.time, d.event, d.stratum)
        assert _rel(br.beta, nw.beta) > 1e-6      # the two tie rules give different estimates here


def test_efron_fit_heavy_ties_one_stratum():
    """Few distinct times: tie groups of hundreds of events, strata crossing workgroup tiles."""
    d = synth.make("iid", 300_000, 8, 1, seed=31, beta_sd=0.4, tie_round=3.0)
    _say(f"efron fit heavy ties n=3e5 K=1 largest tie group={_max_tie(d)}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, tol=1e-13, ties=coxmi.COX_EFRON) as m:
        beta, info = m.fit()
    assert info["status"] == coxmi.COX_OK
    nw = orc.fit_newton(d.X, d.time, d.event, d.stratum, ties="efron", tol=1e-14)
    assert nw.converged
    err = _rel(beta, nw.beta)
    _say(f"  rel err {err:.2e}")
    assert err <= 1e-10


def test_efron_equals_breslow_without_ties():
    d = synth.config_small(n=20_000, K=50, ties=False)
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, tol=1e-13) as m:
        b_br, _ = m.fit()
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, tol=1e-13, ties=coxmi.COX_EFRON) as m:
        b_ef, info = m.fit()
    assert info["status"] == coxmi.COX_OK
    assert _rel(b_ef, b_br) <= 1e-14


def test_efron_indicator_matches_dense():
    d = synth.make("binary", 30_000, 12, 30, seed=41, beta_sd=0.5, tie_round=50.0)
    cols = [np.flatnonzero(d.X[:, j]) for j in range(d.p)]
    col_ptr = np.concatenate([[0], np.cumsum([c.size for c in cols])])
    row_idx = np.concatenate(cols).astype(np.int32)
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, gamma=0.5, tol=1e-13, ties=coxmi.COX_EFRON) as m:
        b_dense, _ = m.fit()
    with coxmi.CoxModel.indicator(d.n, col_ptr, row_idx, d.time, d.event, d.stratum, gamma=0.5, tol=1e-13,
                                  ties=coxmi.COX_EFRON) as m:
        b_bits, info = m.fit()
    assert info["status"] == coxmi.COX_OK
    assert np.array_equal(b_dense, b_bits)
    ref = orc.fit_ccd(d.X, d.time, d.event, d.stratum, gamma=0.5, tol=1e-13, ties="efron")
    assert np.array_equal(b_bits == 0.0, ref.beta == 0.0)
    assert _rel(b_bits, ref.beta) <= 1e-10


# ------------------------------------------------------------------ full evaluation and Newton fits

U_BF16 = 2.0 ** -8
U_FP8 = 2.0 ** -4

EVAL_CASES = [
    ("small-K10-ties", lambda: synth.config_small(K=10, ties=True, gamma=0.0)),
    ("mixed-p97-K1-ties", lambda: synth.make("mixed", 9_001, 97, 1, 4, beta_sd=0.05, tie_round=100.0)),
    ("ar1-p40-K300-ties", lambda: synth.make("ar1", 40_000, 40, 300, 12, beta_sd=0.3, tie_round=20.0)),
    ("iid-p12-K1-heavy-ties", lambda: synth.make("iid", 60_000, 12, 1, 13, beta_sd=0.3, tie_round=4.0)),
]


def _probe(d, seed=11):
    rng = np.random.default_rng(seed)
    return d.beta_true * 0.7 + rng.normal(0.0, 0.02, size=d.p) / np.maximum(d.X.std(0), 1e-3)


def _oracle_efron(d, beta):
    lay = orc.canonical_layout(d.time, d.event, d.stratum)
    return orc.full_eval(orc.to_canonical(d.X, lay), lay, beta, want_info=True, ties="efron")


def _scale(fe):
    f = np.sqrt(np.clip(np.diag(fe.info_first), 0, None))
    s = np.sqrt(np.clip(np.diag(fe.info_second), 0, None))
    return np.outer(f, f) + np.outer(s, s)


def _check_first_order(d, obj, g, hd, fe):
    """As test_gpu_newton.py: the weights w c sum to E over the rows, so 1e-11 * 2 E m_j bounds
    the score's rounding and 1e-11 * E m_j^2 the diagonal's (m_j = max(1, max|x_j|))."""
    E = float(d.event.sum())
    mx = np.maximum(1.0, np.max(np.abs(d.X), axis=0))
    tg, th = 1e-11 * 2.0 * max(1.0, E) * mx, 1e-11 * max(1.0, E) * mx * mx
    assert abs(obj - fe.objective) <= 1e-11 * max(E, abs(fe.objective)), (obj, fe.objective)
    assert np.all(np.abs(g - fe.grad) <= tg), float(np.max(np.abs(g - fe.grad) / tg))
    assert np.all(np.abs(hd - fe.hess_diag) <= th), float(np.max(np.abs(hd - fe.hess_diag) / th))


@pytest.mark.parametrize("name,make", EVAL_CASES, ids=[c[0] for c in EVAL_CASES])
def test_efron_full_evaluation_f64(name, make):
    d = make()
    beta = _probe(d)
    _say(f"efron evaluate_full F64 {name} n={d.n} p={d.p} largest tie group={_max_tie(d)}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, ties=coxmi.COX_EFRON) as m:
        obj, g, hd, info = m.evaluate_full(beta)
    fe = _oracle_efron(d, beta)
    _check_first_order(d, obj, g, hd, fe)
    r = _scale(fe)
    err = np.abs(info - fe.info)
    assert np.all(err <= 1e-11 * r), float(np.max(err / r))
    assert np.array_equal(info, info.T)
    # the scan path's coordinate terms agree with the full evaluation
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, ties=coxmi.COX_EFRON) as m:
        obj2, g2, h2 = m.evaluate(beta)
    _check_first_order(d, obj2, g2, h2, fe)


@pytest.mark.parametrize("name,make", EVAL_CASES, ids=[c[0] for c in EVAL_CASES])
def test_efron_information_bf16_within_bound(name, make):
    """The bound of test_gpu_newton.py: Z's rows here are another factorisation of the same
    PSD second term, so sum_k |z_ki z_kj| <= sqrt(S_ii S_jj) still bounds every product."""
    d = make()
    beta = _probe(d)
    _say(f"efron evaluate_full BF16 {name} n={d.n} p={d.p}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, x_precision=coxmi.COX_BF16, ties=coxmi.COX_EFRON) as m:
        obj, g, hd, info = m.evaluate_full(beta)
    fe = _oracle_efron(d, beta)
    _check_first_order(d, obj, g, hd, fe)
    r = _scale(fe)
    k = math.ceil(d.n / 128) + 16
    lim = 3.5 * U_BF16 + k * 2.0 ** -24
    err = np.abs(info - fe.info)
    assert np.all(err <= lim * r), float(np.max(err / r))
    assert float(np.median(err / r)) <= 0.1 * 3.5 * U_BF16


@pytest.mark.parametrize("prec", [coxmi.COX_F64, coxmi.COX_BF16, coxmi.COX_FP8_E4M3], ids=["f64", "bf16", "fp8"])
@pytest.mark.parametrize("name,make", EVAL_CASES, ids=[c[0] for c in EVAL_CASES])
def test_efron_newton_fit(name, make, prec):
    d = make()
    _say(f"efron Newton fit {name} prec={prec}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE, x_precision=prec,
                        tol=1e-13, max_iter=200, ties=coxmi.COX_EFRON) as m:
        beta, info = m.fit()
    ref = orc.fit_newton(d.X, d.time, d.event, d.stratum, tol=1e-14, ties="efron")
    assert info["status"] == coxmi.COX_OK and ref.converged
    err = _rel(beta, ref.beta)
    _say(f"  {info['iters']} steps, rel err {err:.2e}")
    assert err <= 1e-10


def test_efron_newton_l1_matches_ccd():
    """Proximal Newton with Efron's terms reaches the l1 optimum the CCD path finds."""
    d = synth.config_small(K=10, ties=True, gamma=math.sqrt(2.0))
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, gamma=d.gamma, mode=coxmi.COX_NEWTON_REFINE,
                        tol=1e-13, max_iter=300, ties=coxmi.COX_EFRON) as m:
        b_nt, info = m.fit()
    ref = orc.fit_ccd(d.X, d.time, d.event, d.stratum, gamma=d.gamma, tol=1e-14, max_sweeps=5000, ties="efron")
    assert info["status"] == coxmi.COX_OK and ref.converged
    assert np.array_equal(b_nt == 0.0, ref.beta == 0.0)
    assert _rel(b_nt, ref.beta) <= 1e-10


def test_efron_baseline_hazard_reports_unsupported():
    d = synth.config_small(n=3000, ties=True)
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, ties=coxmi.COX_EFRON) as m:
        with pytest.raises(coxmi.CoxError) as ei:
            m.baseline_hazard(np.zeros(d.p))
    assert ei.value.code == coxmi.COX_EUNSUPPORTED
