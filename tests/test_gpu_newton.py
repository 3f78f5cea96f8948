"""GPU parity of the full evaluation, the information contraction and the Newton fit.

Everything goes through the C ABI (cox_evaluate_full, cox_fit in
COX_NEWTON_REFINE mode) and is compared with the FP64 CPU oracle on the same
seeded inputs.

Tolerances:
* objective, gradient, diagonal Hessian (FP64 on both sides): 1e-11 * max(E, |obj|)
  for the objective (E = number of events); for column j with m_j = max(1, max_r |x_rj|),
  1e-11 * 2 E m_j for the score and 1e-11 * E m_j^2 for the diagonal: the weights
  w_r Lambda_r sum to E over the rows (each event group g contributes d_g S0_g / S0_g),
  so these bound the sums of absolute values of the terms;
* information matrix in FP64: |gpu_ij - oracle_ij| <= 1e-11 * r_ij with
  r_ij = sqrt(F_ii F_jj) + sqrt(S_ii S_jj), where F = X' diag(w Lambda) X and
  S = sum_g d_g xbar_g xbar_g' are the two terms (both PSD, so by Cauchy-Schwarz
  r_ij bounds the sum of absolute values of every product that enters entry ij);
* information matrix with X in BF16 (per-column power-of-two scales): a product
  b_k x_ik x_jk of the first term is formed from three values rounded to 8
  significant bits (x_ik, x_jk and the weighted operand b_k x_ik), a product
  z_gi z_gj of the second from two; FP32 accumulation adds at most k 2^-24
  relative over a K range of k rows (the contraction splits N into 128 ranges
  and the groups into 64).  With u = 2^-8 and a margin for second-order terms,
      |gpu_ij - oracle_ij| <= (3.5 u + k 2^-24) r_ij;
* information matrix with X in FP8 e4m3 (power-of-two column scales) and Z in
  BF16: the first term's products are formed from operands a_rj = (x_rj/s_j)
  sqrt(b_r)/S, each rounded twice to 4 significant bits (the stored x, then the
  weighted value), so a product carries at most 4 such roundings: with
  u8 = 2^-4 the bound is (4.5 u8 + k 2^-24) r_ij plus the BF16 Z term's 3.5 u;
  values that fall below the e4m3 normal range (2^-6 after scaling) add an
  absolute error bounded the same way because |a| <= 224 sets the scale;
* fitted beta (FP64, BF16 or FP8 factor + FP64 refinement): max|gpu - oracle| /
  max|oracle| <= 1e-10, with the oracle's own Newton fit to 1e-14.
"""
import math

import numpy as np
import pytest

from oracle import cox_oracle as orc
from paper_2310_16238_amd import coxmi, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U_BF16 = 2.0 ** -8
U_FP8 = 2.0 ** -4


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


def _oracle_eval(d, beta):
    lay = orc.canonical_layout(d.time, d.event, d.stratum)
    Xc = orc.to_canonical(d.X, lay)
    return orc.full_eval(Xc, lay, beta, want_info=True)


def _scale(fe):
    f = np.sqrt(np.clip(np.diag(fe.info_first), 0, None))
    s = np.sqrt(np.clip(np.diag(fe.info_second), 0, None))
    return np.outer(f, f) + np.outer(s, s)


def _first_order_tols(X, E):
    m = np.maximum(1.0, np.max(np.abs(X), axis=0))
    return 1e-11 * 2.0 * max(1.0, E) * m, 1e-11 * max(1.0, E) * m * m


def _check_first_order(d, obj, g, hd, fe):
    E = float(d.event.sum())
    tg, th = _first_order_tols(d.X, E)
    assert abs(obj - fe.objective) <= 1e-11 * max(E, abs(fe.objective)), (obj, fe.objective)
    assert np.all(np.abs(g - fe.grad) <= tg), float(np.max(np.abs(g - fe.grad) / tg))
    assert np.all(np.abs(hd - fe.hess_diag) <= th), float(np.max(np.abs(hd - fe.hess_diag) / th))


def _mixed(n, p, K, seed, ties=False):
    return synth.make("mixed", n, p, K, seed, beta_sd=0.05, tie_round=100.0 if ties else 0.0)


# (name, data factory): several 64-column and 32-column tiles with ragged tails,
# N not a multiple of the row tile, ties, one and many strata
CASES = [
    ("small-K1", lambda: synth.config_small(K=1, gamma=0.0)),
    ("small-K10-ties", lambda: synth.config_small(K=10, ties=True, gamma=0.0)),
    ("mixed-p70-K37", lambda: _mixed(20_011, 70, 37, 3)),
    ("mixed-p97-K1-ties", lambda: _mixed(9_001, 97, 1, 4, ties=True)),
    ("ar1-p130-K500", lambda: synth.config_ar1(n=30_000, p=130, K=500)),
]


def _beta_probe(d, seed=11):
    rng = np.random.default_rng(seed)
    return d.beta_true * 0.7 + rng.normal(0.0, 0.02, size=d.p) / np.maximum(d.X.std(0), 1e-3)


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_full_evaluation_f64(name, make):
    d = make()
    beta = _beta_probe(d)
    _say(f"evaluate_full F64 {name} n={d.n} p={d.p}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum) as m:
        obj, g, hd, info = m.evaluate_full(beta)
        obj2, g2, hd2, none = m.evaluate_full(beta, want_info=False)
    fe = _oracle_eval(d, beta)
    _check_first_order(d, obj, g, hd, fe)
    assert none is None and obj2 == obj and np.array_equal(g2, g) and np.array_equal(hd2, hd)
    r = _scale(fe)
    err = np.abs(info - fe.info)
    assert np.all(err <= 1e-11 * r), float(np.max(err / r))
    assert np.array_equal(info, info.T)
    # its diagonal is the diagonal Hessian of the scan path
    assert np.all(np.abs(np.diag(info) - hd) <= _first_order_tols(d.X, float(d.event.sum()))[1])


@pytest.mark.parametrize("n,p,K", [(20_011, 300, 13), (12_003, 512, 1), (9_001, 257, 40)])
def test_full_evaluation_f64_wide(n, p, K):
    """FP64 information beyond 256 columns on the matrix cores: several groups of 16 x 16 blocks
    per K range (each staging every row of its chunk), at the 512-column limit and one column
    past a block; the same bound as the narrow FP64 case."""
    d = _mixed(n, p, K, 7)
    beta = _beta_probe(d)
    _say(f"evaluate_full F64 wide n={n} p={p}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE) as m:
        obj, g, hd, info = m.evaluate_full(beta)
    fe = _oracle_eval(d, beta)
    _check_first_order(d, obj, g, hd, fe)
    r = _scale(fe)
    err = np.abs(info - fe.info)
    assert np.all(err <= 1e-11 * r), float(np.max(err / r))
    assert np.array_equal(info, info.T)


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_information_bf16_within_bound(name, make):
    d = make()
    beta = _beta_probe(d)
    _say(f"evaluate_full BF16 {name} n={d.n} p={d.p}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, x_precision=coxmi.COX_BF16) as m:
        obj, g, hd, info = m.evaluate_full(beta)
    fe = _oracle_eval(d, beta)
    # objective, gradient and diagonal stay FP64
    _check_first_order(d, obj, g, hd, fe)
    r = _scale(fe)
    k = math.ceil(d.n / 128) + 16
    bound = (3.5 * U_BF16 + k * 2.0 ** -24) * r
    err = np.abs(info - fe.info)
    worst = float(np.max(err / r))
    _say(f"  max |err| / r = {worst:.3e} (bound {3.5 * U_BF16 + k * 2.0 ** -24:.3e})")
    assert np.all(err <= bound), worst
    assert np.array_equal(info, info.T)
    # rounding errors, not misplaced entries: the typical error is far below the bound
    assert float(np.median(err / r)) <= 0.1 * 3.5 * U_BF16


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_information_fp8_within_bound(name, make):
    d = make()
    beta = _beta_probe(d)
    _say(f"evaluate_full FP8 {name} n={d.n} p={d.p}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE,
                        x_precision=coxmi.COX_FP8_E4M3) as m:
        obj, g, hd, info = m.evaluate_full(beta)
    fe = _oracle_eval(d, beta)
    _check_first_order(d, obj, g, hd, fe)
    r = _scale(fe)
    k = math.ceil(d.n / 128) + 16
    lim = 4.5 * U_FP8 + 3.5 * U_BF16 + k * 2.0 ** -24
    err = np.abs(info - fe.info)
    worst = float(np.max(err / r))
    _say(f"  max |err| / r = {worst:.3e} (bound {lim:.3e}), median {float(np.median(err / r)):.2e}")
    assert np.all(err <= lim * r), worst
    assert np.array_equal(info, info.T)
    assert float(np.median(err / r)) <= 0.1 * lim


@pytest.mark.parametrize("prec", [coxmi.COX_F64, coxmi.COX_BF16, coxmi.COX_FP8_E4M3], ids=["f64", "bf16", "fp8"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_newton_fit(name, make, prec):
    d = make()
    _say(f"newton fit {name} prec={prec}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE, x_precision=prec,
                        tol=1e-13, max_iter=200) as m:
        beta, info = m.fit()
    ref = orc.fit_newton(d.X, d.time, d.event, d.stratum, tol=1e-14)
    assert ref.converged
    assert info["status"] == coxmi.COX_OK, info
    err = _rel(beta, ref.beta)
    _say(f"  iters={info['iters']} evals={info['coord_evals']} rel err {err:.3e}")
    assert err <= 1e-10
    free = ~orc.degenerate_columns(orc.to_canonical(d.X, orc.canonical_layout(d.time, d.event, d.stratum)),
                                   orc.canonical_layout(d.time, d.event, d.stratum))
    assert np.all(beta[~free] == 0.0)
    assert info["n_pinned"] == int(np.count_nonzero(~free))
    assert abs(info["objective"] - ref.objective) <= 1e-11 * max(float(d.event.sum()), abs(ref.objective))


def test_newton_fit_mixed_precision_full_size():
    """N = 1e6, P = 200 AR(1), K = 5e4: BF16 contraction + FP64 refinement vs the oracle's optimum."""
    from conftest import read_golden
    gold = read_golden("newton_mixed_n1e6_p200.txt")
    d = synth.config_mixed()
    _say("newton fit BF16 n=1e6 p=200 K=5e4")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE,
                        x_precision=coxmi.COX_BF16, tol=1e-13, max_iter=200) as m:
        beta, info = m.fit()
        obj, g, _, _ = m.evaluate_full(beta, want_info=False)
    ref = np.array(gold["beta"])
    err = _rel(beta, ref)
    _say(f"  iters={info['iters']} evals={info['coord_evals']} rel err {err:.3e} max|grad| {np.max(np.abs(g)):.3e}")
    assert info["status"] == coxmi.COX_OK
    assert err <= 1e-10
    assert abs(obj - gold["objective"][0]) <= 1e-11 * abs(gold["objective"][0])


def test_newton_options_rejected():
    d = synth.config_small(n=500, K=1)
    wide = np.random.default_rng(0).normal(size=(500, 4097))
    with pytest.raises(coxmi.CoxError) as e:
        coxmi.cox_init(wide, d.time, d.event, mode=coxmi.COX_NEWTON_REFINE, x_precision=coxmi.COX_FP8_E4M3)
    assert e.value.code == coxmi.COX_EUNSUPPORTED
    for prec in (coxmi.COX_F32, coxmi.COX_FP8_E4M3):
        with pytest.raises(coxmi.CoxError) as e:
            coxmi.cox_init(d.X, d.time, d.event, x_precision=prec)
        assert e.value.code == coxmi.COX_EUNSUPPORTED


def test_full_evaluation_edge_cases():
    # no events: zero objective, gradient and information
    n, p = 300, 5
    rng = np.random.default_rng(5)
    X = rng.standard_normal((n, p))
    t = rng.random(n)
    with coxmi.CoxModel(X, t, np.zeros(n, np.uint8)) as m:
        obj, g, hd, info = m.evaluate_full(np.full(p, 0.3))
    assert obj == 0.0 and not np.any(g) and not np.any(hd) and not np.any(info)
    # one row, one column; and a single event per stratum (every xbar is the row itself)
    for (n, p, K) in [(1, 1, 1), (64, 3, 64), (257, 33, 2)]:
        X = rng.standard_normal((n, p))
        t = rng.random(n)
        ev = np.ones(n, np.uint8)
        st = np.arange(n, dtype=np.int32) % K
        beta = rng.normal(0, 0.3, p)
        for prec in (coxmi.COX_F64, coxmi.COX_BF16):
            with coxmi.CoxModel(X, t, ev, st, x_precision=prec) as m:
                obj, g, hd, info = m.evaluate_full(beta)
            lay = orc.canonical_layout(t, ev, st)
            fe = orc.full_eval(orc.to_canonical(X, lay), lay, beta)
            assert abs(obj - fe.objective) <= 1e-11 * max(n, abs(fe.objective))
            tg, _ = _first_order_tols(X, float(n))
            assert np.all(np.abs(g - fe.grad) <= tg)
            r = _scale(fe) + 1e-300
            lim = 1e-11 if prec == coxmi.COX_F64 else 3.5 * U_BF16 + 64 * 2.0 ** -24
            assert np.all(np.abs(info - fe.info) <= lim * r + 1e-12), (n, p, K, prec)


def test_newton_beyond_the_resident_kernel():
    """N = 2.5e6 rows exceeds the persistent kernel's register capacity (256 CUs x 512 x 16):
    the handle takes the tile layout; Newton fits, full evaluations and cox_evaluate (answered
    by the full evaluation) match the oracle; a COX_CCD handle of the same data fits by
    (proximal) Newton steps (fallback 2) to the oracle's optima, unpenalised and with l1
    weights; cox_coordinate reports COX_EUNSUPPORTED."""
    d = synth.make("ar1", 2_500_000, 8, 1000, 21, beta_sd=0.5)
    _say("newton fit beyond the resident kernel n=2.5e6 p=8 K=1000")
    ref = orc.fit_newton(d.X, d.time, d.event, d.stratum, tol=1e-14)
    for prec in (coxmi.COX_F64, coxmi.COX_BF16):
        with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE, x_precision=prec,
                            tol=1e-13) as m:
            n, p, ld = coxmi.cox_shape(m.h)
            assert ld % 4096 == 0 and ld >= n
            beta, info = m.fit()
            assert info["status"] == coxmi.COX_OK
            assert _rel(beta, ref.beta) <= 1e-10
            if prec == coxmi.COX_F64:
                obj, g, hd, info_m = m.evaluate_full(beta)
                fe = _oracle_eval(d, beta)
                _check_first_order(d, obj, g, hd, fe)
                assert np.all(np.abs(info_m - fe.info) <= 1e-11 * _scale(fe))
                obj2, g2, hd2 = m.evaluate(beta)   # the per-coordinate path cannot hold it
                _check_first_order(d, obj2, g2, hd2, fe)
    # the same data on a COX_CCD handle
    L = orc.canonical_layout(d.time, d.event, d.stratum)
    g0 = orc.full_eval(orc.to_canonical(d.X, L), L, np.zeros(d.p), want_info=False).grad
    gam = 0.2 * float(np.max(np.abs(g0)))
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, tol=1e-13) as m:
        beta, info = m.fit()
        assert info["status"] == coxmi.COX_OK and info["fallback"] == 2, info
        assert _rel(beta, ref.beta) <= 1e-10
        with pytest.raises(coxmi.CoxError) as ei:
            m.coordinate(beta, 0)
        assert ei.value.code == coxmi.COX_EUNSUPPORTED
        m.set_penalty(gam)
        beta1, info1 = m.fit()
    assert info1["status"] == coxmi.COX_OK and info1["fallback"] == 2, info1
    # the l1 optimality conditions of the oracle's score (plain C, Eq. strat_g) at the estimate
    fe1 = orc.full_eval(orc.to_canonical(d.X, L), L, beta1, want_info=False)
    E = float(d.event.sum())
    viol = np.where(beta1 != 0.0, np.abs(fe1.grad + gam * np.sign(beta1)), np.maximum(np.abs(fe1.grad) - gam, 0.0))
    _say(f"  CCD handle, l1 at 0.2 gamma_max: {np.count_nonzero(beta1)} nonzero, max violation / E = "
         f"{np.max(viol) / E:.2e}")
    assert np.count_nonzero(beta1) < d.p and np.max(viol) <= 1e-9 * E


def test_newton_fp8_heavy_tailed():
    """The heavy-tailed shape at reduced size: N = 2e5, P = 500 Student-t(3) columns, 50
    nonzero coefficients, K = 1e4; FP8 information matrix + FP64 refinement."""
    d = synth.config_heavy(n=200_000, p=500, K=10_000)
    _say("newton fit FP8 heavy-tailed n=2e5 p=500 K=1e4")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE,
                        x_precision=coxmi.COX_FP8_E4M3, tol=1e-13, max_iter=200) as m:
        beta, info = m.fit()
        prof = m.profile()
    ref = orc.fit_newton(d.X, d.time, d.event, d.stratum, tol=1e-14)
    err = _rel(beta, ref.beta)
    _say(f"  iters={info['iters']} evals={info['coord_evals']} rel err {err:.3e} profile {prof}")
    assert info["status"] == coxmi.COX_OK
    assert err <= 1e-10


@pytest.fixture(scope="module")
def heavy_tile():
    """The heavy-tailed workload past the persistent kernel's register capacity (256 CUs x
    512 x 16 rows): N = 2.5e6 Student-t(3) rows, P = 64, 6 nonzero N(0,1) coefficients,
    K = N/20 strata -- the handle takes the 4096-row tile layout, as at N = 1e7."""
    return synth.config_heavy(n=2_500_000, p=64, K=125_000)


def test_information_fp8_tile_layout_within_bound(heavy_tile):
    """FP8 e4m3 information matrix on a tile-layout handle, element by element within the
    FP8 bound of the module docstring (the contraction's K ranges hold at most
    ceil(N / 128) + 16 rows here too)."""
    d = heavy_tile
    beta = d.beta_true * 0.9
    _say(f"evaluate_full FP8 tile layout n={d.n} p={d.p}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE,
                        x_precision=coxmi.COX_FP8_E4M3) as m:
        n, p, ld = coxmi.cox_shape(m.h)
        assert ld % 4096 == 0 and ld >= n > 256 * 512 * 16
        obj, g, hd, info = m.evaluate_full(beta)
    fe = _oracle_eval(d, beta)
    _check_first_order(d, obj, g, hd, fe)
    r = _scale(fe)
    k = math.ceil(d.n / 128) + 16
    lim = 4.5 * U_FP8 + 3.5 * U_BF16 + k * 2.0 ** -24
    err = np.abs(info - fe.info)
    worst = float(np.max(err / r))
    _say(f"  max |err| / r = {worst:.3e} (bound {lim:.3e}), median {float(np.median(err / r)):.2e}")
    assert np.all(err <= lim * r), worst
    assert np.array_equal(info, info.T)
    assert float(np.median(err / r)) <= 0.1 * lim


def test_newton_fp8_beyond_the_resident_kernel(heavy_tile):
    """The large heavy-tailed configuration's own path at a size the oracle fits in seconds:
    FP8 information matrix on the tile layout + FP64 score and refinement, against the
    oracle's FP64 Newton optimum (1e-10 relative on beta)."""
    d = heavy_tile
    _say(f"newton fit FP8 tile layout n={d.n} p={d.p} K=1.25e5")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE,
                        x_precision=coxmi.COX_FP8_E4M3, tol=1e-13, max_iter=200) as m:
        n, p, ld = coxmi.cox_shape(m.h)
        assert ld % 4096 == 0 and ld >= n
        beta, info = m.fit()
        prof = m.profile()
    ref = orc.fit_newton(d.X, d.time, d.event, d.stratum, tol=1e-14)
    assert ref.converged
    err = _rel(beta, ref.beta)
    _say(f"  iters={info['iters']} evals={info['coord_evals']} rel err {err:.3e} profile {prof}")
    assert info["status"] == coxmi.COX_OK
    assert err <= 1e-10
    assert abs(info["objective"] - ref.objective) <= 1e-11 * max(float(d.event.sum()), abs(ref.objective))


def test_full_evaluation_extreme_linear_predictor():
    """Rows whose X beta is 900 or more above the rest of their stratum: a single
    exponent shift would underflow every other row's weight; the running-maximum
    recurrences keep all risk-set sums in range.  Against the oracle, whose scan
    carries a running maximum as well."""
    rng = np.random.default_rng(41)
    n, p, K = 6000, 4, 60
    X = rng.standard_normal((n, p))
    hot = rng.choice(n, size=12, replace=False)
    X[hot, 0] = rng.choice([-300.0, 300.0], size=12)
    t = rng.exponential(1.0, n)
    e = (rng.random(n) < 0.6).astype(np.uint8)
    st = (np.arange(n) % K).astype(np.int32)
    beta = np.array([3.0, -2.0, 1.0, 0.5])
    d = synth.CoxData(X=np.asfortranarray(X), time=t, event=e, stratum=st, beta_true=beta, gamma=0.0, name="extreme")
    _say("evaluate_full with |X beta| up to 900")
    fe = _oracle_eval(d, beta)
    for prec in (coxmi.COX_F64, coxmi.COX_BF16):
        with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE, x_precision=prec) as m:
            obj, g, hd, info = m.evaluate_full(beta)
        _check_first_order(d, obj, g, hd, fe)
        lim = 1e-11 if prec == coxmi.COX_F64 else 3.5 * U_BF16 + 64 * 2.0 ** -24
        assert np.all(np.abs(info - fe.info) <= lim * _scale(fe) + 1e-300)


@pytest.mark.parametrize("n,K,ties", [(3000, 1, False), (4000, 40, True)])
def test_baseline_hazard_matches_oracle(n, K, ties):
    """Breslow cumulative baseline hazard from the full evaluation against the oracle's
    definition (FP64 on both sides: 1e-12 relative, row by row)."""
    d = synth.make("iid", n, 4, K, 41 + K, beta_sd=0.5, tie_round=50.0 if ties else 0.0)
    beta = np.array([0.4, -0.3, 0.2, 0.1])
    _say(f"baseline hazard n={n} K={K} ties={ties}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum) as m:
        lam = m.baseline_hazard(beta)
    ref = orc.baseline_hazard_brute(d.X, d.time, d.event, d.stratum, beta)
    np.testing.assert_allclose(lam, ref, rtol=1e-12, atol=0)


def test_baseline_hazard_large_identities():
    """At N = 1e6 with 5e4 strata: martingale residuals sum to zero in every stratum, and
    X'(exp(X beta) Lambda_0 - delta) equals the score of cox_evaluate_full."""
    d = synth.config_ar1()
    beta = np.random.default_rng(2).normal(0, 0.1, d.X.shape[1])
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE) as m:
        lam = m.baseline_hazard(beta)
        _, g, _, _ = m.evaluate_full(beta, want_info=False)
    w = np.exp(d.X @ beta)
    res = d.event - w * lam
    per = np.bincount(d.stratum, weights=res)
    E = float(d.event.sum())
    assert np.max(np.abs(per)) <= 1e-10
    score = d.X.T @ (w * lam - d.event)
    assert np.max(np.abs(score - g)) <= 1e-10 * E


L1_CASES = [
    ("small-K1", lambda: synth.config_small(K=1, gamma=0.0)),
    ("small-K10-ties", lambda: synth.config_small(K=10, ties=True, gamma=0.0)),
    ("ar1-p40-K200", lambda: synth.config_ar1(n=10_000, p=40, K=200)),
]


@pytest.mark.parametrize("prec", [coxmi.COX_F64, coxmi.COX_BF16, coxmi.COX_FP8_E4M3], ids=["f64", "bf16", "fp8"])
@pytest.mark.parametrize("name,make", L1_CASES, ids=[c[0] for c in L1_CASES])
def test_newton_l1_fit(name, make, prec):
    """Proximal Newton with the l1 penalty (column 0 unpenalised) against the oracle's CCD fit of
    the same penalised objective: the optimum is unique, so the estimates agree to 1e-10 and
    the zero pattern exactly, whatever the precision of the information matrix.  gamma is a
    fifth of the largest penalised score at 0, so that a share of the coefficients is 0."""
    d = make()
    p = d.X.shape[1]
    pen = np.ones(p, np.uint8)
    pen[0] = 0
    L = orc.canonical_layout(d.time, d.event, d.stratum)
    g0 = orc.full_eval(orc.to_canonical(d.X, L), L, np.zeros(p), want_info=False).grad
    gamma = 0.2 * float(np.max(np.abs(g0[1:])))
    _say(f"newton l1 fit {name} prec={prec} gamma={gamma:.2f}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE, x_precision=prec,
                        gamma=gamma, penalize=pen, tol=1e-13, max_iter=300) as m:
        beta, info = m.fit()
    ref = orc.fit_ccd(d.X, d.time, d.event, d.stratum, gamma=gamma, penalize=pen, tol=1e-14, max_sweeps=5000)
    assert ref.converged and info["status"] == coxmi.COX_OK, info
    assert np.array_equal(beta == 0.0, ref.beta == 0.0)
    err = _rel(beta, ref.beta)
    _say(f"  steps={info['iters']} nonzero={int(np.count_nonzero(beta))} rel err {err:.3e} kkt {info['kkt_inf']:.2e}")
    assert err <= 1e-10


@pytest.mark.parametrize("prec", [coxmi.COX_F64, coxmi.COX_BF16], ids=["f64", "bf16"])
def test_newton_l1_fit_wide(prec):
    """Proximal Newton with more columns than one LDS chunk of the device model solve (1024
    coordinates) and than its prefetched row (1024 entries per row): chunked staging and the
    streamed row tail; the oracle's CCD optimum to 1e-10 and the same zero pattern."""
    d = synth.config_ar1(n=8_000, p=1_100, K=40)
    p = d.X.shape[1]
    pen = np.ones(p, np.uint8)
    pen[0] = 0
    L = orc.canonical_layout(d.time, d.event, d.stratum)
    g0 = orc.full_eval(orc.to_canonical(d.X, L), L, np.zeros(p), want_info=False).grad
    gamma = 0.3 * float(np.max(np.abs(g0[1:])))
    _say(f"newton l1 fit wide p={p} prec={prec} gamma={gamma:.2f}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE, x_precision=prec,
                        gamma=gamma, penalize=pen, tol=1e-13, max_iter=300) as m:
        beta, info = m.fit()
    ref = orc.fit_ccd(d.X, d.time, d.event, d.stratum, gamma=gamma, penalize=pen, tol=1e-14, max_sweeps=5000)
    assert ref.converged and info["status"] == coxmi.COX_OK, info
    assert np.array_equal(beta == 0.0, ref.beta == 0.0)
    err = _rel(beta, ref.beta)
    _say(f"  steps={info['iters']} nonzero={int(np.count_nonzero(beta))} rel err {err:.3e}")
    assert err <= 1e-10


@pytest.mark.parametrize("n,p,K", [(20_011, 600, 13), (12_003, 1000, 1)])
def test_information_bf16_wide_within_bound(n, p, K):
    """More than 16 row tiles (P > 512): the blocked contraction, where each workgroup stages only
    the two row blocks of its tile pairs.  Same bound as the narrow case; the two-factor design
    makes every entry comparable to the diagonal, so a misplaced block would show."""
    d = _mixed(n, p, K, 5)
    beta = _beta_probe(d)
    _say(f"evaluate_full BF16 wide n={n} p={p}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, x_precision=coxmi.COX_BF16) as m:
        obj, g, hd, info = m.evaluate_full(beta)
    fe = _oracle_eval(d, beta)
    _check_first_order(d, obj, g, hd, fe)
    r = _scale(fe)
    k = math.ceil(d.n / 128) + 16
    bound = (3.5 * U_BF16 + k * 2.0 ** -24) * r
    err = np.abs(info - fe.info)
    worst = float(np.max(err / r))
    _say(f"  max |err| / r = {worst:.3e} (bound {3.5 * U_BF16 + k * 2.0 ** -24:.3e})")
    assert np.all(err <= bound), worst
    assert np.array_equal(info, info.T)
    assert float(np.median(err / r)) <= 0.1 * 3.5 * U_BF16


@pytest.mark.parametrize("n,p,K", [(20_011, 900, 13), (12_003, 1000, 1)])
def test_information_fp8_wide_within_bound(n, p, K):
    """More than 800 columns in FP8: the blocked kernel (each workgroup stages only the row
    blocks of its tile pairs); the FP8 bound of the narrow case."""
    d = _mixed(n, p, K, 6)
    beta = _beta_probe(d)
    _say(f"evaluate_full FP8 wide n={n} p={p}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, mode=coxmi.COX_NEWTON_REFINE,
                        x_precision=coxmi.COX_FP8_E4M3) as m:
        obj, g, hd, info = m.evaluate_full(beta)
    fe = _oracle_eval(d, beta)
    _check_first_order(d, obj, g, hd, fe)
    r = _scale(fe)
    k = math.ceil(d.n / 128) + 16
    lim = 4.5 * U_FP8 + 3.5 * U_BF16 + k * 2.0 ** -24
    err = np.abs(info - fe.info)
    worst = float(np.max(err / r))
    _say(f"  max |err| / r = {worst:.3e} (bound {lim:.3e}), median {float(np.median(err / r)):.2e}")
    assert np.all(err <= lim * r), worst
    assert np.array_equal(info, info.T)
    assert float(np.median(err / r)) <= 0.1 * lim
