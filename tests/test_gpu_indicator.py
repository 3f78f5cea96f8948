"""Indicator X (one bit per row; Secs. 3.1-3.2 use 3-5% dense indicators) on the GPU.

With x in {0, 1} every product the CCD kernel forms equals the dense one exactly, so a
handle built from compressed sparse columns must give the same bits as a handle on the
same X stored dense (fits, evaluations, coordinates), and both meet the oracle at the
FP64 fit tolerance (max|gpu - oracle| / max|oracle| <= 1e-10, zero pattern exact).
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


def _csc(X):
    cols = [np.flatnonzero(X[:, j]) for j in range(X.shape[1])]
    ptr = np.zeros(X.shape[1] + 1, np.int64)
    ptr[1:] = np.cumsum([c.size for c in cols])
    return ptr, np.concatenate(cols).astype(np.int32)


@pytest.mark.parametrize("n,p,K,gamma", [(5000, 12, 1, 1.0), (150_000, 40, 7500, 2.0), (600_000, 30, 1, 0.0),
                                         (1_200_000, 20, 60_000, 5.0)])
def test_indicator_equals_dense(n, p, K, gamma):
    d = synth.make("binary", n, p, K, 200 + K, beta_sd=1.0, beta_nonzero=0.3, density=0.05, tie_round=100.0)
    d.X[:, 3] = 0.0                       # an empty column (pinned at zero)
    ptr, idx = _csc(d.X)
    _say(f"indicator vs dense n={n} p={p} K={K} gamma={gamma} nnz={idx.size}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, gamma=gamma, tol=1e-13) as md, \
            coxmi.CoxModel.indicator(n, ptr, idx, d.time, d.event, d.stratum, gamma=gamma, tol=1e-13) as mb:
        assert np.array_equal(md.layout()[0], mb.layout()[0])
        bd, infod = md.fit()
        bb, infob = mb.fit()
        assert np.array_equal(bd, bb) and infod["iters"] == infob["iters"]
        probe = np.random.default_rng(1).normal(0, 0.2, p)
        od, gd, hd = md.evaluate(probe)
        ob, gb, hb = mb.evaluate(probe)
        assert od == ob and np.array_equal(gd, gb) and np.array_equal(hd, hb)
        assert np.array_equal(md.coordinate(probe, 5), mb.coordinate(probe, 5))
    if n <= 150_000:
        ref = orc.fit_ccd(d.X, d.time, d.event, d.stratum, gamma=gamma, tol=1e-13)
        assert ref.converged and np.array_equal(bb == 0.0, ref.beta == 0.0)
        err = _rel(bb, ref.beta)
        _say(f"  sweeps={infob['iters']} rel err vs oracle {err:.3e}")
        assert err <= 1e-10


def test_indicator_repeated_indices_and_errors():
    d = synth.make("binary", 4000, 5, 2, 211, density=0.1)
    ptr, idx = _csc(d.X)
    # every index listed twice, columns in scrambled order: the same matrix
    ptr2 = ptr * 2
    idx2 = np.concatenate([np.random.default_rng(0).permutation(np.repeat(idx[ptr[j]:ptr[j + 1]], 2))
                           for j in range(5)]).astype(np.int32)
    with coxmi.CoxModel.indicator(4000, ptr, idx, d.time, d.event, d.stratum, gamma=1.0) as a, \
            coxmi.CoxModel.indicator(4000, ptr2, idx2, d.time, d.event, d.stratum, gamma=1.0) as b:
        ba, _ = a.fit()
        bb, _ = b.fit()
        assert np.array_equal(ba, bb)
        with pytest.raises(coxmi.CoxError) as e:
            a.evaluate_full(np.zeros(5))
        assert e.value.code == coxmi.COX_EUNSUPPORTED
        with pytest.raises(coxmi.CoxError) as e:
            a.baseline_hazard(np.zeros(5))
        assert e.value.code == coxmi.COX_EUNSUPPORTED
        with pytest.raises(coxmi.CoxError) as e:
            a.intervals(d.time, d.event, d.stratum, [0.5], mode=coxmi.COX_NEWTON_REFINE)
        assert e.value.code == coxmi.COX_EUNSUPPORTED
    bad = idx.copy()
    bad[0] = 4000
    with pytest.raises(coxmi.CoxError) as e:
        coxmi.CoxModel.indicator(4000, ptr, bad, d.time, d.event, d.stratum)
    assert e.value.code == coxmi.COX_EINVAL
    ptr_bad = ptr.copy()
    ptr_bad[2] = ptr_bad[1] - 1
    with pytest.raises(coxmi.CoxError) as e:
        coxmi.CoxModel.indicator(4000, ptr_bad, idx, d.time, d.event, d.stratum)
    assert e.value.code == coxmi.COX_EINVAL


def test_wide_indicator_beyond_4096_columns():
    """P = 6000 (the persistent kernel keeps only beta in LDS): indicator and dense handles
    agree bit for bit, and the oracle's per-column derivatives (plain C, Eq. strat_g) at
    the returned beta satisfy the l1 optimality conditions on sampled columns."""
    n, p = 30_000, 6000
    d = synth.make("binary", n, p, 300, 213, beta_sd=1.0, beta_nonzero=0.02, density=0.03, tie_round=100.0)
    ptr, idx = _csc(d.X)
    gamma = 4.0
    _say(f"wide indicator n={n} p={p} nnz={idx.size}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, gamma=gamma, tol=1e-12) as md, \
            coxmi.CoxModel.indicator(n, ptr, idx, d.time, d.event, d.stratum, gamma=gamma, tol=1e-12) as mb:
        bd, infod = md.fit()
        bb, infob = mb.fit()
    assert infob["status"] == coxmi.COX_OK and np.array_equal(bd, bb)
    lay = orc.canonical_layout(d.time, d.event, d.stratum)
    eta = np.ascontiguousarray((d.X @ bb)[lay.perm])
    E = float(d.event.sum())
    nz = np.flatnonzero(bb)
    cols = list(nz[:5]) + list(np.flatnonzero(bb == 0.0)[:5]) + [p - 1]
    worst = 0.0
    for j in cols:
        g = orc.coord_terms(orc.to_canonical(d.X[:, [j]], lay), lay, 0, eta)["grad"]
        r = abs(g + gamma * np.sign(bb[j])) if bb[j] != 0.0 else max(abs(g) - gamma, 0.0)
        worst = max(worst, r / E)
    _say(f"  sweeps={infob['iters']} nonzero={nz.size} l1 optimality residual / E = {worst:.2e}")
    assert worst <= 1e-10


@pytest.mark.parametrize("n,K", [(20_000, 40), (1_100_000, 11)])
def test_indicator_resample_cv_bootstrap_equal_dense(n, K):
    """Resampled handles of an indicator parent (bits gathered on the device) give the same bits
    as those of a dense parent: a fold fit, the cross-validated likelihood and bootstrap refits;
    n = 1.1e6 takes 16 rows per thread in the parent and 8 in a fold."""
    p = 12
    d = synth.make("binary", n, p, K, 215 + K, beta_sd=1.0, beta_nonzero=0.4, density=0.05, tie_round=100.0)
    ptr, idx = _csc(d.X)
    rng = np.random.default_rng(5)
    fold = rng.integers(0, 4, n).astype(np.int32)
    counts = np.stack([rng.multinomial(n, np.full(n, 1.0 / n)) for _ in range(2)]).astype(np.uint32)
    gammas = [50.0, 10.0, 2.0]
    _say(f"indicator resampling n={n} K={K}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, gamma=3.0, tol=1e-12) as md, \
            coxmi.CoxModel.indicator(n, ptr, idx, d.time, d.event, d.stratum, gamma=3.0, tol=1e-12) as mb:
        keep = (fold != 1).astype(np.uint32)
        with md.resample(keep) as cd, mb.resample(keep) as cb:
            assert np.array_equal(cd.layout()[1], cb.layout()[1])
            bd, _ = cd.fit()
            bb, _ = cb.fit()
            assert np.array_equal(bd, bb)
        cvd, betd, _ = md.cross_validate(fold, gammas)
        cvb, betb, _ = mb.cross_validate(fold, gammas)
        assert np.array_equal(cvd, cvb) and np.array_equal(betd, betb)
        btd, _ = md.bootstrap(counts)
        btb, _ = mb.bootstrap(counts)
        assert np.array_equal(btd, btb)
    if n <= 20_000:
        Xr, tr, er, sr = orc.resample(d.X, d.time, d.event, d.stratum, keep)
        ref = orc.fit_ccd(Xr, tr, er, sr, gamma=3.0, tol=1e-12)
        assert np.array_equal(bb == 0.0, ref.beta == 0.0) and _rel(bb, ref.beta) <= 1e-10


def test_indicator_intervals_equal_dense():
    """The interval-stratified model (Secs. 2.2-2.3, step coefficients on two columns) built on
    the device from an indicator parent equals the one built from a dense parent, bit for bit,
    and meets the oracle's fit of its own split."""
    n, p = 40_000, 16
    d = synth.make("binary", n, p, 8, 221, beta_sd=1.0, beta_nonzero=0.4, density=0.08, tie_round=50.0)
    d.X[:, 0] = (np.random.default_rng(3).random(n) < 0.5).astype(np.float64)    # a treatment indicator
    ptr, idx = _csc(d.X)
    cuts = [float(np.quantile(d.time, 0.2)), float(np.quantile(d.time, 0.6))]
    tv = np.zeros(p, np.uint8)
    tv[[0, 5]] = 1
    r = orc.split_intervals(d.X, d.time, d.event, d.stratum, cuts, tv_coef=tv)
    pa = r["X"].shape[1]
    pen = np.ones(pa, np.uint8)
    pen[r["col_source"] == 0] = 0
    _say(f"indicator intervals n={n} p={p} -> n_aug={r['X'].shape[0]} p_aug={pa}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum) as md, \
            coxmi.CoxModel.indicator(n, ptr, idx, d.time, d.event, d.stratum) as mb:
        with md.intervals(d.time, d.event, d.stratum, cuts, tv, gamma=2.0, penalize=pen, tol=1e-13) as cd, \
                mb.intervals(d.time, d.event, d.stratum, cuts, tv, gamma=2.0, penalize=pen, tol=1e-13) as cb:
            assert np.array_equal(cd.layout()[0], cb.layout()[0]) and np.array_equal(cd.layout()[1], cb.layout()[1])
            bd, _ = cd.fit()
            bb, info = cb.fit()
    assert np.array_equal(bd, bb)
    ref = orc.fit_ccd(r["X"], r["time"], r["event"], r["stratum"], gamma=2.0, penalize=pen, tol=1e-13)
    assert ref.converged and info["status"] == coxmi.COX_OK
    assert np.array_equal(bb == 0.0, ref.beta == 0.0) and _rel(bb, ref.beta) <= 1e-10


def _sparse_values(d, seed):
    """d.X with its ones replaced by N(0, 1) values (a general sparse design) and its CSC form."""
    X = d.X.copy()
    nz = X != 0.0
    X[nz] = np.random.default_rng(seed).normal(0.0, 1.0, int(nz.sum()))
    cols = [np.flatnonzero(X[:, j]) for j in range(X.shape[1])]
    ptr = np.zeros(X.shape[1] + 1, np.int64)
    ptr[1:] = np.cumsum([c.size for c in cols])
    idx = np.concatenate(cols).astype(np.int32)
    vals = np.concatenate([X[c, j] for j, c in enumerate(cols)])
    return X, ptr, idx, vals


@pytest.mark.parametrize("n,p,K,gamma", [(5000, 12, 1, 1.0), (150_000, 40, 7500, 2.0), (300_000, 16, 3, 0.0),
                                         (600_000, 10, 30_000, 0.5), (1_200_000, 8, 60_000, 5.0)])
def test_sparse_values_equal_dense(n, p, K, gamma):
    """General sparse X (cox_init_sparse: the nonzero rows' bits and their values, found by a
    prefix sum of bit counts across each wave) against the same X stored dense: every product
    is formed from the same values, so fits, evaluations and coordinates agree bit for bit, at
    1, 2, 4, 8 and 16 rows per thread; and the oracle's CCD fit to 1e-10."""
    d = synth.make("binary", n, p, K, 300 + K, beta_sd=0.5, beta_nonzero=0.4, density=0.05, tie_round=100.0)
    X, ptr, idx, vals = _sparse_values(d, 17)
    X[:, 2] = 0.0                         # an empty column
    keep = idx >= 0
    keep[ptr[2]:ptr[3]] = False
    ptr2 = ptr.copy()
    ptr2[3:] -= ptr[3] - ptr[2]
    idx, vals = idx[keep], vals[keep]
    perm = np.random.default_rng(3).permutation(ptr2[1])   # column 0's entries in scrambled order
    idx[:ptr2[1]] = idx[:ptr2[1]][perm]
    vals[:ptr2[1]] = vals[:ptr2[1]][perm]
    _say(f"sparse values vs dense n={n} p={p} K={K} gamma={gamma} nnz={idx.size}")
    with coxmi.CoxModel(X, d.time, d.event, d.stratum, gamma=gamma, tol=1e-13) as md, \
            coxmi.CoxModel.sparse(n, ptr2, idx, vals, d.time, d.event, d.stratum, gamma=gamma, tol=1e-13) as ms:
        bd, infod = md.fit()
        bs, infos = ms.fit()
        assert np.array_equal(bd, bs) and infod["iters"] == infos["iters"], (infod, infos)
        probe = np.random.default_rng(1).normal(0, 0.2, p)
        od, gd, hd = md.evaluate(probe)
        os_, gs, hs = ms.evaluate(probe)
        assert od == os_ and np.array_equal(gd, gs) and np.array_equal(hd, hs)
        assert np.array_equal(md.coordinate(probe, p - 1), ms.coordinate(probe, p - 1))
    if n <= 150_000:
        ref = orc.fit_ccd(X, d.time, d.event, d.stratum, gamma=gamma, tol=1e-13)
        assert ref.converged and np.array_equal(bs == 0.0, ref.beta == 0.0)
        err = _rel(bs, ref.beta)
        _say(f"  sweeps={infos['iters']} rel err vs oracle {err:.3e}")
        assert err <= 1e-10


def test_sparse_values_errors():
    d = synth.make("binary", 4000, 5, 2, 221, density=0.1)
    X, ptr, idx, vals = _sparse_values(d, 5)
    bad = idx.copy()
    bad[1] = bad[0]                       # a repeated row in column 0
    with pytest.raises(coxmi.CoxError) as e:
        coxmi.CoxModel.sparse(4000, ptr, bad, vals, d.time, d.event, d.stratum)
    assert e.value.code == coxmi.COX_EINVAL
    v2 = vals.copy()
    v2[0] = np.inf
    with pytest.raises(coxmi.CoxError) as e:
        coxmi.CoxModel.sparse(4000, ptr, idx, v2, d.time, d.event, d.stratum)
    assert e.value.code == coxmi.COX_EINVAL
    with coxmi.CoxModel.sparse(4000, ptr, idx, vals, d.time, d.event, d.stratum) as m:
        for call in (lambda: m.evaluate_full(np.zeros(5)), lambda: m.intervals(d.time, d.event, d.stratum, [0.5]),
                     lambda: m.resample(np.ones(4000, np.uint32))):
            with pytest.raises(coxmi.CoxError) as e:
                call()
            assert e.value.code == coxmi.COX_EUNSUPPORTED
