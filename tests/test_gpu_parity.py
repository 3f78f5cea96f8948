"""GPU parity: the HIP path through the C ABI against the CPU oracle, same seeded inputs.

Tolerances (FP64 on both sides, different summation orders):
* integer work (canonical order, row words, scans of integers): bit-exact;
* per-coordinate sums g', g'': |gpu - oracle| <= 1e-11 * max(1, E) where E is the
  number of events (each sum has E terms of size O(1));
* -log L: |gpu - oracle| <= 1e-11 * max(E, |-log L|): its terms are logs of risk-set
  sums of up to n_k rows, and a sequential n_k-term sum has relative rounding error
  up to n_k * 2^-53 (about 7e-11 for a 6e5-row stratum), correlated across events;
* fitted beta: max|gpu - oracle| / max|oracle| <= 1e-10; l1 zero pattern identical.
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


# ------------------------------------------------------------------ scan primitive

def _gpu_scan(a, f):
    ta = torch.tensor(a, dtype=torch.float64, device="cuda")
    tf = torch.tensor(f, dtype=torch.uint8, device="cuda")
    tb = torch.empty_like(ta)
    torch.cuda.synchronize()
    coxmi.cox_segscan_f64(ta.data_ptr(), tf.data_ptr(), tb.data_ptr(), ta.numel())
    return tb.cpu().numpy()


def test_segscan_paper_example():
    from conftest import read_golden
    g = read_golden("segscan_example.txt")
    _say("segscan paper example")
    np.testing.assert_array_equal(_gpu_scan(np.array(g["a"]), np.array(g["f"], dtype=np.uint8)), np.array(g["b"]))


@pytest.mark.parametrize("n", [1, 2, 63, 64, 1023, 1024, 1025, 3 * 2048 + 17, 262144 + 5, 1 << 21])
@pytest.mark.parametrize("density", [0.0, 1e-4, 0.05, 1.0])
def test_segscan_integers_bit_exact(n, density):
    _say(f"segscan n={n} density={density}")
    rng = np.random.default_rng(n + int(density * 1000))
    a = rng.integers(-1000, 1000, size=n).astype(np.float64)
    f = (rng.random(n) < density).astype(np.uint8)
    expect = orc.segmented_scan_c(a, f)
    np.testing.assert_array_equal(_gpu_scan(a, f), expect)


def test_segscan_empty_is_noop():
    coxmi.cox_segscan_f64(0, 0, 0, 0)


# ------------------------------------------------------------------ layout

@pytest.mark.parametrize("K,ties", [(1, False), (1, True), (37, True), (5000, True)])
def test_layout_bit_exact(K, ties):
    d = synth.config_small(n=20000, K=K, ties=ties)
    d.stratum = (d.stratum * 7 - 100).astype(np.int32)   # labels need not be 0..K-1
    _say(f"layout K={K} ties={ties}")
    L = orc.canonical_layout(d.time, d.event, d.stratum)
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum) as m:
        perm, meta = m.layout()
    np.testing.assert_array_equal(perm, L.perm)
    np.testing.assert_array_equal(meta, L.meta)


# ------------------------------------------------------------------ per-coordinate sums

@pytest.mark.parametrize("n,K", [(5000, 1), (5000, 250), (150_000, 7500), (600_000, 1), (600_000, 30_000)])
def test_coordinate_and_evaluate_parity(n, K):
    d = synth.make("ar1", n, 6, K, seed=100 + K, beta_sd=0.5, tie_round=100.0)
    beta = np.array([0.3, -0.4, 0.25, 0.0, 0.6, -0.2])
    _say(f"coordinate parity n={n} K={K}")
    L = orc.canonical_layout(d.time, d.event, d.stratum)
    Xc = orc.to_canonical(d.X, L)
    eta = Xc @ beta
    tol = 1e-11 * max(1.0, float(d.event.sum()))
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum) as m:
        for j in range(6):
            got = m.coordinate(beta, j)
            ref = orc.coord_terms(Xc, L, j, eta)
            assert abs(got[0] - ref["grad"]) <= tol, (j, got[0], ref["grad"])
            assert abs(got[1] - ref["hess"]) <= tol, (j, got[1], ref["hess"])
            assert abs(got[2] - ref["obj"]) <= 1e-11 * max(d.event.sum(), abs(ref["obj"])), (j, got[2], ref["obj"])
            assert abs(got[3] - ref["m2"]) <= tol
        obj, g, h = m.evaluate(beta)
    fe = orc.full_eval(Xc, L, beta, want_info=False)
    assert abs(obj - fe.objective) <= 1e-11 * max(d.event.sum(), abs(fe.objective))
    np.testing.assert_allclose(g, fe.grad, rtol=0, atol=tol)
    np.testing.assert_allclose(h, fe.hess_diag, rtol=0, atol=tol)


def test_tile_boundary_strata():
    """Strata that end exactly at, one before and one after workgroup tile boundaries."""
    n = 3 * 512 + 40
    bounds = [0, 511, 512, 513, 1024, 1100, 1535, 1536, 1537, n]
    stratum = np.zeros(n, dtype=np.int32)
    for k in range(len(bounds) - 1):
        stratum[bounds[k]:bounds[k + 1]] = k
    rng = np.random.default_rng(5)
    X = np.asfortranarray(rng.standard_normal((n, 3)))
    # decreasing times inside each stratum keep the canonical order equal to the input order
    time = np.concatenate([np.sort(rng.exponential(1.0, bounds[k + 1] - bounds[k]))[::-1]
                           for k in range(len(bounds) - 1)])
    event = (rng.random(n) < 0.6).astype(np.uint8)
    beta = np.array([0.5, -0.3, 0.2])
    L = orc.canonical_layout(time, event, stratum)
    assert np.array_equal(L.perm, np.arange(n))
    Xc = orc.to_canonical(X, L)
    fe = orc.full_eval(Xc, L, beta, want_info=False)
    with coxmi.CoxModel(X, time, event, stratum) as m:
        obj, g, h = m.evaluate(beta)
    tol = 1e-11 * event.sum()
    assert abs(obj - fe.objective) <= tol
    np.testing.assert_allclose(g, fe.grad, atol=tol, rtol=0)
    np.testing.assert_allclose(h, fe.hess_diag, atol=tol, rtol=0)


def test_wave_aligned_layout_edges():
    """Strata of at most one wave's rows (64 at one row per thread): the layout pads them to
    wave boundaries and every wave scans on its own.  Sizes include exactly 64, 63, 65-free
    runs of 1-row strata and strata that would otherwise straddle a wave or tile boundary."""
    rng = np.random.default_rng(17)
    sizes = []
    pattern = [64, 1, 63, 2, 64, 30, 50, 64, 1, 1, 1, 33, 64, 40, 24, 64]
    while sum(sizes) < 20_000:
        sizes.extend(pattern)
    n = sum(sizes)
    stratum = np.repeat(np.arange(len(sizes), dtype=np.int32), sizes)
    perm = rng.permutation(n)
    stratum = stratum[perm]
    X = np.asfortranarray(rng.standard_normal((n, 4)))
    time = np.floor(rng.exponential(1.0, n) * 50) / 50       # ties
    event = (rng.random(n) < 0.6).astype(np.uint8)
    beta = np.array([0.4, -0.3, 0.2, 0.1])
    L = orc.canonical_layout(time, event, stratum)
    Xc = orc.to_canonical(X, L)
    fe = orc.full_eval(Xc, L, beta, want_info=False)
    tol = 1e-11 * max(1.0, float(event.sum()))
    _say(f"wave-aligned layout n={n} strata={len(sizes)}")
    with coxmi.CoxModel(X, time, event, stratum) as m:
        obj, g, h = m.evaluate(beta)
        assert coxmi.cox_shape(m.h)[2] > n   # padded
        b, info = m.fit()
    assert abs(obj - fe.objective) <= 1e-11 * max(event.sum(), abs(fe.objective))
    np.testing.assert_allclose(g, fe.grad, atol=tol, rtol=0)
    np.testing.assert_allclose(h, fe.hess_diag, atol=tol, rtol=0)
    ref = orc.fit_newton(X, time, event, stratum, tol=1e-14)
    assert info["status"] == coxmi.COX_OK and _rel(b, ref.beta) <= 1e-10


# ------------------------------------------------------------------ fits

@pytest.mark.parametrize("K", [1, 10, 500, 5000])
@pytest.mark.parametrize("ties", [False, True])
@pytest.mark.parametrize("gamma", [math.sqrt(2.0), 0.0])
def test_fit_small_config(K, ties, gamma):
    d = synth.config_small(K=K, ties=ties, gamma=gamma)
    _say(f"fit small K={K} ties={ties} gamma={gamma:.3f}")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, gamma=gamma, tol=1e-13) as m:
        beta, info = m.fit()
    ref = orc.fit_ccd(d.X, d.time, d.event, d.stratum, gamma=gamma, tol=1e-13)
    assert info["status"] == coxmi.COX_OK and ref.converged
    assert beta[0] == 0.0                        # ones column stays pinned
    assert np.array_equal(beta == 0.0, ref.beta == 0.0)
    assert _rel(beta, ref.beta) <= 1e-10
    if gamma == 0.0:
        nw = orc.fit_newton(d.X, d.time, d.event, d.stratum)
        assert _rel(beta, nw.beta) <= 1e-10
    assert info["kkt_inf"] <= 1e-8 * max(1.0, d.event.sum())


def test_fit_ar1_full_size():
    """The N = 1e6, P = 50, K = 5e4 AR(1) workload, to convergence, against the Newton optimum."""
    d = synth.config_ar1()
    _say("fit ar1 n=1e6 p=50 K=5e4")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, tol=1e-12) as m:
        beta, info = m.fit()
        ms = m.kernel_ms()
    _say(f"  sweeps={info['iters']} kernel_ms={ms:.2f}")
    assert info["status"] == coxmi.COX_OK
    nw = orc.fit_newton(d.X, d.time, d.event, d.stratum, tol=1e-14)
    assert nw.converged
    err = _rel(beta, nw.beta)
    _say(f"  rel_err vs Newton oracle = {err:.3e}")
    assert err <= 1e-10


def test_fit_deterministic_and_warm_start():
    d = synth.config_small(n=40000, K=400, ties=True)
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, gamma=d.gamma) as m:
        b1, i1 = m.fit()
        b2, i2 = m.fit()
        assert np.array_equal(b1, b2) and i1["iters"] == i2["iters"]
        b3, i3 = m.fit(beta0=b1)          # resume from the estimate: converges at once
        assert i3["iters"] <= 2 and _rel(b3, b1) <= 1e-12


def test_not_converged_status():
    d = synth.config_small(n=5000)
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, max_iter=1) as m:
        beta, info = m.fit()
    assert info["status"] == coxmi.COX_NOT_CONVERGED and info["iters"] == 1
    assert np.all(np.isfinite(beta))


def test_edge_cases():
    # a single row with an event: every ratio is 1, nothing moves
    with coxmi.CoxModel(np.array([[2.0]]), np.array([1.0]), np.array([1], np.uint8)) as m:
        beta, info = m.fit()
        assert beta[0] == 0.0 and info["status"] == 0
    # no events at all: g' = g'' = 0 everywhere
    d = synth.config_small(n=3000)
    with coxmi.CoxModel(d.X, d.time, np.zeros(3000, np.uint8), d.stratum) as m:
        obj, g, h = m.evaluate(np.ones(10) * 0.1)
        assert obj == 0.0 and np.all(g == 0.0) and np.all(h == 0.0)
        beta, info = m.fit()
        assert np.all(beta == 0.0)
    # every row its own stratum
    n = 2000
    rng = np.random.default_rng(3)
    X = rng.standard_normal((n, 2))
    with coxmi.CoxModel(X, rng.exponential(1.0, n), np.ones(n, np.uint8), np.arange(n, dtype=np.int32)) as m:
        obj, g, h = m.evaluate(np.array([0.7, -0.2]))
        assert abs(obj) <= 1e-12 * n and np.all(np.abs(g) <= 1e-12 * n) and np.all(np.abs(h) <= 1e-12 * n)


def test_dynamic_range_falls_back_to_the_full_evaluation():
    """X beta beyond the range one shift per fit can hold in FP64: a stratum-constant offset of
    2000 in a column (the partial likelihood ignores it; exp(x'b - c) of the other stratum
    underflows for any single c).  cox_evaluate then answers from the full evaluation (running-
    maximum scans) and cox_fit finishes by Newton / proximal Newton steps on it -- the oracle's
    values and optima (running-shift scans) to the usual bars."""
    rng = np.random.default_rng(31)
    n = 3000
    st = (np.arange(n) % 2).astype(np.int32)
    z = rng.normal(size=(n, 2))
    X = z.copy()
    X[:, 0] += 2000.0 * st
    lin = z @ np.array([0.6, -0.4])
    T = rng.exponential(1.0 / np.exp(lin))
    C = rng.exponential(1.0, n)
    time = np.minimum(T, C)
    event = (T <= C).astype(np.uint8)
    b0 = np.array([0.6, -0.4])
    with coxmi.CoxModel(X, time, event, st, tol=1e-13) as m:
        obj, g, hd = m.evaluate(b0)
        beta, info = m.fit()
    with coxmi.CoxModel(X, time, event, st, gamma=5.0, tol=1e-13) as m:
        beta1, info1 = m.fit()
    L = orc.canonical_layout(time, event, st)
    fe = orc.full_eval(orc.to_canonical(X, L), L, b0, want_info=False)
    E = float(event.sum())
    assert abs(obj - fe.objective) <= 1e-11 * max(E, abs(fe.objective))
    assert np.max(np.abs(g - fe.grad)) <= 1e-11 * max(1.0, E) * 2000.0
    assert np.max(np.abs(hd - fe.hess_diag)) <= 1e-11 * max(1.0, E) * 2000.0 ** 2
    # the offset is constant within strata, so the optima are those of the data without it
    ref = orc.fit_newton(z, time, event, st, tol=1e-14)
    assert ref.converged and info["status"] == coxmi.COX_OK and info["fallback"] == 1, info
    assert np.max(np.abs(beta - ref.beta)) <= 1e-10 * np.max(np.abs(ref.beta))
    ref1 = orc.fit_ccd(z, time, event, st, gamma=5.0, tol=1e-14, max_sweeps=5000)
    assert ref1.converged and info1["status"] == coxmi.COX_OK and info1["fallback"] == 1, info1
    assert np.array_equal(beta1 == 0.0, ref1.beta == 0.0)
    assert np.max(np.abs(beta1 - ref1.beta)) <= 1e-10 * np.max(np.abs(ref1.beta))
    # a fit within range takes the persistent kernel
    with coxmi.CoxModel(z, time, event, st, tol=1e-13) as m:
        _, info2 = m.fit()
    assert info2["fallback"] == 0
