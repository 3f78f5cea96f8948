"""GPU tests of the fit server's persistent rounds (cox_server_options.fused_rounds > 0:
one cooperative launch runs many rounds of every resident fit, its phases separated by
grid-wide barriers): every fit's estimate, iteration count, objective and status equal,
bit for bit, those of the server that takes every round as separate launches; a fit that
finishes early is reported while the launch still runs; arrivals during a launch join at
the next one; and the served estimates sit at the oracle's optimum.
"""
import time

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


def _l1_weight(d, share=0.2):
    L = orc.canonical_layout(d.time, d.event, d.stratum)
    g0 = orc.full_eval(orc.to_canonical(d.X, L), L, np.zeros(d.p), want_info=False).grad
    return share * float(np.max(np.abs(g0[1:])))


def _workload():
    """Unpenalised requests of uneven size (p from 3 to the server's limit of 128, one
    with many strata) and l1 requests, one warm-started."""
    reqs = [synth.serving_request(i, seed=21, n_range=(400, 30_000), p_range=(3, 100)) for i in range(12)]
    reqs.append(synth.serving_request(0, seed=22, n_range=(9_000, 9_001), p_range=(128, 128)))
    jobs = [(d, {}) for d in reqs]
    for d in reqs[:4]:
        g = _l1_weight(d)
        jobs.append((d, dict(gamma=g)))
    d = reqs[1]
    jobs.append((d, dict(gamma=0.5 * _l1_weight(d), beta0=np.full(d.p, 0.01))))
    return jobs


def _serve(jobs, fused_rounds, stagger=0.0):
    with coxmi.CoxServer(hbm_budget=1 << 30, staging_bytes=256 << 20, prep_threads=4,
                         fused_rounds=fused_rounds) as srv:
        tickets = []
        for d, kw in jobs:
            tickets.append(srv.submit(d.X, d.time, d.event, d.stratum, **kw))
            if stagger:
                time.sleep(stagger)
        assert srv.drain(timeout=150.0)
        out = [srv.poll(t) for t in tickets]
        st = srv.stats()
    return out, st


def _same(a, b, label):
    for k, ((ba, ia, _), (bb, ib, _)) in enumerate(zip(a, b)):
        assert np.array_equal(ba, bb), (label, k, _rel(ba, bb))
        for key in ("status", "iters", "coord_evals", "objective", "kkt_inf", "last_step", "n_pinned"):
            assert ia[key] == ib[key], (label, k, key, ia[key], ib[key])


def test_fused_rounds_equal_separate_launches():
    jobs = _workload()
    _say(f"{len(jobs)} requests, p in [{min(d.p for d, _ in jobs)}, {max(d.p for d, _ in jobs)}], "
         f"n in [{min(d.n for d, _ in jobs)}, {max(d.n for d, _ in jobs)}]")
    ref, st0 = _serve(jobs, 0)
    _say(f"  separate launches: {st0['iterations']} rounds")
    for R in (1, 3, 200):
        out, st = _serve(jobs, R)
        _say(f"  fused_rounds={R}: {st['iterations']} rounds, completed {st['completed']}")
        assert st["completed"] == len(jobs) and st["resident_now"] == 0
        _same(ref, out, f"R={R}")
        for (beta, info, times) in out:
            assert info["status"] == coxmi.COX_OK
            assert times["submit_s"] <= times["admit_s"] <= times["done_s"]
    # the served estimates against the oracle (two unpenalised, one l1)
    for k in (0, 12):
        d = jobs[k][0]
        oref = orc.fit_newton(d.X, d.time, d.event, d.stratum, tol=1e-14)
        assert _rel(ref[k][0], oref.beta) <= 1e-10, (k, _rel(ref[k][0], oref.beta))
    d, kw = jobs[13]
    oref = orc.fit_ccd(d.X, d.time, d.event, d.stratum, gamma=kw["gamma"], tol=1e-14, max_sweeps=5000)
    assert np.array_equal(ref[13][0] == 0.0, oref.beta == 0.0)
    assert _rel(ref[13][0], oref.beta) <= 1e-10


def test_early_finisher_reported_during_the_launch():
    big = synth.serving_request(0, seed=23, n_range=(60_000, 60_001), p_range=(110, 110))
    small = synth.serving_request(1, seed=23, n_range=(500, 501), p_range=(3, 3))
    with coxmi.CoxServer(hbm_budget=1 << 30, prep_threads=2, fused_rounds=500) as srv:
        tb = srv.submit(big.X, big.time, big.event, big.stratum)
        ts = srv.submit(small.X, small.time, small.event, small.stratum)
        assert srv.drain(timeout=120.0)
        rb, rs = srv.poll(tb), srv.poll(ts)
        st = srv.stats()
    _say(f"  big {rb[1]['iters']} steps done {rb[2]['done_s']:.4f}; small {rs[1]['iters']} steps "
         f"done {rs[2]['done_s']:.4f}; rounds {st['iterations']}")
    assert rb[1]["status"] == coxmi.COX_OK and rs[1]["status"] == coxmi.COX_OK
    if rs[1]["coord_evals"] < rb[1]["coord_evals"] and rs[2]["admit_s"] <= rb[2]["admit_s"] + 1e-3:
        assert rs[2]["done_s"] < rb[2]["done_s"]
    for d, (beta, info, _) in ((big, rb), (small, rs)):
        oref = orc.fit_newton(d.X, d.time, d.event, d.stratum, tol=1e-14)
        assert _rel(beta, oref.beta) <= 1e-10


def test_fused_arrivals_join_later_launches():
    jobs = [(synth.serving_request(i, seed=24, n_range=(1_000, 40_000), p_range=(5, 90)), {}) for i in range(14)]
    ref, _ = _serve(jobs, 0)
    out, st = _serve(jobs, 64, stagger=0.003)
    _say(f"  staggered arrivals, fused: {st['iterations']} rounds, mean resident {st['mean_resident']:.2f}")
    _same(ref, out, "staggered")
    admits = [r[2]["admit_s"] for r in out]
    dones = [r[2]["done_s"] for r in out]
    assert any(admits[j] < max(dones[:j]) for j in range(1, len(out)))


def test_fused_rounds_option_checked():
    for bad in (-1, 5000):
        with pytest.raises(coxmi.CoxError) as e:
            coxmi.CoxServer(fused_rounds=bad)
        assert e.value.code == coxmi.COX_EINVAL


def test_fused_edge_cases_and_device_requests():
    """One row, no events, one column with strata, a stratum longer than a scan tile, and
    device-resident requests: the persistent rounds give what the separate launches give."""
    rng = np.random.default_rng(5)
    cases = [
        (np.ones((1, 1)), np.array([1.0]), np.array([1], np.uint8), None),
        (rng.standard_normal((50, 3)), rng.random(50), np.zeros(50, np.uint8), None),
        (rng.standard_normal((400, 1)), rng.exponential(1.0, 400), (rng.random(400) < 0.5).astype(np.uint8),
         (np.arange(400) % 4).astype(np.int32)),
    ]
    long_stratum = synth.make("iid", 9_000, 7, 1, 23, intercept=True)
    multi_tile = synth.serving_request(3, seed=25, n_range=(30_000, 30_001), p_range=(20, 20))

    def run(fused):
        with coxmi.CoxServer(prep_threads=2, fused_rounds=fused) as srv:
            tk = [srv.submit(*c) for c in cases]
            for d in (long_stratum, multi_tile):
                tk.append(srv.submit(d.X, d.time, d.event, d.stratum))
                dev = (torch.from_numpy(np.ascontiguousarray(d.X.T)).cuda().t(),
                       torch.from_numpy(np.ascontiguousarray(d.time)).cuda(),
                       torch.from_numpy(np.ascontiguousarray(d.event, dtype=np.uint8)).cuda(),
                       None if d.stratum is None else
                       torch.from_numpy(np.ascontiguousarray(d.stratum, dtype=np.int32)).cuda())
                torch.cuda.synchronize()
                tk.append(srv.submit_device(*dev))
            assert srv.drain(timeout=100.0)
            return [srv.poll(t) for t in tk]

    ref = run(0)
    out = run(16)
    _same(ref, out, "edge")
    for (X, t, e, s), (beta, info, _) in zip(cases, out):
        assert info["status"] == coxmi.COX_OK, info
        if e.sum() == 0 or X.shape[0] == 1:
            assert np.all(beta == 0.0)
        else:
            assert _rel(beta, orc.fit_newton(X, t, e, s, tol=1e-14).beta) <= 1e-10
    for k, d in enumerate((long_stratum, multi_tile)):
        host, dev = out[3 + 2 * k], out[4 + 2 * k]
        assert np.array_equal(host[0], dev[0]), d.name
        assert _rel(dev[0], orc.fit_newton(d.X, d.time, d.event, d.stratum, tol=1e-14).beta) <= 1e-10
