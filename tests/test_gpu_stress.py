"""Determinism under repetition: the cross-workgroup scan and the persistent CCD kernel
use fixed-order reductions and epoch-tagged exchanges (no float atomics), so repeated
runs must agree bit for bit whatever the arrival order of workgroups.

* the raw segmented scan over 2e6 FP64 values (many tiles, segments that span tiles, so
  every tile's carry comes from the look-back) run 2000 times;
* a few-strata CCD fit (every coordinate's scan crosses tiles) run 25 times, and an
  evaluation 200 times.
"""
import numpy as np
import pytest

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


def test_lookback_scan_repeated_bitwise():
    n = 2_000_000
    rng = np.random.default_rng(3)
    a = rng.standard_normal(n)
    flags = np.zeros(n, np.uint8)
    flags[rng.choice(n, 40, replace=False)] = 1     # 41 segments of ~50k rows: most tiles carry in
    ta = torch.from_numpy(a).cuda()
    tf = torch.from_numpy(flags).cuda()
    first = torch.empty_like(ta)
    torch.cuda.synchronize()
    coxmi.cox_segscan_f64(ta.data_ptr(), tf.data_ptr(), first.data_ptr(), n)
    torch.cuda.synchronize()
    ref = first.cpu().numpy()
    _say("segscan 2e6 x 2000 repetitions")
    out = torch.empty_like(ta)
    mismatches = 0
    for rep in range(2000):
        coxmi.cox_segscan_f64(ta.data_ptr(), tf.data_ptr(), out.data_ptr(), n)
        if not torch.equal(out, first):
            mismatches += 1
        if rep % 500 == 499:
            _say(f"  {rep + 1} repetitions, {mismatches} mismatches")
    assert mismatches == 0
    # and the first result is the plain sequential scan's, to rounding of the sums
    seg = np.cumsum(flags) + (flags[0] == 0)
    for s in np.unique(seg)[:3]:
        idx = np.flatnonzero(seg == s)
        np.testing.assert_allclose(ref[idx], np.cumsum(a[idx]), rtol=0, atol=1e-9)


def test_ccd_fit_repeated_bitwise():
    d = synth.make("ar1", 900_000, 10, 3, 31, beta_sd=0.5)
    _say("few-strata CCD fit x 25, evaluation x 200")
    with coxmi.CoxModel(d.X, d.time, d.event, d.stratum, gamma=1.0, tol=1e-12) as m:
        b0, i0 = m.fit()
        for _ in range(24):
            b, i = m.fit()
            assert np.array_equal(b, b0) and i["iters"] == i0["iters"]
        o0, g0, h0 = m.evaluate(b0)
        for _ in range(199):
            o, g, h = m.evaluate(b0)
            assert o == o0 and np.array_equal(g, g0) and np.array_equal(h, h0)
