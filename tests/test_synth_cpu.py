"""The synthetic-input generators: draws that stay inside the floating-point range."""
import numpy as np

from paper_2310_16238_amd import synth


def test_log_scale_times_match_the_direct_draw():
    """Drawing on the log scale is the same model: on a design whose hazards stay in range,
    the events are identical and exp(log Y) equals Y to rounding."""
    a = synth.make("iid", 20_000, 6, 40, 17, beta_sd=0.5)
    b = synth.make("iid", 20_000, 6, 40, 17, beta_sd=0.5, log_time=True)
    assert np.array_equal(a.event, b.event)
    assert np.allclose(np.exp(b.time), a.time, rtol=1e-12, atol=0.0)
    assert np.array_equal(np.argsort(a.time, kind="stable"), np.argsort(b.time, kind="stable"))


def test_heavy_tailed_draw_has_no_overflow_or_zero_times():
    """Student-t(3) columns with N(0,1) coefficients put X beta beyond exp()'s range; the
    draw must neither overflow nor collapse rows onto a common time."""
    with np.errstate(over="raise", under="ignore", invalid="raise", divide="raise"):
        d = synth.config_heavy(n=200_000, p=500, K=10_000)
    eta = d.X @ d.beta_true
    assert np.max(np.abs(eta)) > 100.0          # the case that overflowed a direct draw in FP32
    assert np.all(np.isfinite(d.time))
    assert np.unique(d.time).size == d.n        # continuous times: no ties at all
    assert 0.3 < d.event.mean() < 0.7
