"""The allocation-free scan (cox_segscan_f64_noalloc) against the allocating entry point
(cox_segscan_f64) through the C ABI: bit-identical outputs on two calls in a row, the
second smaller than the first (the scratch array keeps the first call's packets, which
carry the same epoch, so the clear before each scan is what this checks), and both equal
to the exact segmented sums of integer-valued inputs."""
import numpy as np
import pytest

from paper_2310_16238_amd import coxmi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    coxmi.lib()


def _exact(a, f):
    """Segmented +scan of integer-valued doubles (exact in FP64 below 2^53)."""
    out = np.empty_like(a)
    run = 0.0
    for i in range(a.size):
        run = a[i] if (i == 0 or f[i]) else run + a[i]
        out[i] = run
    return out


def _inputs(n, density, seed):
    rng = np.random.default_rng(seed)
    a = rng.integers(-1000, 1000, size=n).astype(np.float64)
    f = (rng.random(n) < density).astype(np.uint8)
    return a, f


def _scan(fn, a, f):
    ta = torch.tensor(a, dtype=torch.float64, device="cuda")
    tf = torch.tensor(f, dtype=torch.uint8, device="cuda")
    tb = torch.full_like(ta, float("nan"))
    torch.cuda.synchronize()
    fn(ta.data_ptr(), tf.data_ptr(), tb.data_ptr(), ta.numel())
    return tb.cpu().numpy()


@pytest.mark.parametrize("sizes", [(3_000_017, 100_003), (1_048_576, 4_097)], ids=["3e6-then-1e5", "1m-then-4k"])
def test_noalloc_scan_matches_allocating_scan(sizes):
    for k, n in enumerate(sizes):
        # few heads, so most workgroups take their carry from the look-back over the scratch packets
        a, f = _inputs(n, 2e-6, 100 + k)
        print(f"[gpu-test] noalloc segscan call {k + 1}: n={n}", flush=True)
        got = _scan(coxmi.cox_segscan_f64_noalloc, a, f)
        ref = _scan(coxmi.cox_segscan_f64, a, f)
        assert np.array_equal(got, ref)
        if n <= 200_000:
            assert np.array_equal(got, _exact(a, f))
        else:
            # exact segmented sums by cumulative sums per segment
            starts = np.flatnonzero(np.r_[1, f[1:]])
            seg = np.cumsum(np.r_[1, f[1:]]) - 1
            cs = np.cumsum(a)
            base = np.r_[0.0, cs][starts][seg]
            assert np.array_equal(got, cs - base)


def test_noalloc_scan_limits():
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    coxmi.cox_segscan_f64_noalloc(0, 0, 0, 0)          # n = 0 is a no-op
    n = min(cus, 256) * 1024 * 16 + 1
    ta = torch.zeros(n, dtype=torch.float64, device="cuda")
    tf = torch.zeros(n, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    with pytest.raises(coxmi.CoxError) as e:
        coxmi.cox_segscan_f64_noalloc(ta.data_ptr(), tf.data_ptr(), ta.data_ptr(), n)
    assert e.value.code == coxmi.COX_EUNSUPPORTED
