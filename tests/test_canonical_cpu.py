"""The library's host canonical order (Sec. 2.7; cox_canonical_order) against the
oracle's, bit-exact, across the paths of its sort: one stratum of many sizes, dense
and sparse stratum labels (counting sort and radix sort on the label), times equal in
their high bits (the full-key fix-up of the radix sort on the high word), ties, -0
and +0 times, negative and extreme times."""
import numpy as np
import pytest

from oracle import cox_oracle as orc
from paper_2310_16238_amd import coxmi


def _check(time, event, stratum=None):
    perm, meta = coxmi.cox_canonical_order(time, event, stratum)
    L = orc.canonical_layout(time, event, stratum)
    np.testing.assert_array_equal(perm, L.perm)
    np.testing.assert_array_equal(meta, L.meta)


@pytest.mark.parametrize("n", [1, 2, 31, 32, 33, 4096, 4097, 20_000])
def test_one_stratum_all_sort_sizes(n):
    rng = np.random.default_rng(n)
    t = rng.exponential(1.0, n)
    e = (rng.random(n) < 0.6).astype(np.uint8)
    _check(t, e)
    _check(np.round(t, 1), e)   # heavy ties


@pytest.mark.parametrize("K", [2, 37, 500, 5000])
def test_dense_and_shifted_labels(K):
    rng = np.random.default_rng(K)
    n = 30_000
    s = (rng.integers(0, K, n) * 7 - 100).astype(np.int32)
    t = np.round(rng.exponential(1.0, n), 2)
    e = (rng.random(n) < 0.5).astype(np.uint8)
    _check(t, e, s)


def test_sparse_labels_take_the_radix_path():
    rng = np.random.default_rng(5)
    n = 10_000
    s = rng.choice(np.array([-2**31, -7, 0, 3, 2**31 - 1, 123456789], dtype=np.int64), n).astype(np.int32)
    t = rng.standard_normal(n) * 1e300
    e = (rng.random(n) < 0.5).astype(np.uint8)
    _check(t, e, s)


def test_signed_zero_and_extreme_times():
    t = np.array([0.0, -0.0, 1e-308, -1e-308, 5e-324, -5e-324, 1.7e308, -1.7e308, 0.0, -0.0, 2.0, 2.0])
    e = np.array([1, 0, 1, 1, 0, 1, 1, 0, 1, 1, 0, 1], dtype=np.uint8)
    _check(t, e)
    _check(t, e, np.array([1, 1, 0, 0, 1, 1, 0, 0, 1, 1, 0, 0], dtype=np.int32))


def test_errors():
    with pytest.raises(coxmi.CoxError):
        coxmi.cox_canonical_order(np.array([1.0, np.nan]), np.array([1, 0], np.uint8))
    with pytest.raises(coxmi.CoxError):
        coxmi.cox_canonical_order(np.array([1.0, 2.0]), np.array([1, 2], np.uint8))
    with pytest.raises(coxmi.CoxError):
        coxmi.cox_canonical_order(np.zeros(0), np.zeros(0, np.uint8))


@pytest.mark.parametrize("bases,spread", [(4, 8), (4, 1000), (700, 8), (700, 1000)])
def test_times_that_differ_only_in_low_bits(bases, spread):
    """Times equal in their top 32 bits and different below (runs of equal high words, put in
    order by the full time: short runs by insertion, long runs by a stable merge), with exact
    ties among them, one stratum and many."""
    rng = np.random.default_rng(spread + bases)
    n = 5000
    pool = np.concatenate([[1.0, 3.5, -2.25, 1e-300], rng.exponential(1.0, bases)])[:bases]
    base = pool[rng.integers(0, bases, n)]
    t = base + rng.integers(0, spread, n) * np.spacing(np.abs(base))
    e = (rng.random(n) < 0.5).astype(np.uint8)
    _check(t, e)
    _check(t, e, rng.integers(0, 40, n).astype(np.int32))


def test_many_rows_many_strata():
    rng = np.random.default_rng(77)
    n = 300_000
    t = rng.exponential(1.0, n)
    t[rng.random(n) < 0.1] = 1.0   # a heavy tie
    e = (rng.random(n) < 0.5).astype(np.uint8)
    _check(t, e, rng.integers(0, 3000, n).astype(np.int32))
