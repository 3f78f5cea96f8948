"""Breslow cumulative baseline hazard in the oracle, pinned.

* beta = 0, one stratum: the Nelson-Aalen estimator, worked by hand from at-risk counts;
* at any beta, within each stratum sum_i (delta_i - exp(x_i'beta) Lambda_0(Y_i)) = 0 (every
  event group's jump d / S0 is collected back by the rows at risk at it);
* the score: X'(exp(X beta) * Lambda_0 - delta) equals Eq. strat_g by brute force;
* adding c to every linear predictor scales Lambda_0 by exp(-c).
"""
import math

import numpy as np

from oracle import cox_oracle as o
from paper_2310_16238_amd import synth


def test_nelson_aalen_by_hand():
    # event times 1 (6 at risk), 2 (5 at risk; the censored row at 2 is still at risk), 3 (3), 5 (1)
    time = np.array([1.0, 2.0, 2.0, 3.0, 4.0, 5.0])
    event = np.array([1, 1, 0, 1, 0, 1], np.uint8)
    X = np.zeros((6, 1))
    a = 1 / 6
    b = a + 1 / 5
    c = b + 1 / 3
    expect = np.array([a, b, b, c, c, c + 1.0])
    got = o.baseline_hazard_brute(X, time, event, None, [0.0])
    np.testing.assert_allclose(got, expect, rtol=1e-15, atol=0)


def test_martingale_residuals_sum_to_zero_and_score():
    d = synth.make("iid", 120, 3, 3, 4, beta_sd=0.6, tie_round=10.0)
    for seed in range(3):
        beta = np.random.default_rng(seed).normal(0, 0.5, 3)
        lam = o.baseline_hazard_brute(d.X, d.time, d.event, d.stratum, beta)
        w = np.exp(d.X @ beta)
        for k in np.unique(d.stratum):
            r = d.stratum == k
            assert abs(np.sum(d.event[r] - w[r] * lam[r])) <= 1e-12 * max(1, d.event[r].sum())
        score = d.X.T @ (w * lam - d.event)
        np.testing.assert_allclose(score, o.grad_brute(d.X, d.time, d.event, d.stratum, beta), rtol=0, atol=1e-11)


def test_linear_predictor_shift():
    d = synth.make("iid", 80, 2, 2, 6, beta_sd=0.5)
    X1 = np.column_stack([d.X, np.ones(80)])
    beta = np.array([0.3, -0.4, 1.7])      # the ones column adds 1.7 to every linear predictor
    base = o.baseline_hazard_brute(d.X, d.time, d.event, d.stratum, beta[:2])
    shifted = o.baseline_hazard_brute(X1, d.time, d.event, d.stratum, beta)
    np.testing.assert_allclose(shifted, base * math.exp(-1.7), rtol=1e-13, atol=0)
