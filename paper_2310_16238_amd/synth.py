"""Seeded synthetic inputs shaped like the stratified-Cox workloads.

This module only *draws* data: designs, true coefficients, strata and the
(time, event) response.  It holds none of the estimator's arithmetic (no risk
sets, scans, likelihoods or derivatives), so it can feed both the HIP path and
the CPU oracle without coupling them.

Response model (Sec. 2.1, proportional hazards within stratum k):
    T_i ~ Exponential(rate = lambda_k * exp(x_i' beta_true))
    C_i ~ Exponential(rate = lambda_k)          (independent censoring)
    Y_i = min(T_i, C_i),  delta_i = 1[T_i <= C_i]
with lambda_k = exp(u_k), u_k ~ U(-1, 1) (lambda = 1 when K = 1).  The paper
does not state how its synthetic times were drawn; this is the reading used
throughout (about half of the rows are events).

Strata (Sec. 3.1 sweeps the number of strata; equal-sized strata as in the
propensity-score stratification of Sec. 3.2): stratum_i = floor(pi(i) K / N)
for a seeded permutation pi, so stratum sizes differ by at most one.

Draw order for a seed: X column by column, then beta_true, then the stratum
permutation and u_k, then T, then C.

Arrays: X is float64 of shape (n, p) in Fortran (column-major) order, so each
column is contiguous and ``X.ctypes.data`` is a column-major N x P matrix with
leading dimension n.  time float64[n], event uint8[n], stratum int32[n].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class CoxData:
    X: np.ndarray          # (n, p) float64, Fortran order
    time: np.ndarray       # (n,) float64
    event: np.ndarray      # (n,) uint8
    stratum: np.ndarray    # (n,) int32
    beta_true: np.ndarray  # (p,) float64
    gamma: float           # l1 strength used for this workload
    name: str

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def p(self) -> int:
        return int(self.X.shape[1])


# --------------------------------------------------------------------------- designs

def _design_iid_normal(rng, n, p, intercept):
    X = np.empty((n, p), dtype=np.float64, order="F")
    start = 0
    if intercept:
        X[:, 0] = 1.0
        start = 1
    for j in range(start, p):
        X[:, j] = rng.standard_normal(n)
    return X


def _design_ar1(rng, n, p, rho=0.5):
    """Columns x_j = rho x_{j-1} + sqrt(1-rho^2) z_j: unit variance, corr rho^|i-j|."""
    X = np.empty((n, p), dtype=np.float64, order="F")
    X[:, 0] = rng.standard_normal(n)
    c = math.sqrt(1.0 - rho * rho)
    for j in range(1, p):
        X[:, j] = rho * X[:, j - 1] + c * rng.standard_normal(n)
    return X


def _design_t3(rng, n, p, progress=None):
    """iid Student-t(3) scaled to unit variance (variance of t3 is 3)."""
    X = np.empty((n, p), dtype=np.float64, order="F")
    s = 1.0 / math.sqrt(3.0)
    for j in range(p):
        X[:, j] = rng.standard_t(3, n) * s
        if progress is not None:
            progress(j + 1, p)
    return X


def _design_mixed(rng, n, p):
    """Two common factors: x_i = z_i + f_i1 a_1 + f_i2 a_2, column j scaled by 2^(e_j).

    z_i iid N(0, I_p), f iid N(0, 1), a_1, a_2 iid N(0, I_p) loadings and
    e_j uniform in {-3..3}.  The correlation I + a_1 a_1' + a_2 a_2' makes every
    entry of X'X of the order of its diagonal, with varied signs, so a
    misplaced entry of a cross-product stands out, while the condition number
    stays of the order of p.
    """
    a = rng.standard_normal((2, p))
    X = np.empty((n, p), dtype=np.float64, order="F")
    f = rng.standard_normal((n, 2))
    for j in range(p):
        X[:, j] = rng.standard_normal(n) + f @ a[:, j]
    X *= np.exp2(rng.integers(-3, 4, size=p)).astype(np.float64)
    return X


def _design_binary(rng, n, p, density):
    """Binary indicators with P(x=1) = density (Sec. 3.1 uses 5% ones)."""
    X = np.empty((n, p), dtype=np.float64, order="F")
    for j in range(p):
        X[:, j] = (rng.random(n) < density).astype(np.float64)
    return X


# --------------------------------------------------------------------------- response

def _strata(rng, n, K):
    perm = rng.permutation(n)
    stratum = (perm.astype(np.int64) * K // n).astype(np.int32)
    u = rng.uniform(-1.0, 1.0, size=K) if K > 1 else np.zeros(1)
    return stratum, np.exp(u)


def _linear_predictor(X, beta):
    # Data generation only: the true hazard multiplier of each row.
    eta = np.zeros(X.shape[0])
    for j in np.flatnonzero(beta):
        eta += X[:, j] * beta[j]
    return eta


def _times(rng, eta, lam_row, tie_round, log_time=False):
    if log_time:
        # On the log scale: log T = log E - log lambda - eta and log C = log E' - log lambda
        # never overflow, whatever the range of eta (exp(eta) would for |eta| > 709).  The
        # returned time is log Y, a strictly increasing function of Y: the partial
        # likelihood depends on the times only through their order within a stratum.
        log_lam = np.log(lam_row)
        logT = np.log(rng.exponential(1.0, size=eta.shape[0])) - log_lam - eta
        logC = np.log(rng.exponential(1.0, size=eta.shape[0])) - log_lam
        event = (logT <= logC).astype(np.uint8)
        return np.minimum(logT, logC).astype(np.float64), event
    rate_t = lam_row * np.exp(eta)
    T = rng.exponential(1.0, size=eta.shape[0]) / rate_t
    C = rng.exponential(1.0, size=eta.shape[0]) / lam_row
    event = (T <= C).astype(np.uint8)
    Y = np.minimum(T, C)
    if tie_round:
        # Discretised follow-up (e.g. days): many exact ties in Y.
        Y = np.floor(Y * tie_round) / tie_round
    return Y.astype(np.float64), event


def make(design: str, n: int, p: int, K: int, seed: int, *, beta=None,
         beta_kind: str = "normal", beta_sd: float = 0.5, beta_nonzero: float = 1.0,
         intercept: bool = False, density: float = 0.05, tie_round: float = 0.0,
         gamma: float = 0.0, name: str = "", progress=None, log_time: bool = False) -> CoxData:
    """Draw one workload.  See the module docstring for the model and order.
    `progress(j, p)`, if given, is called after each column of the t3 design is drawn.
    With `log_time` the returned times are log Y (drawn on the log scale, see _times)."""
    if n < 1 or p < 1 or K < 1 or K > n:
        raise ValueError("need n >= 1, p >= 1, 1 <= K <= n")
    rng = np.random.default_rng(seed)
    if design == "iid":
        X = _design_iid_normal(rng, n, p, intercept)
    elif design == "ar1":
        X = _design_ar1(rng, n, p)
    elif design == "t3":
        X = _design_t3(rng, n, p, progress)
    elif design == "binary":
        X = _design_binary(rng, n, p, density)
    elif design == "mixed":
        X = _design_mixed(rng, n, p)
    else:
        raise ValueError(f"unknown design {design!r}")
    if beta is not None:
        b = np.asarray(beta, dtype=np.float64).copy()
    elif beta_kind == "normal":
        b = rng.normal(0.0, beta_sd, size=p)
        if beta_nonzero < 1.0:
            b *= rng.random(p) < beta_nonzero
    elif beta_kind == "sparse_count":
        # exactly round(beta_nonzero * p) nonzero N(0, beta_sd^2) entries at seeded positions
        b = np.zeros(p)
        nz = rng.choice(p, size=max(1, int(round(beta_nonzero * p))), replace=False)
        b[nz] = rng.normal(0.0, beta_sd, size=nz.size)
    else:
        raise ValueError(f"unknown beta_kind {beta_kind!r}")
    stratum, lam = _strata(rng, n, K)
    eta = _linear_predictor(X, b)
    Y, event = _times(rng, eta, lam[stratum], tie_round, log_time)
    return CoxData(X=X, time=Y, event=event, stratum=stratum, beta_true=b,
                   gamma=float(gamma), name=name or f"{design}-n{n}-p{p}-K{K}-s{seed}")


# --------------------------------------------------------------------------- named workloads

def config_small(n: int = 10_000, K: int = 1, seed: int = 0, ties: bool = False,
                 gamma: float = math.sqrt(2.0)) -> CoxData:
    """N=1e4, P=10: a ones column plus 9 iid N(0,1) columns, beta_true=linspace(-1,1,10).

    The l1 strength defaults to sqrt(2), the value Sec. 3.1 fixes for its synthetic fits.
    """
    return make("iid", n, 10, K, seed, beta=np.linspace(-1.0, 1.0, 10), intercept=True,
                tie_round=100.0 if ties else 0.0, gamma=gamma,
                name=f"small-n{n}-K{K}{'-ties' if ties else ''}")


def config_ar1(n: int = 1_000_000, p: int = 50, K: int = 50_000, seed: int = 1,
               ties: bool = False) -> CoxData:
    """AR(1) design corr 0.5^|i-j|, beta_true iid N(0, 0.25), default K = N/20."""
    return make("ar1", n, p, K, seed, beta_kind="normal", beta_sd=0.5,
                tie_round=100.0 if ties else 0.0, gamma=0.0,
                name=f"ar1-n{n}-p{p}-K{K}{'-ties' if ties else ''}")


def config_paper(n: int = 100_000, p: int = 1000, K: int = 5000, seed: int = 5) -> CoxData:
    """Sec. 3.1 shape: binary X with 5% ones, beta ~ N(0,1) x Bernoulli(0.2), gamma = sqrt(2)."""
    return make("binary", n, p, K, seed, beta_kind="normal", beta_sd=1.0, beta_nonzero=0.2,
                density=0.05, gamma=math.sqrt(2.0), name=f"paper-n{n}-p{p}-K{K}")


def config_mixed(n: int = 1_000_000, p: int = 200, K: int = 50_000, seed: int = 2) -> CoxData:
    """The AR(1) design at P = 200 for the reduced-precision Newton fit (seed 2)."""
    return make("ar1", n, p, K, seed, beta_kind="normal", beta_sd=0.5, gamma=0.0,
                name=f"mixed-n{n}-p{p}-K{K}")


def serving_request(i: int, seed: int = 3, n_range=(1_000, 100_000), p_range=(5, 100)) -> CoxData:
    """Request i of the serving stream: n log-uniform in n_range, p uniform in p_range,
    a ones column plus p-1 iid N(0,1) columns, beta_true iid N(0, 0.25) (sd 0.5),
    K = max(1, round(n / 100)) strata; drawn from default_rng((seed, i))."""
    rng = np.random.default_rng((seed, i))
    lo, hi = math.log(n_range[0]), math.log(n_range[1])
    n = int(round(math.exp(rng.uniform(lo, hi))))
    p = int(rng.integers(p_range[0], p_range[1] + 1))
    K = max(1, int(round(n / 100)))
    sub = int(rng.integers(0, 2**31 - 1))
    return make("iid", n, p, K, sub, beta_kind="normal", beta_sd=0.5, intercept=True, gamma=0.0,
                name=f"serve-{seed}-{i}-n{n}-p{p}")


def arrival_times(count: int, rate: float, seed: int = 3) -> np.ndarray:
    """Poisson arrivals at `rate` per second: cumulative sums of Exp(rate) gaps (seconds)."""
    rng = np.random.default_rng((seed, 1 << 20))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def config_heavy(n: int = 10_000_000, p: int = 500, K: int = 500_000, seed: int = 4, progress=None) -> CoxData:
    """Student-t(3) columns scaled to unit variance, beta_true with round(0.1 p) nonzero
    N(0, 1) entries at seeded positions (seed 4).  X beta_true spreads beyond the range of
    exp() in FP64, so the times are drawn on the log scale and returned as log Y."""
    return make("t3", n, p, K, seed, beta_kind="sparse_count", beta_sd=1.0, beta_nonzero=0.1, gamma=0.0,
                name=f"heavy-n{n}-p{p}-K{K}", progress=progress, log_time=True)


def config_step_effect(n: int = 407_828, p: int = 1000, seed: int = 6, cut: float = 10.0,
                       log_hr=(math.log(2.0), math.log(1.1)), density: float = 0.05,
                       base_rate: float = 1.0 / 365.0, censor_rate: float = 1.0 / 500.0) -> CoxData:
    """Sec. 3.3 shape: a treatment whose effect changes at `cut` days after initiation.

    Column 0 is the treatment indicator (half the subjects, the 1:1 matched comparison);
    columns 1..p-1 are binary baseline covariates with `density` ones and coefficients
    N(0, 0.25) x Bernoulli(0.2).  The treatment's log hazard ratio is log_hr[0] before the
    cut and log_hr[1] after it, so the event times come from a piecewise-exponential
    hazard: with rate a before the cut and b after, T = E / a if E < a cut, else
    cut + (E - a cut) / b, for E ~ Exp(1).  Censoring C ~ Exp(censor_rate); follow-up
    in whole days (Y = ceil(min(T, C)), at least 1); one stratum.  beta_true holds the
    baseline coefficients with the treatment entry 0 (its effect is log_hr).
    """
    rng = np.random.default_rng(seed)
    X = np.empty((n, p), dtype=np.float64, order="F")
    X[:, 0] = (rng.random(n) < 0.5).astype(np.float64)
    for j in range(1, p):
        X[:, j] = (rng.random(n) < density).astype(np.float64)
    b = rng.normal(0.0, 0.5, size=p) * (rng.random(p) < 0.2)
    b[0] = 0.0
    eta = _linear_predictor(X, b)
    a_rate = base_rate * np.exp(eta + X[:, 0] * log_hr[0])
    b_rate = base_rate * np.exp(eta + X[:, 0] * log_hr[1])
    E = rng.exponential(1.0, size=n)
    T = np.where(E < a_rate * cut, E / a_rate, cut + (E - a_rate * cut) / b_rate)
    C = rng.exponential(1.0, size=n) / censor_rate
    event = (T <= C).astype(np.uint8)
    Y = np.maximum(np.ceil(np.minimum(T, C)), 1.0)
    return CoxData(X=X, time=Y, event=event, stratum=np.zeros(n, dtype=np.int32), beta_true=b,
                   gamma=math.sqrt(2.0), name=f"step-effect-n{n}-p{p}-cut{cut:g}")


def config_legend(n: int = 946_911, p: int = 1000, K: int = 10, seed: int = 7) -> CoxData:
    """Sec. 3.2 shape: p binary covariates with 3% ones (the paper's 97% sparsity),
    coefficients N(0, 0.25) x Bernoulli(0.2), K equal-sized strata (standing in for its
    propensity-score strata); column 0 plays the unpenalised treatment covariate."""
    return make("binary", n, p, K, seed, beta_kind="normal", beta_sd=0.5, beta_nonzero=0.2, density=0.03,
             gamma=math.sqrt(2.0), name=f"legend-n{n}-p{p}-K{K}")


@dataclasses.dataclass
class SparseCoxData:
    """Indicator design in compressed sparse columns: column j is 1 at rows
    row_idx[col_ptr[j]:col_ptr[j + 1]] (ascending) and 0 elsewhere."""
    n: int
    col_ptr: np.ndarray    # (p + 1,) int64
    row_idx: np.ndarray    # (nnz,) int32
    time: np.ndarray
    event: np.ndarray
    stratum: np.ndarray
    beta_true: np.ndarray
    gamma: float
    name: str


def config_legend_sparse(n: int = 946_911, p: int = 9977, K: int = 10, density: float = 0.03,
                         seed: int = 9) -> SparseCoxData:
    """Sec. 3.2 at its full width: p indicator covariates with `density` ones (97% sparse),
    drawn column by column as the gaps between ones (geometric with success probability
    `density`), coefficients N(0, 0.25) x Bernoulli(0.2) with column 0 (the treatment) at
    log 0.8; K equal strata; the response model of make()."""
    rng = np.random.default_rng(seed)
    cols = []
    for _ in range(p):
        gaps = rng.geometric(density, size=int(n * density * 1.2) + 64)
        pos = np.cumsum(gaps) - 1
        while pos[-1] < n - 1:       # rare: draw more gaps
            more = np.cumsum(rng.geometric(density, size=int(n * density * 0.2) + 64)) + pos[-1]
            pos = np.concatenate([pos, more])
        cols.append(pos[pos < n].astype(np.int32))
    col_ptr = np.zeros(p + 1, dtype=np.int64)
    col_ptr[1:] = np.cumsum([c.size for c in cols])
    row_idx = np.concatenate(cols)
    b = rng.normal(0.0, 0.5, size=p) * (rng.random(p) < 0.2)
    b[0] = math.log(0.8)
    eta = np.zeros(n)
    for j in np.flatnonzero(b):
        eta[cols[j]] += b[j]
    stratum, lam = _strata(rng, n, K)
    Y, event = _times(rng, eta, lam[stratum], 0.0)
    return SparseCoxData(n=n, col_ptr=col_ptr, row_idx=row_idx, time=Y, event=event, stratum=stratum,
                         beta_true=b, gamma=math.sqrt(2.0), name=f"legend-sparse-n{n}-p{p}-K{K}")


def config_cough_sparse(n: int = 407_828, p: int = 9666, density: float = 0.03, cut: float = 10.0,
                        log_hr=(math.log(2.0), math.log(1.1)), seed: int = 11) -> SparseCoxData:
    """Sec. 3.3 at its full width on indicator X: column 0 a treatment indicator (half the
    subjects) whose log hazard ratio is log_hr[0] before `cut` days and log_hr[1] after,
    columns 1..p-1 indicators with `density` ones (drawn as geometric gaps), coefficients
    N(0, 0.01) x Bernoulli(0.2) (so the baseline covariates' linear predictor has sd ~0.8, and
    few subjects leave before the cut); piecewise-exponential event times (baseline rate 1/365 per
    day), censoring Exp(1/500), whole days; one stratum.  beta_true[0] = 0 (the treatment
    effect is log_hr)."""
    rng = np.random.default_rng(seed)
    cols = [np.flatnonzero(rng.random(n) < 0.5).astype(np.int32)]
    for _ in range(1, p):
        gaps = rng.geometric(density, size=int(n * density * 1.2) + 64)
        pos = np.cumsum(gaps) - 1
        while pos[-1] < n - 1:
            more = np.cumsum(rng.geometric(density, size=int(n * density * 0.2) + 64)) + pos[-1]
            pos = np.concatenate([pos, more])
        cols.append(pos[pos < n].astype(np.int32))
    col_ptr = np.zeros(p + 1, dtype=np.int64)
    col_ptr[1:] = np.cumsum([c.size for c in cols])
    row_idx = np.concatenate(cols)
    b = rng.normal(0.0, 0.1, size=p) * (rng.random(p) < 0.2)
    b[0] = 0.0
    eta = np.zeros(n)
    for j in np.flatnonzero(b):
        eta[cols[j]] += b[j]
    treat = np.zeros(n)
    treat[cols[0]] = 1.0
    base = 1.0 / 365.0
    a_rate = base * np.exp(eta + treat * log_hr[0])
    b_rate = base * np.exp(eta + treat * log_hr[1])
    E = rng.exponential(1.0, size=n)
    T = np.where(E < a_rate * cut, E / a_rate, cut + (E - a_rate * cut) / b_rate)
    C = rng.exponential(1.0, size=n) * 500.0
    event = (T <= C).astype(np.uint8)
    Y = np.maximum(np.ceil(np.minimum(T, C)), 1.0)
    return SparseCoxData(n=n, col_ptr=col_ptr, row_idx=row_idx, time=Y, event=event,
                         stratum=np.zeros(n, dtype=np.int32), beta_true=b, gamma=math.sqrt(2.0),
                         name=f"cough-sparse-n{n}-p{p}")
