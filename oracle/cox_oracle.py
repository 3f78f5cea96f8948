"""FP64 CPU oracle for the stratified Cox model (arXiv 2310.16238).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP path (``paper_2310_16238_amd``) and never imports it.

Three levels, each citing the passage it follows:

* **Definitions, brute force** (``*_brute``): the negative log partial
  likelihood of Eq. strat_l, its gradient (Eq. strat_g), the diagonal of its
  Hessian (Eq. strat_h) and the full Hessian (the same sums with x x' in place
  of x_j^2), each as an explicit loop over events and their risk sets
  R_k(Y_ki) = {r in stratum k : Y_kr >= Y_ki}.  O(E N P); small inputs only.
* **Scan form** (plain C in ``cox_oracle.c``): rows sorted by stratum and
  decreasing time (Sec. 2.7), the segmented scan of Sec. 2.6, and the
  per-coordinate reductions of Eqs. parallel_g / parallel_h; cyclic coordinate
  descent with trust region and l1 (Sec. 2.4).
* **Full information and Newton**: the Hessian in the form
  X' diag(w Lambda) X - sum_g d_g xbar_g xbar_g' (exchanging the order of the
  sums in Eq. strat_h), evaluated with a matrix product, and a Newton/Cholesky
  fit for the unpenalised optimum.

Readings of points the paper leaves open (ties, ordering, degenerate columns,
convergence) are the ones listed in the project's design notes; the important
ones are restated where they are used.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cox_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liborc.so")
_lib = None


def build_c(force: bool = False) -> str:
    """Compile the plain-C part of the oracle with gcc (single-threaded, -O2)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-fno-fast-math",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def load_library(path: str):
    """Load a compiled copy of cox_oracle.c and declare its signatures."""
    lib = ctypes.CDLL(path)
    i64, dp, u8p, i64p = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), \
        ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int64)
    lib.orc_segscan.argtypes = [i64, dp, u8p, dp]
    lib.orc_segscan.restype = None
    lib.orc_coord_terms.argtypes = [i64, dp, dp, u8p, u8p, i64p, dp]
    lib.orc_coord_terms.restype = None
    lib.orc_ccd_step.argtypes = [ctypes.c_double] * 5 + [dp]
    lib.orc_ccd_step.restype = ctypes.c_double
    lib.orc_ccd_fit.argtypes = [i64, i64, dp, i64, u8p, u8p, i64p, dp, ctypes.c_double,
                                ctypes.c_int, dp, dp, dp]
    lib.orc_ccd_fit.restype = ctypes.c_int
    lib.orc_group_sums.argtypes = [i64, i64, dp, i64, dp, u8p, u8p, i64p,
                                   dp, dp, dp, dp, dp, dp]
    lib.orc_group_sums.restype = i64
    lib.orc_coord_terms_efron.argtypes = [i64, dp, dp, u8p, u8p, i64p, dp]
    lib.orc_coord_terms_efron.restype = None
    lib.orc_ccd_fit_ties.argtypes = [i64, i64, dp, i64, u8p, u8p, i64p, dp, ctypes.c_double,
                                     ctypes.c_int, dp, dp, dp, ctypes.c_int]
    lib.orc_ccd_fit_ties.restype = ctypes.c_int
    lib.orc_group_sums_efron.argtypes = [i64, i64, dp, i64, dp, u8p, u8p, i64p,
                                         dp, dp, dp, dp, dp, dp, dp, dp, dp]
    lib.orc_group_sums_efron.restype = i64
    return lib


def _c():
    global _lib
    if _lib is None:
        _lib = load_library(build_c())
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


# ============================================================== canonical layout (Sec. 2.7)

@dataclasses.dataclass
class Layout:
    """Rows in canonical order: stratum ascending, time descending, original index ascending.

    perm[i]   original index of canonical row i
    head[i]   1 iff canonical row i is the first row of its stratum (head flag f, Sec. 2.7)
    event[i]  delta of canonical row i
    gend[i]   canonical index of the last row of row i's tie group (same stratum, same time)
    dcount[i] number of events in the tie group if row i ends its group, else 0
    meta[i]   packed word: bit 31 head, bit 30 event, bits 0..29 dcount
    """
    perm: np.ndarray
    head: np.ndarray
    event: np.ndarray
    gend: np.ndarray
    dcount: np.ndarray
    meta: np.ndarray
    n_strata: int


def canonical_layout(time, event, stratum=None) -> Layout:
    time = np.asarray(time, dtype=np.float64)
    event = np.asarray(event).astype(np.uint8)
    n = time.shape[0]
    if stratum is None:
        stratum = np.zeros(n, dtype=np.int64)
    stratum = np.asarray(stratum).astype(np.int64)
    # np.lexsort sorts by the last key first: stratum, then -time, then index.
    perm = np.lexsort((np.arange(n), -time, stratum)).astype(np.int64)
    s = stratum[perm]
    t = time[perm]
    ev = event[perm]
    head = np.ones(n, dtype=np.uint8)
    head[1:] = (s[1:] != s[:-1]).astype(np.uint8)
    # a tie group continues while the stratum and the time are unchanged
    new_group = np.ones(n, dtype=bool)
    new_group[1:] = (s[1:] != s[:-1]) | (t[1:] != t[:-1])
    starts = np.flatnonzero(new_group)
    ends = np.append(starts[1:] - 1, n - 1)
    gid = np.cumsum(new_group) - 1
    gend = ends[gid].astype(np.int64)
    dsum = np.add.reduceat(ev.astype(np.int64), starts)
    dcount = np.zeros(n, dtype=np.int64)
    dcount[ends] = dsum
    meta = (head.astype(np.uint32) << np.uint32(31)) | (ev.astype(np.uint32) << np.uint32(30)) \
        | dcount.astype(np.uint32)
    return Layout(perm=perm, head=head, event=ev.astype(np.uint8), gend=gend, dcount=dcount,
                  meta=meta.astype(np.uint32), n_strata=int(head.sum()))


def to_canonical(X, layout: Layout) -> np.ndarray:
    """Rows of X (n, p) permuted to canonical order, column-major."""
    return np.asfortranarray(np.asarray(X, dtype=np.float64)[layout.perm, :])


# ============================================================== scan (Sec. 2.6)

def seg_op(x, y):
    """(f_i, a_i) (+)s (f_j, a_j) = (f_i | f_j, a_j if f_j else a_i + a_j)."""
    return (x[0] | y[0], y[1] if y[0] else x[1] + y[1])


def segmented_scan(a, flags):
    """Inclusive segmented scan by folding seg_op left to right (pure Python)."""
    out = []
    acc = None
    for ai, fi in zip(a, flags):
        cur = (int(fi), ai)
        acc = cur if acc is None else seg_op(acc, cur)
        out.append(acc[1])
    return out


def segmented_scan_c(a, flags) -> np.ndarray:
    """The same scan in the C oracle (FP64)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    f = np.ascontiguousarray(flags, dtype=np.uint8)
    b = np.empty_like(a)
    _c().orc_segscan(a.shape[0], _p(a, ctypes.c_double), _p(f, ctypes.c_uint8), _p(b, ctypes.c_double))
    return b


# ============================================================== definitions (brute force)

def _risk_sets(time, stratum):
    """For each row i, the boolean mask of R(Y_i) = {r : same stratum, Y_r >= Y_i}."""
    time = np.asarray(time, dtype=np.float64)
    n = time.shape[0]
    stratum = np.zeros(n, dtype=np.int64) if stratum is None else np.asarray(stratum)
    for i in range(n):
        yield i, (stratum == stratum[i]) & (time >= time[i])


def neg_loglik_brute(X, time, event, stratum, beta) -> float:
    """-log of Eq. strat_l: -sum_i delta_i [x_i'b - log sum_{r in R(Y_i)} exp(x_r'b)]."""
    X = np.asarray(X, dtype=np.float64)
    eta = X @ np.asarray(beta, dtype=np.float64)
    total = 0.0
    for i, R in _risk_sets(time, stratum):
        if event[i]:
            total -= eta[i] - np.log(np.sum(np.exp(eta[R])))
    return float(total)


def grad_brute(X, time, event, stratum, beta) -> np.ndarray:
    """Eq. strat_g for every j: -sum_i delta_i x_ij + sum_i delta_i (sum_R x_rj w_r)/(sum_R w_r)."""
    X = np.asarray(X, dtype=np.float64)
    eta = X @ np.asarray(beta, dtype=np.float64)
    g = np.zeros(X.shape[1])
    for i, R in _risk_sets(time, stratum):
        if event[i]:
            w = np.exp(eta[R])
            g += -X[i] + (w @ X[R]) / w.sum()
    return g


def hess_diag_brute(X, time, event, stratum, beta) -> np.ndarray:
    """Eq. strat_h for every j: sum_i delta_i [(sum_R x_rj^2 w)/(sum_R w) - ((sum_R x_rj w)/(sum_R w))^2]."""
    X = np.asarray(X, dtype=np.float64)
    eta = X @ np.asarray(beta, dtype=np.float64)
    h = np.zeros(X.shape[1])
    for i, R in _risk_sets(time, stratum):
        if event[i]:
            w = np.exp(eta[R])
            m1 = (w @ X[R]) / w.sum()
            m2 = (w @ (X[R] ** 2)) / w.sum()
            h += m2 - m1 * m1
    return h


def info_brute(X, time, event, stratum, beta) -> np.ndarray:
    """Full Hessian of -log L: sum_i delta_i [ (sum_R w x x')/(sum_R w) - xbar xbar' ]."""
    X = np.asarray(X, dtype=np.float64)
    eta = X @ np.asarray(beta, dtype=np.float64)
    p = X.shape[1]
    H = np.zeros((p, p))
    for i, R in _risk_sets(time, stratum):
        if event[i]:
            w = np.exp(eta[R])
            XR = X[R]
            xbar = (w @ XR) / w.sum()
            H += (XR.T * w) @ XR / w.sum() - np.outer(xbar, xbar)
    return H


# ------------------------------------------------ Efron's approximation for ties (brute force)
#
# Efron (JASA 72, 1977): a tie group g of stratum k at time t with d events D_g and risk
# set R_g = {r in stratum k : Y_r >= t} contributes
#     -sum_{i in D_g} eta_i + sum_{l=0}^{d-1} log( sum_{R_g} w_r - (l/d) sum_{D_g} w_i )
# to -log L (w = exp(eta)).  The paper's risk sets (Eq. strat_l) give Breslow's form,
# where every tied event sees all of R_g; Efron's removes an increasing share of the tied
# events' weight.  With one event per group both are the same.

def _event_groups(time, event, stratum):
    """For each (stratum, time) that holds an event: masks of R_g and D_g."""
    time = np.asarray(time, dtype=np.float64)
    event = np.asarray(event)
    n = time.shape[0]
    stratum = np.zeros(n, dtype=np.int64) if stratum is None else np.asarray(stratum)
    keys = sorted({(int(stratum[i]), float(time[i])) for i in range(n) if event[i]})
    for s_, t_ in keys:
        same = stratum == s_
        yield same & (time >= t_), same & (time == t_) & (event != 0)


def neg_loglik_efron_brute(X, time, event, stratum, beta) -> float:
    """-log L with Efron's tie correction, by explicit loops over tie groups and their events."""
    X = np.asarray(X, dtype=np.float64)
    eta = X @ np.asarray(beta, dtype=np.float64)
    w = np.exp(eta)
    total = 0.0
    for R, D in _event_groups(time, event, stratum):
        d = int(D.sum())
        S0, E0 = w[R].sum(), w[D].sum()
        total -= eta[D].sum()
        for l in range(d):
            total += np.log(S0 - (l / d) * E0)
    return float(total)


def grad_efron_brute(X, time, event, stratum, beta) -> np.ndarray:
    """Gradient of neg_loglik_efron_brute: -sum_D x + sum_l (S1 - a_l E1) / (S0 - a_l E0)."""
    X = np.asarray(X, dtype=np.float64)
    w = np.exp(X @ np.asarray(beta, dtype=np.float64))
    g = np.zeros(X.shape[1])
    for R, D in _event_groups(time, event, stratum):
        d = int(D.sum())
        S0, S1 = w[R].sum(), w[R] @ X[R]
        E0, E1 = w[D].sum(), w[D] @ X[D]
        g -= X[D].sum(axis=0)
        for l in range(d):
            a = l / d
            g += (S1 - a * E1) / (S0 - a * E0)
    return g


def info_efron_brute(X, time, event, stratum, beta) -> np.ndarray:
    """Hessian of neg_loglik_efron_brute: sum_l [(S2 - a_l E2)/A_l - m_l m_l'], m_l = (S1 - a_l E1)/A_l."""
    X = np.asarray(X, dtype=np.float64)
    w = np.exp(X @ np.asarray(beta, dtype=np.float64))
    H = np.zeros((X.shape[1], X.shape[1]))
    for R, D in _event_groups(time, event, stratum):
        d = int(D.sum())
        S0, S1, S2 = w[R].sum(), w[R] @ X[R], (X[R].T * w[R]) @ X[R]
        E0, E1, E2 = w[D].sum(), w[D] @ X[D], (X[D].T * w[D]) @ X[D]
        for l in range(d):
            a = l / d
            A = S0 - a * E0
            m = (S1 - a * E1) / A
            H += (S2 - a * E2) / A - np.outer(m, m)
    return H


# ============================================================== scan form (C)

def _ties_flag(ties: str) -> int:
    if ties not in ("breslow", "efron"):
        raise ValueError("ties must be 'breslow' or 'efron'")
    return int(ties == "efron")


def coord_terms(Xc, layout: Layout, j: int, eta, ties: str = "breslow") -> dict:
    """g'(beta_j), g''(beta_j), objective and second-moment term for column j.

    Xc is the design in canonical order (see to_canonical); eta = Xc @ beta.
    Follows Eqs. parallel_g / parallel_h with the segmented scans of Sec. 2.6;
    ties="efron" takes Efron's tie correction (orc_coord_terms_efron).
    """
    xj = np.ascontiguousarray(Xc[:, j], dtype=np.float64)
    eta = np.ascontiguousarray(eta, dtype=np.float64)
    out = np.zeros(4)
    fn = _c().orc_coord_terms_efron if _ties_flag(ties) else _c().orc_coord_terms
    fn(xj.shape[0], _p(xj, ctypes.c_double), _p(eta, ctypes.c_double),
       _p(layout.head, ctypes.c_uint8), _p(layout.event, ctypes.c_uint8),
       _p(layout.gend, ctypes.c_int64), _p(out, ctypes.c_double))
    return {"grad": out[0], "hess": out[1], "obj": out[2], "m2": out[3]}


def ccd_step(beta_j, g1, g2, m2, gamma, trust):
    """One CCD coordinate step (Sec. 2.4); returns (step, new trust half-width)."""
    t = ctypes.c_double(trust)
    s = _c().orc_ccd_step(beta_j, g1, g2, m2, gamma, ctypes.byref(t))
    return s, t.value


@dataclasses.dataclass
class FitResult:
    beta: np.ndarray
    converged: bool
    iters: int
    objective: float
    last_step: float
    grad: np.ndarray


def _gamma_vec(p, gamma, penalize):
    g = np.full(p, float(gamma))
    if penalize is not None:
        g = np.where(np.asarray(penalize, dtype=bool), g, 0.0)
    return np.ascontiguousarray(g)


def fit_ccd(X, time, event, stratum=None, *, gamma=0.0, penalize=None, beta0=None,
            tol=1e-12, max_sweeps=1000, layout: Layout | None = None, Xc=None,
            ties: str = "breslow") -> FitResult:
    """Cyclic coordinate descent of Sec. 2.4 on -log L + sum_j gamma_j |beta_j| (C oracle);
    ties="efron" descends Efron's -log L instead."""
    efron = _ties_flag(ties)
    layout = layout or canonical_layout(time, event, stratum)
    Xc = to_canonical(X, layout) if Xc is None else Xc
    n, p = Xc.shape
    beta = np.zeros(p) if beta0 is None else np.array(beta0, dtype=np.float64)
    grad = np.zeros(p)
    info = np.zeros(3)
    gam = _gamma_vec(p, gamma, penalize)
    rc = _c().orc_ccd_fit_ties(n, p, _p(Xc, ctypes.c_double), n, _p(layout.head, ctypes.c_uint8),
                               _p(layout.event, ctypes.c_uint8), _p(layout.gend, ctypes.c_int64),
                               _p(gam, ctypes.c_double), float(tol), int(max_sweeps),
                               _p(beta, ctypes.c_double), _p(grad, ctypes.c_double),
                               _p(info, ctypes.c_double), efron)
    return FitResult(beta=beta, converged=(rc == 0), iters=int(info[0]), objective=float(info[2]),
                     last_step=float(info[1]), grad=grad)


@dataclasses.dataclass
class FullEval:
    objective: float
    grad: np.ndarray
    hess_diag: np.ndarray
    info: np.ndarray | None
    info_first: np.ndarray | None = None    # X' diag(w Lambda) X
    info_second: np.ndarray | None = None   # sum_g d_g xbar_g xbar_g'


def full_eval_efron(Xc, layout: Layout, beta, want_info: bool = True) -> FullEval:
    """full_eval with Efron's tie correction (see orc_coord_terms_efron).

    objective = -delta' eta + sum_g sum_l log A_{g,l},  A_{g,l} = S0_g - a_l E0_g, a_l = l/d_g
    gradient  = -X' delta + sum_g sum_l (S1_g - a_l E1_g) / A_{g,l}
    diag      = sum_g sum_l [(S2_g - a_l E2_g) / A_{g,l} - ((S1_g - a_l E1_g) / A_{g,l})^2]
    Hessian   = X' diag(w c) X - Z'Z, the rows of Z being m_{g,l} = (S1_g - a_l E1_g) / A_{g,l}
    for every group g and l < d_g (one row per event), w c from orc_group_sums_efron.
    """
    Xc = np.asfortranarray(Xc, dtype=np.float64)
    n, p = Xc.shape
    beta = np.asarray(beta, dtype=np.float64)
    eta = np.ascontiguousarray(Xc @ beta)
    G = int(np.count_nonzero(layout.dcount))
    S0 = np.zeros(G); S1 = np.zeros((G, p)); S2 = np.zeros((G, p))
    E0 = np.zeros(G); E1 = np.zeros((G, p)); E2 = np.zeros((G, p))
    d = np.zeros(G); m = np.zeros(G); wl = np.zeros(n)
    dp = ctypes.c_double
    g_out = _c().orc_group_sums_efron(n, p, _p(Xc, dp), n, _p(eta, dp), _p(layout.head, ctypes.c_uint8),
                                      _p(layout.event, ctypes.c_uint8), _p(layout.gend, ctypes.c_int64),
                                      _p(S0, dp), _p(S1, dp), _p(S2, dp), _p(E0, dp), _p(E1, dp), _p(E2, dp),
                                      _p(d, dp), _p(m, dp), _p(wl, dp))
    assert g_out == G
    ev = layout.event.astype(np.float64)
    dn = d.astype(np.int64)
    # one row per event: group index and a_l = l / d_g
    gi = np.repeat(np.arange(G), dn)
    a = np.concatenate([np.arange(k) / k for k in dn]) if G else np.zeros(0)
    A = S0[gi] - a * E0[gi]
    M1 = (S1[gi] - a[:, None] * E1[gi]) / A[:, None]
    M2 = (S2[gi] - a[:, None] * E2[gi]) / A[:, None]
    obj = float(-(ev @ eta) + np.sum(np.log(A) + m[gi]))
    grad = -(Xc.T @ ev) + M1.sum(axis=0)
    hdiag = (M2 - M1 * M1).sum(axis=0)
    info = first = second = None
    if want_info:
        first = (Xc.T * wl) @ Xc
        second = M1.T @ M1
        info = first - second
    return FullEval(objective=obj, grad=grad, hess_diag=hdiag, info=info, info_first=first, info_second=second)


def full_eval(Xc, layout: Layout, beta, want_info: bool = True, ties: str = "breslow") -> FullEval:
    """Objective, full gradient, diag Hessian and (optionally) the full Hessian at beta.

    gradient  = -X' delta + sum_g d_g S1_g / S0_g                     (Eq. strat_g, all j)
    diag      = sum_g d_g (S2_g / S0_g - (S1_g / S0_g)^2)              (Eq. strat_h)
    Hessian   = X' diag(w Lambda) X - sum_g d_g xbar_g xbar_g'         (Eq. strat_h, x x')
    where g runs over tie groups with d_g events, S*_g are risk-set sums at the
    group end, xbar_g = S1_g / S0_g and Lambda_r = sum_{g: Y_g <= Y_r} d_g / S0_g
    (same stratum): sum_g d_g S2_g / S0_g = sum_r w_r Lambda_r x_r x_r'.
    ties="efron" gives full_eval_efron.
    """
    if _ties_flag(ties):
        return full_eval_efron(Xc, layout, beta, want_info)
    Xc = np.asfortranarray(Xc, dtype=np.float64)
    n, p = Xc.shape
    beta = np.asarray(beta, dtype=np.float64)
    eta = np.ascontiguousarray(Xc @ beta)
    G = int(np.count_nonzero(layout.dcount))
    S0 = np.zeros(G); S1 = np.zeros((G, p)); S2 = np.zeros((G, p))
    d = np.zeros(G); m = np.zeros(G); wl = np.zeros(n)
    g_out = _c().orc_group_sums(n, p, _p(Xc, ctypes.c_double), n, _p(eta, ctypes.c_double),
                                _p(layout.head, ctypes.c_uint8), _p(layout.event, ctypes.c_uint8),
                                _p(layout.gend, ctypes.c_int64), _p(S0, ctypes.c_double),
                                _p(S1, ctypes.c_double), _p(S2, ctypes.c_double),
                                _p(d, ctypes.c_double), _p(m, ctypes.c_double), _p(wl, ctypes.c_double))
    assert g_out == G
    ev = layout.event.astype(np.float64)
    xbar = S1 / S0[:, None]
    obj = float(-(ev @ eta) + d @ (np.log(S0) + m))
    grad = -(Xc.T @ ev) + d @ xbar
    hdiag = d @ (S2 / S0[:, None] - xbar * xbar)
    info = first = second = None
    if want_info:
        first = (Xc.T * wl) @ Xc
        second = (xbar.T * d) @ xbar
        info = first - second
    return FullEval(objective=obj, grad=grad, hess_diag=hdiag, info=info, info_first=first, info_second=second)


def degenerate_columns(Xc, layout: Layout, beta=None, ties: str = "breslow") -> np.ndarray:
    """Columns with numerically zero curvature (g'' <= 1e-12 * second-moment term)."""
    Xc = np.asfortranarray(Xc, dtype=np.float64)
    n, p = Xc.shape
    beta = np.zeros(p) if beta is None else np.asarray(beta, dtype=np.float64)
    eta = Xc @ beta
    out = np.zeros(p, dtype=bool)
    for j in range(p):
        t = coord_terms(Xc, layout, j, eta, ties)
        out[j] = not (t["hess"] > 1e-12 * abs(t["m2"]))
    return out


def fit_newton(X, time, event, stratum=None, *, beta0=None, tol=1e-14, max_iter=100,
               layout: Layout | None = None, Xc=None, ties: str = "breslow") -> FitResult:
    """Unpenalised optimum by Newton's method on the full Hessian (numpy Cholesky).

    Degenerate columns (a ones column, which cancels from every ratio in
    Eq. strat_l) are held at zero.  Step halving guards the first iterations.
    Stops when max|step| <= tol * max(1, max|beta|).  ties="efron": Efron's -log L.
    """
    layout = layout or canonical_layout(time, event, stratum)
    Xc = to_canonical(X, layout) if Xc is None else Xc
    n, p = Xc.shape
    beta = np.zeros(p) if beta0 is None else np.array(beta0, dtype=np.float64)
    free = ~degenerate_columns(Xc, layout, ties=ties)
    beta[~free] = 0.0
    ev = full_eval(Xc, layout, beta, ties=ties)
    it = 0
    step_max = np.inf
    converged = False
    while it < max_iter:
        it += 1
        H = ev.info[np.ix_(free, free)]
        L = np.linalg.cholesky(H)
        step = np.zeros(p)
        step[free] = -np.linalg.solve(L.T, np.linalg.solve(L, ev.grad[free]))
        t = 1.0
        while True:
            cand = full_eval(Xc, layout, beta + t * step, ties=ties)
            if cand.objective <= ev.objective + 1e-12 * abs(ev.objective) or t < 1e-6:
                break
            t *= 0.5
        beta = beta + t * step
        ev = cand
        step_max = float(np.max(np.abs(t * step))) if p else 0.0
        if step_max <= tol * max(1.0, float(np.max(np.abs(beta)))):
            converged = True
            break
    return FitResult(beta=beta, converged=converged, iters=it, objective=ev.objective,
                     last_step=step_max, grad=ev.grad)


# ============================================================== time intervals (Secs. 2.2-2.3)

def augmented_columns(tv_coef, K: int):
    """Columns of X^(aug) (Sec. 2.3): (source column, interval) pairs, interval -1 for a
    column with a time-fixed coefficient; a step-coefficient column j gives (j, 0..K-1)."""
    cols = []
    for j, t in enumerate(np.asarray(tv_coef).astype(bool)):
        cols += [(j, k) for k in range(K)] if t else [(j, -1)]
    return cols


def split_intervals(X, time, event, stratum=None, cuts=(), tv_coef=None, X_by_interval=None,
                    keep_all_rows: bool = False) -> dict:
    """The augmented data set of Secs. 2.2-2.3, built from their definitions.

    Intervals I_k = [t_{k-1}, t_k), k = 0..K-1 with K = len(cuts) + 1, t_{-1} = -inf and
    the last interval unbounded above (it holds max Y).  For interval k and subject i:
    Y_ki = min(Y_i, t_k), delta_ki = delta_i [Y_i in I_k], stratum (rank of s_i) * K + k,
    covariates x_ki (X_by_interval[k][i] if given, else x_i), with every column j that has
    a step-function coefficient (Sec. 2.3) replaced by K columns, the k-th equal to x_kij on
    interval k's rows and zero elsewhere.  Rows are interval-major, subjects in their
    original order within an interval.

    The paper's augmented matrix has all K N rows.  A row with Y_i < t_{k-1} carries no
    event and its time is below every event time of its stratum, so it is in no risk set:
    it contributes nothing to Eq. time_cov_strat_l, and the result drops it unless
    keep_all_rows.
    """
    X = np.asarray(X, dtype=np.float64)
    n, p = X.shape
    Y = np.asarray(time, dtype=np.float64)
    d = np.asarray(event).astype(np.uint8)
    cuts = np.asarray(cuts, dtype=np.float64)
    K = cuts.shape[0] + 1
    bounds = np.concatenate([[-np.inf], cuts, [np.inf]])
    if stratum is None:
        srank = np.zeros(n, dtype=np.int64)
    else:
        _, srank = np.unique(np.asarray(stratum), return_inverse=True)
    cols = augmented_columns(np.zeros(p) if tv_coef is None else tv_coef, K)

    parts = []
    for k in range(K):
        lo, hi = bounds[k], bounds[k + 1]
        xk = X if X_by_interval is None else np.asarray(X_by_interval[k], dtype=np.float64)
        rows = np.arange(n) if keep_all_rows else np.flatnonzero(Y >= lo)
        in_k = (Y[rows] >= lo) & (Y[rows] < hi)
        Xa = np.zeros((rows.shape[0], len(cols)))
        for c, (j, kc) in enumerate(cols):
            if kc < 0 or kc == k:
                Xa[:, c] = xk[rows, j]
        parts.append(dict(X=Xa, time=np.minimum(Y[rows], hi), event=np.where(in_k, d[rows], 0),
                          stratum=srank[rows] * K + k, row_subject=rows, row_interval=np.full(rows.shape[0], k)))
    cat = {key: np.concatenate([q[key] for q in parts]) for key in parts[0]}
    return {
        "X": np.asfortranarray(cat["X"]),
        "time": cat["time"].astype(np.float64),
        "event": cat["event"].astype(np.uint8),
        "stratum": cat["stratum"].astype(np.int32),
        "row_subject": cat["row_subject"].astype(np.int64),
        "row_interval": cat["row_interval"].astype(np.int32),
        "col_source": np.asarray([c[0] for c in cols], dtype=np.int32),
        "col_interval": np.asarray([c[1] for c in cols], dtype=np.int32),
        "intervals": K,
    }


def neg_loglik_time_varying_brute(X_by_interval, time, event, stratum, cuts, beta_of_interval) -> float:
    """-log of Eq. time_cov_l with piecewise-constant covariates and coefficients, by definition.

    For an event at Y_i in interval I_k, every r in R(Y_i) (same stratum, Y_r >= Y_i)
    contributes exp(x_r(Y_i)' beta(Y_i)) with x_r(Y_i) = X_by_interval[k][r] and
    beta(Y_i) = beta_of_interval[k]: the covariate path of Sec. 2.2 and the step
    coefficients of Sec. 2.3 (Eq. time_coef_l) read at the event time.
    """
    Y = np.asarray(time, dtype=np.float64)
    cuts = np.asarray(cuts, dtype=np.float64)
    n = Y.shape[0]
    st = np.zeros(n, dtype=np.int64) if stratum is None else np.asarray(stratum)
    total = 0.0
    for i in range(n):
        if not event[i]:
            continue
        k = int(np.searchsorted(cuts, Y[i], side="right"))   # number of cuts <= Y_i
        xk = np.asarray(X_by_interval[k], dtype=np.float64)
        b = np.asarray(beta_of_interval[k], dtype=np.float64)
        R = (st == st[i]) & (Y >= Y[i])
        total -= xk[i] @ b - np.log(np.sum(np.exp(xk[R] @ b)))
    return float(total)


# ============================================================== resampling, CV, bootstrap (Secs. 2.1, 3.2)

def resample(X, time, event, stratum, count):
    """The data set in which row i appears count[i] times (copies kept together, rows in
    their original order): the training rows of a cross-validation fold (counts 0/1) or a
    bootstrap sample (multinomial counts)."""
    idx = np.repeat(np.arange(np.asarray(time).shape[0]), np.asarray(count, dtype=np.int64))
    X = np.asarray(X, dtype=np.float64)
    return (np.asfortranarray(X[idx]), np.asarray(time, dtype=np.float64)[idx], np.asarray(event)[idx],
            None if stratum is None else np.asarray(stratum)[idx])


def neg_loglik(X, time, event, stratum, beta) -> float:
    """-log of Eq. strat_l (no penalty) through the scan form."""
    lay = canonical_layout(time, event, stratum)
    return full_eval(to_canonical(X, lay), lay, beta, want_info=False).objective


def cross_validate(X, time, event, stratum, fold, gammas, penalize=None, tol=1e-13, max_sweeps=1000):
    """Cross-validated log partial likelihood of the l1 weight (Sec. 2.1 chooses gamma by
    cross-validation; the criterion is not stated -- this is the one of Verweij and van
    Houwelingen): for fold k, beta_{-k}(gamma) is the CCD fit on the rows outside fold k,
    and cvl(gamma) = sum_k [ l(beta_{-k}) - l_{-k}(beta_{-k}) ], l the log partial
    likelihood on all rows and l_{-k} on the training rows.  Each fold's path starts at 0
    and is warm-started from the previous gamma.
    Returns (cvl[ngamma], betas[nfolds, ngamma, p], converged[nfolds, ngamma])."""
    fold = np.asarray(fold)
    K = int(fold.max()) + 1
    G = len(gammas)
    p = np.asarray(X).shape[1]
    cvl = np.zeros(G)
    betas = np.zeros((K, G, p))
    conv = np.zeros((K, G), dtype=bool)
    for k in range(K):
        Xt, tt, et, st = resample(X, time, event, stratum, (fold != k).astype(np.int64))
        lay = canonical_layout(tt, et, st)
        Xc = to_canonical(Xt, lay)
        beta = np.zeros(p)
        for g, gam in enumerate(gammas):
            r = fit_ccd(Xt, tt, et, st, gamma=gam, penalize=penalize, beta0=beta, tol=tol,
                        max_sweeps=max_sweeps, layout=lay, Xc=Xc)
            beta = r.beta
            betas[k, g] = beta
            conv[k, g] = r.converged
            l_all = -neg_loglik(X, time, event, stratum, beta)
            l_train = -full_eval(Xc, lay, beta, want_info=False).objective
            cvl[g] += l_all - l_train
    return cvl, betas, conv


def bootstrap(X, time, event, stratum, counts, gamma=0.0, penalize=None, beta0=None, tol=1e-13, max_sweeps=1000):
    """Refits on bootstrap samples (Sec. 3.2): replicate b uses the rows with multiplicities
    counts[b].  Returns (betas[B, p], converged[B])."""
    counts = np.asarray(counts)
    p = np.asarray(X).shape[1]
    betas = np.zeros((counts.shape[0], p))
    conv = np.zeros(counts.shape[0], dtype=bool)
    for b in range(counts.shape[0]):
        Xb, tb, eb, sb = resample(X, time, event, stratum, counts[b])
        r = fit_ccd(Xb, tb, eb, sb, gamma=gamma, penalize=penalize, beta0=beta0, tol=tol, max_sweeps=max_sweeps)
        betas[b] = r.beta
        conv[b] = r.converged
    return betas, conv


def percentile_interval(values, level=0.95):
    """Percentile interval of bootstrap values (Sec. 3.2): the (1-level)/2 and (1+level)/2
    empirical quantiles, numpy's default (linear) interpolation."""
    v = np.asarray(values, dtype=np.float64)
    return np.quantile(v, (1.0 - level) / 2.0, axis=0), np.quantile(v, (1.0 + level) / 2.0, axis=0)


# ============================================================== Breslow baseline hazard

def baseline_hazard_brute(X, time, event, stratum, beta) -> np.ndarray:
    """Breslow cumulative baseline hazard at each row's own time, by definition: for row i in
    stratum k, the sum over the distinct event times t <= Y_i of stratum k of
    d(t) / sum_{r in k, Y_r >= t} exp(x_r'beta), d(t) the events at t (the denominators are
    the risk-set sums of Eq. strat_l)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(time, dtype=np.float64)
    ev = np.asarray(event).astype(bool)
    n = Y.shape[0]
    st = np.zeros(n, dtype=np.int64) if stratum is None else np.asarray(stratum)
    w = np.exp(X @ np.asarray(beta, dtype=np.float64))
    out = np.zeros(n)
    for i in range(n):
        same = st == st[i]
        for t in np.unique(Y[same & ev & (Y <= Y[i])]):
            d = np.count_nonzero(same & ev & (Y == t))
            out[i] += d / w[same & (Y >= t)].sum()
    return out
