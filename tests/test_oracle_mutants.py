"""Planted mistakes in a copy of the C oracle must each break at least one pin.

Each mutant edits one line of oracle/cox_oracle.c the way a plausible slip
would (a dropped term, a wrong sign or index, a lost reset), is compiled to a
temporary library and swapped in; the pins below must then fail.  This checks
that the pins constrain the oracle, not that the oracle is right (the pins in
test_oracle_pins.py do that).
"""
import os
import subprocess

import numpy as np
import pytest

from conftest import read_golden
from oracle import cox_oracle as o
from paper_2310_16238_amd import synth

SRC = os.path.join(os.path.dirname(o.__file__), "cox_oracle.c")

MUTANTS = {
    "scan_no_reset": ("r.a = y.f ? y.a : x.a + y.a;", "r.a = x.a + y.a;"),
    "state_no_reset": ("if (b.f) { r.m = b.m;", "if (0) { r.m = b.m;"),
    "ties_ignored": ("const orc_state *g = &S[gend[i]];", "const orc_state *g = &S[i];"),
    "grad_sign": ("out[0] = -dx + g1;", "out[0] = dx + g1;"),
    "hess_no_square": ("out[1] = h1 - h2;", "out[1] = h1;"),
    "obj_no_shift": ("ll += log(g->s0) + g->m;", "ll += log(g->s0);"),
    "rescale_wrong": ("double ea = exp(a.m - M), eb = exp(b.m - M);",
                      "double ea = exp(a.m - M), eb = exp(M - b.m);"),
    "s2_not_squared": ("s2[j] += w * x * x;", "s2[j] += w * x;"),
    "lambda_leaks_strata": ("if (head[s]) la = -INFINITY;", ";"),
    "trust_never_grows": ("*trust = t2 > half ? t2 : half;", "*trust = half;"),
    "l1_wrong_side": ("} else if (g1 + gamma < 0.0) {", "} else if (g1 - gamma < 0.0) {"),
    "newton_sign": ("step = -g1 / g2;", "step = g1 / g2;"),
    # Efron's tie correction
    "efron_denominator_uncorrected": ("double A = g->s0 - a * e0;", "double A = g->s0;"),
    "efron_numerator_uncorrected": ("double r1 = (g->s1 - a * e1) / A;", "double r1 = g->s1 / A;"),
    "efron_objective_uncorrected": ("lsum += log(A) + g->m;", "lsum += log(g->s0) + g->m;"),
    "efron_share_over_all_rows": ("            if (!event[r]) continue;\n            double w = exp(eta[r] - g->m);",
                                  "            double w = exp(eta[r] - g->m);"),
    "efron_k_wrong": ("k += a / A;", "k += 1.0 / A;"),
    "efron_no_event_term_in_weights": ("if (event[q] && lk[e] != -INFINITY) v -= exp(eta[q] + lk[e]);", ";"),
}


def _pins():
    """Run a compact set of the pins; return the names of those that fail."""
    fails = []

    def check(name, fn):
        try:
            with np.errstate(all="ignore"):
                ok = fn()
        except Exception:
            ok = False
        if not ok:
            fails.append(name)

    g = read_golden("segscan_example.txt")
    check("paper_scan", lambda: list(o.segmented_scan_c(np.array(g["a"]), np.array(g["f"], dtype=np.uint8)))
          == g["b"])
    t = read_golden("toy_closed_forms.txt")
    for toy in ("toy1", "toy2"):
        X = np.array(t[toy + ".x"])[:, None]
        tm, ev = np.array(t[toy + ".time"]), np.array(t[toy + ".event"], dtype=np.uint8)
        L = o.canonical_layout(tm, ev)
        Xc = o.to_canonical(X, L)
        c = o.coord_terms(Xc, L, 0, np.zeros(3))
        check(toy + "_grad", lambda: abs(c["grad"] - t[toy + ".grad0"][0]) < 1e-14)
        check(toy + "_hess", lambda: abs(c["hess"] - t[toy + ".hess0"][0]) < 1e-14)
        check(toy + "_obj", lambda: abs(c["obj"] - t[toy + ".negloglik0"][0]) < 1e-14)
    d = synth.make("iid", 150, 3, 5, 7, beta_sd=0.7, tie_round=10.0)
    beta = np.array([0.6, -0.9, 0.4])
    L = o.canonical_layout(d.time, d.event, d.stratum)
    Xc = o.to_canonical(d.X, L)
    fe = o.full_eval(Xc, L, beta)
    tol = 1e-11 * d.event.sum()
    check("brute_obj", lambda: abs(fe.objective - o.neg_loglik_brute(d.X, d.time, d.event, d.stratum, beta)) < tol)
    check("brute_grad", lambda: np.allclose(fe.grad, o.grad_brute(d.X, d.time, d.event, d.stratum, beta), atol=tol))
    check("brute_info", lambda: np.allclose(fe.info, o.info_brute(d.X, d.time, d.event, d.stratum, beta), atol=tol))
    eta = Xc @ beta
    check("brute_coord", lambda: all(
        abs(o.coord_terms(Xc, L, j, eta)["grad"] - gb) < tol and abs(o.coord_terms(Xc, L, j, eta)["obj"] - ob) < tol
        for j, gb, ob in zip(range(3), o.grad_brute(d.X, d.time, d.event, d.stratum, beta),
                             [o.neg_loglik_brute(d.X, d.time, d.event, d.stratum, beta)] * 3)))
    check("brute_hdiag", lambda: np.allclose(fe.hess_diag, o.hess_diag_brute(d.X, d.time, d.event, d.stratum, beta),
                                             atol=tol))
    # strong effects: the optimum is several trust-region widths away from 0
    ds = synth.make("iid", 300, 3, 5, 8, beta=[3.0, -3.0, 2.0])
    Ls = o.canonical_layout(ds.time, ds.event, ds.stratum)
    Xs = o.to_canonical(ds.X, Ls)
    nw = o.fit_newton(ds.X, ds.time, ds.event, ds.stratum, layout=Ls, Xc=Xs)
    cd = o.fit_ccd(ds.X, ds.time, ds.event, ds.stratum, layout=Ls, Xc=Xs, tol=1e-13, max_sweeps=300)
    check("ccd_vs_newton", lambda: cd.converged and np.max(np.abs(cd.beta - nw.beta)) < 1e-9)
    gb = o.grad_brute(ds.X, ds.time, ds.event, ds.stratum, cd.beta)
    check("ccd_zero_score", lambda: np.max(np.abs(gb)) < 1e-8)
    # Efron's correction: toy 3 closed forms and the brute-force definition on tied data
    X3 = np.array(t["toy3.x"])[:, None]
    t3, e3 = np.array(t["toy3.time"]), np.array(t["toy3.event"], dtype=np.uint8)
    L3 = o.canonical_layout(t3, e3)
    X3c = o.to_canonical(X3, L3)
    ce = o.coord_terms(X3c, L3, 0, np.zeros(4), "efron")
    fe3 = o.full_eval(X3c, L3, [0.0], ties="efron")
    check("efron_toy3_grad", lambda: abs(ce["grad"] - t["toy3.efron.grad0"][0]) < 1e-14
          and abs(fe3.grad[0] - t["toy3.efron.grad0"][0]) < 1e-14)
    check("efron_toy3_hess", lambda: abs(ce["hess"] - t["toy3.efron.hess0"][0]) < 1e-14
          and abs(fe3.info[0, 0] - t["toy3.efron.hess0"][0]) < 1e-14)
    check("efron_toy3_obj", lambda: abs(ce["obj"] - t["toy3.efron.negloglik0"][0]) < 1e-14
          and abs(fe3.objective - t["toy3.efron.negloglik0"][0]) < 1e-14)
    de = synth.make("iid", 150, 3, 5, 7, beta_sd=0.7, tie_round=5.0)
    Le = o.canonical_layout(de.time, de.event, de.stratum)
    fee = o.full_eval(o.to_canonical(de.X, Le), Le, beta, ties="efron")
    tole = 1e-11 * de.event.sum()
    check("efron_brute_info", lambda: np.allclose(fee.info, o.info_efron_brute(de.X, de.time, de.event, de.stratum,
                                                                                beta), atol=tole))
    check("efron_brute_grad", lambda: np.allclose(fee.grad, o.grad_efron_brute(de.X, de.time, de.event, de.stratum,
                                                                                beta), atol=tole))
    Xec = o.to_canonical(de.X, Le)
    etae = Xec @ beta
    ge = o.grad_efron_brute(de.X, de.time, de.event, de.stratum, beta)
    oe = o.neg_loglik_efron_brute(de.X, de.time, de.event, de.stratum, beta)
    check("efron_brute_coord", lambda: all(
        abs(o.coord_terms(Xec, Le, j, etae, "efron")["grad"] - ge[j]) < tole
        and abs(o.coord_terms(Xec, Le, j, etae, "efron")["obj"] - oe) < tole for j in range(3)))
    gam = 5.0
    # a weak fourth column so that the l1 optimum has an exact zero (dead zone |g'| <= gamma)
    X4 = np.asfortranarray(np.column_stack([d.X, 0.02 * np.random.default_rng(2).standard_normal(d.n)]))
    L4 = o.canonical_layout(d.time, d.event, d.stratum)
    c1 = o.fit_ccd(X4, d.time, d.event, d.stratum, layout=L4, gamma=gam, tol=1e-13, max_sweeps=300)
    g1 = o.grad_brute(X4, d.time, d.event, d.stratum, c1.beta)
    nz = c1.beta != 0
    check("l1_kkt", lambda: c1.converged and (~nz).any() and nz.any()
          and np.allclose(g1[nz] + gam * np.sign(c1.beta[nz]), 0, atol=1e-8)
          and np.all(np.abs(g1[~nz]) <= gam + 1e-8))
    return fails


def test_unmutated_oracle_passes_compact_pins():
    assert _pins() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mpath = tmp_path / "mut.c"
    mpath.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-std=c99", str(mpath), "-o", str(so), "-lm"])
    monkeypatch.setattr(o, "_lib", o.load_library(str(so)))
    fails = _pins()
    assert fails, f"mutant {name} passed every pin"
