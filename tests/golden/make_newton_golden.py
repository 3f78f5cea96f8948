"""Write the oracle's unpenalised optimum for the full-size mixed-precision workload.

    python tests/golden/make_newton_golden.py

Workload: N = 1e6 rows, P = 200 AR(1) columns (corr 0.5^|i-j|), K = 5e4
strata, seed 2 (synth.config_mixed).  The optimum comes from the FP64 oracle's
Newton iteration (numpy Cholesky of the full information matrix, Eq. strat_h)
run to max|step| <= 1e-14 max(1, max|beta|); no GPU code is involved.  Output:
tests/golden/newton_mixed_n1e6_p200.txt with one 'beta' line of P values
(repr precision) and the objective at the optimum.  Takes about a minute.
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import cox_oracle as orc  # noqa: E402
from paper_2310_16238_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "newton_mixed_n1e6_p200.txt")


def main():
    t0 = time.time()
    d = synth.config_mixed()
    fit = orc.fit_newton(d.X, d.time, d.event, d.stratum, tol=1e-14)
    assert fit.converged, "oracle Newton did not converge"
    with open(OUT, "w") as fh:
        fh.write("# Oracle Newton optimum (FP64 CPU) for synth.config_mixed(): N=1e6, P=200, AR(1) 0.5,\n")
        fh.write(f"# K=5e4 strata, seed 2.  Written by tests/golden/make_newton_golden.py;\n")
        fh.write(f"# {fit.iters} Newton iterations, last max|step| {fit.last_step:.3e}, "
                 f"max|grad| {float(abs(fit.grad).max()):.3e}.\n")
        fh.write("objective " + repr(float(fit.objective)) + "\n")
        fh.write("beta " + " ".join(repr(float(v)) for v in fit.beta) + "\n")
    print(f"wrote {OUT} in {time.time() - t0:.1f}s ({fit.iters} iterations)")


if __name__ == "__main__":
    main()
