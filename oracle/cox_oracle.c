/*
 * cox_oracle.c -- plain, sequential FP64 reference for the stratified Cox model.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP path.
 *
 * Every routine walks the rows one by one in the canonical order of Sec. 2.7:
 * rows grouped by stratum, and inside a stratum sorted by decreasing observed
 * time, so each risk set R_k(Y_ki) = {r in stratum k : Y_kr >= Y_ki} is a
 * prefix of the stratum.  The caller (oracle/cox_oracle.py) builds that order.
 *
 * Ties (reading of R_k(Y) with ">=" taken literally, Breslow): an event at time
 * Y uses the risk-set sum over *all* rows with Y_r >= Y, i.e. the inclusive
 * prefix at the last row of its tie group.  gend[i] is that row's index.
 *
 * exp() is taken after subtracting the running maximum of eta over the
 * risk set; the likelihood ratios are invariant under such a shift, and the
 * log-likelihood adds the shift back, so no exp() overflows or underflows.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ scan (Sec. 2.6) */

typedef struct { int f; double a; } orc_pair;

/* The flag-value operator of Sec. 2.6 with (+) as the base operator:
 * (f_i, a_i) (+)s (f_j, a_j) = (f_i | f_j, f_j ? a_j : a_i + a_j). */
static orc_pair orc_seg_op(orc_pair x, orc_pair y)
{
    orc_pair r;
    r.f = x.f | y.f;
    r.a = y.f ? y.a : x.a + y.a;
    return r;
}

/* Inclusive segmented scan b_i = (f_0,a_0) (+)s ... (+)s (f_i,a_i), value part. */
void orc_segscan(int64_t n, const double *a, const uint8_t *head, double *b)
{
    if (n <= 0) return;
    orc_pair acc = { head[0] ? 1 : 0, a[0] };
    b[0] = acc.a;
    for (int64_t i = 1; i < n; ++i) {
        orc_pair nx = { head[i] ? 1 : 0, a[i] };
        acc = orc_seg_op(acc, nx);
        b[i] = acc.a;
    }
}

/*
 * Risk-set sums kept with a running shift: the triple (s0, s1, s2) holds
 * sum w_r, sum w_r x_r, sum w_r x_r^2 with w_r = exp(eta_r - m), where m is the
 * largest eta seen so far in the stratum.  Combining a new row is the (+) of
 * Sec. 2.6 taken in this scaled representation: when eta_r exceeds m the old
 * sums are rescaled by exp(m - eta_r) first.  In exact arithmetic
 * exp(m) * s_k equals the plain sum, so ratios s1/s0 and s2/s0 are the
 * ratios of Eqs. strat_g / strat_h and log(s0) + m is the log of the risk-set
 * sum of Eq. strat_l, without overflow or underflow of exp().
 */
typedef struct { int f; double m, s0, s1, s2; } orc_state;

/* (f_i, A) (+)s (f_j, B) = (f_i | f_j, f_j ? B : A (+) B), with (+) the shifted sum. */
static orc_state orc_state_op(orc_state a, orc_state b)
{
    orc_state r;
    r.f = a.f | b.f;
    if (b.f) { r.m = b.m; r.s0 = b.s0; r.s1 = b.s1; r.s2 = b.s2; return r; }
    double M = a.m > b.m ? a.m : b.m;
    double ea = exp(a.m - M), eb = exp(b.m - M);
    r.m = M;
    r.s0 = a.s0 * ea + b.s0 * eb;
    r.s1 = a.s1 * ea + b.s1 * eb;
    r.s2 = a.s2 * ea + b.s2 * eb;
    return r;
}

/* Row r as a scan element: D = 1, N1 = x, N2 = x^2 at its own shift m = eta_r
 * (i.e. D = exp(eta_r - m), N1 = x D, N2 = x^2 D of Eqs. parallel_d/n1/n2). */
static orc_state orc_row(int head, double eta, double x)
{
    orc_state r = { head, eta, 1.0, x, x * x };
    return r;
}

/*
 * Coordinate quantities for column x_j (Eqs. parallel_g / parallel_h):
 *   out[0] = g'(beta_j)  = -delta'X_j + delta' (S[N1] / S[D])
 *   out[1] = g''(beta_j) =  delta' (S[N2] / S[D]) - delta' (S[N1] / S[D])^2
 *   out[2] = -log partial likelihood (Eq. strat_l) at this eta
 *   out[3] = delta' (S[N2] / S[D])   (second-moment term; scale for degeneracy)
 * where S is the inclusive segmented scan and each event reads the scan at the
 * end of its tie group.
 */
void orc_coord_terms(int64_t n, const double *xj, const double *eta, const uint8_t *head,
                     const uint8_t *event, const int64_t *gend, double *out)
{
    orc_state *S = (orc_state *)malloc(sizeof(orc_state) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        orc_state e = orc_row(i == 0 ? 1 : head[i], eta[i], xj[i]);
        S[i] = (i == 0) ? e : orc_state_op(S[i - 1], e);
    }
    double dx = 0, de = 0, g1 = 0, h1 = 0, h2 = 0, ll = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!event[i]) continue;
        const orc_state *g = &S[gend[i]];
        double r1 = g->s1 / g->s0;
        dx += xj[i];
        de += eta[i];
        g1 += r1;
        h1 += g->s2 / g->s0;
        h2 += r1 * r1;
        ll += log(g->s0) + g->m;
    }
    out[0] = -dx + g1;
    out[1] = h1 - h2;
    out[2] = -de + ll;
    out[3] = h1;
    free(S);
}

/* ------------------------------------------------------------------ Efron's ties */

/*
 * Efron's approximation for tied event times (B. Efron, "The efficiency of Cox's
 * likelihood function for censored data", JASA 72, 1977), a variant the paper does not
 * discuss.  A tie group g with d events D_g and risk set R_g (the rows of the stratum
 * with Y_r >= Y_g) contributes
 *     -sum_{i in D_g} eta_i + sum_{l=0}^{d-1} log(S0_g - (l/d) E0_g)
 * to -log L, with S0_g = sum_{r in R_g} w_r and E0_g = sum_{i in D_g} w_i: the l-th of
 * the tied events keeps only (1 - l/d) of the tied events' weight in its risk set.  The
 * derivatives in beta_j use the same sums with w x_j (S1, E1) and w x_j^2 (S2, E2):
 *     g'  = -sum_D x_j + sum_l (S1 - a_l E1) / (S0 - a_l E0)
 *     g'' =  sum_l [ (S2 - a_l E2) / (S0 - a_l E0) - ((S1 - a_l E1) / (S0 - a_l E0))^2 ]
 * with a_l = l/d.  A group with one event (d = 1) is Breslow's term exactly.
 * Same outputs as orc_coord_terms; the E sums are taken at the group's shift m.
 */
void orc_coord_terms_efron(int64_t n, const double *xj, const double *eta, const uint8_t *head,
                           const uint8_t *event, const int64_t *gend, double *out)
{
    orc_state *S = (orc_state *)malloc(sizeof(orc_state) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        orc_state e = orc_row(i == 0 ? 1 : head[i], eta[i], xj[i]);
        S[i] = (i == 0) ? e : orc_state_op(S[i - 1], e);
    }
    double sx = 0, se = 0, t1 = 0, t2 = 0, t3 = 0, lsum = 0;
    int64_t i = 0;
    while (i < n) {
        const int64_t e = gend[i];          /* rows i..e form one tie group */
        const orc_state *g = &S[e];
        int nd = 0;
        double e0 = 0, e1 = 0, e2 = 0;
        for (int64_t r = i; r <= e; ++r) {
            if (!event[r]) continue;
            double w = exp(eta[r] - g->m);
            ++nd;
            e0 += w;
            e1 += w * xj[r];
            e2 += w * xj[r] * xj[r];
            sx += xj[r];
            se += eta[r];
        }
        for (int l = 0; l < nd; ++l) {
            double a = (double)l / (double)nd;
            double A = g->s0 - a * e0;
            double r1 = (g->s1 - a * e1) / A;
            t1 += r1;
            t2 += (g->s2 - a * e2) / A;
            t3 += r1 * r1;
            lsum += log(A) + g->m;
        }
        i = e + 1;
    }
    out[0] = t1 - sx;
    out[1] = t2 - t3;
    out[2] = lsum - se;
    out[3] = t2;
    free(S);
}

/* ------------------------------------------------------------------ CCD (Sec. 2.4) */

/* Coordinates whose curvature is numerically zero (a ones column, a column
 * constant within strata) have g'' = 0 in exact arithmetic and carry no
 * information; they are skipped, which pins them at their start value. */
static int degenerate(double g2, double h1)
{
    return !(g2 > 1e-12 * fabs(h1)) || !isfinite(g2);
}

/*
 * One coordinate update.  Newton step -g'/g'' (Eq. newton) on the smooth part;
 * with an l1 weight gamma > 0 at beta_j = 0 the two one-sided directional
 * derivatives g' + gamma and g' - gamma decide the direction (or no move);
 * away from 0 the step uses g' + gamma sgn(beta_j) and stops at 0 if it would
 * cross it.  The step is clipped to the trust region [-Delta_j, Delta_j], and
 * Delta_j <- max(2|step|, Delta_j / 2).
 */
double orc_ccd_step(double beta, double g1, double g2, double h1, double gamma, double *trust)
{
    if (degenerate(g2, h1)) return 0.0;
    double step;
    if (gamma <= 0.0) {
        step = -g1 / g2;
    } else if (beta != 0.0) {
        double sg = beta > 0 ? 1.0 : -1.0;
        step = -(g1 + gamma * sg) / g2;
    } else if (g1 + gamma < 0.0) {
        step = -(g1 + gamma) / g2;
    } else if (g1 - gamma > 0.0) {
        step = -(g1 - gamma) / g2;
    } else {
        step = 0.0;
    }
    double lim = *trust;
    if (fabs(step) > lim) step = step > 0 ? lim : -lim;
    if (gamma > 0.0 && beta != 0.0) {
        double nb = beta + step;
        if ((beta > 0 && nb < 0) || (beta < 0 && nb > 0)) step = -beta;
    }
    double t2 = 2.0 * fabs(step), half = 0.5 * lim;
    *trust = t2 > half ? t2 : half;
    return step;
}

/*
 * Cyclic coordinate descent, coordinates 0..p-1 in order each sweep.  eta is
 * kept up to date with eta += x_j * step after every coordinate
 * (Eq. parallel_xb).  Stops after the first sweep whose largest |step| is at
 * most tol * max(1, max_j |beta_j|).  Returns 0 when converged, 1 otherwise.
 *   X     : column-major n x p, leading dimension ldx, canonical row order
 *   gamma : per-column l1 weight (0 = unpenalised)
 *   beta  : in = start, out = estimate
 *   grad  : out, g' of the last evaluation of each coordinate (may be NULL)
 *   info  : out[0] = sweeps, out[1] = last max |step|, out[2] = objective at exit
 */
int orc_ccd_fit_ties(int64_t n, int64_t p, const double *X, int64_t ldx, const uint8_t *head,
                     const uint8_t *event, const int64_t *gend, const double *gamma, double tol,
                     int max_sweeps, double *beta, double *grad, double *info, int efron);

int orc_ccd_fit(int64_t n, int64_t p, const double *X, int64_t ldx, const uint8_t *head,
                const uint8_t *event, const int64_t *gend, const double *gamma, double tol,
                int max_sweeps, double *beta, double *grad, double *info)
{
    return orc_ccd_fit_ties(n, p, X, ldx, head, event, gend, gamma, tol, max_sweeps, beta, grad, info, 0);
}

/* The same descent with each coordinate's terms from orc_coord_terms (efron = 0, the
 * risk sets of Eq. strat_l) or orc_coord_terms_efron (efron = 1). */
int orc_ccd_fit_ties(int64_t n, int64_t p, const double *X, int64_t ldx, const uint8_t *head,
                     const uint8_t *event, const int64_t *gend, const double *gamma, double tol,
                     int max_sweeps, double *beta, double *grad, double *info, int efron)
{
    double *eta = (double *)calloc((size_t)n, sizeof(double));
    double *trust = (double *)malloc(sizeof(double) * (size_t)p);
    for (int64_t j = 0; j < p; ++j) {
        trust[j] = 1.0;
        if (beta[j] != 0.0)
            for (int64_t i = 0; i < n; ++i) eta[i] += X[j * ldx + i] * beta[j];
    }
    int sweeps = 0, converged = 0;
    double last = 0.0, obj = 0.0;
    while (sweeps < max_sweeps && !converged) {
        double maxstep = 0.0;
        for (int64_t j = 0; j < p; ++j) {
            double t[4];
            const double *xj = X + j * ldx;
            if (efron) orc_coord_terms_efron(n, xj, eta, head, event, gend, t);
            else orc_coord_terms(n, xj, eta, head, event, gend, t);
            if (grad) grad[j] = t[0];
            obj = t[2];
            double s = orc_ccd_step(beta[j], t[0], t[1], t[3], gamma ? gamma[j] : 0.0, &trust[j]);
            if (s != 0.0) {
                beta[j] += s;
                for (int64_t i = 0; i < n; ++i) eta[i] += xj[i] * s;
            }
            if (fabs(s) > maxstep) maxstep = fabs(s);
        }
        ++sweeps;
        double bmax = 1.0;
        for (int64_t j = 0; j < p; ++j) if (fabs(beta[j]) > bmax) bmax = fabs(beta[j]);
        last = maxstep;
        converged = maxstep <= tol * bmax;
    }
    if (info) { info[0] = sweeps; info[1] = last; info[2] = obj; }
    free(trust);
    free(eta);
    return converged ? 0 : 1;
}

/* ------------------------------------------------------------------ full evaluation */

/*
 * Risk-set sums of every column at the end of every tie group that holds an
 * event, for the full gradient and information matrix.  Groups are numbered
 * in canonical order; for group g (ending at row e), with the running shift
 * m_g = max of eta over the risk set (rows of the stratum up to e):
 *   S0g[g]        = sum over the risk set of w_r,        w_r = exp(eta_r - m_g)
 *   S1g[g*p + j]  = sum over the risk set of w_r x_rj
 *   S2dg[g*p + j] = sum over the risk set of w_r x_rj^2
 *   dg[g]         = number of events in the group,  mg[g] = m_g
 * Also returns, per row, wl[r] = exp(eta_r) * Lambda_r, where
 * Lambda_r = sum over the event groups g of r's stratum with Y_g <= Y_r of
 * d_g / (exp(m_g) S0g[g]) (the Breslow cumulative hazard), accumulated in the
 * log domain.  Returns the number of event groups.
 */
int64_t orc_group_sums(int64_t n, int64_t p, const double *X, int64_t ldx, const double *eta,
                       const uint8_t *head, const uint8_t *event, const int64_t *gend,
                       double *S0g, double *S1g, double *S2dg, double *dg, double *mg,
                       double *wl)
{
    double *s1 = (double *)calloc((size_t)p, sizeof(double));
    double *s2 = (double *)calloc((size_t)p, sizeof(double));
    double *lh = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1)); /* log(d_g/S0_g) - m_g */
    double s0 = 0.0, m = -INFINITY;
    int64_t G = 0;
    int64_t i = 0;
    while (i < n) {
        int64_t e = gend[i];          /* rows i..e form one tie group */
        int nd = 0;
        for (int64_t r = i; r <= e; ++r) {
            if (head[r] || r == 0) {
                s0 = 0.0;
                m = -INFINITY;
                memset(s1, 0, sizeof(double) * (size_t)p);
                memset(s2, 0, sizeof(double) * (size_t)p);
            }
            if (eta[r] > m) {
                double sc = (m == -INFINITY) ? 0.0 : exp(m - eta[r]);
                s0 *= sc;
                for (int64_t j = 0; j < p; ++j) { s1[j] *= sc; s2[j] *= sc; }
                m = eta[r];
            }
            double w = exp(eta[r] - m);
            s0 += w;
            for (int64_t j = 0; j < p; ++j) {
                double x = X[j * ldx + r];
                s1[j] += w * x;
                s2[j] += w * x * x;
            }
            nd += event[r] ? 1 : 0;
        }
        if (nd > 0) {
            S0g[G] = s0;
            memcpy(S1g + G * p, s1, sizeof(double) * (size_t)p);
            memcpy(S2dg + G * p, s2, sizeof(double) * (size_t)p);
            dg[G] = nd;
            mg[G] = m;
            for (int64_t r = i; r <= e; ++r) lh[r] = log((double)nd / s0) - m;
            ++G;
        } else {
            for (int64_t r = i; r <= e; ++r) lh[r] = -INFINITY;
        }
        i = e + 1;
    }
    /* Lambda_r sums d_g / S0_g over the event groups at or after row r's group in
     * the same stratum (those have Y_g <= Y_r); accumulate from the stratum's end
     * as a log-sum-exp, then wl_r = exp(eta_r + log Lambda_r). */
    double la = -INFINITY;
    for (int64_t r = n - 1; r >= 0; ) {
        int64_t e = r, s = r;
        while (s > 0 && gend[s - 1] == e) --s;   /* start of r's tie group */
        double t = lh[e];
        if (t != -INFINITY) {
            double M = la > t ? la : t;
            la = M + log(exp(la - M) + exp(t - M));
        }
        for (int64_t q = s; q <= e; ++q) wl[q] = (la == -INFINITY) ? 0.0 : exp(eta[q] + la);
        if (head[s]) la = -INFINITY;
        r = s - 1;
    }
    free(lh);
    free(s2);
    free(s1);
    return G;
}

/*
 * Efron's form of the group sums (see orc_coord_terms_efron).  For every tie group g
 * holding events, at its shift m_g (the running maximum of eta over R_g):
 *   S0g[g], S1g[g*p + j], S2dg[g*p + j]  the risk-set sums of w, w x_j, w x_j^2
 *   E0g[g], E1g[g*p + j], E2dg[g*p + j]  the same sums over the group's events only
 *   dg[g], mg[g]                         event count and shift
 * and per row wl[r] = w_r c_r with w_r = exp(eta_r), where
 *   c_r = sum over the event groups g of r's stratum with Y_g <= Y_r of h_g
 *         - delta_r k_{g(r)},   h_g = sum_l 1/A_{g,l},  k_g = sum_l (l/d_g)/A_{g,l},
 *   A_{g,l} = S0_g - (l/d_g) E0_g (unshifted):
 * exchanging the sums, sum_g sum_l (S2_g - a_l E2_g)/A_{g,l} = sum_r w_r c_r x_r x_r'.
 * log h and log k are accumulated with the shifts, so no exp() overflows.  Returns the
 * number of event groups.
 */
int64_t orc_group_sums_efron(int64_t n, int64_t p, const double *X, int64_t ldx, const double *eta,
                             const uint8_t *head, const uint8_t *event, const int64_t *gend,
                             double *S0g, double *S1g, double *S2dg, double *E0g, double *E1g,
                             double *E2dg, double *dg, double *mg, double *wl)
{
    double *q1 = (double *)calloc((size_t)p, sizeof(double));
    double *q2 = (double *)calloc((size_t)p, sizeof(double));
    double *lh = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1)); /* log h_g per row of g */
    double *lk = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1)); /* log k_g per row of g */
    double s0 = 0.0, m = -INFINITY;
    int64_t G = 0;
    int64_t i = 0;
    while (i < n) {
        int64_t e = gend[i];
        int nd = 0;
        for (int64_t r = i; r <= e; ++r) {
            if (head[r] || r == 0) {
                s0 = 0.0;
                m = -INFINITY;
                memset(q1, 0, sizeof(double) * (size_t)p);
                memset(q2, 0, sizeof(double) * (size_t)p);
            }
            if (eta[r] > m) {
                double sc = (m == -INFINITY) ? 0.0 : exp(m - eta[r]);
                s0 *= sc;
                for (int64_t j = 0; j < p; ++j) { q1[j] *= sc; q2[j] *= sc; }
                m = eta[r];
            }
            double w = exp(eta[r] - m);
            s0 += w;
            for (int64_t j = 0; j < p; ++j) {
                double x = X[j * ldx + r];
                q1[j] += w * x;
                q2[j] += w * x * x;
            }
            nd += event[r] ? 1 : 0;
        }
        if (nd > 0) {
            double e0 = 0.0;
            double *e1 = E1g + G * p, *e2 = E2dg + G * p;
            for (int64_t j = 0; j < p; ++j) { e1[j] = 0.0; e2[j] = 0.0; }
            for (int64_t r = i; r <= e; ++r) {
                if (!event[r]) continue;
                double w = exp(eta[r] - m);
                e0 += w;
                for (int64_t j = 0; j < p; ++j) {
                    double x = X[j * ldx + r];
                    e1[j] += w * x;
                    e2[j] += w * x * x;
                }
            }
            double h = 0.0, k = 0.0;
            for (int l = 0; l < nd; ++l) {
                double a = (double)l / (double)nd;
                double A = s0 - a * e0;
                h += 1.0 / A;
                k += a / A;
            }
            S0g[G] = s0;
            E0g[G] = e0;
            memcpy(S1g + G * p, q1, sizeof(double) * (size_t)p);
            memcpy(S2dg + G * p, q2, sizeof(double) * (size_t)p);
            dg[G] = nd;
            mg[G] = m;
            for (int64_t r = i; r <= e; ++r) {
                lh[r] = log(h) - m;
                lk[r] = k > 0.0 ? log(k) - m : -INFINITY;
            }
            ++G;
        } else {
            for (int64_t r = i; r <= e; ++r) { lh[r] = -INFINITY; lk[r] = -INFINITY; }
        }
        i = e + 1;
    }
    double lacc = -INFINITY;
    for (int64_t r = n - 1; r >= 0; ) {
        int64_t e = r, s = r;
        while (s > 0 && gend[s - 1] == e) --s;
        double t = lh[e];
        if (t != -INFINITY) {
            double M = lacc > t ? lacc : t;
            lacc = M + log(exp(lacc - M) + exp(t - M));
        }
        for (int64_t q = s; q <= e; ++q) {
            double v = (lacc == -INFINITY) ? 0.0 : exp(eta[q] + lacc);
            if (event[q] && lk[e] != -INFINITY) v -= exp(eta[q] + lk[e]);
            wl[q] = v;
        }
        if (head[s]) lacc = -INFINITY;
        r = s - 1;
    }
    free(lk);
    free(lh);
    free(q2);
    free(q1);
    return G;
}
