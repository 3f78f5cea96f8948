/*
 * coxmi.h -- C ABI of the MI355X (gfx950) stratified Cox library.
 *
 * The library fits the stratified Cox proportional-hazards model of Sec. 2.1
 * (partial likelihood Eq. strat_l, optional l1 penalty sum_j gamma_j |beta_j|)
 * by cyclic coordinate descent (Sec. 2.4), evaluating each coordinate's
 * gradient and Hessian (Eqs. strat_g / strat_h) with one segmented scan over
 * rows sorted by stratum and decreasing time (Secs. 2.6 and 2.7).
 *
 * Conventions for every entry point
 *   - Return value: COX_OK (0) on success, a negative COX_E* code on error,
 *     COX_NOT_CONVERGED (1) when an iteration limit is hit (outputs are still
 *     filled).  On error the per-handle message is set (cox_last_error) and
 *     no output is written unless stated.
 *   - Matrices are column-major.  beta, gradients and Hessians are indexed by
 *     the caller's column order; row outputs use the caller's row order unless
 *     stated (cox_layout reports the canonical order itself).
 *   - The caller owns every buffer it passes; the library never keeps a
 *     pointer to a caller buffer after a call returns.  cox_init copies the
 *     data into device memory owned by the handle; cox_release frees it.
 *   - A handle is not thread-safe.  Work is issued on the stream given in
 *     cox_options (NULL = the default stream); calls return after that work
 *     has finished, so host outputs are ready on return.
 *   - Ties in time follow the risk-set definition R_k(Y) = {r : Y_kr >= Y}
 *     literally (Breslow): tied rows are all in each other's risk sets.
 */
#ifndef COXMI_H
#define COXMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define COX_OK 0
#define COX_NOT_CONVERGED 1
#define COX_EINVAL (-1)   /* bad argument: sizes, NaN/inf time, event not 0/1, NULL pointer */
#define COX_ENOMEM (-2)   /* device or host allocation failed */
#define COX_EDEVICE (-3)  /* HIP runtime error or a device-side synchronisation time-out */
#define COX_ENUMERIC (-4) /* a risk-set sum left the normal FP64 range (see cox_fit) */
#define COX_EUNSUPPORTED (-5) /* option or size the library does not support */

/* ---------------------------------------------------------------- options */
/* optimiser: cyclic coordinate descent (Sec. 2.4), or Newton steps on the full
 * information matrix with an FP64 Cholesky solve and iterative refinement */
enum { COX_CCD = 0, COX_NEWTON_REFINE = 1 };
/* storage precision of X for the information-matrix contraction (the
 * gradient and objective are always formed in FP64) */
enum { COX_F64 = 0, COX_F32 = 1, COX_BF16 = 2, COX_FP8_E4M3 = 3 };
/* tie handling: COX_BRESLOW takes the risk sets of Eq. strat_l literally (see above);
 * COX_EFRON is Efron's (1977) approximation, which the paper does not discuss: the l-th of
 * the d tied events of a group sees its risk set less l/d of the tied events' own weight
 * (sums S - (l/d) E, l = 0..d-1).  The two agree when no event times are tied. */
enum { COX_BRESLOW = 0, COX_EFRON = 1 };

typedef struct cox_handle cox_handle; /* opaque; owns all device state of one data set */

typedef struct {
    int64_t n;               /* rows (observations), >= 1 */
    int64_t p;               /* columns (covariates), >= 1 */
    const double *x;         /* column-major n x p, leading dimension ldx >= n */
    int64_t ldx;
    const double *time;      /* n observed times Y (finite) */
    const uint8_t *event;    /* n event indicators delta in {0, 1} */
    const int32_t *stratum;  /* n stratum labels (any int32 values); NULL = one stratum */
    int on_device;           /* 0: the four arrays are host memory; 1: device memory of the
                                current device (e.g. torch tensors), see cox_init */
} cox_data;

typedef struct {
    double gamma;             /* l1 strength gamma >= 0 (Sec. 2.1); 0 = unpenalised */
    const uint8_t *penalize;  /* host, p flags: 1 = column penalised; NULL = all columns */
    int mode;                 /* COX_CCD or COX_NEWTON_REFINE */
    int x_precision;          /* contraction precision: COX_F64 or COX_BF16; COX_FP8_E4M3 in mode
                                 COX_NEWTON_REFINE only (p <= 4096); COX_F32: COX_EUNSUPPORTED
                                 (the fit server's precision) */
    int ties;                 /* COX_BRESLOW or COX_EFRON */
    double tol;               /* stop when the largest |step| of a CCD sweep or Newton step <= tol * max(1, max|beta|) */
    int max_iter;             /* maximum number of CCD sweeps or Newton iterations */
    void *stream;             /* hipStream_t to issue work on; NULL = default stream */
} cox_options;

typedef struct {
    int status;               /* return code of the fit */
    int iters;                /* CCD sweeps or Newton iterations performed */
    int64_t coord_evals;      /* CCD: coordinate (g', g'') evaluations = iters * p; Newton: full evaluations */
    double objective;         /* -log partial likelihood + penalty, at the start of the last sweep */
    double kkt_inf;           /* max_j of the l1 KKT residual from the last sweep's gradients */
    double last_step;         /* largest |step| of the last sweep */
    int n_pinned;             /* columns skipped as degenerate (g'' numerically 0) in the last sweep */
    int fallback;             /* 1: a COX_CCD fit whose X beta left the range one shift per fit can hold in
                                 FP64 (the persistent kernel's exp(x'beta - c)) was finished by (proximal)
                                 Newton steps on the full evaluation, whose running-maximum scans hold any
                                 range -- the same optimum; iters and coord_evals then count Newton steps
                                 and full evaluations.  2: the same for a COX_CCD handle of dense X with
                                 more rows than the persistent kernel holds (every fit on it) */
} cox_fit_info;

/* Fill *o with defaults: gamma 0, all columns penalised, COX_CCD, COX_F64,
 * COX_BRESLOW, tol 1e-12, max_iter 1000, default stream. */
void cox_default_options(cox_options *o);

/*
 * Create a handle for data set d (Sec. 2.1: rows (Y_ki, delta_ki, x_ki) in K
 * strata).  Validates the inputs, sorts rows by (stratum ascending, time
 * descending, original index ascending) (Sec. 2.7), marks stratum heads and
 * tie groups, copies X into device memory in that order, and precomputes
 * delta'X_j for every column (first term of Eq. strat_g; summed on the device in
 * a fixed order, so both sources of X below give the same handle bit for bit).
 *   out : receives the handle (set to NULL on error)
 *   d   : data, read only during the call.  d->on_device = 0: host arrays.
 *         d->on_device = 1: device memory of the current device, read after the
 *         work already queued on o->stream (the caller orders any other producer
 *         stream before the call); the keys (time, event, stratum) are copied to the
 *         host for the canonical order, X is gathered into that order on the device
 *         (only a 4-byte source index per row crosses PCIe).  Each array must lie
 *         inside one allocation (x: ldx * (p - 1) + n doubles), else COX_EINVAL.
 *   o   : options (NULL = defaults); penalize is copied
 * Errors: COX_EINVAL (n < 1, p < 1, ldx < n, NULL x/time/event, non-finite
 * time, event not 0/1, on_device arrays not in device memory of the current
 * device), COX_EUNSUPPORTED (p > 12288, or p > 4096 in mode
 * COX_NEWTON_REFINE -- cox_evaluate_full also needs p <= 4096; in mode COX_CCD with
 * p > 4096, n beyond the persistent kernel's register-resident capacity of about
 * CUs x 512 x 16 rows -- a handle of that size and p <= 4096 is created in either mode
 * and then serves cox_fit by (proximal) Newton steps on the full evaluation
 * (info->fallback = 2 in mode COX_CCD: the same optimum), cox_evaluate and
 * cox_evaluate_full, but not cox_coordinate; x_precision COX_F32, or
 * COX_FP8_E4M3 outside mode COX_NEWTON_REFINE),
 * COX_ENOMEM, COX_EDEVICE.  On error *out is NULL and the
 * message is available through cox_last_error(NULL).
 */
int cox_init(cox_handle **out, const cox_data *d, const cox_options *o);

/*
 * Fit beta by cyclic coordinate descent (Sec. 2.4): for j = 0..p-1 in turn,
 * evaluate g'(beta_j) and g''(beta_j) by segmented scan (Eqs. parallel_g,
 * parallel_h), take the Newton step -g'/g'' (Eq. newton) with the l1
 * directional-derivative rule and the trust-region limit, and update
 * X beta incrementally (Eq. parallel_xb).  The whole fit runs in one
 * persistent kernel; only the final result crosses to the host.
 *   beta0    : host, p start values (NULL = zeros)
 *   beta_out : host, p entries, receives the estimate
 *   info     : host, optional (may be NULL)
 * Degenerate columns (g'' <= 1e-12 * delta'(S[N2]/S[D])) are not moved.
 * With mode COX_NEWTON_REFINE: Newton steps beta -= I^{-1} grad with I from
 * cox_evaluate_full's contraction in x_precision, factored by an FP64 Cholesky
 * on the device; once a step is below 1e-3 * max(1, max|beta|) the factor is
 * kept and only the FP64 gradient is recomputed (iterative refinement), until
 * the step is below tol * max(1, max|beta|).  A step that raises the objective
 * is halved.  With l1 weights (gamma != 0) the steps are proximal Newton steps:
 * the quadratic model g'D + D'ID/2 plus the l1 term is minimised by coordinate
 * descent with soft thresholding on the device (one wave, I where the contraction
 * left it), and the penalised objective decides the halving; the fixed point meets the l1
 * optimality conditions on the FP64 score, so a reduced-precision I (kept once
 * steps are small) still gives the FP64 optimum.
 * In mode COX_CCD, when an event's risk-set sum under- or overflows FP64 after the
 * persistent kernel's single shift of X beta, the fit is finished by (proximal)
 * Newton steps on the full evaluation, whose running-maximum scans hold any range
 * (the same optimum; info->fallback = 1); a COX_CCD handle of dense X too long for the
 * persistent kernel fits that way from the start (info->fallback = 2).
 * Returns COX_OK, COX_NOT_CONVERGED (max_iter sweeps done; beta_out filled),
 * COX_ENUMERIC (out of range on a handle of indicator X, which has no full
 * evaluation, or in the full evaluation itself), COX_EDEVICE.
 */
int cox_fit(cox_handle *h, const double *beta0, double *beta_out, cox_fit_info *info);

/*
 * Evaluate at beta (host, p): the negative log partial likelihood of
 * Eq. strat_l plus the l1 penalty (objective, may be NULL), the gradient of
 * the unpenalised part (Eq. strat_g, grad: host p, may be NULL) and the
 * diagonal of its Hessian (Eq. strat_h, hess_diag: host p, may be NULL).
 * Each column is one segmented-scan evaluation, as inside a CCD sweep but
 * without moving beta.  Beyond the single shift's FP64 range the values come from
 * cox_evaluate_full (dense X; indicator X returns COX_ENUMERIC).
 */
int cox_evaluate(cox_handle *h, const double *beta, double *objective, double *grad,
                 double *hess_diag);

/*
 * Full evaluation at beta (host, p) through the exchanged-sum form of
 * Eqs. strat_g / strat_h: with Lambda_r the Breslow cumulative hazard of row
 * r's stratum at Y_r and w = exp(X beta),
 *   gradient = X'(w o Lambda - delta),
 *   Hessian  = X' diag(w o Lambda) X - sum_g d_g xbar_g xbar_g',
 * xbar_g the risk-set mean of x at event group g (Sec. 2.7 scans, one pass
 * over X per product).  Outputs (host, any may be NULL): objective (-log L of
 * Eq. strat_l plus the l1 penalty), grad (p), hess_diag (p), info (p x p,
 * row-major, symmetric).  objective, grad and hess_diag are FP64; info is
 * formed in the handle's x_precision (FP64; BF16, or FP8 e4m3 for a
 * COX_NEWTON_REFINE handle, on the matrix cores with FP32 accumulation) and
 * returned as FP64.
 */
int cox_evaluate_full(cox_handle *h, const double *beta, double *objective, double *grad, double *hess_diag,
                      double *info);

/*
 * The quantities one CCD coordinate step uses, for column j at beta (host, p):
 *   out[0] = g'(beta_j)   (Eq. strat_g / parallel_g)
 *   out[1] = g''(beta_j)  (Eq. strat_h / parallel_h)
 *   out[2] = -log partial likelihood at beta (Eq. strat_l, no penalty)
 *   out[3] = delta'(S[N2]/S[D])  (scale used for the degeneracy test)
 * out: host, 4 doubles.  COX_EINVAL if j is out of range.
 */
int cox_coordinate(cox_handle *h, const double *beta, int64_t j, double *out);

/*
 * Canonical order chosen by cox_init (Sec. 2.7).  perm (host, n, may be NULL)
 * receives the original row index of each canonical row; meta (host, n, may
 * be NULL) the packed row word: bit 31 = first row of its stratum (head flag),
 * bit 30 = event, bits 0..28 = number of events in the row's tie group if the
 * row is the last of that group, else 0.  Padding rows are not reported.
 */
int cox_layout(const cox_handle *h, int64_t *perm, uint32_t *meta);

/* The canonical order of Sec. 2.7 on the host, without a handle or a device:
 * the same perm and meta as cox_layout reports after cox_init of these data
 * (rows by stratum ascending, time descending, original index ascending;
 * -0 and +0 are the same time).  time, event, stratum (NULL = one stratum):
 * host, n entries; perm, meta: host, n entries, written on success.
 * Errors: COX_EINVAL (n < 1 or > 2^29 - 1, a NULL pointer, a non-finite time,
 * an event other than 0 or 1), nothing written. */
int cox_canonical_order(int64_t n, const double *time, const uint8_t *event, const int32_t *stratum,
                        int64_t *perm, uint32_t *meta);

/* ---------------------------------------------------------------- time intervals
 * Secs. 2.2-2.3: a model with piecewise-constant time-varying covariates or
 * step-function coefficients is a Cox model stratified on time intervals over an
 * augmented data set.  Given cut points t_1 < ... < t_{K-1} (K = ncuts + 1
 * intervals [t_{k-1}, t_k), t_0 = -inf, the last interval closed at max Y):
 *   rows     : (interval k, subject i) for every i with Y_i >= t_{k-1} (a subject
 *              that left before t_{k-1} is in no risk set of interval k), interval
 *              by interval, subjects in their original order within one;
 *   time     : min(Y_i, t_k) (Y_i in the last interval);
 *   event    : delta_i if Y_i lies in interval k, else 0;
 *   stratum  : the pair (original stratum, k), numbered s * K + k with s the rank
 *              of the original label among the distinct labels (one stratum: s = 0);
 *   columns  : in the original order; a column j with tv_coef[j] = 1 becomes K
 *              columns, the k-th equal to x_ij on interval k's rows and 0 elsewhere
 *              (its coefficient beta_jk applies on interval k); other columns keep
 *              x_ij, or x_by_interval[k][i][j] when given (time-varying covariates).
 * d         : host data as for cox_init; cuts: host, ncuts strictly increasing
 *             finite values (ncuts >= 0); tv_coef: host, p flags, or NULL (none);
 *             x_by_interval: host, K blocks of n x p column-major (leading
 *             dimension d->ldx), or NULL (x applies on every interval).
 * out       : receives a library-owned result; release it with
 *             cox_intervals_release.  Its `data` is ready for cox_init (which copies
 *             it); the maps give the origin of every augmented row and column.
 * Errors: COX_EINVAL (the checks of cox_init, bad cuts, more than 2^31 - 1
 * augmented rows or strata), COX_ENOMEM. */
typedef struct {
    cox_data data;                 /* the augmented data set (library-owned host arrays) */
    int intervals;                 /* K */
    const int64_t *row_subject;    /* [data.n]: original row of each augmented row */
    const int32_t *row_interval;   /* [data.n]: its interval, 0..K-1 */
    const int32_t *col_source;     /* [data.p]: original column of each augmented column */
    const int32_t *col_interval;   /* [data.p]: its interval for a step coefficient, -1 otherwise */
} cox_intervals;

int cox_split_intervals(const cox_data *d, int ncuts, const double *cuts, const uint8_t *tv_coef,
                        const double *x_by_interval, cox_intervals **out);
void cox_intervals_release(cox_intervals *s);

/* ---------------------------------------------------------------- indicator X
 * The paper's covariates are mostly indicators with 3-5% ones (Secs. 3.1-3.2); its
 * kernels touch only the nonzeros of x_j.  A handle on indicator X stores one bit per
 * row (X given as compressed sparse columns of the rows holding a 1; every other entry
 * is 0), so 1e6 rows x 10,000 columns take 1.25 GB instead of 80 GB of FP64, and the
 * persistent CCD kernel reads a thread's rows of x_j from one byte.  With x in {0, 1}
 * every product the kernel forms is exact, so fits equal those on the same X stored
 * dense, bit for bit.
 *   n, p     : rows and columns (1 <= n <= 2^29 - 1, 1 <= p <= 12288)
 *   col_ptr  : host, p + 1 non-decreasing offsets into row_idx, col_ptr[0] = 0
 *   row_idx  : host, col_ptr[p] row indices in [0, n) (order free; repeats count once)
 *   time, event, stratum : as in cox_data
 *   o        : options (mode COX_CCD, x_precision COX_F64; NULL = defaults)
 * The handle runs cox_fit (COX_CCD), cox_evaluate, cox_coordinate, cox_set_penalty,
 * cox_init_resample and cox_init_intervals (the bits are gathered on the device; the
 * children hold indicator X too), cox_cross_validate, cox_bootstrap and the bookkeeping
 * calls; cox_evaluate_full, cox_baseline_hazard and Newton fits return COX_EUNSUPPORTED.  Errors: COX_EINVAL (bad arrays), COX_EUNSUPPORTED (sizes, options,
 * n beyond the resident kernel), COX_ENOMEM, COX_EDEVICE. */
int cox_init_indicator(cox_handle **out, int64_t n, int64_t p, const int64_t *col_ptr, const int32_t *row_idx,
                       const double *time, const uint8_t *event, const int32_t *stratum, const cox_options *o);

/* ---------------------------------------------------------------- sparse X
 * General sparse covariates (Sec. 2.7: the kernels need the nonzeros of x_j only), given
 * as compressed sparse columns with values.  The handle stores the indicator bits of the
 * nonzero rows (as cox_init_indicator) and the nonzero values in device-row order, with
 * per-wave offsets; the persistent CCD kernel reads a thread's bits, finds its values by
 * a prefix sum of bit counts across the wave, and forms every product from the values
 * themselves, so fits equal those on the same X stored dense, bit for bit.  Storage:
 * n/8 bytes per column + 8 bytes per nonzero (+ 4 bytes per 64 threads' rows per column).
 *   n, p     : rows and columns (1 <= n <= 2^29 - 1, 1 <= p <= 12288)
 *   col_ptr  : host, p + 1 non-decreasing offsets into row_idx and values, col_ptr[0] = 0
 *   row_idx  : host, col_ptr[p] row indices in [0, n), distinct within a column (order free)
 *   values   : host, col_ptr[p] finite values (explicit zeros are dropped)
 *   time, event, stratum : as in cox_data
 *   o        : options (mode COX_CCD, x_precision COX_F64; NULL = defaults)
 * The handle runs cox_fit (COX_CCD), cox_evaluate, cox_coordinate, cox_set_penalty and the
 * bookkeeping calls; cox_init_resample, cox_init_intervals (and so cross-validation and
 * bootstrap), cox_evaluate_full, cox_baseline_hazard and Newton fits return
 * COX_EUNSUPPORTED, as does the range fallback of cox_fit (COX_ENUMERIC stays).
 * Errors: COX_EINVAL (bad arrays, a repeated row in a column), COX_EUNSUPPORTED (sizes,
 * options, n beyond the resident kernel), COX_ENOMEM, COX_EDEVICE. */
int cox_init_sparse(cox_handle **out, int64_t n, int64_t p, const int64_t *col_ptr, const int32_t *row_idx,
                    const double *values, const double *time, const uint8_t *event, const int32_t *stratum,
                    const cox_options *o);

/* ---------------------------------------------------------------- resampling, CV, bootstrap
 * Sec. 2.1 chooses the common l1 weight gamma by cross-validation; Sec. 3.2 adds
 * bootstrap percentile intervals.  Both refit the model on resampled data sets:
 * the data set in which original row i of the parent appears count[i] times
 * (0 drops it; copies are tied subjects under the Breslow rule).
 *
 * cox_init_resample: a new handle for that data set, built on the device from
 * the parent's resident X (a gather; X does not cross PCIe again).  Its rows
 * are numbered as if the caller had repeated every row count[i] times in
 * order (cox_layout's perm refers to that numbering), and its canonical order
 * equals cox_canonical_order of those repeated data.  delta'X_j is summed on
 * the device (fixed order), so with every count 1 the child equals the parent
 * up to the rounding of that sum.
 *   parent : a handle on the current device (not modified; must outlive no child)
 *   count  : host, parent n entries; their sum in [1, 2^29 - 1]
 *   o      : options of the child (penalize copied); NULL = the parent's options
 *            and l1 weights
 * Errors: COX_EINVAL (NULL pointer, no rows, another device), COX_EUNSUPPORTED
 * (too many rows, options as for cox_init), COX_ENOMEM, COX_EDEVICE; message via
 * cox_last_error(NULL). */
int cox_init_resample(cox_handle **out, const cox_handle *parent, const uint32_t *count, const cox_options *o);

/* The interval-stratified model of Secs. 2.2-2.3 (step-function coefficients) built on
 * the device from a handle on the original data, without the augmented X ever
 * existing on the host or crossing PCIe: rows, strata, times and events are those of
 * cox_split_intervals (same cuts and tv_coef rules, same row and column order, so
 * cox_layout's perm numbers its augmented rows), and each augmented column is
 * gathered from the parent's resident column (zero outside its interval for a step
 * coefficient; a parent on indicator X gives an indicator child, COX_CCD in FP64).
 * Covariates that change between intervals need cox_split_intervals.
 *   parent           : a handle on the current device, built from n rows
 *   time, event,
 *   stratum          : host, the n rows the parent was built from (stratum may be NULL);
 *                      checked against the parent's event pattern
 *   ncuts, cuts,
 *   tv_coef          : as for cox_split_intervals (tv_coef: parent p flags or NULL)
 *   o                : options of the child (penalize indexes the augmented columns);
 *                      NULL = the parent's options, each augmented column taking its
 *                      source column's l1 weight
 * Errors: COX_EINVAL (NULL pointer, bad cuts, data that do not match the parent),
 * COX_EUNSUPPORTED (more than 2^29 - 1 rows, or more than 12288 columns after the split
 * (4096 for COX_NEWTON_REFINE)),
 * COX_ENOMEM, COX_EDEVICE; message via cox_last_error(NULL). */
int cox_init_intervals(cox_handle **out, const cox_handle *parent, const double *time, const uint8_t *event,
                       const int32_t *stratum, int ncuts, const double *cuts, const uint8_t *tv_coef,
                       const cox_options *o);

/* Replace h's l1 weights: gamma_j = gamma for penalised columns (penalize: host,
 * p flags, NULL = all), 0 otherwise.  COX_EINVAL for a negative or non-finite
 * gamma.  On a COX_NEWTON_REFINE handle nonzero weights make cox_fit take proximal
 * Newton steps (see cox_fit). */
int cox_set_penalty(cox_handle *h, double gamma, const uint8_t *penalize);

/* K-fold cross-validation of the l1 weight along a path (Sec. 2.1).  For fold k
 * the model is fitted (CCD, warm-started along gammas in the given order, from
 * 0 at gammas[0]) on the rows with fold[i] != k, giving beta_{-k}(gamma), and the
 * cross-validated log partial likelihood
 *     cvl[g] = sum_k [ l(beta_{-k}) - l_{-k}(beta_{-k}) ]
 * is accumulated, l being the log of Eq. strat_l on all rows and l_{-k} on the
 * training rows (the held-out rows' contribution given the rest).
 *   h       : handle on the full data (used for l; its options give the mode --
 *             COX_CCD, or COX_NEWTON_REFINE for proximal Newton fits --, tol, max_iter,
 *             precision and stream of the fold fits)
 *   fold    : host, n entries in [0, nfolds); every fold non-empty and not all rows.  On
 *             a handle from cox_init_intervals all rows of one subject must share a fold
 *             (a subject is held out whole; else COX_EINVAL); on rows split by
 *             cox_split_intervals and passed to cox_init, the caller keeps subjects whole
 *   gammas  : host, ngamma finite values >= 0 (a decreasing path warm-starts best)
 *   penalize: host, p flags or NULL (all columns penalised)
 *   cvl     : host, ngamma outputs; betas: host [nfolds][ngamma][p] or NULL;
 *   status  : host [nfolds][ngamma] fit statuses or NULL
 * Returns COX_OK, COX_NOT_CONVERGED (some fit hit max_iter; outputs filled), or
 * an error. */
int cox_cross_validate(cox_handle *h, int nfolds, const int32_t *fold, int ngamma, const double *gammas,
                       const uint8_t *penalize, double *cvl, double *betas, int *status);

/* Bootstrap refits (Sec. 3.2): replicate b is the data set with row
 * multiplicities counts[b * n .. b * n + n - 1] (host; e.g. a multinomial draw
 * of n rows), fitted with h's options and l1 weights from beta0 (host p, NULL =
 * 0); betas: host [nrep][p]; status: host [nrep] or NULL.  Percentile intervals
 * are quantiles of the betas.  Returns COX_OK, COX_NOT_CONVERGED, or an error. */
int cox_bootstrap(cox_handle *h, int nrep, const uint32_t *counts, const double *beta0, double *betas, int *status);

/* Duration in milliseconds of the last persistent-kernel launch on h, from
 * HIP events recorded on the handle's stream immediately around the launch. */
int cox_last_kernel_ms(const cox_handle *h, double *ms);

/* Device time of the last cox_fit / cox_evaluate / cox_evaluate_full call on
 * h, by phase, from HIP events recorded on the handle's stream around each
 * launch sequence. */
typedef struct {
    double kernel_ms;        /* the persistent CCD / evaluation kernel */
    int evaluations;         /* full evaluations (cox_evaluate_full, COX_NEWTON_REFINE fits) */
    double evaluation_ms;
    int contractions;        /* information-matrix contractions */
    double contraction_ms;
    int solves;              /* Cholesky factor-and-solve or solve-only launches */
    double solve_ms;
} cox_profile;

int cox_last_profile(const cox_handle *h, cox_profile *out);

/* Breslow estimate of the cumulative baseline hazard at beta (the step function whose
 * jump at an event time of stratum k is d / sum_{r in R_k} exp(x_r'beta), the sums of
 * Eq. strat_l): cumhaz[i] = Lambda_0k(Y_i) for original row i in stratum k, the jumps
 * of its stratum at times <= Y_i.  From one full evaluation (the reverse scan Lambda of
 * the score X'(w Lambda - delta), with exp(X beta) taken relative to the running maximum
 * within the stratum and scaled back).  beta: host p; cumhaz: host n.  Needs dense X and
 * p <= 4096 (else COX_EUNSUPPORTED); COX_ENUMERIC as for cox_evaluate_full. */
int cox_baseline_hazard(cox_handle *h, const double *beta, double *cumhaz);

/* Number of rows and columns of the handle; the device row stride (>= n). */
int cox_shape(const cox_handle *h, int64_t *n, int64_t *p, int64_t *ld);

/*
 * Segmented inclusive scan of Sec. 2.6 with + on FP64, on device memory:
 * b[i] = a[i] if head[i] != 0 (or i == 0), else b[i-1] + a[i].
 *   a, head, b : device pointers to n doubles, n bytes, n doubles (b may not alias a)
 *   n          : 0 <= n <= 2^31 - 1 (n = 0 is a no-op)
 *   stream     : hipStream_t or NULL; the call waits for completion.
 * Uses the same device scan as the Cox kernels.  No handle; errors are
 * returned as codes only.
 */
int cox_segscan_f64(const double *a, const uint8_t *head, double *b, int64_t n, void *stream);

/*
 * cox_segscan_f64 for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments, scan and results, but the scan's synchronisation words live in a fixed
 * 4,352-byte array of the library's device memory (one copy per GPU, held until the
 * process ends) instead of a per-call allocation.  A fill kernel on `stream` clears
 * the array before each scan.  Calls no hipMalloc, hipFree or other allocating
 * routine.  Limit: n <= CUs x 1024 x 16 rows (4,194,304 on 256 compute units), else
 * COX_EUNSUPPORTED (as for cox_segscan_f64).  Calls that overlap on one GPU (other
 * streams or threads) share the array and race: the caller serialises them.
 */
int cox_segscan_f64_noalloc(const double *a, const uint8_t *head, double *b, int64_t n, void *stream);

/* Free the handle and all device memory it owns.  NULL is a no-op. */
void cox_release(cox_handle *h);

/* Message for the last error on h (NULL: the last cox_init failure of this thread). */
const char *cox_last_error(const cox_handle *h);

/* ------------------------------------------------------------------ fit server
 *
 * Continuous batching of many independent stratified Cox fits of uneven size
 * (Eq. strat_l per request; unpenalised, or with l1 weights through
 * cox_server_submit_fit).  Each request is put
 * in the canonical order of Sec. 2.7 by a host thread pool and admitted to
 * the device as soon as a slot is free and its footprint fits in the
 * server's device budget; every resident fit then takes one Newton step per
 * round of batched kernels (FP64 objective and score by the segmented scans
 * of Sec. 2.6-2.7; information matrix in FP32 on the matrix cores; FP64
 * Cholesky and iterative refinement as in COX_NEWTON_REFINE).  Requests that
 * arrive while others run join at the next round.  No work item mixes two
 * fits and each fit's sums run in an order fixed by its own (n, p), so a
 * result does not depend on what else is resident.
 */
typedef struct cox_server cox_server;

typedef struct {
    size_t hbm_budget;      /* device bytes for resident fits (default 8 GiB) */
    size_t staging_bytes;   /* pinned host bytes for staged uploads (default 1 GiB) */
    int max_resident;       /* fits resident at once (default 1024) */
    int prep_threads;       /* host threads that canonicalise requests (default 8) */
    int x_precision;        /* COX_F32 (the only value accepted) */
    double tol;             /* stop when max|step| <= tol * max(1, max|beta|) (default 1e-12) */
    int max_iter;           /* Newton steps per fit (default 100) */
    int device;             /* HIP device ordinal, -1 = the current device */
    int fused_rounds;       /* 0: every round is six batched launches driven by the host thread;
                               R in 1..4096: one persistent cooperative launch runs up to R rounds
                               of every resident fit, its phases separated by grid-wide barriers,
                               finished fits reported while it runs; it ends early when all its
                               fits are done or new fits are ready to join.  Results are
                               bit-identical either way (default 0) */
} cox_server_options;

typedef struct {
    double submit_s;        /* seconds on the server's monotonic clock */
    double admit_s;         /* the fit was given device memory */
    double done_s;          /* its result was available */
} cox_request_times;

typedef struct {
    int64_t submitted, completed, iterations;
    int64_t resident_now, resident_peak;
    double mean_resident;   /* resident fits per round, averaged over rounds */
    size_t arena_bytes, arena_peak;
    double gpu_busy_s;      /* sum over rounds of launch-to-completion time */
    double now_s;           /* the server's clock */
    int64_t launches;       /* persistent launches (fused_rounds > 0), else 0 */
    double phase_s[6];      /* fused_rounds > 0: seconds from one grid barrier to the next, by the
                               phase it ends (X beta, row scans, column pass, contraction, information
                               sums, step), summed over launches (workgroup 0's constant-rate clock) */
} cox_server_counters;

/* cox_server_submit flags.
 * COX_SUBMIT_BORROW: do not copy the inputs; the caller keeps x, time, event
 *   and stratum valid and unchanged until the ticket's result is ready.
 * COX_SUBMIT_DEVICE: the four pointers are device memory of the server's
 *   device, already written (the stream that wrote them synchronised).  They
 *   are read in place -- borrowed as above, whatever the other flag says: the
 *   keys (time, event, stratum) are copied to the host for the canonical
 *   order, and the fit's rows of x are gathered into the server's arena on the
 *   device when the fit is admitted, so x crosses no host link.  Keys that fail
 *   the checks of cox_init complete the request with status COX_EINVAL. */
#define COX_SUBMIT_BORROW 1
#define COX_SUBMIT_DEVICE 2

void cox_server_default_options(cox_server_options *o);

/* Allocate the device arena (hbm_budget) and pinned staging, start the
 * threads.  Errors: COX_EINVAL (bad options), COX_EUNSUPPORTED (x_precision
 * other than COX_F32), COX_ENOMEM, COX_EDEVICE; message via
 * cox_server_last_error(NULL). */
int cox_server_create(cox_server **out, const cox_server_options *o);

/* Queue one fit; returns at once with its ticket (tickets start at 1).
 *   d     : data as for cox_init (stratum may be NULL): host memory, or device
 *           memory with COX_SUBMIT_DEVICE (d->on_device = 1 means the same); each
 *           device array must lie inside one allocation, as for cox_init
 *   flags : 0 (inputs copied), COX_SUBMIT_BORROW and/or COX_SUBMIT_DEVICE
 * Errors: COX_EINVAL (the checks of cox_init), COX_EUNSUPPORTED (p > 128),
 * or the server's fatal device error.  A request whose device footprint
 * exceeds hbm_budget (or staging_bytes) completes with status COX_EUNSUPPORTED. */
int cox_server_submit(cox_server *s, const cox_data *d, int flags, uint64_t *ticket);

/* Per-request options of cox_server_submit_fit. */
typedef struct {
    double gamma;             /* l1 weight (Sec. 2.1, R5): 0 = unpenalised */
    const uint8_t *penalize;  /* host, p flags or NULL (every column penalised when gamma > 0) */
    const double *beta0;      /* host, p start values (original column order) or NULL (zeros) */
} cox_fit_request;

/* cox_server_submit with per-request options: an l1-penalised fit (gamma > 0) takes
 * proximal Newton steps, as on a COX_NEWTON_REFINE handle: the quadratic model with the
 * FP64 score and the FP32 information matrix, minimised by cyclic coordinate descent with
 * soft thresholding (the l1 rule of Sec. 2.4) on the device, a step that raises the
 * penalised objective halved; info->objective is the penalised objective and kkt_inf the
 * largest violation of the l1 optimality conditions.  beta0 starts the fit elsewhere than
 * at zero (a warm start along a path of weights).  r = NULL is cox_server_submit.
 * Errors: those of cox_server_submit, COX_EINVAL (gamma < 0 or not finite, beta0 not finite). */
int cox_server_submit_fit(cox_server *s, const cox_data *d, int flags, const cox_fit_request *r, uint64_t *ticket);

/* cox_cross_validate with the fold fits batched through a fit server (Sec. 3.2's 10-fold
 * l1 path as many small independent fits): for each weight in turn the nfolds training-set
 * fits are submitted together (cox_server_submit_fit: proximal Newton steps, FP32
 * information matrix, FP64 score), each warm-started from its fold's fit at the previous
 * weight; the criterion is cox_cross_validate's, from FP64 evaluations on h and on a
 * training-set handle per fold.
 *   h   : handle made by cox_init from d (not an interval or resampled handle)
 *   srv : the server (p <= 128); its tol and max_iter rule the fold fits
 *   d   : the same data in host memory
 * Other arguments and outputs as cox_cross_validate.  Errors: those of
 * cox_cross_validate, COX_EINVAL (srv or d missing, d on the device or not h's shape),
 * the server's (COX_EUNSUPPORTED for p > 128). */
int cox_cross_validate_served(cox_handle *h, cox_server *srv, const cox_data *d, int nfolds, const int32_t *fold,
                              int ngamma, const double *gammas, const uint8_t *penalize, double *cvl, double *betas,
                              int *status);

/* Collect a result: returns COX_OK and fills beta_out (p doubles, original
 * column order), info (status COX_OK, COX_NOT_CONVERGED, COX_ENUMERIC, ...;
 * iters = Newton steps, coord_evals = evaluations) and times (each may be
 * NULL); the result is then released.  Returns 1 while the fit is pending and
 * COX_EINVAL for an unknown or already collected ticket. */
int cox_server_poll(cox_server *s, uint64_t ticket, double *beta_out, cox_fit_info *info,
                    cox_request_times *times);

/* Block until the ticket's result is ready (COX_OK), the timeout passes
 * (1; timeout_s < 0 waits for ever) or the server failed (its error code). */
int cox_server_wait(cox_server *s, uint64_t ticket, double timeout_s);

/* Block until every submitted fit has finished and its device slot has been released (a
 * result can be ready a little before its slot is: fits are reported as soon as their final
 * state reaches the host); codes as cox_server_wait. */
int cox_server_drain(cox_server *s, double timeout_s);

int cox_server_stats(cox_server *s, cox_server_counters *st);

/* Message for the last error on s (NULL: the last failed cox_server_create of this thread). */
const char *cox_server_last_error(cox_server *s);

/* Stop the threads (fits still running are abandoned) and free everything. */
void cox_server_destroy(cox_server *s);

#ifdef __cplusplus
}
#endif

#endif /* COXMI_H */
