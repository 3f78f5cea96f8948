// serve.h -- device-side layout of the fit server (kernels in serve.hip, host
// engine in server.cpp).
//
// Every resident fit owns a block of the server's device arena holding its
// canonical data and its Newton state; one launch of each batched kernel
// covers all resident fits through a list of (fit, piece) work items, so fits
// of any size and at any stage of their iteration share the same launches.
// No work item mixes two fits, and each fit's sums are taken in an order that
// depends only on its own (n, p), so a fit's result is the same whatever else
// is resident.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace coxmi {
namespace serve {

constexpr int kMaxP = 128;        // columns of a served fit (its Cholesky factor lives in LDS)
constexpr int kRowPad = 64;       // rows are padded to a multiple of this
constexpr int kEtaRows = 256;     // rows per work item of the X beta kernel
constexpr int kMaxRange = 4096;   // rows (event groups) per K range of the contraction, at most
constexpr int kMinRange = 1024;   //   and at least: a fit's range is about an eighth of its rows, in
                                  //   steps of 256, so that a small fit's contraction still spreads
                                  //   over several workgroups
constexpr int kColBlock = 4;      // columns per wave of the column pass
constexpr int kTile = 32;         // edge of a contraction tile (one MFMA block)
constexpr int kScanTile = 4096;   // rows of a scan tile: a fit whose strata all fit one tile is laid
                                  // out so that every scan tile starts with a stratum head

// FitState.flags
enum : int {
    kHaveFree = 1,   // the non-degenerate columns have been chosen
    kFrozen = 2,     // the Cholesky factor is kept; only the FP64 score is recomputed
    kDone = 4,       // status is final
};

// Written by the kernels, read back by the host after every iteration.
struct alignas(16) FitState {
    double obj_eval;    // objective at the current beta (rows kernel)
    double obj;         // objective at the last accepted point
    double obj_prev;    // objective where the last accepted step started
    double last_step;   // max |step| of the last accepted step
    double kkt;         // max |score| over the free columns at the last evaluation (with l1 weights:
                        // the largest violation of the l1 optimality conditions there)
    int iters;          // accepted Newton steps
    int evals;          // evaluations (accepted steps + halvings)
    int halvings;       // consecutive halvings of the current step
    int flags;
    int status;         // COX_OK / COX_NOT_CONVERGED / COX_ENUMERIC once kDone
    unsigned range;     // set when an event's risk-set sum left the FP64 normal range
    int n_pinned;       // columns held at zero
    int pad_;
};

// Everything a kernel needs to know about one resident fit (device pointers).
struct FitDesc {
    double *x;              // [p][ld] FP64, canonical rows, padding rows zero
    const double *xs;       // device-resident request: the caller's X (column-major, leading dimension ldxs),
    const int32_t *src;     //   gathered into x at admission: row r of x is row src[r] of xs (-1: padding);
    int64_t ldxs;           //   xs = nullptr when X came up with the request's image
    float *xf;              // [p][ld] FP32 copy for the contraction
    const uint32_t *meta;   // [ld] row words (padding rows: head | pad)
    const int32_t *gidx;    // [ld] event-group index at group ends, else -1
    double *eta, *w, *zq, *hz, *b;   // [ld] row vectors (zq = (d/S0)/sqrt(d) at group ends, b = w Lambda)
    float *bf;              // [ld] b rounded to FP32: the contraction's weights
    float *z;               // [p][ldz] sqrt(d_g) xbar_g
    double *beta, *prev, *grad, *diag1, *diag2;   // [p]
    uint8_t *free_col;      // [p]
    double *L;              // [p][p] information matrix (info kernel), then its Cholesky factor (row-major, lower)
    float *part;            // [(nxr + nzr) * npairs][32 * 32] contraction partials
    double *tilemax;        // [ntile]
    double *tpart;          // [ntc][2] per scan tile: objective part, range flag
    double *cpart;          // [ntc][p][3] per scan tile and column: score, the two diagonal parts
    FitState *st;
    FitState *hst;          // host-mapped mirror of *st, written by the step kernel every iteration
    double *hbeta;          // host-mapped [p]: the estimate, written when the fit is final
    int64_t n, ld, ldz;
    int64_t tile;           // rows per scan tile (ld = ntc * tile)
    int ntc;                // scan tiles
    int p, G;               // columns, event groups
    int nxr, nzr;           // K ranges of the two products (nzr = 0 without events)
    int xrange, zrange;     // rows of X, event groups of Z per K range (multiples of 256)
    int npairs, ntile;      // tile pairs of the upper triangle; X beta work items
    const double *gam;      // [p] l1 weights (0 for unpenalised columns); nullptr: an unpenalised fit
    const double *beta0;    // [p] start point; nullptr: zeros
    double tol;
    int max_iter;
    int freeze;             // 1: keep the factor (with l1: the information matrix) once steps are small
};

static_assert(sizeof(FitDesc) % 8 == 0, "descriptors are copied in 8-byte words");

// Launchers (return a hipError_t value).  Work-item arrays are device memory.
// admit: `joining` holds the descriptors of the fits that join (copied to
// fits[slots[k]] by the kernel); items are (k, 256-row tile).
int launch_admit(FitDesc *fits, const FitDesc *joining, const int *slots, const int2 *items, int nitems,
                 hipStream_t s);
int launch_eta(const FitDesc *fits, const int2 *items, int nitems, hipStream_t s);
int launch_rows(const FitDesc *fits, const int2 *items, int nitems, hipStream_t s);
int launch_cols(const FitDesc *fits, const int2 *items, int nitems, hipStream_t s);
// syrk: counts[0] per-pair items (fit, tile pair, K range, product), then items (fit, 0, K range,
// product) grouped by the fit's tile count, counts[t] of fits with t tiles (host array of 5);
// both forms give the same partials
int launch_syrk(const FitDesc *fits, const int4 *items, const int *counts, hipStream_t s);
int launch_info(const FitDesc *fits, const int2 *items, int nitems, hipStream_t s);
int launch_step(const FitDesc *fits, const int *slots, int nslots, int max_p, hipStream_t s);

// Persistent rounds: one cooperative launch runs up to max_rounds iterations of every fit in
// the lists, the phases separated by grid-wide barriers; it ends early when every fit has
// finished or when the host writes a nonzero hold word.  Results equal those of the
// separate launches above, bit for bit.
constexpr int kRoundThreads = 512;   // threads of a workgroup of the round kernel
constexpr int kRoundMaxGrid = 2048;

struct RoundWork {
    const FitDesc *fits;
    const int2 *eta, *rows, *cols;   // work items as for the separate launches
    const int4 *syrk;                // items of the fits not frozen when the launch starts
    const int2 *info;
    const int *slots;                // the fits of the launch
    int ne, nr, nc, ns, ni, nf;
    int syrk_per_pair;               // 1: syrk items are per tile pair (light rounds), else per fit and K range
    int max_rounds;
    int max_p;                       // largest p among the fits (sizes the step's LDS)
    const uint32_t *hold;            // host-mapped: nonzero asks the launch to end after the current round
    void *ctl;                       // device, round_ctl_bytes(), cleared before every launch
    uint64_t *hout;                  // host-mapped [8]: rounds completed; 1 if a bounded wait timed out;
                                     // clock ticks (100 MHz) of the six phases, by workgroup 0
};

size_t round_ctl_bytes();
// Workgroups of a round launch for fits of at most max_p columns (all resident at once).
int round_grid(int max_p, int *grid);
int launch_rounds(const RoundWork &w, int grid, hipStream_t s);

}  // namespace serve
}  // namespace coxmi
