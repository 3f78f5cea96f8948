// newton.h -- interface of the full evaluation (newton.hip) and the
// information contraction and Cholesky solve (contraction.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace coxmi {

// Columns of the FP8 contraction (up to 800 every workgroup stages all p rows, beyond that
// blocks of tile pairs stage only their own rows): the Newton path's limit.
constexpr int64_t kMaxFp8P = 4096;

// ------------------------------------------------------------------ full evaluation (newton.hip)

enum ZType { kZF64 = 0, kZF32 = 1, kZBF16 = 2 };

// Buffers and sizes of one full evaluation (device pointers).
struct FullEvalArgs {
    const double *x = nullptr;        // [p][ld]
    const uint32_t *meta = nullptr;   // [ld]
    const int32_t *gidx = nullptr;    // [ld] index of the event group ending at the row, else -1
    const double *beta = nullptr;     // [p]
    int64_t ld = 0;
    int p = 0;
    int max_blocks = 0;               // capacity of blockbuf
    // row vectors [ld]: X beta, its running maximum m within the stratum, alpha and
    // u = exp(eta - m) (see affscan.hpp), S0' = S0 exp(-m), h' = d / S0', the reverse
    // recurrence R (w Lambda = u R), b = w Lambda, zq = h' / sqrt(d)
    double *eta = nullptr, *m = nullptr, *alpha = nullptr, *w = nullptr, *s0 = nullptr, *h = nullptr;
    double *lam = nullptr, *b = nullptr, *zq = nullptr;
    double *blockbuf = nullptr;       // [max_blocks]
    // column pass: tiles of `tile` rows (ld = ntiles * tile)
    int64_t tile = 0;
    int ntiles = 0;
    const uint8_t *tile_carry = nullptr;   // [ntiles] 1: the tile's first row continues a stratum
    const int32_t *lasthead = nullptr;     // [ntiles] row of the tile's last stratum head, -1 if none
    const int32_t *agg_tiles = nullptr;    // [n_agg] tiles whose successor needs a carry
    int n_agg = 0;
    double *agg = nullptr;                 // [ntiles][p][2]: map S -> A S + B of the tile's tail rows
    double *carry = nullptr;               // [ntiles][p]
    double *colpart = nullptr;             // [ntiles][p][3]
    double *grad = nullptr, *diag1 = nullptr, *diag2 = nullptr;   // [p] each
    double *scal = nullptr;           // [0] shift c, [1] objective
    unsigned *flags = nullptr;        // bit 0: a risk-set sum left the FP64 normal range
    int ztype = kZF64;
    void *z = nullptr;                // [p][ldz] sqrt(d_g) xbar_g / zscale_j, event groups in order
    int64_t ldz = 0;
    const float *zscale = nullptr;    // [p] power-of-two column scales (NULL for FP64)
    bool want_xbar = true;            // form xbar, Z and the second diagonal part
    void *scan_scratch = nullptr;     // sync scratch of the row scans
    size_t scan_scratch_bytes = 0;
    // Efron's tie correction: row vectors [ld] E0' (the group's own event weights, relative to
    // exp(m)), k', and the Cholesky factor (zq = l11, l21, l22) of sum_l (1, -a_l)(1, -a_l)' / A_l^2;
    // the multi-event groups (d >= 2) as lists of their event rows (see FullEvalArgs users)
    bool efron = false;
    double *e0 = nullptr, *kq = nullptr, *zq2 = nullptr, *zq3 = nullptr;
    const int32_t *gidx2 = nullptr, *gend = nullptr;
    const int32_t *me_ptr = nullptr, *me_row = nullptr, *me_end = nullptr;
    double *me_w = nullptr, *s1me = nullptr, *epart = nullptr;
    int64_t n_groups = 0, n_multi = 0, n_me_rows = 0;
    int eblocks = 0;
};

// Objective, gradient and the two parts of the Hessian diagonal at beta,
// plus the scaled xbar matrix for the information contraction.  Asynchronous.
int full_eval_launch(const FullEvalArgs &A, hipStream_t stream);

// Inclusive segmented +scan over n rows (n a multiple of tile, tile a multiple
// of 256) with the head flags of meta (reverse: from the last row backwards,
// segments starting at each stratum's last row).  Three launches.
int rowscan(const double *a, const uint32_t *meta, double *out, int64_t n, int64_t tile, bool reverse,
            void *scratch, size_t scratch_bytes, hipStream_t stream);
size_t rowscan_scratch_bytes(int ntiles);

// ------------------------------------------------------------------ contraction (contraction.hip)

// Bytes of the split partials of a p x p symmetric product (FP64 tiles; BF16 tiles).
size_t syrk_partial_bytes(int p, int splits);
size_t syrk_bf16_partial_bytes(int p, int splits);

// K splits of the contractions: X' diag(b) X and Z'Z, FP64 and BF16.
constexpr int kSplitsXF64 = 128, kSplitsZF64 = 128, kSplitsXBF16 = 256, kSplitsZBF16 = 256;
// C (+)= sign * sum_k c_k u_k u_k' in FP64 (u: [p][ldu]; c NULL means 1).  `part` must hold
// syrk_partial_bytes(p, 2 * splits) for p <= 256, where the matrix cores take 2 * splits K slices
// (syrk_partial_bytes(p, splits) beyond).
int syrk_f64(const double *u, int64_t ldu, int p, const double *c, int64_t K, int splits, double *part,
             double sign, int accumulate, double *C, hipStream_t stream);
// BF16 copy of X with power-of-two column scales (zscale receives the same scales).
int make_bf16_copy(const double *x, int64_t ld, int p, void *xlp, float *xscale, float *zscale, hipStream_t stream);
// C (+)= sign * scale_i scale_j sum_k c_k u_ik u_jk with BF16 u on the matrix cores (FP32 accumulate).
// `part` must hold syrk_bf16_partial_bytes(p, 2 * splits): up to 256 columns the K range is cut
// into 2 * splits slices (two workgroups per compute unit).
int syrk_bf16(const uint16_t *u, int64_t ldu, int p, const float *scale, const double *c, int64_t K, int splits,
              double *part, double sign, int accumulate, double *C, hipStream_t stream);
// Bytes of the blocked e4m3 copy of an ld x p matrix (make_fp8_copy, syrk_fp8).
size_t fp8_copy_bytes(int64_t ld, int p);
// e4m3 copy of X with power-of-two column scales (|x / s| <= 224), in blocks of 64 rows
// (each block: the 64 bytes of every column, p rounded up to 32, in turn; ld a multiple of
// 64); zscale gets the BF16 scales.
int make_fp8_copy(const double *x, int64_t ld, int p, uint8_t *x8, float *xscale, float *zscale, hipStream_t stream);
// C (+)= sign * scale_i scale_j sum_k c_k u_ik u_jk with e4m3 u and sqrt(c) on both operands
// (blockmax: 256 doubles of scratch; wsc: 1 double receiving the weight scale).
int syrk_fp8(const uint8_t *u, int64_t ldu, int p, const float *scale, const double *c, int64_t K, int splits,
             double *part, double *blockmax, double *wsc, double sign, int accumulate, double *C, hipStream_t stream);
constexpr int kSplitsXFP8 = 256;
// Factor A (unless factored) and solve dx = -A^{-1} g on the free columns.
int chol_solve(double *A, int p, const double *g, const uint8_t *free_col, int factored, double *dx, int *status,
               hipStream_t stream);

// Proximal Newton's model solve on the device (one wave): D minimising
// g'D + D'HD/2 + sum_j gam_j |beta_j + D_j| by cyclic coordinate descent with soft thresholding,
// free columns only (H: p x p symmetric; g, beta, gam: p; D: p out; sweeps: 1 int out).
// Stops after a sweep whose largest change is <= tol, or after max_sweeps.  p <= 4096.
int prox_model_solve(const double *H, int p, const double *g, const double *beta, const double *gam,
                     const uint8_t *free_col, double tol, int max_sweeps, double *D, int *sweeps, hipStream_t stream);

}  // namespace coxmi
