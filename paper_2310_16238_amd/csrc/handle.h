// handle.h -- the library-owned state behind a cox_handle (private to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "coxmi.h"
#include "internal.h"

// Device buffers of the full-evaluation / Newton path, allocated on first use.
struct NewtonState {
    bool ready = false;
    int max_blocks = 0;
    int64_t tile = 0;              // rows per column-pass tile
    int ntiles = 0, n_agg = 0;
    int64_t n_groups = 0, ldz = 0;
    int32_t *gidx = nullptr;       // [ld]
    double *rows = nullptr;        // 9 x [ld]: eta, u, s0', h', R, alpha, b, zq, m
    double *blockbuf = nullptr;    // [max_blocks]
    uint8_t *tile_carry = nullptr; // [ntiles]
    int32_t *lasthead = nullptr;   // [ntiles]
    int32_t *agg_tiles = nullptr;  // [n_agg]
    double *agg = nullptr;         // [ntiles][p][2]
    double *carry = nullptr;       // [ntiles][p]
    double *colpart = nullptr;     // [ntiles][p][3]
    double *vec = nullptr;         // beta, grad, diag1, diag2, dx (p each), scal (8)
    double *hvec = nullptr;        // pinned host mirror of vec, then flags and status (one double each)
    unsigned *flags = nullptr;
    int *status = nullptr;
    uint8_t *free_col = nullptr;   // [p]
    void *z = nullptr;             // [p][ldz] in the contraction type
    float *zscale = nullptr;       // [p]
    void *xlp = nullptr;           // [p][ld] low-precision copy of X (BF16 or e4m3)
    double *wscratch = nullptr;    // FP8: 256 block maxima of the weights, then the weight scale
    float *xscale = nullptr;       // [p]
    double *syrk_part = nullptr;   // split partials of the contraction
    size_t syrk_part_bytes = 0;
    double *info = nullptr;        // [p][p] information matrix, then its Cholesky factor
    void *scan_scratch = nullptr;
    size_t scan_scratch_bytes = 0;
    hipEvent_t ev[6] = {};         // around evaluation, contraction, solve
    // Efron's tie correction (see newton.hip): groups with two or more events get a second row of Z
    bool efron = false;
    int64_t n_multi = 0;           // tie groups with >= 2 events
    int64_t n_zrows = 0;           // rows of Z in use: n_groups (+ n_multi with Efron)
    int32_t *gidx2 = nullptr;      // [ld] index of the multi-event group ending at the row, else -1
    int32_t *gend = nullptr;       // [ld] end row of an event row's tie group, else -1
    int32_t *me_ptr = nullptr;     // [n_multi + 1] event rows of each multi-event group (me_row ranges)
    int32_t *me_row = nullptr;     // [me_ptr[n_multi]]
    int32_t *me_end = nullptr;     // [n_multi] end row of each multi-event group
    double *me_w = nullptr;        // [me_ptr[n_multi]] exp(eta_r - m_end) of those rows
    double *s1me = nullptr;        // [n_multi][p] S1' at the multi-event group ends
    double *erows = nullptr;       // 4 x [ld]: E0', k', l21, l22 at event-group ends
    double *epart = nullptr;       // [p][eblocks] diagonal parts of the multi-event groups
    int eblocks = 0;
    double *prox = nullptr;        // proximal Newton: g, beta, gamma, D (p each), then the sweep count
};

struct cox_handle {
    int64_t n = 0, p = 0;
    int device = 0;
    coxmi::LaunchShape shape;
    hipStream_t stream = nullptr;
    double *d_x = nullptr;         // dense X [p][ld]; NULL for a handle on indicator X
    void *d_xbits = nullptr;       // indicator X: [p][ldb] units of ipt bits (uint8, uint16 for ipt 16)
    int64_t ldb = 0;
    double *d_xvals = nullptr;     // sparse X (cox_init_sparse): the values of the rows d_xbits marks
    int64_t *d_xvoff = nullptr;    // [p] start of each column's values
    int32_t *d_woff = nullptr;     // [p][ld / (64 ipt)] values of the column before each wave's rows
    uint32_t *d_meta = nullptr;
    double *d_vec = nullptr;       // q, gamma, beta, g1, g2, m2 (p each), result (8), exp table (64)
    void *d_sync = nullptr;
    double *d_trust = nullptr;     // [grid][p] trust half-widths of the persistent kernel
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    float last_kernel_ms = 0.0f;
    cox_profile prof{};
    std::vector<int64_t> perm;     // canonical row -> original row
    std::vector<uint32_t> meta;    // canonical row words
    std::vector<int64_t> pos;      // canonical row -> row of the device layout
    std::vector<double> gamma;
    std::vector<int64_t> subject;  // cox_init_intervals: subject (row of the parent) of each row; else empty
    cox_options opt{};
    std::string err;
    NewtonState nt;

    double *q() const { return d_vec; }
    double *gam() const { return d_vec + p; }
    double *beta() const { return d_vec + 2 * p; }
    double *g1() const { return d_vec + 3 * p; }
    double *g2() const { return d_vec + 4 * p; }
    double *m2() const { return d_vec + 5 * p; }
    double *result() const { return d_vec + 6 * p; }
    double *exp_tab() const { return d_vec + 6 * p + coxmi::kResultSlots; }
};

int handle_fail(cox_handle *h, int code, const std::string &msg);
int handle_hip_fail(cox_handle *h, hipError_t e, const char *what);
void newton_free(cox_handle *h);
int newton_fit(cox_handle *h, const double *beta0, double *beta_out, cox_fit_info *info);
