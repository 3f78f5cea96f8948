// internal.h -- interface between the C ABI (coxmi.cpp) and the kernels (ccd_kernel.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace coxmi {

// Row word in canonical order (see cox_layout in include/coxmi.h).
constexpr uint32_t kHeadBit = 0x80000000u;
constexpr uint32_t kEventBit = 0x40000000u;
constexpr uint32_t kPadBit = 0x20000000u;     // device layout only: a padding row
constexpr uint32_t kCountMask = 0x1fffffffu;

constexpr int kThreads = 512;           // threads per workgroup of the CCD kernel
constexpr int kMaxGroups = 256;         // workgroups of one persistent launch (one per compute unit)

enum KernelMode { kModeFit = 0, kModeEval = 1 };

// Resident launch shape of a data set: `grid` workgroups of kThreads threads,
// each thread owning `ipt` consecutive rows; ld = grid * kThreads * ipt rows.
struct LaunchShape {
    int ipt = 0;
    int grid = 0;
    int64_t ld = 0;
};

// Workgroups that fit on the device at once for the persistent kernel with
// `ipt` rows per thread (0 if it does not fit); at most one per compute unit.
int max_resident_groups(int ipt, int p, int *groups, std::string &err);

// Arguments of one persistent launch (device pointers unless noted).
struct CcdLaunch {
    const double *x = nullptr;       // [p][ld] canonical rows, padding rows zero
    const uint32_t *meta = nullptr;  // [ld]
    const double *q = nullptr;       // [p] delta' X_j
    const double *gamma = nullptr;   // [p] l1 weights
    const double *exp_tab = nullptr; // [64] 2^(j/64)
    int64_t n = 0;                   // real rows (rows n..ld-1 are padding)
    int p = 0;
    int mode = kModeFit;
    int j0 = 0, j1 = 0;              // evaluation: columns [j0, j1)
    int max_sweeps = 0;
    double tol = 0.0;
    double *beta = nullptr;          // [p] in: start point; out (fit): estimate
    double *g1 = nullptr;            // [p] g' of each coordinate's last evaluation
    double *g2 = nullptr;            // [p] g''
    double *m2 = nullptr;            // [p] delta'(S[N2]/S[D])
    double *result = nullptr;        // [kResultSlots] see ResultSlot
    void *agg = nullptr;             // [grid][3] packets: tile aggregates for the look-back
    void *part = nullptr;            // [grid][5] packets: per-workgroup partial sums
    void *res = nullptr;             // [2] packets: the step broadcast by workgroup 0
    void *ctl = nullptr;             // control words
};

// Bytes of the per-launch synchronisation scratch for `grid` workgroups.
size_t sync_scratch_bytes(int grid);
// Carve the scratch block into the CcdLaunch fields (agg, stat1, part, stat2, ctl).
void carve_sync_scratch(void *base, int grid, CcdLaunch &L);


// Launch the persistent CCD / evaluation kernel; returns a hipError_t value.
// Zeroes the synchronisation words first; records ev0/ev1 around the kernel if non-null.
int launch_ccd(const LaunchShape &shape, const CcdLaunch &L, hipStream_t stream,
               hipEvent_t ev0, hipEvent_t ev1);

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
    int splits = 1;                   // row splits of the X' products
    int max_blocks = 0;               // capacity of blockbuf
    double *eta = nullptr, *w = nullptr, *s0 = nullptr, *h = nullptr, *lam = nullptr;  // [ld] each
    double *a = nullptr, *b = nullptr;                                                // [ld] each
    double *blockbuf = nullptr;       // [max_blocks]
    double *xtpart = nullptr;         // [splits][p][2]
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
};

// Objective, gradient and the two parts of the Hessian diagonal at beta,
// plus the scaled xbar matrix for the information contraction.  Asynchronous.
int full_eval_launch(const FullEvalArgs &A, hipStream_t stream);

// Inclusive segmented +scan over rows with the head flags of meta (reverse:
// from the last row backwards, segments starting at each stratum's last row).
int rowscan(const double *a, const uint32_t *meta, double *out, int64_t n, bool reverse, void *scratch,
            size_t scratch_bytes, hipStream_t stream);

// ------------------------------------------------------------------ contraction (contraction.hip)

// Bytes of the split partials of a p x p symmetric product.
size_t syrk_partial_bytes(int p, int splits);
// C (+)= sign * sum_k c_k u_k u_k' in FP64 (u: [p][ldu]; c NULL means 1).
int syrk_f64(const double *u, int64_t ldu, int p, const double *c, int64_t K, int splits, double *part,
             double sign, int accumulate, double *C, hipStream_t stream);
// BF16 copy of X with power-of-two column scales (zscale receives the same scales).
int make_bf16_copy(const double *x, int64_t ld, int p, void *xlp, float *xscale, float *zscale, hipStream_t stream);
// C (+)= sign * scale_i scale_j sum_k c_k u_ik u_jk with BF16 u on the matrix cores (FP32 accumulate).
int syrk_bf16(const uint16_t *u, int64_t ldu, int p, const float *scale, const double *c, int64_t K, int splits,
              double *part, double sign, int accumulate, double *C, hipStream_t stream);
// Factor A (unless factored) and solve dx = -A^{-1} g on the free columns.
int chol_solve(double *A, int p, const double *g, const uint8_t *free_col, int factored, double *dx, int *status,
               hipStream_t stream);

// Segmented +scan of n doubles on device memory; returns a COX_* code.
int segscan_f64(const double *a, const uint8_t *head, double *b, int64_t n, hipStream_t stream);

// Result slots written by the persistent kernel.
enum ResultSlot {
    kResSweeps = 0, kResLastStep = 1, kResObjective = 2, kResPinned = 3,
    kResConverged = 4, kResNumeric = 5, kResCompleted = 6
};
constexpr int kResultSlots = 8;

}  // namespace coxmi
