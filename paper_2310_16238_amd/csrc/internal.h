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
constexpr int kWaveRows = 64;           // threads per wave: a wave owns kWaveRows * ipt consecutive rows
constexpr int kMaxGroups = 256;         // workgroups of one persistent launch (one per compute unit)
constexpr int64_t kMaxCcdP = 12288;     // columns of the persistent kernel (beta in LDS: 96 KB)
constexpr int64_t kMaxNewtonP = 4096;   // columns of the Newton / full-evaluation path

enum KernelMode { kModeFit = 0, kModeEval = 1 };

// Resident launch shape of a data set: `grid` workgroups of kThreads threads,
// each thread owning `ipt` consecutive rows; ld = grid * kThreads * ipt rows.
struct LaunchShape {
    int ipt = 0;
    int grid = 0;
    int64_t ld = 0;
    bool wave = false;   // every stratum lies within one wave's rows (kWaveRows(ipt)): wave-local scans
};

// Workgroups that fit on the device at once for the persistent kernel with
// `ipt` rows per thread (0 if it does not fit); at most one per compute unit.
int max_resident_groups(int ipt, int p, int *groups, std::string &err);

// Arguments of one persistent launch (device pointers unless noted).
struct CcdLaunch {
    const double *x = nullptr;       // [p][ld] canonical rows, padding rows zero (dense X)
    const void *xbits = nullptr;     // indicator X instead: [p][ldb] units of IPT bits (uint8, uint16 for IPT 16)
    int64_t ldb = 0;                 // units per indicator column (grid * threads)
    const double *xvals = nullptr;   // sparse values instead: the nonzeros the bits mark, column by column
    const int64_t *xvoff = nullptr;  // [p] start of column j in xvals
    const int32_t *woff = nullptr;   // [p][nwaves] nonzeros of column j before wave w's first row
    int64_t nwaves = 0;              // waves of the launch (ld / (64 ipt))
    const uint32_t *meta = nullptr;  // [ld]
    const double *q = nullptr;       // [p] delta' X_j
    const double *gamma = nullptr;   // [p] l1 weights
    double *trust = nullptr;         // [grid][p] trust half-widths, one copy per workgroup
    const double *exp_tab = nullptr; // [64] 2^(j/64)
    int64_t n = 0;                   // real rows (rows n..ld-1 are padding)
    int p = 0;
    int mode = kModeFit;
    int efron = 0;                   // 1: Efron's tie correction instead of the plain risk sets
    int wave = 0;                    // 1: the layout is wave-aligned (LaunchShape::wave)
    int j0 = 0, j1 = 0;              // evaluation: columns [j0, j1)
    int max_sweeps = 0;
    double tol = 0.0;
    double *beta = nullptr;          // [p] in: start point; out (fit): estimate
    double *g1 = nullptr;            // [p] g' of each coordinate's last evaluation
    double *g2 = nullptr;            // [p] g''
    double *m2 = nullptr;            // [p] delta'(S[N2]/S[D])
    double *result = nullptr;        // [kResultSlots] see ResultSlot
    void *agg = nullptr;             // [grid][6] packets: tile aggregates for the look-back
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

// Resampled data sets (resample.hip); return hipError_t values.
// x_out[j][r] = src[r] >= 0 ? x_in[col_src[j]][src[r]] : 0 for r < ld_out (device arrays: src
// and rint ld_out entries, col_src and col_int p entries; col_src NULL = identity).  With
// rint and col_int, column j is also zero where col_int[j] >= 0 and rint[r] != col_int[j].
int launch_gather_rows(const double *x_in, int64_t ld_in, const int32_t *src, const int32_t *rint,
                       const int32_t *col_src, const int32_t *col_int, double *x_out, int64_t ld_out, int p,
                       hipStream_t stream);
// q[j] = sum of x[j][r] over the rows whose word has the event bit (fixed-order sums: thread t of
// kEventSumThreads adds rows r = t (mod kEventSumThreads) in increasing r, then a halving tree).
constexpr int kEventSumThreads = 256;
int launch_event_sums(const double *x, int64_t ld, const uint32_t *meta, double *q, int p, hipStream_t stream);

// True when [ptr, ptr + bytes) lies inside one device (or managed) allocation of `device`
// (host code; clears the HIP error state when the pointer is not device memory).
bool device_range_ok(const void *ptr, size_t bytes, int device);

// Segmented +scan of n doubles on device memory; returns a COX_* code.
int segscan_f64(const double *a, const uint8_t *head, double *b, int64_t n, hipStream_t stream);
// The same scan with its synchronisation words in a fixed library-owned device array
// (no allocation); calls that overlap on one device race on that array.
int segscan_f64_noalloc(const double *a, const uint8_t *head, double *b, int64_t n, hipStream_t stream);

// Result slots written by the persistent kernel.
enum ResultSlot {
    kResSweeps = 0, kResLastStep = 1, kResObjective = 2, kResPinned = 3,
    kResConverged = 4, kResNumeric = 5, kResCompleted = 6
};
constexpr int kResultSlots = 8;

}  // namespace coxmi
