// resample.hip -- device side of cox_init_resample and cox_init_intervals: a
// resampled data set (row multiplicities, e.g. the training rows of a
// cross-validation fold or a bootstrap sample) or an interval-stratified one
// (Secs. 2.2-2.3) is built from a handle's device-resident X by a gather,
// without sending X over PCIe again.
#include "internal.h"
#include "resample.h"

namespace coxmi {

namespace {

constexpr int kGatherBlock = 256;
constexpr int kGatherRows = 4;     // rows per thread
constexpr int kGatherCols = 8;     // columns per workgroup (the source index is loaded once for them)

// x_out[j][r] = src[r] >= 0 ? x_in[cs(j)][src[r]] : 0 for r < ld_out, j < p, where
// cs(j) = col_src[j] (identity when col_src is null); with col_int and rint given, a
// column with col_int[j] >= 0 is also zero on rows whose rint[r] differs (a step
// coefficient's column outside its interval).
// Grid: (ceil(ld_out / (kGatherBlock * kGatherRows)), ceil(p / kGatherCols)).
__global__ __launch_bounds__(kGatherBlock) void gather_rows_kernel(const double *__restrict__ x_in, int64_t ld_in,
                                                                   const int32_t *__restrict__ src,
                                                                   const int32_t *__restrict__ rint,
                                                                   const int32_t *__restrict__ col_src,
                                                                   const int32_t *__restrict__ col_int,
                                                                   double *__restrict__ x_out, int64_t ld_out, int p)
{
    const int64_t r0 = (int64_t)blockIdx.x * (kGatherBlock * kGatherRows) + threadIdx.x;
    const int j0 = blockIdx.y * kGatherCols;
    int32_t s[kGatherRows], ki[kGatherRows];
#pragma unroll
    for (int k = 0; k < kGatherRows; ++k) {
        const int64_t r = r0 + (int64_t)k * kGatherBlock;
        s[k] = r < ld_out ? src[r] : -1;
        ki[k] = (rint && r < ld_out) ? rint[r] : -1;
    }
#pragma unroll
    for (int c = 0; c < kGatherCols; ++c) {
        const int j = j0 + c;
        if (j >= p) break;
        const int js = col_src ? col_src[j] : j;
        const int jk = col_int ? col_int[j] : -1;
        const double *xi = x_in + (int64_t)js * ld_in;
        double *xo = x_out + (int64_t)j * ld_out;
#pragma unroll
        for (int k = 0; k < kGatherRows; ++k) {
            const int64_t r = r0 + (int64_t)k * kGatherBlock;
            const bool live = s[k] >= 0 && (jk < 0 || jk == ki[k]);
            if (r < ld_out) xo[r] = live ? xi[s[k]] : 0.0;
        }
    }
}

constexpr int kQBlock = kEventSumThreads;

// q[j] = sum over rows with the event bit of x[j][r], one workgroup per column;
// each thread sums a fixed stride of rows and the workgroup folds the thread
// sums in a fixed tree, so the result does not depend on timing.
__global__ __launch_bounds__(kQBlock) void event_sums_kernel(const double *__restrict__ x, int64_t ld,
                                                             const uint32_t *__restrict__ meta, double *__restrict__ q)
{
    __shared__ double s[kQBlock];
    const int j = blockIdx.x;
    const double *xj = x + (int64_t)j * ld;
    double acc = 0.0;
    for (int64_t r = threadIdx.x; r < ld; r += kQBlock)
        if (meta[r] & kEventBit) acc += xj[r];
    s[threadIdx.x] = acc;
    __syncthreads();
#pragma unroll
    for (int w = kQBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) q[j] = s[0];
}

// Indicator columns: child unit u of column j (ipt_out bits, unit of us_out bytes) takes
// bit i from the parent's row src[u * ipt_out + i] (bit (s % ipt_in) of the parent's unit
// s / ipt_in, units of us_in bytes, little-endian).  Grid: (ceil(ldb_out / 256), p).
// With rint / col_src / col_int (device, may be NULL), column j takes the parent's column
// col_src[j] and, when col_int[j] >= 0, only the rows whose rint equals it (a step coefficient).
__global__ __launch_bounds__(256) void gather_bits_kernel(const uint8_t *__restrict__ b_in, int64_t ldb_in, int ipt_in,
                                                          int us_in, const int32_t *__restrict__ src,
                                                          const int32_t *__restrict__ rint,
                                                          const int32_t *__restrict__ col_src,
                                                          const int32_t *__restrict__ col_int,
                                                          uint8_t *__restrict__ b_out, int64_t ldb_out, int ipt_out,
                                                          int us_out)
{
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (u >= ldb_out) return;
    const int64_t j = blockIdx.y;
    const int64_t js = col_src ? col_src[j] : j;
    const int jk = col_int ? col_int[j] : -1;
    uint32_t v = 0u;
    for (int i = 0; i < ipt_out; ++i) {
        const int64_t r = u * ipt_out + i;
        const int32_t s = src[r];
        if (s < 0) continue;
        if (jk >= 0 && rint[r] != jk) continue;
        const int bit = s % ipt_in;
        const uint8_t byte = b_in[(js * ldb_in + s / ipt_in) * us_in + bit / 8];
        v |= (uint32_t)((byte >> (bit % 8)) & 1u) << i;
    }
    uint8_t *o = b_out + (j * ldb_out + u) * us_out;
    o[0] = (uint8_t)(v & 0xffu);
    if (us_out == 2) o[1] = (uint8_t)(v >> 8);
}

// q[j] = number of rows with the event bit whose indicator bit is set (fixed-order sums).
__global__ __launch_bounds__(kQBlock) void event_sums_bits_kernel(const uint8_t *__restrict__ bits, int64_t ldb,
                                                                  int ipt, int us, const uint32_t *__restrict__ meta,
                                                                  double *__restrict__ q)
{
    __shared__ double s[kQBlock];
    const int64_t j = blockIdx.x;
    const int64_t ld = ldb * ipt;
    double acc = 0.0;
    for (int64_t r = threadIdx.x; r < ld; r += kQBlock) {
        if (!(meta[r] & kEventBit)) continue;
        const int bit = (int)(r % ipt);
        const uint8_t byte = bits[(j * ldb + r / ipt) * us + bit / 8];
        if ((byte >> (bit % 8)) & 1u) acc += 1.0;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
#pragma unroll
    for (int w = kQBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) q[j] = s[0];
}

}  // namespace

int launch_gather_rows(const double *x_in, int64_t ld_in, const int32_t *src, const int32_t *rint,
                       const int32_t *col_src, const int32_t *col_int, double *x_out, int64_t ld_out, int p,
                       hipStream_t stream)
{
    if (ld_out <= 0 || p <= 0) return (int)hipSuccess;
    const int64_t per = (int64_t)kGatherBlock * kGatherRows;
    const dim3 grid((unsigned)((ld_out + per - 1) / per), (unsigned)((p + kGatherCols - 1) / kGatherCols));
    hipLaunchKernelGGL(gather_rows_kernel, grid, dim3(kGatherBlock), 0, stream, x_in, ld_in, src, rint, col_src,
                       col_int, x_out, ld_out, p);
    return (int)hipGetLastError();
}

int launch_gather_bits(const void *b_in, int64_t ldb_in, int ipt_in, const int32_t *src, const int32_t *rint,
                       const int32_t *col_src, const int32_t *col_int, void *b_out, int64_t ldb_out, int ipt_out, int p,
                       hipStream_t stream)
{
    if (ldb_out <= 0 || p <= 0) return (int)hipSuccess;
    const dim3 grid((unsigned)((ldb_out + 255) / 256), (unsigned)p);
    hipLaunchKernelGGL(gather_bits_kernel, grid, dim3(256), 0, stream, static_cast<const uint8_t *>(b_in), ldb_in,
                       ipt_in, ipt_in > 8 ? 2 : 1, src, rint, col_src, col_int, static_cast<uint8_t *>(b_out), ldb_out,
                       ipt_out, ipt_out > 8 ? 2 : 1);
    return (int)hipGetLastError();
}

int launch_event_sums_bits(const void *bits, int64_t ldb, int ipt, const uint32_t *meta, double *q, int p,
                           hipStream_t stream)
{
    if (p <= 0) return (int)hipSuccess;
    hipLaunchKernelGGL(event_sums_bits_kernel, dim3((unsigned)p), dim3(kQBlock), 0, stream,
                       static_cast<const uint8_t *>(bits), ldb, ipt, ipt > 8 ? 2 : 1, meta, q);
    return (int)hipGetLastError();
}

int launch_event_sums(const double *x, int64_t ld, const uint32_t *meta, double *q, int p, hipStream_t stream)
{
    if (p <= 0) return (int)hipSuccess;
    hipLaunchKernelGGL(event_sums_kernel, dim3((unsigned)p), dim3(kQBlock), 0, stream, x, ld, meta, q);
    return (int)hipGetLastError();
}

}  // namespace coxmi
