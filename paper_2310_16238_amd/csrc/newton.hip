// newton.hip -- full evaluation of the stratified Cox objective, gradient and
// information matrix on gfx950, and the FP64 Cholesky solve of a Newton step.
//
// Exchanging the order of the sums in Eqs. strat_g / strat_h (every event
// group g adds d_g x_r w_r / S0_g for each row r of its risk set) gives, with
// Lambda_r = sum over the event groups g of r's stratum with Y_g <= Y_r of
// d_g / S0_g (a reverse segmented scan of d_g / S0_g):
//   gradient     = X'(w o Lambda - delta)
//   Hessian      = X' diag(w o Lambda) X - sum_g d_g xbar_g xbar_g',  xbar_g = S1_g / S0_g
//   diagonal     = sum_r x_rj^2 w_r Lambda_r - sum_g d_g xbar_gj^2
//   objective    = -delta'eta + sum_g d_g (log S0_g + c)
// where S0_g, S1_g are the forward segmented scans of w and w x at the end of
// group g, w = exp(eta - c).  One pass over X forms eta, one more forms the
// X' products, and one per-column scan forms xbar; the information matrix is
// two symmetric rank-K products (contraction.hip).
//
// Kernels here are ordinary (non-persistent) launches except the row scans,
// which reuse the cooperative single-pass scan with look-back.
#include <hip/hip_bf16.h>
#include <math.h>

#include <type_traits>

#include "internal.h"
#include "segscan.hpp"

namespace coxmi {

namespace {

constexpr int kRowBlock = 256;   // threads of the elementwise and reduction kernels

__device__ __forceinline__ double block_sum(double v, double *red)
{
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) s += red[k];
    __syncthreads();
    return s;
}

__device__ __forceinline__ double block_max(double v, double *red)
{
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = -INFINITY;
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) s = fmax(s, red[k]);
    __syncthreads();
    return s;
}

// eta = X beta over all ld rows; per-block max of eta over real rows.
__global__ __launch_bounds__(kRowBlock) void eta_kernel(const double *x, int64_t ld, int p, const double *beta,
                                                        const uint32_t *meta, double *eta, double *blockmax)
{
    __shared__ double red[kRowBlock / kWave];
    const int64_t r = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    double e = 0.0, mx = -INFINITY;
    if (r < ld) {
        for (int j = 0; j < p; ++j) {
            const double bj = beta[j];
            if (bj != 0.0) e = fma(x[(int64_t)j * ld + r], bj, e);
        }
        eta[r] = e;
        if (!(meta[r] & kPadBit)) mx = e;
    }
    mx = block_max(mx, red);
    if (threadIdx.x == 0) blockmax[blockIdx.x] = mx;
}

// Single workgroup: scal[0] = max of blockmax (the shift c), fixed order.
__global__ __launch_bounds__(kRowBlock) void max_kernel(const double *blockmax, int nb, double *scal)
{
    __shared__ double red[kRowBlock / kWave];
    double mx = -INFINITY;
    for (int i = threadIdx.x; i < nb; i += kRowBlock) mx = fmax(mx, blockmax[i]);
    mx = block_max(mx, red);
    if (threadIdx.x == 0) scal[0] = mx;
}

// w = exp(eta - c)
__global__ __launch_bounds__(kRowBlock) void weight_kernel(const double *eta, const double *scal, int64_t ld,
                                                           double *w)
{
    const int64_t r = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (r < ld) w[r] = exp(eta[r] - scal[0]);
}

// At event-group ends: h = d / S0 and the per-block objective part
// d (log S0 + c); at event rows: -eta.  Range check of S0 as in the CCD kernel.
__global__ __launch_bounds__(kRowBlock) void hazard_kernel(const double *s0, const double *eta, const uint32_t *meta,
                                                           const double *scal, int64_t ld, double *h,
                                                           double *blockobj, unsigned *flags)
{
    __shared__ double red[kRowBlock / kWave];
    const int64_t r = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    double obj = 0.0;
    if (r < ld) {
        const uint32_t m = meta[r];
        const uint32_t d = m & kCountMask;
        double hv = 0.0;
        if (d != 0u) {
            const double s = s0[r];
            if (!(s >= 1e-300) || !(s <= 1e300)) atomicOr(flags, 1u);
            hv = (double)d / s;
            obj += (double)d * (log(s) + scal[0]);
        }
        if (m & kEventBit) obj -= eta[r];
        h[r] = hv;
    }
    obj = block_sum(obj, red);
    if (threadIdx.x == 0) blockobj[blockIdx.x] = obj;
}

// a = w Lambda - delta, b = w Lambda
__global__ __launch_bounds__(kRowBlock) void rowweight_kernel(const double *w, const double *lam, const uint32_t *meta,
                                                              int64_t ld, double *a, double *b)
{
    const int64_t r = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (r < ld) {
        const double wl = w[r] * lam[r];
        b[r] = wl;
        a[r] = wl - ((meta[r] & kEventBit) ? 1.0 : 0.0);
    }
}

// Split sums over rows: part[(s * p + j) * 2 + {0,1}] = sum over rows of split s
// of x_rj a_r and x_rj^2 b_r.  Grid (p, S).
__global__ __launch_bounds__(kRowBlock) void xt_kernel(const double *x, int64_t ld, int p, const double *a,
                                                       const double *b, int64_t rows_per_split, double *part)
{
    __shared__ double red[kRowBlock / kWave];
    const int j = blockIdx.x, s = blockIdx.y;
    const int64_t r0 = (int64_t)s * rows_per_split;
    const int64_t r1 = r0 + rows_per_split < ld ? r0 + rows_per_split : ld;
    const double *xj = x + (int64_t)j * ld;
    double ga = 0.0, gb = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kRowBlock) {
        const double v = xj[r];
        ga = fma(v, a[r], ga);
        gb = fma(v * v, b[r], gb);
    }
    ga = block_sum(ga, red);
    gb = block_sum(gb, red);
    if (threadIdx.x == 0) {
        part[((int64_t)s * p + j) * 2] = ga;
        part[((int64_t)s * p + j) * 2 + 1] = gb;
    }
}

// Fixed-order sums of the split partials: out_a[j], out_b[j]; also the
// objective (sum of blockobj, by workgroup 0).
__global__ __launch_bounds__(kRowBlock) void xt_reduce_kernel(const double *part, int p, int S, double *out_a,
                                                              double *out_b, const double *blockobj, int nb,
                                                              double *scal)
{
    __shared__ double red[kRowBlock / kWave];
    const int j = blockIdx.x;
    if (j < p) {
        if (threadIdx.x == 0) {
            double sa = 0.0, sb = 0.0;
            for (int s = 0; s < S; ++s) {
                sa += part[((int64_t)s * p + j) * 2];
                sb += part[((int64_t)s * p + j) * 2 + 1];
            }
            out_a[j] = sa;
            out_b[j] = sb;
        }
    } else {
        double o = 0.0;
        for (int i = threadIdx.x; i < nb; i += kRowBlock) o += blockobj[i];
        o = block_sum(o, red);
        if (threadIdx.x == 0) scal[1] = o;
    }
}

template <typename ZT>
__device__ __forceinline__ void store_z(ZT *p, double v, float inv_scale)
{
    if constexpr (std::is_same<ZT, double>::value) *p = v;
    else if constexpr (std::is_same<ZT, float>::value) *p = (float)v * inv_scale;
    else *p = __float2bfloat16((float)v * inv_scale);
}

// Per column j (one workgroup of 1024 threads): forward segmented scan of
// w x_j over the rows, tile by tile with the carry in registers; at each
// event-group end (gidx >= 0): xbar = S1 / S0, diag2_j += d xbar^2, and
// z[j][g] = sqrt(d) xbar in the contraction's storage type.
template <typename ZT>
__global__ __launch_bounds__(1024) void xbar_kernel(const double *x, int64_t ld, const double *w, const double *s0,
                                                    const uint32_t *meta, const int32_t *gidx, int64_t ldz,
                                                    const float *zscale, ZT *z, double *diag2)
{
    constexpr int NW = 1024 / kWave, IPT = 4, TILE = 1024 * IPT;
    __shared__ SegVal<1> wtot[NW];
    __shared__ double red[NW];
    const int j = blockIdx.x, t = threadIdx.x;
    const double *xj = x + (int64_t)j * ld;
    const float zs = zscale ? 1.0f / zscale[j] : 1.0f;
    SegVal<1> carry = seg_identity<1>();
    double d2 = 0.0;
    for (int64_t base = 0; base < ld; base += TILE) {
        SegVal<1> e[IPT];
        SegVal<1> tagg = seg_identity<1>();
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const int64_t r = base + (int64_t)t * IPT + i;
            if (r < ld) {
                e[i].f = meta[r] >> 31;
                e[i].v[0] = w[r] * xj[r];
            } else {
                e[i] = seg_identity<1>();
                e[i].f = 1u;
            }
            tagg = seg_combine(tagg, e[i]);
        }
        SegVal<1> btot;
        SegVal<1> exc = block_exclusive_scan<1, NW>(tagg, wtot, btot);
        SegVal<1> run = seg_combine(carry, exc);
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const int64_t r = base + (int64_t)t * IPT + i;
            run = seg_combine(run, e[i]);
            if (r < ld) {
                const int32_t g = gidx[r];
                if (g >= 0) {
                    const double d = (double)(meta[r] & kCountMask);
                    const double xb = run.v[0] / s0[r];
                    d2 = fma(d * xb, xb, d2);
                    store_z<ZT>(&z[(int64_t)j * ldz + g], sqrt(d) * xb, zs);
                }
            }
        }
        carry = seg_combine(carry, btot);
        __syncthreads();   // wtot is rewritten by the next tile
    }
    // fixed-order workgroup sum of the diag2 parts
    for (int off = 32; off >= 1; off >>= 1) d2 += __shfl_xor(d2, off, kWave);
    if ((t & (kWave - 1)) == 0) red[t / kWave] = d2;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int k = 0; k < NW; ++k) s += red[k];
        diag2[j] = s;
    }
}

// ------------------------------------------------------------------ row scans (forward / reverse)

// Inclusive segmented +scan of `a` over rows 0..n-1 with the head flags of
// `meta`; REV scans from the last row backwards, a segment then starting at
// the last row of each stratum.  Same single-pass cooperative scheme as the
// scan primitive.
template <int IPT, bool REV>
__global__ __launch_bounds__(1024) void rowscan_kernel(const double *a, const uint32_t *meta, double *out, int64_t n,
                                                       Packet *aggp, SyncCtl *ctl)
{
    constexpr int NW = 1024 / kWave;
    __shared__ SegVal<1> s_wtot[NW];
    __shared__ SegVal<1> s_win[kMaxGroups / kWave];
    __shared__ int s_abort;
    const PacketArray agg = packet_array(aggp, sizeof(Packet) * gridDim.x);
    const int b = blockIdx.x, t = threadIdx.x;
    const int64_t tile0 = (int64_t)b * 1024 * IPT;
    const int64_t row0 = tile0 + (int64_t)t * IPT;
    auto head_at = [&](int64_t i) -> uint32_t {   // i in scan order
        if (!REV) return (i == 0 || (meta[i] & kHeadBit)) ? 1u : 0u;
        const int64_t r = n - 1 - i;   // row; a reverse segment starts at a stratum's last row
        return (i == 0 || (meta[r + 1] & kHeadBit)) ? 1u : 0u;
    };
    SegVal<1> e[IPT];
    SegVal<1> tagg = seg_identity<1>();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int64_t k = row0 + i;
        if (k < n) {
            e[i].f = head_at(k);
            e[i].v[0] = a[REV ? n - 1 - k : k];
        } else {
            e[i].f = 1u;
            e[i].v[0] = 0.0;
        }
        tagg = seg_combine(tagg, e[i]);
    }
    if (t == 0) s_abort = 0;
    const uint32_t epoch = 1;
    SegVal<1> btot;
    SegVal<1> exc = block_exclusive_scan<1, NW>(tagg, s_wtot, btot);
    if (t == 0) publish_aggregate<1>(agg, b, btot, epoch);
    const bool tile_head = tile0 >= n || head_at(tile0) != 0u;
    if (!tile_head) {
        SegVal<1> carry;
        if (!look_back<1>(b, epoch, agg, ctl, s_win, &s_abort, carry)) return;
        exc = seg_combine(carry, exc);
    }
    SegVal<1> run = exc;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        run = seg_combine(run, e[i]);
        const int64_t k = row0 + i;
        if (k < n) out[REV ? n - 1 - k : k] = run.v[0];
    }
}

}  // namespace

// ------------------------------------------------------------------ host launchers

int rowscan(const double *a, const uint32_t *meta, double *out, int64_t n, bool reverse, void *scratch,
            size_t scratch_bytes, hipStream_t stream)
{
    int cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -3;
    const int ipts[] = {1, 2, 4, 8, 16};
    int ipt = 0;
    int64_t grid = 0;
    for (int c : ipts) {
        grid = (n + 1024LL * c - 1) / (1024LL * c);
        if (grid <= cus && grid <= kMaxGroups) {
            ipt = c;
            break;
        }
    }
    if (!ipt) return -5;
    const size_t need = 256 + sizeof(Packet) * (size_t)grid;
    if (need > scratch_bytes) return -5;
    SyncCtl *ctl = static_cast<SyncCtl *>(scratch);
    Packet *agg = reinterpret_cast<Packet *>(static_cast<char *>(scratch) + 256);
    hipError_t e = hipMemsetAsync(scratch, 0, need, stream);
    if (e != hipSuccess) return -3;
    void *args[] = {(void *)&a, (void *)&meta, (void *)&out, (void *)&n, (void *)&agg, (void *)&ctl};
    const void *fn = nullptr;
#define COXMI_PICK(I) (reverse ? reinterpret_cast<const void *>(&rowscan_kernel<I, true>) \
                               : reinterpret_cast<const void *>(&rowscan_kernel<I, false>))
    switch (ipt) {
    case 1: fn = COXMI_PICK(1); break;
    case 2: fn = COXMI_PICK(2); break;
    case 4: fn = COXMI_PICK(4); break;
    case 8: fn = COXMI_PICK(8); break;
    default: fn = COXMI_PICK(16); break;
    }
#undef COXMI_PICK
    e = hipLaunchCooperativeKernel(fn, dim3((unsigned)grid), dim3(1024), args, 0, stream);
    return e == hipSuccess ? 0 : -3;
}

int full_eval_launch(const FullEvalArgs &A, hipStream_t stream)
{
    const int64_t ld = A.ld;
    const int nb = (int)((ld + kRowBlock - 1) / kRowBlock);
    if (nb > A.max_blocks) return -5;
    hipError_t e = hipMemsetAsync(A.flags, 0, sizeof(unsigned), stream);
    if (e != hipSuccess) return -3;
    eta_kernel<<<nb, kRowBlock, 0, stream>>>(A.x, ld, A.p, A.beta, A.meta, A.eta, A.blockbuf);
    max_kernel<<<1, kRowBlock, 0, stream>>>(A.blockbuf, nb, A.scal);
    weight_kernel<<<nb, kRowBlock, 0, stream>>>(A.eta, A.scal, ld, A.w);
    int rc = rowscan(A.w, A.meta, A.s0, ld, false, A.scan_scratch, A.scan_scratch_bytes, stream);
    if (rc) return rc;
    hazard_kernel<<<nb, kRowBlock, 0, stream>>>(A.s0, A.eta, A.meta, A.scal, ld, A.h, A.blockbuf, A.flags);
    rc = rowscan(A.h, A.meta, A.lam, ld, true, A.scan_scratch, A.scan_scratch_bytes, stream);
    if (rc) return rc;
    rowweight_kernel<<<nb, kRowBlock, 0, stream>>>(A.w, A.lam, A.meta, ld, A.a, A.b);
    const int64_t rps = (ld + A.splits - 1) / A.splits;
    xt_kernel<<<dim3(A.p, A.splits), kRowBlock, 0, stream>>>(A.x, ld, A.p, A.a, A.b, rps, A.xtpart);
    xt_reduce_kernel<<<A.p + 1, kRowBlock, 0, stream>>>(A.xtpart, A.p, A.splits, A.grad, A.diag1, A.blockbuf, nb,
                                                        A.scal);
    if (!A.want_xbar) return hipGetLastError() == hipSuccess ? 0 : -3;
    switch (A.ztype) {
    case kZF64:
        xbar_kernel<double><<<A.p, 1024, 0, stream>>>(A.x, ld, A.w, A.s0, A.meta, A.gidx, A.ldz, nullptr,
                                                      static_cast<double *>(A.z), A.diag2);
        break;
    case kZF32:
        xbar_kernel<float><<<A.p, 1024, 0, stream>>>(A.x, ld, A.w, A.s0, A.meta, A.gidx, A.ldz, A.zscale,
                                                     static_cast<float *>(A.z), A.diag2);
        break;
    default:
        xbar_kernel<__hip_bfloat16><<<A.p, 1024, 0, stream>>>(A.x, ld, A.w, A.s0, A.meta, A.gidx, A.ldz,
                                                              A.zscale, static_cast<__hip_bfloat16 *>(A.z),
                                                              A.diag2);
        break;
    }
    e = hipGetLastError();
    return e == hipSuccess ? 0 : -3;
}

}  // namespace coxmi
