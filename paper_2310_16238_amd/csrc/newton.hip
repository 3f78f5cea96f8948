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
// All kernels here are ordinary launches (no cross-workgroup waits).
#include <hip/hip_bf16.h>
#include <math.h>

#include <type_traits>

#include "internal.h"
#include "newton.h"
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
// also zq = (d/S0) / sqrt(d) at group ends: xbar_j sqrt(d) = S1_j zq and
// d xbar_j^2 = (S1_j zq)^2, so the column pass needs no division per column
__global__ __launch_bounds__(kRowBlock) void hazard_kernel(const double *s0, const double *eta, const uint32_t *meta,
                                                           const double *scal, int64_t ld, double *h, double *zq,
                                                           double *blockobj, unsigned *flags)
{
    __shared__ double red[kRowBlock / kWave];
    const int64_t r = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    double obj = 0.0;
    if (r < ld) {
        const uint32_t m = meta[r];
        const uint32_t d = m & kCountMask;
        double hv = 0.0, qv = 0.0;
        if (d != 0u) {
            const double s = s0[r];
            if (!(s >= 1e-300) || !(s <= 1e300)) atomicOr(flags, 1u);
            hv = (double)d / s;
            qv = hv / sqrt((double)d);
            obj += (double)d * (log(s) + scal[0]);
        }
        if (m & kEventBit) obj -= eta[r];
        h[r] = hv;
        zq[r] = qv;
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

template <typename ZT>
__device__ __forceinline__ void store_z(ZT *p, double v, float inv_scale)
{
    if constexpr (std::is_same<ZT, double>::value) *p = v;
    else if constexpr (std::is_same<ZT, float>::value) *p = (float)v * inv_scale;
    else *p = __float2bfloat16((float)v * inv_scale);
}

// ------------------------------------------------------------------ column pass
//
// Rows are cut into tiles of `tile` rows (the persistent kernel's tiles, so in
// the stratum-aligned layout most tiles start with a stratum head).  One wave
// handles one (tile, column): the forward segmented scan of w x_j over the
// tile's rows (S1, carried in from the previous tiles when the tile's first
// row continues a stratum), xbar = S1/S0 at event-group ends with
// z = sqrt(d) xbar and sum d xbar^2, and the tile's parts of x'(w Lambda - delta)
// and (x o x)'(w Lambda).  The carries come from a masked sum per (tile,
// column) -- the rows after the tile's last head -- chained per column.

constexpr int kColWaves = 4, kColIpt = 4, kColChunk = kWave * kColIpt;

__device__ __forceinline__ void load4(const double *p, double *v)
{
    const double2 lo = *reinterpret_cast<const double2 *>(p);
    const double2 hi = *reinterpret_cast<const double2 *>(p + 2);
    v[0] = lo.x;
    v[1] = lo.y;
    v[2] = hi.x;
    v[3] = hi.y;
}

// agg[t][j] = sum of w x_j over the rows of tile t from its last head (or its
// first row) to its end, for the tiles listed in `tiles`.
__global__ __launch_bounds__(kWave * kColWaves) void colagg_kernel(const double *x, int64_t ld, int p, const double *w,
                                                                   int64_t tile, const int32_t *tiles, int ntl,
                                                                   const int32_t *lasthead, double *agg)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int item = __builtin_amdgcn_readfirstlane(blockIdx.x * kColWaves + threadIdx.x / kWave);
    if (item >= ntl * p) return;
    const int t = tiles[item / p], j = item % p;
    const int64_t r1 = (int64_t)(t + 1) * tile;
    const int64_t r0 = lasthead[t] >= 0 ? (int64_t)lasthead[t] : (int64_t)t * tile;
    const double *xj = x + (int64_t)j * ld;
    double s = 0.0;
    for (int64_t r = r0 + lane; r < r1; r += kWave) s = fma(w[r], xj[r], s);
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, kWave);
    if (lane == 0) agg[(int64_t)t * p + j] = s;
}

// carry[t][j] = the S1 running sum entering tile t (for tiles whose first row
// continues a stratum).  One thread per column, tiles in order.
__global__ __launch_bounds__(256) void colcarry_kernel(int p, int ntiles, const uint8_t *tile_carry,
                                                       const int32_t *lasthead, const double *agg, double *carry)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= p) return;
    double c = 0.0;
    for (int t = 0; t < ntiles; ++t) {
        carry[(int64_t)t * p + j] = c;
        if (t + 1 < ntiles && tile_carry[t + 1]) c = (lasthead[t] >= 0 ? 0.0 : c) + agg[(int64_t)t * p + j];
        else c = 0.0;
    }
}

// kColBlock columns per wave: the row vectors (w, b, zq, row words, group
// indices) are loaded once per chunk for all of them.
constexpr int kColBlock = 4;

template <typename ZT, bool XBAR>
__global__ __launch_bounds__(kWave * kColWaves) void colpass_kernel(const double *x, int64_t ld, int p, int64_t tile,
                                                                    int ntiles, const double *w, const double *zq,
                                                                    const double *b, const uint32_t *meta,
                                                                    const int32_t *gidx, const uint8_t *tile_carry,
                                                                    const double *carry, int64_t ldz,
                                                                    const float *zscale, ZT *z, double *part)
{
    constexpr int CB = kColBlock;
    const int lane = threadIdx.x & (kWave - 1);
    // XCD-aware order: workgroups are dealt to the 8 XCDs in turn, so workgroup
    // wg runs on XCD wg % 8; every column group of a tile goes to one XCD, whose
    // L2 then holds that tile's row vectors for all of its columns
    const int per_wg = kColWaves * CB;
    const int cgroups = (p + per_wg - 1) / per_wg;
    const int wg = blockIdx.x, xcd = wg & 7, k = wg >> 3;
    const int t = (k / cgroups) * 8 + xcd;
    const int j0 = __builtin_amdgcn_readfirstlane((k % cgroups) * per_wg + (int)(threadIdx.x / kWave) * CB);
    if (t >= ntiles || j0 >= p) return;   // whole wave; no workgroup barrier below
    const int64_t r_begin = (int64_t)t * tile, r_end = r_begin + tile;
    const double *xc[CB];
    bool live[CB];
    float zs[CB];
    double g[CB], d1[CB], d2[CB];
    SegVal<1> run_carry[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        const int j = j0 + c;
        live[c] = j < p;
        xc[c] = x + (int64_t)(live[c] ? j : j0) * ld;
        zs[c] = (zscale && live[c]) ? 1.0f / zscale[j] : 1.0f;
        g[c] = d1[c] = d2[c] = 0.0;
        run_carry[c] = seg_identity<1>();
        if (XBAR && live[c] && tile_carry[t]) run_carry[c].v[0] = carry[(int64_t)t * p + j];
    }
    for (int64_t base = r_begin; base < r_end; base += kColChunk) {
        const int64_t r0 = base + (int64_t)lane * kColIpt;   // 4 consecutive rows per lane: 16-byte loads
        double xv[CB][kColIpt], bv[kColIpt], wv[kColIpt], qv[kColIpt];
        uint32_t m[kColIpt];
        int32_t gi[kColIpt];
#pragma unroll
        for (int c = 0; c < CB; ++c) load4(xc[c] + r0, xv[c]);
        load4(b + r0, bv);
        {
            const uint4 mm = *reinterpret_cast<const uint4 *>(meta + r0);
            m[0] = mm.x;
            m[1] = mm.y;
            m[2] = mm.z;
            m[3] = mm.w;
        }
        if (XBAR) {
            load4(w + r0, wv);
            load4(zq + r0, qv);
            const int4 gg = *reinterpret_cast<const int4 *>(gidx + r0);
            gi[0] = gg.x;
            gi[1] = gg.y;
            gi[2] = gg.z;
            gi[3] = gg.w;
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) {
#pragma unroll
            for (int i = 0; i < kColIpt; ++i) {
                const double av = bv[i] - ((m[i] & kEventBit) ? 1.0 : 0.0);   // w Lambda - delta
                g[c] = fma(xv[c][i], av, g[c]);
                d1[c] = fma(xv[c][i] * xv[c][i], bv[i], d1[c]);
            }
        }
        if (XBAR) {
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                SegVal<1> e[kColIpt];
                SegVal<1> tot = seg_identity<1>();
#pragma unroll
                for (int i = 0; i < kColIpt; ++i) {
                    e[i].f = m[i] >> 31;
                    e[i].v[0] = wv[i] * xv[c][i];
                    tot = seg_combine(tot, e[i]);
                }
                const SegVal<1> inc = wave_inclusive_scan(tot);
                SegVal<1> run = seg_combine(run_carry[c], wave_shift_right(inc));
#pragma unroll
                for (int i = 0; i < kColIpt; ++i) {
                    run = seg_combine(run, e[i]);
                    if ((m[i] & kCountMask) && live[c]) {
                        const double zv = run.v[0] * qv[i];   // sqrt(d) xbar
                        d2[c] = fma(zv, zv, d2[c]);
                        store_z<ZT>(&z[(int64_t)(j0 + c) * ldz + gi[i]], zv, zs[c]);
                    }
                }
                run_carry[c] = seg_combine(run_carry[c], lane63_seg(inc));
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        double gc = g[c], s1 = d1[c], s2 = d2[c];
        for (int off = 32; off >= 1; off >>= 1) {
            gc += __shfl_xor(gc, off, kWave);
            s1 += __shfl_xor(s1, off, kWave);
            s2 += __shfl_xor(s2, off, kWave);
        }
        if (lane == 0 && live[c]) {
            double *o = part + ((int64_t)t * p + j0 + c) * 3;
            o[0] = gc;
            o[1] = s1;
            o[2] = s2;
        }
    }
}

// Fixed-order sums over tiles: grad[j], diag1[j], diag2[j] (thread k sums
// tiles k, k + 256, ... in order, then a fixed-order tree over the threads);
// workgroup p sums the objective parts.
__device__ __forceinline__ double tree_sum_256(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kRowBlock) void colreduce_kernel(const double *part, int p, int ntiles, double *grad,
                                                              double *diag1, double *diag2, const double *blockobj,
                                                              int nb, double *scal)
{
    __shared__ double red[kRowBlock / kWave];
    __shared__ double tree[256];
    const int j = blockIdx.x;
    if (j < p) {
        double sg = 0.0, s1 = 0.0, s2 = 0.0;
        for (int t = threadIdx.x; t < ntiles; t += kRowBlock) {
            const double *o = part + ((int64_t)t * p + j) * 3;
            sg += o[0];
            s1 += o[1];
            s2 += o[2];
        }
        sg = tree_sum_256(sg, tree);
        s1 = tree_sum_256(s1, tree);
        s2 = tree_sum_256(s2, tree);
        if (threadIdx.x == 0) {
            grad[j] = sg;
            diag1[j] = s1;
            diag2[j] = s2;
        }
    } else {
        double o = 0.0;
        for (int i = threadIdx.x; i < nb; i += kRowBlock) o += blockobj[i];
        o = block_sum(o, red);
        if (threadIdx.x == 0) scal[1] = o;
    }
}

// ------------------------------------------------------------------ row scans (forward / reverse)
//
// Segmented +scan of one FP64 value per row over all ld rows, in tiles of
// `tile` rows: (1) each workgroup folds its tile into one aggregate, (2) one
// workgroup scans the aggregates into the carry entering every tile, (3) each
// workgroup rescans its tile from its carry.  REV scans from the last row
// backwards, a segment then starting at the last row of each stratum.

constexpr int kScanThreads = 256, kScanWaves = kScanThreads / kWave;

template <bool REV>
__device__ __forceinline__ uint32_t scan_head(const uint32_t *meta, int64_t n, int64_t k)
{
    if (k == 0) return 1u;
    if (!REV) return (meta[k] & kHeadBit) ? 1u : 0u;
    return (meta[n - k] & kHeadBit) ? 1u : 0u;   // row n-1-k is a stratum's last row
}

template <bool REV>
__global__ __launch_bounds__(kScanThreads) void tileagg_kernel(const double *a, const uint32_t *meta, int64_t n,
                                                                 int64_t tile, double *aggv, uint32_t *aggf)
{
    __shared__ SegVal<1> wtot[kScanWaves];
    const int t = blockIdx.x;
    const int64_t per = tile / kScanThreads;
    const int64_t k0 = (int64_t)t * tile + (int64_t)threadIdx.x * per;
    SegVal<1> f = seg_identity<1>();
    for (int64_t i = 0; i < per; ++i) {
        const int64_t k = k0 + i;
        SegVal<1> e;
        e.f = scan_head<REV>(meta, n, k);
        e.v[0] = a[REV ? n - 1 - k : k];
        f = seg_combine(f, e);
    }
    SegVal<1> total;
    (void)block_exclusive_scan<1, kScanWaves>(f, wtot, total);
    if (threadIdx.x == 0) {
        aggv[t] = total.v[0];
        aggf[t] = total.f;
    }
}

// carry[t] = the running segment sum entering tile t (one workgroup)
__global__ __launch_bounds__(1024) void tilecarry_kernel(const double *aggv, const uint32_t *aggf, int ntiles,
                                                         double *carry)
{
    __shared__ SegVal<1> wtot[1024 / kWave];
    const int per = (ntiles + 1023) / 1024;
    const int t0 = threadIdx.x * per;
    SegVal<1> f = seg_identity<1>();
    for (int i = 0; i < per; ++i) {
        const int t = t0 + i;
        if (t < ntiles) {
            SegVal<1> e;
            e.f = aggf[t];
            e.v[0] = aggv[t];
            f = seg_combine(f, e);
        }
    }
    SegVal<1> total;
    SegVal<1> run = block_exclusive_scan<1, 1024 / kWave>(f, wtot, total);
    for (int i = 0; i < per; ++i) {
        const int t = t0 + i;
        if (t < ntiles) {
            carry[t] = run.v[0];
            SegVal<1> e;
            e.f = aggf[t];
            e.v[0] = aggv[t];
            run = seg_combine(run, e);
        }
    }
}

template <bool REV>
__global__ __launch_bounds__(kScanThreads) void tileapply_kernel(const double *a, const uint32_t *meta, double *out,
                                                                   int64_t n, int64_t tile, const double *carry)
{
    __shared__ SegVal<1> wtot[kScanWaves];
    const int t = blockIdx.x;
    const int64_t per = tile / kScanThreads;
    const int64_t k0 = (int64_t)t * tile + (int64_t)threadIdx.x * per;
    SegVal<1> f = seg_identity<1>();
    for (int64_t i = 0; i < per; ++i) {
        const int64_t k = k0 + i;
        SegVal<1> e;
        e.f = scan_head<REV>(meta, n, k);
        e.v[0] = a[REV ? n - 1 - k : k];
        f = seg_combine(f, e);
    }
    SegVal<1> total;
    const SegVal<1> exc = block_exclusive_scan<1, kScanWaves>(f, wtot, total);
    SegVal<1> run = seg_identity<1>();
    run.v[0] = carry[t];
    run = seg_combine(run, exc);
    for (int64_t i = 0; i < per; ++i) {
        const int64_t k = k0 + i;
        SegVal<1> e;
        e.f = scan_head<REV>(meta, n, k);
        e.v[0] = a[REV ? n - 1 - k : k];
        run = seg_combine(run, e);
        out[REV ? n - 1 - k : k] = run.v[0];
    }
}

}  // namespace

// ------------------------------------------------------------------ host launchers

int rowscan(const double *a, const uint32_t *meta, double *out, int64_t n, int64_t tile, bool reverse,
            void *scratch, size_t scratch_bytes, hipStream_t stream)
{
    if (tile <= 0 || tile % kScanThreads != 0 || n % tile != 0) return -5;
    const int ntiles = (int)(n / tile);
    if (rowscan_scratch_bytes(ntiles) > scratch_bytes) return -5;
    double *aggv = static_cast<double *>(scratch);
    double *carry = aggv + ntiles;
    uint32_t *aggf = reinterpret_cast<uint32_t *>(carry + ntiles);
    if (reverse) tileagg_kernel<true><<<ntiles, kScanThreads, 0, stream>>>(a, meta, n, tile, aggv, aggf);
    else tileagg_kernel<false><<<ntiles, kScanThreads, 0, stream>>>(a, meta, n, tile, aggv, aggf);
    tilecarry_kernel<<<1, 1024, 0, stream>>>(aggv, aggf, ntiles, carry);
    if (reverse) tileapply_kernel<true><<<ntiles, kScanThreads, 0, stream>>>(a, meta, out, n, tile, carry);
    else tileapply_kernel<false><<<ntiles, kScanThreads, 0, stream>>>(a, meta, out, n, tile, carry);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

size_t rowscan_scratch_bytes(int ntiles) { return (sizeof(double) * 2 + sizeof(uint32_t)) * (size_t)ntiles + 256; }

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
    int rc = rowscan(A.w, A.meta, A.s0, ld, A.tile, false, A.scan_scratch, A.scan_scratch_bytes, stream);
    if (rc) return rc;
    hazard_kernel<<<nb, kRowBlock, 0, stream>>>(A.s0, A.eta, A.meta, A.scal, ld, A.h, A.zq, A.blockbuf, A.flags);
    rc = rowscan(A.h, A.meta, A.lam, ld, A.tile, true, A.scan_scratch, A.scan_scratch_bytes, stream);
    if (rc) return rc;
    rowweight_kernel<<<nb, kRowBlock, 0, stream>>>(A.w, A.lam, A.meta, ld, A.a, A.b);
    if (A.n_agg > 0) {
        colagg_kernel<<<(A.n_agg * A.p + kColWaves - 1) / kColWaves, kWave * kColWaves, 0, stream>>>(
            A.x, ld, A.p, A.w, A.tile, A.agg_tiles, A.n_agg, A.lasthead, A.agg);
        colcarry_kernel<<<(A.p + 255) / 256, 256, 0, stream>>>(A.p, A.ntiles, A.tile_carry, A.lasthead, A.agg,
                                                               A.carry);
    }
    const int grid = 8 * ((A.ntiles + 7) / 8) * ((A.p + kColWaves * kColBlock - 1) / (kColWaves * kColBlock));
#define COXMI_COLPASS(ZT, XB)                                                                                  \
    colpass_kernel<ZT, XB><<<grid, kWave * kColWaves, 0, stream>>>(                                            \
        A.x, ld, A.p, A.tile, A.ntiles, A.w, A.zq, A.b, A.meta, A.gidx, A.tile_carry, A.carry, A.ldz,          \
        A.zscale, static_cast<ZT *>(A.z), A.colpart)
    if (!A.want_xbar) COXMI_COLPASS(double, false);
    else if (A.ztype == kZF64) COXMI_COLPASS(double, true);
    else if (A.ztype == kZF32) COXMI_COLPASS(float, true);
    else COXMI_COLPASS(__hip_bfloat16, true);
#undef COXMI_COLPASS
    colreduce_kernel<<<A.p + 1, kRowBlock, 0, stream>>>(A.colpart, A.p, A.ntiles, A.grad, A.diag1, A.diag2,
                                                        A.blockbuf, nb, A.scal);
    e = hipGetLastError();
    return e == hipSuccess ? 0 : -3;
}

}  // namespace coxmi
