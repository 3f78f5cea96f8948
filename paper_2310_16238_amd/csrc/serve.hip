// serve.hip -- batched kernels of the fit server (gfx950).
//
// One Newton iteration of every resident fit is five launches:
//   eta   (fit, 256-row tile)  X beta in FP64 and the tile's max of X beta
//   rows  (fit, scan tile)     w = exp(X beta - c), forward segmented scan of w
//                              (S0), d/S0 and (d/S0)/sqrt(d) at group ends and the
//                              objective, reverse
//                              segmented scan of d/S0 (Lambda), a = w Lambda - delta,
//                              b = w Lambda
//   cols  (fit, scan tile, column)
//                              one wave: forward segmented scan of w x_j (S1),
//                              xbar = S1/S0 at group ends, z = sqrt(d) xbar,
//                              score X'a, diagonal (X o X)'b - sum d xbar^2
//   syrk  (fit, tile pair, K range, product)
//                              one wave: a 32 x 32 tile of X' diag(b) X or Z'Z on
//                              the matrix cores (v_mfma_f32_32x32x2f32, FP32)
//   step  (fit)                the information matrix from the partials (FP64),
//                              Cholesky in LDS, the Newton step and the fit's
//                              state machine (halving, freezing, convergence)
// The sums follow Eqs. strat_l, strat_g and strat_h with the order of the sums
// over events and risk sets exchanged (the Lambda form).
#include <math.h>

#include "coxmi.h"
#include "internal.h"
#include "segscan.hpp"
#include "serve.h"

namespace coxmi {
namespace serve {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
    return v;
}

// ------------------------------------------------------------------ admit: FP32 copy of X

__global__ __launch_bounds__(256) void admit_kernel(const FitDesc *fits, const int2 *items)
{
    const int2 it = items[blockIdx.x];
    const FitDesc F = fits[it.x];
    const int64_t r = (int64_t)it.y * 256 + threadIdx.x;
    if (r >= F.ld) return;
    for (int j = 0; j < F.p; ++j) F.xf[(int64_t)j * F.ld + r] = (float)F.x[(int64_t)j * F.ld + r];
}

// ------------------------------------------------------------------ eta

__global__ __launch_bounds__(kEtaRows) void eta_kernel(const FitDesc *fits, const int2 *items)
{
    __shared__ double red[kEtaRows / kWave];
    const int2 it = items[blockIdx.x];
    const FitDesc F = fits[it.x];
    const int64_t r = (int64_t)it.y * kEtaRows + threadIdx.x;
    double mx = -INFINITY;
    if (r < F.ld) {
        double e = 0.0;
        for (int j = 0; j < F.p; ++j) {
            const double bj = F.beta[j];
            if (bj != 0.0) e = fma(F.x[(int64_t)j * F.ld + r], bj, e);
        }
        F.eta[r] = e;
        if (!(F.meta[r] & kPadBit)) mx = e;
    }
    mx = wave_max(mx);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int k = 1; k < kEtaRows / kWave; ++k) m = fmax(m, red[k]);
        F.tilemax[it.y] = m;
    }
}

// ------------------------------------------------------------------ rows

constexpr int kRowThreads = 512, kRowIpt = 4, kRowTile = kRowThreads * kRowIpt, kRowWaves = kRowThreads / kWave;

__device__ __forceinline__ double block_sum_rows(double v, double *red)
{
    v = wave_sum(v);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < kRowWaves; ++k) s += red[k];
    __syncthreads();
    return s;
}

__device__ __forceinline__ double block_max_rows(double v, double *red)
{
    v = wave_max(v);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    double s = -INFINITY;
    for (int k = 0; k < kRowWaves; ++k) s = fmax(s, red[k]);
    __syncthreads();
    return s;
}

// One workgroup per (fit, scan tile): every scan tile starts with a stratum
// head (or is the fit's only tile), so its scans need no carry.  The tile's
// objective part and range flag go to tpart; the step kernel adds them up.
__global__ __launch_bounds__(kRowThreads) void rows_kernel(const FitDesc *fits, const int2 *items)
{
    __shared__ SegVal<1> wtot[kRowWaves];
    __shared__ double red[kRowWaves];
    const int2 it = items[blockIdx.x];
    const FitDesc F = fits[it.x];
    const int t = threadIdx.x;
    const int64_t r_begin = (int64_t)it.y * F.tile;
    const int64_t r_end = r_begin + F.tile < F.ld ? r_begin + F.tile : F.ld;
    const int64_t len = r_end - r_begin;

    double c = -INFINITY;
    for (int i = t; i < F.ntile; i += kRowThreads) c = fmax(c, F.tilemax[i]);
    c = block_max_rows(c, red);
    if (!(c > -INFINITY)) c = 0.0;   // a fit of padding rows only cannot occur; guard the shift anyway

    // forward: S0 = segmented scan of w; at group ends d/S0 and d (log S0 + c); -eta at events
    double obj = 0.0;
    unsigned bad = 0u;
    SegVal<1> carry = seg_identity<1>();
    for (int64_t base = 0; base < len; base += kRowTile) {
        SegVal<1> e[kRowIpt];
        SegVal<1> tagg = seg_identity<1>();
#pragma unroll
        for (int i = 0; i < kRowIpt; ++i) {
            const int64_t k = base + (int64_t)t * kRowIpt + i;
            if (k < len) {
                const int64_t r = r_begin + k;
                const uint32_t mw = F.meta[r];
                e[i].f = (k == 0) ? 1u : (mw >> 31);
                e[i].v[0] = (mw & kPadBit) ? 0.0 : exp(F.eta[r] - c);   // padding rows carry no weight
            } else {
                e[i] = seg_identity<1>();
            }
            tagg = seg_combine(tagg, e[i]);
        }
        SegVal<1> btot;
        const SegVal<1> exc = block_exclusive_scan<1, kRowWaves>(tagg, wtot, btot);
        SegVal<1> run = seg_combine(carry, exc);
#pragma unroll
        for (int i = 0; i < kRowIpt; ++i) {
            const int64_t k = base + (int64_t)t * kRowIpt + i;
            run = seg_combine(run, e[i]);
            if (k < len) {
                const int64_t r = r_begin + k;
                const uint32_t m = F.meta[r];
                const uint32_t d = m & kCountMask;
                F.w[r] = e[i].v[0];
                double hv = 0.0, qv = 0.0;
                if (d != 0u) {
                    const double s = run.v[0];
                    if (!(s >= 1e-300) || !(s <= 1e300)) bad = 1u;
                    hv = (double)d / s;
                    qv = hv / sqrt((double)d);
                    obj += (double)d * (log(s) + c);
                }
                if (m & kEventBit) obj -= F.eta[r];
                F.hz[r] = hv;
                F.zq[r] = qv;
            }
        }
        carry = seg_combine(carry, btot);
        __syncthreads();   // wtot is rewritten by the next chunk; w / hz visible to the reverse pass
    }

    // reverse: Lambda = segmented scan of d/S0 from each stratum's last row backwards
    carry = seg_identity<1>();
    for (int64_t base = 0; base < len; base += kRowTile) {
        SegVal<1> e[kRowIpt];
        SegVal<1> tagg = seg_identity<1>();
#pragma unroll
        for (int i = 0; i < kRowIpt; ++i) {
            const int64_t k = base + (int64_t)t * kRowIpt + i;   // scan position; row r_end-1-k
            if (k < len) {
                const int64_t r = r_end - 1 - k;
                e[i].f = (k == 0 || (F.meta[r + 1] & kHeadBit)) ? 1u : 0u;
                e[i].v[0] = F.hz[r];
            } else {
                e[i] = seg_identity<1>();
            }
            tagg = seg_combine(tagg, e[i]);
        }
        SegVal<1> btot;
        const SegVal<1> exc = block_exclusive_scan<1, kRowWaves>(tagg, wtot, btot);
        SegVal<1> run = seg_combine(carry, exc);
#pragma unroll
        for (int i = 0; i < kRowIpt; ++i) {
            const int64_t k = base + (int64_t)t * kRowIpt + i;
            run = seg_combine(run, e[i]);
            if (k < len) {
                const int64_t r = r_end - 1 - k;
                const double wl = F.w[r] * run.v[0];
                F.b[r] = wl;
                F.a[r] = wl - ((F.meta[r] & kEventBit) ? 1.0 : 0.0);
            }
        }
        carry = seg_combine(carry, btot);
        __syncthreads();
    }
    obj = block_sum_rows(obj, red);
    const double anybad = block_max_rows(bad ? 1.0 : 0.0, red);
    if (t == 0) {
        F.tpart[2 * it.y] = obj;
        F.tpart[2 * it.y + 1] = anybad;
    }
}

// ------------------------------------------------------------------ cols

constexpr int kColWaves = 4, kColIpt = 4, kColChunk = kWave * kColIpt;

__global__ __launch_bounds__(kWave * kColWaves) void cols_kernel(const FitDesc *fits, const int2 *items, int nitems)
{
    const int lane = threadIdx.x & (kWave - 1);
    // the item index is the same in all lanes of a wave
    const int item = __builtin_amdgcn_readfirstlane(blockIdx.x * kColWaves + threadIdx.x / kWave);
    if (item >= nitems) return;   // whole wave; no workgroup barrier below
    const int2 it = items[item];
    const FitDesc F = fits[it.x];
    const int tt = it.y >> 10, j = it.y & 1023;   // (scan tile, column)
    const int64_t r_begin = (int64_t)tt * F.tile;
    const int64_t n = r_begin + F.tile < F.ld ? r_begin + F.tile : F.ld;
    const double *xj = F.x + (int64_t)j * F.ld;
    float *zj = F.z + (int64_t)j * F.ldz;
    double g = 0.0, d1 = 0.0, d2 = 0.0;
    SegVal<1> carry = seg_identity<1>();
    for (int64_t base = r_begin; base < n; base += kColChunk) {
        const int64_t r0 = base + (int64_t)lane * kColIpt;
        SegVal<1> e[kColIpt];
        uint32_t m[kColIpt];
        SegVal<1> tot = seg_identity<1>();
#pragma unroll
        for (int i = 0; i < kColIpt; ++i) {
            const int64_t r = r0 + i;
            if (r < n) {
                m[i] = F.meta[r];
                const double xv = xj[r];
                e[i].f = m[i] >> 31;
                e[i].v[0] = F.w[r] * xv;
                g = fma(xv, F.a[r], g);
                d1 = fma(xv * xv, F.b[r], d1);
            } else {
                m[i] = 0u;
                e[i] = seg_identity<1>();
            }
            tot = seg_combine(tot, e[i]);
        }
        const SegVal<1> inc = wave_inclusive_scan(tot);
        SegVal<1> run = seg_combine(carry, wave_shift_right(inc));
#pragma unroll
        for (int i = 0; i < kColIpt; ++i) {
            run = seg_combine(run, e[i]);
            if (m[i] & kCountMask) {
                const int64_t r = r0 + i;
                const double zv = run.v[0] * F.zq[r];   // sqrt(d) xbar
                d2 = fma(zv, zv, d2);
                zj[F.gidx[r]] = (float)zv;
            }
        }
        carry = seg_combine(carry, lane63_seg(inc));
    }
    g = wave_sum(g);
    d1 = wave_sum(d1);
    d2 = wave_sum(d2);
    if (lane == 0) {
        double *o = F.cpart + ((int64_t)tt * F.p + j) * 3;
        o[0] = g;
        o[1] = d1;
        o[2] = d2;
    }
}

// ------------------------------------------------------------------ syrk (FP32 matrix cores)

__host__ __device__ __forceinline__ int tile_count(int p) { return (p + kTile - 1) / kTile; }

__device__ __forceinline__ void pair_tiles(int pair, int nt, int &ti, int &tj)
{
    int i = 0, rem = pair;
    while (rem >= nt - i) {
        rem -= nt - i;
        ++i;
    }
    ti = i;
    tj = i + rem;
}

__device__ __forceinline__ int pair_index(int ti, int tj, int nt)
{
    // row-major order of the upper triangle (ti <= tj)
    return ti * nt - ti * (ti - 1) / 2 + (tj - ti);
}

constexpr int kSyrkWaves = 4;

__global__ __launch_bounds__(kWave * kSyrkWaves) void syrk_kernel(const FitDesc *fits, const int4 *items, int nitems)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int item = __builtin_amdgcn_readfirstlane(blockIdx.x * kSyrkWaves + threadIdx.x / kWave);
    if (item >= nitems) return;   // whole wave
    const int4 it = items[item];
    const FitDesc F = fits[it.x];
    const int nt = tile_count(F.p);
    int ti, tj;
    pair_tiles(it.y, nt, ti, tj);
    const bool zpart = it.w != 0;
    const float *u = zpart ? F.z : F.xf;
    const int64_t ldu = zpart ? F.ldz : F.ld;
    const int64_t k0 = (int64_t)it.z * (zpart ? kZRange : kXRange);
    const int64_t kend = k0 + (zpart ? kZRange : kXRange);
    const int64_t k1 = kend < ldu ? kend : ldu;
    const double *c = zpart ? nullptr : F.b;
    const int ra = ti * kTile + (lane & 31), rb = tj * kTile + (lane & 31);
    const int kofs = 4 * (lane >> 5);
    const float *ua = u + (int64_t)(ra < F.p ? ra : 0) * ldu;
    const float *ub = u + (int64_t)(rb < F.p ? rb : 0) * ldu;
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    for (int64_t k = k0; k < k1; k += 8) {
        const int64_t kk = k + kofs;
        float4 av = *reinterpret_cast<const float4 *>(ua + kk);
        float4 bv = *reinterpret_cast<const float4 *>(ub + kk);
        if (ra >= F.p) av = make_float4(0.f, 0.f, 0.f, 0.f);
        if (rb >= F.p) bv = make_float4(0.f, 0.f, 0.f, 0.f);
        if (c) {
            av.x *= (float)c[kk];
            av.y *= (float)c[kk + 1];
            av.z *= (float)c[kk + 2];
            av.w *= (float)c[kk + 3];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, bv.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, bv.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.z, bv.z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.w, bv.w, acc, 0, 0, 0);
    }
    const int slot = zpart ? F.nxr + it.z : it.z;
    float *out = F.part + ((int64_t)slot * F.npairs + it.y) * (kTile * kTile);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int m = 8 * (i / 4) + 4 * (lane >> 5) + (i % 4), nn = lane & 31;
        out[m * kTile + nn] = acc[i];
    }
}

// ------------------------------------------------------------------ step

constexpr int kStepThreads = 256;

__global__ __launch_bounds__(kStepThreads) void step_kernel(const FitDesc *fits, const int *slots)
{
    extern __shared__ double lds[];   // A[p * p], y[p]
    __shared__ int s_action, s_bad, s_frozen;
    __shared__ double s_red[kStepThreads / kWave];
    __shared__ double s_piv;
    const FitDesc F = fits[slots[blockIdx.x]];
    FitState *st = F.st;
    const int t = threadIdx.x, p = F.p;
    double *A = lds;
    double *y = lds + (int64_t)p * p;

    // per-column sums of the scan-tile partials, and the objective, in tile order
    for (int j = t; j < p; j += kStepThreads) {
        double sg = 0.0, s1 = 0.0, s2 = 0.0;
        for (int q = 0; q < F.ntc; ++q) {
            const double *o = F.cpart + ((int64_t)q * p + j) * 3;
            sg += o[0];
            s1 += o[1];
            s2 += o[2];
        }
        F.grad[j] = sg;
        F.diag1[j] = s1;
        F.diag2[j] = s2;
    }
    if (t == 0) {
        double o = 0.0, bad = 0.0;
        for (int q = 0; q < F.ntc; ++q) {
            o += F.tpart[2 * q];
            bad = fmax(bad, F.tpart[2 * q + 1]);
        }
        st->obj_eval = o;
        st->range = bad > 0.0 ? 1u : 0u;
    }
    __syncthreads();
    if (t == 0) {
        st->evals += 1;
        int action = 2;   // 0 stop, 1 halve, 2 step
        if (st->range) {
            st->status = COX_ENUMERIC;
            st->flags |= kDone;
            action = 0;
        } else if (st->iters > 0 && st->halvings < 40 &&
                   st->obj_eval > st->obj_prev + 1e-12 * fabs(st->obj_prev)) {
            st->halvings += 1;
            action = 1;
        }
        s_action = action;
        s_frozen = (st->flags & kFrozen) ? 1 : 0;
        s_bad = 0;
    }
    __syncthreads();
    const int action = s_action;
    if (action == 0) return;
    if (action == 1) {
        for (int j = t; j < p; j += kStepThreads) F.beta[j] = F.prev[j] + 0.5 * (F.beta[j] - F.prev[j]);
        return;
    }
    // the columns that move: chosen once, at the first evaluation (g'' > 1e-12 S2-term)
    if (!(st->flags & kHaveFree)) {
        for (int j = t; j < p; j += kStepThreads) {
            const double hd = F.diag1[j] - F.diag2[j];
            F.free_col[j] = (hd > 1e-12 * fabs(F.diag1[j]) && isfinite(hd)) ? 1 : 0;
        }
        __syncthreads();
    }
    const bool frozen = s_frozen != 0;
    if (!frozen) {
        // I = X' diag(b) X - Z'Z from the upper-triangle tiles, partials summed in FP64 in range order
        const int nt = tile_count(p);
        for (int e = t; e < p * p; e += kStepThreads) {
            const int i = e / p, j = e % p;
            if (j < i) continue;
            const int ti = i / kTile, tj = j / kTile;
            const int pair = pair_index(ti, tj, nt);
            const int off = (i % kTile) * kTile + (j % kTile);
            double sx = 0.0, sz = 0.0;
            for (int r = 0; r < F.nxr; ++r) sx += (double)F.part[((int64_t)r * F.npairs + pair) * (kTile * kTile) + off];
            for (int r = 0; r < F.nzr; ++r)
                sz += (double)F.part[((int64_t)(F.nxr + r) * F.npairs + pair) * (kTile * kTile) + off];
            double v = sx - sz;
            if (!F.free_col[i] || !F.free_col[j]) v = (i == j) ? 1.0 : 0.0;
            A[i * p + j] = v;
            A[j * p + i] = v;
        }
        __syncthreads();
        // right-looking Cholesky, lower triangle
        for (int k = 0; k < p; ++k) {
            if (t == 0) {
                double d = A[k * p + k];
                if (!(d > 0.0)) {
                    s_bad = 1;
                    d = 1.0;
                }
                s_piv = sqrt(d);
                A[k * p + k] = s_piv;
            }
            __syncthreads();
            const double piv = s_piv;
            for (int i = k + 1 + t; i < p; i += kStepThreads) A[i * p + k] /= piv;
            __syncthreads();
            const int m = p - k - 1;
            for (int e = t; e < m * m; e += kStepThreads) {
                const int i = k + 1 + e / m, j = k + 1 + e % m;
                if (j <= i) A[i * p + j] -= A[i * p + k] * A[j * p + k];
            }
            __syncthreads();
        }
        for (int e = t; e < p * p; e += kStepThreads) F.L[e] = A[e];
    } else {
        for (int e = t; e < p * p; e += kStepThreads) A[e] = F.L[e];
    }
    // score on the free columns; kkt = max |score|
    double kk = 0.0;
    for (int j = t; j < p; j += kStepThreads) {
        const double gj = F.free_col[j] ? F.grad[j] : 0.0;
        y[j] = -gj;
        kk = fmax(kk, fabs(gj));
    }
    kk = wave_max(kk);
    if ((t & (kWave - 1)) == 0) s_red[t / kWave] = kk;
    __syncthreads();
    // L y = -g, then L' dx = y
    for (int k = 0; k < p; ++k) {
        if (t == 0) y[k] /= A[k * p + k];
        __syncthreads();
        const double yk = y[k];
        for (int i = k + 1 + t; i < p; i += kStepThreads) y[i] -= A[i * p + k] * yk;
        __syncthreads();
    }
    for (int k = p - 1; k >= 0; --k) {
        if (t == 0) y[k] /= A[k * p + k];
        __syncthreads();
        const double xk = y[k];
        for (int i = t; i < k; i += kStepThreads) y[i] -= A[k * p + i] * xk;
        __syncthreads();
    }
    double smax = 0.0, bmax = 0.0;
    for (int j = t; j < p; j += kStepThreads) {
        const double dx = F.free_col[j] ? y[j] : 0.0;
        const double b0 = F.beta[j];
        const double b1 = b0 + dx;
        F.prev[j] = b0;
        F.beta[j] = b1;
        smax = fmax(smax, fabs(dx));
        bmax = fmax(bmax, fabs(b1));
    }
    smax = wave_max(smax);
    bmax = wave_max(bmax);
    __shared__ double s_s[kStepThreads / kWave], s_b[kStepThreads / kWave];
    if ((t & (kWave - 1)) == 0) {
        s_s[t / kWave] = smax;
        s_b[t / kWave] = bmax;
    }
    __syncthreads();
    if (t == 0) {
        double step = 0.0, bm = 1.0, kkt = 0.0;
        for (int k = 0; k < kStepThreads / kWave; ++k) {
            step = fmax(step, s_s[k]);
            bm = fmax(bm, s_b[k]);
            kkt = fmax(kkt, s_red[k]);
        }
        int flags = st->flags | kHaveFree;
        int pinned = 0;
        for (int j = 0; j < p; ++j) pinned += F.free_col[j] ? 0 : 1;
        st->n_pinned = pinned;
        st->kkt = kkt;
        st->obj = st->obj_eval;
        st->obj_prev = st->obj_eval;
        st->halvings = 0;
        st->iters += 1;
        st->last_step = step;
        if (s_bad) {
            st->status = COX_ENUMERIC;
            flags |= kDone;
        } else if (step <= F.tol * bm) {
            st->status = COX_OK;
            flags |= kDone;
        } else {
            if (F.freeze && !frozen && step <= 1e-3 * bm) flags |= kFrozen;
            if (st->iters >= F.max_iter) {
                st->status = COX_NOT_CONVERGED;
                flags |= kDone;
            }
        }
        st->flags = flags;
    }
}

}  // namespace

int launch_admit(const FitDesc *fits, const int2 *items, int nitems, hipStream_t s)
{
    if (nitems > 0) admit_kernel<<<nitems, 256, 0, s>>>(fits, items);
    return (int)hipGetLastError();
}

int launch_eta(const FitDesc *fits, const int2 *items, int nitems, hipStream_t s)
{
    if (nitems > 0) eta_kernel<<<nitems, kEtaRows, 0, s>>>(fits, items);
    return (int)hipGetLastError();
}

int launch_rows(const FitDesc *fits, const int2 *items, int nitems, hipStream_t s)
{
    if (nitems > 0) rows_kernel<<<nitems, kRowThreads, 0, s>>>(fits, items);
    return (int)hipGetLastError();
}

int launch_cols(const FitDesc *fits, const int2 *items, int nitems, hipStream_t s)
{
    if (nitems > 0) cols_kernel<<<(nitems + kColWaves - 1) / kColWaves, kWave * kColWaves, 0, s>>>(fits, items, nitems);
    return (int)hipGetLastError();
}

int launch_syrk(const FitDesc *fits, const int4 *items, int nitems, hipStream_t s)
{
    if (nitems > 0)
        syrk_kernel<<<(nitems + kSyrkWaves - 1) / kSyrkWaves, kWave * kSyrkWaves, 0, s>>>(fits, items, nitems);
    return (int)hipGetLastError();
}

int launch_step(const FitDesc *fits, const int *slots, int nslots, int max_p, hipStream_t s)
{
    if (nslots <= 0) return 0;
    const size_t lds = sizeof(double) * ((size_t)max_p * max_p + max_p);
    static bool attr_set = false;
    if (!attr_set) {
        const size_t most = sizeof(double) * ((size_t)kMaxP * kMaxP + kMaxP);
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&step_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)most);
        if (e != hipSuccess) return (int)e;
        attr_set = true;
    }
    step_kernel<<<nslots, kStepThreads, lds, s>>>(fits, slots);
    return (int)hipGetLastError();
}

}  // namespace serve
}  // namespace coxmi
