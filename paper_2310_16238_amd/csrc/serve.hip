// serve.hip -- batched kernels of the fit server (gfx950).
//
// Fits join through `admit` (descriptor, FP32 copy of X, cleared state).  One
// Newton iteration of every resident fit is six launches (or one phase each of
// the persistent round kernel at the end of this file):
//   eta   (fit, 256-row tile)  X beta in FP64 and the tile's max of X beta
//   rows  (fit, scan tile)     w = exp(X beta - c), forward segmented scan of w
//                              (S0), d/S0 and (d/S0)/sqrt(d) at group ends and the
//                              objective, reverse
//                              segmented scan of d/S0 (Lambda), a = w Lambda - delta,
//                              b = w Lambda
//   cols  (fit, scan tile, 4 columns)
//                              one wave: forward segmented scan of w x_j (S1),
//                              xbar = S1/S0 at group ends, z = sqrt(d) xbar,
//                              score X'a, diagonal (X o X)'b - sum d xbar^2
//   syrk  (fit, K range, product), or (fit, tile pair, K range, product) in light rounds
//                              four waves: the 32 x 32 tile pairs of X' diag(b) X or
//                              Z'Z over 1024-4096 rows (event groups)
//                              on the matrix cores (v_mfma_f32_32x32x2f32, FP32)
//   info  (fit, tile pair)     the K-range partials summed in FP64 in range order:
//                              the information matrix
//   step  (fit)                Cholesky in LDS, the Newton step and the fit's
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

// x of lane src, for a src that is the same in every lane of the wave (two v_readlane, no
// trip through the LDS crossbar as for a per-lane source)
__device__ __forceinline__ double lane_value(double x, int src)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// ------------------------------------------------------------------ admit: FP32 copy of X

// Item (k, t): rows [256 t, 256 t + 256) of joining fit k (X gathered from the
// caller's device memory for a device-resident request; the FP32 copy).  The items of a fit
// also clear its z (grid-stride over the fit's items); item 0 installs the
// descriptor in the fit's slot and clears beta, the previous beta and the state.
__global__ __launch_bounds__(256) void admit_kernel(FitDesc *fits, const FitDesc *joining, const int *slots,
                                                    const int2 *items)
{
    const int2 it = items[blockIdx.x];
    const FitDesc &F = joining[it.x];
    const int x = threadIdx.x;
    const int64_t r = (int64_t)it.y * 256 + x;
    if (r < F.ld) {
        if (F.xs) {
            // device-resident request: gather the canonical rows from the caller's X
            const int32_t sr = F.src[r];
            for (int j0 = 0; j0 < F.p; j0 += 8) {   // 8 loads in flight per thread
                double v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    v[q] = (j0 + q < F.p && sr >= 0) ? F.xs[(int64_t)(j0 + q) * F.ldxs + sr] : 0.0;
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (j0 + q < F.p) {
                        F.x[(int64_t)(j0 + q) * F.ld + r] = v[q];
                        F.xf[(int64_t)(j0 + q) * F.ld + r] = (float)v[q];
                    }
            }
        } else {
            for (int j = 0; j < F.p; ++j) F.xf[(int64_t)j * F.ld + r] = (float)F.x[(int64_t)j * F.ld + r];
        }
    }
    const int64_t nz = (int64_t)F.p * F.ldz, stride = (int64_t)F.ntile * 256;
    for (int64_t e = (int64_t)it.y * 256 + x; e < nz; e += stride) F.z[e] = 0.0f;
    if (it.y == 0) {
        if (x < F.p) {
            const double b0 = F.beta0 ? F.beta0[x] : 0.0;
            F.beta[x] = b0;
            F.prev[x] = b0;
        }
        if (x < (int)(sizeof(FitState) / 4)) reinterpret_cast<uint32_t *>(F.st)[x] = 0u;
        uint64_t *dst = reinterpret_cast<uint64_t *>(fits + slots[it.x]);
        const uint64_t *src = reinterpret_cast<const uint64_t *>(&F);
        if (x < (int)(sizeof(FitDesc) / 8)) dst[x] = src[x];
    }
}

// ------------------------------------------------------------------ eta

// The fit's state flags as the last step left them.  Rounds may be queued before the
// previous one has finished, so every kernel leaves out the items of fits that have
// finished (and the contraction those whose information matrix is frozen).
__device__ __forceinline__ int fit_flags(const FitDesc *fits, int slot) { return fits[slot].st->flags; }


// The phases of a round are device functions shared by the separate launches
// below and by the persistent round kernel; a phase body makes the same sums in
// the same order in both, so a fit's result does not depend on which runs it.

// Item (fit, 256-row tile) of X beta, run by kEtaRows threads (t = 0 .. 255).
// Every thread of the workgroup calls it the same number of times (the
// barriers inside); `live` false leaves the item out.
__device__ __forceinline__ void eta_item(const FitDesc *fits, int2 it, bool live, int t, double *red)
{
    double mx = -INFINITY;
    if (live) {
        const FitDesc F = fits[it.x];
        const int64_t r = (int64_t)it.y * kEtaRows + t;
        if (r < F.ld) {
            // every column, in order (X is finite, so a zero coefficient adds a zero)
            const double *xr = F.x + r;
            double e = 0.0;
            int j = 0;
            for (; j + 8 <= F.p; j += 8) {
                double v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) v[q] = xr[(int64_t)(j + q) * F.ld];
#pragma unroll
                for (int q = 0; q < 8; ++q) e = fma(v[q], F.beta[j + q], e);
            }
            for (; j < F.p; ++j) e = fma(xr[(int64_t)j * F.ld], F.beta[j], e);
            F.eta[r] = e;
            if (!(F.meta[r] & kPadBit)) mx = e;
        }
    }
    mx = wave_max(mx);
    if ((t & (kWave - 1)) == 0) red[t / kWave] = mx;
    __syncthreads();
    if (live && t == 0) {
        double m = red[0];
        for (int k = 1; k < kEtaRows / kWave; ++k) m = fmax(m, red[k]);
        fits[it.x].tilemax[it.y] = m;
    }
    __syncthreads();   // red is rewritten by the next item
}

__global__ __launch_bounds__(kEtaRows) void eta_kernel(const FitDesc *fits, const int2 *items)
{
    __shared__ double red[kEtaRows / kWave];
    const int2 it = items[blockIdx.x];
    eta_item(fits, it, !(fit_flags(fits, it.x) & kDone), threadIdx.x, red);
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
// Run by kRowThreads threads; the whole workgroup takes the item.
__device__ __forceinline__ void rows_item(const FitDesc *fits, int2 it)
{
    __shared__ SegVal<1> wtot[kRowWaves];
    __shared__ double red[kRowWaves];
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
                const double bw = F.w[r] * run.v[0];
                F.b[r] = bw;
                F.bf[r] = (float)bw;
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

__global__ __launch_bounds__(kRowThreads) void rows_kernel(const FitDesc *fits, const int2 *items)
{
    const int2 it = items[blockIdx.x];
    if (!(fit_flags(fits, it.x) & kDone)) rows_item(fits, it);
}

// ------------------------------------------------------------------ cols

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

// One wave per (fit, scan tile, block of kColBlock columns): the row vectors
// (w, b, zq, row words, group indices) are loaded once per chunk for all the
// block's columns, whose scans share one flag.  Lanes own 4 consecutive rows
// (scan tiles and the padded row count are multiples of 64, so a lane's rows
// are all in the tile or all past it).
// Run by one wave (no workgroup barrier inside).  PF: the next chunk's loads are issued
// before this chunk is processed (more registers; same arithmetic).
template <bool PF>
__device__ __forceinline__ void cols_item(const FitDesc *fits, int2 it)
{
    constexpr int CB = kColBlock;
    const int lane = threadIdx.x & (kWave - 1);
    const FitDesc F = fits[it.x];
    const int tt = it.y >> 10, j0 = it.y & 1023;   // (scan tile, first column of the block)
    const int64_t r_begin = (int64_t)tt * F.tile;
    const int64_t r_end = r_begin + F.tile < F.ld ? r_begin + F.tile : F.ld;
    const double *xc[CB];
    bool live[CB];
    double g[CB], d1[CB], d2[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        live[c] = j0 + c < F.p;
        xc[c] = F.x + (int64_t)(live[c] ? j0 + c : j0) * F.ld;
        g[c] = d1[c] = d2[c] = 0.0;
    }
    // one chunk's loads; the next chunk's loads are issued before this chunk is processed
    struct Chunk {
        double xv[CB][kColIpt], wv[kColIpt], bv[kColIpt], qv[kColIpt];
        uint32_t m[kColIpt];
        int32_t gi[kColIpt];
    };
    auto load_chunk = [&](Chunk &k, int64_t r0) {
        if (r0 < r_end) {
#pragma unroll
            for (int c = 0; c < CB; ++c) load4(xc[c] + r0, k.xv[c]);
            load4(F.w + r0, k.wv);
            load4(F.b + r0, k.bv);
            load4(F.zq + r0, k.qv);
            const uint4 mm = *reinterpret_cast<const uint4 *>(F.meta + r0);
            const int4 gg = *reinterpret_cast<const int4 *>(F.gidx + r0);
            k.m[0] = mm.x;
            k.m[1] = mm.y;
            k.m[2] = mm.z;
            k.m[3] = mm.w;
            k.gi[0] = gg.x;
            k.gi[1] = gg.y;
            k.gi[2] = gg.z;
            k.gi[3] = gg.w;
        } else {
#pragma unroll
            for (int i = 0; i < kColIpt; ++i) {
#pragma unroll
                for (int c = 0; c < CB; ++c) k.xv[c][i] = 0.0;
                k.wv[i] = k.bv[i] = k.qv[i] = 0.0;
                k.m[i] = 0u;
                k.gi[i] = 0;
            }
        }
    };
    SegVal<CB> carry = seg_identity<CB>();
    Chunk cur;
    load_chunk(cur, r_begin + (int64_t)lane * kColIpt);
    for (int64_t base = r_begin; base < r_end; base += kColChunk) {
        const int64_t r0 = base + (int64_t)lane * kColIpt;
        Chunk nxt;
        const bool more = base + kColChunk < r_end;
        if (PF && more) load_chunk(nxt, r0 + kColChunk);
        double(&xv)[CB][kColIpt] = cur.xv;
        double(&wv)[kColIpt] = cur.wv;
        double(&bv)[kColIpt] = cur.bv;
        double(&qv)[kColIpt] = cur.qv;
        uint32_t(&m)[kColIpt] = cur.m;
        int32_t(&gi)[kColIpt] = cur.gi;
        SegVal<CB> e[kColIpt];
        SegVal<CB> tot = seg_identity<CB>();
#pragma unroll
        for (int i = 0; i < kColIpt; ++i) {
            const double aw = bv[i] - ((m[i] & kEventBit) ? 1.0 : 0.0);   // w Lambda - delta
            e[i].f = m[i] >> 31;
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                g[c] = fma(xv[c][i], aw, g[c]);
                d1[c] = fma(xv[c][i] * xv[c][i], bv[i], d1[c]);
                e[i].v[c] = wv[i] * xv[c][i];
            }
            tot = seg_combine(tot, e[i]);
        }
        const SegVal<CB> inc = wave_inclusive_scan(tot);
        SegVal<CB> run = seg_combine(carry, wave_shift_right(inc));
#pragma unroll
        for (int i = 0; i < kColIpt; ++i) {
            run = seg_combine(run, e[i]);
            if (m[i] & kCountMask) {
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    const double zv = run.v[c] * qv[i];   // sqrt(d) xbar
                    if (live[c]) {
                        d2[c] = fma(zv, zv, d2[c]);
                        F.z[(int64_t)(j0 + c) * F.ldz + gi[i]] = (float)zv;
                    }
                }
            }
        }
        carry = seg_combine(carry, lane63_seg(inc));
        if (PF && more) cur = nxt;
        else if (!PF && more) load_chunk(cur, r0 + kColChunk);
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        const double gc = wave_sum(g[c]), s1 = wave_sum(d1[c]), s2 = wave_sum(d2[c]);
        if (lane == 0 && live[c]) {
            double *o = F.cpart + ((int64_t)tt * F.p + j0 + c) * 3;
            o[0] = gc;
            o[1] = s1;
            o[2] = s2;
        }
    }
}

__global__ __launch_bounds__(kWave * kColWaves) void cols_kernel(const FitDesc *fits, const int2 *items, int nitems)
{
    // the item index is the same in all lanes of a wave
    const int item = __builtin_amdgcn_readfirstlane(blockIdx.x * kColWaves + threadIdx.x / kWave);
    if (item >= nitems) return;   // whole wave
    const int2 it = items[item];
    if (!(fit_flags(fits, it.x) & kDone)) cols_item<true>(fits, it);
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

// Wave v's share of item (fit, K range, product): the v-th quarter of the range for every
// tile pair (ti <= tj) of the fit.  Rows of X (event groups of Z) come in steps of 32 -- 16
// consecutive per half-wave, as float4s.  A step loads the fragments of all NT tiles and the
// weights once, then runs each pair's 16 products (A the weighted rows of tile ti, B the rows
// of tile tj) in the order a loop over one pair would, so every pair's sums are those of such
// a loop.  The next step's operands are loaded before this step's products.
template <int NT>
__device__ __forceinline__ void syrk_pairs(const FitDesc &F, int4 it, int v, int lane,
                                           f32x16 (&acc)[NT * (NT + 1) / 2])
{
    constexpr int NP = NT * (NT + 1) / 2;
    constexpr bool PF = true;
    const bool zpart = it.w != 0;
    const float *u = zpart ? F.z : F.xf;
    const int64_t ldu = zpart ? F.ldz : F.ld;
    const int64_t range = zpart ? F.zrange : F.xrange, quarter = range / kSyrkWaves;
    const int64_t k0 = (int64_t)it.z * range + v * quarter;
    // k0 is a multiple of 64 and ldu a multiple of 64: steps of 32 fit exactly
    const int64_t k1 = k0 + quarter < ldu ? k0 + quarter : ldu;
    const int kofs = 16 * (lane >> 5);
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 *ut[NT];
    bool lt[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int row = t * kTile + (lane & 31);
        lt[t] = row < F.p;
        ut[t] = reinterpret_cast<const float4 *>(u + (int64_t)(lt[t] ? row : 0) * ldu + kofs);
    }
    const float4 *uc = zpart ? nullptr : reinterpret_cast<const float4 *>(F.bf + kofs);
#pragma unroll
    for (int pr = 0; pr < NP; ++pr)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[pr][i] = 0.0f;
    float4 fn[NT][4], cn[4];
    auto load = [&](float4(&f)[NT][4], float4(&c)[4], int64_t k) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) f[t][q] = ut[t][k / 4 + q];
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] = uc ? uc[k / 4 + q] : zero4;
    };
    if (PF && k0 < k1) load(fn, cn, k0);
    for (int64_t k = k0; k < k1; k += 32) {
        float4 fv[NT][4], cv[4];
        if (PF) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) fv[t][q] = fn[t][q];
#pragma unroll
            for (int q = 0; q < 4; ++q) cv[q] = cn[q];
            if (k + 32 < k1) load(fn, cn, k + 32);
        } else {
            load(fv, cv, k);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
            if (!lt[t]) {
#pragma unroll
                for (int q = 0; q < 4; ++q) fv[t][q] = zero4;   // rows beyond p (loaded from row 0)
            }
        int pr = 0;
#pragma unroll
        for (int ti = 0; ti < NT; ++ti) {
            float4 av[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                av[q] = fv[ti][q];
                if (uc) {
                    av[q].x *= cv[q].x;
                    av[q].y *= cv[q].y;
                    av[q].z *= cv[q].z;
                    av[q].w *= cv[q].w;
                }
            }
#pragma unroll
            for (int tj = ti; tj < NT; ++tj, ++pr) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    acc[pr] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[q].x, fv[tj][q].x, acc[pr], 0, 0, 0);
                    acc[pr] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[q].y, fv[tj][q].y, acc[pr], 0, 0, 0);
                    acc[pr] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[q].z, fv[tj][q].z, acc[pr], 0, 0, 0);
                    acc[pr] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[q].w, fv[tj][q].w, acc[pr], 0, 0, 0);
                }
            }
        }
    }
}

// Wave v's product over the v-th quarter of the K range of a per-pair item (fit, tile
// pair, K range, product): the same products, in the same order, as syrk_pairs makes for
// that pair.  Rows of X (event groups of Z) come in steps of 32
// -- 16 consecutive per half-wave, as float4s -- with the next step's operands
// loaded before this step's 16 products.
__device__ __forceinline__ f32x16 syrk_partial(const FitDesc &F, int4 it, int v, int lane)
{
    const int nt = tile_count(F.p);
    int ti, tj;
    pair_tiles(it.y, nt, ti, tj);
    const bool zpart = it.w != 0;
    const float *u = zpart ? F.z : F.xf;
    const int64_t ldu = zpart ? F.ldz : F.ld;
    const int64_t range = zpart ? F.zrange : F.xrange, quarter = range / kSyrkWaves;
    const int64_t k0 = (int64_t)it.z * range + v * quarter;
    // k0 is a multiple of 64 and ldu a multiple of 64: steps of 32 fit exactly
    const int64_t k1 = k0 + quarter < ldu ? k0 + quarter : ldu;
    const int ra = ti * kTile + (lane & 31), rb = tj * kTile + (lane & 31);
    const bool la = ra < F.p, lb = rb < F.p;
    const int kofs = 16 * (lane >> 5);
    const float4 *ua = reinterpret_cast<const float4 *>(u + (int64_t)(la ? ra : 0) * ldu + kofs);
    const float4 *ub = reinterpret_cast<const float4 *>(u + (int64_t)(lb ? rb : 0) * ldu + kofs);
    const float4 *uc = zpart ? nullptr : reinterpret_cast<const float4 *>(F.bf + kofs);
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    float4 an[4], bn[4], cn[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) an[q] = bn[q] = cn[q] = zero4;
    if (k0 < k1) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            an[q] = ua[k0 / 4 + q];
            bn[q] = ub[k0 / 4 + q];
            if (uc) cn[q] = uc[k0 / 4 + q];
        }
    }
    for (int64_t k = k0; k < k1; k += 32) {
        float4 av[4], bv[4], cv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            av[q] = an[q];
            bv[q] = bn[q];
            cv[q] = cn[q];
        }
        if (k + 32 < k1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                an[q] = ua[(k + 32) / 4 + q];
                bn[q] = ub[(k + 32) / 4 + q];
                if (uc) cn[q] = uc[(k + 32) / 4 + q];
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (!la) av[q] = zero4;
            if (!lb) bv[q] = zero4;
            if (uc) {
                av[q].x *= cv[q].x;
                av[q].y *= cv[q].y;
                av[q].z *= cv[q].z;
                av[q].w *= cv[q].w;
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[q].x, bv[q].x, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[q].y, bv[q].y, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[q].z, bv[q].z, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[q].w, bv[q].w, acc, 0, 0, 0);
        }
    }
    return acc;
}

constexpr int kSyrkRed = (kSyrkWaves - 1) * 16 * kWave;   // floats of red

// Per-pair item (fit, tile pair, K range, product) for light rounds, where spreading a fit's
// pairs over workgroups shortens the round: the four wave accumulators are added in wave order
// through red, as in syrk_item_nt, so the pair's partial is the same either way.
__device__ void syrk_pair_item(const FitDesc *fits, int4 it, bool live, bool compute, int v, int lane,
                               float *red)
{
    if (!live) return;
    const FitDesc &F = fits[it.x];
    f32x16 acc;
    if (compute) {
        acc = syrk_partial(F, it, v, lane);
        if (v > 0) {
#pragma unroll
            for (int i = 0; i < 16; ++i) red[((v - 1) * 16 + i) * kWave + lane] = acc[i];
        }
    }
    __syncthreads();
    if (compute && v == 0) {
#pragma unroll
        for (int w = 0; w < kSyrkWaves - 1; ++w) {
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[i] += red[(w * 16 + i) * kWave + lane];
        }
        const int slot = it.w != 0 ? F.nxr + it.z : it.z;
        float *out = F.part + ((int64_t)slot * F.npairs + it.y) * (kTile * kTile);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int m = 8 * (i / 4) + 4 * (lane >> 5) + (i % 4), nn = lane & 31;
            out[m * kTile + nn] = acc[i];
        }
    }
    __syncthreads();   // red is rewritten by the next item
}



// Item (fit, K range, product) of a fit with NT tiles: kSyrkWaves waves (v = 0 .. 3) compute;
// in the persistent kernel the workgroup's other waves only keep the barrier count
// (compute = false).  Each pair's four wave accumulators are added in wave order through
// red ([3][16][64] floats), one pair after another, into the pair's partial of the range.
template <int NT>
__device__ __forceinline__ void syrk_item_nt(const FitDesc &F, int4 it, bool compute, int v, int lane,
                                             float *red)
{
    constexpr int NP = NT * (NT + 1) / 2;
    f32x16 acc[NP];
    if (compute) {
        syrk_pairs<NT>(F, it, v, lane, acc);
    } else {
#pragma unroll
        for (int pr = 0; pr < NP; ++pr)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[pr][i] = 0.0f;
    }
    const int slot = it.w != 0 ? F.nxr + it.z : it.z;
#pragma unroll
    for (int pr = 0; pr < NP; ++pr) {
        if (compute && v > 0) {
#pragma unroll
            for (int i = 0; i < 16; ++i) red[((v - 1) * 16 + i) * kWave + lane] = acc[pr][i];
        }
        __syncthreads();
        if (compute && v == 0) {
            f32x16 sum = acc[pr];
#pragma unroll
            for (int w = 0; w < kSyrkWaves - 1; ++w) {
#pragma unroll
                for (int i = 0; i < 16; ++i) sum[i] += red[(w * 16 + i) * kWave + lane];
            }
            float *out = F.part + ((int64_t)slot * F.npairs + pr) * (kTile * kTile);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int m = 8 * (i / 4) + 4 * (lane >> 5) + (i % 4), nn = lane & 31;
                out[m * kTile + nn] = sum[i];
            }
        }
        __syncthreads();   // red is rewritten for the next pair
    }
}

// Item (fit, K range, product); the whole workgroup calls it (the barriers inside depend only
// on the fit's tile count), `live` uniform: false leaves the item out.  Not inlined into the
// persistent kernel, which would otherwise hold the registers of all four tile counts at once.
__device__ __noinline__ void syrk_item(const FitDesc *fits, int4 it, bool live, bool compute, int v, int lane,
                                       float *red)
{
    if (!live) return;
    const FitDesc &F = fits[it.x];
    switch (tile_count(F.p)) {
    case 1: syrk_item_nt<1>(F, it, compute, v, lane, red); break;
    case 2: syrk_item_nt<2>(F, it, compute, v, lane, red); break;
    case 3: syrk_item_nt<3>(F, it, compute, v, lane, red); break;
    default: syrk_item_nt<4>(F, it, compute, v, lane, red); break;   // p <= kMaxP = 128
    }
}

// One workgroup per per-pair item.
__global__ __launch_bounds__(kWave * kSyrkWaves) void syrk_pair_kernel(const FitDesc *fits, const int4 *items)
{
    __shared__ float red[kSyrkRed];
    const int4 it = items[blockIdx.x];
    const bool live = !(fit_flags(fits, it.x) & (kDone | kFrozen));
    syrk_pair_item(fits, it, live, true, threadIdx.x / kWave, threadIdx.x & (kWave - 1), red);
}

// One workgroup per item of a fit with NT tiles (the items come grouped by tile count, so
// each launch holds the registers its own tile count needs).
template <int NT>
__global__ __launch_bounds__(kWave * kSyrkWaves, NT <= 3 ? 2 : 1) void syrk_kernel(const FitDesc *fits,
                                                                                  const int4 *items)
{
    __shared__ float red[kSyrkRed];
    const int4 it = items[blockIdx.x];
    if (fit_flags(fits, it.x) & (kDone | kFrozen)) return;   // the whole workgroup
    syrk_item_nt<NT>(fits[it.x], it, true, threadIdx.x / kWave, threadIdx.x & (kWave - 1), red);
}

// ------------------------------------------------------------------ info

// One workgroup per (fit, tile pair): entry (m, n) of the pair's 32 x 32 block
// of I = X' diag(b) X - Z'Z is the FP64 sum of its K-range partials in range
// order, written to both triangles of F.L (entries below the diagonal of a
// diagonal block are taken from above it).
// Run by 256 threads (t = 0 .. 255); no barrier inside.
__device__ __forceinline__ void info_item(const FitDesc *fits, int2 it, int t)
{
    const FitDesc F = fits[it.x];
    const int nt = tile_count(F.p), p = F.p;
    int ti, tj;
    pair_tiles(it.y, nt, ti, tj);
    const int e0 = t * 4;   // entries e0 .. e0 + 3: one row m, columns n .. n + 3
    double sx[4] = {0.0, 0.0, 0.0, 0.0}, sz[4] = {0.0, 0.0, 0.0, 0.0};
    const float *base = F.part + (int64_t)it.y * (kTile * kTile) + e0;
    const int64_t step = (int64_t)F.npairs * (kTile * kTile);
    for (int r = 0; r < F.nxr; ++r) {
        const float4 q = *reinterpret_cast<const float4 *>(base + r * step);
        sx[0] += (double)q.x;
        sx[1] += (double)q.y;
        sx[2] += (double)q.z;
        sx[3] += (double)q.w;
    }
    for (int r = 0; r < F.nzr; ++r) {
        const float4 q = *reinterpret_cast<const float4 *>(base + (F.nxr + r) * step);
        sz[0] += (double)q.x;
        sz[1] += (double)q.y;
        sz[2] += (double)q.z;
        sz[3] += (double)q.w;
    }
    const int m = e0 / kTile, i = ti * kTile + m;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int n = (e0 % kTile) + q, j = tj * kTile + n;
        if (i < p && j < p && (ti < tj || m <= n)) {
            const double val = sx[q] - sz[q];
            F.L[(int64_t)i * p + j] = val;
            F.L[(int64_t)j * p + i] = val;
        }
    }
}

__global__ __launch_bounds__(256) void info_kernel(const FitDesc *fits, const int2 *items)
{
    const int2 it = items[blockIdx.x];
    if (!(fit_flags(fits, it.x) & (kDone | kFrozen))) info_item(fits, it, threadIdx.x);
}

// ------------------------------------------------------------------ step

constexpr int kStepThreads = 256;

// The step of an l1-penalised fit (proximal Newton): the quadratic model
//   g'D + D'HD/2 + sum_j gamma_j |beta_j + D_j|
// (FP64 score g, information H from the info kernel, kept once frozen) minimised by cyclic
// coordinate descent with soft thresholding (the l1 rule of Sec. 2.4) over the free columns,
// by wave 0 with H in LDS: lane l keeps (HD)_l and (HD)_{l+64} and D_l, D_{l+64} in registers,
// and every lane takes the same decision for coordinate j from values it reads or receives by
// shuffle.  The model is solved to a thousandth of the last step (or of max(1, |beta|) at the
// first), at least to 1e-3 tol.  D goes to y; s_red[w] receives the largest violation of the
// l1 optimality conditions at the current point (wave w's columns).
template <int NT>
__device__ void prox_step(const FitDesc &F, double *A, double *y, const uint8_t *s_free, double *s_red, int t,
                          int wv, int lane)
{
    __shared__ double s_g[kMaxP], s_b[kMaxP], s_gm[kMaxP], s_a[kMaxP];
    const int p = F.p;
    constexpr int kWaves = NT / kWave;
    for (int i = wv; i < p; i += kWaves)
        for (int j = lane; j < p; j += kWave)
            A[i * p + j] = i >= j ? F.L[(int64_t)i * p + j] : F.L[(int64_t)j * p + i];   // lower triangle, mirrored
    double viol = 0.0, bmax = 1.0;
    for (int j = t; j < p; j += NT) {
        const double g = F.grad[j], b = F.beta[j], gm = F.gam[j], a = F.L[(int64_t)j * p + j];
        s_g[j] = g;
        s_b[j] = b;
        s_gm[j] = gm;
        s_a[j] = (s_free[j] && a > 0.0) ? a : 0.0;   // 0: the coordinate stays
        bmax = fmax(bmax, fabs(b));
        if (!s_free[j]) continue;
        const double r = gm <= 0.0 ? fabs(g) : (b != 0.0 ? fabs(g + (b > 0.0 ? gm : -gm)) : fmax(fabs(g) - gm, 0.0));
        viol = fmax(viol, r);
    }
    viol = wave_max(viol);
    bmax = wave_max(bmax);
    __shared__ double s_bm[NT / kWave];
    if (lane == 0) {
        s_red[wv] = viol;
        s_bm[wv] = bmax;
    }
    __syncthreads();
    if (wv == 0) {
        const FitState *st = F.st;
        double bm = 1.0;
        for (int k = 0; k < kWaves; ++k) bm = fmax(bm, s_bm[k]);
        const double tol = fmax(1e-3 * F.tol * bm, st->iters ? 1e-3 * st->last_step : 1e-3 * bm);
        double hd0 = 0.0, hd1 = 0.0, d0 = 0.0, d1 = 0.0;
        for (int sweep = 0; sweep < 1000; ++sweep) {
            double change = 0.0;
            for (int j = 0; j < p; ++j) {
                const double a = s_a[j];
                if (a == 0.0) continue;
                const int src = j & (kWave - 1);
                const double hj = lane_value(j < kWave ? hd0 : hd1, src);
                const double dj = lane_value(j < kWave ? d0 : d1, src);
                const double bj = s_b[j], gm = s_gm[j];
                const double bb = s_g[j] + hj - a * dj;   // the model's slope at D with D_j removed
                const double u = a * bj - bb;
                const double z = u > gm ? (u - gm) / a : (u < -gm ? (u + gm) / a : 0.0);
                const double dn = z - bj;
                const double delta = dn - dj;
                if (delta != 0.0) {
                    if (lane == src) {
                        if (j < kWave) d0 = dn;
                        else d1 = dn;
                    }
                    if (lane < p) hd0 = fma(A[j * p + lane], delta, hd0);
                    if (lane + kWave < p) hd1 = fma(A[j * p + lane + kWave], delta, hd1);
                    change = fmax(change, fabs(delta));
                }
            }
            if (change <= tol) break;
        }
        if (lane < p) y[lane] = d0;
        if (lane + kWave < p) y[lane + kWave] = d1;
    }
}

// The fit's state goes to host-mapped memory with kDone set last, after a system-scope
// fence: a host that finds kDone while kernels still run reads the rest of the state, and
// the estimate written before it, complete.
__device__ __forceinline__ void publish_state(const FitDesc &F, const FitState &st)
{
    FitState v = st;
    const int flags = v.flags;
    v.flags = flags & ~kDone;
    *F.hst = v;
    if (flags & kDone) {
        __threadfence_system();
        __hip_atomic_store(&F.hst->flags, flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Every entry of beta to host-mapped memory (each thread the entries it owns), then the
// state; ndone (if given) counts the fits that finished.
template <int NT>
__device__ __forceinline__ void publish_final(const FitDesc &F, const FitState *st, int t, uint32_t *ndone)
{
    for (int j = t; j < F.p; j += NT) F.hbeta[j] = F.beta[j];
    __threadfence_system();
    __syncthreads();
    if (t == 0) {
        publish_state(F, *st);
        if (ndone) __hip_atomic_fetch_add(ndone, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// One fit's step, run by NT threads (the whole workgroup) with lds = A[p * p], y[p].
template <int NT>
__device__ __forceinline__ void step_fit(const FitDesc *fits, int slot, double *lds, uint32_t *ndone)
{
    __shared__ int s_action, s_bad, s_frozen;
    __shared__ uint8_t s_free[kMaxP];
    __shared__ double s_red[NT / kWave];
    __syncthreads();   // the shared words of the previous fit have been read
    const FitDesc F = fits[slot];
    FitState *st = F.st;
    const int t = threadIdx.x, p = F.p;
    double *A = lds;
    double *y = lds + (int64_t)p * p;

    // per-column sums of the scan-tile partials, and the objective, in tile order; with l1
    // weights the objective includes sum_j gamma_j |beta_j| (summed by wave 0 in column order)
    for (int j = t; j < p; j += NT) {
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
        if (F.gam)
            for (int j = 0; j < p; ++j) o += F.gam[j] * fabs(F.beta[j]);
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
    if (action == 0) {   // final: the estimate and the state go to the host
        publish_final<NT>(F, st, t, ndone);
        return;
    }
    if (action == 1) {
        for (int j = t; j < p; j += NT) F.beta[j] = F.prev[j] + 0.5 * (F.beta[j] - F.prev[j]);
        if (t == 0) publish_state(F, *st);
        return;
    }
    // the columns that move: chosen once, at the first evaluation (g'' > 1e-12 S2-term)
    if (!(st->flags & kHaveFree)) {
        __shared__ int s_moved;
        if (t == 0) s_moved = 0;
        __syncthreads();
        for (int j = t; j < p; j += NT) {
            const double hd = F.diag1[j] - F.diag2[j];
            const bool fr = hd > 1e-12 * fabs(F.diag1[j]) && isfinite(hd);
            F.free_col[j] = fr ? 1 : 0;
            if (F.gam && !fr && F.beta[j] != 0.0) {   // l1 fits hold such columns at zero
                F.beta[j] = 0.0;
                F.prev[j] = 0.0;
                s_moved = 1;
            }
        }
        __syncthreads();
        if (s_moved) {   // evaluate again at the start point with those columns at zero
            if (t == 0) {
                st->flags |= kHaveFree;
                publish_state(F, *st);
            }
            return;
        }
    }
    const bool frozen = s_frozen != 0;
    const int wv = t / kWave, lane = t & (kWave - 1);
    constexpr int kWaves = NT / kWave;
    for (int j = t; j < p; j += NT) s_free[j] = F.free_col[j];
    __syncthreads();
    if (F.gam) {
        prox_step<NT>(F, A, y, s_free, s_red, t, wv, lane);
    } else if (!frozen) {
        // Blocked right-looking Cholesky of the information matrix (info kernel; rows and
        // columns not free become unit rows) in LDS, lower triangle, panels of 16 columns:
        // wave 0 factors the diagonal block (lane r holds its row r, columns passed by
        // shuffles), every thread solves rows below it against that block, and the threads
        // update the trailing triangle in 4 x 4 tiles -- three barriers per panel.
        constexpr int NB = 16;
        for (int i = wv; i < p; i += kWaves)
            for (int j = lane; j <= i; j += kWave) {
                double v = F.L[(int64_t)i * p + j];
                if (!s_free[i] || !s_free[j]) v = (i == j) ? 1.0 : 0.0;
                A[i * p + j] = v;
            }
        __syncthreads();
        for (int k0 = 0; k0 < p; k0 += NB) {
            const int kb = p - k0 < NB ? p - k0 : NB;
            if (wv == 0) {
                double r[NB];
#pragma unroll
                for (int c = 0; c < NB; ++c) r[c] = (lane < kb && c <= lane) ? A[(k0 + lane) * p + k0 + c] : 0.0;
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    if (c < kb) {
                        double d = lane_value(r[c], c);
                        const bool ok = d > 0.0;
                        if (!ok) {
                            d = 1.0;
                            if (lane == 0) s_bad = 1;
                        }
                        const double piv = sqrt(d), inv = 1.0 / piv;
                        r[c] = lane == c ? piv : (lane > c ? r[c] * inv : r[c]);
                        const double lc = r[c];   // L[k0 + lane][k0 + c] below the pivot
#pragma unroll
                        for (int cc = c + 1; cc < NB; ++cc) {
                            const double lcc = lane_value(lc, cc);   // L[k0 + cc][k0 + c]
                            if (cc < kb && lane >= cc) r[cc] = fma(-lc, lcc, r[cc]);
                        }
                    }
                }
#pragma unroll
                for (int c = 0; c < NB; ++c)
                    if (lane < kb && c <= lane) A[(k0 + lane) * p + k0 + c] = r[c];
            }
            __syncthreads();
            // rows below the block: x L_kk' = A[i][k0 .. k0 + kb)
            for (int i = k0 + kb + t; i < p; i += NT) {
                double x[NB];
#pragma unroll
                for (int c = 0; c < NB; ++c) x[c] = c < kb ? A[i * p + k0 + c] : 0.0;
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    if (c < kb) {
                        double v = x[c];
#pragma unroll
                        for (int cc = 0; cc < c; ++cc) v = fma(-x[cc], A[(k0 + c) * p + k0 + cc], v);
                        x[c] = v / A[(k0 + c) * p + k0 + c];
                    }
                }
#pragma unroll
                for (int c = 0; c < NB; ++c)
                    if (c < kb) A[i * p + k0 + c] = x[c];
            }
            __syncthreads();
            // trailing triangle rows/columns m0 .. p-1, 4 x 4 tiles (ti >= tj)
            const int m0 = k0 + kb, mt = (p - m0 + 3) / 4;
            const int ntile = mt * (mt + 1) / 2;
            for (int q = t; q < ntile; q += NT) {
                int ti = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
                while (ti * (ti + 1) / 2 > q) --ti;
                while ((ti + 1) * (ti + 2) / 2 <= q) ++ti;
                const int tj = q - ti * (ti + 1) / 2;
                const int i0 = m0 + 4 * ti, j0 = m0 + 4 * tj;
                double acc[4][4];
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int s2 = 0; s2 < 4; ++s2) acc[r][s2] = 0.0;
                for (int c = 0; c < kb; ++c) {
                    double av[4], bv[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        av[r] = i0 + r < p ? A[(i0 + r) * p + k0 + c] : 0.0;
                        bv[r] = j0 + r < p ? A[(j0 + r) * p + k0 + c] : 0.0;
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int s2 = 0; s2 < 4; ++s2) acc[r][s2] = fma(av[r], bv[s2], acc[r][s2]);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int s2 = 0; s2 < 4; ++s2) {
                        const int i = i0 + r, j = j0 + s2;
                        if (i < p && j <= i) A[i * p + j] -= acc[r][s2];
                    }
            }
            __syncthreads();
        }
        for (int i = wv; i < p; i += kWaves)
            for (int j = lane; j <= i; j += kWave) F.L[(int64_t)i * p + j] = A[i * p + j];
        __syncthreads();
    } else {
        for (int i = wv; i < p; i += kWaves)
            for (int j = lane; j < p; j += kWave) A[i * p + j] = F.L[(int64_t)i * p + j];
    }
    if (!F.gam) {
        // score on the free columns; kkt = max |score|
        double kk = 0.0;
        for (int j = t; j < p; j += NT) {
            const double gj = s_free[j] ? F.grad[j] : 0.0;
            y[j] = -gj;
            kk = fmax(kk, fabs(gj));
        }
        kk = wave_max(kk);
        if (lane == 0) s_red[wv] = kk;
        __syncthreads();
        // L y = -g, then L' dx = y, by wave 0: lane l holds entries l and l + 64
        if (wv == 0) {
            double y0 = lane < p ? y[lane] : 0.0, y1 = lane + kWave < p ? y[lane + kWave] : 0.0;
            for (int k = 0; k < p; ++k) {
                const double own = k < kWave ? y0 : y1;
                const double yk = lane_value(own, k & (kWave - 1)) / A[k * p + k];
                if (lane == (k & (kWave - 1))) {
                    if (k < kWave) y0 = yk;
                    else y1 = yk;
                }
                if (lane > k && lane < p) y0 -= A[lane * p + k] * yk;
                if (lane + kWave > k && lane + kWave < p) y1 -= A[(lane + kWave) * p + k] * yk;
            }
            for (int k = p - 1; k >= 0; --k) {
                const double own = k < kWave ? y0 : y1;
                const double xk = lane_value(own, k & (kWave - 1)) / A[k * p + k];
                if (lane == (k & (kWave - 1))) {
                    if (k < kWave) y0 = xk;
                    else y1 = xk;
                }
                if (lane < k) y0 -= A[k * p + lane] * xk;
                if (lane + kWave < k) y1 -= A[k * p + lane + kWave] * xk;
            }
            if (lane < p) y[lane] = y0;
            if (lane + kWave < p) y[lane + kWave] = y1;
        }
    }
    __syncthreads();
    double smax = 0.0, bmax = 0.0;
    for (int j = t; j < p; j += NT) {
        const double dx = s_free[j] ? y[j] : 0.0;
        const double b0 = F.beta[j];
        const double b1 = b0 + dx;
        F.prev[j] = b0;
        F.beta[j] = b1;
        smax = fmax(smax, fabs(dx));
        bmax = fmax(bmax, fabs(b1));
    }
    smax = wave_max(smax);
    bmax = wave_max(bmax);
    __shared__ double s_s[NT / kWave], s_b[NT / kWave];
    if ((t & (kWave - 1)) == 0) {
        s_s[t / kWave] = smax;
        s_b[t / kWave] = bmax;
    }
    __syncthreads();
    if (t == 0) {
        double step = 0.0, bm = 1.0, kkt = 0.0;
        for (int k = 0; k < NT / kWave; ++k) {
            step = fmax(step, s_s[k]);
            bm = fmax(bm, s_b[k]);
            kkt = fmax(kkt, s_red[k]);
        }
        int flags = st->flags | kHaveFree;
        int pinned = 0;
        for (int j = 0; j < p; ++j) pinned += s_free[j] ? 0 : 1;
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
        s_action = (flags & kDone) ? 1 : 0;
    }
    __syncthreads();
    if (s_action) {   // final: every thread sends the entries of beta it wrote, then the state
        publish_final<NT>(F, st, t, ndone);
    } else if (t == 0) {
        publish_state(F, *st);
    }
}

__global__ __launch_bounds__(kStepThreads) void step_kernel(const FitDesc *fits, const int *slots)
{
    extern __shared__ double lds[];   // A[p * p], y[p]
    const int slot = slots[blockIdx.x];
    if (fit_flags(fits, slot) & kDone) return;   // the whole workgroup
    step_fit<kStepThreads>(fits, slot, lds, nullptr);
}

// ------------------------------------------------------------------ persistent rounds

// Control block of one persistent launch (device memory, cleared before the launch).
struct RoundCtl {
    SyncCtl sync;                  // abort word of the bounded waits
    uint32_t ndone;                // fits that finished during the launch
    uint32_t hold[2];              // the host's hold word as workgroup 0 read it, by round parity
    uint32_t pad[61];
    Packet arrive[kRoundMaxGrid];  // epoch of the last barrier each workgroup reached
};

// Grid-wide barrier of the persistent round kernel.  Every wave waits for its
// stores to reach the L2 of its XCD; one thread per workgroup then writes that
// L2 back (agent-scope fence: the XCDs' L2 caches are kept coherent only
// through such fences, and one write-back covers the stores of all the
// workgroup's waves) and publishes its arrival packet; wave 0 of every
// workgroup polls all arrival packets (a workgroup that has gone on to a later
// barrier counts as arrived) and fences again before anything written by
// another workgroup is read.  At the barrier that ends a round every workgroup
// takes the same decision from the same data: go on while rounds remain, fits
// remain unfinished (the counter the step phase raises) and the host had not
// asked for the launch to end when workgroup 0 arrived (its reading of the hold
// word, stored before its arrival).  Every wait is bounded.  Returns 1 to go
// on, 0 to stop, -1 when a wait timed out.
__device__ int round_barrier(const RoundWork &w, RoundCtl *ctl, uint32_t epoch, bool end_of_round, int round,
                             int *s_word)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int t = threadIdx.x;
    const PacketArray arrive = packet_array(ctl->arrive, sizeof(Packet) * gridDim.x);
    if (t == 0) {
        if (end_of_round && blockIdx.x == 0) {
            const uint32_t h = __hip_atomic_load(w.hold, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&ctl->hold[round & 1], h != 0u ? 1u : 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __threadfence();
        packet_put(arrive, blockIdx.x, 0.0, epoch, 0u);
    }
    if (t < kWave) {
        bool ok = true;
        for (int k = t; k < (int)gridDim.x && ok; k += kWave) {
            WaitBudget wb;
            while (packet_get(arrive, (uint32_t)k).z < epoch)
                if (!wb.keep_waiting(&ctl->sync)) {
                    ok = false;
                    break;
                }
        }
        const bool all_ok = __all(ok ? 1 : 0) != 0;
        if (t == 0) {
            int go = -1;
            if (all_ok) {
                __threadfence();
                go = 1;
                if (end_of_round) {
                    const uint32_t nd = __hip_atomic_load(&ctl->ndone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t hold = __hip_atomic_load(&ctl->hold[round & 1], __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                    go = (round + 1 < w.max_rounds && (int)nd < w.nf && hold == 0u) ? 1 : 0;
                }
            }
            *s_word = go;
        }
    }
    __syncthreads();
    const int go = *s_word;
    __syncthreads();   // s_word is rewritten by the next barrier
    return go;
}

// Persistent round kernel: up to max_rounds Newton iterations of every fit in the work
// lists, the six phases of a round separated by grid-wide barriers (one cooperative
// launch; every workgroup resident).  Each phase's items are dealt out over the workgroups
// first (eta, syrk, info: to half-workgroups of 256 threads; cols: to waves; rows and step:
// to whole workgroups), so a light phase spreads over many CUs, and run the same bodies as
// the separate launches, so every fit's sums are the same.  Fits that finish are left out of the later rounds, fits whose information
// matrix is frozen out of the contraction.  lds: the step's A[p * p], y[p], and during the
// contraction the two half-workgroups' reduction buffers.
__global__ __launch_bounds__(kRoundThreads) void round_kernel(RoundWork w)
{
    extern __shared__ double lds[];
    __shared__ double s_eta_red[2][kEtaRows / kWave];
    __shared__ int s_word;
    RoundCtl *ctl = static_cast<RoundCtl *>(w.ctl);
    const int t = threadIdx.x, half = t / 256, th = t & 255, lane = t & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(t / kWave);
    const int G = gridDim.x, b = blockIdx.x;
    constexpr int kWaves = kRoundThreads / kWave;
    uint32_t epoch = 0;
    int rounds = 0, status = 0;
    // workgroup 0 times the phases between barrier releases (constant-rate clock)
    __shared__ uint64_t s_ticks[7];   // six phases, then the last release
    const bool timer = b == 0 && t == 0;
    if (timer) {
        for (int k = 0; k < 6; ++k) s_ticks[k] = 0;
        s_ticks[6] = wall_clock64();
    }
    auto lap = [&](int ph) {
        if (timer) {
            const uint64_t now = wall_clock64();
            s_ticks[ph] += now - s_ticks[6];
            s_ticks[6] = now;
        }
    };
    for (int round = 0;; ++round) {
        // X beta: half-workgroup items
        for (int base = 0; base < w.ne; base += 2 * G) {
            const int i = __builtin_amdgcn_readfirstlane(base + half * G + b);
            int2 it = make_int2(0, 0);
            bool live = false;
            if (i < w.ne) {
                it = w.eta[i];
                live = !(fit_flags(w.fits, it.x) & kDone);
            }
            eta_item(w.fits, it, live, th, s_eta_red[half]);
        }
        if (round_barrier(w, ctl, ++epoch, false, round, &s_word) < 0) {
            status = -1;
            break;
        }
        lap(0);
        // row scans: workgroup items
        for (int i = b; i < w.nr; i += G) {
            const int2 it = w.rows[i];
            if (!(fit_flags(w.fits, it.x) & kDone)) rows_item(w.fits, it);
        }
        if (round_barrier(w, ctl, ++epoch, false, round, &s_word) < 0) {
            status = -1;
            break;
        }
        lap(1);
        // column pass: wave items
        for (int i = wv * G + b; i < w.nc; i += kWaves * G) {
            const int2 it = w.cols[i];
            if (!(fit_flags(w.fits, it.x) & kDone)) cols_item<false>(w.fits, it);
        }
        if (round_barrier(w, ctl, ++epoch, false, round, &s_word) < 0) {
            status = -1;
            break;
        }
        lap(2);
        if (w.ns > 0) {
            // contraction: workgroup items, computed by waves 0-3 (the others keep the barriers)
            float *red = reinterpret_cast<float *>(lds);
            for (int i = b; i < w.ns; i += G) {
                const int4 it = w.syrk[i];
                const bool live = !(fit_flags(w.fits, it.x) & (kDone | kFrozen));
                if (w.syrk_per_pair) syrk_pair_item(w.fits, it, live, wv < kSyrkWaves, wv & (kSyrkWaves - 1), lane, red);
                else syrk_item(w.fits, it, live, wv < kSyrkWaves, wv & (kSyrkWaves - 1), lane, red);
            }
            if (round_barrier(w, ctl, ++epoch, false, round, &s_word) < 0) {
                status = -1;
                break;
            }
            lap(3);
            for (int base = 0; base < w.ni; base += 2 * G) {
                const int i = __builtin_amdgcn_readfirstlane(base + half * G + b);
                if (i < w.ni) {
                    const int2 it = w.info[i];
                    if (!(fit_flags(w.fits, it.x) & (kDone | kFrozen))) info_item(w.fits, it, th);
                }
            }
            if (round_barrier(w, ctl, ++epoch, false, round, &s_word) < 0) {
                status = -1;
                break;
            }
            lap(4);
        }
        // step: workgroup items
        for (int i = b; i < w.nf; i += G) {
            const int slot = w.slots[i];
            if (!(fit_flags(w.fits, slot) & kDone)) step_fit<kRoundThreads>(w.fits, slot, lds, &ctl->ndone);
        }
        const int go = round_barrier(w, ctl, ++epoch, true, round, &s_word);
        if (go < 0) {
            status = -1;
            break;
        }
        lap(5);
        rounds = round + 1;
        if (go == 0) break;
    }
    if (b == 0 && t == 0) {
        w.hout[0] = (uint64_t)rounds;
        w.hout[1] = status < 0 ? 1u : 0u;
        for (int k = 0; k < 6; ++k) w.hout[2 + k] = s_ticks[k];
    }
}

}  // namespace

int launch_admit(FitDesc *fits, const FitDesc *joining, const int *slots, const int2 *items, int nitems,
                 hipStream_t s)
{
    if (nitems > 0) admit_kernel<<<nitems, 256, 0, s>>>(fits, joining, slots, items);
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

int launch_syrk(const FitDesc *fits, const int4 *items, const int *counts, hipStream_t s)
{
    const int4 *at = items;
    if (counts[0] > 0) syrk_pair_kernel<<<counts[0], kWave * kSyrkWaves, 0, s>>>(fits, at);
    at += counts[0];
    if (counts[1] > 0) syrk_kernel<1><<<counts[1], kWave * kSyrkWaves, 0, s>>>(fits, at);
    at += counts[1];
    if (counts[2] > 0) syrk_kernel<2><<<counts[2], kWave * kSyrkWaves, 0, s>>>(fits, at);
    at += counts[2];
    if (counts[3] > 0) syrk_kernel<3><<<counts[3], kWave * kSyrkWaves, 0, s>>>(fits, at);
    at += counts[3];
    if (counts[4] > 0) syrk_kernel<4><<<counts[4], kWave * kSyrkWaves, 0, s>>>(fits, at);
    return (int)hipGetLastError();
}

int launch_info(const FitDesc *fits, const int2 *items, int nitems, hipStream_t s)
{
    if (nitems > 0) info_kernel<<<nitems, 256, 0, s>>>(fits, items);
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

size_t round_ctl_bytes() { return sizeof(RoundCtl); }

size_t round_lds_bytes(int max_p)
{
    const size_t step = sizeof(double) * ((size_t)max_p * max_p + max_p);
    const size_t red = sizeof(float) * 2 * kSyrkRed;
    return step > red ? step : red;
}

int round_grid(int max_p, int *grid)
{
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&round_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)round_lds_bytes(kMaxP));
        if (e != hipSuccess) return (int)e;
        attr_set = true;
    }
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(&round_kernel),
                                                         kRoundThreads, round_lds_bytes(max_p));
    if (e != hipSuccess) return (int)e;
    const int g = cus * per_cu;
    *grid = g < kRoundMaxGrid ? g : kRoundMaxGrid;
    return 0;
}

int launch_rounds(const RoundWork &w, int grid, hipStream_t s)
{
    if (w.nf <= 0 || grid < 1 || grid > kRoundMaxGrid) return (int)hipErrorInvalidValue;
    RoundWork a = w;
    void *args[] = {(void *)&a};
    hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&round_kernel), dim3((unsigned)grid),
                                              dim3(kRoundThreads), args, (unsigned)round_lds_bytes(w.max_p), s);
    return (int)e;
}

}  // namespace serve
}  // namespace coxmi
