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
// Efron's tie correction (Efron 1977; the paper's risk sets are Breslow's): the l-th of the
// d events of group g sees A_l = S0_g - (l/d) E0_g, E the sums over the group's own events.
// With h_g = sum_l 1/A_l and k_g = sum_l (l/d)/A_l the same exchange of sums gives
//   gradient     = X'(w o c - delta),  c_r = sum_{g: r in R_g} h_g - delta_r k_{g(r)}
//   Hessian      = X' diag(w o c) X - sum_g [S1 E1] M_g [S1 E1]',  M_g = sum_l (1, -a_l)(1, -a_l)' / A_l^2
//   objective    = -delta'eta + sum_g sum_l (log A_l + c)
// and M_g = L L' (2 x 2 Cholesky) turns each group's term into two rows of Z: l11 S1 + l21 E1
// and l22 E1.  For d = 1, a_0 = 0 and these are the plain terms (h = 1/S0, one row S1/S0), so
// E1 is needed only for the groups with two or more events, whose event rows are listed.
//
// All kernels here are ordinary launches (no cross-workgroup waits).
#include <hip/hip_bf16.h>
#include <math.h>

#include <type_traits>

#include "internal.h"
#include "newton.h"
#include "affscan.hpp"
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

// eta = X beta over all ld rows.
__global__ __launch_bounds__(kRowBlock) void eta_kernel(const double *x, int64_t ld, int p, const double *beta,
                                                        double *eta)
{
    const int64_t r = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (r < ld) {
        double e = 0.0;
        for (int j = 0; j < p; ++j) {
            const double bj = beta[j];
            if (bj != 0.0) e = fma(x[(int64_t)j * ld + r], bj, e);
        }
        eta[r] = e;
    }
}

// With m the running maximum of eta within the stratum: alpha_r =
// exp(m_{r-1} - m_r) (1 at a head) and u_r = exp(eta_r - m_r), both in (0, 1].
__global__ __launch_bounds__(kRowBlock) void prep_kernel(const double *eta, const double *m, const uint32_t *meta,
                                                         int64_t ld, double *alpha, double *u)
{
    const int64_t r = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (r < ld) {
        const double mr = m[r];
        alpha[r] = (meta[r] & kHeadBit) ? 1.0 : exp(m[r - 1] - mr);
        u[r] = exp(eta[r] - mr);
    }
}

// At event-group ends, with S0' = S0 exp(-m) in [1, n]: h' = d / S0', its
// objective part d (log S0' + m), and zq = h' / sqrt(d) (so that
// sqrt(d) xbar_j = S1'_j zq and d xbar_j^2 = (S1'_j zq)^2: no division per
// column); -eta at event rows.  A non-finite S0' (non-finite X beta) is flagged.
__global__ __launch_bounds__(kRowBlock) void hazard_kernel(const double *s0, const double *eta, const double *m,
                                                           const uint32_t *meta, int64_t ld, double *h, double *zq,
                                                           double *blockobj, unsigned *flags)
{
    __shared__ double red[kRowBlock / kWave];
    const int64_t r = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    double obj = 0.0;
    if (r < ld) {
        const uint32_t mw = meta[r];
        const uint32_t d = mw & kCountMask;
        double hv = 0.0, qv = 0.0;
        if (d != 0u) {
            const double s = s0[r];
            if (!(s >= 0.5) || !(s <= 1e300)) atomicOr(flags, 1u);
            hv = (double)d / s;
            qv = hv / sqrt((double)d);
            obj += (double)d * (log(s) + m[r]);
        }
        if (mw & kEventBit) obj -= eta[r];
        h[r] = hv;
        zq[r] = qv;
    }
    obj = block_sum(obj, red);
    if (threadIdx.x == 0) blockobj[blockIdx.x] = obj;
}

// b = w Lambda = u R, with R the reverse recurrence of h' (relative to exp(m_r))
__global__ __launch_bounds__(kRowBlock) void rowweight_kernel(const double *u, const double *R, int64_t ld, double *b)
{
    const int64_t r = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (r < ld) b[r] = u[r] * R[r];
}

// Efron at event-group ends, everything relative to exp(m_r) as above: A'_l = S0' - (l/d) E0',
// h' = sum_l 1/A'_l, k' = sum_l (l/d)/A'_l, objective sum_l (log A'_l + m), and the factor of
// M' = sum_l (1, -a_l)(1, -a_l)' / A'_l^2 (l11 in zq, l21, l22); -eta at event rows.
__global__ __launch_bounds__(kRowBlock) void hazard_efron_kernel(const double *s0, const double *e0, const double *eta,
                                                                 const double *m, const uint32_t *meta, int64_t ld,
                                                                 double *h, double *kq, double *zq, double *zq2,
                                                                 double *zq3, double *blockobj, unsigned *flags)
{
    __shared__ double red[kRowBlock / kWave];
    const int64_t r = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    double obj = 0.0;
    if (r < ld) {
        const uint32_t mw = meta[r];
        const uint32_t d = mw & kCountMask;
        double hv = 0.0, kv = 0.0, l11 = 0.0, l21 = 0.0, l22 = 0.0;
        if (d != 0u) {
            const double s = s0[r], ev = e0[r], mr = m[r], dd = (double)d;
            if (!(s >= 0.5) || !(s <= 1e300)) atomicOr(flags, 1u);
            double m11 = 0.0, m21 = 0.0, m22 = 0.0;
            for (uint32_t l = 0; l < d; ++l) {
                const double a = (double)l / dd;
                const double A = s - a * ev;
                const double iA = 1.0 / A, iA2 = iA * iA;
                hv += iA;
                kv += a * iA;
                m11 += iA2;
                m21 -= a * iA2;
                m22 += a * a * iA2;
                obj += log(A) + mr;
            }
            l11 = sqrt(m11);
            l21 = m21 / l11;
            l22 = sqrt(fmax(m22 - l21 * l21, 0.0));
        }
        if (mw & kEventBit) obj -= eta[r];
        h[r] = hv;
        kq[r] = kv;
        zq[r] = l11;
        zq2[r] = l21;
        zq3[r] = l22;
    }
    obj = block_sum(obj, red);
    if (threadIdx.x == 0) blockobj[blockIdx.x] = obj;
}

// b = w c = u R - delta exp(eta - m_e) k'_e, e the end row of the row's tie group
__global__ __launch_bounds__(kRowBlock) void rowweight_efron_kernel(const double *u, const double *R, const double *eta,
                                                                    const double *m, const double *kq,
                                                                    const int32_t *gend, int64_t ld, double *b)
{
    const int64_t r = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (r < ld) {
        double v = u[r] * R[r];
        const int32_t e = gend[r];
        if (e >= 0) v -= exp(eta[r] - m[e]) * kq[e];
        b[r] = v;
    }
}

// me_w[q] = exp(eta - m_end) of the listed event rows of the multi-event groups
__global__ __launch_bounds__(kRowBlock) void efron_w_kernel(const double *eta, const double *m, const int32_t *me_ptr,
                                                            const int32_t *me_row, const int32_t *me_end,
                                                            int64_t n_multi, double *me_w)
{
    const int64_t k = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (k < n_multi) {
        const double me = m[me_end[k]];
        for (int32_t q = me_ptr[k]; q < me_ptr[k + 1]; ++q) me_w[q] = exp(eta[me_row[q]] - me);
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

// agg[t][j] = the map S -> A S + B of the rows of tile t from its last head (or
// its first row) to its end for the recurrence S'_r = alpha_r S'_{r-1} + u_r x_rj
// (stored as A, B), for the tiles listed in `tiles`.
__global__ __launch_bounds__(kWave * kColWaves) void colagg_kernel(const double *x, int64_t ld, int p, const double *alpha,
                                                                   const double *u, const uint32_t *meta, int64_t tile,
                                                                   const int32_t *tiles, int ntl,
                                                                   const int32_t *lasthead, double *agg)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int item = __builtin_amdgcn_readfirstlane(blockIdx.x * kColWaves + threadIdx.x / kWave);
    if (item >= ntl * p) return;
    const int t = tiles[item / p], j = item % p;
    const int64_t r1 = (int64_t)(t + 1) * tile;
    const int64_t r0 = lasthead[t] >= 0 ? (int64_t)lasthead[t] : (int64_t)t * tile;
    const double *xj = x + (int64_t)j * ld;
    AffE acc = AffOp::id();
    for (int64_t base = r0; base < r1; base += kWave) {
        const int64_t r = base + lane;
        AffE e = AffOp::id();
        if (r < r1) e = AffE{(meta[r] & kHeadBit) ? 1u : 0u, alpha[r], u[r] * xj[r]};
        const AffE tot = lane63_e(wave_scan_e<AffOp>(e));
        acc = AffOp::combine(acc, tot);
    }
    if (lane == 0) {
        agg[((int64_t)t * p + j) * 2] = acc.a;
        agg[((int64_t)t * p + j) * 2 + 1] = acc.b;
    }
}

// carry[t][j] = S'_j entering tile t (for tiles whose first row continues a
// stratum).  One thread per column, tiles in order.
__global__ __launch_bounds__(256) void colcarry_kernel(int p, int ntiles, const uint8_t *tile_carry,
                                                       const int32_t *lasthead, const double *agg, double *carry)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= p) return;
    double c = 0.0;
    for (int t = 0; t < ntiles; ++t) {
        carry[(int64_t)t * p + j] = c;
        if (t + 1 < ntiles && tile_carry[t + 1]) {
            const double A = agg[((int64_t)t * p + j) * 2], B = agg[((int64_t)t * p + j) * 2 + 1];
            c = lasthead[t] >= 0 ? B : fma(A, c, B);
        } else {
            c = 0.0;
        }
    }
}

// kColBlock columns per wave: the row vectors (alpha, u, b, zq, row words,
// group indices) are loaded once per chunk for all of them, and the
// column-independent parts (flags, products of alpha) of the wave scan are
// formed once.
constexpr int kColBlock = 4;

// One DPP step of the shared-multiplier scan: every column's b uses the same
// (f, a) of the element it extends.
template <int CTRL, int ROWS, int CB>
__device__ __forceinline__ void aff_step(uint32_t &f, double &a, double (&b)[CB])
{
    const uint32_t sf = dpp_keep_u32<CTRL, ROWS>(0u, f);
    const double sa = dpp_keep<CTRL, ROWS>(1.0, a);
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        const double sb = dpp_keep<CTRL, ROWS>(0.0, b[c]);
        b[c] = f ? b[c] : fma(a, sb, b[c]);
    }
    a = f ? a : sa * a;
    f = f | sf;
}

// EFRON: at the end of a group with two or more events S1' goes to s1me (its rows of Z
// are formed with E1 by efron_z_kernel); the other groups' rows are the plain ones.
template <typename ZT, bool XBAR, bool EFRON>
__global__ __launch_bounds__(kWave * kColWaves) void colpass_kernel(const double *x, int64_t ld, int p, int64_t tile,
                                                                    int ntiles, const double *alpha, const double *u,
                                                                    const double *zq, const double *b,
                                                                    const uint32_t *meta, const int32_t *gidx,
                                                                    const uint8_t *tile_carry, const double *carry,
                                                                    int64_t ldz, const float *zscale, ZT *z, double *part,
                                                                    const int32_t *gidx2, double *s1me)
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
    double g[CB], d1[CB], d2[CB], cb[CB];   // cb: S'_j entering the chunk
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        const int j = j0 + c;
        live[c] = j < p;
        xc[c] = x + (int64_t)(live[c] ? j : j0) * ld;
        zs[c] = (zscale && live[c]) ? 1.0f / zscale[j] : 1.0f;
        g[c] = d1[c] = d2[c] = 0.0;
        cb[c] = (XBAR && live[c] && tile_carry[t]) ? carry[(int64_t)t * p + j] : 0.0;
    }
    // one chunk's loads: 4 consecutive rows per lane (16-byte loads); the next
    // chunk's loads are issued before this chunk is processed
    struct Chunk {
        double xv[CB][kColIpt], bv[kColIpt], av[kColIpt], uv[kColIpt], qv[kColIpt];
        uint32_t m[kColIpt];
        int32_t gi[kColIpt], g2[EFRON ? kColIpt : 1];
    };
    auto load_chunk = [&](Chunk &k, int64_t r0) {
#pragma unroll
        for (int c = 0; c < CB; ++c) load4(xc[c] + r0, k.xv[c]);
        load4(b + r0, k.bv);
        const uint4 mm = *reinterpret_cast<const uint4 *>(meta + r0);
        k.m[0] = mm.x;
        k.m[1] = mm.y;
        k.m[2] = mm.z;
        k.m[3] = mm.w;
        if (XBAR) {
            load4(alpha + r0, k.av);
            load4(u + r0, k.uv);
            load4(zq + r0, k.qv);
            const int4 gg = *reinterpret_cast<const int4 *>(gidx + r0);
            k.gi[0] = gg.x;
            k.gi[1] = gg.y;
            k.gi[2] = gg.z;
            k.gi[3] = gg.w;
            if constexpr (EFRON) {
                const int4 g2 = *reinterpret_cast<const int4 *>(gidx2 + r0);
                k.g2[0] = g2.x;
                k.g2[1] = g2.y;
                k.g2[2] = g2.z;
                k.g2[3] = g2.w;
            }
        }
    };
    Chunk cur;
    load_chunk(cur, r_begin + (int64_t)lane * kColIpt);
    for (int64_t base = r_begin; base < r_end; base += kColChunk) {
        Chunk nxt;
        const bool more = base + kColChunk < r_end;
        if (more) load_chunk(nxt, base + kColChunk + (int64_t)lane * kColIpt);
        double(&xv)[CB][kColIpt] = cur.xv;
        double(&bv)[kColIpt] = cur.bv;
        double(&av)[kColIpt] = cur.av;
        double(&uv)[kColIpt] = cur.uv;
        double(&qv)[kColIpt] = cur.qv;
        uint32_t(&m)[kColIpt] = cur.m;
        int32_t(&gi)[kColIpt] = cur.gi;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
#pragma unroll
            for (int i = 0; i < kColIpt; ++i) {
                const double aw = bv[i] - ((m[i] & kEventBit) ? 1.0 : 0.0);   // w Lambda - delta
                g[c] = fma(xv[c][i], aw, g[c]);
                d1[c] = fma(xv[c][i] * xv[c][i], bv[i], d1[c]);
            }
        }
        if (XBAR) {
            // this lane's 4 rows folded: flags, product of alphas, and per column the map's offset
            uint32_t f = 0u;
            double a = 1.0, bb[CB];
#pragma unroll
            for (int c = 0; c < CB; ++c) bb[c] = 0.0;
#pragma unroll
            for (int i = 0; i < kColIpt; ++i) {
                const uint32_t fi = m[i] >> 31;
#pragma unroll
                for (int c = 0; c < CB; ++c) bb[c] = fi ? uv[i] * xv[c][i] : fma(av[i], bb[c], uv[i] * xv[c][i]);
                a = fi ? av[i] : a * av[i];
                f |= fi;
            }
            // inclusive scan across the wave
            aff_step<0x111, 0xF, CB>(f, a, bb);
            aff_step<0x112, 0xF, CB>(f, a, bb);
            aff_step<0x114, 0xF, CB>(f, a, bb);
            aff_step<0x118, 0xF, CB>(f, a, bb);
            aff_step<0x142, 0xA, CB>(f, a, bb);
            aff_step<0x143, 0xC, CB>(f, a, bb);
            // exclusive prefix of this lane = the inclusive value of lane - 1
            const uint32_t ef = dpp_keep_u32<0x138, 0xF>(0u, f);
            const double ea = dpp_keep<0x138, 0xF>(1.0, a);
            const uint32_t tf = (uint32_t)__builtin_amdgcn_readlane((int)f, 63);
            const double ta = readlane63(a);
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const double eb = dpp_keep<0x138, 0xF>(0.0, bb[c]);
                double run = ef ? eb : fma(ea, cb[c], eb);   // S' entering this lane's first row
#pragma unroll
                for (int i = 0; i < kColIpt; ++i) {
                    const double ux = uv[i] * xv[c][i];
                    run = (m[i] >> 31) ? ux : fma(av[i], run, ux);
                    if ((m[i] & kCountMask) && live[c]) {
                        if (EFRON && cur.g2[EFRON ? i : 0] >= 0) {
                            s1me[(int64_t)cur.g2[EFRON ? i : 0] * p + j0 + c] = run;
                        } else {
                            const double zv = run * qv[i];   // sqrt(d) xbar
                            d2[c] = fma(zv, zv, d2[c]);
                            store_z<ZT>(&z[(int64_t)(j0 + c) * ldz + gi[i]], zv, zs[c]);
                        }
                    }
                }
                const double tb = readlane63(bb[c]);
                cb[c] = tf ? tb : fma(ta, cb[c], tb);
            }
        }
        if (more) cur = nxt;
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

// Rows of Z of the multi-event groups (Efron): for group k and column j = blockIdx.y,
// E1' = sum over its event rows of exp(eta_r - m_end) x_rj, then z1 = l11 S1' + l21 E1' at the
// group's own row and z2 = l22 E1' at row n_groups + k; the workgroup's sum of z1^2 + z2^2 goes
// to epart[j][blockIdx.x] (fixed-order tree).
template <typename ZT>
__global__ __launch_bounds__(kRowBlock) void efron_z_kernel(const double *x, int64_t ld, int p, const int32_t *me_ptr,
                                                            const int32_t *me_row, const int32_t *me_end,
                                                            const double *me_w, const double *s1me,
                                                            const double *zq, const double *zq2, const double *zq3,
                                                            const int32_t *gidx, int64_t n_groups, int64_t n_multi,
                                                            int64_t ldz, const float *zscale, ZT *z, double *epart,
                                                            int eblocks)
{
    __shared__ double tree[kRowBlock];
    const int j = blockIdx.y;
    const int64_t k = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    double sq = 0.0;
    if (k < n_multi && j < p) {
        const double *xj = x + (int64_t)j * ld;
        double e1 = 0.0;
        for (int32_t q = me_ptr[k]; q < me_ptr[k + 1]; ++q) e1 = fma(me_w[q], xj[me_row[q]], e1);
        const int32_t e = me_end[k];
        const double s1 = s1me[k * p + j];
        const double z1 = fma(zq[e], s1, zq2[e] * e1), z2 = zq3[e] * e1;
        const float inv = zscale ? 1.0f / zscale[j] : 1.0f;
        store_z<ZT>(&z[(int64_t)j * ldz + gidx[e]], z1, inv);
        store_z<ZT>(&z[(int64_t)j * ldz + n_groups + k], z2, inv);
        sq = fma(z1, z1, z2 * z2);
    }
    tree[threadIdx.x] = sq;
    __syncthreads();
    for (int h = kRowBlock / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) tree[threadIdx.x] += tree[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0 && j < p) epart[(int64_t)j * eblocks + blockIdx.x] = tree[0];
}

// diag2[j] += the multi-event groups' parts, summed in block order
__global__ __launch_bounds__(kWave) void efron_d2_kernel(const double *epart, int eblocks, int p, double *diag2)
{
    const int j = blockIdx.x * kWave + threadIdx.x;
    if (j < p) {
        double s = 0.0;
        for (int k = 0; k < eblocks; ++k) s += epart[(int64_t)j * eblocks + k];
        diag2[j] += s;
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

// ------------------------------------------------------------------ row scans
//
// Segmented scans over all ld rows in tiles of `tile` rows: (1) each workgroup
// folds its tile into one aggregate, (2) one workgroup scans the aggregates
// into the value entering every tile, (3) each workgroup rescans its tile from
// there.  The element type and its operator come from affscan.hpp; a loader
// gives the element at scan position k and a writer stores the inclusive value.

constexpr int kScanThreads = 256, kScanWaves = kScanThreads / kWave;

template <class Op, class Ld, int PER>
__global__ __launch_bounds__(kScanThreads) void tscan_agg_kernel(Ld ldr, int64_t tile, typename Op::E *agg)
{
    using E = typename Op::E;
    __shared__ E wtot[kScanWaves];
    const int t = blockIdx.x;
    const int64_t per = PER > 0 ? PER : tile / kScanThreads;
    const int64_t k0 = (int64_t)t * tile + (int64_t)threadIdx.x * per;
    E f = Op::id();
    if constexpr (PER > 0) {
        E v[PER];   // all of the thread's rows in flight at once, in ascending address order
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = Ld::kReverse ? PER - 1 - q : q;
            v[i] = ldr(k0 + i);
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) f = Op::combine(f, v[i]);
    } else {
        for (int64_t i = 0; i < per; ++i) f = Op::combine(f, ldr(k0 + i));
    }
    E total;
    (void)block_exclusive_e<Op, kScanWaves>(f, wtot, total);
    if (threadIdx.x == 0) agg[t] = total;
}

template <class Op>
__global__ __launch_bounds__(1024) void tscan_carry_kernel(const typename Op::E *agg, int ntiles,
                                                           typename Op::E *carry)
{
    using E = typename Op::E;
    __shared__ E wtot[1024 / kWave];
    const int per = (ntiles + 1023) / 1024;
    const int t0 = threadIdx.x * per;
    E f = Op::id();
    for (int i = 0; i < per; ++i)
        if (t0 + i < ntiles) f = Op::combine(f, agg[t0 + i]);
    E total;
    E run = block_exclusive_e<Op, 1024 / kWave>(f, wtot, total);
    for (int i = 0; i < per; ++i) {
        const int t = t0 + i;
        if (t < ntiles) {
            carry[t] = run;
            run = Op::combine(run, agg[t]);
        }
    }
}

template <class Op, class Ld, class Wr, int PER>
__global__ __launch_bounds__(kScanThreads) void tscan_apply_kernel(Ld ldr, Wr wr, int64_t tile,
                                                                   const typename Op::E *carry)
{
    using E = typename Op::E;
    __shared__ E wtot[kScanWaves];
    const int t = blockIdx.x;
    const int64_t per = PER > 0 ? PER : tile / kScanThreads;
    const int64_t k0 = (int64_t)t * tile + (int64_t)threadIdx.x * per;
    if constexpr (PER > 0) {
        E v[PER];   // the thread's rows, loaded once, all in flight at once, in ascending address order
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = Ld::kReverse ? PER - 1 - q : q;
            v[i] = ldr(k0 + i);
        }
        E f = Op::id();
#pragma unroll
        for (int i = 0; i < PER; ++i) f = Op::combine(f, v[i]);
        E total;
        const E exc = block_exclusive_e<Op, kScanWaves>(f, wtot, total);
        E run = Op::combine(carry[t], exc);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            run = Op::combine(run, v[i]);
            wr(k0 + i, run);
        }
    } else {
        E f = Op::id();
        for (int64_t i = 0; i < per; ++i) f = Op::combine(f, ldr(k0 + i));
        E total;
        const E exc = block_exclusive_e<Op, kScanWaves>(f, wtot, total);
        E run = Op::combine(carry[t], exc);
        for (int64_t i = 0; i < per; ++i) {
            run = Op::combine(run, ldr(k0 + i));
            wr(k0 + i, run);
        }
    }
}

// running maximum of eta within each stratum (forward)
struct MaxLoad {
    static constexpr bool kReverse = false;   // scan position k is row k
    const double *eta;
    const uint32_t *meta;
    __device__ MaxE operator()(int64_t k) const { return MaxE{(meta[k] & kHeadBit) ? 1u : 0u, eta[k]}; }
};
struct MaxWrite {
    double *m;
    __device__ void operator()(int64_t k, const MaxE &e) const { m[k] = e.m; }
};

// S0' (forward): S0'_r = alpha_r S0'_{r-1} + u_r
struct S0Load {
    static constexpr bool kReverse = false;
    const double *alpha, *u;
    const uint32_t *meta;
    __device__ AffE operator()(int64_t k) const { return AffE{(meta[k] & kHeadBit) ? 1u : 0u, alpha[k], u[k]}; }
};
struct BWrite {
    double *out;
    __device__ void operator()(int64_t k, const AffE &e) const { out[k] = e.b; }
};

// Efron's E0' (forward): the running sum of u over event rows, restarting at stratum heads and
// after every row that ends a tie group with events, so at a group end it is the group's own
// E0 relative to exp(m_end): E0'_r = alpha_r E0'_{r-1} + delta_r u_r
struct E0Load {
    static constexpr bool kReverse = false;
    const double *alpha, *u;
    const uint32_t *meta;
    __device__ AffE operator()(int64_t k) const
    {
        const uint32_t mk = meta[k];
        const bool restart = (mk & kHeadBit) || k == 0 || (meta[k - 1] & kCountMask) != 0u;
        return AffE{restart ? 1u : 0u, alpha[k], (mk & kEventBit) ? u[k] : 0.0};
    }
};

// R (reverse, scan position k = row n-1-k): R_r = h'_r + alpha_{r+1} R_{r+1},
// a segment starting at each stratum's last row
struct RLoad {
    static constexpr bool kReverse = true;    // scan position k is row n - 1 - k
    const double *alpha, *h;
    const uint32_t *meta;
    int64_t n;
    __device__ AffE operator()(int64_t k) const
    {
        const int64_t r = n - 1 - k;
        const bool start = k == 0 || (meta[r + 1] & kHeadBit);
        return AffE{start ? 1u : 0u, start ? 1.0 : alpha[r + 1], h[r]};
    }
};
struct RWrite {
    double *out;
    int64_t n;
    __device__ void operator()(int64_t k, const AffE &e) const { out[n - 1 - k] = e.b; }
};

template <class Op, class Ld, class Wr>
int tile_scan(Ld ldr, Wr wr, int64_t n, int64_t tile, void *scratch, size_t scratch_bytes, hipStream_t stream)
{
    using E = typename Op::E;
    if (tile <= 0 || tile % kScanThreads != 0 || n % tile != 0) return -5;
    const int ntiles = (int)(n / tile);
    if (sizeof(E) * 2 * (size_t)ntiles > scratch_bytes) return -5;
    E *agg = static_cast<E *>(scratch);
    E *carry = agg + ntiles;
    // rows per thread as a compile-time count for the tile lengths of the layouts
    // (4096, 2048, 1024 and 512 rows), so that a thread's loads are all issued together
    const int64_t per = tile / kScanThreads;
#define COXMI_TSCAN(P)                                                                                     \
    do {                                                                                                   \
        tscan_agg_kernel<Op, Ld, P><<<ntiles, kScanThreads, 0, stream>>>(ldr, tile, agg);                 \
        tscan_carry_kernel<Op><<<1, 1024, 0, stream>>>(agg, ntiles, carry);                              \
        tscan_apply_kernel<Op, Ld, Wr, P><<<ntiles, kScanThreads, 0, stream>>>(ldr, wr, tile, carry);    \
    } while (0)
    if (per == 16) COXMI_TSCAN(16);
    else if (per == 8) COXMI_TSCAN(8);
    else if (per == 4) COXMI_TSCAN(4);
    else if (per == 2) COXMI_TSCAN(2);
    else COXMI_TSCAN(0);
#undef COXMI_TSCAN
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace

// ------------------------------------------------------------------ host launchers

size_t rowscan_scratch_bytes(int ntiles) { return sizeof(AffE) * 2 * (size_t)ntiles + 256; }

int full_eval_launch(const FullEvalArgs &A, hipStream_t stream)
{
    const int64_t ld = A.ld;
    const int nb = (int)((ld + kRowBlock - 1) / kRowBlock);
    if (nb > A.max_blocks) return -5;
    hipError_t e = hipMemsetAsync(A.flags, 0, sizeof(unsigned), stream);
    if (e != hipSuccess) return -3;
    eta_kernel<<<nb, kRowBlock, 0, stream>>>(A.x, ld, A.p, A.beta, A.eta);
    int rc = tile_scan<MaxOp>(MaxLoad{A.eta, A.meta}, MaxWrite{A.m}, ld, A.tile, A.scan_scratch,
                              A.scan_scratch_bytes, stream);
    if (rc) return rc;
    prep_kernel<<<nb, kRowBlock, 0, stream>>>(A.eta, A.m, A.meta, ld, A.alpha, A.w);
    rc = tile_scan<AffOp>(S0Load{A.alpha, A.w, A.meta}, BWrite{A.s0}, ld, A.tile, A.scan_scratch,
                          A.scan_scratch_bytes, stream);
    if (rc) return rc;
    if (A.efron) {
        rc = tile_scan<AffOp>(E0Load{A.alpha, A.w, A.meta}, BWrite{A.e0}, ld, A.tile, A.scan_scratch,
                              A.scan_scratch_bytes, stream);
        if (rc) return rc;
        hazard_efron_kernel<<<nb, kRowBlock, 0, stream>>>(A.s0, A.e0, A.eta, A.m, A.meta, ld, A.h, A.kq, A.zq, A.zq2,
                                                          A.zq3, A.blockbuf, A.flags);
    } else {
        hazard_kernel<<<nb, kRowBlock, 0, stream>>>(A.s0, A.eta, A.m, A.meta, ld, A.h, A.zq, A.blockbuf, A.flags);
    }
    rc = tile_scan<AffOp>(RLoad{A.alpha, A.h, A.meta, ld}, RWrite{A.lam, ld}, ld, A.tile, A.scan_scratch,
                          A.scan_scratch_bytes, stream);
    if (rc) return rc;
    if (A.efron)
        rowweight_efron_kernel<<<nb, kRowBlock, 0, stream>>>(A.w, A.lam, A.eta, A.m, A.kq, A.gend, ld, A.b);
    else
        rowweight_kernel<<<nb, kRowBlock, 0, stream>>>(A.w, A.lam, ld, A.b);
    if (A.n_agg > 0) {
        colagg_kernel<<<(A.n_agg * A.p + kColWaves - 1) / kColWaves, kWave * kColWaves, 0, stream>>>(
            A.x, ld, A.p, A.alpha, A.w, A.meta, A.tile, A.agg_tiles, A.n_agg, A.lasthead, A.agg);
        colcarry_kernel<<<(A.p + 255) / 256, 256, 0, stream>>>(A.p, A.ntiles, A.tile_carry, A.lasthead, A.agg,
                                                               A.carry);
    }
    const int grid = 8 * ((A.ntiles + 7) / 8) * ((A.p + kColWaves * kColBlock - 1) / (kColWaves * kColBlock));
#define COXMI_COLPASS(ZT, XB, EF)                                                                              \
    colpass_kernel<ZT, XB, EF><<<grid, kWave * kColWaves, 0, stream>>>(                                        \
        A.x, ld, A.p, A.tile, A.ntiles, A.alpha, A.w, A.zq, A.b, A.meta, A.gidx, A.tile_carry, A.carry, A.ldz, \
        A.zscale, static_cast<ZT *>(A.z), A.colpart, A.gidx2, A.s1me)
    const bool ef = A.efron && A.n_multi > 0;
    if (!A.want_xbar) COXMI_COLPASS(double, false, false);
    else if (A.ztype == kZF64) {
        if (ef) COXMI_COLPASS(double, true, true);
        else COXMI_COLPASS(double, true, false);
    } else if (A.ztype == kZF32) {
        COXMI_COLPASS(float, true, false);
    } else {
        if (ef) COXMI_COLPASS(__hip_bfloat16, true, true);
        else COXMI_COLPASS(__hip_bfloat16, true, false);
    }
#undef COXMI_COLPASS
    colreduce_kernel<<<A.p + 1, kRowBlock, 0, stream>>>(A.colpart, A.p, A.ntiles, A.grad, A.diag1, A.diag2,
                                                        A.blockbuf, nb, A.scal);
    if (ef && A.want_xbar) {
        if (A.ztype == kZF32) return -5;
        efron_w_kernel<<<(unsigned)((A.n_multi + kRowBlock - 1) / kRowBlock), kRowBlock, 0, stream>>>(
            A.eta, A.m, A.me_ptr, A.me_row, A.me_end, A.n_multi, A.me_w);
        const dim3 zg((unsigned)A.eblocks, (unsigned)A.p);
        if (A.ztype == kZF64)
            efron_z_kernel<double><<<zg, kRowBlock, 0, stream>>>(
                A.x, ld, A.p, A.me_ptr, A.me_row, A.me_end, A.me_w, A.s1me, A.zq, A.zq2, A.zq3, A.gidx, A.n_groups,
                A.n_multi, A.ldz, A.zscale, static_cast<double *>(A.z), A.epart, A.eblocks);
        else
            efron_z_kernel<__hip_bfloat16><<<zg, kRowBlock, 0, stream>>>(
                A.x, ld, A.p, A.me_ptr, A.me_row, A.me_end, A.me_w, A.s1me, A.zq, A.zq2, A.zq3, A.gidx, A.n_groups,
                A.n_multi, A.ldz, A.zscale, static_cast<__hip_bfloat16 *>(A.z), A.epart, A.eblocks);
        efron_d2_kernel<<<(A.p + kWave - 1) / kWave, kWave, 0, stream>>>(A.epart, A.eblocks, A.p, A.diag2);
    }
    e = hipGetLastError();
    return e == hipSuccess ? 0 : -3;
}

}  // namespace coxmi
