// contraction.hip -- the information matrix as two symmetric rank-K products,
// and the FP64 Cholesky solve of a Newton step (gfx950).
//
//   I = X' diag(b) X - Z'Z,   b_r = w_r Lambda_r,   Z_gj = sqrt(d_g) xbar_gj
// (the Hessian of Eq. strat_h with the order of its sums exchanged; see
// newton.hip).  Both products have the form C = sum_k c_k u_k u_k' over K
// rows with u_k in R^p stored column-wise ([p][ld], k contiguous).
//
// FP64 reference kernel: 64x64 tiles of the upper triangle, K split across
// workgroups, 32-row chunks staged in LDS, each thread owning a 4x4 block;
// the split partials are summed in split order (deterministic).
//
// BF16 kernel (matrix cores): u is stored as BF16 with a power-of-two scale
// per column; v_mfma_f32_32x32x16_bf16 accumulates 32x32 tiles in FP32.  The
// weights c_k multiply one operand in FP32 before it is rounded to BF16.
// Each wave owns up to 8 tiles of the upper triangle, a workgroup's 4 waves
// share one K range, and the FP32 partials of the K ranges are summed in FP64
// in range order with the column scales applied.
#include <hip/hip_bf16.h>
#include <math.h>

#include "internal.h"
#include "newton.h"

namespace coxmi {

namespace {

constexpr int kTile = 64, kKc = 32, kSyrkThreads = 256, kWaveC = 64;

// x of lane src, for a src that is the same in every lane of the wave (two v_readlane, no
// trip through the LDS crossbar as for a per-lane source)
__device__ __forceinline__ double lane_value(double x, int src)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ void tile_pair(int pair, int nt, int &ti, int &tj)
{
    // pairs (ti <= tj) in row-major order of the upper triangle
    int i = 0, rem = pair;
    while (rem >= nt - i) {
        rem -= nt - i;
        ++i;
    }
    ti = i;
    tj = i + rem;
}

// (K range, group) of a workgroup of a (splits, groups) grid.  Workgroups go to the 8 XCDs in
// turn by linear id; when splits is a multiple of 8 the ids are renumbered so that every group
// of one K range runs on one XCD at nearly the same time, and the rows of the range that each
// of them stages are read from HBM once and from that XCD's L2 after.  Only the assignment of
// work to workgroups changes, not the work.
__device__ __forceinline__ void split_group(int &split, int &group)
{
    const int nsplit = gridDim.x, ngroup = gridDim.y;
    if (ngroup == 1 || nsplit % 8 != 0) {
        split = blockIdx.x;
        group = blockIdx.y;
        return;
    }
    const int L = blockIdx.x + nsplit * blockIdx.y;
    const int x = L % 8, r = L / 8;
    split = x + 8 * (r / ngroup);
    group = r % ngroup;
}


__global__ __launch_bounds__(kSyrkThreads) void syrk_f64_kernel(const double *u, int64_t ldu, int p,
                                                                const double *c, int64_t K, int64_t kchunk,
                                                                double *part)
{
    __shared__ double As[kTile][kKc + 1];
    __shared__ double Bs[kTile][kKc + 1];
    const int nt = (p + kTile - 1) / kTile;
    const int npairs = nt * (nt + 1) / 2;
    const int pair = blockIdx.x, s = blockIdx.y;
    int ti, tj;
    tile_pair(pair, nt, ti, tj);
    const int t = threadIdx.x, tx = t % 16, ty = t / 16;
    const int64_t k0 = (int64_t)s * kchunk;
    const int64_t k1 = k0 + kchunk < K ? k0 + kchunk : K;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) acc[a][bb] = 0.0;
    for (int64_t k = k0; k < k1; k += kKc) {
#pragma unroll
        for (int e = 0; e < kTile * kKc / kSyrkThreads; ++e) {
            const int idx = t + kSyrkThreads * e;
            const int i = idx / kKc, kk = idx % kKc;
            const int64_t kr = k + kk;
            const int ri = ti * kTile + i, rj = tj * kTile + i;
            double av = 0.0, bv = 0.0;
            if (kr < k1) {
                const double ck = c ? c[kr] : 1.0;
                if (ri < p) av = u[(int64_t)ri * ldu + kr] * ck;
                if (rj < p) bv = u[(int64_t)rj * ldu + kr];
            }
            As[i][kk] = av;
            Bs[i][kk] = bv;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < kKc; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = As[ty * 4 + a][kk];
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) bv[bb] = Bs[tx * 4 + bb][kk];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int bb = 0; bb < 4; ++bb) acc[a][bb] = fma(av[a], bv[bb], acc[a][bb]);
        }
        __syncthreads();
    }
    double *out = part + ((int64_t)s * npairs + pair) * (kTile * kTile);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) out[(ty * 4 + a) * kTile + tx * 4 + bb] = acc[a][bb];
}

// FP64 on the matrix cores (v_mfma_f64_16x16x4_f64), for p <= 512: per K chunk of kF64KC
// rows the workgroup stages every row of u once in LDS (FP64, as stored); its 8 waves own
// 16 x 16 blocks (bi <= bj) of the upper triangle in turn (block q of the workgroup's group
// to wave q mod 8) and run them from LDS, the A operand multiplied by c_k as it is read.  A
// group holds up to kF64Group blocks (p <= 256: all of them; beyond, the groups of one K range
// run on one XCD, see split_group).  An MFMA step takes 4 K values: lane l supplies
// A[bi*16 + l%16][k + l/16] and B[bj*16 + l%16][k + l/16] and holds D[l/16 + 4 r][l%16],
// r = 0..3, of its block (rows interleaved by 4).  The partials go to the 64 x 64 tile-pair
// layout of syrk_f64_kernel (blocks below the diagonal of a diagonal tile are never
// written, and syrk_reduce_kernel never reads them).
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int kF64Waves = 8, kF64KC = 32;
constexpr int kF64PerWave = 17, kF64Group = kF64Waves * kF64PerWave;   // 136 = all blocks at p <= 256

// MAXB: the most 16-row blocks (16: p <= 256, staged rows 256 x 33 doubles; 32: p <= 512, 135 KB)
template <int MAXB>
__global__ __launch_bounds__(64 * kF64Waves, 1) void syrk_f64_mfma_kernel(const double *u, int64_t ldu, int p,
                                                                         const double *c, int64_t K,
                                                                         int64_t kchunk, double *part)
{
    __shared__ double xs[MAXB * 16][kF64KC + 1];
    __shared__ double cs[kF64KC];
    const int nb = (p + 15) / 16;
    const int nblk = nb * (nb + 1) / 2;
    const int nt = (p + kTile - 1) / kTile;
    const int npairs = nt * (nt + 1) / 2;
    const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
    int s, grp;
    split_group(s, grp);
    const int q0 = grp * kF64Group;
    const int64_t k0 = (int64_t)s * kchunk;
    const int64_t k1 = k0 + kchunk < K ? k0 + kchunk : K;
    int bi[kF64PerWave], bj[kF64PerWave];
    f64x4 acc[kF64PerWave];
#pragma unroll
    for (int m = 0; m < kF64PerWave; ++m) {
        const int q = q0 + w + kF64Waves * m;
        int i = 0, rem = q < nblk ? q : 0;
        while (rem >= nb - i) {
            rem -= nb - i;
            ++i;
        }
        bi[m] = i;
        bj[m] = i + rem;
        acc[m] = f64x4{0.0, 0.0, 0.0, 0.0};
    }
    const int rows = nb * 16;
    const int r16 = lane & 15, kq = lane >> 4;
    for (int64_t kc = k0; kc < k1; kc += kF64KC) {
        // stage rows x kF64KC (zero beyond p and beyond k1)
        for (int e = threadIdx.x; e < rows * kF64KC; e += 64 * kF64Waves) {
            const int r = e / kF64KC, kk = e % kF64KC;
            const int64_t kr = kc + kk;
            xs[r][kk] = (r < p && kr < k1) ? u[(int64_t)r * ldu + kr] : 0.0;
        }
        if (threadIdx.x < kF64KC) cs[threadIdx.x] = (c && kc + threadIdx.x < k1) ? c[kc + threadIdx.x] : 1.0;
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kF64KC; ks += 4) {
            const int kk = ks + kq;
            const double ck = cs[kk];
#pragma unroll
            for (int m = 0; m < kF64PerWave; ++m) {
                if (q0 + w + kF64Waves * m < nblk) {
                    const double a = xs[bi[m] * 16 + r16][kk] * ck;
                    const double b = xs[bj[m] * 16 + r16][kk];
                    acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[m], 0, 0, 0);
                }
            }
        }
        __syncthreads();   // the next chunk rewrites the staged rows
    }
#pragma unroll
    for (int m = 0; m < kF64PerWave; ++m) {
        if (q0 + w + kF64Waves * m < nblk) {
            const int ti = bi[m] / 4, tj = bj[m] / 4;
            const int pair = ti * nt - ti * (ti - 1) / 2 + (tj - ti);
            double *out = part + ((int64_t)s * npairs + pair) * (kTile * kTile);
            const int col = (bj[m] % 4) * 16 + r16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = (bi[m] % 4) * 16 + kq + 4 * r;
                out[row * kTile + col] = acc[m][r];
            }
        }
    }
}

// C (p x p, row-major, symmetric) = sign * sum over splits of the partial tiles, added to C
// when accumulate != 0.  Grid (npairs, 64): a workgroup takes 64 entries of one 64 x 64 tile;
// its 16 waves sum the splits q = w, w + 16, ... in order and the 16 sums are added in wave
// order (a fixed order: results do not vary run to run).  Entries below the diagonal of a
// diagonal tile are neither read nor written.
constexpr int kRedWaves = 16;

__global__ __launch_bounds__(64 * kRedWaves) void syrk_reduce_kernel(const double *part, int p, int S, double sign,
                                                                     int accumulate, double *C)
{
    __shared__ double red[kRedWaves][64];
    const int nt = (p + kTile - 1) / kTile;
    const int npairs = nt * (nt + 1) / 2;
    const int pair = blockIdx.x;
    int ti, tj;
    tile_pair(pair, nt, ti, tj);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int e = blockIdx.y * 64 + lane;
    const int a = e / kTile, bb = e % kTile;
    const int i = ti * kTile + a, j = tj * kTile + bb;
    const bool live = i < p && j < p && !(ti == tj && j < i);
    double s = 0.0;
    if (live)
        for (int q = w; q < S; q += kRedWaves) s += part[((int64_t)q * npairs + pair) * (kTile * kTile) + e];
    red[w][lane] = s;
    __syncthreads();
    if (w != 0 || !live) return;
    s = red[0][lane];
    for (int v = 1; v < kRedWaves; ++v) s += red[v][lane];
    s *= sign;
    if (accumulate) {
        C[(int64_t)i * p + j] += s;
        if (i != j) C[(int64_t)j * p + i] += s;
    } else {
        C[(int64_t)i * p + j] = s;
        if (i != j) C[(int64_t)j * p + i] = s;
    }
}

// One workgroup: A (p x p, row-major, symmetric positive definite on the free
// columns) is overwritten by its Cholesky factor L (lower triangle) unless
// `factored`; then dx = -A^{-1} g on the free columns, 0 on the others.
// status[0] = 1 if a pivot was not positive.
__global__ __launch_bounds__(256) void chol_solve_kernel(double *A, int p, const double *g, const uint8_t *free_col,
                                                         int factored, double *dx, int *status)
{
    extern __shared__ double sy[];   // [p]
    __shared__ double s_piv;
    __shared__ int s_bad;
    const int t = threadIdx.x;
    if (t == 0) s_bad = 0;
    if (!factored) {
        for (int64_t e = t; e < (int64_t)p * p; e += 256) {
            const int i = (int)(e / p), j = (int)(e % p);
            if (!free_col[i] || !free_col[j]) A[e] = (i == j) ? 1.0 : 0.0;
        }
        __syncthreads();
        for (int k = 0; k < p; ++k) {
            if (t == 0) {
                double d = A[(int64_t)k * p + k];
                if (!(d > 0.0)) {
                    s_bad = 1;
                    d = 1.0;
                }
                s_piv = sqrt(d);
                A[(int64_t)k * p + k] = s_piv;
            }
            __syncthreads();
            const double piv = s_piv;
            for (int i = k + 1 + t; i < p; i += 256) A[(int64_t)i * p + k] /= piv;
            __syncthreads();
            const int m = p - k - 1;
            for (int64_t e = t; e < (int64_t)m * m; e += 256) {
                const int i = k + 1 + (int)(e / m), j = k + 1 + (int)(e % m);
                if (j <= i) A[(int64_t)i * p + j] -= A[(int64_t)i * p + k] * A[(int64_t)j * p + k];
            }
            __syncthreads();
        }
    }
    for (int i = t; i < p; i += 256) sy[i] = free_col[i] ? -g[i] : 0.0;
    __syncthreads();
    for (int k = 0; k < p; ++k) {          // L y = -g
        if (t == 0) sy[k] /= A[(int64_t)k * p + k];
        __syncthreads();
        const double yk = sy[k];
        for (int i = k + 1 + t; i < p; i += 256) sy[i] -= A[(int64_t)i * p + k] * yk;
        __syncthreads();
    }
    for (int k = p - 1; k >= 0; --k) {     // L' x = y
        if (t == 0) sy[k] /= A[(int64_t)k * p + k];
        __syncthreads();
        const double xk = sy[k];
        for (int i = t; i < k; i += 256) sy[i] -= A[(int64_t)k * p + i] * xk;
        __syncthreads();
    }
    for (int i = t; i < p; i += 256) dx[i] = free_col[i] ? sy[i] : 0.0;
    if (t == 0) status[0] = s_bad;
}

// Blocked variant for p <= kCholMaxP, 16-column panels, three barriers each:
//   1. wave 0 factors the 16 x 16 diagonal block, a row per lane in registers
//      (each scaled column goes through LDS to the lanes below it);
//   2. every thread takes one row below the block and solves x L11' = a for it
//      (L11 read from LDS by all lanes at once), giving the panel L21;
//   3. all threads update the trailing lower triangle in 4 x 4 register blocks
//      from L21 (kept in LDS): A22 -= L21 L21'.
// Triangular solves by 32-row blocks (one wave solves the diagonal block with
// lane shuffles).  Same contract as chol_solve_kernel.
constexpr int kCholNB = 32, kCholThreads = 512, kCholMaxP = 512, kPanNB = 16;

__global__ __launch_bounds__(kCholThreads) void chol_blocked_kernel(double *A, int p, const double *g,
                                                                    const uint8_t *free_col, int factored,
                                                                    double *dx, int *status)
{
    // panel L21 [kPanNB][p] (column-major: entry (i, c) at c * p + i), then y at p * kCholNB
    extern __shared__ double lds[];
    double *pan = lds;
    double *y = lds + (size_t)p * kCholNB;
    __shared__ double s_l11[kPanNB][kPanNB + 1];   // the factored diagonal block, row-major
    __shared__ double s_inv[kPanNB];                 // 1 / its diagonal
    __shared__ double s_col[kPanNB];                 // one scaled column of the block
    __shared__ int s_bad;
    const int t = threadIdx.x;
    const int lane = t & (kWaveC - 1), wv = t / kWaveC;
    constexpr int kWaves = kCholThreads / kWaveC;
    if (t == 0) s_bad = 0;
    if (!factored) {
        // rows and columns not free become unit rows
        for (int i = wv; i < p; i += kWaves)
            for (int j = lane; j < p; j += kWaveC)
                if (!free_col[i] || !free_col[j]) A[(int64_t)i * p + j] = (i == j) ? 1.0 : 0.0;
        __syncthreads();
        for (int c0 = 0; c0 < p; c0 += kPanNB) {
            const int nb = p - c0 < kPanNB ? p - c0 : kPanNB;
            // 1. diagonal block: lane r holds row c0 + r (entries up to the diagonal)
            if (wv == 0) {
                double D[kPanNB];
#pragma unroll
                for (int c = 0; c < kPanNB; ++c)
                    D[c] = (lane < nb && c <= lane) ? A[(int64_t)(c0 + lane) * p + c0 + c] : 0.0;
#pragma unroll
                for (int kk = 0; kk < kPanNB; ++kk) {
                    if (kk < nb) {
                        double d = lane_value(D[kk], kk);
                        const bool ok = d > 0.0;
                        if (!ok) d = 1.0;
                        const double piv = sqrt(d), inv = 1.0 / piv;
                        if (lane == 0) {
                            if (!ok) s_bad = 1;
                            s_inv[kk] = inv;
                        }
                        if (lane == kk) D[kk] = piv;
                        else if (lane > kk) D[kk] *= inv;
                        if (lane < kPanNB) s_col[lane] = D[kk];
                        __builtin_amdgcn_wave_barrier();
#pragma unroll
                        for (int jj = kk + 1; jj < kPanNB; ++jj)
                            if (jj < nb && lane >= jj) D[jj] = fma(-D[kk], s_col[jj], D[jj]);
                        __builtin_amdgcn_wave_barrier();
                    }
                }
                if (lane < nb) {
#pragma unroll
                    for (int c = 0; c < kPanNB; ++c)
                        if (c <= lane) {
                            s_l11[lane][c] = D[c];
                            A[(int64_t)(c0 + lane) * p + c0 + c] = D[c];
                        }
                }
            }
            __syncthreads();
            // 2. the rows below the block: x L11' = a, one row per thread
            const int r0 = c0 + nb;
            for (int i = r0 + t; i < p; i += kCholThreads) {
                double a[kPanNB];
                const double *row = A + (int64_t)i * p + c0;
#pragma unroll
                for (int c = 0; c < kPanNB; ++c) a[c] = c < nb ? row[c] : 0.0;
#pragma unroll
                for (int c = 0; c < kPanNB; ++c) {
                    if (c < nb) {
                        double v = a[c];
#pragma unroll
                        for (int q = 0; q < c; ++q) v = fma(-a[q], s_l11[c][q], v);
                        a[c] = v * s_inv[c];
                    }
                    // keep the LDS reads of row c + 1 of L11 from being hoisted above this
                    // point (hoisting all of them would not fit in registers)
                    __builtin_amdgcn_sched_barrier(0);
                }
                double *wrow = A + (int64_t)i * p + c0;
#pragma unroll
                for (int c = 0; c < kPanNB; ++c)
                    if (c < nb) {
                        wrow[c] = a[c];
                        pan[c * p + i] = a[c];
                    }
            }
            __syncthreads();
            // 3. trailing update of the lower triangle: A22 -= L21 L21'
            const int m2 = p - r0;
            if (m2 > 0) {
                const int nb4 = (m2 + 3) / 4;
                const int nblk = nb4 * (nb4 + 1) / 2;
                for (int bk = t; bk < nblk; bk += kCholThreads) {
                    // block (bi, bj), bj <= bi, in row-major order of the lower triangle
                    int bi = (int)((sqrt(8.0 * bk + 1.0) - 1.0) * 0.5);
                    while ((bi + 1) * (bi + 2) / 2 <= bk) ++bi;
                    while (bi * (bi + 1) / 2 > bk) --bi;
                    const int bj = bk - bi * (bi + 1) / 2;
                    double acc[4][4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
                    for (int c = 0; c < nb; ++c) {
                        double ai[4], aj[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int ii = r0 + 4 * bi + u, jj = r0 + 4 * bj + u;
                            ai[u] = ii < p ? pan[c * p + ii] : 0.0;
                            aj[u] = jj < p ? pan[c * p + jj] : 0.0;
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u)
#pragma unroll
                            for (int v = 0; v < 4; ++v) acc[u][v] = fma(ai[u], aj[v], acc[u][v]);
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int i = r0 + 4 * bi + u, j = r0 + 4 * bj + v;
                            if (i < p && j <= i) A[(int64_t)i * p + j] -= acc[u][v];
                        }
                }
            }
            __syncthreads();
        }
    }
    // solves: L y = -g, then L' x = y (free columns only)
    for (int i = t; i < p; i += kCholThreads) y[i] = free_col[i] ? -g[i] : 0.0;
    __syncthreads();
    // the diagonal block's entries a lane needs are loaded into registers first
    // (all loads in flight together), so the sequential steps wait only on shuffles
    for (int k0 = 0; k0 < p; k0 += kCholNB) {
        const int nb = p - k0 < kCholNB ? p - k0 : kCholNB;
        if (wv == 0) {
            double Lr[kCholNB];   // row k0 + lane of the block (entries up to the diagonal)
#pragma unroll
            for (int c = 0; c < kCholNB; ++c)
                Lr[c] = (lane < nb && c <= lane) ? A[(int64_t)(k0 + lane) * p + k0 + c] : 1.0;
            double yi = lane < nb ? y[k0 + lane] : 0.0;
#pragma unroll
            for (int c = 0; c < kCholNB; ++c) {
                if (c < nb) {
                    if (lane == c) yi /= Lr[c];
                    const double yc = lane_value(yi, c);
                    if (lane > c && lane < nb) yi = fma(-Lr[c], yc, yi);
                }
            }
            if (lane < nb) y[k0 + lane] = yi;
        }
        __syncthreads();
        for (int i = k0 + nb + t; i < p; i += kCholThreads) {
            const double *row = A + (int64_t)i * p + k0;
            double s = 0.0;
            for (int c = 0; c < nb; ++c) s = fma(row[c], y[k0 + c], s);
            y[i] -= s;
        }
        __syncthreads();
    }
    for (int k0 = ((p - 1) / kCholNB) * kCholNB; k0 >= 0; k0 -= kCholNB) {
        const int nb = p - k0 < kCholNB ? p - k0 : kCholNB;
        if (wv == 0) {
            double Lc[kCholNB];   // column k0 + lane of the block (entries from the diagonal down)
#pragma unroll
            for (int c = 0; c < kCholNB; ++c)
                Lc[c] = (lane < nb && c >= lane && c < nb) ? A[(int64_t)(k0 + c) * p + k0 + lane] : 1.0;
            double xi = lane < nb ? y[k0 + lane] : 0.0;
#pragma unroll
            for (int c = kCholNB - 1; c >= 0; --c) {
                if (c < nb) {
                    if (lane == c) xi /= Lc[c];
                    const double xc = lane_value(xi, c);
                    if (lane < c) xi = fma(-Lc[c], xc, xi);
                }
            }
            if (lane < nb) y[k0 + lane] = xi;
        }
        __syncthreads();
        for (int i = t; i < k0; i += kCholThreads) {
            double s = 0.0;
            for (int c = 0; c < nb; ++c) s = fma(A[(int64_t)(k0 + c) * p + i], y[k0 + c], s);
            y[i] -= s;
        }
        __syncthreads();
    }
    for (int i = t; i < p; i += kCholThreads) dx[i] = free_col[i] ? y[i] : 0.0;
    if (t == 0) status[0] = s_bad;
}

// ------------------------------------------------------------------ BF16 on the matrix cores

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));

constexpr int kMT = 32;              // MFMA tile edge
constexpr int kTilesPerWave = 8;
constexpr int kSyrkBfWaves = 4;
constexpr int kPairsPerGroup = kTilesPerWave * kSyrkBfWaves;

__host__ __device__ __forceinline__ int npairs32(int p)
{
    const int nt = (p + kMT - 1) / kMT;
    return nt * (nt + 1) / 2;
}

// Fragment of 8 consecutive K values of row `row` (0 beyond p).
__device__ __forceinline__ bf16x8 load_frag(const uint16_t *u, int64_t ldu, int p, int row, int64_t k)
{
    if (row >= p) {
        bf16x8 z;
#pragma unroll
        for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.0f;
        return z;
    }
    const u32x4v v = *reinterpret_cast<const u32x4v *>(u + (int64_t)row * ldu + k);
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ bf16x8 weight_frag(bf16x8 a, const double *c, int64_t k)
{
    bf16x8 r;
#pragma unroll
    for (int i = 0; i < 8; ++i) r[i] = (__bf16)((float)a[i] * (float)c[k + i]);
    return r;
}

// part[(s * npairs + pair) * 1024 + m * 32 + n] = sum over K range s of
// c_k u[ti*32+m][k] u[tj*32+n][k] (scaled units).  Grid (S, pair groups).
__global__ __launch_bounds__(64 * kSyrkBfWaves) void syrk_bf16_kernel(const uint16_t *u, int64_t ldu, int p,
                                                                      const double *c, int64_t K,
                                                                      int64_t kchunk, float *part)
{
    const int nt = (p + kMT - 1) / kMT;
    const int npairs = nt * (nt + 1) / 2;
    const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
    int s, grp;
    split_group(s, grp);
    const int pair0 = grp * kPairsPerGroup + w * kTilesPerWave;
    const int64_t k0 = (int64_t)s * kchunk;
    const int64_t k1 = k0 + kchunk < K ? k0 + kchunk : K;
    int ti[kTilesPerWave], tj[kTilesPerWave];
    f32x16 acc[kTilesPerWave];
#pragma unroll
    for (int q = 0; q < kTilesPerWave; ++q) {
        tile_pair(pair0 + q < npairs ? pair0 + q : 0, nt, ti[q], tj[q]);
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[q][i] = 0.0f;
    }
    const int nq = npairs - pair0 < kTilesPerWave ? (npairs - pair0 > 0 ? npairs - pair0 : 0) : kTilesPerWave;
    const int rsub = lane % 32, ksub = 8 * (lane / 32);
    for (int64_t k = k0; k < k1; k += 16) {
        const int64_t kk = k + ksub;
#pragma unroll
        for (int q = 0; q < kTilesPerWave; ++q) {
            if (q < nq) {
                bf16x8 a = load_frag(u, ldu, p, ti[q] * kMT + rsub, kk);
                if (c) a = weight_frag(a, c, kk);
                const bf16x8 bv = load_frag(u, ldu, p, tj[q] * kMT + rsub, kk);
                acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv, acc[q], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kTilesPerWave; ++q) {
        if (q < nq) {
            float *out = part + ((int64_t)s * npairs + pair0 + q) * (kMT * kMT);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int m = 8 * (i / 4) + 4 * (lane / 32) + (i % 4), n = lane % 32;
                out[m * kMT + n] = acc[q][i];
            }
        }
    }
}

// LDS-staged variant for p <= 256 (at most 8 row tiles): per 128-row K chunk
// the workgroup stages all row tiles of u once (and once more multiplied by
// the weights, rounded to BF16), then every wave runs its tile pairs' MFMAs
// from LDS.  The next chunk's global loads are issued into registers before
// the current chunk's MFMAs.  Same partial layout as syrk_bf16_kernel.
// KC rows per chunk: 128 for up to 8 row tiles, 64 for up to 16 (the LDS then
// holds 16 tiles x 32 rows x 72 BF16, twice with weights: 147 KB).
constexpr int kLdsMaxTiles = 16;

// MAXT: the most row tiles the launch may have (the LDS holds MAXT x 32 rows); OCC: the waves
// per SIMD the register budget is cut for (with NWV waves of TPW tile pairs each: two
// workgroups of 8 waves per compute unit need 4, so one workgroup's loads overlap the
// other's matrix-core work).
template <bool WEIGHT, int KC, int MAXT = (KC == 128 ? 8 : 16), int OCC = 1, int NWV = kSyrkBfWaves,
          int TPW = kTilesPerWave>
__global__ __launch_bounds__(64 * NWV, OCC) void syrk_bf16_lds_kernel(const uint16_t *u, int64_t ldu, int p,
                                                                               const double *c, int64_t K,
                                                                               int64_t kchunk, float *part)
{
    constexpr int kLdsKC = KC, kLdsStride = KC + 8, kLdsPieces = KC / 8;
    static_assert(NWV * TPW == kPairsPerGroup, "a group holds kPairsPerGroup tile pairs");
    constexpr int kLdsPerThread = (MAXT * kMT * kLdsPieces + 64 * NWV - 1) / (64 * NWV);
    extern __shared__ uint16_t sh[];   // [nt*32][kLdsStride] plain, then weighted (WEIGHT)
    __shared__ float cw[kLdsKC];
    const int nt = (p + kMT - 1) / kMT;
    const int rows = nt * kMT;
    uint16_t *plain = sh;
    uint16_t *wtd = sh + (size_t)rows * kLdsStride;
    const int npairs = nt * (nt + 1) / 2;
    const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
    int s, grp;
    split_group(s, grp);
    const int pair0 = grp * kPairsPerGroup + w * TPW;
    const int nq = npairs - pair0 < TPW ? (npairs - pair0 > 0 ? npairs - pair0 : 0) : TPW;
    const int64_t k0 = (int64_t)s * kchunk;
    const int64_t k1 = k0 + kchunk < K ? k0 + kchunk : K;
    const int rsub = lane & 31, ksub = 8 * (lane >> 5);
    // LDS offsets of this lane's A (weighted) and B (plain) rows for each tile pair, packed
    // 16 bits each (at most 16 x 32 rows of kLdsStride elements: < 2^16)
    uint32_t offs[TPW];
    f32x16 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        int ti, tj;
        tile_pair(pair0 + q < npairs ? pair0 + q : 0, nt, ti, tj);
        offs[q] = (uint32_t)((ti * kMT + rsub) * kLdsStride) | ((uint32_t)((tj * kMT + rsub) * kLdsStride) << 16);
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[q][i] = 0.0f;
    }
    const int npieces = rows * kLdsPieces;
    // prefetch registers: this thread's pieces e = tid + 256 m, one chunk ahead
    u32x4v reg[kLdsPerThread];
    float creg = 0.0f;
    auto load_chunk = [&](int64_t kc) {
#pragma unroll
        for (int m = 0; m < kLdsPerThread; ++m) {
            const int e = threadIdx.x + 64 * NWV * m;
            const int r = e / kLdsPieces, piece = e % kLdsPieces;
            u32x4v v = {0u, 0u, 0u, 0u};
            if (e < npieces && r < p) v = *reinterpret_cast<const u32x4v *>(u + (int64_t)r * ldu + kc + 8 * piece);
            reg[m] = v;
        }
        if (WEIGHT && threadIdx.x < kLdsKC) creg = (float)c[kc + threadIdx.x];
    };
    if (k0 < k1) load_chunk(k0);
    for (int64_t kc = k0; kc < k1; kc += kLdsKC) {
        if (WEIGHT && threadIdx.x < kLdsKC) cw[threadIdx.x] = creg;
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kLdsPerThread; ++m) {
            const int e = threadIdx.x + 64 * NWV * m;
            if (e < npieces) {
                const int r = e / kLdsPieces, piece = e % kLdsPieces;
                *reinterpret_cast<u32x4v *>(plain + r * kLdsStride + 8 * piece) = reg[m];
                if (WEIGHT) {
                    const bf16x8 x = __builtin_bit_cast(bf16x8, reg[m]);
                    bf16x8 y;
#pragma unroll
                    for (int i = 0; i < 8; ++i) y[i] = (__bf16)((float)x[i] * cw[8 * piece + i]);
                    *reinterpret_cast<u32x4v *>(wtd + r * kLdsStride + 8 * piece) = __builtin_bit_cast(u32x4v, y);
                }
            }
        }
        __syncthreads();
        if (kc + kLdsKC < k1) load_chunk(kc + kLdsKC);   // in flight during the MFMAs below
        const uint16_t *asrc = WEIGHT ? wtd : plain;
#pragma unroll
        for (int sub = 0; sub < kLdsKC / 16; ++sub) {
            const int kk = 16 * sub + ksub;
            // a wave's pairs run along rows of the upper triangle: the A fragment (row tile ti)
            // is read from LDS only when ti changes
            bf16x8 a;
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                if (q < nq) {
                    if (q == 0 || (offs[q] & 0xffffu) != (offs[q - 1] & 0xffffu))
                        a = __builtin_bit_cast(bf16x8,
                                               *reinterpret_cast<const u32x4v *>(asrc + (offs[q] & 0xffffu) + kk));
                    const bf16x8 b = __builtin_bit_cast(
                        bf16x8, *reinterpret_cast<const u32x4v *>(plain + (offs[q] >> 16) + kk));
                    acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[q], 0, 0, 0);
                }
            }
        }
        __syncthreads();   // the next chunk rewrites the LDS tiles
    }
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        if (q < nq) {
            float *out = part + ((int64_t)s * npairs + pair0 + q) * (kMT * kMT);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int m = 8 * (i / 4) + 4 * (lane / 32) + (i % 4), n = lane % 32;
                out[m * kMT + n] = acc[q][i];
            }
        }
    }
}

// Wide X (more than kLdsMaxTiles row tiles): the tile pairs are cut into blocks of
// kBlkTiles x kBlkTiles pairs (row block I, column block J >= I), and a workgroup stages
// only the 2 kBlkTiles row tiles its block touches (kBlkTiles on the diagonal), so the
// LDS holds 8 tiles x 32 rows x (KC + 8) BF16, twice with weights: 139 KB at KC = 128.
// Waves take kBlkPairsPerWave pairs of the block; same partial layout as the kernels above.
constexpr int kBlkTiles = 4;
constexpr int kBlkPairsPerWave = kBlkTiles * kBlkTiles / kSyrkBfWaves;   // 4

__host__ __device__ __forceinline__ int pair_index(int ti, int tj, int nt)
{
    return ti * nt - ti * (ti - 1) / 2 + (tj - ti);   // row-major upper triangle, ti <= tj
}

template <bool WEIGHT, int KC>
__global__ __launch_bounds__(64 * kSyrkBfWaves) void syrk_bf16_blk_kernel(const uint16_t *u, int64_t ldu, int p,
                                                                          const double *c, int64_t K, int64_t kchunk,
                                                                          float *part)
{
    constexpr int kStride = KC + 8, kPieces = KC / 8;
    constexpr int kRows = 2 * kBlkTiles * kMT;                                // staged rows (off-diagonal block)
    constexpr int kPerThread = kRows * kPieces / (64 * kSyrkBfWaves);      // 16 at KC = 128
    extern __shared__ uint16_t sh[];   // [kRows][kStride] plain, then weighted (WEIGHT)
    __shared__ float cw[KC];
    uint16_t *plain = sh;
    uint16_t *wtd = sh + (size_t)kRows * kStride;
    const int nt = (p + kMT - 1) / kMT;
    const int nb = (nt + kBlkTiles - 1) / kBlkTiles;
    const int npairs = nt * (nt + 1) / 2;
    int I, J;
    int s, grp;
    split_group(s, grp);
    tile_pair(grp, nb, I, J);
    const bool diag = I == J;
    const int nst = diag ? kBlkTiles : 2 * kBlkTiles;     // staged tiles
    const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
    const int64_t k0 = (int64_t)s * kchunk;
    const int64_t k1 = k0 + kchunk < K ? k0 + kchunk : K;
    // this wave's pairs: local tiles (la, lb) of the staged rows, global pair index, valid flag
    int la[kBlkPairsPerWave], lb[kBlkPairsPerWave], gp[kBlkPairsPerWave];
    bool ok[kBlkPairsPerWave];
    f32x16 acc[kBlkPairsPerWave];
#pragma unroll
    for (int q = 0; q < kBlkPairsPerWave; ++q) {
        const int idx = w * kBlkPairsPerWave + q;
        int a, b;
        if (diag) {
            tile_pair(idx < kBlkTiles * (kBlkTiles + 1) / 2 ? idx : 0, kBlkTiles, a, b);
            ok[q] = idx < kBlkTiles * (kBlkTiles + 1) / 2;
            la[q] = a;
            lb[q] = b;
        } else {
            a = idx / kBlkTiles;
            b = idx % kBlkTiles;
            ok[q] = true;
            la[q] = a;
            lb[q] = kBlkTiles + b;
        }
        const int ti = I * kBlkTiles + a, tj = J * kBlkTiles + b;
        ok[q] = ok[q] && ti < nt && tj < nt;
        gp[q] = ok[q] ? pair_index(ti, tj, nt) : 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[q][i] = 0.0f;
    }
    const int rsub = lane & 31, ksub = 8 * (lane >> 5);
    const int npieces = nst * kMT * kPieces;
    u32x4v reg[kPerThread];
    float creg = 0.0f;
    auto global_row = [&](int lr) {
        const int lt = lr / kMT;
        const int gt = lt < kBlkTiles ? I * kBlkTiles + lt : J * kBlkTiles + (lt - kBlkTiles);
        return gt * kMT + lr % kMT;
    };
    auto load_chunk = [&](int64_t kc) {
#pragma unroll
        for (int m = 0; m < kPerThread; ++m) {
            const int e = threadIdx.x + 64 * kSyrkBfWaves * m;
            const int lr = e / kPieces, piece = e % kPieces;
            u32x4v v = {0u, 0u, 0u, 0u};
            if (e < npieces) {
                const int r = global_row(lr);
                if (r < p) v = *reinterpret_cast<const u32x4v *>(u + (int64_t)r * ldu + kc + 8 * piece);
            }
            reg[m] = v;
        }
        if (WEIGHT && threadIdx.x < KC) creg = (float)c[kc + threadIdx.x];
    };
    if (k0 < k1) load_chunk(k0);
    for (int64_t kc = k0; kc < k1; kc += KC) {
        if (WEIGHT && threadIdx.x < KC) cw[threadIdx.x] = creg;
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kPerThread; ++m) {
            const int e = threadIdx.x + 64 * kSyrkBfWaves * m;
            if (e < npieces) {
                const int lr = e / kPieces, piece = e % kPieces;
                *reinterpret_cast<u32x4v *>(plain + lr * kStride + 8 * piece) = reg[m];
                if (WEIGHT) {
                    const bf16x8 x = __builtin_bit_cast(bf16x8, reg[m]);
                    bf16x8 y;
#pragma unroll
                    for (int i = 0; i < 8; ++i) y[i] = (__bf16)((float)x[i] * cw[8 * piece + i]);
                    *reinterpret_cast<u32x4v *>(wtd + lr * kStride + 8 * piece) = __builtin_bit_cast(u32x4v, y);
                }
            }
        }
        __syncthreads();
        if (kc + KC < k1) load_chunk(kc + KC);   // in flight during the MFMAs below
        const uint16_t *asrc = WEIGHT ? wtd : plain;
#pragma unroll
        for (int sub = 0; sub < KC / 16; ++sub) {
            const int kk = 16 * sub + ksub;
#pragma unroll
            for (int q = 0; q < kBlkPairsPerWave; ++q) {
                if (ok[q]) {
                    const bf16x8 a = __builtin_bit_cast(
                        bf16x8, *reinterpret_cast<const u32x4v *>(asrc + (la[q] * kMT + rsub) * kStride + kk));
                    const bf16x8 b = __builtin_bit_cast(
                        bf16x8, *reinterpret_cast<const u32x4v *>(plain + (lb[q] * kMT + rsub) * kStride + kk));
                    acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[q], 0, 0, 0);
                }
            }
        }
        __syncthreads();   // the next chunk rewrites the LDS tiles
    }
#pragma unroll
    for (int q = 0; q < kBlkPairsPerWave; ++q) {
        if (ok[q]) {
            float *out = part + ((int64_t)s * npairs + gp[q]) * (kMT * kMT);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int m = 8 * (i / 4) + 4 * (lane / 32) + (i % 4), n = lane % 32;
                out[m * kMT + n] = acc[q][i];
            }
        }
    }
}

// ------------------------------------------------------------------ FP8 (e4m3) on the matrix cores
//
// X is stored as e4m3 with a power-of-two scale per column (|x / s| <= 224).
// For X' diag(b) X both operands are the same matrix a_rj = (x_rj / s_j)
// sqrt(b_r) / S, with S the power of two >= sqrt(max b): each 64-row K chunk
// of every row tile is read once, multiplied by sqrt(b_r)/S in FP32 and
// rounded to e4m3 into LDS, and the waves run v_mfma_scale_f32_32x32x64_f8f6f4
// (unit block scales) on their tile pairs.  The FP32 partials are summed in
// FP64 times s_i s_j S^2.

constexpr float kFp8Max = 224.0f;   // below the e4m3 maximum of either encoding
constexpr int kF8KC = 64, kF8Stride = 80;   // bytes per LDS row (64 + 16 pad)
constexpr int kF8MaxRows = 800;                // p <= 800 (rows = p rounded up to 32)
typedef int i32x8v __attribute__((ext_vector_type(8)));

// The e4m3 copy is stored in blocks of kF8KC rows of X: block k holds, for each
// of the prow (= p rounded up to 32) columns in turn, its kF8KC bytes (zero for
// the padding columns), so the contraction reads each chunk as one contiguous
// stretch of prow * kF8KC bytes.
__global__ __launch_bounds__(256) void to_fp8_kernel(const double *x, int64_t ld, int p, int prow,
                                                     const float *xscale, uint8_t *x8)
{
    const int j = blockIdx.y;
    const int64_t r = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (r >= ld) return;
    int v = 0;
    if (j < p) {
        const double inv = 1.0 / (double)xscale[j];
        const double *src = x + (int64_t)j * ld + r;
        v = __builtin_amdgcn_cvt_pk_fp8_f32((float)(src[0] * inv), (float)(src[1] * inv), 0, false);
        v = __builtin_amdgcn_cvt_pk_fp8_f32((float)(src[2] * inv), (float)(src[3] * inv), v, true);
    }
    *reinterpret_cast<int *>(x8 + ((r / kF8KC) * prow + j) * kF8KC + r % kF8KC) = v;
}

// wsc[0] = S = 2^ceil(log2(sqrt(max b))) (1 if b is all zero), in two launches
__global__ __launch_bounds__(256) void bmax_kernel(const double *b, int64_t n, double *blockmax)
{
    __shared__ double red[4];
    double m = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256) m = fmax(m, b[r]);
    for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) blockmax[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ __launch_bounds__(256) void wscale_kernel(const double *blockmax, int nb, double *wsc)
{
    __shared__ double red[4];
    double m = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) m = fmax(m, blockmax[i]);
    for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        wsc[0] = m > 0.0 ? exp2(ceil(log2(sqrt(m)))) : 1.0;
    }
}

// Two waves per SIMD (registers capped at 256, accumulators included): the
// products of one chunk overlap the other wave's staging.
// MAXR: the most staged rows (p rounded up to 32) the launch may have; it sizes the prefetch
// registers.  NWV waves of TPW tile pairs each, registers cut for two workgroups per compute unit.
template <int MAXR, int NWV = kSyrkBfWaves, int TPW = kTilesPerWave>
__global__ __launch_bounds__(64 * NWV, NWV / 2) void syrk_fp8_lds_kernel(const uint8_t *u, int p,
                                                                        const double *c, const double *wsc,
                                                                        int64_t K, int64_t kchunk, float *part)
{
    extern __shared__ uint8_t sh8[];   // [nt*32][kF8Stride]
    __shared__ float cw[kF8KC];
    const int nt = (p + kMT - 1) / kMT;
    const int rows = nt * kMT;
    const int npairs = nt * (nt + 1) / 2;
    const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
    int s, grp;
    split_group(s, grp);
    const int pair0 = grp * kPairsPerGroup + w * TPW;
    const int nq = npairs - pair0 < TPW ? (npairs - pair0 > 0 ? npairs - pair0 : 0) : TPW;
    const int64_t k0 = (int64_t)s * kchunk;
    const int64_t k1 = k0 + kchunk < K ? k0 + kchunk : K;
    const double invS = 1.0 / wsc[0];
    const int rsub = lane & 31, kofs = 32 * (lane >> 5);
    // LDS byte offsets of this lane's A and B rows for each tile pair, packed 16 bits each
    // (at most kF8MaxRows rows of kF8Stride bytes: < 2^16)
    uint32_t offs[TPW];
    f32x16 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        int ti, tj;
        tile_pair(pair0 + q < npairs ? pair0 + q : 0, nt, ti, tj);
        offs[q] = (uint32_t)((ti * kMT + rsub) * kF8Stride + kofs) |
                  ((uint32_t)((tj * kMT + rsub) * kF8Stride + kofs) << 16);
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[q][i] = 0.0f;
    }
    // the chunk is one contiguous block of rows x 64 bytes (padding rows are zero), read
    // as 16-byte pieces e = tid + 256 m into registers one chunk ahead
    static_assert(NWV * TPW == kPairsPerGroup, "a group holds kPairsPerGroup tile pairs");
    constexpr int kPieces = (MAXR * 4 + 64 * NWV - 1) / (64 * NWV);
    const int npieces = rows * 4;
    u32x4v reg[kPieces];
    double creg = 0.0;
    auto load_chunk = [&](int64_t kc) {
        const u32x4v *blk = reinterpret_cast<const u32x4v *>(u + (kc / kF8KC) * (int64_t)rows * kF8KC);
#pragma unroll
        for (int m = 0; m < kPieces; ++m) {
            const int e = threadIdx.x + 64 * NWV * m;
            u32x4v v = {0u, 0u, 0u, 0u};
            if (e < npieces) v = blk[e];
            reg[m] = v;
        }
        if (threadIdx.x < kF8KC) creg = c[kc + threadIdx.x];
    };
    if (k0 < k1) load_chunk(k0);
    for (int64_t kc = k0; kc < k1; kc += kF8KC) {
        if (threadIdx.x < kF8KC) cw[threadIdx.x] = (float)(sqrt(creg) * invS);
        __syncthreads();
        // decode, weight, re-encode into LDS; every piece of this thread covers the same
        // 16 rows of the chunk (piece = tid mod 4), so it needs 16 weights
        const int piece = threadIdx.x & 3;
        const float *wk = cw + 16 * piece;
#pragma unroll
        for (int m = 0; m < kPieces; ++m) {
            const int e = threadIdx.x + 64 * NWV * m;
            if (e < npieces) {
                const u32x4v raw = reg[m];
                u32x4v v;
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const int word = (int)raw[d];
                    int o = __builtin_amdgcn_cvt_pk_fp8_f32(__builtin_amdgcn_cvt_f32_fp8(word, 0) * wk[4 * d],
                                                            __builtin_amdgcn_cvt_f32_fp8(word, 1) * wk[4 * d + 1], 0,
                                                            false);
                    o = __builtin_amdgcn_cvt_pk_fp8_f32(__builtin_amdgcn_cvt_f32_fp8(word, 2) * wk[4 * d + 2],
                                                        __builtin_amdgcn_cvt_f32_fp8(word, 3) * wk[4 * d + 3], o, true);
                    v[d] = (unsigned)o;
                }
                *reinterpret_cast<u32x4v *>(sh8 + (e >> 2) * kF8Stride + 16 * piece) = v;
            }
        }
        __syncthreads();
        if (kc + kF8KC < k1) load_chunk(kc + kF8KC);   // in flight during the products below
        // a wave's pairs run along rows of the upper triangle: the A fragment (row tile ti) is
        // read from LDS only when ti changes
        i32x8v av;
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            if (q < nq) {
                if (q == 0 || (offs[q] & 0xffffu) != (offs[q - 1] & 0xffffu)) {
                    const uint8_t *pa = sh8 + (offs[q] & 0xffffu);
                    const u32x4v a0 = *reinterpret_cast<const u32x4v *>(pa);
                    const u32x4v a1 = *reinterpret_cast<const u32x4v *>(pa + 16);
                    av = i32x8v{(int)a0[0], (int)a0[1], (int)a0[2], (int)a0[3],
                                (int)a1[0], (int)a1[1], (int)a1[2], (int)a1[3]};
                }
                const uint8_t *pb = sh8 + (offs[q] >> 16);
                const u32x4v b0 = *reinterpret_cast<const u32x4v *>(pb), b1 = *reinterpret_cast<const u32x4v *>(pb + 16);
                const i32x8v bv = {(int)b0[0], (int)b0[1], (int)b0[2], (int)b0[3],
                                   (int)b1[0], (int)b1[1], (int)b1[2], (int)b1[3]};
                acc[q] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc[q], 0, 0, 0, 127, 0, 127);
            }
        }
        __syncthreads();   // the next chunk rewrites the LDS tiles
    }
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        if (q < nq) {
            float *out = part + ((int64_t)s * npairs + pair0 + q) * (kMT * kMT);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int m = 8 * (i / 4) + 4 * (lane / 32) + (i % 4), n = lane % 32;
                out[m * kMT + n] = acc[q][i];
            }
        }
    }
}

// Wide X in FP8 (more than kF8MaxRows rows): blocks of kBlkTiles x kBlkTiles tile pairs as in
// syrk_bf16_blk_kernel; a workgroup stages only the row tiles of its block (8 tiles x 32 rows
// x 80 bytes of LDS) with the same decode / weight / re-encode as syrk_fp8_lds_kernel.
__global__ __launch_bounds__(64 * kSyrkBfWaves) void syrk_fp8_blk_kernel(const uint8_t *u, int p, const double *c,
                                                                         const double *wsc, int64_t K, int64_t kchunk,
                                                                         float *part)
{
    constexpr int kRows = 2 * kBlkTiles * kMT;                                   // staged rows
    constexpr int kPieces = kRows * 4 / (64 * kSyrkBfWaves);                    // 4 per thread
    __shared__ uint8_t sh8[kRows * kF8Stride];
    __shared__ float cw[kF8KC];
    const int nt = (p + kMT - 1) / kMT;
    const int rows = nt * kMT;
    const int nb = (nt + kBlkTiles - 1) / kBlkTiles;
    const int npairs = nt * (nt + 1) / 2;
    int I, J;
    int s, grp;
    split_group(s, grp);
    tile_pair(grp, nb, I, J);
    const bool diag = I == J;
    const int nst = diag ? kBlkTiles : 2 * kBlkTiles;
    const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
    const int64_t k0 = (int64_t)s * kchunk;
    const int64_t k1 = k0 + kchunk < K ? k0 + kchunk : K;
    const double invS = 1.0 / wsc[0];
    int la[kBlkPairsPerWave], lb[kBlkPairsPerWave], gp[kBlkPairsPerWave];
    bool ok[kBlkPairsPerWave];
    f32x16 acc[kBlkPairsPerWave];
#pragma unroll
    for (int q = 0; q < kBlkPairsPerWave; ++q) {
        const int idx = w * kBlkPairsPerWave + q;
        int a, b;
        if (diag) {
            ok[q] = idx < kBlkTiles * (kBlkTiles + 1) / 2;
            tile_pair(ok[q] ? idx : 0, kBlkTiles, a, b);
            la[q] = a;
            lb[q] = b;
        } else {
            a = idx / kBlkTiles;
            b = idx % kBlkTiles;
            ok[q] = true;
            la[q] = a;
            lb[q] = kBlkTiles + b;
        }
        const int ti = I * kBlkTiles + a, tj = J * kBlkTiles + b;
        ok[q] = ok[q] && ti < nt && tj < nt;
        gp[q] = ok[q] ? pair_index(ti, tj, nt) : 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[q][i] = 0.0f;
    }
    const int rsub = lane & 31, kofs = 32 * (lane >> 5);
    const int npieces = nst * kMT * 4;
    u32x4v reg[kPieces];
    double creg = 0.0;
    auto load_chunk = [&](int64_t kc) {
        const uint8_t *blk = u + (kc / kF8KC) * (int64_t)rows * kF8KC;
#pragma unroll
        for (int m = 0; m < kPieces; ++m) {
            const int e = threadIdx.x + 64 * kSyrkBfWaves * m;
            u32x4v v = {0u, 0u, 0u, 0u};
            if (e < npieces) {
                const int lr = e >> 2, lt = lr / kMT;
                const int gt = lt < kBlkTiles ? I * kBlkTiles + lt : J * kBlkTiles + (lt - kBlkTiles);
                if (gt < nt)
                    v = *reinterpret_cast<const u32x4v *>(blk + (int64_t)(gt * kMT + lr % kMT) * kF8KC + 16 * (e & 3));
            }
            reg[m] = v;
        }
        if (threadIdx.x < kF8KC) creg = c[kc + threadIdx.x];
    };
    if (k0 < k1) load_chunk(k0);
    for (int64_t kc = k0; kc < k1; kc += kF8KC) {
        if (threadIdx.x < kF8KC) cw[threadIdx.x] = (float)(sqrt(creg) * invS);
        __syncthreads();
        const int piece = threadIdx.x & 3;
        float wk[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) wk[i] = cw[16 * piece + i];
#pragma unroll
        for (int m = 0; m < kPieces; ++m) {
            const int e = threadIdx.x + 64 * kSyrkBfWaves * m;
            if (e < npieces) {
                const u32x4v raw = reg[m];
                u32x4v v;
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const int word = (int)raw[d];
                    int o = __builtin_amdgcn_cvt_pk_fp8_f32(__builtin_amdgcn_cvt_f32_fp8(word, 0) * wk[4 * d],
                                                            __builtin_amdgcn_cvt_f32_fp8(word, 1) * wk[4 * d + 1], 0,
                                                            false);
                    o = __builtin_amdgcn_cvt_pk_fp8_f32(__builtin_amdgcn_cvt_f32_fp8(word, 2) * wk[4 * d + 2],
                                                        __builtin_amdgcn_cvt_f32_fp8(word, 3) * wk[4 * d + 3], o, true);
                    v[d] = (unsigned)o;
                }
                *reinterpret_cast<u32x4v *>(sh8 + (e >> 2) * kF8Stride + 16 * piece) = v;
            }
        }
        __syncthreads();
        if (kc + kF8KC < k1) load_chunk(kc + kF8KC);   // in flight during the products below
#pragma unroll
        for (int q = 0; q < kBlkPairsPerWave; ++q) {
            if (ok[q]) {
                const uint8_t *pa = sh8 + (la[q] * kMT + rsub) * kF8Stride + kofs;
                const uint8_t *pb = sh8 + (lb[q] * kMT + rsub) * kF8Stride + kofs;
                const u32x4v a0 = *reinterpret_cast<const u32x4v *>(pa), a1 = *reinterpret_cast<const u32x4v *>(pa + 16);
                const u32x4v b0 = *reinterpret_cast<const u32x4v *>(pb), b1 = *reinterpret_cast<const u32x4v *>(pb + 16);
                const i32x8v av = {(int)a0[0], (int)a0[1], (int)a0[2], (int)a0[3],
                                   (int)a1[0], (int)a1[1], (int)a1[2], (int)a1[3]};
                const i32x8v bv = {(int)b0[0], (int)b0[1], (int)b0[2], (int)b0[3],
                                   (int)b1[0], (int)b1[1], (int)b1[2], (int)b1[3]};
                acc[q] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc[q], 0, 0, 0, 127, 0, 127);
            }
        }
        __syncthreads();   // the next chunk rewrites the LDS tiles
    }
#pragma unroll
    for (int q = 0; q < kBlkPairsPerWave; ++q) {
        if (ok[q]) {
            float *out = part + ((int64_t)s * npairs + gp[q]) * (kMT * kMT);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int m = 8 * (i / 4) + 4 * (lane / 32) + (i % 4), n = lane % 32;
                out[m * kMT + n] = acc[q][i];
            }
        }
    }
}

// C (+)= sign * scale_i * scale_j * sum over ranges of the partial tiles (FP64).
// Grid (npairs, 16): each workgroup takes 64 entries of one tile; its 16
// waves sum the splits q = w, w + 16, ... in order, then the 16 sums are
// added in wave order (a fixed order, so results do not vary run to run).
__global__ __launch_bounds__(64 * kRedWaves) void syrk_bf16_reduce_kernel(const float *part, int p, int S,
                                                                          const float *scale, double sign,
                                                                          int accumulate, double *C, const double *wsc)
{
    __shared__ double red[kRedWaves][64];
    const int nt = (p + kMT - 1) / kMT;
    const int npairs = nt * (nt + 1) / 2;
    const int pair = blockIdx.x;
    int ti, tj;
    tile_pair(pair, nt, ti, tj);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int e = blockIdx.y * 64 + lane;
    double s = 0.0;
    for (int q = w; q < S; q += kRedWaves) s += (double)part[((int64_t)q * npairs + pair) * (kMT * kMT) + e];
    red[w][lane] = s;
    __syncthreads();
    if (w != 0) return;
    s = red[0][lane];
    for (int v = 1; v < kRedWaves; ++v) s += red[v][lane];
    const int a = e / kMT, bb = e % kMT;
    const int i = ti * kMT + a, j = tj * kMT + bb;
    if (i >= p || j >= p) return;
    if (ti == tj && j < i) return;
    s *= sign * (double)scale[i] * (double)scale[j];
    if (wsc) s *= wsc[0] * wsc[0];
    if (accumulate) {
        C[(int64_t)i * p + j] += s;
        if (i != j) C[(int64_t)j * p + i] += s;
    } else {
        C[(int64_t)i * p + j] = s;
        if (i != j) C[(int64_t)j * p + i] = s;
    }
}

// xscale_j = the power of two s with max|x_j| / s <= xmax (1 for a zero column);
// zscale_j = the power of two >= max|x_j| (the BF16 scale of xbar_j).
__global__ __launch_bounds__(256) void colscale_kernel(const double *x, int64_t ld, float xmax, float *xscale,
                                                       float *zscale)
{
    __shared__ double red[4];
    const int j = blockIdx.x;
    double m = 0.0;
    for (int64_t r = threadIdx.x; r < ld; r += 256) m = fmax(m, fabs(x[(int64_t)j * ld + r]));
    for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        xscale[j] = m > 0.0 ? (float)exp2(ceil(log2(m / (double)xmax))) : 1.0f;
        zscale[j] = m > 0.0 ? (float)exp2(ceil(log2(m))) : 1.0f;
    }
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const double *x, int64_t ld, const float *xscale,
                                                      uint16_t *xlp)
{
    const int j = blockIdx.y;
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r < ld) {
        const __hip_bfloat16 v = __float2bfloat16((float)(x[(int64_t)j * ld + r] / (double)xscale[j]));
        xlp[(int64_t)j * ld + r] = __builtin_bit_cast(uint16_t, v);
    }
}

}  // namespace

size_t syrk_bf16_partial_bytes(int p, int splits)
{
    return sizeof(float) * (size_t)splits * (size_t)npairs32(p) * kMT * kMT;
}

size_t syrk_partial_bytes(int p, int splits)
{
    const int nt = (p + kTile - 1) / kTile;
    return sizeof(double) * (size_t)splits * (size_t)(nt * (nt + 1) / 2) * kTile * kTile;
}

int syrk_f64(const double *u, int64_t ldu, int p, const double *c, int64_t K, int splits, double *part,
             double sign, int accumulate, double *C, hipStream_t stream)
{
    const int nt = (p + kTile - 1) / kTile;
    const int npairs = nt * (nt + 1) / 2;
    int64_t kchunk = (K + splits - 1) / splits;
    if (p <= 512) {
        // matrix cores, every row of u staged once per K chunk: 2 * splits K ranges at p <= 256
        // (one group of blocks), splits ranges of 4 groups beyond; fewer ranges when K is short
        // (at least 4 chunks each), the reduction reading every range's tiles
        const int nb = (p + 15) / 16, ngroups = (nb * (nb + 1) / 2 + kF64Group - 1) / kF64Group;
        int s2 = p <= 256 ? 2 * splits : splits;
        const int64_t most = (K + 4 * kF64KC - 1) / (4 * kF64KC);
        if (most < s2) s2 = most > 1 ? (int)most : 1;
        if (ngroups > 1 && s2 >= 8) s2 = s2 / 8 * 8;   // whole groups of 8 ranges: one XCD runs all groups of a range
        kchunk = (K + s2 - 1) / s2;
        kchunk = (kchunk + kF64KC - 1) / kF64KC * kF64KC;
        if (p <= 256) syrk_f64_mfma_kernel<16><<<dim3(s2, ngroups), 64 * kF64Waves, 0, stream>>>(u, ldu, p, c, K, kchunk, part);
        else syrk_f64_mfma_kernel<32><<<dim3(s2, ngroups), 64 * kF64Waves, 0, stream>>>(u, ldu, p, c, K, kchunk, part);
        syrk_reduce_kernel<<<dim3(npairs, kTile * kTile / 64), 64 * kRedWaves, 0, stream>>>(part, p, s2, sign,
                                                                                           accumulate, C);
        return hipGetLastError() == hipSuccess ? 0 : -3;
    }
    kchunk = (kchunk + kKc - 1) / kKc * kKc;
    syrk_f64_kernel<<<dim3(npairs, splits), kSyrkThreads, 0, stream>>>(u, ldu, p, c, K, kchunk, part);
    syrk_reduce_kernel<<<dim3(npairs, kTile * kTile / 64), 64 * kRedWaves, 0, stream>>>(part, p, splits, sign,
                                                                                       accumulate, C);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int make_bf16_copy(const double *x, int64_t ld, int p, void *xlp, float *xscale, float *zscale, hipStream_t stream)
{
    colscale_kernel<<<p, 256, 0, stream>>>(x, ld, 1.0f, xscale, zscale);
    to_bf16_kernel<<<dim3((unsigned)((ld + 255) / 256), p), 256, 0, stream>>>(x, ld, xscale,
                                                                             static_cast<uint16_t *>(xlp));
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int syrk_bf16(const uint16_t *u, int64_t ldu, int p, const float *scale, const double *c, int64_t K, int splits,
              double *part, double sign, int accumulate, double *C, hipStream_t stream)
{
    if (ldu % 16 != 0) return -1;
    const int npairs = npairs32(p);
    const int ngroups = (npairs + kPairsPerGroup - 1) / kPairsPerGroup;
    const int64_t K16 = (K + 15) / 16 * 16;          // entries K..K16-1 are zero (padding)
    if (K16 > ldu) return -1;
    float *fpart = reinterpret_cast<float *>(part);
    const int nt = (p + kMT - 1) / kMT;
    const int KC = nt <= 8 ? 128 : 64;
    const int64_t K64 = (K + KC - 1) / KC * KC;
    if (nt <= 8 && (K + 63) / 64 * 64 <= ldu && ldu % 8 == 0) {
        // two workgroups per compute unit, 64-row chunks (64.5 KB of LDS each with the weighted copy)
        const int64_t KB = (K + 63) / 64 * 64;
        const int s2 = 2 * splits;
        int64_t kchunk = (KB + s2 - 1) / s2;
        kchunk = (kchunk + 63) / 64 * 64;
        const size_t lds = sizeof(uint16_t) * (size_t)nt * kMT * (64 + 8) * (c ? 2 : 1);
        static bool attr2 = false;
        if (!attr2) {
            const size_t most = sizeof(uint16_t) * (size_t)8 * kMT * (64 + 8) * 2;
            const void *fns[] = {reinterpret_cast<const void *>(&syrk_bf16_lds_kernel<true, 64, 8, 4, 8, 4>),
                                 reinterpret_cast<const void *>(&syrk_bf16_lds_kernel<false, 64, 8, 4, 8, 4>)};
            for (const void *fn : fns)
                if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)most) != hipSuccess)
                    return -3;
            attr2 = true;
        }
        splits = s2;   // the reduce below sums the slices this launch writes
        const dim3 grid(s2, ngroups);
        if (c) syrk_bf16_lds_kernel<true, 64, 8, 4, 8, 4><<<grid, 64 * 8, lds, stream>>>(u, ldu, p, c, KB, kchunk, fpart);
        else syrk_bf16_lds_kernel<false, 64, 8, 4, 8, 4><<<grid, 64 * 8, lds, stream>>>(u, ldu, p, c, KB, kchunk, fpart);
    } else if (nt <= kLdsMaxTiles && K64 <= ldu && ldu % 8 == 0) {
        int64_t kchunk = (K64 + splits - 1) / splits;
        kchunk = (kchunk + KC - 1) / KC * KC;
        const size_t lds = sizeof(uint16_t) * (size_t)nt * kMT * (KC + 8) * (c ? 2 : 1);
        static bool attr = false;
        if (!attr) {
            const size_t most = sizeof(uint16_t) * (size_t)16 * kMT * (64 + 8) * 2;   // the largest of both shapes
            const void *fns[] = {reinterpret_cast<const void *>(&syrk_bf16_lds_kernel<true, 128>),
                                 reinterpret_cast<const void *>(&syrk_bf16_lds_kernel<false, 128>),
                                 reinterpret_cast<const void *>(&syrk_bf16_lds_kernel<true, 64>),
                                 reinterpret_cast<const void *>(&syrk_bf16_lds_kernel<false, 64>)};
            for (const void *fn : fns)
                if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)most) != hipSuccess)
                    return -3;
            attr = true;
        }
        const dim3 grid(splits, ngroups);
        if (KC == 128) {
            if (c) syrk_bf16_lds_kernel<true, 128><<<grid, 64 * kSyrkBfWaves, lds, stream>>>(u, ldu, p, c, K64, kchunk, fpart);
            else syrk_bf16_lds_kernel<false, 128><<<grid, 64 * kSyrkBfWaves, lds, stream>>>(u, ldu, p, c, K64, kchunk, fpart);
        } else {
            if (c) syrk_bf16_lds_kernel<true, 64><<<grid, 64 * kSyrkBfWaves, lds, stream>>>(u, ldu, p, c, K64, kchunk, fpart);
            else syrk_bf16_lds_kernel<false, 64><<<grid, 64 * kSyrkBfWaves, lds, stream>>>(u, ldu, p, c, K64, kchunk, fpart);
        }
    } else if (nt > kLdsMaxTiles && ldu % 8 == 0 && (K + 63) / 64 * 64 <= ldu) {
        // wide X: blocks of tile pairs, each staging only its row blocks
        const int BKC = (K + 127) / 128 * 128 <= ldu ? 128 : 64;
        const int64_t KB = (K + BKC - 1) / BKC * BKC;
        const int nb = (nt + kBlkTiles - 1) / kBlkTiles;
        const int nblocks = nb * (nb + 1) / 2;
        int bsplits = splits;
        if (bsplits * (int64_t)nblocks > 16384) bsplits = 16384 / nblocks > 1 ? 16384 / nblocks : 1;
        int64_t kchunk = (KB + bsplits - 1) / bsplits;
        kchunk = (kchunk + BKC - 1) / BKC * BKC;
        const size_t lds = sizeof(uint16_t) * (size_t)2 * kBlkTiles * kMT * (BKC + 8) * (c ? 2 : 1);
        static bool battr = false;
        if (!battr) {
            const size_t most = sizeof(uint16_t) * (size_t)2 * kBlkTiles * kMT * (128 + 8) * 2;
            const void *fns[] = {reinterpret_cast<const void *>(&syrk_bf16_blk_kernel<true, 128>),
                                 reinterpret_cast<const void *>(&syrk_bf16_blk_kernel<false, 128>),
                                 reinterpret_cast<const void *>(&syrk_bf16_blk_kernel<true, 64>),
                                 reinterpret_cast<const void *>(&syrk_bf16_blk_kernel<false, 64>)};
            for (const void *fn : fns)
                if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)most) != hipSuccess)
                    return -3;
            battr = true;
        }
        splits = bsplits;   // the reduce below sums the slices this launch writes
        const dim3 grid(bsplits, nblocks);
        if (BKC == 128) {
            if (c) syrk_bf16_blk_kernel<true, 128><<<grid, 64 * kSyrkBfWaves, lds, stream>>>(u, ldu, p, c, KB, kchunk, fpart);
            else syrk_bf16_blk_kernel<false, 128><<<grid, 64 * kSyrkBfWaves, lds, stream>>>(u, ldu, p, c, KB, kchunk, fpart);
        } else {
            if (c) syrk_bf16_blk_kernel<true, 64><<<grid, 64 * kSyrkBfWaves, lds, stream>>>(u, ldu, p, c, KB, kchunk, fpart);
            else syrk_bf16_blk_kernel<false, 64><<<grid, 64 * kSyrkBfWaves, lds, stream>>>(u, ldu, p, c, KB, kchunk, fpart);
        }
    } else {
        int64_t kchunk = (K16 + splits - 1) / splits;
        kchunk = (kchunk + 15) / 16 * 16;
        syrk_bf16_kernel<<<dim3(splits, ngroups), 64 * kSyrkBfWaves, 0, stream>>>(u, ldu, p, c, K16, kchunk, fpart);
    }
    syrk_bf16_reduce_kernel<<<dim3(npairs, 16), 64 * kRedWaves, 0, stream>>>(fpart, p, splits, scale, sign, accumulate, C,
                                                                 nullptr);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

size_t fp8_copy_bytes(int64_t ld, int p)
{
    return (size_t)ld * (size_t)((p + kMT - 1) / kMT * kMT);
}

int make_fp8_copy(const double *x, int64_t ld, int p, uint8_t *x8, float *xscale, float *zscale, hipStream_t stream)
{
    if (ld % kF8KC != 0) return -1;
    const int prow = (p + kMT - 1) / kMT * kMT;
    colscale_kernel<<<p, 256, 0, stream>>>(x, ld, kFp8Max, xscale, zscale);
    to_fp8_kernel<<<dim3((unsigned)((ld / 4 + 255) / 256), prow), 256, 0, stream>>>(x, ld, p, prow, xscale, x8);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int syrk_fp8(const uint8_t *u, int64_t ldu, int p, const float *scale, const double *c, int64_t K, int splits,
             double *part, double *blockmax, double *wsc, double sign, int accumulate, double *C, hipStream_t stream)
{
    const int nt = (p + kMT - 1) / kMT;
    const int npairs = nt * (nt + 1) / 2;
    const int ngroups = (npairs + kPairsPerGroup - 1) / kPairsPerGroup;
    const int64_t K64 = (K + kF8KC - 1) / kF8KC * kF8KC;
    if (K64 > ldu || ldu % kF8KC != 0) return -1;
    bmax_kernel<<<256, 256, 0, stream>>>(c, K, blockmax);
    wscale_kernel<<<1, 256, 0, stream>>>(blockmax, 256, wsc);
    if (nt * kMT > kF8MaxRows) {
        // wide X: blocks of tile pairs, each staging only its row blocks
        const int nb = (nt + kBlkTiles - 1) / kBlkTiles;
        const int nblocks = nb * (nb + 1) / 2;
        int bsplits = splits;
        if (bsplits * (int64_t)nblocks > 16384) bsplits = 16384 / nblocks > 1 ? 16384 / nblocks : 1;
        int64_t kchunk = (K64 + bsplits - 1) / bsplits;
        kchunk = (kchunk + kF8KC - 1) / kF8KC * kF8KC;
        float *fpart = reinterpret_cast<float *>(part);
        syrk_fp8_blk_kernel<<<dim3(bsplits, nblocks), 64 * kSyrkBfWaves, 0, stream>>>(u, p, c, wsc, K64, kchunk, fpart);
        syrk_bf16_reduce_kernel<<<dim3(npairs, 16), 64 * kRedWaves, 0, stream>>>(fpart, p, bsplits, scale, sign, accumulate, C,
                                                                     wsc);
        return hipGetLastError() == hipSuccess ? 0 : -3;
    }
    // two workgroups per compute unit are resident: size the grid to whole rounds of them
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    int fit = (4 * cus) / ngroups;
    if (fit >= 8) fit = fit / 8 * 8;   // whole groups of 8 K ranges: one XCD runs all groups of a range
    if (fit >= 1 && fit < splits) splits = fit;
    int64_t kchunk = (K64 + splits - 1) / splits;
    kchunk = (kchunk + kF8KC - 1) / kF8KC * kF8KC;
    const size_t lds = (size_t)nt * kMT * kF8Stride;
    float *fpart = reinterpret_cast<float *>(part);
    if (nt * kMT <= 512)
        syrk_fp8_lds_kernel<512><<<dim3(splits, ngroups), 64 * kSyrkBfWaves, lds, stream>>>(u, p, c, wsc, K64, kchunk,
                                                                                          fpart);
    else
        syrk_fp8_lds_kernel<kF8MaxRows><<<dim3(splits, ngroups), 64 * kSyrkBfWaves, lds, stream>>>(u, p, c, wsc, K64,
                                                                                                 kchunk, fpart);
    syrk_bf16_reduce_kernel<<<dim3(npairs, 16), 64 * kRedWaves, 0, stream>>>(fpart, p, splits, scale, sign, accumulate, C, wsc);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// Proximal Newton's model solve: cyclic coordinate descent with soft thresholding (the l1
// rule of Sec. 2.4, applied to the quadratic model of the objective)
//   min_D  g'D + D'HD/2 + sum_j gamma_j |beta_j + D_j|
// in one wave.  Every lane takes the same scalar decision for coordinate j from inputs
// broadcast out of LDS; lane l keeps HD[k] (k = l mod 64) up to date from row j of the
// symmetric H when D_j moves.  Row j+1's first kProxPre * 64 entries are loaded into
// registers while coordinate j is decided.  Coordinates not free, or with H_jj <= 0 or not
// finite, stay at 0.  Stops after the first sweep whose largest |change| is <= tol, or after
// max_sweeps sweeps.
constexpr int kProxChunk = 1024;   // coordinates whose inputs are staged in LDS at a time
constexpr int kProxPre = 16;       // prefetched entries of a row per lane (1024 columns)

__global__ __launch_bounds__(64) void prox_cd_kernel(const double *H, int p, const double *g, const double *beta,
                                                     const double *gam, const uint8_t *free_col, double tol,
                                                     int max_sweeps, double *D, int *sweeps_out)
{
    extern __shared__ double sm[];   // HD[p], Dv[p]
    double *HD = sm, *Dv = sm + p;
    __shared__ double cg[kProxChunk], cb[kProxChunk], cgam[kProxChunk], ca[kProxChunk];
    const int lane = threadIdx.x;
    for (int k = lane; k < p; k += 64) {
        HD[k] = 0.0;
        Dv[k] = 0.0;
    }
    double nxt[kProxPre];
    auto load_row = [&](int j) {
        const double *row = H + (size_t)j * p;
#pragma unroll
        for (int m = 0; m < kProxPre; ++m) {
            const int k = lane + 64 * m;
            nxt[m] = k < p ? row[k] : 0.0;
        }
    };
    int sweep = 0;
    while (sweep < max_sweeps) {
        ++sweep;
        double change = 0.0;
        for (int j0 = 0; j0 < p; j0 += kProxChunk) {
            const int jn = p - j0 < kProxChunk ? p - j0 : kProxChunk;
            __syncthreads();
            for (int i = lane; i < jn; i += 64) {
                const int j = j0 + i;
                const double a = H[(size_t)j * p + j];
                cg[i] = g[j];
                cb[i] = beta[j];
                cgam[i] = gam[j];
                ca[i] = (free_col[j] && a > 0.0 && a < INFINITY) ? a : 0.0;
            }
            load_row(j0);
            __syncthreads();
            for (int i = 0; i < jn; ++i) {
                const int j = j0 + i;
                double cur[kProxPre];
#pragma unroll
                for (int m = 0; m < kProxPre; ++m) cur[m] = nxt[m];
                if (i + 1 < jn) load_row(j + 1);
                const double a = ca[i];
                if (a == 0.0) continue;
                const double bj = cb[i], gm = cgam[i], dj = Dv[j];
                const double b = cg[i] + HD[j] - a * dj;   // the model's slope at D with D_j removed
                const double u = a * bj - b;
                const double z = u > gm ? (u - gm) / a : (u < -gm ? (u + gm) / a : 0.0);
                const double dn = z - bj;
                const double delta = dn - dj;
                if (delta != 0.0) {
                    __syncthreads();   // every lane has read Dv[j] and HD[j]
                    if (lane == 0) Dv[j] = dn;
#pragma unroll
                    for (int m = 0; m < kProxPre; ++m) {
                        const int k = lane + 64 * m;
                        if (k < p) HD[k] += cur[m] * delta;
                    }
                    for (int k = lane + 64 * kProxPre; k < p; k += 64) HD[k] += H[(size_t)j * p + k] * delta;
                    change = fmax(change, fabs(delta));
                    __syncthreads();   // HD and Dv written before the next coordinate reads them
                }
            }
        }
        if (change <= tol) break;
    }
    __syncthreads();
    for (int k = lane; k < p; k += 64) D[k] = Dv[k];
    if (lane == 0) *sweeps_out = sweep;
}

int prox_model_solve(const double *H, int p, const double *g, const double *beta, const double *gam,
                     const uint8_t *free_col, double tol, int max_sweeps, double *D, int *sweeps, hipStream_t stream)
{
    if (p < 1 || p > 4096) return -1;
    const size_t lds = sizeof(double) * 2 * (size_t)p;
    static bool attr = false;
    if (!attr) {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(&prox_cd_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)(sizeof(double) * 2 * 4096)) !=
            hipSuccess)
            return -3;
        attr = true;
    }
    prox_cd_kernel<<<1, 64, lds, stream>>>(H, p, g, beta, gam, free_col, tol, max_sweeps, D, sweeps);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int chol_solve(double *A, int p, const double *g, const uint8_t *free_col, int factored, double *dx, int *status,
               hipStream_t stream)
{
    if (p <= kCholMaxP) {
        const size_t lds = sizeof(double) * ((size_t)p * kCholNB + 2 * (size_t)p);
        static bool attr = false;
        if (!attr) {
            const size_t most = sizeof(double) * ((size_t)kCholMaxP * kCholNB + 2 * (size_t)kCholMaxP);
            if (hipFuncSetAttribute(reinterpret_cast<const void *>(&chol_blocked_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)most) != hipSuccess)
                return -3;
            attr = true;
        }
        chol_blocked_kernel<<<1, kCholThreads, lds, stream>>>(A, p, g, free_col, factored, dx, status);
    } else {
        chol_solve_kernel<<<1, 256, sizeof(double) * (size_t)p, stream>>>(A, p, g, free_col, factored, dx, status);
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace coxmi
