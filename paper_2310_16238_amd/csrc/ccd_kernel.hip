// ccd_kernel.hip -- persistent cyclic-coordinate-descent kernel for the stratified Cox model (gfx950).
//
// What one coordinate j computes (Sec. 2.7):
//   D = exp(X beta), N1 = X_j * D, N2 = X_j^2 * D            (Eqs. parallel_d, parallel_n1, parallel_n2)
//   segmented scans S[D], S[N1], S[N2] over the canonical rows  (Sec. 2.6)
//   g'  = -delta'X_j + delta'(S[N1]/S[D])                      (Eq. parallel_g)
//   g'' =  delta'(S[N2]/S[D]) - delta'(S[N1]/S[D])^2           (Eq. parallel_h)
//   Newton step with trust region and l1 rule                   (Sec. 2.4, Eq. newton)
//   X beta += X_j * step                                        (Eq. parallel_xb)
// Ties: an event reads the scans at the last row of its tie group; the row
// word carries d = number of events of the group on that row, so the
// reductions are sum over group ends of d * (...).
//
// How it maps onto the MI355X (our design, not the paper's):
//   * One persistent cooperative launch runs the whole fit.  Workgroup b of
//     BLOCK threads owns rows [b*BLOCK*IPT, (b+1)*BLOCK*IPT); each thread keeps
//     its IPT rows of X beta and of the row word in registers for the whole
//     fit, so a coordinate reads only x_j from HBM (8 B/row).  x_{j+1} is
//     loaded while coordinate j synchronises.
//   * Rows inside a workgroup: thread fold -> wave64 shuffle scan -> LDS scan
//     of the 16 wave totals.  Between workgroups: each publishes its tile
//     aggregate with an agent-scope release; a workgroup whose first row is
//     not a stratum head folds its predecessors' aggregates back to the
//     nearest one containing a head (look-back, one wave, 64 tiles per step).
//   * The per-coordinate sums are reduced per workgroup (shuffles + LDS) and
//     published into a double-buffered array; every workgroup gathers all of
//     them in the same fixed order and computes the same scalar step, so no
//     broadcast round trip is needed and results are bit-reproducible.
//   * exp() uses one global shift c (the largest X beta of the previous
//     coordinate); ratios are shift-invariant and the objective adds c back.
//     A risk-set sum outside [1e-300, 1e300] stops the fit with a flag.
#include <math.h>

#include "internal.h"
#include "segscan.hpp"

namespace coxmi {

// Per-workgroup partial record.
enum { kPC1 = 0, kPC2 = 1, kPM2 = 2, kPObj = 3, kPEtaMax = 4, kPErr = 5 };

struct alignas(16) CtlBlock {
    SyncCtl ctl;
};

size_t sync_scratch_bytes(int grid)
{
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    size_t s = up(sizeof(SyncCtl));
    s += up(sizeof(TileAgg<3>) * (size_t)grid);
    s += up(sizeof(uint32_t) * (size_t)grid);
    s += up(sizeof(double) * kPartialDoubles * 2 * (size_t)grid);
    s += up(sizeof(uint32_t) * 2 * (size_t)grid);
    return s;
}

void carve_sync_scratch(void *base, int grid, CcdLaunch &L)
{
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    char *c = static_cast<char *>(base);
    L.ctl = c;
    c += up(sizeof(SyncCtl));
    L.agg = c;
    c += up(sizeof(TileAgg<3>) * (size_t)grid);
    L.stat1 = reinterpret_cast<uint32_t *>(c);
    c += up(sizeof(uint32_t) * (size_t)grid);
    L.part = reinterpret_cast<double *>(c);
    c += up(sizeof(double) * kPartialDoubles * 2 * (size_t)grid);
    L.stat2 = reinterpret_cast<uint32_t *>(c);
}

// ------------------------------------------------------------------ small helpers

template <int IPT>
__device__ __forceinline__ void load_rows(double (&v)[IPT], const double *p)
{
    if constexpr (IPT % 2 == 0) {
        const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
        for (int i = 0; i < IPT / 2; ++i) {
            double2 t = q[i];
            v[2 * i] = t.x;
            v[2 * i + 1] = t.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < IPT; ++i) v[i] = p[i];
    }
}

template <int IPT>
__device__ __forceinline__ void load_words(uint32_t (&v)[IPT], const uint32_t *p)
{
    if constexpr (IPT % 4 == 0) {
        const uint4 *q = reinterpret_cast<const uint4 *>(p);
#pragma unroll
        for (int i = 0; i < IPT / 4; ++i) {
            uint4 t = q[i];
            v[4 * i] = t.x; v[4 * i + 1] = t.y; v[4 * i + 2] = t.z; v[4 * i + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < IPT; ++i) v[i] = p[i];
    }
}

__device__ __forceinline__ void partial_identity(double (&v)[kPartialDoubles])
{
    v[kPC1] = 0.0; v[kPC2] = 0.0; v[kPM2] = 0.0; v[kPObj] = 0.0;
    v[kPEtaMax] = -INFINITY; v[kPErr] = 0.0;
}

__device__ __forceinline__ void partial_combine(double (&a)[kPartialDoubles], const double (&b)[kPartialDoubles])
{
    a[kPC1] += b[kPC1];
    a[kPC2] += b[kPC2];
    a[kPM2] += b[kPM2];
    a[kPObj] += b[kPObj];
    a[kPEtaMax] = fmax(a[kPEtaMax], b[kPEtaMax]);
    a[kPErr] = fmax(a[kPErr], b[kPErr]);
}

// Butterfly reduction: every lane ends with the same total (+ and max commute).
__device__ __forceinline__ void wave_allreduce_partial(double (&v)[kPartialDoubles])
{
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) {
        double o[kPartialDoubles];
#pragma unroll
        for (int k = 0; k < kPartialDoubles; ++k) o[k] = __shfl_xor(v[k], off, kWave);
        partial_combine(v, o);
    }
}

// Workgroup reduction; the total is valid in every lane of wave 0.
template <int NW>
__device__ __forceinline__ void block_reduce_partial(double (&v)[kPartialDoubles],
                                                     double (*red)[kPartialDoubles])
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    wave_allreduce_partial(v);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < kPartialDoubles; ++k) red[w][k] = v[k];
    }
    __syncthreads();
    if (w == 0) {
        double x[kPartialDoubles];
        if (lane < NW) {
#pragma unroll
            for (int k = 0; k < kPartialDoubles; ++k) x[k] = red[lane][k];
        } else {
            partial_identity(x);
        }
        wave_allreduce_partial(x);
#pragma unroll
        for (int k = 0; k < kPartialDoubles; ++k) v[k] = x[k];
    }
}

// Publish this workgroup's record for `epoch` and gather the records of all
// workgroups (wave 0 only).  Sums in a fixed order, so every workgroup gets a
// bit-identical total.  Returns false on abort.
__device__ __forceinline__ bool exchange_partials(double (&v)[kPartialDoubles], int b, int G,
                                                  uint32_t epoch, double *part, uint32_t *stat2,
                                                  SyncCtl *ctl)
{
    const int lane = threadIdx.x & (kWave - 1);
    const size_t par = epoch & 1u;
    double *base = part + par * (size_t)G * kPartialDoubles;
    uint32_t *st = stat2 + par * (size_t)G;
    if (lane == 0) {
        double *mine = base + (size_t)b * kPartialDoubles;
#pragma unroll
        for (int k = 0; k < kPartialDoubles; ++k) mine[k] = v[k];
        store_release(&st[b], epoch);
    }
    bool ok = true;
    for (int q = lane; q < G; q += kWave)
        if (ok) ok = wait_equal(&st[q], epoch, ctl);
    if (__any(!ok)) return false;
    double acc[kPartialDoubles];
    partial_identity(acc);
    for (int q = lane; q < G; q += kWave) {
        double o[kPartialDoubles];
        const double *pq = base + (size_t)q * kPartialDoubles;
#pragma unroll
        for (int k = 0; k < kPartialDoubles; ++k) o[k] = pq[k];
        partial_combine(acc, o);
    }
    wave_allreduce_partial(acc);
#pragma unroll
    for (int k = 0; k < kPartialDoubles; ++k) v[k] = acc[k];
    return true;
}

// One CCD coordinate update (Sec. 2.4).  Newton step on the smooth part; with
// an l1 weight the step uses g' + gamma sgn(beta) away from 0, and at 0 the
// one-sided directional derivatives g' + gamma / g' - gamma pick the side (or
// no move).  The step is limited to the trust-region half-width, a step that
// would carry beta through 0 stops at 0, and the half-width becomes
// max(2 |step|, half-width / 2).  Columns with numerically zero curvature
// (g'' <= 1e-12 delta'(S[N2]/S[D])) do not move.
__device__ __forceinline__ double ccd_step(double beta, double g1, double g2, double m2, double gamma,
                                           double *trust, int *pinned)
{
    if (!(g2 > 1e-12 * fabs(m2)) || !isfinite(g2)) {
        *pinned = 1;
        return 0.0;
    }
    double d;
    if (gamma <= 0.0)
        d = -g1 / g2;
    else if (beta > 0.0)
        d = -(g1 + gamma) / g2;
    else if (beta < 0.0)
        d = -(g1 - gamma) / g2;
    else if (g1 + gamma < 0.0)
        d = -(g1 + gamma) / g2;
    else if (g1 - gamma > 0.0)
        d = -(g1 - gamma) / g2;
    else
        d = 0.0;
    const double lim = *trust;
    double s = fabs(d) > lim ? lim : fabs(d);
    s = d < 0.0 ? -s : s;
    if (gamma > 0.0 && beta != 0.0) {
        const double nb = beta + s;
        if ((beta > 0.0 && nb < 0.0) || (beta < 0.0 && nb > 0.0)) s = -beta;
    }
    const double t2 = 2.0 * fabs(s), half = 0.5 * lim;
    *trust = t2 > half ? t2 : half;
    return s;
}

// ------------------------------------------------------------------ the persistent kernel

template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void ccd_kernel(CcdLaunch L)
{
    constexpr int NW = BLOCK / kWave;
    extern __shared__ double smem_dyn[];
    __shared__ BlockScanSmem<3, NW> ss;
    __shared__ double red[NW][kPartialDoubles];
    __shared__ SegVal<3> s_carry;
    __shared__ double s_step, s_shift;
    __shared__ int s_flag;   // 0 go on, 1 abort, 2 numeric stop, 3 converged, 4 sweep limit

    const int p = L.p;
    const int G = gridDim.x, b = blockIdx.x, t = threadIdx.x;
    const int lane = t & (kWave - 1), w = t / kWave;
    SyncCtl *ctl = static_cast<SyncCtl *>(L.ctl);
    TileAgg<3> *agg = static_cast<TileAgg<3> *>(L.agg);
    const int64_t ld = (int64_t)G * BLOCK * IPT;
    const int64_t tile0 = (int64_t)b * BLOCK * IPT;
    const int64_t row0 = tile0 + (int64_t)t * IPT;

    double *sbeta = smem_dyn, *strust = smem_dyn + p, *sgamma = smem_dyn + 2 * p;
    for (int j = t; j < p; j += BLOCK) {
        sbeta[j] = L.beta[j];
        strust[j] = 1.0;
        sgamma[j] = L.gamma[j];
    }
    uint32_t meta[IPT];
    double eta[IPT];
    load_words<IPT>(meta, L.meta + row0);
#pragma unroll
    for (int i = 0; i < IPT; ++i) eta[i] = 0.0;
    const bool tile_head = (L.meta[tile0] & kHeadBit) != 0u;
    __syncthreads();

    // X beta0 (columns with beta0_j = 0 are skipped)
    for (int j = 0; j < p; ++j) {
        const double bj = sbeta[j];
        if (bj != 0.0) {
            double xv[IPT];
            load_rows<IPT>(xv, L.x + (int64_t)j * ld + row0);
#pragma unroll
            for (int i = 0; i < IPT; ++i) eta[i] = fma(xv[i], bj, eta[i]);
        }
    }

    // initial shift: the largest X beta over the real rows
    uint32_t epoch = 1;
    {
        double v[kPartialDoubles];
        partial_identity(v);
#pragma unroll
        for (int i = 0; i < IPT; ++i)
            if (row0 + i < L.n) v[kPEtaMax] = fmax(v[kPEtaMax], eta[i]);
        block_reduce_partial<NW>(v, red);
        if (w == 0) {
            const bool ok = exchange_partials(v, b, G, epoch, L.part, L.stat2, ctl);
            if (lane == 0) {
                s_flag = ok ? 0 : 1;
                s_shift = v[kPEtaMax];
            }
        }
        __syncthreads();
        if (s_flag == 1) return;
    }
    double c = s_shift;

    const bool fit = (L.mode == kModeFit);
    const int jfirst = fit ? 0 : L.j0;
    const int jend = fit ? p : L.j1;
    double xc[IPT];
    load_rows<IPT>(xc, L.x + (int64_t)jfirst * ld + row0);

    // bookkeeping held by thread 0 of every workgroup (identical everywhere)
    int sweeps = 0, pinned = 0, pinned_last = 0;
    double maxstep = 0.0, last_maxstep = 0.0, objective = 0.0;
    int stop = 0;

    for (;;) {
        for (int j = jfirst; j < jend; ++j) {
            ++epoch;
            const int jn = (j + 1 < jend) ? j + 1 : jfirst;
            double xn[IPT];
            load_rows<IPT>(xn, L.x + (int64_t)jn * ld + row0);
            const bool want_obj = (j == jfirst);

            // pass 1: D, N1, N2 of the thread's rows and their fold
            double wv[IPT];
            SegVal<3> tagg = seg_identity<3>();
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                wv[i] = exp(eta[i] - c);
                SegVal<3> r;
                r.f = meta[i] >> 31;
                r.v[0] = wv[i];
                r.v[1] = xc[i] * wv[i];
                r.v[2] = xc[i] * r.v[1];
                tagg = seg_combine(tagg, r);
            }
            SegVal<3> exc = block_exclusive_scan(tagg, ss);
            if (t == 0) {
                agg[b].f = ss.block_total.f ? 1.0 : 0.0;
                agg[b].v[0] = ss.block_total.v[0];
                agg[b].v[1] = ss.block_total.v[1];
                agg[b].v[2] = ss.block_total.v[2];
                store_release(&L.stat1[b], epoch);
            }
            if (!tile_head) {
                if (w == 0) {
                    SegVal<3> carry;
                    const bool ok = look_back<3>(b, epoch, agg, L.stat1, ctl, carry);
                    if (lane == 0) {
                        s_carry = carry;
                        s_flag = ok ? 0 : 1;
                    }
                }
                __syncthreads();
                if (s_flag == 1) return;
                exc = seg_combine(s_carry, exc);
            }

            // pass 2: inclusive prefixes at group ends -> per-coordinate sums
            double v[kPartialDoubles];
            partial_identity(v);
            SegVal<3> run = exc;
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                SegVal<3> r;
                r.f = meta[i] >> 31;
                r.v[0] = wv[i];
                r.v[1] = xc[i] * wv[i];
                r.v[2] = xc[i] * r.v[1];
                run = seg_combine(run, r);
                if (row0 + i < L.n) v[kPEtaMax] = fmax(v[kPEtaMax], eta[i]);
                const uint32_t d = meta[i] & kCountMask;
                if (d != 0u) {
                    const double s0 = run.v[0];
                    if (!(s0 >= 1e-300) || !(s0 <= 1e300)) v[kPErr] = 1.0;
                    const double inv = 1.0 / s0;
                    const double r1 = run.v[1] * inv, r2 = run.v[2] * inv;
                    const double dd = (double)d;
                    v[kPC1] += dd * r1;
                    v[kPC2] += dd * (r2 - r1 * r1);
                    v[kPM2] += dd * r2;
                    if (want_obj) v[kPObj] += dd * (log(s0) + c);
                }
                if (want_obj && (meta[i] & kEventBit)) v[kPObj] -= eta[i];
            }
            block_reduce_partial<NW>(v, red);
            if (w == 0) {
                const bool ok = exchange_partials(v, b, G, epoch, L.part, L.stat2, ctl);
                if (lane == 0) {
                    int flag = ok ? 0 : 1;
                    double step = 0.0;
                    if (ok) {
                        const double g1 = -L.q[j] + v[kPC1], g2 = v[kPC2], m2 = v[kPM2];
                        if (v[kPErr] != 0.0) flag = 2;
                        if (b == 0) {
                            L.g1[j] = g1;
                            L.g2[j] = g2;
                            L.m2[j] = m2;
                        }
                        if (want_obj) {
                            objective = v[kPObj];
                            if (fit)
                                for (int k = 0; k < p; ++k) objective += sgamma[k] * fabs(sbeta[k]);
                        }
                        if (fit && flag == 0) {
                            int pin = 0;
                            step = ccd_step(sbeta[j], g1, g2, m2, sgamma[j], &strust[j], &pin);
                            sbeta[j] += step;
                            maxstep = fmax(maxstep, fabs(step));
                            pinned += pin;
                        }
                    }
                    s_step = step;
                    s_shift = v[kPEtaMax];
                    s_flag = flag;
                }
            }
            __syncthreads();
            if (s_flag == 1) return;
            if (s_flag == 2) {
                stop = 2;
                break;
            }
            const double step = s_step;
            c = s_shift;
            if (step != 0.0) {
#pragma unroll
                for (int i = 0; i < IPT; ++i) eta[i] = fma(xc[i], step, eta[i]);
            }
#pragma unroll
            for (int i = 0; i < IPT; ++i) xc[i] = xn[i];
        }
        if (stop || !fit) break;
        ++sweeps;
        if (t == 0) {
            double bmax = 1.0;
            for (int k = 0; k < p; ++k) bmax = fmax(bmax, fabs(sbeta[k]));
            int flag = 0;
            if (maxstep <= L.tol * bmax) flag = 3;
            else if (sweeps >= L.max_sweeps) flag = 4;
            last_maxstep = maxstep;
            pinned_last = pinned;
            maxstep = 0.0;
            pinned = 0;
            s_flag = flag;
        }
        __syncthreads();
        if (s_flag != 0) {
            stop = s_flag;
            break;
        }
    }

    if (b == 0) {
        __syncthreads();
        if (fit)
            for (int j = t; j < p; j += BLOCK) L.beta[j] = sbeta[j];
        if (t == 0) {
            L.result[kResSweeps] = sweeps;
            L.result[kResLastStep] = last_maxstep;
            L.result[kResObjective] = objective;
            L.result[kResPinned] = pinned_last;
            L.result[kResConverged] = (stop == 3) ? 1.0 : 0.0;
            L.result[kResNumeric] = (stop == 2) ? 1.0 : 0.0;
            L.result[kResCompleted] = 1.0;
        }
    }
}

// ------------------------------------------------------------------ raw segmented scan

constexpr int kScanBlock = 1024;

template <int IPT>
__global__ __launch_bounds__(kScanBlock) void segscan_kernel(const double *a, const uint8_t *head,
                                                             double *out, int64_t n, TileAgg<1> *agg,
                                                             uint32_t *stat, SyncCtl *ctl)
{
    constexpr int kBlock = kScanBlock;
    __shared__ BlockScanSmem<1, kBlock / kWave> ss;
    __shared__ SegVal<1> s_carry;
    __shared__ int s_flag;
    const int b = blockIdx.x, t = threadIdx.x;
    const int lane = t & (kWave - 1), w = t / kWave;
    const int64_t tile0 = (int64_t)b * kBlock * IPT;
    const int64_t row0 = tile0 + (int64_t)t * IPT;
    SegVal<1> e[IPT];
    SegVal<1> tagg = seg_identity<1>();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int64_t r = row0 + i;
        if (r < n) {
            e[i].f = (r == 0 || head[r] != 0) ? 1u : 0u;
            e[i].v[0] = a[r];
        } else {
            e[i].f = 1u;
            e[i].v[0] = 0.0;
        }
        tagg = seg_combine(tagg, e[i]);
    }
    const uint32_t epoch = 1;
    SegVal<1> exc = block_exclusive_scan(tagg, ss);
    if (t == 0) {
        agg[b].f = ss.block_total.f ? 1.0 : 0.0;
        agg[b].v[0] = ss.block_total.v[0];
        store_release(&stat[b], epoch);
    }
    const bool tile_head = tile0 >= n || tile0 == 0 || head[tile0] != 0;
    if (!tile_head) {
        if (w == 0) {
            SegVal<1> carry;
            const bool ok = look_back<1>(b, epoch, agg, stat, ctl, carry);
            if (lane == 0) {
                s_carry = carry;
                s_flag = ok ? 0 : 1;
            }
        }
        __syncthreads();
        if (s_flag) return;
        exc = seg_combine(s_carry, exc);
    }
    SegVal<1> run = exc;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        run = seg_combine(run, e[i]);
        if (row0 + i < n) out[row0 + i] = run.v[0];
    }
}

// ------------------------------------------------------------------ host launchers

namespace {

constexpr int kCcdBlock = kThreads;

template <int IPT>
int occupancy_ccd(int p, int *blocks)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, ccd_kernel<kCcdBlock, IPT>, kCcdBlock,
                                                        sizeof(double) * 3 * (size_t)p);
}

int occupancy_for(int ipt, int p, int *blocks)
{
    switch (ipt) {
    case 1: return occupancy_ccd<1>(p, blocks);
    case 2: return occupancy_ccd<2>(p, blocks);
    case 4: return occupancy_ccd<4>(p, blocks);
    case 8: return occupancy_ccd<8>(p, blocks);
    case 16: return occupancy_ccd<16>(p, blocks);
    default: return (int)hipErrorInvalidValue;
    }
}

int device_cus(int *cus)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    return (int)hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
}

}  // namespace

int choose_shape(int64_t n, int p, LaunchShape &shape, std::string &err)
{
    int cus = 0;
    int e = device_cus(&cus);
    if (e != (int)hipSuccess || cus <= 0) {
        err = "cannot query the device's compute-unit count";
        return -3;
    }
    const int ipts[] = {1, 2, 4, 8, 16};
    for (int ipt : ipts) {
        const int64_t rows_per_wg = (int64_t)kCcdBlock * ipt;
        const int64_t grid = (n + rows_per_wg - 1) / rows_per_wg;
        if (grid > cus) continue;
        int blocks = 0;
        e = occupancy_for(ipt, p, &blocks);
        if (e != (int)hipSuccess) {
            err = "occupancy query failed";
            return -3;
        }
        if (blocks < 1) {
            err = "the persistent kernel does not fit on one compute unit for this p";
            return -5;
        }
        shape.ipt = ipt;
        shape.grid = (int)grid;
        shape.ld = grid * rows_per_wg;
        return 0;
    }
    err = "n exceeds the register-resident limit of the persistent kernel (CUs x 512 x 16 rows)";
    return -5;
}

int launch_ccd(const LaunchShape &shape, const CcdLaunch &L, hipStream_t stream, hipEvent_t ev0,
               hipEvent_t ev1)
{
    hipError_t e = hipMemsetAsync(L.ctl, 0, sync_scratch_bytes(shape.grid), stream);
    if (e != hipSuccess) return (int)e;
    if (ev0 && (e = hipEventRecord(ev0, stream)) != hipSuccess) return (int)e;
    CcdLaunch arg = L;
    void *args[] = {&arg};
    const size_t smem = sizeof(double) * 3 * (size_t)L.p;
    const void *fn = nullptr;
    switch (shape.ipt) {
    case 1: fn = reinterpret_cast<const void *>(&ccd_kernel<kCcdBlock, 1>); break;
    case 2: fn = reinterpret_cast<const void *>(&ccd_kernel<kCcdBlock, 2>); break;
    case 4: fn = reinterpret_cast<const void *>(&ccd_kernel<kCcdBlock, 4>); break;
    case 8: fn = reinterpret_cast<const void *>(&ccd_kernel<kCcdBlock, 8>); break;
    case 16: fn = reinterpret_cast<const void *>(&ccd_kernel<kCcdBlock, 16>); break;
    default: return (int)hipErrorInvalidValue;
    }
    e = hipLaunchCooperativeKernel(fn, dim3(shape.grid), dim3(kCcdBlock), args, (unsigned)smem, stream);
    if (e != hipSuccess) return (int)e;
    if (ev1 && (e = hipEventRecord(ev1, stream)) != hipSuccess) return (int)e;
    return (int)hipSuccess;
}

int segscan_f64(const double *a, const uint8_t *head, double *b, int64_t n, hipStream_t stream)
{
    if (n < 0 || (n > 0 && (!a || !head || !b))) return -1;
    if (n == 0) return 0;
    int cus = 0;
    if (device_cus(&cus) != (int)hipSuccess || cus <= 0) return -3;
    const int ipts[] = {1, 2, 4, 8, 16};
    int ipt = 0;
    int64_t grid = 0;
    for (int c : ipts) {
        grid = (n + (int64_t)kScanBlock * c - 1) / ((int64_t)kScanBlock * c);
        if (grid <= cus) {
            ipt = c;
            break;
        }
    }
    if (!ipt) return -5;
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t bytes = up(sizeof(SyncCtl)) + up(sizeof(TileAgg<1>) * grid) + up(sizeof(uint32_t) * grid);
    void *scratch = nullptr;
    if (hipMalloc(&scratch, bytes) != hipSuccess) return -2;
    char *cb = static_cast<char *>(scratch);
    SyncCtl *ctl = reinterpret_cast<SyncCtl *>(cb);
    TileAgg<1> *agg = reinterpret_cast<TileAgg<1> *>(cb + up(sizeof(SyncCtl)));
    uint32_t *stat = reinterpret_cast<uint32_t *>(cb + up(sizeof(SyncCtl)) + up(sizeof(TileAgg<1>) * grid));
    int rc = 0;
    hipError_t e = hipMemsetAsync(scratch, 0, bytes, stream);
    if (e == hipSuccess) {
        void *args[] = {(void *)&a, (void *)&head, (void *)&b, (void *)&n, (void *)&agg, (void *)&stat,
                        (void *)&ctl};
        const void *fn = nullptr;
        switch (ipt) {
        case 1: fn = reinterpret_cast<const void *>(&segscan_kernel<1>); break;
        case 2: fn = reinterpret_cast<const void *>(&segscan_kernel<2>); break;
        case 4: fn = reinterpret_cast<const void *>(&segscan_kernel<4>); break;
        case 8: fn = reinterpret_cast<const void *>(&segscan_kernel<8>); break;
        default: fn = reinterpret_cast<const void *>(&segscan_kernel<16>); break;
        }
        e = hipLaunchCooperativeKernel(fn, dim3((unsigned)grid), dim3(kScanBlock), args, 0, stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    uint32_t aborted = 0;
    if (e == hipSuccess) e = hipMemcpy(&aborted, &ctl->abort, sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess || aborted) rc = -3;
    (void)hipFree(scratch);
    return rc;
}

}  // namespace coxmi
