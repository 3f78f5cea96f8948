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
// reductions are sums over group ends of d * (...).
//
// How it maps onto the MI355X (our design, not the paper's):
//   * One persistent cooperative launch runs the whole fit.  Workgroup b of
//     BLOCK threads owns rows [b*BLOCK*IPT, (b+1)*BLOCK*IPT); each thread keeps
//     its IPT rows of X beta and of the row word in registers for the whole
//     fit, so a coordinate reads only x_j from HBM (8 B/row).  x_{j+1} is
//     loaded while coordinate j synchronises.
//   * Rows inside a workgroup: thread fold -> DPP wave scan -> LDS fold of the
//     wave totals.  A workgroup whose first row is not a stratum head takes
//     its carry from its predecessors' published tile aggregates (look-back,
//     one wave, 64 tiles per round).  When strata fit in a tile the host pads
//     the row layout so no stratum crosses a tile boundary, and the look-back
//     never runs.
//   * Per-coordinate sums are reduced per workgroup (DPP + LDS) and published
//     as epoch-tagged packets (two per workgroup, double-buffered by epoch
//     parity).  In every workgroup one wave gathers all of them -- four
//     workgroups' records per lane, all in flight at once -- reduces them in a
//     fixed order and takes the same scalar CCD step, which one barrier hands
//     to the other waves: one memory round trip after the last workgroup
//     publishes, everyone can move on.  Results are bit-reproducible.
//   * exp() uses one global shift c (the largest X beta of the previous
//     coordinate); ratios are shift-invariant and the objective adds c back.
//     A risk-set sum outside [1e-300, 1e300] stops the fit with a flag.
#include <math.h>

#include <mutex>
#include <type_traits>

#include "internal.h"
#include "segscan.hpp"

namespace coxmi {

// Per-workgroup partial record (5 doubles + an error flag).
enum { kPC1 = 0, kPC2 = 1, kPM2 = 2, kPObj = 3, kPEtaMax = 4, kPN = 5 };

struct Partial {
    double v[kPN];
    uint32_t err;
};

// Stop flags decided after a coordinate.
enum : uint32_t { kFlagNumeric = 1u, kFlagConverged = 2u, kFlagSweepLimit = 4u };

// A published record is 4 packet slots:
//   [0] (sum d S1/S0,              epoch, float(max eta))
//   [1] (sum d (S2/S0 - (S1/S0)^2), epoch, float(sum d S2/S0), NaN if a risk-set sum left range)
//   [2] (objective part,            epoch, 0)   -- only when the objective is wanted
//   [3] (sum d S2/S0,               epoch, 0)   -- only when evaluating (exact value for the caller)
// In a fit the side words only steer the shift and the degeneracy
// threshold, for which single precision is ample.
constexpr int kRecPackets = 4;

namespace {

size_t up256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

// Tile aggregates of the look-back: up to 6 packets per workgroup (Efron's scan element).
constexpr int kAggPackets = 6;

size_t sync_scratch_bytes(int grid)
{
    return up256(sizeof(SyncCtl)) + up256(sizeof(Packet) * kAggPackets * (size_t)grid) +
           up256(sizeof(Packet) * kRecPackets * 2 * (size_t)grid);
}

void carve_sync_scratch(void *base, int grid, CcdLaunch &L)
{
    char *c = static_cast<char *>(base);
    L.ctl = c;
    c += up256(sizeof(SyncCtl));
    L.agg = c;
    c += up256(sizeof(Packet) * kAggPackets * (size_t)grid);
    L.part = c;
    L.res = nullptr;
}

// ------------------------------------------------------------------ small helpers

// exp(x) by the table-driven method of Tang (ACM TOMS 15(2), 1989):
// x = (64 m + j) ln2/64 + r with |r| <= ln2/128, exp(x) = 2^m 2^(j/64) e^r, and
// e^r from its degree-5 Taylor polynomial (truncation below 2^-54 there).
// ln2/64 is split in two (the high part has 30 trailing zero bits, so n times
// it is exact) to form r without cancellation.  tab[j] = 2^(j/64), rounded
// to nearest, built on the host.  Accuracy about 1 ulp, like the libm exp.
__device__ __forceinline__ double exp_table(double x, const double *tab)
{
    x = fmin(fmax(x, -746.0), 710.0);                 // keeps n an int; results saturate to 0 / inf
    const double n = rint(x * 0x1.71547652b82fep+6);   // 64 / ln 2
    double r = fma(-n, 0x1.62e42c0000000p-7, x);       // ln2/64, high part
    r = fma(-n, 0x1.f7d1cf79abc9ep-30, r);             // ln2/64, low part
    const double p = r * fma(r, fma(r, fma(r, fma(r, 1.0 / 120.0, 1.0 / 24.0), 1.0 / 6.0), 0.5), 1.0);
    const int k = (int)n;
    const double t = tab[k & 63];
    return ldexp(fma(t, p, t), k >> 6);
}

// 1/a from the hardware estimate refined by two Newton steps (each squares
// the relative error), ending within about 1 ulp.
__device__ __forceinline__ double recip(double a)
{
    double r = __builtin_amdgcn_rcp(a);
    double e = fma(-a, r, 1.0);
    r = fma(r, e, r);
    e = fma(-a, r, 1.0);
    return fma(r, e, r);
}

template <int IPT>
__device__ __forceinline__ void load_rows(double (&v)[IPT], const double *p)
{
    if constexpr (IPT % 2 == 0) {
        const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
        for (int i = 0; i < IPT / 2; ++i) {
            const double2 t = q[i];
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
            const uint4 t = q[i];
            v[4 * i] = t.x; v[4 * i + 1] = t.y; v[4 * i + 2] = t.z; v[4 * i + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < IPT; ++i) v[i] = p[i];
    }
}

// One column's values at a thread's IPT rows (XK, the kind of X).  Dense (0): IPT doubles
// from the column-major X.  Indicator (1): one bit per row, a thread's IPT bits in one unit
// (uint8 for IPT <= 8, uint16 for 16) at xbits[j * ldb + thread]; the value is 0.0 or 1.0,
// so every product formed with it equals the dense one exactly.  Sparse values (2): the
// same bits mark the nonzero rows, whose values lie in row order in xvals from xvoff[j];
// a wave's first one is at woff[j * nwaves + wave], a lane's after the nonzeros of the
// lanes below it (a prefix sum of bit counts across the wave) -- the values themselves,
// so every product again equals the dense one.
template <int IPT, int XK>
struct XCol;

template <int IPT>
struct XCol<IPT, 0> {
    double v[IPT];
    __device__ __forceinline__ void load(const CcdLaunch &L, int64_t ld, int64_t j, int64_t row0, int64_t)
    {
        load_rows<IPT>(v, L.x + j * ld + row0);
    }
    __device__ __forceinline__ double operator[](int i) const { return v[i]; }
};

template <int IPT>
struct XCol<IPT, 1> {
    using Unit = typename std::conditional<(IPT > 8), uint16_t, uint8_t>::type;
    uint32_t bits;
    __device__ __forceinline__ void load(const CcdLaunch &L, int64_t, int64_t j, int64_t, int64_t tg)
    {
        bits = static_cast<const Unit *>(L.xbits)[j * L.ldb + tg];
    }
    __device__ __forceinline__ double operator[](int i) const { return ((bits >> i) & 1u) ? 1.0 : 0.0; }
};

template <int IPT>
struct XCol<IPT, 2> {
    using Unit = typename std::conditional<(IPT > 8), uint16_t, uint8_t>::type;
    double v[IPT];
    // called by every lane of the wave (the prefix sum below is across the whole wave)
    __device__ __forceinline__ void load(const CcdLaunch &L, int64_t, int64_t j, int64_t, int64_t tg)
    {
        const uint32_t bits = static_cast<const Unit *>(L.xbits)[j * L.ldb + tg];
        const int lane = (int)(threadIdx.x & (kWave - 1));
        const int cnt = __popc(bits);
        int incl = cnt;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int up = __shfl_up(incl, d, kWave);
            if (lane >= d) incl += up;
        }
        const double *src = L.xvals + L.xvoff[j] + L.woff[j * L.nwaves + tg / kWave] + (incl - cnt);
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const uint32_t below = bits & ((1u << i) - 1u);
            v[i] = ((bits >> i) & 1u) ? src[__popc(below)] : 0.0;
        }
    }
    __device__ __forceinline__ double operator[](int i) const { return v[i]; }
};

__device__ __forceinline__ Partial partial_identity()
{
    Partial r;
    r.v[kPC1] = 0.0; r.v[kPC2] = 0.0; r.v[kPM2] = 0.0; r.v[kPObj] = 0.0;
    r.v[kPEtaMax] = -INFINITY;
    r.err = 0u;
    return r;
}

__device__ __forceinline__ void partial_combine(Partial &a, const Partial &b)
{
    a.v[kPC1] += b.v[kPC1];
    a.v[kPC2] += b.v[kPC2];
    a.v[kPM2] += b.v[kPM2];
    a.v[kPObj] += b.v[kPObj];
    a.v[kPEtaMax] = fmax(a.v[kPEtaMax], b.v[kPEtaMax]);
    a.err |= b.err;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ Partial dpp_partial(const Partial &x)
{
    Partial r;
    r.v[kPC1] = dpp_f64<CTRL, ROWS>(x.v[kPC1]);
    r.v[kPC2] = dpp_f64<CTRL, ROWS>(x.v[kPC2]);
    r.v[kPM2] = dpp_f64<CTRL, ROWS>(x.v[kPM2]);
    r.v[kPObj] = dpp_f64<CTRL, ROWS>(x.v[kPObj]);
    // lanes without a source must see the identity of max
    r.v[kPEtaMax] = __builtin_amdgcn_update_dpp(-(double)INFINITY, x.v[kPEtaMax], CTRL, ROWS, 0xF, false);
    r.err = dpp_u32<CTRL, ROWS>(x.err);
    return r;
}

// Wave reduction in a fixed lane order; the total ends in lane 63.
__device__ __forceinline__ Partial wave_reduce_partial(Partial x)
{
    Partial o;
    o = dpp_partial<0x111, 0xF>(x); partial_combine(x, o);
    o = dpp_partial<0x112, 0xF>(x); partial_combine(x, o);
    o = dpp_partial<0x114, 0xF>(x); partial_combine(x, o);
    o = dpp_partial<0x118, 0xF>(x); partial_combine(x, o);
    o = dpp_partial<0x142, 0xA>(x); partial_combine(x, o);
    o = dpp_partial<0x143, 0xC>(x); partial_combine(x, o);
    return x;
}

// Workgroup reduction; every thread receives the same total.  One barrier.
template <int NW>
__device__ __forceinline__ Partial block_reduce_partial(const Partial &x, Partial *red)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const Partial wr = wave_reduce_partial(x);
    if (lane == kWave - 1) red[w] = wr;
    __syncthreads();
    Partial tot = red[0];
#pragma unroll
    for (int k = 1; k < NW; ++k) partial_combine(tot, red[k]);
    return tot;
}

// Publish this workgroup's record for `epoch` (thread 0); `extra` adds
// slots [2] and [3].
__device__ __forceinline__ void publish_partial(const PacketArray &part, int G, int b, const Partial &x,
                                                uint32_t epoch, bool extra)
{
    const uint32_t slot = (uint32_t)(kRecPackets * ((epoch & 1u) * (uint32_t)G + (uint32_t)b));
    const float emax = (float)x.v[kPEtaMax];
    const float m2 = x.err ? __builtin_nanf("") : (float)fmin(x.v[kPM2], 3.0e38);
    packet_put(part, slot, x.v[kPC1], epoch, __float_as_uint(emax));
    packet_put(part, slot + 1, x.v[kPC2], epoch, __float_as_uint(m2));
    if (extra) {
        packet_put(part, slot + 2, x.v[kPObj], epoch, 0u);
        packet_put(part, slot + 3, x.v[kPM2], epoch, 0u);
    }
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

// One wave gathers the records of all G <= 256 workgroups for `epoch`: lane L
// waits for the records of workgroups L, L + 64, L + 128, L + 192 (every packet of
// every pending record in flight at once, re-polled together until all carry the
// epoch), folds them in that order, and the wave reduces the lane totals in a
// fixed DPP order -- so every workgroup obtains the same bits regardless of
// arrival times.  Every lane of the wave receives the total.  Returns false
// (uniformly) once a wait has timed out or another workgroup aborted.  Packets
// first .. first + NP - 1 of each record are polled.
constexpr int kGatherPer = kMaxGroups / kWave;

template <int NP>
__device__ __forceinline__ bool poll_records(const PacketArray &part, int G, uint32_t epoch, SyncCtl *ctl,
                                             u32x4 (&r)[kGatherPer][NP], int first = 0)
{
    const int lane = threadIdx.x & (kWave - 1);
    bool done[kGatherPer];
    uint32_t slot[kGatherPer];
#pragma unroll
    for (int k = 0; k < kGatherPer; ++k) {
        const int q = lane + kWave * k;
        done[k] = q >= G;
        slot[k] = (uint32_t)(kRecPackets * ((epoch & 1u) * (uint32_t)G + (uint32_t)q) + first);
    }
    WaitBudget wb;
    bool ok = true;
    for (;;) {
#pragma unroll
        for (int k = 0; k < kGatherPer; ++k)
            if (!done[k])
#pragma unroll
                for (int pk = 0; pk < NP; ++pk) r[k][pk] = packet_get(part, slot[k] + pk);
        bool all = true;
#pragma unroll
        for (int k = 0; k < kGatherPer; ++k) {
            if (!done[k]) {
                bool fresh = true;
#pragma unroll
                for (int pk = 0; pk < NP; ++pk) fresh = fresh && r[k][pk].z == epoch;
                done[k] = fresh;
                all = all && fresh;
            }
        }
        if (all) break;
        if (!wb.keep_waiting(ctl)) {
            ok = false;
            break;
        }
    }
    return __builtin_amdgcn_ballot_w64(!ok) == 0;
}

__device__ __forceinline__ Partial broadcast_lane63(const Partial &x)
{
    Partial r;
#pragma unroll
    for (int k = 0; k < kPN; ++k) r.v[k] = lane63_f64(x.v[k]);
    r.err = (uint32_t)__builtin_amdgcn_readlane((int)x.err, 63);
    return r;
}

__device__ __forceinline__ bool gather_wave(const PacketArray &part, int G, uint32_t epoch, bool extra,
                                            SyncCtl *ctl, Partial &total)
{
    const int lane = threadIdx.x & (kWave - 1);
    Partial x = partial_identity();
    {
        u32x4 r[kGatherPer][2];
        if (!poll_records<2>(part, G, epoch, ctl, r)) return false;
#pragma unroll
        for (int k = 0; k < kGatherPer; ++k) {
            if (lane + kWave * k < G) {
                Partial y;
                y.v[kPC1] = packet_value(r[k][0]);
                y.v[kPEtaMax] = (double)__uint_as_float(r[k][0].w);
                y.v[kPC2] = packet_value(r[k][1]);
                const float m2 = __uint_as_float(r[k][1].w);
                y.err = (m2 == m2) ? 0u : 1u;
                y.v[kPM2] = (double)m2;
                y.v[kPObj] = 0.0;
                partial_combine(x, y);
            }
        }
    }
    if (extra) {
        // the objective and the exact second moment (written with the two above): a second,
        // short poll on the first coordinate of a sweep and in evaluations only
        u32x4 r[kGatherPer][2];
        if (!poll_records<2>(part, G, epoch, ctl, r, 2)) return false;
        double obj = 0.0, m2 = 0.0;
#pragma unroll
        for (int k = 0; k < kGatherPer; ++k) {
            if (lane + kWave * k < G) {
                obj += packet_value(r[k][0]);
                m2 += packet_value(r[k][1]);
            }
        }
        x.v[kPObj] = obj;
        x.v[kPM2] = m2;
    }
    total = broadcast_lane63(wave_reduce_partial(x));
    return true;
}

// Tie-group terms of one row, added to v (Sec. 2.4 derivatives).  S = (S0, S1, S2): the
// inclusive risk-set sums at the row; d: the events of the tie group ending at the row (0 when
// the row ends no group with events, and then nothing is added).
//   Breslow (the risk sets of Eq. strat_l taken literally): every tied event sees S,
//     so the group adds d S1/S0, d (S2/S0 - (S1/S0)^2), d S2/S0, d (log S0 + c).  Evaluated
//     on every row without branches (d = 0 adds zeros; S0 is replaced by 1 there so that
//     no infinity enters).
//   Efron (1977): E = (E0, E1, E2), the same sums over the group's own events; the l-th
//     of its d events sees S - (l/d) E, l = 0..d-1 (d = 1 is Breslow's term exactly).
template <bool EFRON, bool WANT_OBJ>
__device__ __forceinline__ void group_terms(Partial &v, uint32_t d, const double (&S)[3], const double (&E)[3],
                                            double c)
{
    const double s0 = S[0];
    if constexpr (!EFRON) {
        const bool end = d != 0u;
        if (end && (!(s0 >= 1e-300) || !(s0 <= 1e300))) v.err = 1u;
        const double sg = end ? s0 : 1.0;
        const double inv = recip(sg);
        const double r1 = S[1] * inv, r2 = S[2] * inv;
        const double dd = (double)d;
        v.v[kPC1] = fma(dd, r1, v.v[kPC1]);
        v.v[kPC2] = fma(dd, fma(-r1, r1, r2), v.v[kPC2]);
        v.v[kPM2] = fma(dd, r2, v.v[kPM2]);
        if constexpr (WANT_OBJ) v.v[kPObj] = fma(dd, log(sg) + c, v.v[kPObj]);
    } else {
        if (d == 0u) return;
        if (!(s0 >= 1e-300) || !(s0 <= 1e300)) v.err = 1u;
        const double dd = (double)d;
        for (uint32_t l = 0; l < d; ++l) {
            const double a = (double)l / dd;
            const double A = s0 - a * E[0];
            const double inv = recip(A);
            const double r1 = (S[1] - a * E[1]) * inv, r2 = (S[2] - a * E[2]) * inv;
            v.v[kPC1] += r1;
            v.v[kPC2] += r2 - r1 * r1;
            v.v[kPM2] += r2;
            if constexpr (WANT_OBJ) v.v[kPObj] += log(A) + c;
        }
    }
}

// Scan element of one row.  Components 0..2: (D, N1, N2) restarting at stratum heads
// (flag bit 0).  Efron adds components 3..5: the same values on event rows only, restarting
// after every row that ends a tie group with events (flag bit 1; such a row contributes 0
// itself, so the running value before it plus its own values are its group's event sums).
// An event-free stretch adds nothing, so these sums need no restart at stratum heads.
template <bool EFRON>
using RowVal = SegVal<EFRON ? 6 : 3, 3>;

template <bool EFRON>
__device__ __forceinline__ RowVal<EFRON> row_value(uint32_t m, double w, double x)
{
    RowVal<EFRON> r;
    r.f = m >> 31;
    r.v[0] = w;
    r.v[1] = x * w;
    r.v[2] = x * r.v[1];
    if constexpr (EFRON) {
        const bool end = (m & kCountMask) != 0u, ev = (m & kEventBit) != 0u;
        r.f |= end ? 2u : 0u;
        const bool keep = ev && !end;
        r.v[3] = keep ? r.v[0] : 0.0;
        r.v[4] = keep ? r.v[1] : 0.0;
        r.v[5] = keep ? r.v[2] : 0.0;
    }
    return r;
}

// Pass 2 over a thread's rows: the inclusive prefixes from the thread's exclusive prefix
// `run`, the group-end terms, the largest X beta over real rows, and (WANT_OBJ, the first
// coordinate of a sweep) the objective's parts.
template <int IPT, int XK, bool EFRON, bool WANT_OBJ>
__device__ __forceinline__ Partial pass2(RowVal<EFRON> run, const uint32_t (&meta)[IPT], const double (&wv)[IPT],
                                         const XCol<IPT, XK> &xc, const double (&eta)[IPT], double c)
{
    Partial v = partial_identity();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const RowVal<EFRON> r = row_value<EFRON>(meta[i], wv[i], xc[i]);
        double E[3] = {0.0, 0.0, 0.0};
        if constexpr (EFRON) {
            // this row's group's event sums: the running value before it plus its own share
            const bool ev = (meta[i] & kEventBit) != 0u;
#pragma unroll
            for (int k = 0; k < 3; ++k) E[k] = run.v[3 + k] + (ev ? r.v[k] : 0.0);
        }
        run = seg_combine(run, r);
        v.v[kPEtaMax] = (meta[i] & kPadBit) ? v.v[kPEtaMax] : fmax(v.v[kPEtaMax], eta[i]);
        const double S[3] = {run.v[0], run.v[1], run.v[2]};
        group_terms<EFRON, WANT_OBJ>(v, meta[i] & kCountMask, S, E, c);
        if constexpr (WANT_OBJ) v.v[kPObj] -= (meta[i] & kEventBit) ? eta[i] : 0.0;
    }
    return v;
}

// ------------------------------------------------------------------ the persistent kernel

// WAVE: the layout puts every stratum inside one wave's rows, so a wave's first row is a
// stratum head and its scan needs nothing from the other waves: no workgroup scan, no barrier.
template <int BLOCK, int IPT, int XK, bool EFRON, bool WAVE>
__global__ __launch_bounds__(BLOCK) void ccd_kernel(CcdLaunch L)
{
    constexpr int NW = BLOCK / kWave;
    constexpr int KV = EFRON ? 6 : 3;
    using RV = RowVal<EFRON>;
    static_assert(BLOCK % kWave == 0 && NW <= 16, "block shape");
    extern __shared__ double smem_dyn[];     // beta (the same in every workgroup)
    __shared__ RV s_wtot[NW];
    __shared__ Partial s_red[NW];        // this workgroup's own reduction
    __shared__ RV s_win[kMaxGroups / kWave];
    __shared__ int s_abort;
    __shared__ double s_exptab[64];
    __shared__ double s_step, s_shift;   // wave 0's step and shift for the next coordinate
    __shared__ uint32_t s_flags;

    const int p = L.p;
    const int G = gridDim.x, b = blockIdx.x, t = threadIdx.x;
    const int lane = t & (kWave - 1), w = t / kWave;
    const bool writer = (b == 0 && t == 0);   // writes the outputs
    SyncCtl *ctl = static_cast<SyncCtl *>(L.ctl);
    const PacketArray agg = packet_array(L.agg, sizeof(Packet) * KV * (size_t)G);
    const PacketArray part = packet_array(L.part, sizeof(Packet) * kRecPackets * 2 * (size_t)G);
    const int64_t ld = (int64_t)G * BLOCK * IPT;
    const int64_t tile0 = (int64_t)b * BLOCK * IPT;
    const int64_t row0 = tile0 + (int64_t)t * IPT;
    const int64_t tg = (int64_t)b * BLOCK + t;      // the thread's unit in an indicator column
    const bool fit = (L.mode == kModeFit);

    double *sbeta = smem_dyn;
    double *trust = L.trust + (int64_t)b * p;      // this workgroup's copy of the trust half-widths
    for (int j = t; j < p; j += BLOCK) {
        sbeta[j] = L.beta[j];
        trust[j] = 1.0;
    }
    if (t == 0) s_abort = 0;
    if (t < 64) s_exptab[t] = L.exp_tab[t];
    uint32_t meta[IPT];
    double eta[IPT];
    load_words<IPT>(meta, L.meta + row0);
#pragma unroll
    for (int i = 0; i < IPT; ++i) eta[i] = 0.0;
    const bool tile_head = (L.meta[tile0] & kHeadBit) != 0u;

    // X beta0 (columns with beta0_j = 0 are skipped)
    for (int j = 0; j < p; ++j) {
        const double bj = L.beta[j];
        if (bj != 0.0) {
            XCol<IPT, XK> xv;
            xv.load(L, ld, j, row0, tg);
#pragma unroll
            for (int i = 0; i < IPT; ++i) eta[i] = fma(xv[i], bj, eta[i]);
        }
    }
    __syncthreads();

    // epoch 1: the initial shift, the largest X beta over the real rows
    uint32_t epoch = 1;
    double c;
    {
        Partial v = partial_identity();
#pragma unroll
        for (int i = 0; i < IPT; ++i)
            if (!(meta[i] & kPadBit)) v.v[kPEtaMax] = fmax(v.v[kPEtaMax], eta[i]);
        v = block_reduce_partial<NW>(v, s_red);
        if (t == 0) publish_partial(part, G, b, v, epoch, false);
        if (w == 0) {
            Partial tot;
            if (gather_wave(part, G, epoch, false, ctl, tot)) {
                if (lane == 0) s_shift = tot.v[kPEtaMax];
            } else if (lane == 0) {
                s_abort = 1;
            }
        }
        __syncthreads();
        if (s_abort) return;
        c = s_shift;
    }

    const int jfirst = fit ? 0 : L.j0;
    const int jend = fit ? p : L.j1;
    XCol<IPT, XK> xc;
    xc.load(L, ld, jfirst, row0, tg);

    // Wave 0 keeps the bookkeeping (the same in every lane) and takes the step: its
    // inputs are read at the start of the coordinate, and lane 0 writes beta_j and the
    // half-width after the gather, for the next sweep.
    int sweeps = 0, pinned = 0, pinned_last = 0;
    double maxstep = 0.0, last_maxstep = 0.0, objective = 0.0;
    uint32_t stop = 0;

    for (;;) {
        for (int j = jfirst; j < jend; ++j) {
            ++epoch;
            const int jn = (j + 1 < jend) ? j + 1 : jfirst;
            XCol<IPT, XK> xn;
            xn.load(L, ld, jn, row0, tg);
            const bool want_obj = (j == jfirst);
            // the step's per-column inputs: issued here, they arrive during the passes
            const double bj = sbeta[j];
            const double qj = L.q[j], gj = L.gamma[j];
            double trj = trust[j];

            // pass 1: D, N1, N2 of the thread's rows and their fold
            RV tagg = seg_identity<KV, 3>();
            double wv[IPT];
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                wv[i] = exp_table(eta[i] - c, s_exptab);
                tagg = seg_combine(tagg, row_value<EFRON>(meta[i], wv[i], xc[i]));
            }
            RV exc;
            if constexpr (WAVE) {
                exc = wave_shift_right(wave_inclusive_scan(tagg));
            } else {
                RV btot;
                exc = block_exclusive_scan<KV, NW, 3>(tagg, s_wtot, btot);
                if (t == 0) publish_aggregate(agg, b, btot, epoch);
                if (!tile_head) {
                    RV carry;
                    if (!look_back<KV, 3>(b, epoch, agg, ctl, s_win, &s_abort, carry)) return;
                    exc = seg_combine(carry, exc);
                }
            }

            // pass 2: inclusive prefixes at group ends -> per-coordinate sums
            Partial v = want_obj ? pass2<IPT, XK, EFRON, true>(exc, meta, wv, xc, eta, c)
                                 : pass2<IPT, XK, EFRON, false>(exc, meta, wv, xc, eta, c);
            v = block_reduce_partial<NW>(v, s_red);
            const bool extra = want_obj || !fit;
            if (t == 0) publish_partial(part, G, b, v, epoch, extra);

            // wave 0 gathers every workgroup's record and takes the step; the others wait for it
            if (w == 0) {
                Partial tot;
                if (!gather_wave(part, G, epoch, extra, ctl, tot)) {
                    if (lane == 0) s_abort = 1;
                } else {
                    uint32_t flags = tot.err ? kFlagNumeric : 0u;
                    const double g1 = -qj + tot.v[kPC1], g2 = tot.v[kPC2], m2 = tot.v[kPM2];
                    if (writer) {
                        L.g1[j] = g1;
                        L.g2[j] = g2;
                        L.m2[j] = m2;
                    }
                    if (want_obj) {
                        objective = tot.v[kPObj];
                        if (fit)
                            for (int k = 0; k < p; ++k) objective += L.gamma[k] * fabs(sbeta[k]);
                    }
                    double step = 0.0;
                    if (fit && !(flags & kFlagNumeric)) {
                        int pin = 0;
                        step = ccd_step(bj, g1, g2, m2, gj, &trj, &pin);
                        maxstep = fmax(maxstep, fabs(step));
                        pinned += pin;
                        if (j == jend - 1) {
                            ++sweeps;
                            double bmax = 1.0;
                            for (int k = 0; k < p; ++k) bmax = fmax(bmax, fabs(k == j ? bj + step : sbeta[k]));
                            if (maxstep <= L.tol * bmax) flags |= kFlagConverged;
                            else if (sweeps >= L.max_sweeps) flags |= kFlagSweepLimit;
                            last_maxstep = maxstep;
                            pinned_last = pinned;
                            maxstep = 0.0;
                            pinned = 0;
                        }
                    }
                    if (lane == 0) {
                        if (fit && !(flags & kFlagNumeric)) {
                            trust[j] = trj;
                            sbeta[j] = bj + step;
                        }
                        s_step = step;
                        s_shift = tot.v[kPEtaMax];
                        s_flags = flags;
                    }
                }
            }
            __syncthreads();
            if (s_abort) return;
            const uint32_t flags = s_flags;
            if (flags & kFlagNumeric) {
                stop = kFlagNumeric;
                break;
            }
            const double step = s_step;
            c = s_shift;
            if (step != 0.0) {
#pragma unroll
                for (int i = 0; i < IPT; ++i) eta[i] = fma(xc[i], step, eta[i]);
            }
            xc = xn;
            if (flags & (kFlagConverged | kFlagSweepLimit)) {
                stop = flags;
                break;
            }
        }
        if (stop || !fit) break;
    }

    if (b == 0) {
        // wave 0 holds the bookkeeping; beta is in LDS (written before the last barrier)
        if (fit)
            for (int j = t; j < p; j += BLOCK) L.beta[j] = sbeta[j];
        if (t == 0) {
            L.result[kResSweeps] = sweeps;
            L.result[kResLastStep] = last_maxstep;
            L.result[kResObjective] = objective;
            L.result[kResPinned] = pinned_last;
            L.result[kResConverged] = (stop & kFlagConverged) ? 1.0 : 0.0;
            L.result[kResNumeric] = (stop & kFlagNumeric) ? 1.0 : 0.0;
            L.result[kResCompleted] = 1.0;
        }
    }
}

// ------------------------------------------------------------------ raw segmented scan

constexpr int kScanBlock = 1024;

template <int IPT>
__global__ __launch_bounds__(kScanBlock) void segscan_kernel(const double *a, const uint8_t *head,
                                                             double *out, int64_t n, Packet *aggp,
                                                             SyncCtl *ctl)
{
    const PacketArray agg = packet_array(aggp, sizeof(Packet) * gridDim.x);
    constexpr int NW = kScanBlock / kWave;
    __shared__ SegVal<1> s_wtot[NW];
    __shared__ SegVal<1> s_win[kMaxGroups / kWave];
    __shared__ int s_abort;
    const int b = blockIdx.x, t = threadIdx.x;
    const int lane = t & (kWave - 1), w = t / kWave;
    const int64_t tile0 = (int64_t)b * kScanBlock * IPT;
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
    if (t == 0) s_abort = 0;
    const uint32_t epoch = 1;
    SegVal<1> btot;
    SegVal<1> exc = block_exclusive_scan<1, NW>(tagg, s_wtot, btot);
    if (t == 0) publish_aggregate<1>(agg, b, btot, epoch);
    const bool tile_head = tile0 >= n || tile0 == 0 || head[tile0] != 0;
    if (!tile_head) {
        SegVal<1> carry;
        if (!look_back<1>(b, epoch, agg, ctl, s_win, &s_abort, carry)) return;
        exc = seg_combine(carry, exc);
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

// Dynamic LDS of one persistent workgroup: beta.
size_t ccd_smem_bytes(int, int p)
{
    return sizeof(double) * (size_t)p;
}

template <int IPT, int XK, bool EFRON, bool WAVE>
const void *ccd_fn()
{
    return reinterpret_cast<const void *>(&ccd_kernel<kCcdBlock, IPT, XK, EFRON, WAVE>);
}

template <int XK, bool EFRON, bool WAVE>
const void *ccd_fn_ipt(int ipt)
{
    switch (ipt) {
    case 1: return ccd_fn<1, XK, EFRON, WAVE>();
    case 2: return ccd_fn<2, XK, EFRON, WAVE>();
    case 4: return ccd_fn<4, XK, EFRON, WAVE>();
    case 8: return ccd_fn<8, XK, EFRON, WAVE>();
    case 16: return ccd_fn<16, XK, EFRON, WAVE>();
    default: return nullptr;
    }
}

template <bool WAVE>
const void *ccd_function_w(int ipt, int xk, bool efron)
{
    if (xk == 2) return efron ? ccd_fn_ipt<2, true, WAVE>(ipt) : ccd_fn_ipt<2, false, WAVE>(ipt);
    if (xk == 1) return efron ? ccd_fn_ipt<1, true, WAVE>(ipt) : ccd_fn_ipt<1, false, WAVE>(ipt);
    return efron ? ccd_fn_ipt<0, true, WAVE>(ipt) : ccd_fn_ipt<0, false, WAVE>(ipt);
}

// xk: 0 dense X, 1 indicator X, 2 sparse values (see XCol)
const void *ccd_function(int ipt, int xk, bool efron, bool wave)
{
    return wave ? ccd_function_w<true>(ipt, xk, efron) : ccd_function_w<false>(ipt, xk, efron);
}

// Workgroups of the persistent kernel that fit on one compute unit; every variant
// (indicator or sparse X, Efron, wave-aligned layout) must fit, since a handle may run any of them.
int occupancy_for(int ipt, int p, int *blocks)
{
    *blocks = 1 << 30;
    for (int v = 0; v < 12; ++v) {
        const void *fn = ccd_function(ipt, v % 3, ((v / 3) & 1) != 0, ((v / 3) & 2) != 0);
        if (!fn) return (int)hipErrorInvalidValue;
        int nb = 0;
        const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kCcdBlock, ccd_smem_bytes(ipt, p));
        if (e != hipSuccess) return (int)e;
        *blocks = nb < *blocks ? nb : *blocks;
    }
    return (int)hipSuccess;
}

int device_cus(int *cus)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    return (int)hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
}

}  // namespace

int max_resident_groups(int ipt, int p, int *groups, std::string &err)
{
    *groups = 0;
    int cus = 0;
    if (device_cus(&cus) != (int)hipSuccess || cus <= 0) {
        err = "cannot query the device's compute-unit count";
        return -3;
    }
    int blocks = 0;
    if (occupancy_for(ipt, p, &blocks) != (int)hipSuccess) {
        err = "occupancy query failed";
        return -3;
    }
    *groups = blocks >= 1 ? (cus < kMaxGroups ? cus : kMaxGroups) : 0;   // one workgroup per compute unit
    return 0;
}

int launch_ccd(const LaunchShape &shape, const CcdLaunch &L, hipStream_t stream, hipEvent_t ev0,
               hipEvent_t ev1)
{
    hipError_t e = hipMemsetAsync(L.ctl, 0, sync_scratch_bytes(shape.grid), stream);
    if (e != hipSuccess) return (int)e;
    if (ev0 && (e = hipEventRecord(ev0, stream)) != hipSuccess) return (int)e;
    CcdLaunch arg = L;
    void *args[] = {&arg};
    const size_t smem = ccd_smem_bytes(shape.ipt, L.p);
    const void *fn = ccd_function(shape.ipt, L.xvals ? 2 : (L.xbits ? 1 : 0), L.efron != 0, shape.wave);
    if (!fn) return (int)hipErrorInvalidValue;
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
        if (grid <= cus && grid <= kMaxGroups) {
            ipt = c;
            break;
        }
    }
    if (!ipt) return -5;
    const size_t bytes = up256(sizeof(SyncCtl)) + up256(sizeof(Packet) * (size_t)grid);
    void *scratch = nullptr;
    if (hipMalloc(&scratch, bytes) != hipSuccess) return -2;
    char *cb = static_cast<char *>(scratch);
    SyncCtl *ctl = reinterpret_cast<SyncCtl *>(cb);
    Packet *agg = reinterpret_cast<Packet *>(cb + up256(sizeof(SyncCtl)));
    int rc = 0;
    hipError_t e = hipMemsetAsync(scratch, 0, bytes, stream);
    if (e == hipSuccess) {
        void *args[] = {(void *)&a, (void *)&head, (void *)&b, (void *)&n, (void *)&agg, (void *)&ctl};
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

// ------------------------------------------------------------------ the scan without allocation

// Synchronisation words of segscan_f64_noalloc: the control block and one aggregate
// packet per workgroup (at most kMaxGroups), in library-owned device memory that
// exists once per GPU for the life of the process.  Host code never uses this name
// as an address: its per-device address comes from hipGetSymbolAddress.
constexpr size_t kNoAllocScratchBytes = 256 + sizeof(Packet) * kMaxGroups;
static_assert(sizeof(SyncCtl) <= 256, "control block");
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per device.
int scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return -3;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return -3;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

// Zero `words` 32-bit words (a fill kernel rather than a memset node, so the call can
// sit in captured work).
__global__ __launch_bounds__(256) void zero_words_kernel(uint32_t *p, int words)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < words) p[i] = 0u;
}

}  // namespace

int segscan_f64_noalloc(const double *a, const uint8_t *head, double *b, int64_t n, hipStream_t stream)
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
        if (grid <= cus && grid <= kMaxGroups) {
            ipt = c;
            break;
        }
    }
    if (!ipt) return -5;
    void *base = nullptr;
    if (scratch_address(&base) != 0) return -3;
    const size_t bytes = up256(sizeof(SyncCtl)) + up256(sizeof(Packet) * (size_t)grid);
    if (bytes > kNoAllocScratchBytes) return -5;
    char *cb = static_cast<char *>(base);
    SyncCtl *ctl = reinterpret_cast<SyncCtl *>(cb);
    Packet *agg = reinterpret_cast<Packet *>(cb + up256(sizeof(SyncCtl)));
    // the previous call's packets carry the same epoch: clear them before this scan reads any
    const int words = (int)(bytes / sizeof(uint32_t));
    hipLaunchKernelGGL(zero_words_kernel, dim3((words + 255) / 256), dim3(256), 0, stream,
                       reinterpret_cast<uint32_t *>(base), words);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        void *args[] = {(void *)&a, (void *)&head, (void *)&b, (void *)&n, (void *)&agg, (void *)&ctl};
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
    uint32_t aborted = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&aborted, &ctl->abort, sizeof(uint32_t), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    return (e != hipSuccess || aborted) ? -3 : 0;
}

}  // namespace coxmi
