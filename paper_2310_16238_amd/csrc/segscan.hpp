// segscan.hpp -- device building blocks for the segmented scan of Sec. 2.6 on gfx950.
//
// A scan element is a flag-value pair (f, v) with v a small tuple of doubles.
// The operator is the flag-value operator of Sec. 2.6 with + as the base:
//     (f_a, a) (+)s (f_b, b) = (f_a | f_b, f_b ? b : a + b)
// It is associative but not commutative: the left operand is the earlier row.
// (0, 0) -- all bits zero -- is its identity on both sides.
//
// Layout of work on the chip (ours, not the paper's): a workgroup of NW
// wave64s owns a contiguous tile of rows, each thread IPT consecutive rows.
// The tile's scan is
//   thread-sequential fold over its IPT rows
//   -> wave64 inclusive scan with DPP lane moves (row_shr 1/2/4/8 inside each
//      16-lane row, then row_bcast 15 and 31 across rows: 6 steps, no LDS)
//   -> the NW wave totals through LDS, folded by every wave (one barrier).
//
// Between workgroups, values travel as 16-byte packets (a double, the epoch
// it belongs to, and a 32-bit side word) written and read with single
// 16-byte buffer accesses that go through to the device coherence point
// (the sc1 cache policy).  A 16-byte aligned dwordx4 access is performed as
// one transaction, so a reader sees a packet either whole-old or whole-new
// and the epoch inside it says which: no flag, fence or cache write-back is
// needed, and a wait costs one round trip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace coxmi {

constexpr int kWave = 64;

// Components 0..KS-1 restart at elements whose flag has bit 0 set, components KS..K-1
// at elements whose flag has bit 1 set: two segmented scans with different segment
// boundaries carried in one element.  With KS = K it is one scan, restarting at any
// nonzero flag.  Each is the flag-value operator above, so the pair is associative too.
template <int K, int KS = K>
struct SegVal {
    uint32_t f;
    double v[K];
};

template <int K, int KS = K>
__device__ __forceinline__ SegVal<K, KS> seg_identity()
{
    SegVal<K, KS> r;
    r.f = 0u;
#pragma unroll
    for (int k = 0; k < K; ++k) r.v[k] = 0.0;
    return r;
}

// a is the earlier (left) element, b the later one.
template <int K, int KS>
__device__ __forceinline__ SegVal<K, KS> seg_combine(const SegVal<K, KS> &a, const SegVal<K, KS> &b)
{
    SegVal<K, KS> r;
    r.f = a.f | b.f;
    if constexpr (KS == K) {
        // one scan: any flag bit restarts.  a * keep + b with keep = 0 or 1 is b or a + b
        // exactly (one rounding, as the sum), for finite a: one FMA per component
        const double keep = b.f ? 0.0 : 1.0;
#pragma unroll
        for (int k = 0; k < K; ++k) r.v[k] = fma(a.v[k], keep, b.v[k]);
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) r.v[k] = (b.f & (k < KS ? 1u : 2u)) ? b.v[k] : a.v[k] + b.v[k];
    }
    return r;
}

// ------------------------------------------------------------------ DPP lane moves
// dpp_ctrl codes (GFX9 encoding): row_shr:n = 0x110 + n, wave_shr:1 = 0x138,
// row_bcast:15 = 0x142, row_bcast:31 = 0x143.  Lanes without a source (or in
// rows masked off) receive 0, which is the identity of every operator here.

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double x)
{
    return __builtin_amdgcn_update_dpp(0.0, x, CTRL, ROWS, 0xF, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xF, false);
}

template <int CTRL, int ROWS, int K, int KS>
__device__ __forceinline__ SegVal<K, KS> dpp_seg(const SegVal<K, KS> &x)
{
    SegVal<K, KS> r;
    r.f = dpp_u32<CTRL, ROWS>(x.f);
#pragma unroll
    for (int k = 0; k < K; ++k) r.v[k] = dpp_f64<CTRL, ROWS>(x.v[k]);
    return r;
}

// Inclusive segmented scan across the 64 lanes (lane order = row order).
// All 64 lanes must be active.
template <int K, int KS>
__device__ __forceinline__ SegVal<K, KS> wave_inclusive_scan(SegVal<K, KS> x)
{
    x = seg_combine(dpp_seg<0x111, 0xF>(x), x);
    x = seg_combine(dpp_seg<0x112, 0xF>(x), x);
    x = seg_combine(dpp_seg<0x114, 0xF>(x), x);
    x = seg_combine(dpp_seg<0x118, 0xF>(x), x);
    x = seg_combine(dpp_seg<0x142, 0xA>(x), x);
    x = seg_combine(dpp_seg<0x143, 0xC>(x), x);
    return x;
}

// Lane i receives lane i-1's value; lane 0 receives the identity.
template <int K, int KS>
__device__ __forceinline__ SegVal<K, KS> wave_shift_right(const SegVal<K, KS> &x)
{
    return dpp_seg<0x138, 0xF, K, KS>(x);
}

__device__ __forceinline__ double lane63_f64(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int K, int KS>
__device__ __forceinline__ SegVal<K, KS> lane63_seg(const SegVal<K, KS> &x)
{
    SegVal<K, KS> r;
    r.f = (uint32_t)__builtin_amdgcn_readlane((int)x.f, 63);
#pragma unroll
    for (int k = 0; k < K; ++k) r.v[k] = lane63_f64(x.v[k]);
    return r;
}

// Exclusive scan of one element per thread over the workgroup (NW waves).
// Returns the thread's exclusive prefix; `total` receives the workgroup's
// total in every thread.  One barrier.  `wtot` is LDS of NW elements that
// must not be rewritten before a later barrier.
template <int K, int NW, int KS = K>
__device__ __forceinline__ SegVal<K, KS> block_exclusive_scan(const SegVal<K, KS> &x, SegVal<K, KS> *wtot,
                                                              SegVal<K, KS> &total)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const SegVal<K, KS> inc = wave_inclusive_scan(x);
    const SegVal<K, KS> exc = wave_shift_right(inc);
    if (lane == kWave - 1) wtot[w] = inc;
    __syncthreads();
    SegVal<K, KS> pre = seg_identity<K, KS>(), tot = seg_identity<K, KS>();
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const SegVal<K, KS> t = wtot[k];
        if (k < w) pre = seg_combine(pre, t);
        tot = seg_combine(tot, t);
    }
    total = tot;
    return seg_combine(pre, exc);
}

// ------------------------------------------------------------------ packets

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct alignas(16) Packet {
    double v;
    uint32_t epoch;
    uint32_t aux;
};

// A packet array addressed through a buffer resource: accesses beyond
// `bytes` are dropped (stores) or read as zero (loads) by the hardware, so a
// wrong index can never touch other memory.
struct PacketArray {
    __amdgpu_buffer_rsrc_t rsrc;
};

// gfx9 raw-buffer descriptor word 3 (32-bit data format, no swizzle)
constexpr int kBufferWord3 = 0x00020000;
// cache-policy bits of the buffer builtins: sc1 = device-coherent; bit 31 = volatile
constexpr int kPolicyCoherent = 1 << 4;
constexpr int kPolicyVolatile = 1 << 31;

__device__ __forceinline__ PacketArray packet_array(const void *base, size_t bytes)
{
    PacketArray a;
    a.rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kBufferWord3);
    return a;
}

__device__ __forceinline__ void packet_put(const PacketArray &a, uint32_t index, double v, uint32_t epoch,
                                           uint32_t aux)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const u32x4 d = {(unsigned)b, (unsigned)(b >> 32), epoch, aux};
    __builtin_amdgcn_raw_buffer_store_b128(d, a.rsrc, (int)(index * sizeof(Packet)), 0, kPolicyCoherent);
}

__device__ __forceinline__ u32x4 packet_get(const PacketArray &a, uint32_t index)
{
    return __builtin_amdgcn_raw_buffer_load_b128(a.rsrc, (int)(index * sizeof(Packet)), 0,
                                                 kPolicyCoherent | kPolicyVolatile);
}

__device__ __forceinline__ double packet_value(const u32x4 &r)
{
    return __longlong_as_double((long long)(((unsigned long long)r.y << 32) | r.x));
}

// Control words shared by all workgroups of one launch.
struct SyncCtl {
    uint32_t abort;        // set to 1 by any workgroup whose wait timed out
    uint32_t pad[63];
};

// Wall-clock bound on any single wait (the constant-rate 100 MHz counter).
constexpr uint64_t kWaitTicks = 200000000ull;   // 2 s
// Polls between checks of the clock and of the abort word.
constexpr int kPollsPerCheck = 256;

__device__ __forceinline__ bool abort_raised(const SyncCtl *ctl)
{
    return __hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
}

__device__ __forceinline__ void raise_abort(SyncCtl *ctl)
{
    __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait used by every poll loop: call once per failed poll; returns
// false once the wait has exceeded kWaitTicks (raising abort) or another
// workgroup has aborted.  Every wait therefore ends.
struct WaitBudget {
    uint64_t t0;
    int polls;
    __device__ __forceinline__ WaitBudget() : t0(wall_clock64()), polls(0) {}
    __device__ __forceinline__ bool keep_waiting(SyncCtl *ctl)
    {
        if (++polls % kPollsPerCheck == 0) {
            if (abort_raised(ctl)) return false;
            if (wall_clock64() - t0 > kWaitTicks) {
                raise_abort(ctl);
                return false;
            }
        }
        __builtin_amdgcn_s_sleep(1);
        return true;
    }
};

// Wait until the N packets starting at `index` all carry `epoch`.
template <int N>
__device__ __forceinline__ bool packets_wait(const PacketArray &a, uint32_t index, uint32_t epoch, SyncCtl *ctl,
                                             u32x4 (&r)[N])
{
    WaitBudget wb;
    for (;;) {
        bool ready = true;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            r[k] = packet_get(a, index + k);
            ready = ready && (r[k].z == epoch);
        }
        if (ready) return true;
        if (!wb.keep_waiting(ctl)) return false;
    }
}

// ------------------------------------------------------------------ look-back

// Publish a tile aggregate as K packets at index K*b: (v0, epoch, f), (v1, epoch), ...
template <int K, int KS>
__device__ __forceinline__ void publish_aggregate(const PacketArray &agg, int b, const SegVal<K, KS> &a, uint32_t epoch)
{
#pragma unroll
    for (int k = 0; k < K; ++k) packet_put(agg, (uint32_t)(K * b + k), a.v[k], epoch, k == 0 ? a.f : 0u);
}

// Carry into tile b: the ordered combination of the aggregates published by
// tiles 0..b-1 for `epoch`.  Called by every thread of the workgroup (b
// uniform, 1 <= b <= 256).  Wave k reads the window of predecessors
// [b - 64(k+1), b - 64k - 1] -- all windows in flight at once -- with lane
// order equal to row order, scans it, and leaves the window total in
// win[k]; after one barrier every thread folds the windows from the
// farthest to the nearest.  Heads inside a window cut the carry as the
// operator requires.  Returns false (uniformly) on abort.
template <int K, int KS = K>
__device__ __forceinline__ bool look_back(int b, uint32_t epoch, const PacketArray &agg, SyncCtl *ctl,
                                          SegVal<K, KS> *win, int *abort_flag, SegVal<K, KS> &carry)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int nwin = (b + kWave - 1) / kWave;
    if (w < nwin) {
        const int q = b - kWave * (w + 1) + lane;
        SegVal<K, KS> x = seg_identity<K, KS>();
        bool ok = true;
        if (q >= 0) {
            u32x4 r[K];
            ok = packets_wait<K>(agg, (uint32_t)(K * q), epoch, ctl, r);
            if (ok) {
                x.f = r[0].w;
#pragma unroll
                for (int k = 0; k < K; ++k) x.v[k] = packet_value(r[k]);
            }
        }
        if (!ok) *abort_flag = 1;
        const SegVal<K, KS> inc = wave_inclusive_scan(x);
        if (lane == kWave - 1) win[w] = inc;
    }
    __syncthreads();
    if (*abort_flag) return false;
    carry = seg_identity<K, KS>();
    for (int k = nwin - 1; k >= 0; --k) carry = seg_combine(carry, win[k]);
    return true;
}

}  // namespace coxmi
