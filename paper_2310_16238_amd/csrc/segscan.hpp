// segscan.hpp -- device building blocks for the segmented scan of Sec. 2.6 on gfx950.
//
// A scan element is a flag-value pair (f, v) with v a small tuple of doubles.
// The operator is the flag-value operator of Sec. 2.6 with + as the base:
//     (f_a, a) (+)s (f_b, b) = (f_a | f_b, f_b ? b : a + b)
// It is associative but not commutative: the left operand is the earlier row.
// (0, 0) is its identity on both sides.
//
// Layout of work on the chip (ours, not the paper's): a workgroup of NW
// wave64s owns a contiguous tile of rows, each thread IPT consecutive rows.
// The tile's scan is
//   thread-sequential fold over its IPT rows
//   -> wave64 inclusive scan with cross-lane shuffles (6 steps)
//   -> scan of the NW wave totals through LDS
// and the carry between tiles comes from the preceding tiles' published
// aggregates (look-back), read with agent-scope acquire loads.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace coxmi {

constexpr int kWave = 64;

template <int K>
struct SegVal {
    uint32_t f;
    double v[K];
};

template <int K>
__device__ __forceinline__ SegVal<K> seg_identity()
{
    SegVal<K> r;
    r.f = 0u;
#pragma unroll
    for (int k = 0; k < K; ++k) r.v[k] = 0.0;
    return r;
}

// a is the earlier (left) element, b the later one.
template <int K>
__device__ __forceinline__ SegVal<K> seg_combine(const SegVal<K> &a, const SegVal<K> &b)
{
    SegVal<K> r;
    r.f = a.f | b.f;
#pragma unroll
    for (int k = 0; k < K; ++k) r.v[k] = b.f ? b.v[k] : a.v[k] + b.v[k];
    return r;
}

template <int K>
__device__ __forceinline__ SegVal<K> shfl_up_seg(const SegVal<K> &x, int off)
{
    SegVal<K> r;
    r.f = __shfl_up(x.f, off, kWave);
#pragma unroll
    for (int k = 0; k < K; ++k) r.v[k] = __shfl_up(x.v[k], off, kWave);
    return r;
}

template <int K>
__device__ __forceinline__ SegVal<K> shfl_down_seg(const SegVal<K> &x, int off)
{
    SegVal<K> r;
    r.f = __shfl_down(x.f, off, kWave);
#pragma unroll
    for (int k = 0; k < K; ++k) r.v[k] = __shfl_down(x.v[k], off, kWave);
    return r;
}

// Inclusive scan across the 64 lanes of a wave (lane order = row order).
template <int K>
__device__ __forceinline__ SegVal<K> wave_inclusive_scan(SegVal<K> x, int lane)
{
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        SegVal<K> o = shfl_up_seg(x, off);
        if (lane >= off) x = seg_combine(o, x);
    }
    return x;
}

// Ordered reduction where lane 63 holds the leftmost element and lane 0 the
// rightmost: lane 0 ends with x[63] (+)s x[62] (+)s ... (+)s x[0].
template <int K>
__device__ __forceinline__ SegVal<K> wave_reduce_right_to_left(SegVal<K> x, int lane)
{
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        SegVal<K> o = shfl_down_seg(x, off);
        if (lane + off < kWave) x = seg_combine(o, x);
    }
    return x;
}

template <int K, int NW>
struct BlockScanSmem {
    SegVal<K> wave_total[NW];
    SegVal<K> wave_prefix[NW];
    SegVal<K> block_total;
};

// Exclusive scan of one element per thread over the whole workgroup.
// Returns the thread's exclusive prefix (identity for thread 0); the block
// total is left in sm.block_total.  Contains two workgroup barriers.
template <int K, int NW>
__device__ __forceinline__ SegVal<K> block_exclusive_scan(const SegVal<K> &x, BlockScanSmem<K, NW> &sm)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    SegVal<K> inc = wave_inclusive_scan(x, lane);
    SegVal<K> exc = shfl_up_seg(inc, 1);
    if (lane == 0) exc = seg_identity<K>();
    if (lane == kWave - 1) sm.wave_total[w] = inc;
    __syncthreads();
    if (w == 0) {
        SegVal<K> t = lane < NW ? sm.wave_total[lane] : seg_identity<K>();
        SegVal<K> ti = wave_inclusive_scan(t, lane);
        SegVal<K> te = shfl_up_seg(ti, 1);
        if (lane == 0) te = seg_identity<K>();
        if (lane < NW) sm.wave_prefix[lane] = te;
        if (lane == NW - 1) sm.block_total = ti;
    }
    __syncthreads();
    return seg_combine(sm.wave_prefix[w], exc);
}

// ---------------------------------------------------------------- cross-workgroup flags

// Control words shared by all workgroups of one launch.
struct SyncCtl {
    uint32_t abort;        // set to 1 by any workgroup whose wait timed out
    uint32_t numeric;      // set to 1 if a risk-set sum left the FP64 normal range
    uint32_t pad[62];
};

__device__ __forceinline__ uint32_t load_acquire(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_release(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Wall-clock bound on any single wait (the constant-rate 100 MHz counter).
constexpr uint64_t kWaitTicks = 200000000ull;   // 2 s

// Wait until *flag == want.  Returns false (and raises ctl->abort) if the wait
// exceeds kWaitTicks or another workgroup has raised abort; the caller must
// then leave the kernel.  Every wait therefore ends.
__device__ __forceinline__ bool wait_equal(const uint32_t *flag, uint32_t want, SyncCtl *ctl)
{
    if (load_acquire(flag) == want) return true;
    const uint64_t t0 = wall_clock64();
    for (;;) {
        __builtin_amdgcn_s_sleep(1);
        if (load_acquire(flag) == want) return true;
        if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return false;
        if (wall_clock64() - t0 > kWaitTicks) {
            __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
}

// Published tile aggregate for the look-back: flag and values as doubles.
template <int K>
struct alignas(16) TileAgg {
    double f;
    double v[K];
};

// Carry into tile `b` = ordered combination of the aggregates of tiles
// 0..b-1, stopping at the nearest tile that contains a head flag (everything
// before it is discarded by the operator anyway).  Executed by one whole wave;
// the result is valid in lane 0.  Returns false on abort.
template <int K>
__device__ __forceinline__ bool look_back(int b, uint32_t epoch, const TileAgg<K> *agg,
                                          const uint32_t *status, SyncCtl *ctl, SegVal<K> &carry)
{
    const int lane = threadIdx.x & (kWave - 1);
    carry = seg_identity<K>();
    int base = b - 1;
    bool ok = true;
    while (base >= 0) {
        const int q = base - lane;
        SegVal<K> x = seg_identity<K>();
        if (q >= 0) {
            ok = wait_equal(&status[q], epoch, ctl);
            if (ok) {
                x.f = agg[q].f != 0.0 ? 1u : 0u;
#pragma unroll
                for (int k = 0; k < K; ++k) x.v[k] = agg[q].v[k];
            }
        }
        if (__any(!ok)) return false;
        SegVal<K> win = wave_reduce_right_to_left(x, lane);
        // broadcast lane 0's window total
        win.f = __shfl(win.f, 0, kWave);
#pragma unroll
        for (int k = 0; k < K; ++k) win.v[k] = __shfl(win.v[k], 0, kWave);
        carry = seg_combine(win, carry);
        if (win.f) break;
        base -= kWave;
    }
    return true;
}

}  // namespace coxmi
