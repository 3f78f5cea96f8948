// affscan.hpp -- segmented scans whose elements are not plain sums: the
// running maximum of X beta, and first-order linear recurrences
// S_r = alpha_r S_{r-1} + b_r (composition of affine maps), used by the full
// evaluation to keep every risk-set sum relative to the running maximum of
// X beta within its stratum.
//
// For rows in canonical order with m_r the running maximum of eta over the
// stratum up to row r, alpha_r = exp(m_{r-1} - m_r) <= 1 and
// u_r = exp(eta_r - m_r) <= 1, the recurrence with b_r = u_r (or u_r x_rj)
// gives S0_r exp(-m_r) (or S1_rj exp(-m_r)): the same risk-set sums as the
// segmented scan of Sec. 2.6, scaled by a factor that depends only on the row,
// so ratios S1/S0 are unchanged and S0 exp(-m_r) lies in [1, n].
//
// A segmented element (f, a, b) stands for the map S -> a S + b restricted to a
// run of rows (f: the run contains a stratum head, after which the incoming S
// is dropped).  combine(A, B) applies A's rows first, then B's.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace coxmi {

struct MaxE {
    uint32_t f;
    double m;
};

struct AffE {
    uint32_t f;
    double a, b;
};

struct MaxOp {
    using E = MaxE;
    __device__ static E id() { return E{0u, -INFINITY}; }
    __device__ static E combine(const E &x, const E &y) { return E{x.f | y.f, y.f ? y.m : fmax(x.m, y.m)}; }
};

struct AffOp {
    using E = AffE;
    __device__ static E id() { return E{0u, 1.0, 0.0}; }
    __device__ static E combine(const E &x, const E &y)
    {
        return E{x.f | y.f, y.f ? y.a : x.a * y.a, y.f ? y.b : fma(y.a, x.b, y.b)};
    }
};

// DPP move whose lanes without a source (or in rows masked off) keep `old`.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_keep(double old, double x)
{
    return __builtin_amdgcn_update_dpp(old, x, CTRL, ROWS, 0xF, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_keep_u32(uint32_t old, uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)x, CTRL, ROWS, 0xF, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ MaxE dpp_e(const MaxE &x)
{
    return MaxE{dpp_keep_u32<CTRL, ROWS>(0u, x.f), dpp_keep<CTRL, ROWS>(-INFINITY, x.m)};
}

template <int CTRL, int ROWS>
__device__ __forceinline__ AffE dpp_e(const AffE &x)
{
    return AffE{dpp_keep_u32<CTRL, ROWS>(0u, x.f), dpp_keep<CTRL, ROWS>(1.0, x.a), dpp_keep<CTRL, ROWS>(0.0, x.b)};
}

__device__ __forceinline__ double readlane63(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ MaxE lane63_e(const MaxE &x)
{
    return MaxE{(uint32_t)__builtin_amdgcn_readlane((int)x.f, 63), readlane63(x.m)};
}

__device__ __forceinline__ AffE lane63_e(const AffE &x)
{
    return AffE{(uint32_t)__builtin_amdgcn_readlane((int)x.f, 63), readlane63(x.a), readlane63(x.b)};
}

// Inclusive scan across the 64 lanes (lane order = scan order); all lanes active.
template <class Op>
__device__ __forceinline__ typename Op::E wave_scan_e(typename Op::E x)
{
    x = Op::combine(dpp_e<0x111, 0xF>(x), x);
    x = Op::combine(dpp_e<0x112, 0xF>(x), x);
    x = Op::combine(dpp_e<0x114, 0xF>(x), x);
    x = Op::combine(dpp_e<0x118, 0xF>(x), x);
    x = Op::combine(dpp_e<0x142, 0xA>(x), x);
    x = Op::combine(dpp_e<0x143, 0xC>(x), x);
    return x;
}

// Lane i receives lane i-1's value, lane 0 the identity.
template <class E>
__device__ __forceinline__ E wave_shr1_e(const E &x)
{
    return dpp_e<0x138, 0xF>(x);
}

// Exclusive scan over the workgroup (NW waves, one element per thread); `total`
// receives the workgroup's total.  wtot: LDS of NW elements.  One barrier.
template <class Op, int NW>
__device__ __forceinline__ typename Op::E block_exclusive_e(const typename Op::E &x, typename Op::E *wtot,
                                                            typename Op::E &total)
{
    using E = typename Op::E;
    const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
    const E inc = wave_scan_e<Op>(x);
    const E exc = wave_shr1_e(inc);
    if (lane == 63) wtot[w] = inc;
    __syncthreads();
    E pre = Op::id(), tot = Op::id();
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const E t = wtot[k];
        if (k < w) pre = Op::combine(pre, t);
        tot = Op::combine(tot, t);
    }
    total = tot;
    return Op::combine(pre, exc);
}

}  // namespace coxmi
