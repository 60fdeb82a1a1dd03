// Device building blocks shared by the resampling kernels (gfx950, wave64).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11), counter-based, so any draw is
// addressed by (seed, counter) with no per-thread state. Counter words are
// (c0, c1, c2, c3) = (particle or particle group, instance, draw block, tag).
#pragma once

#include <hip/hip_runtime.h>

#include "launch.h"
#include <stdint.h>

namespace rs {

constexpr int kWave = 64;

// Counter tags: which step of the method a Philox block feeds.
constexpr uint32_t kTagMetropolis = 1u;
constexpr uint32_t kTagStratified = 2u;
constexpr uint32_t kTagSystematic = 3u;
constexpr uint32_t kTagMultinomial = 4u;
constexpr uint32_t kTagFilterNoise = 5u;

// Status bits (mirror RS_FLAG_* in resample.h).
constexpr int kFlagNan = 1;
constexpr int kFlagPosInf = 2;
constexpr int kFlagAllNegInf = 4;
constexpr int kFlagBadAncestor = 8;
constexpr int kFlagInternal = 16;

struct Block4 {
    uint32_t r0, r1, r2, r3;
};

// Ten Philox rounds: two 32x32->64 products per round (multipliers from the
// SC'11 paper); the key advances by the Weyl increments between rounds.
__device__ __forceinline__ Block4 philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                                         uint32_t c3)
{
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Block4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t word(const Block4 &b, uint32_t k)
{
    return k == 0 ? b.r0 : k == 1 ? b.r1 : k == 2 ? b.r2 : b.r3;
}

// Uniform index in [0, P): the high word of r * P.
__device__ __forceinline__ uint32_t uniform_index(uint32_t r, uint32_t P)
{
    return (uint32_t)(((uint64_t)r * (uint64_t)P) >> 32);
}

// Uniform on the open binary32 grid (2m + 1) 2^-24, m = r >> 9.
__device__ __forceinline__ float grid_uniform(uint32_t r)
{
    return (float)(2u * (r >> 9) + 1u) * 0x1p-24f;
}

// Correctly rounded binary32 log of a grid uniform, via the binary64 log.
__device__ __forceinline__ float exact_log_u(float u)
{
    return (float)log((double)u);
}

// Uniform in [0, 1) with 32 random bits, as binary64.
__device__ __forceinline__ double unit32(uint32_t r)
{
    return (double)r * 0x1p-32;
}

// Uniform in [0, 1) with 53 random bits, as binary64.
__device__ __forceinline__ double unit53(uint32_t a, uint32_t b)
{
    return (double)(((uint64_t)a << 21) | (uint64_t)(b >> 11)) * 0x1p-53;
}

// ---------------------------------------------------------------- wave ops
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x / kWave); }

// Lane moves by DPP (GFX9 controls): the source lane is read inside the VALU
// instruction, with no LDS round trip as a ds_bpermute shuffle takes. A lane
// whose source lies outside the pattern, or in a row the row mask leaves
// out, receives `fill`. Wave ops below run in uniform control flow (all 64
// lanes active).
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114,
              kDppRowShr8 = 0x118, kDppWaveShr1 = 0x138, kDppRowBcast15 = 0x142,
              kDppRowBcast31 = 0x143;

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v, uint32_t fill)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, CTRL, ROW_MASK, 0xf, false);
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v, uint64_t fill)
{
    const uint64_t lo = dpp_u32<CTRL, ROW_MASK>((uint32_t)v, (uint32_t)fill);
    const uint64_t hi = dpp_u32<CTRL, ROW_MASK>((uint32_t)(v >> 32), (uint32_t)(fill >> 32));
    return (hi << 32) | lo;
}

template <int CTRL, int ROW_MASK = 0xf, typename T>
__device__ __forceinline__ T dpp_move(T v, T fill)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit lanes");
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, dpp_u64<CTRL, ROW_MASK>(__builtin_bit_cast(uint64_t, v),
                                                             __builtin_bit_cast(uint64_t, fill)));
    else
        return __builtin_bit_cast(T, dpp_u32<CTRL, ROW_MASK>(__builtin_bit_cast(uint32_t, v),
                                                             __builtin_bit_cast(uint32_t, fill)));
}

// Inclusive scan over the 64 lanes with an associative op and its identity:
// Hillis-Steele inside each row of 16 lanes (shifts 1, 2, 4, 8), then row
// 0's total into row 1 and row 2's into row 3, then rows 0-1's total into
// rows 2 and 3. A fixed order, so the same bits on every call.
template <typename T, typename Op>
__device__ __forceinline__ T wave_scan(T v, T id, Op op)
{
    v = op(v, dpp_move<kDppRowShr1>(v, id));
    v = op(v, dpp_move<kDppRowShr2>(v, id));
    v = op(v, dpp_move<kDppRowShr4>(v, id));
    v = op(v, dpp_move<kDppRowShr8>(v, id));
    v = op(v, dpp_move<kDppRowBcast15, 0xa>(v, id));
    v = op(v, dpp_move<kDppRowBcast31, 0xc>(v, id));
    return v;
}

// Lane 63's value, in every lane.
__device__ __forceinline__ double lane63(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
    return __longlong_as_double((long long)((hi << 32) | lo));
}
__device__ __forceinline__ float lane63(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ int lane63(int v) { return __builtin_amdgcn_readlane(v, 63); }

struct AddOp { template <typename T> __device__ T operator()(T a, T b) const { return a + b; } };
struct MaxOp {
    __device__ float operator()(float a, float b) const { return fmaxf(a, b); }
    __device__ double operator()(double a, double b) const { return fmax(a, b); }
};
struct OrOp { __device__ int operator()(int a, int b) const { return a | b; } };

__device__ __forceinline__ double wave_inclusive_sum(double v) { return wave_scan(v, 0.0, AddOp{}); }

// Inclusive prefix maximum of non-negative values (0 is the identity).
__device__ __forceinline__ double wave_inclusive_max_nonneg(double v)
{
    return wave_scan(v, 0.0, MaxOp{});
}

// Each lane gets its left neighbour's value, lane 0 gets 0.
template <typename T>
__device__ __forceinline__ T wave_shift_up(T v) { return dpp_move<kDppWaveShr1>(v, (T)0); }

__device__ __forceinline__ double wave_sum(double v) { return lane63(wave_scan(v, 0.0, AddOp{})); }

__device__ __forceinline__ float wave_max(float v)
{
    return lane63(wave_scan(v, -(float)INFINITY, MaxOp{}));
}

__device__ __forceinline__ double wave_max(double v)
{
    return lane63(wave_scan(v, -(double)INFINITY, MaxOp{}));
}

__device__ __forceinline__ int wave_or(int v) { return lane63(wave_scan(v, 0, OrOp{})); }

// Largest binary64 strictly below a positive finite b.
__device__ __forceinline__ double below(double b)
{
    return __longlong_as_double(__double_as_longlong(b) - 1);
}

__device__ __forceinline__ void raise_flags(int32_t *status, int flags)
{
    if (flags && status) atomicOr(status, flags);
}

// Row dst of x_out from row src of x_in, elements first, first + step, ...
// (16-byte vectors when the rows allow).
__device__ __forceinline__ void copy_row(const Rows &r, int64_t dst, int64_t src, int first,
                                         int step)
{
    const int D = r.D;
    if ((D & 3) == 0 && ((((uintptr_t)r.x_in) | ((uintptr_t)r.x_out)) & 15) == 0) {
        const float4 *in = reinterpret_cast<const float4 *>(r.x_in) + src * (D / 4);
        float4 *out = reinterpret_cast<float4 *>(r.x_out) + dst * (D / 4);
        for (int c = first; c < D / 4; c += step) out[c] = in[c];
    } else {
        for (int c = first; c < D; c += step) r.x_out[dst * D + c] = r.x_in[src * D + c];
    }
}

}  // namespace rs
