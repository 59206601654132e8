// mhar_device.hpp -- device building blocks of the MHAR step on gfx950:
// counter-based random streams, matrix-core wrappers and operand splitting.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mhar {

constexpr uint32_t kTagDir = 0;
constexpr uint32_t kTagTheta = 1;
constexpr uint32_t kTagLowRank = 2;

struct Block4 {
    uint32_t w0, w1, w2, w3;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Each round multiplies
// counter words 0 and 2 by the two published constants; the high halves are
// xor-ed with the other two words and the round key, the low halves are
// passed through; the key advances by the two published Weyl increments.
__device__ __forceinline__ Block4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // one 32 x 32 -> 64 multiply (v_mad_u64_u32) per product instead
        // of separate high and low multiplies
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Block4{c0, c1, c2, c3};
}

// Block `block` of stream (seed, tag, chain, step); counter words are
// (block, chain, step low, tag | step high << 4), key is the seed.
__device__ __forceinline__ Block4 stream_block(uint64_t seed, uint32_t tag, uint32_t chain,
                                               uint64_t step, uint32_t block)
{
    return philox4x32_10(block, chain, (uint32_t)step, tag | (uint32_t)((step >> 32) << 4),
                         (uint32_t)seed, (uint32_t)(seed >> 32));
}

// 52 random bits -> (k + 1/2) 2^-52: exact in binary64, strictly in (0, 1).
__device__ __forceinline__ double open_unit(uint32_t hi, uint32_t lo)
{
    uint64_t k = ((((uint64_t)hi) << 32) | (uint64_t)lo) >> 12;
    return __dmul_rn(__dadd_rn((double)k, 0.5), 0x1.0p-52);
}

// Two N(0,1) variates from one block by the Box-Muller transform.
__device__ __forceinline__ void gauss_pair(const Block4& w, double& even, double& odd)
{
    double ua = open_unit(w.w0, w.w1);
    double ub = open_unit(w.w2, w.w3);
    double radius = sqrt(__dmul_rn(-2.0, log(ua)));
    // the angle 2 pi ub is taken as pi times the exact 2 ub: no rounded
    // product with 2 pi, and sinpi/cospi reduce their argument exactly in
    // about half the instructions of sin/cos of a general argument
    double sn, cs;
    sincospi(__dmul_rn(2.0, ub), &sn, &cs);
    even = __dmul_rn(radius, cs);
    odd = __dmul_rn(radius, sn);
}

// ---------------------------------------------------------------------------
// Matrix-core wrappers (16 x 16 output tile per wave, 4 values per lane).
// Operand lane layouts (lane l, g = l / 16, c = l % 16), checked on gfx950:
//   f32 16x16x4 : a = A[c][g], b = B[g][c], out[r] = C[4g + r][c]
//   bf16 16x16x32: a = A[c][8g + e], b = B[8g + e][c] (e < 8), out as f32
//   f64 16x16x4 : a = A[c][g], b = B[g][c], out[r] = C[4r + g][c]
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 mma_f32(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f64x4 mma_f64(double a, double b, f64x4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mma_bf16(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Row (within a 16-row block) of output value r held by lane group g.
template <bool F64>
__device__ __forceinline__ int out_row(int g, int r)
{
    return F64 ? (4 * r + g) : (4 * g + r);
}

// Split an FP32 value into bf16 hi + lo with hi = rn(v), lo = rn(v - hi).
__device__ __forceinline__ void split_bf16(float v, __bf16& hi, __bf16& lo)
{
    hi = (__bf16)v;
    lo = (__bf16)(v - (float)hi);
}

// Wave-wide reductions (64 lanes).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

constexpr float kInf = __builtin_huge_valf();
constexpr double kInfD = __builtin_huge_val();
constexpr float kLowShrink = 1.0f - 0x1.0p-20f;  // turns rounded lower bounds into safe ones
constexpr float kHighGrow = 1.0f + 0x1.0p-20f;
constexpr float kScreenSlack = 1.0f + 0x1.0p-18f;  // product form of the candidate test
constexpr float kTinySlack = 0x1.0p-100f;         // slack lower bounds below this are always candidates

// Interval bounds of the two chord-end ratios of one (row, walk) entry.
//   s, g   : approximate slack and directional derivative
//   dl     : bound on |s_hat - s|;  e: bound on |g_hat - g|
// plus side (g > 0):   lo_p <= s/g <= hi_p   (hi_p finite only if g surely > 0)
// minus side (g < 0):  lo_m <= s/(-g) <= hi_m
__device__ __forceinline__ void ratio_bounds(float s, float g, float dl, float e, float& lo_p,
                                             float& hi_p, float& lo_m, float& hi_m)
{
    float s_lo = fmaxf(s - dl, 0.0f);
    float s_hi = s + dl;
    float g_hi = g + e, g_lo = g - e;    // g in [g_lo, g_hi]
    // two reciprocals serve both signs: 1/(-x) = -(1/x) (the approximation
    // is odd), within the error the shrink and grow factors cover
    const float r_hi = __builtin_amdgcn_rcpf(g_hi), r_lo = __builtin_amdgcn_rcpf(g_lo);
    lo_p = (g_hi > 0.0f) ? s_lo * r_hi * kLowShrink : kInf;
    hi_p = (g_lo > 0.0f) ? s_hi * r_lo * kHighGrow : kInf;
    // -g in [-g_hi, -g_lo]
    lo_m = (g_lo < 0.0f) ? s_lo * -r_lo * kLowShrink : kInf;
    hi_m = (g_hi < 0.0f) ? s_hi * -r_hi * kHighGrow : kInf;
}

}  // namespace mhar
