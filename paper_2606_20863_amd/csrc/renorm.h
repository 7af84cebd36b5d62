// Exact greedy round-to-nearest of a multi-word integer into m doubles: the
// renormalisation step of the m-double product (the paper's postponed
// renormalisation, done once per output entry).
//
// The value is X 2^scale with X an integer held as 4 beta-bit columns
// (carried, the top one signed) and then as the magnitude in 32-bit limbs
// L[0..NL).
// Word t is RN(X_t 2^scale), X_0 = X, X_(t+1) = X_t - word t, round to
// nearest with ties to even and the unit clamped at 2^-1074 (subnormal
// words).  Every limb index is a compile-time constant, so the limbs stay in
// registers: data-dependent positions become selects and shift networks.
//
// Plain C++ apart from the __device__ __forceinline__ annotations, so that a
// host build of this header can be checked against an exact reference.
#pragma once

#include <cmath>
#include <cstdint>

namespace mdg {

__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }

// Register layout for S diagonals of B-bit digits (B = 7 or 8): four
// diagonals per column, kCols columns of weight 2^(kCW j) (the top one takes
// only carries and is signed) and the kLimbs 32-bit limbs of the magnitude
// (kCols-1 columns of kCW bits, a top one below 2^64).
template <int S, int B = 7>
struct Tri {
    static constexpr int kCW = 4 * B;
    static constexpr int kCols = (S + 3) / 4 + 1;
    static constexpr int kLimbs = (kCW * (kCols - 1) + 64 + 31) / 32;
};

// Carry every column but the top one into [0, 2^CW).
template <int CW, int NC>
__device__ __forceinline__ void carry_cols(int64_t (&x)[NC])
{
#pragma unroll
    for (int j = 0; j + 1 < NC; ++j) {
        x[j + 1] += x[j] >> CW;
        x[j] &= ((int64_t)1 << CW) - 1;
    }
}

// Limb k of the integer whose limb 0 is zero and limbs 1..NL are L[0..NL-1]
// (bits of X shifted up by 32, so that bit unit-1 >= -1 of X has a place).
template <int NL>
__device__ __forceinline__ uint32_t shifted_limb(const uint32_t (&L)[NL], int k)
{
    return (k >= 1 && k <= NL) ? L[k - 1] : 0u;
}

// One greedy round-to-nearest step on (-1)^neg X 2^scale, X >= 0 held in
// 32-bit limbs L: returns the word RN(X 2^scale) (with sign) and leaves the
// remainder in L and its sign in sgn.  Any unit (clamped at 2^-1074 and at
// bit 0 of X); no branches, so that the steps of several outputs interleave.
template <int NL>
__device__ __forceinline__ double rn_step(uint32_t (&L)[NL], double& sgn, int umin, int scale)
{
    int top = -1;
#pragma unroll
    for (int k = 0; k < NL; ++k)
        top = L[k] ? 32 * k + 31 - __builtin_clz(L[k]) : top;
    const int unit = imax(imax(top - 52, umin), 0);
    // 64 bits of X from bit unit-1: the round bit, then the 53-bit
    // significand; sticky: any bit below unit-1
    const int P = unit + 31, q = P >> 5, r = P & 31;
    uint32_t l0 = 0, l1 = 0, l2 = 0, st = 0;
#pragma unroll
    for (int k = 0; k <= NL; ++k) {
        const uint32_t v = shifted_limb(L, k);
        st |= k < q ? v : (k == q ? v & ((1u << r) - 1u) : 0u);
        l0 = k == q ? v : l0;
        l1 = k == q ? shifted_limb(L, k + 1) : l1;
        l2 = k == q ? shifted_limb(L, k + 2) : l2;
    }
    const uint64_t lo = (uint64_t)l0 | ((uint64_t)l1 << 32);
    const uint64_t win = r ? ((lo >> r) | ((uint64_t)l2 << (64 - r))) : lo;
    uint64_t n = win >> 1;
    const bool up = (win & 1) && (st || (n & 1));
    n += up;
    const double w = top >= 0 ? sgn * ldexp((double)n, unit + scale) : 0.0;
    // remainder: the bits below unit; rounded up, 2^unit minus them with the
    // sign flipped
    uint64_t cy = 1;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int b = unit - 32 * k;
        const uint32_t keep = b >= 32 ? ~0u : (b <= 0 ? 0u : (1u << b) - 1u);
        const uint64_t v = (uint64_t)(~L[k]) + cy;
        cy = v >> 32;
        L[k] = (up ? (uint32_t)v : L[k]) & keep;
    }
    sgn = up ? -sgn : sgn;
    return w;
}

// Shift the limbs left so that the top set bit lands on bit 32 NL - 1; the
// value L 2^scale is kept (scale drops by the shift).  False if L is zero.
template <int NL>
__device__ __forceinline__ bool align_left(uint32_t (&L)[NL], int& scale)
{
    int top = -1;
#pragma unroll
    for (int k = 0; k < NL; ++k)
        top = L[k] ? 32 * k + 31 - __builtin_clz(L[k]) : top;
    const int d = top < 0 ? 0 : 32 * NL - 1 - top;
    const int q = d >> 5, r = d & 31;
    // whole limbs: a shift by q as a network of shifts by 1, 2, 4, 8 limbs
#pragma unroll
    for (int b = 1; b < NL; b <<= 1) {
        const bool on = (q & b) != 0;
#pragma unroll
        for (int k = NL - 1; k >= 0; --k)
            L[k] = on ? (k >= b ? L[k - b] : 0u) : L[k];
    }
    // then r bits
#pragma unroll
    for (int k = NL - 1; k >= 0; --k) {
        const uint32_t lo = k ? L[k - 1] : 0u;
        L[k] = r ? (uint32_t)((((uint64_t)L[k] << 32) | lo) >> (32 - r)) : L[k];
    }
    scale -= d;
    return top >= 0;
}

// One greedy round-to-nearest step on left-aligned limbs whose unit
// 2^(32 NL - 53 + scale) is not below 2^-1074: the significand, the round
// bit and the sticky bits sit at fixed places.  Returns the word; the
// remainder (sign in sgn) is left in L.
template <int NL>
__device__ __forceinline__ double rn_step_aligned(uint32_t (&L)[NL], double& sgn, int scale)
{
    static_assert(NL >= 3, "at least three limbs");
    const uint64_t n = ((uint64_t)L[NL - 1] << 21) | (L[NL - 2] >> 11);
    const bool rnd = (L[NL - 2] >> 10) & 1u;
    uint32_t st = L[NL - 2] & 0x3ffu;
#pragma unroll
    for (int k = 0; k < NL - 2; ++k)
        st |= L[k];
    const bool up = rnd && (st || (n & 1));
    const double w = sgn * ldexp((double)(n + up), 32 * NL - 53 + scale);
    // remainder: the bits below the unit; rounded up, 2^unit minus them with
    // the sign flipped
    L[NL - 1] = 0;
    L[NL - 2] &= 0x7ffu;
    uint64_t cy = 1;
#pragma unroll
    for (int k = 0; k < NL - 1; ++k) {
        const uint64_t v = (uint64_t)(~L[k]) + cy;
        cy = v >> 32;
        L[k] = up ? (uint32_t)v & (k == NL - 2 ? 0x7ffu : ~0u) : L[k];
    }
    sgn = up ? -sgn : sgn;
    return w;
}

// Shift the limbs left by 53 bits (one limb and 21 bits, fixed places);
// the caller has checked that no set bit lies above bit 32 NL - 54.
template <int NL>
__device__ __forceinline__ void shift_left_53(uint32_t (&L)[NL])
{
#pragma unroll
    for (int k = NL - 1; k >= 0; --k)
        L[k] = k >= 2 ? (L[k - 1] << 21) | (L[k - 2] >> 11) : (k == 1 ? L[0] << 21 : 0u);
}

// Greedy step on any limbs: aligned, then the fixed-place step, or the
// general one where the unit would fall below 2^-1074.  A remainder left
// by a step has no set bit above bit 32 NL - 54 (the step cleared its unit
// and everything above), so it is first moved up by those 53 bits at fixed
// places, and where its top bit then lies in the top limb, a shift by that
// limb's leading zeros finishes the alignment without the limb network:
// the same total shift as align_left's, so the same word.  FAST = false
// keeps the limb network for every word (fewer live registers).
template <int NL, bool FAST = true>
__device__ __forceinline__ double rn_next(uint32_t (&L)[NL], double& sgn, int& scale)
{
    static_assert(NL >= 3, "at least three limbs");
    bool aligned = false;
    if (FAST && L[NL - 1] == 0 && (L[NL - 2] >> 11) == 0) {
        shift_left_53(L);
        scale -= 53;
        if (L[NL - 1] != 0) {
            const int z = __builtin_clz(L[NL - 1]);
#pragma unroll
            for (int k = NL - 1; k >= 0; --k) {
                const uint32_t lo = k ? L[k - 1] : 0u;
                L[k] = z ? (L[k] << z) | (lo >> (32 - z)) : L[k];
            }
            scale -= z;
            aligned = true;
        }
    }
    if (!aligned && !align_left(L, scale))
        return 0.0;
    if (32 * NL - 53 + scale >= -1074)
        return rn_step_aligned(L, sgn, scale);
    return rn_step(L, sgn, -1074 - scale, scale);
}

// Magnitude limbs of the carried CW-bit columns; returns the sign.
template <int CW, int NC, int NL>
__device__ __forceinline__ bool to_limbs(int64_t (&x)[NC], uint32_t (&L)[NL])
{
    const bool neg = x[NC - 1] < 0;
#pragma unroll
    for (int j = 0; j < NC; ++j)
        x[j] = neg ? -x[j] : x[j];
    carry_cols<CW>(x);
#pragma unroll
    for (int k = 0; k < NL; ++k)
        L[k] = 0;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        const uint64_t v = (uint64_t)x[j];
        const int b = CW * j, k = b >> 5, r = b & 31;
        L[k] |= (uint32_t)(v << r);
        if (k + 1 < NL)
            L[k + 1] |= (uint32_t)(r ? v >> (32 - r) : v >> 32);
        if (k + 2 < NL && r)
            L[k + 2] |= (uint32_t)(v >> (64 - r));
    }
    return neg;
}


}  // namespace mdg
