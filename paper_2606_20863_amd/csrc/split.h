// Word decoding and bit-field gathering shared by the digit splits: the
// slices of an m-double entry on its row's grid are cut word by word (the
// paper's quarters, Section 2), each word's bits being a field of its
// significand shifted to the grid.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mdg {
namespace {

// |x| = mant * 2^ex with mant < 2^53; returns true if x < 0
__device__ __forceinline__ bool decode(double x, uint64_t& mant, int& ex)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const int eb = (int)((b >> 52) & 0x7ff);
    const uint64_t f = b & ((1ull << 52) - 1);
    mant = eb ? (f | (1ull << 52)) : f;
    ex = eb ? eb - 1075 : -1074;
    return (b >> 63) != 0;
}

// floor(mant * 2^sh) mod 2^W, W <= 63, mant < 2^53; branch-free (clamped
// shift counts and selects), as the word offsets differ from lane to lane
__device__ __forceinline__ uint64_t field(uint64_t mant, int sh, uint64_t wmask)
{
    const uint64_t up = mant << (sh & 63);                     // used for 0 <= sh < 63
    const uint64_t down = mant >> (sh < -63 ? 63 : -sh & 63);   // used for sh < 0
    const uint64_t v = sh >= 63 ? 0 : (sh >= 0 ? up : down);
    return v & wmask;
}

// Gather limb j (digits [D j, D j + D)) of the positive and the negative
// words of one entry.
template <int MW>
__device__ __forceinline__ void limb_pair(const uint64_t (&mant)[MW], const int (&sh0)[MW],
                                          const bool (&neg)[MW], int shift, uint64_t wmask,
                                          uint64_t& P, uint64_t& N)
{
    P = 0;
    N = 0;
#pragma unroll
    for (int w = 0; w < MW; ++w) {
        const uint64_t v = field(mant[w], sh0[w] + shift, wmask);
        N |= neg[w] ? v : 0;
        P |= neg[w] ? 0 : v;
    }
}

}  // namespace
}  // namespace mdg
