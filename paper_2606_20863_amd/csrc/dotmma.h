// Batched INT8 inner products for many slices (the paper's experiment,
// Section 3, at m = 8 and 16): the digits of x and of y as two matrices whose
// rows are the digit positions and whose columns are the entries, so that
// one matrix product over the entries gives every sum of slice products
// sum_k x_s[k] y_t[k] at once; the diagonal sums D_g of the method are the
// sums of that S x S matrix along its anti-diagonals s + t = g < S.  The
// 16 x 16 tiles of the product that hold any s + t <= SC - 1 are computed
// on the matrix cores, about half the tiles for large S (against a sixteenth
// of a matrix instruction's outputs kept when the pairs are put on the tile
// rows), and the digits never leave the workgroup.
//
// A workgroup of two waves takes one pair and a range of its depth, 128
// entries per round: wave 0 cuts two entries of x per lane, wave 1 two of y
// (word placement, one entry per byte), and each writes its digits to LDS,
// row s holding digit s of the round's entries, 32 words of four: lanes l
// and l + 32 fill the low and the high half of word l % 32, so byte 2 h + q
// of word c holds entry 64 q + 32 h + c.  After a barrier each wave
// multiplies its half of the needed tiles over the round's two 64-entry
// sub-blocks: the fragment of tile row I in sub-block j is, for lane L, the
// 16 bytes at words 16 j + 4 (L / 16) .. +3 of row 16 I + L % 16, for x and
// for y alike, so the instruction pairs entry with entry (whatever its order
// of the 64 entries inside).  A wave's limb store lives in its own digit
// rows where they hold it (cleared at the start of a round, overwritten by
// the digits once the cut has left it zero), else beside them: at SC = 112 a
// workgroup holds about 34 KB of LDS and a CU four workgroups.  Tile sums
// stay in int32: each adds at most 2^14 per
// entry, and the host caps the depth per workgroup at 65536 entries.  At the
// end every tile element goes into the int64 sum of its diagonal by an LDS
// atomic.  The rest is the lane kernel's: whole-pair mode (exponents found
// here, in-kernel rounding) or several depth ranges added into a zeroed D.
#pragma once

#include "dotlane.h"

namespace mdg {
namespace {

typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr int kMmaRound = 128;   // entries per round: two per lane
constexpr int kMmaRow = 36;      // 32-bit words per digit row (32 and 4 of padding)
constexpr int64_t kMmaMaxDepth = 65536;

// the needed tiles (I, J), I + J <= NT - 1, by anti-diagonal, dealt
// alternately to the two waves (tile 2 k + w is slot k of wave w; the last
// slot of wave 1 is empty, I = -1, when the count is odd)
template <int NT>
struct MmaTiles {
    static constexpr int N = NT * (NT + 1) / 2;
    static constexpr int SLOTS = (N + 1) / 2;
    int I[2 * SLOTS], J[2 * SLOTS];
    constexpr MmaTiles() : I(), J()
    {
        int k = 0;
        for (int d = 0; d < NT; ++d)
            for (int i = 0; i <= d; ++i) {
                I[k] = i;
                J[k] = d - i;
                ++k;
            }
        for (; k < 2 * SLOTS; ++k) {
            I[k] = -1;
            J[k] = -1;
        }
    }
};

// Wave W's tiles over the 64-entry sub-blocks of a round (xa, ya: this lane's
// fragment bytes in row 0 of the x and y digit rows; every offset from
// there a compile-time constant)
template <int NT, int W>
__device__ __forceinline__ void mma_round(i32x4 (&acc)[MmaTiles<NT>::SLOTS], const uint32_t* xa, const uint32_t* ya)
{
    constexpr MmaTiles<NT> kT{};
    unroll<kMmaRound / 64>([&](auto JJ) {
        constexpr int j = decltype(JJ)::value;
        unroll<MmaTiles<NT>::SLOTS>([&](auto KK) {
            constexpr int k = decltype(KK)::value, I = kT.I[2 * k + W], J = kT.J[2 * k + W];
            if constexpr (I >= 0) {
                const i32x4 fa = *(const i32x4*)(xa + 16 * I * kMmaRow + 16 * j);
                const i32x4 fb = *(const i32x4*)(ya + 16 * J * kMmaRow + 16 * j);
                acc[k] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa, fb, acc[k], 0, 0, 0);
            }
        });
    });
}

// wave W's tile sums added into the diagonal sums dsum[g], g < S
template <int NT, int W>
__device__ __forceinline__ void mma_fold(const i32x4 (&acc)[MmaTiles<NT>::SLOTS], int64_t* dsum, int S, int lane)
{
    constexpr MmaTiles<NT> kT{};
    const int g0 = 4 * (lane >> 4) + (lane & 15);
    unroll<MmaTiles<NT>::SLOTS>([&](auto KK) {
        constexpr int k = decltype(KK)::value, I = kT.I[2 * k + W], J = kT.J[2 * k + W];
        if constexpr (I >= 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int g = 16 * (I + J) + g0 + r;
                if (g < S)
                    atomicAdd(reinterpret_cast<unsigned long long*>(dsum + g),
                              (unsigned long long)(int64_t)acc[k][r]);
            }
        }
    });
}

template <int MW, int SC, bool BAL>
__global__ __launch_bounds__(128) void k_dot_mma(LaneDotArgs a)
{
    static_assert(SC % 16 == 0 && SC >= 16 && SC <= 128, "whole tiles; one thread per diagonal");
    constexpr int NT = SC / 16;
    constexpr int SLOTS = MmaTiles<NT>::SLOTS;
    constexpr int NS = store_limbs<SC, BAL>();
    // a wave's limb store inside its operand's digit rows where it fits
    // (decided at compile time: the balanced containers of 32 digits or more,
    // the sign-magnitude ones of 64 or more), else beside them
    constexpr bool kInRows = NS * 64 * 2 <= SC * kMmaRow;
    __shared__ __attribute__((aligned(16))) uint32_t dig[2][SC][kMmaRow];
    __shared__ uint64_t beside[2][kInRows ? 1 : NS][kInRows ? 1 : 64];
    __shared__ uint32_t magw[2][64];
    __shared__ int32_t xch[16];
    __shared__ int64_t dsum[SC];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t b = a.b0 + blockIdx.x;
    const int64_t c0 = (int64_t)blockIdx.y * a.chunk;
    const int64_t c1 = c0 + a.chunk < a.n ? c0 + a.chunk : a.n;
    const double* xb = a.X + b * a.ldx;
    const double* yb = a.Y + b * a.ldy;
    if (t < SC)
        dsum[t] = 0;

    int Ex, Ey;
    if (a.full) {
        int h[4];
        pair_exponents(xb, yb, a.n, h, xch);
        Ex = (h[0] == INT_MIN ? 0 : h[0]) + a.eoff;
        Ey = (h[2] == INT_MIN ? 0 : h[2]) + a.eoff;
        if (t == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                a.ph[i * a.batch + b] = h[i];
        }
    } else {
        Ex = a.E[b];
        Ey = a.F[b];
    }

    constexpr int bits = BAL ? 8 : 7;
    const int S = a.S;
    // this wave's operand: x for wave 0, y for wave 1
    const int Eo = wave == 0 ? Ex : Ey;
    const int kn = Eo + 1075 - bits * S;
    const int pad = bits * (SC - S);
    const int Er = Eo - a.eoff;
    const bool mag = a.mag != 0;
    const int64_t ps = wave == 0 ? a.psx : a.psy;

    // the wave's limb store inside its operand's digit rows: its limbs are
    // zero again once the round's entries are cut, the digit words then
    // overwrite them, and the next round clears them first
    LdsLimbs L{kInRows ? reinterpret_cast<uint64_t*>(&dig[wave][0][0]) + lane : &beside[wave][0][0] + lane};
    i32x4 acc[SLOTS];
#pragma unroll
    for (int k = 0; k < SLOTS; ++k)
        acc[k] = i32x4{0, 0, 0, 0};
    uint32_t macc = 0;

    const int64_t nrounds = (c1 - c0 + kMmaRound - 1) / kMmaRound;
    const int64_t off = c0 + lane;
    const int64_t lim = c1 - off;
    const int64_t elast = c1 - 1 - off;
    const double* p = (wave == 0 ? xb : yb) + off;
    // the next NB entries' words in flight (entry g of the lane's sequence:
    // byte g % 2 of round g / 2, in buffer g % NB)
    constexpr int NB = MW <= 4 ? 2 : 1;
    double bw[NB][MW];
#pragma unroll
    for (int g = 0; g < NB; ++g)
        lane_load(bw[g], p, ps, (int64_t)(g / 2) * kMmaRound + 64 * (g % 2), lim, elast);

    // this lane's fragment words in the first row of each operand's digits,
    // and where its two digit bytes go: half lane / 32 of word lane % 32
    const uint32_t* xa = &dig[0][lane & 15][4 * (lane >> 4)];
    const uint32_t* ya = &dig[1][lane & 15][4 * (lane >> 4)];
    uint16_t* own = reinterpret_cast<uint16_t*>(&dig[wave][0][lane & 31]) + (lane >> 5);
    uint16_t* ownm = reinterpret_cast<uint16_t*>(&magw[wave][lane & 31]) + (lane >> 5);
    for (int64_t it = 0; it < nrounds; ++it) {
#pragma unroll
        for (int i = 0; i < NS; ++i)
            L.col[i * 64] = 0;
        uint32_t xs[SC], mx = 0;
#pragma unroll
        for (int s = 0; s < SC; ++s)
            xs[s] = 0;
        const int64_t e0 = it * kMmaRound;
        unroll<2>([&](auto QQ) {
            constexpr int q = decltype(QQ)::value, slot = q % NB;
            const int64_t en = e0 + ((q + NB) / 2) * kMmaRound + 64 * ((q + NB) % 2);
            if (mag)
                mx = byte_insert<q, 0>(mx, mag_digit(bw[slot][0], Er));
            lane_digits<q, MW, SC, BAL>(bw[slot], kn, pad, xs, L);
            pin(xs, mx);
            lane_load(bw[slot], p, ps, en, lim, elast);
        });
#pragma unroll
        for (int s = 0; s < SC; ++s)
            own[2 * s * kMmaRow] = (uint16_t)(BAL ? xs[s] ^ 0x8080u : xs[s]);
        *ownm = (uint16_t)mx;
        __syncthreads();
        if (mag && wave == 0 && lane < 32)
            macc = __builtin_amdgcn_udot4(magw[0][lane], magw[1][lane], macc, false);
        if (wave == 0)
            mma_round<NT, 0>(acc, xa, ya);
        else
            mma_round<NT, 1>(acc, xa, ya);
        __syncthreads();
    }

    // tile (I, J): lane L holds rows 16 I + 4 (L / 16) + r, column 16 J + L % 16,
    // on diagonal 16 (I + J) + 4 (L / 16) + r + L % 16; sums of one
    // diagonal meet in int64 by LDS atomics
    if (wave == 0)
        mma_fold<NT, 0>(acc, dsum, S, lane);
    else
        mma_fold<NT, 1>(acc, dsum, S, lane);
    __syncthreads();
    if (a.atomic) {
        if (t < S)
            atomicAdd(reinterpret_cast<unsigned long long*>(a.D + (int64_t)t * a.batch + b),
                      (unsigned long long)dsum[t]);
    } else if (t == 0) {
        lane_round<SC, bits>(dsum, Ex + Ey - bits * (SC + 1), MW, a.out + b, a.pso);
    }
    if (mag && wave == 0) {
        unsigned long long mm = macc;
        for (int o = 1; o < 64; o <<= 1)
            mm += __shfl_xor(mm, o);
        if (lane == 0)
            a.pm[b] = mm;
    }
}

// SC in [LO, HI], a multiple of 16
template <int MW, int HI, int LO>
struct DispatchMma {
    static hipError_t run(const LaneDotArgs& a0, int SC, bool bal, int64_t nch, hipStream_t st)
    {
        if (SC == HI) {
            LaneDotArgs a = a0;
            for (int64_t b0 = 0; b0 < a.batch; b0 += INT64_C(1) << 30) {
                a.b0 = b0;
                const dim3 grid((unsigned)std::min<int64_t>(a.batch - b0, INT64_C(1) << 30), (unsigned)nch);
                if (bal)
                    hipLaunchKernelGGL((k_dot_mma<MW, HI, true>), grid, dim3(128), 0, st, a);
                else
                    hipLaunchKernelGGL((k_dot_mma<MW, HI, false>), grid, dim3(128), 0, st, a);
                const hipError_t e = hipGetLastError();
                if (e != hipSuccess)
                    return e;
            }
            return hipSuccess;
        }
        if constexpr (HI - 16 >= LO)
            return DispatchMma<MW, HI - 16, LO>::run(a0, SC, bal, nch, st);
        return hipErrorInvalidValue;
    }
};

}  // namespace
}  // namespace mdg
