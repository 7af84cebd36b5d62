// The whole-triangle INT8 slice contraction (S <= 32 diagonals at once) with
// its register fold and renormalisation: kernel templates, instantiated over
// ranges of S by tri_*.hip so that the compiles run in parallel.
#pragma once

#include "slice_common.h"

namespace mdg {
namespace {

// Whole triangle of one depth-chunk run [c0, c1): all S diagonals at once
// (INT8, S <= 32), for R row blocks of op(A) against one column block of
// op(B).  The window holds B_0 .. B_{S-1} of the chunk; step p multiplies
// A_p of every row block with B_{g-p} into diagonal g for g >= p (g
// descending), so B_{S-p} is read for the last time at step p-1 and its slot
// takes the next chunk's B_{S-p} at step p (B_0 after the last step).
// Fragment (kc, s) of a stream is at byte (kc S + s) 1024.
//
// Step p carries R (S - p) matrix instructions, so A loads are scheduled by
// work, not by steps: A_q is issued at the latest step that leaves at least
// LA instructions before its use (tri_issue_a); the next chunk's first A
// fragments are issued inside this chunk.
constexpr int tri_work(int S, int R, int p) { return R * (p < S ? S - p : S - (p - S)); }

// Step (0 .. S-1 of this chunk) at which A of position q is issued, where
// q = 0 .. S-1 are this chunk's steps and q = S .. S+1 the next chunk's
// steps 0 and 1; -1: issued before the chunk starts (prologue or the end of
// the previous chunk; only for q < S).
constexpr int tri_issue_a(int S, int R, int LA, int q)
{
    int w = 0;
    for (int l = q - 1; l >= 0; --l) {
        w += tri_work(S, R, l);
        if (w >= LA)
            return l < S ? l : S - 1;
    }
    return q < S ? -1 : 0;   // the next chunk's A cannot precede this chunk
}

// SS: slices per depth chunk in memory (S when the triangle is the whole
// contraction; more when it is the first band of a longer split).
template <int S, int R, int LA, int SS = S>
__device__ __forceinline__ void tri_run_i8(v4i (&acc)[R][S], const FragStream (&LDA)[R],
                                           const FragStream& LDB, int64_t c0, int64_t c1)
{
    constexpr uint32_t F = 1024, CS = (uint32_t)SS * F;
    uint32_t ck = (uint32_t)c0 * CS;
    v4i win[S], ar[R][S + 2];
#pragma unroll
    for (int g = S - 1; g >= 0; --g)
        win[g] = LDB(ck + g * F);
    // A of this first chunk issued "before" it: positions with no issue step
#pragma unroll
    for (int q = 0; q < S; ++q)
        if (tri_issue_a(S, R, LA, q) < 0)
#pragma unroll
            for (int r = 0; r < R; ++r)
                ar[r][q] = LDA[r](ck + q * F);
    for (int64_t kc = c0; kc < c1; ++kc) {
        const uint32_t cn = kc + 1 < c1 ? ck + CS : ck;
#pragma unroll
        for (int p = 0; p < S; ++p) {
            // issue the loads scheduled at this step
#pragma unroll
            for (int q = p + 1; q < S + 2; ++q)
                if (tri_issue_a(S, R, LA, q) == p)
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        ar[r][q] = q < S ? LDA[r](ck + q * F) : LDA[r](cn + (q - S) * F);
            if (p >= 1)
                win[S - p] = LDB(cn + (S - p) * F);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int g = S - 1; g >= p; --g)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    acc[r][g] = FormI8::mma(ar[r][p], win[g - p], acc[r][g]);
            __builtin_amdgcn_sched_barrier(0);
        }
        win[0] = LDB(cn);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            ar[r][0] = ar[r][S];
            ar[r][1] = ar[r][S + 1];
        }
#pragma unroll
        for (int q = 2; q < S; ++q)
            if (tri_issue_a(S, R, LA, q) < 0)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    ar[r][q] = LDA[r](cn + q * F);
        ck = cn;
    }
}

// Register-resident fold of the whole-triangle kernel for digits of B bits
// (7: sign-magnitude, 8: balanced).  The band starts at t = 0, so diagonal
// t lands at bit B e, e = S-1-t, which is column e / 4 (weight
// 2^(4 B (e / 4))) shifted left by the static amount B (e mod 4).  One depth
// chunk adds less than 2^31 (1 + 2^B + 2^2B + 2^3B) < 2^56 to a column;
// after every chunk the columns are carried back to 4 B bits.  The top
// column takes only carries and is the signed one.  x[4 r + o] holds output
// o of the lane in row block rb0 + r.
template <int S, int R, bool DBG, int B>
__device__ __forceinline__ void tri_fold(const v4i (&acc)[R][S], int64_t (&x)[4 * R][Tri<S, B>::kCols],
                                         const GemmArgs& a, int64_t rb0, int64_t cb, int lane)
{
#pragma unroll
    for (int g = 0; g < S; ++g) {
        const int e = S - 1 - g;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                x[4 * r + o][e >> 2] += (int64_t)acc[r][g][o] * ((int64_t)1 << (B * (e & 3)));
                if constexpr (DBG) {
                    const int64_t i = (rb0 + r) * 16 + FormI8::row(lane, o), j = cb * 16 + (lane & 15);
                    if (i < a.M && j < a.N)
                        a.dbgD[((int64_t)g * a.M + i) * a.N + j] += acc[r][g][o];
                }
            }
    }
#pragma unroll
    for (int n = 0; n < 4 * R; ++n)
        carry_cols<Tri<S, B>::kCW>(x[n]);
}

// Greedy renormalisation of the lane's 4 R outputs, their steps interleaved.
// FIX: instead, the exact integers as two's complement limb planes
// (a.fixX[k * M N + i N + j], limbs past the register ones filled with the
// sign) and their scales (a.fixScale[i N + j]).  FAST: rn_next's fixed-place
// alignment of the remainders (off where the kernel has no registers left).
// G: outputs whose steps interleave (groups of G one after the other).
template <int S, int R, int B, bool FIX = false, bool FAST = true, int G = 4 * R>
__device__ __forceinline__ void tri_outputs(int64_t (&x)[4 * R][(Tri<S, B>::kCols)], const GemmArgs& a,
                                            int64_t rb0, int64_t cb, int lane)
{
    constexpr int NL = Tri<S, B>::kLimbs, NO = 4 * R;
    uint32_t L[NO][NL];
    double sgn[NO], *out[NO];
    int scale[NO];
    bool ok[NO];
#pragma unroll
    for (int n = 0; n < NO; ++n) {
        const int64_t i = (rb0 + n / 4) * 16 + FormI8::row(lane, n % 4), j = cb * 16 + (lane & 15);
        ok[n] = i < a.M && j < a.N;
        scale[n] = ok[n] ? a.E[i] + a.F[j] - B * (S + 1) : 0;
        out[n] = a.C + (ok[n] ? i * a.ldc + j : 0);
        sgn[n] = to_limbs<Tri<S, B>::kCW>(x[n], L[n]) ? -1.0 : 1.0;
    }
    if constexpr (FIX) {
        const int64_t count = a.M * a.N;
#pragma unroll
        for (int n = 0; n < NO; ++n) {
            const int64_t e = ((rb0 + n / 4) * 16 + FormI8::row(lane, n % 4)) * a.N + cb * 16 + (lane & 15);
            const bool neg = sgn[n] < 0.0;
            uint64_t cy = 1;
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const uint64_t v = (uint64_t)(~L[n][k]) + cy;
                cy = v >> 32;
                L[n][k] = neg ? (uint32_t)v : L[n][k];
            }
            if (!ok[n])
                continue;
            for (int k = 0; k < a.fixNL; ++k) {
                uint32_t v = neg ? 0xffffffffu : 0u;
#pragma unroll
                for (int q = 0; q < NL; ++q)
                    v = q == k ? L[n][q] : v;
                a.fixX[(int64_t)k * count + e] = (int32_t)v;
            }
            a.fixScale[e] = scale[n];
        }
        return;
    }
    static_assert(NO % G == 0, "whole groups of outputs");
#pragma unroll
    for (int g0 = 0; g0 < NO; g0 += G)
        for (int t = 0; t < a.m; ++t) {
#pragma unroll
            for (int n = g0; n < g0 + G; ++n) {
                const double wv = rn_next<NL, FAST>(L[n], sgn[n], scale[n]);
                if (ok[n])
                    out[n][t * a.psc] = wv;
            }
        }
}

// Load lead of the triangle kernels' A fragments, in matrix instructions.
constexpr int kLeadA = 48;

// Whole-triangle INT8 contraction, S <= 32 diagonals in one band, one row
// block per wave (32 x 32 workgroup tile), any number of exactness chunks;
// B-bit digits.
template <int S, bool DBG, int B>
__global__ __launch_bounds__(256, 1) void k_tri_i8(GemmArgs a)
{
    const WaveTile w(a, 1);
    const uint64_t bytes = (uint64_t)a.nkc * S * 1024;   // one row block of fragments
    const FragStream LA[1] = {frag_stream((const char*)a.A + w.rb * bytes, bytes, w.lane)};
    const FragStream LB = frag_stream((const char*)a.B + w.cb * bytes, bytes, w.lane);
    int64_t x[4][Tri<S, B>::kCols];
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
        for (int j = 0; j < Tri<S, B>::kCols; ++j)
            x[o][j] = 0;
    for (int64_t c0 = 0; c0 < a.nkc; c0 += a.kcc) {
        v4i acc[1][S];
#pragma unroll
        for (int g = 0; g < S; ++g)
            acc[0][g] = FormI8::zero();
        tri_run_i8<S, 1, kLeadA>(acc, LA, LB, c0, min(c0 + a.kcc, a.nkc));
        tri_fold<S, 1, DBG, B>(acc, x, a, w.rb, w.cb, w.lane);
    }
    tri_outputs<S, 1, B>(x, a, w.rb, w.cb, w.lane);
}

// The same with two row blocks per wave (64 x 32 workgroup tile), which
// share the B window: half the B loads per matrix instruction.  The whole
// depth is one exactness chunk, so the fold columns exist only after the
// contraction.  A row block past the digit array (M padded to 32 rows) reads
// through an empty descriptor: zeros.
template <int S, int B>
__global__ __launch_bounds__(256, 1) void k_tri2_i8(GemmArgs a)
{
    const WaveTile w(a, 2);
    const uint64_t bytes = (uint64_t)a.nkc * S * 1024;
    const int64_t nrb = 2 * ((a.M + kTile - 1) / kTile);
    FragStream LA[2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
        LA[r] = frag_stream((const char*)a.A + (w.rb + r) * bytes, w.rb + r < nrb ? bytes : 0,
                            w.lane);
    const FragStream LB = frag_stream((const char*)a.B + w.cb * bytes, bytes, w.lane);
    v4i acc[2][S];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int g = 0; g < S; ++g)
            acc[r][g] = FormI8::zero();
    tri_run_i8<S, 2, kLeadA>(acc, LA, LB, 0, a.nkc);
    int64_t x[8][Tri<S, B>::kCols];
#pragma unroll
    for (int n = 0; n < 8; ++n)
#pragma unroll
        for (int j = 0; j < Tri<S, B>::kCols; ++j)
            x[n][j] = 0;
    tri_fold<S, 2, false, B>(acc, x, a, w.rb, w.cb, w.lane);
    tri_outputs<S, 2, B>(x, a, w.rb, w.cb, w.lane);
}

// The same contraction returning the exact integers (a.fixX, a.fixScale)
// instead of rounded words.  (Its own copy of the body: the rounding
// kernel's code stays exactly as it is tuned.)
template <int S, int B>
__global__ __launch_bounds__(256, 1) void k_tri2_i8_fixed(GemmArgs a)
{
    const WaveTile w(a, 2);
    const uint64_t bytes = (uint64_t)a.nkc * S * 1024;
    const int64_t nrb = 2 * ((a.M + kTile - 1) / kTile);
    FragStream LA[2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
        LA[r] = frag_stream((const char*)a.A + (w.rb + r) * bytes, w.rb + r < nrb ? bytes : 0,
                            w.lane);
    const FragStream LB = frag_stream((const char*)a.B + w.cb * bytes, bytes, w.lane);
    v4i acc[2][S];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int g = 0; g < S; ++g)
            acc[r][g] = FormI8::zero();
    tri_run_i8<S, 2, kLeadA>(acc, LA, LB, 0, a.nkc);
    int64_t x[8][Tri<S, B>::kCols];
#pragma unroll
    for (int n = 0; n < 8; ++n)
#pragma unroll
        for (int j = 0; j < Tri<S, B>::kCols; ++j)
            x[n][j] = 0;
    tri_fold<S, 2, false, B>(acc, x, a, w.rb, w.cb, w.lane);
    tri_outputs<S, 2, B, true>(x, a, w.rb, w.cb, w.lane);
}

// Launch the triangle kernel for a.S in [LO, S], B-bit digits: two row
// blocks per wave when the whole depth is one exactness chunk (and no debug
// dump is asked for), else one.
template <int S, int LO, int B>
struct DispatchTriRange {
    static hipError_t run(const GemmArgs& a, hipStream_t st)
    {
        if (a.S == S) {
            if (a.kcc >= a.nkc && !a.dbgD)
                return launch_kernel(k_tri2_i8<S, B>, a, st, false, 2 * kTile);
            return a.dbgD ? launch_kernel(k_tri_i8<S, true, B>, a, st, false)
                          : launch_kernel(k_tri_i8<S, false, B>, a, st, false);
        }
        if constexpr (S > LO)
            return DispatchTriRange<S - 1, LO, B>::run(a, st);
        return hipErrorInvalidValue;
    }
};

// The fixed-point variant for a.S in [LO, S]: the whole depth must be one
// exactness chunk.
template <int S, int LO, int B>
struct DispatchTriFixRange {
    static hipError_t run(const GemmArgs& a, hipStream_t st)
    {
        if (a.kcc < a.nkc || !a.fixX || !a.fixScale)
            return hipErrorInvalidValue;
        if (a.S == S)
            return launch_kernel(k_tri2_i8_fixed<S, B>, a, st, false, 2 * kTile);
        if constexpr (S > LO)
            return DispatchTriFixRange<S - 1, LO, B>::run(a, st);
        return hipErrorInvalidValue;
    }
};

}  // namespace
}  // namespace mdg
