// The INT8 slice contraction for 33 to 64 slices in two bands of G = S/2
// diagonals, each over the whole depth with compile-time bit positions, so
// that the exact fold stays in registers and no diagonal sum leaves the
// kernel (instantiated over S by duo_*.hip).
//
//   band 1: diagonals t = 0 .. G-1, the triangle of slices 0 .. G-1 (the
//           whole-triangle kernel's loop with the chunk stride of S slices);
//   band 2: diagonals t = G .. 2G-1, a parallelogram over all S slices.
//
// Per depth chunk a wave (two row blocks, one column block) loads 3 G
// fragments for band 1 and 3 S for band 2 (9 G in all, against 12 G + ...
// for bands of at most 16 diagonals that each re-stream the slices below
// them), and issues S (S+1) matrix instructions.  Band 1's fold columns wait
// in LDS while band 2 runs.
#pragma once

#include "tri.h"

#include <utility>

namespace mdg {
namespace {

// Work of band 2's step s (R row blocks): all G diagonals while s <= G,
// then 2G - s; s in [2G, 2G+2) are the next chunk's steps 0 and 1.
constexpr int par_work(int G, int R, int s)
{
    const int q = s >= 2 * G ? s - 2 * G : s;
    return R * (q <= G ? G : 2 * G - q);
}

// Step at which the fragments of step q are issued: the latest one that
// leaves at least LA matrix instructions before step q (-1: before the
// chunk; q = 2G, 2G+1: the next chunk's steps 0 and 1).
constexpr int par_issue(int G, int R, int LA, int q)
{
    int w = 0;
    for (int l = q - 1; l >= 0; --l) {
        w += par_work(G, R, l);
        if (w >= LA)
            return l < 2 * G ? l : 2 * G - 1;
    }
    return q < 2 * G ? -1 : 0;
}

// Band 2 over the depth chunks [c0, c1): diagonals t = G + g, g = 0..G-1.
// Step s multiplies A_s of every row block with B_u, u = G + g - s, for
// every g with 0 <= u <= 2G-1 (all g while s <= G, g >= s - G after).  The
// window slot of B_u is u mod G: at chunk start it holds B_G .. B_{2G-1};
// B_{G-s} enters at step s (1 <= s <= G) into the slot B_{2G-s} left after
// step s-1; from step G+1 on, the slot of B_{2G-s} (last read at step s-1)
// takes the next chunk's B_{3G-s}, and slot 0 the next chunk's B_G after the
// last step.  A_s and the entering B_{G-s} are loaded together, LA matrix
// instructions ahead (par_issue).  Fragment (kc, s) of a stream is at byte
// (kc 2G + s) 1024.  The steps are template instances, so every schedule
// decision and every register index is a compile-time constant.
template <int G, int R, int LA>
struct Par {
    static constexpr int S = 2 * G;
    static constexpr uint32_t F = 1024, CS = (uint32_t)S * F;
    struct Sched {
        int issue[2 * G + 2];
    };
    static constexpr Sched make()
    {
        Sched x{};
        for (int q = 0; q < S + 2; ++q)
            x.issue[q] = par_issue(G, R, LA, q);
        return x;
    }
    static constexpr Sched kSched = make();

    struct State {
        v4i win[G], ar[R][S + 2], bn[S + 2];
    };

    // fragments of step q (this chunk's for q < S, the next chunk's steps
    // 0 and 1 for q = S, S+1)
    template <int Q>
    static __device__ __forceinline__ void load_step(State& z, const FragStream (&LDA)[R],
                                                     const FragStream& LDB, uint32_t ck, uint32_t cn)
    {
#pragma unroll
        for (int r = 0; r < R; ++r)
            z.ar[r][Q] = Q < S ? LDA[r](ck + Q * F) : LDA[r](cn + (Q - S) * F);
        if constexpr (Q >= 1 && Q <= G)
            z.bn[Q] = LDB(ck + (G - Q) * F);
        if constexpr (Q == S + 1)
            z.bn[Q] = LDB(cn + (G - 1) * F);
    }

    // the loads scheduled at step P, positions Q .. S+1
    template <int P, int Q>
    static __device__ __forceinline__ void issue(State& z, const FragStream (&LDA)[R],
                                                 const FragStream& LDB, uint32_t ck, uint32_t cn)
    {
        if constexpr (Q < S + 2) {
            if constexpr (kSched.issue[Q] == P)
                load_step<Q>(z, LDA, LDB, ck, cn);
            issue<P, Q + 1>(z, LDA, LDB, ck, cn);
        }
    }

    // positions with no issue step: loaded before a chunk (prologue: from
    // 0; between chunks: from 2, as 0 and 1 were issued in the chunk before)
    template <int Q>
    static __device__ __forceinline__ void preload(State& z, const FragStream (&LDA)[R],
                                                   const FragStream& LDB, uint32_t ck)
    {
        if constexpr (Q < S) {
            if constexpr (kSched.issue[Q] < 0)
                load_step<Q>(z, LDA, LDB, ck, ck);
            preload<Q + 1>(z, LDA, LDB, ck);
        }
    }

    template <int P>
    static __device__ __forceinline__ void step(v4i (&acc)[R][G], State& z, const FragStream (&LDA)[R],
                                                const FragStream& LDB, uint32_t ck, uint32_t cn)
    {
        issue<P, P + 1>(z, LDA, LDB, ck, cn);
        if constexpr (P >= 1 && P <= G)
            z.win[(G - P) % G] = z.bn[P];
        if constexpr (P > G)
            z.win[S - P] = LDB(cn + (3 * G - P) * F);
        __builtin_amdgcn_sched_barrier(0);
        constexpr int g0 = P > G ? P - G : 0;
#pragma unroll
        for (int g = G - 1; g >= g0; --g)
#pragma unroll
            for (int r = 0; r < R; ++r)
                acc[r][g] = FormI8::mma(z.ar[r][P], z.win[(G + g - P) % G], acc[r][g]);
        __builtin_amdgcn_sched_barrier(0);
    }

    template <int... P>
    static __device__ __forceinline__ void chunk(v4i (&acc)[R][G], State& z, const FragStream (&LDA)[R],
                                                 const FragStream& LDB, uint32_t ck, uint32_t cn,
                                                 std::integer_sequence<int, P...>)
    {
        (step<P>(acc, z, LDA, LDB, ck, cn), ...);
    }

    static __device__ __forceinline__ void run(v4i (&acc)[R][G], const FragStream (&LDA)[R],
                                               const FragStream& LDB, int64_t c0, int64_t c1)
    {
        State z;
        uint32_t ck = (uint32_t)c0 * CS;
#pragma unroll
        for (int v = G - 1; v >= 0; --v)
            z.win[v] = LDB(ck + (G + v) * F);
        preload<0>(z, LDA, LDB, ck);
        for (int64_t kc = c0; kc < c1; ++kc) {
            const uint32_t cn = kc + 1 < c1 ? ck + CS : ck;
            chunk(acc, z, LDA, LDB, ck, cn, std::make_integer_sequence<int, S>{});
            z.win[0] = LDB(cn + G * F);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                z.ar[r][0] = z.ar[r][S];
                z.ar[r][1] = z.ar[r][S + 1];
            }
            z.bn[1] = z.bn[S + 1];
            preload<2>(z, LDA, LDB, cn);
            ck = cn;
        }
    }
};

// Fold columns of one band: diagonal t = t0 + g lands at bit B e,
// e = S-1-t, i.e. column e / 4 shifted by B (e mod 4); this band's columns
// start at J0 = e_min / 4 (NC of them, the last one for carries only).
template <int S, int B, int G, int T0>
struct DuoBand {
    static constexpr int kEmin = S - T0 - G, kEmax = S - 1 - T0;
    static constexpr int kJ0 = kEmin / 4;
    static constexpr int kNC = kEmax / 4 - kJ0 + 2;
};

template <int S, int B, int G, int T0>
__device__ __forceinline__ void duo_fold(const v4i (&acc)[2][G], int64_t (&x)[8][DuoBand<S, B, G, T0>::kNC])
{
    typedef DuoBand<S, B, G, T0> D;
#pragma unroll
    for (int n = 0; n < 8; ++n)
#pragma unroll
        for (int c = 0; c < D::kNC; ++c)
            x[n][c] = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int e = S - 1 - T0 - g;
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int o = 0; o < 4; ++o)
                x[4 * r + o][(e >> 2) - D::kJ0] += (int64_t)acc[r][g][o] * ((int64_t)1 << (B * (e & 3)));
    }
#pragma unroll
    for (int n = 0; n < 8; ++n)
        carry_cols<4 * B>(x[n]);
}

// Two bands of G = S/2 diagonals, two row blocks per wave (64 x 32
// workgroup tile), the whole depth one exactness chunk; B-bit digits.
// Band 1's carried columns (each below 2^(4B) but the signed top one, so
// 32 bits hold them) wait in LDS, one 256-byte row of lanes per column and
// output, while band 2 runs.
template <int S, int B>
__global__ __launch_bounds__(256, 1) void k_duo_i8(GemmArgs a)
{
    constexpr int G = S / 2;
    static_assert(S % 2 == 0 && G > 16 && G <= 32, "two bands of 17 to 32 diagonals");
    typedef DuoBand<S, B, G, 0> D1;
    typedef DuoBand<S, B, G, G> D2;
    constexpr int NC = Tri<S, B>::kCols;
    static_assert(D1::kJ0 + D1::kNC <= NC && D2::kJ0 == 0 && D2::kNC <= NC, "fold columns");
    __shared__ int32_t park[4 * D1::kNC * 8 * 64];
    const WaveTile w(a, 2);
    const uint64_t bytes = (uint64_t)a.nkc * S * 1024;
    const int64_t nrb = 2 * ((a.M + kTile - 1) / kTile);
    FragStream LA[2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
        LA[r] = frag_stream((const char*)a.A + (w.rb + r) * bytes, w.rb + r < nrb ? bytes : 0,
                            w.lane);
    const FragStream LB = frag_stream((const char*)a.B + w.cb * bytes, bytes, w.lane);
    int32_t* mine = park + w.wave * (D1::kNC * 8 * 64) + w.lane;
    v4i acc[2][G];
    {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int g = 0; g < G; ++g)
                acc[r][g] = FormI8::zero();
        tri_run_i8<G, 2, kLeadA, S>(acc, LA, LB, 0, a.nkc);
        int64_t x1[8][D1::kNC];
        duo_fold<S, B, G, 0>(acc, x1);
#pragma unroll
        for (int n = 0; n < 8; ++n)
#pragma unroll
            for (int c = 0; c < D1::kNC; ++c)
                mine[(c * 8 + n) * 64] = (int32_t)x1[n][c];
    }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int g = 0; g < G; ++g)
            acc[r][g] = FormI8::zero();
    Par<G, 2, kLeadA>::run(acc, LA, LB, 0, a.nkc);
    int64_t x2[8][D2::kNC];
    duo_fold<S, B, G, G>(acc, x2);
    int64_t x[8][NC];
#pragma unroll
    for (int n = 0; n < 8; ++n)
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            int64_t v = j < D2::kNC ? x2[n][j] : 0;
            const int c = j - D1::kJ0;
            if (c >= 0 && c < D1::kNC) {
                const int32_t p = mine[(c * 8 + n) * 64];
                // the band's top column is signed, the others are 4B-bit
                // magnitudes
                v += c == D1::kNC - 1 ? (int64_t)p : (int64_t)(uint32_t)p;
            }
            x[n][j] = v;
        }
#pragma unroll
    for (int n = 0; n < 8; ++n)
        carry_cols<Tri<S, B>::kCW>(x[n]);
    // the register file is full here: the outputs' rounding steps
    // interleave in groups of four (balanced digits) or two, so that the
    // remainders' fixed-place alignment fits without spilling
    tri_outputs<S, 2, B, false, true, B == 8 ? 4 : 2>(x, a, w.rb, w.cb, w.lane);
}

// Launch the two-band kernel for a.S in {LO, LO+4, ..., S}, B-bit digits.
template <int S, int LO, int B>
struct DispatchDuoRange {
    static hipError_t run(const GemmArgs& a, hipStream_t st)
    {
        if (a.S == S)
            return launch_kernel(k_duo_i8<S, B>, a, st, false, 2 * kTile);
        if constexpr (S - 4 >= LO)
            return DispatchDuoRange<S - 4, LO, B>::run(a, st);
        return hipErrorInvalidValue;
    }
};

}  // namespace
}  // namespace mdg
