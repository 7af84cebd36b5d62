// The whole-triangle INT8 slice contraction with the workgroup's fragments
// staged in LDS: each digit fragment crosses the texture path once per
// workgroup instead of once per wave that reads it.
//
// The workgroup (4 waves, 64 x 32 outputs: row blocks 0..3, column blocks
// 0..1) walks the depth chunks step by step as the register version does
// (step p of chunk c multiplies A_p with the window B_0 .. B_{S-1-p}).  The
// steps are grouped in stages of BS (BS divides S).  A record holds what one
// step needs from memory: A_p of the 4 row blocks and the next chunk's
// B_{S-1-p} of the 2 column blocks (the window slot that step p reads for
// the last time), 6 fragments of 1 KB.  Three LDS slots of BS records
// rotate.  Stage j's global loads are issued into registers at the start of
// stage j-4 (three register buffers rotate), written to its LDS slot at the
// start of stage j-2, and read in stage j (its first step's A operands
// already at the end of stage j-1).  The stages per chunk are a multiple of
// 3, so every slot and buffer index is fixed by the stage's place in the
// chunk.  A barrier starts every stage; before it
// each wave waits only for its own LDS writes (LDS operations complete in
// order), so the reads issued after them stay in flight.  Wave w loads A of
// row block w for every record and B of its own column block for every
// other record.
#pragma once

#include "tri.h"

#include <utility>

namespace mdg {
namespace {

// s_waitcnt with vmcnt and expcnt left at their maxima and lgkmcnt = n
// (gfx9 encoding: vmcnt [3:0] and [15:14], expcnt [6:4], lgkmcnt [11:8])
template <int N>
__device__ __forceinline__ void wait_lgkm()
{
    static_assert(N >= 0 && N < 16, "lgkmcnt field");
    __builtin_amdgcn_s_waitcnt((0x3 << 14) | (N << 8) | (0x7 << 4) | 0xf);
}

// workgroup barrier that orders the compiler's memory operations too
__device__ __forceinline__ void stage_barrier()
{
    asm volatile("s_barrier" ::: "memory");
}

template <int S, int BS>
struct TriL {
    static_assert(S % BS == 0, "stages of whole steps");
    static constexpr int NST = S / BS;          // stages per chunk
    static_assert(NST % 3 == 0, "slot and register buffer of a stage fixed by its place in the chunk");
    static_assert((S - 1) % 3 != 0, "A operand buffers of the last step and the next chunk's first differ");
    static constexpr uint32_t F = 1024, REC = 6 * F, SLOT = BS * REC;
    static constexpr uint32_t CS = (uint32_t)S * F;
    static constexpr int NB = (BS + 1) / 2;     // B loads per wave and stage, at most

    struct Staged {
        v4i a[BS];        // A (row block w) of a stage's records
        v4i b[NB];        // B (own column block) of records half, half+2, ..
    };
    struct State {
        v4i win[S];       // the B window
        Staged st[3];     // stages in flight from memory, by stage mod 3
        v4i ar[3][2];     // A operands, by step mod 3
    };
    // this wave's places in a record (byte offsets, lane included)
    struct Lanes {
        uint32_t wr_a, wr_b, rd_a, rd_b;
        int half;
    };

    // global loads of stage H of chunk c (H may run past the chunk: the next
    // chunk's stages): A of every record, B of the records of this half
    template <int H>
    static __device__ __forceinline__ void load_stage(Staged& z, const FragStream& LAL, const FragStream& LBL,
                                                      uint32_t c, int half)
    {
        const uint32_t cc = c + H / NST;
        constexpr uint32_t p0 = (H % NST) * BS;
#pragma unroll
        for (int r = 0; r < BS; ++r)
            z.a[r] = LAL(cc * CS + (p0 + r) * F);
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int r = 2 * q + half;
            if (r < BS)
                z.b[q] = LBL((cc + 1) * CS + (S - 1 - (p0 + r)) * F);
        }
    }

    // the staged fragments of stage H into its LDS slot (H mod 3)
    template <int H>
    static __device__ __forceinline__ void write_stage(const Staged& z, char* lds, const Lanes& ln)
    {
        char* slot = lds + (H % 3) * SLOT;
#pragma unroll
        for (int r = 0; r < BS; ++r)
            *(v4i*)(slot + r * REC + ln.wr_a) = z.a[r];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int r = 2 * q + ln.half;
            if (r < BS)
                *(v4i*)(slot + r * REC + ln.wr_b) = z.b[q];
        }
    }

    // the A operands of record R of stage H into ar[Q]
    template <int H, int R, int Q>
    static __device__ __forceinline__ void read_a(State& z, const char* lds, const Lanes& ln)
    {
        const char* rec = lds + (H % 3) * SLOT + R * REC + ln.rd_a;
        z.ar[Q][0] = *(const v4i*)(rec);
        z.ar[Q][1] = *(const v4i*)(rec + F);
    }

    template <int P>
    static __device__ __forceinline__ void step(v4i (&acc)[2][S], State& z, char* lds, uint32_t c,
                                                const FragStream& LAL, const FragStream& LBL, const Lanes& ln)
    {
        constexpr int H = P / BS, R = P % BS;
        if constexpr (R == 0) {
            // stage H+2 to LDS from its register buffer, then stage H+4's
            // loads into that buffer (H+2 and H+4 differ by 2 mod 3: the
            // buffer of H+4 is the one of H+1, written a stage ago)
            write_stage<H + 2>(z.st[(H + 2) % 3], lds, ln);
            load_stage<H + 4>(z.st[(H + 4) % 3], LAL, LBL, c, ln.half);
        }
        // the next step's A operands (the next stage's first one from a slot
        // written a stage before this stage's barrier)
        if constexpr (P + 1 < S)
            read_a<(P + 1) / BS, (P + 1) % BS, (P + 1) % 3>(z, lds, ln);
        else
            read_a<NST, 0, 0>(z, lds, ln);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int g = S - 1; g >= P; --g)
#pragma unroll
            for (int rr = 0; rr < 2; ++rr)
                acc[rr][g] = FormI8::mma(z.ar[P % 3][rr], z.win[g - P], acc[rr][g]);
        __builtin_amdgcn_sched_barrier(0);
        // slot S-1-P was read for the last time: the next chunk's fragment
        z.win[S - 1 - P] = *(const v4i*)(lds + (H % 3) * SLOT + R * REC + ln.rd_b);
        if constexpr (R == BS - 1) {
            // this stage's LDS writes done (the 3 reads after them may stay
            // in flight), then the barrier that starts the next stage
            wait_lgkm<3>();
            stage_barrier();
        }
        __builtin_amdgcn_sched_barrier(0);
    }

    template <int... P>
    static __device__ __forceinline__ void chunk(v4i (&acc)[2][S], State& z, char* lds, uint32_t c,
                                                 const FragStream& LAL, const FragStream& LBL, const Lanes& ln,
                                                 std::integer_sequence<int, P...>)
    {
        (step<P>(acc, z, lds, c, LAL, LBL, ln), ...);
    }

    // the whole depth (nkc chunks) for this wave's two row blocks
    static __device__ __forceinline__ void run(v4i (&acc)[2][S], char* lds, const FragStream& LAL,
                                               const FragStream& LB, int64_t nkc, int wave, int lane)
    {
        State z;
        Lanes ln;
        ln.half = wave >> 1;
        ln.wr_a = wave * F + lane * 16;
        ln.wr_b = (4 + (wave & 1)) * F + lane * 16;
        ln.rd_a = 2 * (wave >> 1) * F + lane * 16;
        ln.rd_b = ln.wr_b;
#pragma unroll
        for (int g = S - 1; g >= 0; --g)
            z.win[g] = LB(g * F);
        // stages 0 and 1 in LDS, 2 and 3 in their register buffers
        load_stage<0>(z.st[0], LAL, LB, 0, ln.half);
        load_stage<1>(z.st[1], LAL, LB, 0, ln.half);
        write_stage<0>(z.st[0], lds, ln);
        write_stage<1>(z.st[1], lds, ln);
        load_stage<2>(z.st[2], LAL, LB, 0, ln.half);
        load_stage<3>(z.st[0], LAL, LB, 0, ln.half);
        wait_lgkm<0>();
        stage_barrier();
        read_a<0, 0, 0>(z, lds, ln);
        for (int64_t c = 0; c < nkc; ++c)
            chunk(acc, z, lds, (uint32_t)c, LAL, LB, ln, std::make_integer_sequence<int, S>{});
    }
};

// Whole-triangle INT8 contraction through LDS, two row blocks per wave, the
// whole depth one exactness chunk (the register kernel k_tri2_i8's contract).
template <int S, int B, int BS>
__global__ __launch_bounds__(256, 1) void k_tri2l_i8(GemmArgs a)
{
    __shared__ __attribute__((aligned(16))) char lds[3 * TriL<S, BS>::SLOT];
    const WaveTile w(a, 2);
    const uint64_t bytes = (uint64_t)a.nkc * S * 1024;
    const int64_t nrb = 2 * ((a.M + kTile - 1) / kTile);
    const int64_t rb0 = (w.rb / 4) * 4;   // the workgroup's first row block
    const FragStream LAL = frag_stream((const char*)a.A + (rb0 + w.wave) * bytes,
                                       rb0 + w.wave < nrb ? bytes : 0, w.lane);
    const FragStream LB = frag_stream((const char*)a.B + w.cb * bytes, bytes, w.lane);
    v4i acc[2][S];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int g = 0; g < S; ++g)
            acc[r][g] = FormI8::zero();
    TriL<S, BS>::run(acc, lds, LAL, LB, a.nkc, w.wave, w.lane);
    int64_t x[8][Tri<S, B>::kCols];
#pragma unroll
    for (int n = 0; n < 8; ++n)
#pragma unroll
        for (int j = 0; j < Tri<S, B>::kCols; ++j)
            x[n][j] = 0;
    tri_fold<S, 2, false, B>(acc, x, a, w.rb, w.cb, w.lane);
    tri_outputs<S, 2, B>(x, a, w.rb, w.cb, w.lane);
}

}  // namespace
}  // namespace mdg
