// The whole-triangle INT8 contraction with the A fragments shared through
// LDS by direct-to-LDS buffer loads: of the two waves that multiply the same
// two row blocks (against different column blocks), each loads one row
// block's fragment per step straight into LDS (no register round trip), and
// both read both from there; the B window stays in registers, loaded per
// wave as in k_tri2_i8.  Per wave and step this is two fragment loads
// through the texture path instead of three.
//
// The steps of a depth chunk are grouped in stages of BS steps (S = NST BS,
// NST a multiple of 3, so every stage's slot is fixed by its place in the
// chunk).  Three LDS slots of BS records rotate; a record holds one step's
// four A fragments (two row-block pairs x two row blocks, 4 KB).  Stage j's
// loads are issued right after the barrier that starts stage j-2; at the
// start of stage j each wave waits until its own loads of stage j are done
// (a vector-memory count fixed at compile time by the issue order below),
// then the barrier makes every wave's loads of stage j visible.  Slot j mod
// 3 is written again by stage j+3's loads, issued after the barrier that
// starts stage j+1, by which time every wave has consumed its reads of
// stage j.
#pragma once

#include "tri.h"

namespace mdg {
namespace {

// s_waitcnt with lgkmcnt and expcnt at their maxima and vmcnt = N (gfx9
// encoding: vmcnt in bits [3:0] and [15:14], expcnt [6:4], lgkmcnt [11:8])
template <int N>
__device__ __forceinline__ void wait_vm()
{
    static_assert(N >= 0 && N < 64, "vmcnt field");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (0x7 << 4) | (0xf << 8));
}

// workgroup barrier that also keeps the compiler's memory operations on
// their side of it
__device__ __forceinline__ void stage_barrier()
{
    asm volatile("s_barrier" ::: "memory");
}

template <int S, int BS>
struct TriD {
    static constexpr int NST = S / BS;
    static_assert(S % BS == 0 && NST % 3 == 0 && NST >= 3, "stages of whole steps, slots fixed per stage");
    static constexpr uint32_t F = 1024, CS = (uint32_t)S * F;
    static constexpr uint32_t REC = 4 * F, SLOT = BS * REC;

    // vector-memory operations a wave issues in stage s of a chunk besides
    // its stage loads: one B window load per step, the one of step 0 being
    // the previous chunk's last (counted in stage NST-1)
    static constexpr int b_loads(int s) { return BS - (s == 0 ? 1 : 0) + (s == NST - 1 ? 1 : 0); }
    // issued after stage j's loads and before the wait that starts stage j
    // (steady state: stage j's loads were issued at the start of stage j-2)
    static constexpr int younger(int j)
    {
        return BS + b_loads((j + NST - 2) % NST) + b_loads((j + NST - 1) % NST);
    }

    // this wave's row-block fragment of the BS steps of stage H (H may pass
    // the chunk: the next chunk's stages) into its LDS slot
    template <int H>
    static __device__ __forceinline__ void issue_stage(const FragStream& LAL, char* lds, uint32_t ck,
                                                       uint32_t cn, uint32_t mine)
    {
        const uint32_t base = H < NST ? ck : cn;
        constexpr int h = H % NST;
#pragma unroll
        for (int r = 0; r < BS; ++r) {
            __attribute__((address_space(3))) void* dst =
                (__attribute__((address_space(3))) void*)(lds + (h % 3) * SLOT + r * REC + mine);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(LAL.rsrc, dst, 16, LAL.voff, (int)(base + (h * BS + r) * F), 0,
                                                     0);
        }
    }

    // A of step P for the wave's two row blocks, from LDS (pair: the pair's
    // offset in a record plus this lane's 16 bytes)
    template <int P>
    static __device__ __forceinline__ void read_a(v4i (&ar)[2], const char* lds, uint32_t pair)
    {
        const char* rec = lds + ((P / BS) % 3) * SLOT + (P % BS) * REC + pair;
        ar[0] = *(const v4i*)(rec);
        ar[1] = *(const v4i*)(rec + F);
    }

    template <int P>
    static __device__ __forceinline__ void step(v4i (&acc)[2][S], v4i (&win)[S], v4i (&ar)[2][2], char* lds,
                                                uint32_t ck, uint32_t cn, const FragStream& LAL,
                                                const FragStream& LDB, uint32_t mine, uint32_t pair)
    {
        constexpr int H = P / BS;
        if constexpr (P % BS == 0) {
            // start of stage H: this wave's loads of it done, then everyone's
            wait_vm<younger(H)>();
            stage_barrier();
            // the stage loads stay together, ahead of this step's B load (the
            // wait counts above depend on that order)
            __builtin_amdgcn_sched_barrier(0);
            issue_stage<H + 2>(LAL, lds, ck, cn, mine);
            __builtin_amdgcn_sched_barrier(0);
            read_a<P>(ar[P & 1], lds, pair);
        }
        // the next step's A, inside this stage
        if constexpr ((P + 1) % BS != 0)
            read_a<P + 1>(ar[(P + 1) & 1], lds, pair);
        if constexpr (P >= 1)
            win[S - P] = LDB(cn + (S - P) * F);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int g = S - 1; g >= P; --g)
#pragma unroll
            for (int r = 0; r < 2; ++r)
                acc[r][g] = FormI8::mma(ar[P & 1][r], win[g - P], acc[r][g]);
        __builtin_amdgcn_sched_barrier(0);
    }

    template <int... P>
    static __device__ __forceinline__ void chunk(v4i (&acc)[2][S], v4i (&win)[S], v4i (&ar)[2][2], char* lds,
                                                 uint32_t ck, uint32_t cn, const FragStream& LAL,
                                                 const FragStream& LDB, uint32_t mine, uint32_t pair,
                                                 std::integer_sequence<int, P...>)
    {
        (step<P>(acc, win, ar, lds, ck, cn, LAL, LDB, mine, pair), ...);
    }

    // the whole depth [0, nkc) for the wave's two row blocks; LAL streams the
    // one row block this wave loads for its pair (wave & 1 of rows rb, rb+1)
    static __device__ __forceinline__ void run(v4i (&acc)[2][S], char* lds, const FragStream& LAL,
                                               const FragStream& LDB, int64_t nkc, int wave, int lane)
    {
        // the pair's two fragments in a record, the one this wave loads (the
        // loads place lane l's 16 bytes at byte 16 l of the fragment), and
        // this lane's bytes of the pair's first fragment for the reads
        const uint32_t base = (uint32_t)(wave >> 1) * 2 * F;
        const uint32_t mine = base + (uint32_t)(wave & 1) * F;
        const uint32_t pair = base + (uint32_t)lane * 16;
        v4i win[S], ar[2][2];
        // stages 0 and 1 of the first chunk, then its window: at least as many
        // loads follow each stage's as in the steady state, so the waits of the
        // first two stages are conservative
        const uint32_t c1 = nkc > 1 ? CS : 0;
        issue_stage<0>(LAL, lds, 0, c1, mine);
        issue_stage<1>(LAL, lds, 0, c1, mine);
#pragma unroll
        for (int g = S - 1; g >= 0; --g)
            win[g] = LDB(g * F);
        uint32_t ck = 0;
        for (int64_t kc = 0; kc < nkc; ++kc) {
            const uint32_t cn = kc + 1 < nkc ? ck + CS : ck;
            chunk(acc, win, ar, lds, ck, cn, LAL, LDB, mine, pair, std::make_integer_sequence<int, S>{});
            win[0] = LDB(cn);
            ck = cn;
        }
        // every stage load issued has landed before the workgroup ends
        wait_vm<0>();
    }
};

// Whole-triangle INT8 contraction with the A fragments through LDS, two row
// blocks per wave (64 x 32 workgroup tile), the whole depth one exactness
// chunk: k_tri2_i8's contract.
template <int S, int B, int BS>
__global__ __launch_bounds__(256, 1) void k_tri2d_i8(GemmArgs a)
{
    __shared__ __attribute__((aligned(16))) char lds[3 * TriD<S, BS>::SLOT];
    const WaveTile w(a, 2);
    const uint64_t bytes = (uint64_t)a.nkc * S * 1024;
    const int64_t nrb = 2 * ((a.M + kTile - 1) / kTile);
    const int64_t rbl = w.rb + (w.wave & 1);   // the row block this wave loads for its pair
    const FragStream LAL = frag_stream((const char*)a.A + rbl * bytes, rbl < nrb ? bytes : 0, w.lane);
    const FragStream LB = frag_stream((const char*)a.B + w.cb * bytes, bytes, w.lane);
    v4i acc[2][S];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int g = 0; g < S; ++g)
            acc[r][g] = FormI8::zero();
    TriD<S, BS>::run(acc, lds, LAL, LB, a.nkc, w.wave, w.lane);
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
