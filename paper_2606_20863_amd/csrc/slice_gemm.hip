// Banded slice contraction (FP64 form, and INT8 beyond 32 diagonals) and the
// dispatch of the INT8 contraction between the banded and the whole-triangle
// kernels.
#include "slice_common.h"

namespace mdg {
namespace {

// Banded contraction: S = nbands * G diagonals, G at a time.  GLOBAL: the
// diagonal sums go to a.gD and launch_gemm_final rounds them.
template <class Form, int G, bool DBG, bool GLOBAL>
__global__ __launch_bounds__(256, 1) void k_slice_gemm(GemmArgs a)
{
    typedef typename Form::frag Frag;
    typedef typename Form::acc Acc;
    extern __shared__ int64_t lds[];
    WaveTile w(a, 1);
    if constexpr (!GLOBAL)
        w.init_cols(a, lds);
    const int64_t fstride = (int64_t)a.S * 64;   // fragments of one depth chunk
    const Frag* Ab = (const Frag*)a.A + w.rb * a.nkc * fstride + w.lane;
    const Frag* Bb = (const Frag*)a.B + w.cb * a.nkc * fstride + w.lane;

    for (int b = 0; b < a.nbands; ++b) {
        const int t0 = b * G;
        for (int64_t c0 = 0; c0 < a.nkc; c0 += a.kcc) {
            Acc acc[G];
#pragma unroll
            for (int g = 0; g < G; ++g)
                acc[g] = Form::zero();
            const int64_t c1 = min(c0 + a.kcc, a.nkc);
            if constexpr (Form::kPipelined && G > 3) {
                band_run<Form, G, 3>(acc, Ab, Bb, fstride, c0, c1, t0);
            } else {
                for (int64_t kc = c0; kc < c1; ++kc)
                    band_chunk<Form, G>(acc, Ab + kc * fstride, Bb + kc * fstride, t0);
            }
            fold_chunk<Form, G, DBG, GLOBAL>(acc, t0, a, w, c0 == 0);
        }
    }
    if constexpr (!GLOBAL)
        write_outputs<Form>(a, w);
}

// INT8 bands with R row blocks of op(A) sharing one window of B fragments
// (as the whole-triangle kernel does), over the depth chunks [c0, c1).  A
// chunk runs steps s = 0 .. t0+G-1: step s multiplies A_s of every row block
// with B_{t0+g-s} into diagonal t0+g for every g with a partner (all g
// while s < t0, g >= s - t0 after).  The window slot of B_u is u mod G; the
// B fragment entering at step s (1 <= s <= t0) is B_{t0-s}.  A fragments and
// entering B fragments are loaded P steps ahead into small rings, across
// chunk boundaries; the next chunk's window is loaded in place during the
// tail steps, slot G-p at tail step p (its last use was the step before).  Buffer
// descriptors bound every load (offsets past a stream read zeros).
template <int G, int R, int P>
__device__ __forceinline__ void band_run_r(v4i (&acc)[R][G], const FragStream (&LDA)[R],
                                           const FragStream& LDB, int64_t c0, int64_t c1, int t0,
                                           int S)
{
    static_assert(P >= 1 && P < G, "prefetch distance must be below the band width");
    constexpr uint32_t F = 1024;
    const uint32_t CS = (uint32_t)S * F;
    uint32_t ck = (uint32_t)c0 * CS;
    v4i win[G], pa[R][P], pb[P];
#pragma unroll
    for (int g = G - 1; g >= 0; --g)
        win[g] = LDB(ck + (uint32_t)(t0 + g) * F);
#pragma unroll
    for (int q = 0; q < P; ++q) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            pa[r][q] = LDA[r](ck + q * F);
        pb[q] = LDB(q <= t0 ? ck + (uint32_t)(t0 - q) * F : ck);
    }
    for (int64_t kc = c0; kc < c1; ++kc) {
        const uint32_t cn = kc + 1 < c1 ? ck + CS : ck;
        // steps s = 0 .. t0-1: every diagonal of the band has a partner
        for (int s0 = 0; s0 < t0; s0 += G) {
#pragma unroll
            for (int r = 0; r < G; ++r) {
                const int s = s0 + r;
                v4i a[R];
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    a[rr] = pa[rr][0];
                const v4i b = pb[0];
#pragma unroll
                for (int q = 0; q + 1 < P; ++q) {
#pragma unroll
                    for (int rr = 0; rr < R; ++rr)
                        pa[rr][q] = pa[rr][q + 1];
                    pb[q] = pb[q + 1];
                }
                // step s + P < t0 + G is this chunk's
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    pa[rr][P - 1] = LDA[rr](ck + (uint32_t)(s + P) * F);
                if (s + P <= t0)
                    pb[P - 1] = LDB(ck + (uint32_t)(t0 - s - P) * F);
                if (r > 0 || s0 > 0)
                    win[(G - r) % G] = b;
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int g = G - 1; g >= 0; --g)
#pragma unroll
                    for (int rr = 0; rr < R; ++rr)
                        acc[rr][g] = FormI8::mma(a[rr], win[(g - r + G) % G], acc[rr][g]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // step t0: B_0 enters
        {
            v4i a[R];
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
                a[rr] = pa[rr][0];
            const v4i b = pb[0];
#pragma unroll
            for (int q = 0; q + 1 < P; ++q) {
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    pa[rr][q] = pa[rr][q + 1];
                pb[q] = pb[q + 1];
            }
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
                pa[rr][P - 1] = LDA[rr](ck + (uint32_t)(t0 + P) * F);
            if (t0 > 0)
                win[0] = b;
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int g = G - 1; g >= 0; --g)
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    acc[rr][g] = FormI8::mma(a[rr], win[g], acc[rr][g]);
            __builtin_amdgcn_sched_barrier(0);
        }
        // tail steps t0 + p, p = 1 .. G-1: diagonals g >= p read slots
        // 0 .. G-1-p, so slot G-p takes the next chunk's B_{t0+G-p}
#pragma unroll
        for (int p = 1; p < G; ++p) {
            v4i a[R];
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
                a[rr] = pa[rr][0];
#pragma unroll
            for (int q = 0; q + 1 < P; ++q) {
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    pa[rr][q] = pa[rr][q + 1];
                pb[q] = pb[q + 1];
            }
            const int nq = p + P - G;   // step of the next chunk, if >= 0
            if (nq < 0) {
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    pa[rr][P - 1] = LDA[rr](ck + (uint32_t)(t0 + p + P) * F);
            } else {
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    pa[rr][P - 1] = LDA[rr](cn + (uint32_t)nq * F);
                if (nq >= 1 && nq <= t0)
                    pb[P - 1] = LDB(cn + (uint32_t)(t0 - nq) * F);
            }
            win[G - p] = LDB(cn + (uint32_t)(t0 + G - p) * F);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int g = G - 1; g >= p; --g)
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
                    acc[rr][g] = FormI8::mma(a[rr], win[g - p], acc[rr][g]);
            __builtin_amdgcn_sched_barrier(0);
        }
        win[0] = LDB(cn + (uint32_t)t0 * F);
        ck = cn;
    }
}

// Banded INT8 contraction (S > 32 diagonals, bands of G) with two row blocks
// per wave, 64 x 32 workgroup tiles; the diagonal sums of every exactness
// chunk are added into a.gD (the first chunk masks the old contents to zero:
// every slot belongs to exactly one band, so the buffer needs no clearing),
// and launch_gemm_final folds and rounds.
template <int G>
__global__ __launch_bounds__(256, 1) void k_band2_i8(GemmArgs a)
{
    const WaveTile w(a, 2);
    const uint64_t bytes = (uint64_t)a.nkc * a.S * 1024;
    const int64_t nrb = 2 * ((a.M + kTile - 1) / kTile);
    FragStream LA[2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
        LA[r] = frag_stream((const char*)a.A + (w.rb + r) * bytes, w.rb + r < nrb ? bytes : 0,
                            w.lane);
    const FragStream LB = frag_stream((const char*)a.B + w.cb * bytes, bytes, w.lane);
    for (int b = 0; b < a.nbands; ++b) {
        const int t0 = b * G;
        for (int64_t c0 = 0; c0 < a.nkc; c0 += a.kcc) {
            v4i acc[2][G];
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int g = 0; g < G; ++g)
                    acc[r][g] = FormI8::zero();
            band_run_r<G, 2, 3>(acc, LA, LB, c0, min(c0 + a.kcc, a.nkc), t0, a.S);
            // the lane's eight slots of each diagonal (private, padded: no
            // bounds checks), one diagonal at a time
            int64_t* D = gd_lane(a, w) + (int64_t)t0 * 512;
            const int64_t keep = c0 == 0 ? 0 : -1;   // the first chunk overwrites
#pragma unroll
            for (int g = 0; g < G; ++g) {
#pragma unroll
                for (int r = 0; r < 2; ++r)
#pragma unroll
                    for (int o = 0; o < 4; ++o)
                        D[r * 4 + o] = (D[r * 4 + o] & keep) + acc[r][g][o];
                D += 512;
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
}

template <int G>
struct DispatchBand2 {
    static hipError_t run(const GemmArgs& a, hipStream_t st)
    {
        if (a.band == G)
            return launch_kernel(k_band2_i8<G>, a, st, false, 2 * kTile);
        return DispatchBand2<G - 1>::run(a, st);
    }
};
template <>
struct DispatchBand2<3> {   // the pipeline needs bands wider than its depth
    static hipError_t run(const GemmArgs&, hipStream_t) { return hipErrorInvalidValue; }
};

template <class Form, int G>
struct Dispatch {
    static hipError_t run(const GemmArgs& a, hipStream_t st)
    {
        if (a.band == G) {
            if (a.gD)
                return launch_kernel(k_slice_gemm<Form, G, false, true>, a, st, false);
            return a.dbgD ? launch_kernel(k_slice_gemm<Form, G, true, false>, a, st)
                          : launch_kernel(k_slice_gemm<Form, G, false, false>, a, st);
        }
        return Dispatch<Form, G - 1>::run(a, st);
    }
};
template <class Form>
struct Dispatch<Form, 0> {
    static hipError_t run(const GemmArgs&, hipStream_t) { return hipErrorInvalidValue; }
};

}  // namespace

hipError_t launch_gemm_i8(const GemmArgs& a, hipStream_t st)
{
    // the triangle kernel's register fold holds |X| / 2^(4 beta ceil(S/4))
    // < K 2^9 in its signed top column
    if (a.nbands == 1 && a.S <= kTriMaxI8 && a.nkc * kKcI8 < ((int64_t)1 << 48)) {
        if (a.fixX) {
            if (a.beta == 8)
                return a.S <= 22 ? launch_trifix8_s1_22(a, st) : launch_trifix8_s23_32(a, st);
            if (a.beta != 7)
                return hipErrorInvalidValue;
            return a.S <= 22 ? launch_trifix_s1_22(a, st) : launch_trifix_s23_32(a, st);
        }
        if (a.kcc >= a.nkc && !a.dbgD && trid_shape(a.S, a.beta))
            return launch_trid(a, st);
        if (a.beta == 8) {
            if (a.S <= 22)
                return launch_tri8_s1_22(a, st);
            if (a.S <= 28)
                return launch_tri8_s23_28(a, st);
            return launch_tri8_s29_32(a, st);
        }
        if (a.beta != 7)
            return hipErrorInvalidValue;
        if (a.S <= 22)
            return launch_tri_s1_22(a, st);
        if (a.S <= 28)
            return launch_tri_s23_28(a, st);
        return launch_tri_s29_32(a, st);
    }
    // two bands over the whole depth, folded in registers
    if (duo_shape(a.S, a.band)) {
        if (a.kcc < a.nkc || a.dbgD || a.fixX || a.gD)
            return hipErrorInvalidValue;
        if (a.beta == 8)
            return a.S <= 48 ? launch_duo8_s36_48(a, st) : launch_duo8_s52_64(a, st);
        if (a.beta != 7)
            return hipErrorInvalidValue;
        return a.S <= 48 ? launch_duo_s36_48(a, st) : launch_duo_s52_64(a, st);
    }
    // bands: the diagonal sums go through a.gD
    if (!a.gD)
        return hipErrorInvalidValue;
    return DispatchBand2<kGmaxI8>::run(a, st);
}

hipError_t launch_gemm_f64(const GemmArgs& a, hipStream_t st)
{
    return Dispatch<FormF64, kGmaxF64>::run(a, st);
}


}  // namespace mdg
