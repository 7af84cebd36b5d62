// Banded slice contraction (FP64 form, and INT8 beyond 32 diagonals) and the
// dispatch of the INT8 contraction between the banded and the whole-triangle
// kernels.
#include "slice_common.h"

namespace mdg {
namespace {

// Banded contraction: S = nbands * G diagonals, G at a time.
template <class Form, int G, bool DBG>
__global__ __launch_bounds__(256, 1) void k_slice_gemm(GemmArgs a)
{
    typedef typename Form::frag Frag;
    typedef typename Form::acc Acc;
    extern __shared__ int64_t lds[];
    WaveTile w(a, 1);
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
            fold_chunk<Form, G, DBG>(acc, t0, a, w);
        }
    }
    write_outputs<Form>(a, w);
}

template <class Form, int G>
struct Dispatch {
    static hipError_t run(const GemmArgs& a, hipStream_t st)
    {
        if (a.band == G)
            return a.dbgD ? launch_kernel(k_slice_gemm<Form, G, true>, a, st)
                          : launch_kernel(k_slice_gemm<Form, G, false>, a, st);
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
    // the triangle kernel's register fold holds |X| / 2^(28 ceil(S/4)) < K 2^9
    // in its signed top column
    if (a.nbands == 1 && a.S <= kTriMaxI8 && a.nkc * kKcI8 < ((int64_t)1 << 48)) {
        if (a.S <= 22)
            return launch_tri_s1_22(a, st);
        if (a.S <= 28)
            return launch_tri_s23_28(a, st);
        return launch_tri_s29_32(a, st);
    }
    return Dispatch<FormI8, kGmaxI8>::run(a, st);
}

hipError_t launch_gemm_f64(const GemmArgs& a, hipStream_t st)
{
    return Dispatch<FormF64, kGmaxF64>::run(a, st);
}

}  // namespace mdg
