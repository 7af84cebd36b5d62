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
            fold_chunk<Form, G, DBG, GLOBAL>(acc, t0, a, w);
        }
    }
    if constexpr (!GLOBAL)
        write_outputs<Form>(a, w);
}

// Fold and round every output from the diagonal sums in a.gD: one thread per
// entry, its fold columns in LDS (ncol x 256).
__global__ __launch_bounds__(256) void k_gemm_final(GemmArgs a)
{
    extern __shared__ int64_t lds[];
    const int t = threadIdx.x;
    const int64_t e = (int64_t)blockIdx.x * 256 + t;
    const int64_t MN = a.M * a.N;
    const bool ok = e < MN;
    const int64_t i = ok ? e / a.N : 0, j = ok ? e % a.N : 0;
    int64_t* cols = lds + t;
    for (int q = 0; q < a.ncol; ++q)
        cols[q * 256] = 0;
    if (ok)
        for (int s = 0; s < a.S; ++s)
            fold_add(cols, 0, a.gD[(int64_t)s * MN + e], a.beta * (a.S - 1 - s));
    const int scale = ok ? a.E[i] + a.F[j] - a.beta * (a.S + 1) : 0;
    renormalise(cols, a.ncol, scale, a.m, ok ? a.C + i * a.ldc + j : nullptr, a.psc, ok);
}

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

hipError_t launch_gemm_final(const GemmArgs& a, hipStream_t st)
{
    const size_t lds = (size_t)a.ncol * 256 * sizeof(int64_t);
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_gemm_final,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    const int64_t blocks = (a.M * a.N + 255) / 256;
    hipLaunchKernelGGL(k_gemm_final, dim3((unsigned)blocks), dim3(256), lds, st, a);
    return hipGetLastError();
}

}  // namespace mdg
