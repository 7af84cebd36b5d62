// Ordinary hexa-double (m = 16) inner products: the expansion arithmetic of
// the octo-doubles on 16 words, in a unit of its own (its product keeps a
// few hundred doubles per thread in scratch and takes minutes to compile).
#include "ordinary.h"

namespace mdg {
namespace {

template <>
struct Ordinary<16> {
    static __device__ __forceinline__ void add(const double (&x)[16], const double (&y)[16], double (&r)[16])
    {
        Expansion<16>::add(x, y, r);
    }
    static __device__ __forceinline__ void mul(const double (&x)[16], const double (&y)[16], double (&r)[16])
    {
        Expansion<16>::mul(x, y, r);
    }
};

}  // namespace

hipError_t launch_ordinary_dot16(const double* X, const double* Y, double* out, int64_t pso, int64_t batch,
                                 int64_t n, hipStream_t st)
{
    const int64_t blocks = (batch + 3) / 4;
    if (blocks > 0x7fffffff)
        return hipErrorInvalidValue;
    const int64_t ps = batch * n;
    hipLaunchKernelGGL(k_ordinary_dot<16>, dim3((unsigned)blocks), dim3(256), 0, st, X, ps, Y, ps, out, pso, batch,
                       n);
    return hipGetLastError();
}

}  // namespace mdg
