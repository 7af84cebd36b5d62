// Exact fixed-point results: the product's sum before its one rounding, as
// a multiword integer X with a power-of-two scale (the paper's "multiple
// integers", Section 1, on the grids of Section 2).  With every depth block
// split on the same shared exponents, the integers of the blocks add up
// exactly to the integer of the whole product, so a product cut along its
// depth is summed here without any rounding and rounded once at the end.
//
// Layout: limb planes.  Limb k of entry e is X[k * count + e] (32-bit two's
// complement, least significant first), so one thread per entry reads and
// writes contiguous runs across the block.
#include "mdgemm_internal.h"
#include "renorm.h"

namespace mdg {
namespace {

// X_e = sum_t D_t 2^(beta (S-1-t)) from D [S][count]: a signed 128-bit
// window slides up in 32-bit steps (the sums enter least significant
// first), NL >= the fold width so that the window ends as the sign, which
// fills the limbs from NL up.
template <int NL>
__global__ __launch_bounds__(256) void k_fixed_from_D(const int64_t* D, int S, int beta, int64_t M,
                                                      int64_t N, const int32_t* E, const int32_t* F,
                                                      int eoff, int32_t* X, int nlimb, int32_t* scale)
{
    const int64_t count = M * N;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count)
        return;
    const int64_t i = e / N, j = e % N;
    __int128 win = 0;
    int t = S - 1, p = 0;
    uint32_t L[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        while (t >= 0 && p < 32 * (k + 1)) {
            win += (__int128)D[(int64_t)t * count + e] << (p - 32 * k);
            --t;
            p += beta;
        }
        L[k] = (uint32_t)(uint64_t)win;
        win >>= 32;
    }
    const uint32_t fill = win < 0 ? 0xffffffffu : 0u;
    for (int k = 0; k < nlimb; ++k) {
        uint32_t v = fill;
#pragma unroll
        for (int q = 0; q < NL; ++q)
            v = q == k ? L[q] : v;
        X[(int64_t)k * count + e] = (int32_t)v;
    }
    scale[e] = E[i] + F[j] + 2 * eoff - beta * (S + 1);
}

__global__ __launch_bounds__(256) void k_fixed_add(int64_t count, int nlimb, const int32_t* X,
                                                   const int32_t* Y, int32_t* Z)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count)
        return;
    uint64_t cy = 0;
    for (int k = 0; k < nlimb; ++k) {
        const int64_t o = (int64_t)k * count + e;
        const uint64_t v = (uint64_t)(uint32_t)X[o] + (uint32_t)Y[o] + cy;
        Z[o] = (int32_t)(uint32_t)v;
        cy = v >> 32;
    }
}

// Magnitude in NL >= nlimb register limbs (sign-extended), then the greedy
// rounding steps of the product's own fold.
template <int NL>
__global__ __launch_bounds__(256) void k_fixed_round(int m, int64_t count, int nlimb, const int32_t* X,
                                                     const int32_t* scale, double* C, int64_t psc)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count)
        return;
    const bool neg = X[(int64_t)(nlimb - 1) * count + e] < 0;
    uint32_t L[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k)
        L[k] = k < nlimb ? (uint32_t)X[(int64_t)k * count + e] : (neg ? 0xffffffffu : 0u);
    uint64_t cy = 1;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const uint64_t v = (uint64_t)(~L[k]) + cy;
        cy = v >> 32;
        L[k] = neg ? (uint32_t)v : L[k];
    }
    double sgn = neg ? -1.0 : 1.0;
    int sc = scale[e];
    for (int w = 0; w < m; ++w)
        C[w * psc + e] = rn_next(L, sgn, sc);
}

unsigned blocks_of(int64_t count) { return (unsigned)((count + 255) / 256); }

template <int NL>
hipError_t from_D(const int64_t* D, int S, int beta, int64_t M, int64_t N, const int32_t* E,
                  const int32_t* F, int eoff, int32_t* X, int nlimb, int32_t* scale, hipStream_t st)
{
    hipLaunchKernelGGL(k_fixed_from_D<NL>, dim3(blocks_of(M * N)), dim3(256), 0, st, D, S, beta, M, N, E,
                       F, eoff, X, nlimb, scale);
    return hipGetLastError();
}

template <int NL>
hipError_t round_nl(int m, int64_t count, int nlimb, const int32_t* X, const int32_t* scale, double* C,
                    int64_t psc, hipStream_t st)
{
    hipLaunchKernelGGL(k_fixed_round<NL>, dim3(blocks_of(count)), dim3(256), 0, st, m, count, nlimb, X,
                       scale, C, psc);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fixed_from_D(const int64_t* D, int S, int beta, int64_t M, int64_t N,
                               const int32_t* E, const int32_t* F, int eoff, int ncol, int32_t* X,
                               int nlimb, int32_t* scale, hipStream_t st)
{
    if ((M * N + 255) / 256 > 0x7fffffff)
        return hipErrorInvalidValue;
    if (ncol <= 8) return from_D<8>(D, S, beta, M, N, E, F, eoff, X, nlimb, scale, st);
    if (ncol <= 12) return from_D<12>(D, S, beta, M, N, E, F, eoff, X, nlimb, scale, st);
    if (ncol <= 16) return from_D<16>(D, S, beta, M, N, E, F, eoff, X, nlimb, scale, st);
    if (ncol <= 20) return from_D<20>(D, S, beta, M, N, E, F, eoff, X, nlimb, scale, st);
    if (ncol <= 24) return from_D<24>(D, S, beta, M, N, E, F, eoff, X, nlimb, scale, st);
    if (ncol <= 32) return from_D<32>(D, S, beta, M, N, E, F, eoff, X, nlimb, scale, st);
    if (ncol <= 48) return from_D<48>(D, S, beta, M, N, E, F, eoff, X, nlimb, scale, st);
    if (ncol <= 80) return from_D<80>(D, S, beta, M, N, E, F, eoff, X, nlimb, scale, st);
    return hipErrorInvalidValue;
}

hipError_t launch_fixed_add(int64_t count, int nlimb, const int32_t* X, const int32_t* Y, int32_t* Z,
                            hipStream_t st)
{
    if ((count + 255) / 256 > 0x7fffffff)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fixed_add, dim3(blocks_of(count)), dim3(256), 0, st, count, nlimb, X, Y, Z);
    return hipGetLastError();
}

hipError_t launch_fixed_round(int m, int64_t count, int nlimb, const int32_t* X, const int32_t* scale,
                              double* C, int64_t psc, hipStream_t st)
{
    if ((count + 255) / 256 > 0x7fffffff)
        return hipErrorInvalidValue;
    if (nlimb <= 8) return round_nl<8>(m, count, nlimb, X, scale, C, psc, st);
    if (nlimb <= 12) return round_nl<12>(m, count, nlimb, X, scale, C, psc, st);
    if (nlimb <= 16) return round_nl<16>(m, count, nlimb, X, scale, C, psc, st);
    if (nlimb <= 20) return round_nl<20>(m, count, nlimb, X, scale, C, psc, st);
    if (nlimb <= 24) return round_nl<24>(m, count, nlimb, X, scale, C, psc, st);
    if (nlimb <= 32) return round_nl<32>(m, count, nlimb, X, scale, C, psc, st);
    if (nlimb <= 48) return round_nl<48>(m, count, nlimb, X, scale, C, psc, st);
    if (nlimb <= 80) return round_nl<80>(m, count, nlimb, X, scale, C, psc, st);
    return hipErrorInvalidValue;
}

}  // namespace mdg
