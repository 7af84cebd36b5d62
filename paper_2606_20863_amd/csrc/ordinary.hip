// Ordinary m-double matrix product: the paper's comparison baseline
// (Section 1, Table 1; the "ordinary" columns of Table 2), in which every
// multiplication and addition renormalises its result to m words.
//
//   C_ij = add(...add(add(0, mul(a_i0, b_0j)), mul(a_i1, b_1j))..., mul(a_i,K-1, b_K-1,j))
//
// accumulated in increasing k (m = 1: plain double arithmetic).  The building blocks are the published
// error-free transformations: Knuth's TwoSum, Dekker's Fast2Sum, Veltkamp's
// split and Dekker's product (no fused multiply-add: the library is built
// with contraction off, so every operation is one IEEE rounding).
//   m = 2: the accurate double-double addition (TwoSum of the high and of
//          the low words, two Fast2Sum renormalisations) and the
//          double-double product (Dekker product of the high words plus the
//          two cross products, one Fast2Sum);
//   m = 4: quad-double addition and multiplication with the terms grouped
//          by order, error-free transformations through the orders a
//          quad-double keeps, plain sums beyond, and one branch-free
//          renormalisation of five terms into four words.
//
// Work split: one thread per output entry, a workgroup a 16 x 16 block; the
// A and B words of a depth tile go through LDS.  Every product is at least a
// few hundred dependent double operations, so the kernel is bound by the
// vector FP64 rate.
#include "ordinary.h"

namespace mdg {
namespace {

// m = 1: plain IEEE double arithmetic
template <>
struct Ordinary<1> {
    static __device__ __forceinline__ void add(const double (&x)[1], const double (&y)[1],
                                               double (&r)[1])
    {
        r[0] = x[0] + y[0];
    }
    static __device__ __forceinline__ void mul(const double (&x)[1], const double (&y)[1],
                                               double (&r)[1])
    {
        r[0] = x[0] * y[0];
    }
};

template <>
struct Ordinary<2> {
    static __device__ __forceinline__ void add(const double (&x)[2], const double (&y)[2],
                                               double (&r)[2])
    {
        double s1, s2, t1, t2;
        two_sum(x[0], y[0], s1, s2);
        two_sum(x[1], y[1], t1, t2);
        s2 = s2 + t1;
        fast_two_sum(s1, s2, s1, s2);
        s2 = s2 + t2;
        fast_two_sum(s1, s2, r[0], r[1]);
    }
    static __device__ __forceinline__ void mul(const double (&x)[2], const double (&y)[2],
                                               double (&r)[2])
    {
        double p1, p2;
        two_prod(x[0], y[0], p1, p2);
        const double cross = x[0] * y[1] + x[1] * y[0];
        p2 = p2 + cross;
        fast_two_sum(p1, p2, r[0], r[1]);
    }
};

template <>
struct Ordinary<4> {
    // five terms of decreasing order to four words
    static __device__ __forceinline__ void renorm5(double x0, double x1, double x2, double x3,
                                                   double x4, double (&y)[4])
    {
        double s, t0, t1, t2, t3, t4, e;
        fast_two_sum(x3, x4, s, t4);
        fast_two_sum(x2, s, s, t3);
        fast_two_sum(x1, s, s, t2);
        fast_two_sum(x0, s, t0, t1);
        fast_two_sum(t0, t1, y[0], e);
        fast_two_sum(e, t2, y[1], e);
        fast_two_sum(e, t3, y[2], e);
        y[3] = e + t4;
    }
    static __device__ __forceinline__ void add(const double (&x)[4], const double (&y)[4],
                                               double (&r)[4])
    {
        double s0, s1, s2, s3, e0, e1, e2, e3, u, v;
        two_sum(x[0], y[0], s0, e0);
        two_sum(x[1], y[1], s1, e1);
        two_sum(x[2], y[2], s2, e2);
        two_sum(x[3], y[3], s3, e3);
        two_sum(s1, e0, s1, e0);             // order 1; e0 now order 2
        three_sum(s2, e0, e1, s2, e0, e1);   // order 2; e0 order 3, e1 order 4
        two_sum(s3, e0, s3, u);              // order 3
        two_sum(s3, e2, s3, v);
        const double t = ((e1 + e3) + u) + v;   // order 4
        renorm5(s0, s1, s2, s3, t, r);
    }
    static __device__ __forceinline__ void mul(const double (&x)[4], const double (&y)[4],
                                               double (&r)[4])
    {
        double p0, q0, p1, q1, p2, q2, p3, q3, p4, q4, p5, q5;
        two_prod(x[0], y[0], p0, q0);        // order 0
        two_prod(x[0], y[1], p1, q1);        // order 1
        two_prod(x[1], y[0], p2, q2);
        two_prod(x[0], y[2], p3, q3);        // order 2
        two_prod(x[1], y[1], p4, q4);
        two_prod(x[2], y[0], p5, q5);
        const double p6 = ((x[0] * y[3] + x[1] * y[2]) + x[2] * y[1]) + x[3] * y[0];   // order 3
        double r1, u1, v1, r2, w1, w2, z1, z2, z3;
        three_sum(p1, p2, q0, r1, u1, v1);   // order 1; u1 order 2, v1 order 3
        three_sum(p3, p4, p5, r2, w1, w2);   // order 2; w1, w2 order 3
        two_sum(r2, q1, r2, z1);
        two_sum(r2, q2, r2, z2);
        two_sum(r2, u1, r2, z3);
        double r3 = p6;                      // order 3, left to right
        r3 = r3 + q3;
        r3 = r3 + q4;
        r3 = r3 + q5;
        r3 = r3 + v1;
        r3 = r3 + w1;
        r3 = r3 + w2;
        r3 = r3 + z1;
        r3 = r3 + z2;
        r3 = r3 + z3;
        renorm5(p0, r1, r2, r3, 0.0, r);
    }
};

template <>
struct Ordinary<8> {
    static __device__ __forceinline__ void add(const double (&x)[8], const double (&y)[8], double (&r)[8])
    {
        Expansion<8>::add(x, y, r);
    }
    static __device__ __forceinline__ void mul(const double (&x)[8], const double (&y)[8], double (&r)[8])
    {
        Expansion<8>::mul(x, y, r);
    }
};

constexpr int kOrdTile = 16, kOrdDepth = 32;

template <int MW>
__global__ __launch_bounds__(256) void k_ordinary(const double* __restrict__ A, int64_t psa,
                                                  const double* __restrict__ B, int64_t psb,
                                                  double* __restrict__ C, int64_t psc, int64_t M,
                                                  int64_t N, int64_t K)
{
    __shared__ double sa[MW][kOrdTile][kOrdDepth + 1];
    __shared__ double sb[MW][kOrdDepth][kOrdTile + 1];
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int64_t gx = (N + kOrdTile - 1) / kOrdTile;
    const int64_t i0 = ((int64_t)blockIdx.x / gx) * kOrdTile, j0 = ((int64_t)blockIdx.x % gx) * kOrdTile;
    double acc[MW];
#pragma unroll
    for (int w = 0; w < MW; ++w)
        acc[w] = 0.0;
    for (int64_t k0 = 0; k0 < K; k0 += kOrdDepth) {
        for (int e = t; e < kOrdTile * kOrdDepth; e += 256) {
            const int r = e / kOrdDepth, kk = e % kOrdDepth;
            const bool ok = i0 + r < M && k0 + kk < K;
#pragma unroll
            for (int w = 0; w < MW; ++w)
                sa[w][r][kk] = ok ? A[w * psa + (i0 + r) * K + k0 + kk] : 0.0;
        }
        for (int e = t; e < kOrdDepth * kOrdTile; e += 256) {
            const int kk = e / kOrdTile, c = e % kOrdTile;
            const bool ok = k0 + kk < K && j0 + c < N;
#pragma unroll
            for (int w = 0; w < MW; ++w)
                sb[w][kk][c] = ok ? B[w * psb + (k0 + kk) * N + j0 + c] : 0.0;
        }
        __syncthreads();
        // only the real depths: an added zero product could still change the
        // accumulator's representation
        const int kend = (int)min((int64_t)kOrdDepth, K - k0);
        for (int kk = 0; kk < kend; ++kk) {
            double x[MW], y[MW], p[MW];
#pragma unroll
            for (int w = 0; w < MW; ++w) {
                x[w] = sa[w][ty][kk];
                y[w] = sb[w][kk][tx];
            }
            Ordinary<MW>::mul(x, y, p);
            Ordinary<MW>::add(acc, p, acc);
        }
        __syncthreads();
    }
    const int64_t i = i0 + ty, j = j0 + tx;
    if (i < M && j < N)
#pragma unroll
        for (int w = 0; w < MW; ++w)
            C[w * psc + i * N + j] = acc[w];
}

}  // namespace

hipError_t launch_ordinary(int m, const double* A, const double* B, double* C, int64_t M,
                           int64_t N, int64_t K, hipStream_t st)
{
    const dim3 grid((unsigned)(((N + kOrdTile - 1) / kOrdTile) * ((M + kOrdTile - 1) / kOrdTile)));
    if (m == 1)
        hipLaunchKernelGGL(k_ordinary<1>, grid, dim3(256), 0, st, A, M * K, B, K * N, C, M * N, M, N, K);
    else if (m == 2)
        hipLaunchKernelGGL(k_ordinary<2>, grid, dim3(256), 0, st, A, M * K, B, K * N, C, M * N, M, N, K);
    else if (m == 4)
        hipLaunchKernelGGL(k_ordinary<4>, grid, dim3(256), 0, st, A, M * K, B, K * N, C, M * N, M, N, K);
    else if (m == 8)
        hipLaunchKernelGGL(k_ordinary<8>, grid, dim3(256), 0, st, A, M * K, B, K * N, C, M * N, M, N, K);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_ordinary_dot(int m, const double* X, const double* Y, double* out, int64_t pso, int64_t batch,
                               int64_t n, hipStream_t st)
{
    const int64_t blocks = (batch + 3) / 4;
    if (blocks > 0x7fffffff)
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks);
    const int64_t ps = batch * n;
    if (m == 1)
        hipLaunchKernelGGL(k_ordinary_dot<1>, grid, dim3(256), 0, st, X, ps, Y, ps, out, pso, batch, n);
    else if (m == 2)
        hipLaunchKernelGGL(k_ordinary_dot<2>, grid, dim3(256), 0, st, X, ps, Y, ps, out, pso, batch, n);
    else if (m == 4)
        hipLaunchKernelGGL(k_ordinary_dot<4>, grid, dim3(256), 0, st, X, ps, Y, ps, out, pso, batch, n);
    else if (m == 8)
        hipLaunchKernelGGL(k_ordinary_dot<8>, grid, dim3(256), 0, st, X, ps, Y, ps, out, pso, batch, n);
    else if (m == 16)
        return launch_ordinary_dot16(X, Y, out, pso, batch, n, st);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace mdg
