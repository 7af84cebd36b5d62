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
#include "mdgemm_internal.h"

#include <utility>

namespace mdg {
namespace {

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void fast_two_sum(double a, double b, double& s, double& e)
{
    s = a + b;
    e = b - (s - a);
}

__device__ __forceinline__ void split(double a, double& hi, double& lo)
{
    const double t = 134217729.0 * a;   // 2^27 + 1
    hi = t - (t - a);
    lo = a - hi;
}

__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e)
{
    p = a * b;
    double ah, al, bh, bl;
    split(a, ah, al);
    split(b, bh, bl);
    e = ah * bh - p;
    e = e + ah * bl;
    e = e + al * bh;
    e = e + al * bl;
}

__device__ __forceinline__ void three_sum(double a, double b, double d, double& s, double& e1,
                                          double& e2)
{
    double u, v, w;
    two_sum(a, b, u, v);
    two_sum(u, d, s, w);
    two_sum(v, w, e1, e2);
}

template <int MW>
struct Ordinary;

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

// m = 8: floating-point expansion arithmetic (CAMPARY's building blocks,
// Joldes, Muller, Popescu and Tucker): VecSum (TwoSum of each term with the
// running sum, from the last term up), VecSumErrBranch (Fast2Sum down the
// terms, a new output word whenever the error is nonzero, until 8 words are
// out), addition by merging both operands' words by decreasing magnitude
// (Batcher's odd-even merge network: fixed compare-exchanges, no branches)
// and renormalising, multiplication by the product of expansions truncated
// at order 8 (TwoProd of every product of order n < 8, each order's high
// parts and the carried errors through VecSum, the order-8 products and the
// remaining errors added plainly, then renormalised).

// Batcher's odd-even merge of two sorted runs of N = 2^k: the compare-
// exchange pairs, in order.
template <int N>
struct MergeNet {
    int lo[N * 8], hi[N * 8];   // room for the pairs (N log2(N) + 1 at most)
    int n = 0;
    constexpr void run(int l, int h, int r)
    {
        const int step = 2 * r;
        if (step < h - l) {
            run(l, h, step);
            run(l + r, h, step);
            for (int i = l + r; i < h - r; i += step) {
                lo[n] = i;
                hi[n] = i + r;
                ++n;
            }
        } else {
            lo[n] = l;
            hi[n] = l + r;
            ++n;
        }
    }
    constexpr MergeNet() : lo(), hi() { run(0, 2 * N - 1, 1); }
};

template <int MW>
struct Expansion {
    static constexpr MergeNet<MW> kNet{};

    // x becomes (s_0, e_1, .., e_(N-1)), the same exact sum
    template <int N>
    static __device__ __forceinline__ void vec_sum(double (&x)[N])
    {
        double s = x[N - 1];
#pragma unroll
        for (int i = N - 2; i >= 0; --i) {
            double e;
            two_sum(x[i], s, s, e);
            x[i + 1] = e;
        }
        x[0] = s;
    }

    // MW words from a VecSum output; per lane, the output slot advances
    // where the error is nonzero (selects, so that the words stay in
    // registers), and the walk stops when MW words are out
    template <int N>
    static __device__ __forceinline__ void err_branch(const double (&e)[N], double (&r)[MW])
    {
#pragma unroll
        for (int q = 0; q < MW; ++q)
            r[q] = 0.0;
        int j = 0;
        bool done = false;
        double eps = e[0];
#pragma unroll
        for (int i = 0; i + 1 < N; ++i) {
            double rj, nxt;
            fast_two_sum(eps, e[i + 1], rj, nxt);
#pragma unroll
            for (int q = 0; q < MW; ++q)
                r[q] = !done && q == j ? rj : r[q];
            const bool more = nxt != 0.0;
            const bool full = more && j >= MW - 1;
            eps = done ? eps : (more ? nxt : rj);
            j = !done && more && !full ? j + 1 : j;
            done = done || full;
        }
#pragma unroll
        for (int q = 0; q < MW; ++q)
            r[q] = !done && q == j ? eps : r[q];
    }

    template <int N>
    static __device__ __forceinline__ void renormalize(double (&x)[N], double (&r)[MW])
    {
        vec_sum(x);
        err_branch(x, r);
    }

    template <int P>
    static __device__ __forceinline__ void exchange(double (&z)[2 * MW])
    {
        constexpr int i = kNet.lo[P], k = kNet.hi[P];
        const bool c = fabs(z[i]) < fabs(z[k]);
        const double a = z[i], b = z[k];
        z[i] = c ? b : a;
        z[k] = c ? a : b;
    }
    template <int... P>
    static __device__ __forceinline__ void merge(double (&z)[2 * MW], std::integer_sequence<int, P...>)
    {
        (exchange<P>(z), ...);
    }

    static __device__ __forceinline__ void add(const double (&x)[MW], const double (&y)[MW], double (&r)[MW])
    {
        double z[2 * MW];
#pragma unroll
        for (int w = 0; w < MW; ++w) {
            z[w] = x[w];
            z[MW + w] = y[w];
        }
        merge(z, std::make_integer_sequence<int, kNet.n>{});
        renormalize(z, r);
    }

    // order n of the product: errs are the n^2 words carried from below
    template <int n>
    static __device__ __forceinline__ void mul_order(const double (&x)[MW], const double (&y)[MW],
                                                     double (&t)[MW + 1], const double (&errs)[n * n])
    {
        if constexpr (n < MW) {
            double v[n + 1 + n * n], eh[n + 1];
#pragma unroll
            for (int i = 0; i <= n; ++i)
                two_prod(x[i], y[n - i], v[i], eh[i]);
#pragma unroll
            for (int q = 0; q < n * n; ++q)
                v[n + 1 + q] = errs[q];
            vec_sum(v);
            t[n] = v[0];
            double next[(n + 1) * (n + 1)];
#pragma unroll
            for (int q = 0; q < n + n * n; ++q)
                next[q] = v[q + 1];
#pragma unroll
            for (int i = 0; i <= n; ++i)
                next[n + n * n + i] = eh[i];
            mul_order<n + 1>(x, y, t, next);
        } else {
            double u = x[1] * y[MW - 1];
#pragma unroll
            for (int i = 2; i < MW; ++i)
                u = u + x[i] * y[MW - i];
#pragma unroll
            for (int q = 0; q < n * n; ++q)
                u = u + errs[q];
            t[MW] = u;
        }
    }

    static __device__ __forceinline__ void mul(const double (&x)[MW], const double (&y)[MW], double (&r)[MW])
    {
        double t[MW + 1], e0[1];
        two_prod(x[0], y[0], t[0], e0[0]);
        mul_order<1>(x, y, t, e0);
        renormalize(t, r);
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

namespace {

// Batched ordinary inner products: one wave per pair, lane l accumulating
// add(acc, mul(x_k, y_k)) over k = l, l + 64, .. in increasing k from zero;
// then the lanes' sums meet pairwise, lane l < h taking add(acc_l,
// acc_(l+h)) for h = 32, 16, .., 1.  Four pairs per 256-thread block.
template <int MW>
__global__ __launch_bounds__(256) void k_ordinary_dot(const double* __restrict__ X, int64_t psx,
                                                      const double* __restrict__ Y, int64_t psy,
                                                      double* __restrict__ out, int64_t pso, int64_t batch,
                                                      int64_t n)
{
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= batch)
        return;   // whole waves leave together
    const double* x = X + b * n;
    const double* y = Y + b * n;
    double acc[MW];
#pragma unroll
    for (int w = 0; w < MW; ++w)
        acc[w] = 0.0;
    for (int64_t k = lane; k < n; k += 64) {
        double xv[MW], yv[MW], p[MW];
#pragma unroll
        for (int w = 0; w < MW; ++w) {
            xv[w] = x[w * psx + k];
            yv[w] = y[w * psy + k];
        }
        Ordinary<MW>::mul(xv, yv, p);
        Ordinary<MW>::add(acc, p, acc);
    }
#pragma unroll
    for (int h = 32; h >= 1; h >>= 1) {
        double other[MW], sum[MW];
#pragma unroll
        for (int w = 0; w < MW; ++w)
            other[w] = __shfl_down(acc[w], h);
        Ordinary<MW>::add(acc, other, sum);
#pragma unroll
        for (int w = 0; w < MW; ++w)
            acc[w] = lane < h ? sum[w] : acc[w];
    }
    if (lane == 0)
#pragma unroll
        for (int w = 0; w < MW; ++w)
            out[w * pso + b] = acc[w];
}

}  // namespace

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
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace mdg
