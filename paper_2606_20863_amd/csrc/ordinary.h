// Ordinary m-double arithmetic on the GPU: the error-free transformations,
// the floating-point expansion operations (any word count a power of two)
// and the batched inner-product kernel, shared by the units that instantiate
// them for the word counts they serve (the paper's comparison baseline,
// Section 1, Table 1, and the "ordinary" columns of Table 2).
#pragma once

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

// m = 8 and 16: floating-point expansion arithmetic (CAMPARY's building
// blocks, Joldes, Muller, Popescu and Tucker): VecSum (TwoSum of each term
// with the running sum, from the last term up), VecSumErrBranch (Fast2Sum
// down the terms, a new output word whenever the error is nonzero, until m
// words are out), addition by merging both operands' words by decreasing
// magnitude (Batcher's odd-even merge network: fixed compare-exchanges, no
// branches) and renormalising, multiplication by the product of expansions
// truncated at order m (TwoProd of every product of order n < m, each
// order's high parts and the carried errors through VecSum, the order-m
// products and the remaining errors added plainly, then renormalised).

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
}  // namespace mdg
