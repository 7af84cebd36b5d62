// Magnitude products for the ratio certificate (all outputs of a matrix
// product, or the pairs of a batch of inner products) and the batched
// inner-product contraction and fold.
#include "slice_common.h"
#include "dotlane.h"
#include "dotmma.h"

#include <climits>

namespace mdg {
namespace {

// min over the outputs of P_ij = sum_k qA_ik qB_kj, depth up to 2^11 depth
// fragments (INT32 exact: one fragment adds below 64 * 127^2 < 2^20): a wave
// computes RX x CY fragments (16 RX x 16 CY outputs), a workgroup of four
// waves 32 RX x 32 CY.  The fragments of the next D depth steps are in
// flight while the current one multiplies.  A wave issues RX + CY fragment
// loads for RX CY matrix instructions per step, so wider tiles relieve the
// texture path once there are enough of them to fill the chip.  Row or
// column blocks past the padded arrays read through empty descriptors
// (zeros; those outputs are not counted).
template <int RX, int CY, int D>
__global__ __launch_bounds__(256) void k_mag_min_short(const v4i* __restrict__ qA,
                                                       const v4i* __restrict__ qB, int64_t M,
                                                       int64_t N, int64_t nkc,
                                                       unsigned long long* minP, int64_t y0)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t rb0 = ((y0 + blockIdx.y) * 2 + (wave >> 1)) * RX;
    const int64_t cb0 = ((int64_t)blockIdx.x * 2 + (wave & 1)) * CY;
    const int64_t nrb = 2 * ((M + kTile - 1) / kTile), ncb = 2 * ((N + kTile - 1) / kTile);
    const uint64_t bytes = (uint64_t)nkc * 1024;
    FragStream SA[RX], SB[CY];
#pragma unroll
    for (int x = 0; x < RX; ++x)
        SA[x] = frag_stream((const char*)qA + (rb0 + x) * bytes, rb0 + x < nrb ? bytes : 0, lane);
#pragma unroll
    for (int y = 0; y < CY; ++y)
        SB[y] = frag_stream((const char*)qB + (cb0 + y) * bytes, cb0 + y < ncb ? bytes : 0, lane);
    v4i acc[RX][CY], pa[D][RX], pb[D][CY];
#pragma unroll
    for (int x = 0; x < RX; ++x)
#pragma unroll
        for (int y = 0; y < CY; ++y)
            acc[x][y] = v4i{0, 0, 0, 0};
#pragma unroll
    for (int d = 0; d < D; ++d) {
#pragma unroll
        for (int x = 0; x < RX; ++x)
            pa[d][x] = SA[x](d * 1024u);
#pragma unroll
        for (int y = 0; y < CY; ++y)
            pb[d][y] = SB[y](d * 1024u);
    }
    for (int64_t kc = 0; kc < nkc; kc += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            // depth steps past nkc read zeros and add nothing
#pragma unroll
            for (int x = 0; x < RX; ++x)
#pragma unroll
                for (int y = 0; y < CY; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_i32_16x16x64_i8(pa[d][x], pb[d][y], acc[x][y],
                                                                      0, 0, 0);
            const uint32_t nxt = (uint32_t)(kc + d + D) * 1024u;
#pragma unroll
            for (int x = 0; x < RX; ++x)
                pa[d][x] = SA[x](nxt);
#pragma unroll
            for (int y = 0; y < CY; ++y)
                pb[d][y] = SB[y](nxt);
        }
    }
    unsigned long long best = ~0ull;
#pragma unroll
    for (int x = 0; x < RX; ++x)
#pragma unroll
        for (int y = 0; y < CY; ++y)
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                const int64_t i = (rb0 + x) * 16 + FormI8::row(lane, o);
                const int64_t j = (cb0 + y) * 16 + (lane & 15);
                const unsigned long long v = (unsigned long long)(uint32_t)acc[x][y][o];
                if (i < M && j < N && v < best)
                    best = v;
            }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(best, off);
        best = o < best ? o : best;
    }
    if (lane == 0 && best != ~0ull)
        atomicMin(minP, best);
}

// The same for longer depths (not pipelined): partial sums carried into
// int64 every 2^11 depth fragments.
__global__ __launch_bounds__(256) void k_mag_min(const v4i* __restrict__ qA,
                                                 const v4i* __restrict__ qB, int64_t M, int64_t N,
                                                 int64_t nkc, unsigned long long* minP, int64_t y0)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t rb0 = ((y0 + blockIdx.y) * 2 + (wave >> 1)) * 4;
    const int64_t cb0 = ((int64_t)blockIdx.x * 2 + (wave & 1)) * 4;
    const int64_t nrb = (M + 15) / 16, ncb = (N + 15) / 16;
    v4i acc[4][4];
    int64_t tot[4][4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            acc[x][y] = v4i{0, 0, 0, 0};
#pragma unroll
            for (int o = 0; o < 4; ++o)
                tot[x][y][o] = 0;
        }
    for (int64_t kc = 0; kc < nkc; ++kc) {
        v4i a[4], b[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const int64_t rb = min(rb0 + x, nrb - 1);
            const int64_t cb = min(cb0 + x, ncb - 1);
            a[x] = qA[(rb * nkc + kc) * 64 + lane];
            b[x] = qB[(cb * nkc + kc) * 64 + lane];
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
                acc[x][y] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[x], b[y], acc[x][y], 0, 0, 0);
        if ((kc & 2047) == 2047 || kc == nkc - 1) {
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) {
#pragma unroll
                    for (int o = 0; o < 4; ++o)
                        tot[x][y][o] += acc[x][y][o];
                    acc[x][y] = v4i{0, 0, 0, 0};
                }
        }
    }
    unsigned long long best = ~0ull;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                const int64_t i = (rb0 + x) * 16 + FormI8::row(lane, o);
                const int64_t j = (cb0 + y) * 16 + (lane & 15);
                if (i < M && j < N && (unsigned long long)tot[x][y][o] < best)
                    best = (unsigned long long)tot[x][y][o];
            }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(best, off);
        best = o < best ? o : best;
    }
    if (lane == 0 && best != ~0ull)
        atomicMin(minP, best);
}

// ---------------------------------------------------------------------------
// Batched inner products out_b = sum_k x_bk y_bk (the paper's experiment,
// Section 3): both operands are split with the vectors as rows, so the slice
// product of row block rb of X with row block rb of Y holds pair rb*16 + i
// at its diagonal entry (i, i); the other 15/16 of the entries are
// discarded, which costs matrix-core time the inner products do not miss.

// Diagonal sums t0 .. t0+G-1 of the 16 pairs of row block y0 + blockIdx.y over the
// depth fragments [c0, c0 + range), range within one exactness chunk.  The
// partial sums are added into D with 64-bit integer atomics: integer
// addition is associative, so D does not depend on their order.
template <class Form, int G>
__global__ __launch_bounds__(64) void k_dot_band(DotArgs a, int64_t y0)
{
    typedef typename Form::frag Frag;
    typedef typename Form::acc Acc;
    const int lane = threadIdx.x;
    const int64_t rb = y0 + blockIdx.y;
    const int64_t c0 = (int64_t)blockIdx.x * a.range, c1 = min(c0 + a.range, a.nkc);
    const int t0 = (int)blockIdx.z * G;
    const int64_t fstride = (int64_t)a.S * 64;
    const Frag* Xb = (const Frag*)a.X + rb * a.nkc * fstride + lane;
    const Frag* Yb = (const Frag*)a.Y + rb * a.nkc * fstride + lane;
    Acc acc[G];
#pragma unroll
    for (int g = 0; g < G; ++g)
        acc[g] = Form::zero();
    if constexpr (Form::kPipelined && G > 3) {
        if (c1 > c0)
            band_run<Form, G, 3>(acc, Xb, Yb, fstride, c0, c1, t0);
    } else {
        for (int64_t kc = c0; kc < c1; ++kc)
            band_chunk<Form, G>(acc, Xb + kc * fstride, Yb + kc * fstride, t0);
    }
    const int64_t b = rb * 16 + (lane & 15);
    if constexpr (std::is_same<Form, FormF64Lane>::value) {
        // lanes l, l+16, l+32, l+48 hold the four depth quarters of pair l%16
#pragma unroll
        for (int g = 0; g < G; ++g) {
            double v = acc[g];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (lane < 16 && b < a.batch)
                atomicAdd(reinterpret_cast<unsigned long long*>(a.D + (int64_t)(t0 + g) * a.batch + b),
                          (unsigned long long)(int64_t)v);
        }
    } else if (b < a.batch) {
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int o = 0; o < 4; ++o)
                if (Form::row(lane, o) == (lane & 15))
                    atomicAdd(reinterpret_cast<unsigned long long*>(a.D + (int64_t)(t0 + g) * a.batch + b),
                              (unsigned long long)Form::value(acc[g], o));
    }
}

__global__ void k_fill_zero_i64(int64_t* p, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0;
}

// Exact fold X_b = sum_t D_tb 2^(beta (S-1-t)) into LDS columns (one thread
// per pair) and greedy rounding of X_b 2^(E_b + F_b - beta (S+1)) into m words.
__global__ __launch_bounds__(256) void k_dot_final(const int64_t* __restrict__ D,
                                                   const int32_t* __restrict__ E,
                                                   const int32_t* __restrict__ F, int64_t batch,
                                                   int S, int beta, int ncol, int m, double* out,
                                                   int64_t pso)
{
    extern __shared__ int64_t lds[];
    const int t = threadIdx.x;
    const int64_t b = (int64_t)blockIdx.x * 256 + t;
    int64_t* cols = lds + t;
    for (int q = 0; q < ncol; ++q)
        cols[q * 256] = 0;
    const bool ok = b < batch;
    if (ok)
        for (int s = 0; s < S; ++s)
            fold_add(cols, 0, D[(int64_t)s * batch + b], beta * (S - 1 - s));
    const int scale = ok ? E[b] + F[b] - beta * (S + 1) : 0;
    renormalise(cols, ncol, scale, m, ok ? out + b : nullptr, pso, ok);
}

// min over the pairs of P_b = sum_k qX_bk qY_bk (magnitude digits in [0, 127],
// fragment order: lane l holds row l%16 at depths 16(l/16) .. +15).  One wave
// per block of 16 pairs.
__global__ __launch_bounds__(64) void k_mag_min_diag(const v4i* __restrict__ qX,
                                                     const v4i* __restrict__ qY, int64_t batch,
                                                     int64_t nkc, unsigned long long* minP)
{
    const int lane = threadIdx.x;
    const int64_t rb = blockIdx.x;
    const v4i* x = qX + rb * nkc * 64 + lane;
    const v4i* y = qY + rb * nkc * 64 + lane;
    unsigned long long acc = 0;
#pragma unroll 4
    for (int64_t kc = 0; kc < nkc; ++kc) {
        const v4i u = x[kc * 64], v = y[kc * 64];
        uint32_t sum = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w)
#pragma unroll
            for (int by = 0; by < 32; by += 8)
                sum += (((uint32_t)u[w] >> by) & 0xffu) * (((uint32_t)v[w] >> by) & 0xffu);
        acc += sum;
    }
    // lanes l, l+16, l+32, l+48 hold the four depth quarters of row l%16
    acc += __shfl_xor(acc, 16);
    acc += __shfl_xor(acc, 32);
    unsigned long long best = rb * 16 + (lane & 15) < batch ? acc : ~0ull;
    for (int off = 8; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(best, off);
        best = o < best ? o : best;
    }
    if (lane == 0 && best != ~0ull)
        atomicMin(minP, best);
}

template <class Form, int G>
struct DispatchDot {
    static hipError_t run(const DotArgs& a, hipStream_t st)
    {
        if (a.band == G) {
            // pair blocks on the grid's second dimension, at most 65535 per launch
            const int64_t nyb = (a.batch + 15) / 16, gx = (a.nkc + a.range - 1) / a.range;
            if (gx > 0x7fffffff)
                return hipErrorInvalidValue;
            for (int64_t y0 = 0; y0 < nyb; y0 += 65535) {
                dim3 grid((unsigned)gx, (unsigned)std::min<int64_t>(nyb - y0, 65535), (unsigned)a.nbands);
                hipLaunchKernelGGL((k_dot_band<Form, G>), grid, dim3(64), 0, st, a, y0);
                const hipError_t e = hipGetLastError();
                if (e != hipSuccess)
                    return e;
            }
            return hipSuccess;
        }
        return DispatchDot<Form, G - 1>::run(a, st);
    }
};
template <class Form>
struct DispatchDot<Form, 0> {
    static hipError_t run(const DotArgs&, hipStream_t) { return hipErrorInvalidValue; }
};

}  // namespace

hipError_t launch_mag_min(const void* qA, const void* qB, int64_t M, int64_t N, int64_t nkc,
                          unsigned long long* minP, hipStream_t st)
{
    // 256 x 256 outputs per workgroup where that still gives every compute
    // unit one (4096^2 outputs and up), else 128 x 128
    const bool wide = nkc <= 2048 && ((N + 255) / 256) * ((M + 255) / 256) >= 256;
    const int64_t tile = wide ? 256 : 128;
    const int64_t gx = (N + tile - 1) / tile, ny = (M + tile - 1) / tile;
    if (gx > 0x7fffffff)
        return hipErrorInvalidValue;
    for (int64_t y0 = 0; y0 < ny; y0 += 65535) {
        dim3 grid((unsigned)gx, (unsigned)std::min<int64_t>(ny - y0, 65535));
        if (wide)
            hipLaunchKernelGGL((k_mag_min_short<8, 8, 2>), grid, dim3(256), 0, st, (const v4i*)qA,
                               (const v4i*)qB, M, N, nkc, minP, y0);
        else if (nkc <= 2048)
            hipLaunchKernelGGL((k_mag_min_short<4, 4, 4>), grid, dim3(256), 0, st, (const v4i*)qA,
                               (const v4i*)qB, M, N, nkc, minP, y0);
        else
            hipLaunchKernelGGL(k_mag_min, grid, dim3(256), 0, st, (const v4i*)qA, (const v4i*)qB, M, N,
                               nkc, minP, y0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_dot_diag(const DotArgs& a, int form_int8, hipStream_t st)
{
    if (form_int8)
        return DispatchDot<FormI8, kTriMaxI8>::run(a, st);
    return DispatchDot<FormF64Lane, kGmaxF64>::run(a, st);
}

hipError_t launch_fill_zero_i64(int64_t* p, int64_t n, hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    if (blocks > 0)
        hipLaunchKernelGGL(k_fill_zero_i64, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_dot_final(const int64_t* D, const int32_t* E, const int32_t* F, int64_t batch,
                            int S, int beta, int ncol, int m, double* out, int64_t pso,
                            hipStream_t st)
{
    const size_t lds = (size_t)ncol * 256 * sizeof(int64_t);
    if (lds > 64 * 1024) {
        const hipError_t e = ensure_dynamic_lds((const void*)k_dot_final, lds);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_dot_final, dim3((unsigned)((batch + 255) / 256)), dim3(256), lds, st, D, E,
                       F, batch, S, beta, ncol, m, out, pso);
    return hipGetLastError();
}

hipError_t launch_mag_min_diag(const void* qX, const void* qY, int64_t batch, int64_t nkc,
                               unsigned long long* minP, hipStream_t st)
{
    hipLaunchKernelGGL(k_mag_min_diag, dim3((unsigned)((batch + 15) / 16)), dim3(64), 0, st,
                       (const v4i*)qX, (const v4i*)qY, batch, nkc, minP);
    return hipGetLastError();
}

hipError_t launch_dot_pre(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t batch, int64_t n,
                          int eoff, int32_t* E, int32_t* F, int32_t* ph, unsigned long long* pm, hipStream_t st)
{
    if (batch > 0x7fffffff)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dot_pre, dim3((unsigned)batch), dim3(256), 0, st, X, ldx, Y, ldy, batch, n, eoff, E,
                       F, ph, pm);
    return hipGetLastError();
}

void lane_sc_range(int m, int& lo, int& hi)
{
    switch (m) {
    case 1: lo = 8; hi = 24; return;
    case 2: lo = 8; hi = 32; return;
    case 4: lo = 8; hi = 48; return;
    default: lo = hi = 0; return;
    }
}

void mma_sc_range(int m, int& lo, int& hi)
{
    lo = m == 16 ? 80 : m == 8 ? 32 : 0;
    hi = m == 16 ? 128 : m == 8 ? 64 : 0;
}

int64_t mma_depth_limit()
{
    return kMmaMaxDepth;
}

hipError_t launch_dot_mma(const LaneDotArgs& a, int m, int SC, bool balanced, int64_t nch, hipStream_t st)
{
    switch (m) {
    case 8: return launch_dot_mma_m8(a, SC, balanced, nch, st);
    case 16: return launch_dot_mma_m16(a, SC, balanced, nch, st);
    default: return hipErrorInvalidValue;
    }
}

int64_t lane_steps_limit(int SC)
{
    return lane_max_steps(SC);
}

hipError_t launch_dot_lane(const LaneDotArgs& a, int m, int SC, bool balanced, int nw, int64_t nch,
                           hipStream_t st)
{
    switch (m) {
    case 1: return launch_dot_lane_m1(a, SC, balanced, nw, nch, st);
    case 2: return launch_dot_lane_m2(a, SC, balanced, nw, nch, st);
    case 4: return launch_dot_lane_m4(a, SC, balanced, nw, nch, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mdg
