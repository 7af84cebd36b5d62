// Batched INT8 inner products with the split in registers (the paper's
// experiment, Section 3; m = 1, 2, 4 words, the matrix-core kernel of
// dotmma.h taking m = 8 and 16): a workgroup takes one pair and a range of its
// depth; each lane cuts four entries of x and four of y into digits (four
// entries per 32-bit word, one per byte, by word placement) and multiplies
// them lane-wise with 4-way byte dot products, every pair of slices (s, t)
// with s + t < S into diagonal sum t + s.  The digits never reach memory,
// and no matrix-core output is thrown away: inner products have no reuse,
// so the contraction is bound by reading the words, not by multiplies.
//
// A lane's entries in step `it`: offsets it * 4 T + 256 w + 64 q + lane of
// the workgroup's range (T threads, wave w, byte q), so every load of a
// word is 512 contiguous bytes per wave.  The words of the next four
// entries of x and of y are in flight while one is cut.  Diagonal sums
// stay in int32 per lane: a step adds at most S 4-way products of digits
// of magnitude <= 128, S 2^16, and the host caps the steps per lane so the
// sums stay below 2^31 (lane_max_steps); the workgroup then adds its lanes
// in int64.
//
// Whole-pair mode (one workgroup per pair, a.full): the workgroup first
// finds the pair's two shared exponents (the largest frexp exponent of the
// nonzero leading words) and writes them with the pair's smallest leading
// exponents and, with a.mag, its magnitude product of the ratio
// certificate (sum_k qx_k qy_k, q the leading word's magnitude digit
// floor(|x^(0)| 2^(7 - E))); the certificate kernel reduces those to the
// call statistics (plain stores here: atomics of every pair on the same few
// words would queue behind each other).  With one depth range per pair the
// workgroup also folds its diagonal sums and rounds the pair's product
// (lane_round); with several, a zeroed D takes 64-bit atomic adds and
// launch_dot_final rounds.  Otherwise the exponents come from the exponent
// pass, and with several depth ranges per pair the sums are added into a
// zeroed D with 64-bit atomics.
#pragma once

#include "mdgemm_internal.h"
#include "renorm.h"
#include "split.h"
#include "ldslimbs.h"

#include <climits>

namespace mdg {
namespace {

// steps per lane whose int32 diagonal sums cannot overflow
constexpr int64_t lane_max_steps(int SC)
{
    return ((INT64_C(1) << 31) - 1) / ((int64_t)SC << 16);
}

// the words of entry e of a lane (base p, e inside iff e < lim, elast the
// last entry inside): every lane loads, from the clamped entry, and keeps
// zeros outside (no branch around the loads)
template <int MW>
__device__ __forceinline__ void lane_load(double (&w)[MW], const double* p, int64_t ps, int64_t e, int64_t lim,
                                          int64_t elast)
{
    const bool ok = e < lim;
    const double* q = p + (ok ? e : elast);
#pragma unroll
    for (int i = 0; i < MW; ++i) {
        const double v = q[i * ps];
        w[i] = ok ? v : 0.0;
    }
}

template <int Q, int MW, int SC, bool BAL>
__device__ __forceinline__ void lane_digits(const double (&w)[MW], int kn, int pad, uint32_t (&xs)[SC],
                                            LdsLimbs& L)
{
    if constexpr (BAL)
        digits_bal<Q, MW, SC>(w, kn, pad, xs, L);
    else
        digits_sm<Q, MW, SC>(w, kn, pad, xs, L);
}

// the pair's largest and smallest frexp exponents of the nonzero leading
// words of x and y (INT_MIN / INT_MAX if none), every thread of the workgroup
__device__ __forceinline__ void pair_exponents(const double* xb, const double* yb, int64_t n, int (&h)[4],
                                               int32_t* xch)
{
    const int t = threadIdx.x, nw = blockDim.x >> 6;
    int hx = INT_MIN, lx = INT_MAX, hy = INT_MIN, ly = INT_MAX;
    auto take = [](double v, int& h, int& l) {
        if (v != 0.0) {
            const int e = frexp_exponent(v);
            h = max(h, e);
            l = min(l, e);
        }
    };
    // every workgroup starts here at once: many loads per round trip, two
    // entries per 16-byte load where both vectors are 16-byte aligned (the
    // odd last entry, or everything otherwise, one at a time)
    int64_t k0 = 0;
    if (((reinterpret_cast<uintptr_t>(xb) | reinterpret_cast<uintptr_t>(yb)) & 15) == 0) {
        const int64_t n2 = n >> 1;
        const double2* x2 = reinterpret_cast<const double2*>(xb);
        const double2* y2 = reinterpret_cast<const double2*>(yb);
#pragma unroll 16
        for (int64_t i = t; i < n2; i += blockDim.x) {
            const double2 xv = x2[i], yv = y2[i];
            take(xv.x, hx, lx);
            take(xv.y, hx, lx);
            take(yv.x, hy, ly);
            take(yv.y, hy, ly);
        }
        k0 = 2 * n2;
    }
#pragma unroll 8
    for (int64_t k = k0 + t; k < n; k += blockDim.x) {
        take(xb[k], hx, lx);
        take(yb[k], hy, ly);
    }
    for (int o = 1; o < 64; o <<= 1) {
        hx = max(hx, __shfl_xor(hx, o));
        lx = min(lx, __shfl_xor(lx, o));
        hy = max(hy, __shfl_xor(hy, o));
        ly = min(ly, __shfl_xor(ly, o));
    }
    if ((t & 63) == 0) {
        xch[4 * (t >> 6) + 0] = hx;
        xch[4 * (t >> 6) + 1] = lx;
        xch[4 * (t >> 6) + 2] = hy;
        xch[4 * (t >> 6) + 3] = ly;
    }
    __syncthreads();
    h[0] = INT_MIN;
    h[1] = INT_MAX;
    h[2] = INT_MIN;
    h[3] = INT_MAX;
    for (int w = 0; w < nw; ++w) {
        h[0] = max(h[0], xch[4 * w + 0]);
        h[1] = min(h[1], xch[4 * w + 1]);
        h[2] = max(h[2], xch[4 * w + 2]);
        h[3] = min(h[3], xch[4 * w + 3]);
    }
}

// Exact fold X 2^(B (SC - S)) = sum_g D_g 2^(B (SC-1-g)) (D_g = 0 for g >= S:
// the container's positions, so every column is a compile-time index) into
// columns of 4 B bits, then greedy rounding of X 2^scale into m words.  A
// diagonal sum goes in as its low column's worth and the rest (arithmetic),
// each below 2^56 after its shift, so a column adds at most 8 of them.
template <int SC, int B>
__device__ __forceinline__ void lane_round(const int64_t* dsum, int scale, int m, double* out, int64_t pso)
{
    constexpr int CW = 4 * B, NC = (SC + 3) / 4 + 2;
    constexpr int NL = (CW * (NC - 1) + 64 + 31) / 32;
    int64_t x[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j)
        x[j] = 0;
#pragma unroll
    for (int g = 0; g < SC; ++g) {
        const int e = SC - 1 - g, col = e >> 2;
        const int64_t w = (int64_t)1 << (B * (e & 3));
        const int64_t d = dsum[g];
        x[col] += (int64_t)((uint64_t)d & ((1ull << CW) - 1)) * w;
        x[col + 1] += (d >> CW) * w;
    }
    carry_cols<CW>(x);
    uint32_t L[NL];
    double sgn = to_limbs<CW>(x, L) ? -1.0 : 1.0;
    for (int t = 0; t < m; ++t)
        out[t * pso] = rn_next(L, sgn, scale);
}

template <int MW, int SC, bool BAL>
__global__ __launch_bounds__(256) void k_dot_lane(LaneDotArgs a)
{
    static_assert(SC % 8 == 0 && SC <= 64, "diagonals reduced eight at a time, 8 per thread group");
    static_assert(MW <= 4, "four entries' words in flight per operand");
    constexpr int NS = store_limbs<SC, BAL>();
    __shared__ uint64_t limbs[4][NS][64];
    __shared__ int32_t red[4 * 8 * 64];
    __shared__ int32_t xch[16];
    __shared__ unsigned long long mxch[4];
    __shared__ int64_t dsum[SC];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = blockDim.x >> 6;
    const int64_t b = a.b0 + blockIdx.x;
    const int64_t c0 = (int64_t)blockIdx.y * a.chunk;
    const int64_t c1 = c0 + a.chunk < a.n ? c0 + a.chunk : a.n;
    const double* xb = a.X + b * a.ldx;
    const double* yb = a.Y + b * a.ldy;

    int Ex, Ey;
    if (a.full) {
        int h[4];
        pair_exponents(xb, yb, a.n, h, xch);
        Ex = (h[0] == INT_MIN ? 0 : h[0]) + a.eoff;
        Ey = (h[2] == INT_MIN ? 0 : h[2]) + a.eoff;
        if (t == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                a.ph[i * a.batch + b] = h[i];
        }
    } else {
        Ex = a.E[b];
        Ey = a.F[b];
    }

    constexpr int bits = BAL ? 8 : 7;
    const int S = a.S;
    const int knx = Ex + 1075 - bits * S, kny = Ey + 1075 - bits * S;
    const int pad = bits * (SC - S);
    const int Erx = Ex - a.eoff, Ery = Ey - a.eoff;
    const bool mag = a.mag != 0;

    LdsLimbs L{&limbs[wave][0][lane]};
#pragma unroll
    for (int i = 0; i < NS; ++i)
        L.col[i * 64] = 0;
    int32_t acc[SC];
#pragma unroll
    for (int g = 0; g < SC; ++g)
        acc[g] = 0;
    uint32_t macc = 0;

    const int64_t stepw = (int64_t)blockDim.x * 4;
    const int64_t nsteps = (c1 - c0 + stepw - 1) / stepw;
    const int64_t off = c0 + 256 * wave + lane;
    const int64_t lim = c1 - off;          // a lane's entry offset e is inside iff e < lim
    const int64_t elast = c1 - 1 - off;   // a lane's offset of the range's last entry
    const double* px = xb + off;
    const double* py = yb + off;
    // words of the next NB entries of x and of y in flight: entry g (byte
    // g % 4 of step g / 4) lives in buffer g % NB, refilled with entry g + NB
    // as soon as it is cut
    constexpr int NB = 4;
    double bx[NB][MW], by[NB][MW];
#pragma unroll
    for (int g = 0; g < NB; ++g) {
        lane_load(bx[g], px, a.psx, 64 * g, lim, elast);
        lane_load(by[g], py, a.psy, 64 * g, lim, elast);
    }
    for (int64_t it = 0; it < nsteps; ++it) {
        uint32_t xs[SC], ys[SC], mx = 0, my = 0;
#pragma unroll
        for (int s = 0; s < SC; ++s) {
            xs[s] = 0;
            ys[s] = 0;
        }
        const int64_t e0 = it * stepw;
        unroll<4>([&](auto QQ) {
            constexpr int q = decltype(QQ)::value, slot = q % NB;
            // entry q + NB of this step's sequence: (q + NB) / 4 steps on, byte (q + NB) % 4
            const int64_t en = e0 + ((q + NB) / 4) * stepw + 64 * ((q + NB) % 4);
            // one entry cut at a time, its buffer refilled after it
            if (mag)
                mx = byte_insert<q, 0>(mx, mag_digit(bx[slot][0], Erx));
            lane_digits<q, MW, SC, BAL>(bx[slot], knx, pad, xs, L);
            pin(xs, mx);
            lane_load(bx[slot], px, a.psx, en, lim, elast);
            if (mag)
                my = byte_insert<q, 0>(my, mag_digit(by[slot][0], Ery));
            lane_digits<q, MW, SC, BAL>(by[slot], kny, pad, ys, L);
            pin(ys, my);
            lane_load(by[slot], py, a.psy, en, lim, elast);
        });
        if constexpr (BAL) {
#pragma unroll
            for (int s = 0; s < SC; ++s) {
                xs[s] ^= 0x80808080u;
                ys[s] ^= 0x80808080u;
            }
        }
        macc = __builtin_amdgcn_udot4(mx, my, macc, false);
        unroll<SC>([&](auto G) {
            constexpr int g = decltype(G)::value;
            if (g < S) {
                unroll<g + 1>([&](auto Sx) {
                    constexpr int s = decltype(Sx)::value;
                    acc[g] = __builtin_amdgcn_sdot4((int)xs[s], (int)ys[g - s], acc[g], false);
                });
            }
        });
    }

    // the workgroup's diagonal sums, eight at a time: lanes' values through
    // LDS, 8 nw threads per diagonal adding 8 values each, then shuffles
    const int parts = 8 * nw, gl = t / parts, part = t % parts;
    unroll<SC / 8>([&](auto G0) {
        constexpr int g0 = 8 * decltype(G0)::value;
#pragma unroll
        for (int gg = 0; gg < 8; ++gg)
            red[(wave * 8 + gg) * 64 + lane] = acc[g0 + gg];
        __syncthreads();
        int64_t s = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int f = part * 8 + i;
            s += red[((f >> 6) * 8 + gl) * 64 + (f & 63)];
        }
        for (int o = 1; o < parts; o <<= 1)
            s += __shfl_xor(s, o);
        if (part == 0) {
            if (a.atomic) {
                if (g0 + gl < S)
                    atomicAdd(reinterpret_cast<unsigned long long*>(a.D + (int64_t)(g0 + gl) * a.batch + b),
                              (unsigned long long)s);
            } else {
                dsum[g0 + gl] = g0 + gl < S ? s : 0;
            }
        }
        __syncthreads();
    });
    if (!a.atomic && t == 0)
        lane_round<SC, bits>(dsum, Ex + Ey - bits * (SC + 1), MW, a.out + b, a.pso);
    if (mag) {
        unsigned long long mm = macc;
        for (int o = 1; o < 64; o <<= 1)
            mm += __shfl_xor(mm, o);
        if (lane == 0)
            mxch[wave] = mm;
        __syncthreads();
        if (t == 0) {
            unsigned long long tot = 0;
            for (int w = 0; w < nw; ++w)
                tot += mxch[w];
            a.pm[b] = tot;
        }
    }
}

// The statistics pass of the slice rule for inner products, one workgroup
// per pair: the pair's shared exponents (E, F: plus eoff) and its largest
// and smallest leading exponents (ph, as whole-pair mode writes them), and
// with pm its magnitude product sum_k qx_k qy_k.  One read of the leading
// words serves both (for the first kPreCache values of each thread and
// operand): a value's frexp exponent e and top seven bits t = floor(|x|
// 2^(7 - e)) stay in a register, and once the vector's exponent E is known
// its magnitude digit floor(|x| 2^(7 - E)) is t >> (E - e) (a floor of a
// floor by a power of two); values past the cache are read again.
constexpr int kPreCache = 32;

// (e + 2048) 2^8 + t, or 0 for a zero word; h, l: running largest and
// smallest frexp exponent
__device__ __forceinline__ uint32_t pre_pack(double x, int& h, int& l)
{
    if (x == 0.0)
        return 0u;
    const int e = frexp_exponent(x);
    h = max(h, e);
    l = min(l, e);
    return ((uint32_t)(e + 2048) << 8) | mag_digit(x, e);
}

__device__ __forceinline__ uint32_t pre_digit(uint32_t c, int E)
{
    const int d = E - ((int)(c >> 8) - 2048);
    return c == 0u || d > 7 ? 0u : (c & 255u) >> d;
}

__global__ __launch_bounds__(256) void k_dot_pre(const double* X, int64_t ldx, const double* Y, int64_t ldy,
                                                 int64_t batch, int64_t n, int eoff, int32_t* E, int32_t* F,
                                                 int32_t* ph, unsigned long long* pm)
{
    __shared__ int32_t xch[16];
    __shared__ unsigned long long mxch[4];
    const int t = threadIdx.x;
    const int64_t b = blockIdx.x;
    const double* xb = X + b * ldx;
    const double* yb = Y + b * ldy;
    int hx = INT_MIN, lx = INT_MAX, hy = INT_MIN, ly = INT_MAX;
    uint32_t cx[kPreCache], cy[kPreCache];
#pragma unroll
    for (int i = 0; i < kPreCache; ++i) {
        const int64_t k = t + (int64_t)i * 256;
        const bool ok = k < n;
        const double x = ok ? xb[k] : 0.0, y = ok ? yb[k] : 0.0;
        cx[i] = pre_pack(x, hx, lx);
        cy[i] = pre_pack(y, hy, ly);
    }
    const int64_t k1 = (int64_t)kPreCache * 256;
    for (int64_t k = k1 + t; k < n; k += 256) {
        pre_pack(xb[k], hx, lx);
        pre_pack(yb[k], hy, ly);
    }
    for (int o = 1; o < 64; o <<= 1) {
        hx = max(hx, __shfl_xor(hx, o));
        lx = min(lx, __shfl_xor(lx, o));
        hy = max(hy, __shfl_xor(hy, o));
        ly = min(ly, __shfl_xor(ly, o));
    }
    if ((t & 63) == 0) {
        xch[4 * (t >> 6) + 0] = hx;
        xch[4 * (t >> 6) + 1] = lx;
        xch[4 * (t >> 6) + 2] = hy;
        xch[4 * (t >> 6) + 3] = ly;
    }
    __syncthreads();
    int h[4] = {INT_MIN, INT_MAX, INT_MIN, INT_MAX};
    for (int w = 0; w < 4; ++w) {
        h[0] = max(h[0], xch[4 * w + 0]);
        h[1] = min(h[1], xch[4 * w + 1]);
        h[2] = max(h[2], xch[4 * w + 2]);
        h[3] = min(h[3], xch[4 * w + 3]);
    }
    const int Ex = h[0] == INT_MIN ? 0 : h[0], Ey = h[2] == INT_MIN ? 0 : h[2];
    if (t == 0) {
        E[b] = Ex + eoff;
        F[b] = Ey + eoff;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            ph[i * batch + b] = h[i];
    }
    if (!pm)
        return;
    unsigned long long acc = 0;
#pragma unroll
    for (int i = 0; i < kPreCache; ++i)
        acc += (unsigned long long)(pre_digit(cx[i], Ex) * pre_digit(cy[i], Ey));
    for (int64_t k = k1 + t; k < n; k += 256)
        acc += (unsigned long long)(mag_digit(xb[k], Ex) * mag_digit(yb[k], Ey));
    for (int o = 1; o < 64; o <<= 1)
        acc += __shfl_xor(acc, o);
    if ((t & 63) == 0)
        mxch[t >> 6] = acc;
    __syncthreads();
    if (t == 0)
        pm[b] = mxch[0] + mxch[1] + mxch[2] + mxch[3];
}

// SC in [LO, HI], a multiple of 8
template <int MW, int HI, int LO>
struct DispatchLane {
    static hipError_t run(const LaneDotArgs& a0, int SC, bool bal, int nw, int64_t nch, hipStream_t st)
    {
        if (SC == HI) {
            LaneDotArgs a = a0;
            for (int64_t b0 = 0; b0 < a.batch; b0 += INT64_C(1) << 30) {
                a.b0 = b0;
                const dim3 grid((unsigned)std::min<int64_t>(a.batch - b0, INT64_C(1) << 30), (unsigned)nch);
                if (bal)
                    hipLaunchKernelGGL((k_dot_lane<MW, HI, true>), grid, dim3(64 * nw), 0, st, a);
                else
                    hipLaunchKernelGGL((k_dot_lane<MW, HI, false>), grid, dim3(64 * nw), 0, st, a);
                const hipError_t e = hipGetLastError();
                if (e != hipSuccess)
                    return e;
            }
            return hipSuccess;
        }
        if constexpr (HI - 8 >= LO)
            return DispatchLane<MW, HI - 8, LO>::run(a0, SC, bal, nw, nch, st);
        return hipErrorInvalidValue;
    }
};

}  // namespace
}  // namespace mdg
