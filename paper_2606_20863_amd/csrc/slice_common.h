// Shared device code of the slice contraction kernels: operand forms,
// fragment streams, the banded contraction loops, the LDS fold and its
// renormalisation, and the workgroup-to-tile mapping.
//
// Slice contraction, exact fold and renormalisation (one fused kernel).
//
// For every output entry the kernel forms the diagonal sums
//   D_t = sum_{s+u=t} sum_k dA_{ik,s} dB_{kj,u},  t = 0..S-1,
// the paper's convolution sums s_i (Section 2; the Conclusions recast them
// as matrix products, which here run on the matrix cores), adds
//   X = sum_t D_t 2^(beta (S-1-t))
// exactly in a multi-word integer, and rounds C~ = X 2^(E_i + F_j - beta(S+1))
// greedily to nearest into m words (one renormalisation per entry, the
// paper's postponed renormalisation).
//
// Work split: a workgroup of 4 waves owns a 32 x 32 block of C, each wave a
// 16 x 16 tile.  Diagonals are processed in bands of G consecutive t; for a
// band starting at t0 (a multiple of G) the wave keeps G accumulators and a
// sliding window of G B-fragments: at step s it multiplies A_s with
// B_{t0+g-s} into accumulator g, so each A fragment is loaded once per band
// and each B fragment enters the window once.  The window slot of B_u is
// u mod G, which the fully unrolled steps resolve at compile time.
//
// Exactness: INT8 products accumulate in INT32 and FP64 products in FP64;
// the host chooses the depth chunk kcc so that every diagonal sum of a chunk
// stays below 2^31 (INT8) or 2^53 (FP64).  After each chunk the accumulators
// are added into the exact fold.
//
// The banded kernels keep the fold in LDS: per wave, per output, ncol signed
// 64-bit columns with weights 2^(32 q) (carry-save; normalised once at the
// end).  The whole-triangle INT8 kernel, whose bit positions are all known at
// compile time, keeps it in registers and renormalises there.
#pragma once

#include "mdgemm_internal.h"
#include "renorm.h"

#include <algorithm>
#include <type_traits>

namespace mdg {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

struct FormI8 {
    typedef v4i frag;
    typedef v4i acc;
    static constexpr bool kPipelined = true;
    static __device__ __forceinline__ acc mma(const frag& a, const frag& b, const acc& c)
    {
        return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ acc zero() { return acc{0, 0, 0, 0}; }
    static __device__ __forceinline__ int64_t value(const acc& c, int o) { return (int64_t)c[o]; }
    // accumulator element o of lane l is row 4 (l/16) + o, column l%16
    static __device__ __forceinline__ int row(int lane, int o) { return 4 * (lane >> 4) + o; }
};

struct FormF64 {
    typedef v4d frag;   // four depth steps of 4
    typedef v4d acc;
    static constexpr bool kPipelined = false;
    static __device__ __forceinline__ acc mma(const frag& a, const frag& b, acc c)
    {
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[2], b[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3], b[3], c, 0, 0, 0);
        return c;
    }
    static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
    // exact: an integer of magnitude below 2^53
    static __device__ __forceinline__ int64_t value(const acc& c, int o) { return (int64_t)c[o]; }
    // accumulator element o of lane l is row 4 o + l/16, column l%16
    static __device__ __forceinline__ int row(int lane, int o) { return 4 * o + (lane >> 4); }
};

// FP64 digits multiplied lane by lane on the vector units: lane l's four
// doubles of an A fragment and of a B fragment sit at the same row l%16 and
// depths, so for the batched inner products (row block of X against the same
// row block of Y) the lane-wise products are exactly the pair products, with
// none of the 16 x 16 tile's off-diagonal work.  The accumulator is one
// double per lane and diagonal; exact while the sums stay below 2^53.
struct FormF64Lane {
    typedef v4d frag;
    typedef double acc;
    static constexpr bool kPipelined = false;
    static __device__ __forceinline__ acc mma(const frag& a, const frag& b, acc c)
    {
        c = __builtin_fma(a[0], b[0], c);
        c = __builtin_fma(a[1], b[1], c);
        c = __builtin_fma(a[2], b[2], c);
        return __builtin_fma(a[3], b[3], c);
    }
    static __device__ __forceinline__ acc zero() { return 0.0; }
};

// One depth chunk of one band: diagonals t0..t0+G-1, t0 a multiple of G.
// A and B point at slice 0 of the chunk (plus the lane); slice s is at +64 s.
template <class Form, int G>
__device__ __forceinline__ void band_chunk(typename Form::acc (&acc)[G],
                                           const typename Form::frag* __restrict__ A,
                                           const typename Form::frag* __restrict__ B, int t0)
{
    typedef typename Form::frag Frag;
    Frag win[G];
#pragma unroll
    for (int g = 0; g < G; ++g)
        win[g] = B[(t0 + g) * 64];
    // steps s = 0 .. t0-1: every diagonal of the band has a partner
    for (int s0 = 0; s0 < t0; s0 += G) {
#pragma unroll
        for (int r = 0; r < G; ++r) {
            const int s = s0 + r;
            if (r > 0 || s0 > 0)
                win[(G - r) % G] = B[(t0 - s) * 64];
            const Frag a = A[s * 64];
#pragma unroll
            for (int g = G - 1; g >= 0; --g)
                acc[g] = Form::mma(a, win[(g - r + G) % G], acc[g]);
        }
    }
    // step s = t0: B_0 enters
    if (t0 > 0)
        win[0] = B[0];
    {
        const Frag a = A[t0 * 64];
#pragma unroll
        for (int g = G - 1; g >= 0; --g)
            acc[g] = Form::mma(a, win[g], acc[g]);
    }
    // steps s = t0 + p: only diagonals g >= p have a partner
#pragma unroll
    for (int p = 1; p < G; ++p) {
        const Frag a = A[(t0 + p) * 64];
#pragma unroll
        for (int g = G - 1; g >= p; --g)
            acc[g] = Form::mma(a, win[g - p], acc[g]);
    }
}

// Buffer-resource loads of INT8 fragments: one descriptor per wave spans the
// wave's row block of fragments; the lane's 16 bytes sit at lane * 16 and the
// fragment at a scalar byte offset, so no per-load address registers are
// needed.  Offsets past the descriptor's range read zeros.
struct FragStream {
    __amdgpu_buffer_rsrc_t rsrc;
    int voff;
    __device__ __forceinline__ v4i operator()(uint32_t soff) const
    {
        return __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff, (int)soff, 0);
    }
};

__device__ __forceinline__ FragStream frag_stream(const void* base, uint64_t bytes, int lane)
{
    FragStream f;
    // word 3 of a raw (untyped) buffer descriptor on gfx9-class targets
    f.rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0,
                                               (int)(bytes > 0xffffffffull ? 0xffffffffu : bytes),
                                               0x00020000);
    f.voff = lane * 16;
    return f;
}

// Software-pipelined run of depth chunks [c0, c1) for one band (t0 a
// multiple of G, P < G).  A step s of a chunk uses A_s and, for 1 <= s <= t0,
// the entering fragment B_{t0-s}; both are loaded P steps ahead into a small
// ring (pa, pb), across chunk boundaries.  The next chunk's window is loaded
// one fragment per tail step into the slot whose last use was the step
// before.  Scheduling barriers keep each step's loads ahead of its matrix
// instructions.  Loads past the last chunk re-read the current chunk.
template <class Form, int G, int P>
__device__ __forceinline__ void band_run(typename Form::acc (&acc)[G],
                                         const typename Form::frag* __restrict__ A,
                                         const typename Form::frag* __restrict__ B,
                                         int64_t fstride, int64_t c0, int64_t c1, int t0)
{
    static_assert(P >= 1 && P < G, "prefetch distance must be below the band width");
    typedef typename Form::frag Frag;
    const Frag* Ak = A + c0 * fstride;
    const Frag* Bk = B + c0 * fstride;
    Frag win[G], pa[P], pb[P];
#pragma unroll
    for (int g = G - 1; g >= 0; --g)
        win[g] = Bk[(t0 + g) * 64];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        pa[q] = Ak[q * 64];
        pb[q] = (q >= 1 && q <= t0) ? Bk[(t0 - q) * 64] : pa[q];
    }
    for (int64_t kc = c0; kc < c1; ++kc) {
        const bool more = kc + 1 < c1;
        const Frag* An = more ? Ak + fstride : Ak;
        const Frag* Bn = more ? Bk + fstride : Bk;
        // steps s = 0 .. t0-1
        for (int s0 = 0; s0 < t0; s0 += G) {
#pragma unroll
            for (int r = 0; r < G; ++r) {
                const int s = s0 + r;
                const Frag a = pa[0];
                const Frag b = pb[0];
#pragma unroll
                for (int q = 0; q + 1 < P; ++q) {
                    pa[q] = pa[q + 1];
                    pb[q] = pb[q + 1];
                }
                pa[P - 1] = Ak[(s + P) * 64];
                if (s + P <= t0)
                    pb[P - 1] = Bk[(t0 - s - P) * 64];
                if (r > 0 || s0 > 0)
                    win[(G - r) % G] = b;
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int g = G - 1; g >= 0; --g)
                    acc[g] = Form::mma(a, win[(g - r + G) % G], acc[g]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // step s = t0: B_0 enters
        {
            const Frag a = pa[0];
            const Frag b = pb[0];
#pragma unroll
            for (int q = 0; q + 1 < P; ++q) {
                pa[q] = pa[q + 1];
                pb[q] = pb[q + 1];
            }
            pa[P - 1] = Ak[(t0 + P) * 64];
            if (t0 > 0)
                win[0] = b;
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int g = G - 1; g >= 0; --g)
                acc[g] = Form::mma(a, win[g], acc[g]);
            __builtin_amdgcn_sched_barrier(0);
        }
        // tail steps s = t0 + p, p = 1 .. G-1: diagonals g >= p
        Frag nwin[G];
#pragma unroll
        for (int p = 1; p < G; ++p) {
            const Frag a = pa[0];
#pragma unroll
            for (int q = 0; q + 1 < P; ++q) {
                pa[q] = pa[q + 1];
                pb[q] = pb[q + 1];
            }
            const int nq = p + P - G;       // step of the next chunk, if >= 0
            if (nq < 0) {
                pa[P - 1] = Ak[(t0 + p + P) * 64];
            } else {
                pa[P - 1] = An[nq * 64];
                if (nq >= 1 && nq <= t0)
                    pb[P - 1] = Bn[(t0 - nq) * 64];
            }
            // slot G-p was last read at step t0 + p - 1
            nwin[G - p] = Bn[(t0 + G - p) * 64];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int g = G - 1; g >= p; --g)
                acc[g] = Form::mma(a, win[g - p], acc[g]);
            __builtin_amdgcn_sched_barrier(0);
        }
        nwin[0] = Bn[t0 * 64];
#pragma unroll
        for (int g = 0; g < G; ++g)
            win[g] = nwin[g];
        Ak = An;
        Bk = Bn;
    }
}

// column q of output o of this lane: cols[q * 256 + o * 64]
__device__ __forceinline__ void col_add(int64_t* cols, int o, int q, int64_t v)
{
    cols[q * 256 + o * 64] += v;
}

// X += v * 2^p exactly (carry-save), |v| < 2^63
__device__ __forceinline__ void fold_add(int64_t* cols, int o, int64_t v, int p)
{
    const int q = p >> 5, r = p & 31;
    const int64_t lo = v & 0xffffffffLL;    // in [0, 2^32)
    const int64_t hi = v >> 32;             // |hi| < 2^31
    const int64_t x = lo << r;              // < 2^63
    const int64_t y = hi << r;              // |y| < 2^62
    col_add(cols, o, q, x & 0xffffffffLL);
    col_add(cols, o, q + 1, (x >> 32) + (y & 0xffffffffLL));
    col_add(cols, o, q + 2, y >> 32);
}

__device__ __forceinline__ uint32_t limb(const int64_t* c, int q, int ncol)
{
    return q < ncol ? (uint32_t)c[q * 256] : 0u;
}

// 64 bits of the (nonnegative, normalised) integer starting at bit pos
__device__ __forceinline__ uint64_t window64(const int64_t* c, int pos, int ncol)
{
    const int q = pos >> 5, r = pos & 31;
    const uint64_t lo = (uint64_t)limb(c, q, ncol) | ((uint64_t)limb(c, q + 1, ncol) << 32);
    const uint64_t hi = limb(c, q + 2, ncol);
    return r ? ((lo >> r) | (hi << (64 - r))) : lo;
}

// Greedy round-to-nearest of X 2^scale into m words; c is one output's
// column set (stride 256), consumed.
__device__ void renormalise(int64_t* c, int ncol, int scale, int m, double* out, int64_t psc,
                            bool write)
{
    // carry propagation: 32-bit limbs, the top one signed
    int64_t carry = 0;
    for (int q = 0; q < ncol; ++q) {
        int64_t v = c[q * 256] + carry;
        if (q < ncol - 1) {
            carry = v >> 32;
            v -= carry * 4294967296LL;
        }
        c[q * 256] = v;
    }
    const bool neg = c[(ncol - 1) * 256] < 0;
    if (neg) {
        carry = 0;
        for (int q = 0; q < ncol; ++q) {
            int64_t v = -c[q * 256] + carry;
            if (q < ncol - 1) {
                carry = v >> 32;
                v -= carry * 4294967296LL;
            }
            c[q * 256] = v;
        }
    }
    double sgn = neg ? -1.0 : 1.0;
    const int umin = -1074 - scale;
    for (int t = 0; t < m; ++t) {
        int top = -1;
        for (int q = ncol - 1; q >= 0; --q) {
            const uint32_t v = (uint32_t)c[q * 256];
            if (v) {
                top = 32 * q + 31 - __clz((int)v);
                break;
            }
        }
        double w = 0.0;
        if (top >= 0) {
            int unit = max(top - 52, umin);
            if (unit < 0)
                unit = 0;
            uint64_t n = window64(c, unit, ncol);
            int rnd = 0, sticky = 0;
            if (unit > 0) {
                const int rb = unit - 1;
                rnd = (int)((limb(c, rb >> 5, ncol) >> (rb & 31)) & 1u);
                const int qs = rb >> 5;
                for (int q = 0; q < qs && !sticky; ++q)
                    sticky = limb(c, q, ncol) != 0;
                if (!sticky && (rb & 31))
                    sticky = (limb(c, qs, ncol) & ((1u << (rb & 31)) - 1u)) != 0;
            }
            const bool up = rnd && (sticky || (n & 1));
            if (up)
                n += 1;
            w = sgn * ldexp((double)n, unit + scale);
            // remainder: clear the bits at and above unit
            const int qu = unit >> 5;
            for (int q = qu + 1; q < ncol; ++q)
                c[q * 256] = 0;
            if (qu < ncol)
                c[qu * 256] = (int64_t)(limb(c, qu, ncol) & ((unit & 31) ? ((1u << (unit & 31)) - 1u) : 0u));
            if (up) {
                // |remainder| = 2^unit - low, and its sign flips
                uint64_t cy = 1;
                const int qe = (unit + 31) >> 5;
                for (int q = 0; q < qe && q < ncol; ++q) {
                    const uint64_t v = (uint64_t)(~limb(c, q, ncol)) + cy;
                    c[q * 256] = (int64_t)(v & 0xffffffffull);
                    cy = v >> 32;
                }
                if ((unit & 31) && qe - 1 < ncol)
                    c[(qe - 1) * 256] &= (int64_t)((1u << (unit & 31)) - 1u);
                sgn = -sgn;
            }
        }
        if (write)
            out[t * psc] = w;
    }
}

// Workgroup -> 32 x 32 output tile.  Workgroups are dispatched round-robin
// over the 8 XCDs (each with its own L2), so linear id L runs on XCD L % 8.
// The mapping gives XCD x the contiguous range x T/8 .. (x+1) T/8 - 1 of a
// grouped order in which runs of kGroupRows tile rows advance column by
// column: the workgroups resident on one XCD at a time then cover a compact
// block of tiles and share their A row panels and B column panels in L2.
constexpr int kXcds = 8, kGroupRows = 4;

__device__ __forceinline__ void tile_of_workgroup(int64_t gx, int64_t gy, int64_t& ty, int64_t& tx)
{
    const int64_t T = gx * gy;
    int64_t L = blockIdx.x;
    if (T % kXcds == 0)
        L = (L % kXcds) * (T / kXcds) + L / kXcds;
    const int64_t per_group = (int64_t)kGroupRows * gx;
    const int64_t group = L / per_group;
    const int64_t first = group * kGroupRows;
    const int64_t rows = min((int64_t)kGroupRows, gy - first);
    const int64_t r = L % per_group;
    ty = first + r % rows;
    tx = r / rows;
}

// Wave geometry shared by the contraction kernels: 4 waves, a 2 x 2 grid of
// 16 x 16 output tiles per workgroup.
struct WaveTile {
    int lane, wave;
    int64_t ty, tx;     // workgroup tile
    int64_t rb, cb;     // row block of op(A), column block of op(B)
    int64_t* cols;      // this lane's fold columns: cols[q * 256 + o * 64]

    // R row blocks per wave (rb .. rb+R-1): a 32 R x 32 workgroup tile
    __device__ __forceinline__ WaveTile(const GemmArgs& a, int R)
    {
        lane = threadIdx.x & 63;
        wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
        tile_of_workgroup((a.N + kTile - 1) / kTile, (a.M + kTile * R - 1) / (kTile * R), ty, tx);
        rb = (ty * 2 + (wave >> 1)) * R;
        cb = tx * 2 + (wave & 1);
        cols = nullptr;
    }

    // zeroed LDS fold columns (the banded kernels)
    __device__ __forceinline__ void init_cols(const GemmArgs& a, int64_t* lds)
    {
        cols = lds + (int64_t)wave * a.ncol * 256 + lane;
        for (int q = 0; q < a.ncol; ++q)
#pragma unroll
            for (int o = 0; o < 4; ++o)
                cols[q * 256 + o * 64] = 0;
    }
};

// This lane's diagonal 0 in the diagonal-sum buffer (layout in GemmArgs);
// diagonal t is 256 gR elements further.
__device__ __forceinline__ int64_t* gd_lane(const GemmArgs& a, const WaveTile& w)
{
    const int64_t gx = (a.N + kTile - 1) / kTile;
    return a.gD + ((((w.ty * gx + w.tx) * 4 + w.wave) * (int64_t)a.S) * 64 + w.lane) * (4 * a.gR);
}

// Exact fold of one depth chunk's diagonal sums t0 .. t0+G-1.  DBG kernels
// also add them into the debug buffer (a separate instantiation, so that the
// production kernels carry no debug addressing).  GLOBAL kernels (one row
// block per wave) only add them into the lane's slots of a.gD (private to
// the lane, so the read-modify-writes do not race) and keep no LDS fold; the
// first exactness chunk (first) masks the old contents to zero, and as every
// slot belongs to one band the buffer needs no clearing.
template <class Form, int G, bool DBG, bool GLOBAL = false>
__device__ __forceinline__ void fold_chunk(const typename Form::acc (&acc)[G], int t0,
                                           const GemmArgs& a, const WaveTile& w, bool first = false)
{
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int t = t0 + g;
        const int p = a.beta * (a.S - 1 - t);
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int64_t v = Form::value(acc[g], o);
            if constexpr (GLOBAL) {
                int64_t* d = gd_lane(a, w) + (int64_t)t * 256 + o;
                *d = (*d & (first ? 0 : -1)) + v;
            } else {
                fold_add(w.cols, o, v, p);
                if constexpr (DBG) {
                    const int64_t i = w.rb * 16 + Form::row(w.lane, o), j = w.cb * 16 + (w.lane & 15);
                    if (i < a.M && j < a.N)
                        a.dbgD[((int64_t)t * a.M + i) * a.N + j] += v;
                }
            }
        }
    }
}

template <class Form>
__device__ __forceinline__ void write_outputs(const GemmArgs& a, const WaveTile& w)
{
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        const int64_t i = w.rb * 16 + Form::row(w.lane, o), j = w.cb * 16 + (w.lane & 15);
        const bool ok = i < a.M && j < a.N;
        const int scale = ok ? a.E[i] + a.F[j] - a.beta * (a.S + 1) : 0;
        renormalise(w.cols + o * 64, a.ncol, scale, a.m, ok ? a.C + i * a.ldc + j : nullptr, a.psc,
                    ok);
    }
}

// lds_fold: the kernel keeps its fold columns in LDS (4 waves x ncol x 256)
template <class Kernel>
hipError_t launch_kernel(Kernel k, const GemmArgs& a, hipStream_t st, bool lds_fold = true,
                         int tile_rows = kTile)
{
    const size_t lds = lds_fold ? (size_t)4 * a.ncol * 256 * sizeof(int64_t) : 0;
    if (lds) {
        const hipError_t e = ensure_dynamic_lds((const void*)k, lds);
        if (e != hipSuccess)
            return e;
    }
    const int64_t tiles = ((a.N + kTile - 1) / kTile) * ((a.M + tile_rows - 1) / tile_rows);
    hipLaunchKernelGGL(k, dim3((unsigned)tiles), dim3(256), lds, st, a);
    return hipGetLastError();
}

}  // namespace
}  // namespace mdg
