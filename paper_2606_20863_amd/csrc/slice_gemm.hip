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

// Whole triangle of one depth-chunk run [c0, c1): all S diagonals at once
// (INT8, S <= 32), for R row blocks of op(A) against one column block of
// op(B).  The window holds B_0 .. B_{S-1} of the chunk; step p multiplies
// A_p of every row block with B_{g-p} into diagonal g for g >= p (g
// descending), so B_{S-p} is read for the last time at step p-1 and its slot
// takes the next chunk's B_{S-p} at step p (B_0 after the last step).
// Fragment (kc, s) of a stream is at byte (kc S + s) 1024.
//
// Step p carries R (S - p) matrix instructions, so A loads are scheduled by
// work, not by steps: A_q is issued at the latest step that leaves at least
// LA instructions before its use (tri_issue_a); the next chunk's first A
// fragments are issued inside this chunk.
constexpr int tri_work(int S, int R, int p) { return R * (p < S ? S - p : S - (p - S)); }

// Step (0 .. S-1 of this chunk) at which A of position q is issued, where
// q = 0 .. S-1 are this chunk's steps and q = S .. S+1 the next chunk's
// steps 0 and 1; -1: issued before the chunk starts (prologue or the end of
// the previous chunk; only for q < S).
constexpr int tri_issue_a(int S, int R, int LA, int q)
{
    int w = 0;
    for (int l = q - 1; l >= 0; --l) {
        w += tri_work(S, R, l);
        if (w >= LA)
            return l < S ? l : S - 1;
    }
    return q < S ? -1 : 0;   // the next chunk's A cannot precede this chunk
}

template <int S, int R, int LA>
__device__ __forceinline__ void tri_run_i8(v4i (&acc)[R][S], const FragStream (&LDA)[R],
                                           const FragStream& LDB, int64_t c0, int64_t c1)
{
    constexpr uint32_t F = 1024, CS = (uint32_t)S * F;
    uint32_t ck = (uint32_t)c0 * CS;
    v4i win[S], ar[R][S + 2];
#pragma unroll
    for (int g = S - 1; g >= 0; --g)
        win[g] = LDB(ck + g * F);
    // A of this first chunk issued "before" it: positions with no issue step
#pragma unroll
    for (int q = 0; q < S; ++q)
        if (tri_issue_a(S, R, LA, q) < 0)
#pragma unroll
            for (int r = 0; r < R; ++r)
                ar[r][q] = LDA[r](ck + q * F);
    for (int64_t kc = c0; kc < c1; ++kc) {
        const uint32_t cn = kc + 1 < c1 ? ck + CS : ck;
#pragma unroll
        for (int p = 0; p < S; ++p) {
            // issue the loads scheduled at this step
#pragma unroll
            for (int q = p + 1; q < S + 2; ++q)
                if (tri_issue_a(S, R, LA, q) == p)
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        ar[r][q] = q < S ? LDA[r](ck + q * F) : LDA[r](cn + (q - S) * F);
            if (p >= 1)
                win[S - p] = LDB(cn + (S - p) * F);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int g = S - 1; g >= p; --g)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    acc[r][g] = FormI8::mma(ar[r][p], win[g - p], acc[r][g]);
            __builtin_amdgcn_sched_barrier(0);
        }
        win[0] = LDB(cn);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            ar[r][0] = ar[r][S];
            ar[r][1] = ar[r][S + 1];
        }
#pragma unroll
        for (int q = 2; q < S; ++q)
            if (tri_issue_a(S, R, LA, q) < 0)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    ar[r][q] = LDA[r](cn + q * F);
        ck = cn;
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
    int64_t rb, cb;     // row block of op(A), column block of op(B)
    int64_t* cols;      // this lane's fold columns: cols[q * 256 + o * 64]

    // R row blocks per wave (rb .. rb+R-1): a 32 R x 32 workgroup tile
    __device__ __forceinline__ WaveTile(const GemmArgs& a, int R)
    {
        lane = threadIdx.x & 63;
        wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
        int64_t ty, tx;
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

// Exact fold of one depth chunk's diagonal sums t0 .. t0+G-1.  DBG kernels
// also add them into the debug buffer (a separate instantiation, so that the
// production kernels carry no debug addressing).
template <class Form, int G, bool DBG>
__device__ __forceinline__ void fold_chunk(const typename Form::acc (&acc)[G], int t0,
                                           const GemmArgs& a, const WaveTile& w)
{
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int t = t0 + g;
        const int p = a.beta * (a.S - 1 - t);
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int64_t v = Form::value(acc[g], o);
            fold_add(w.cols, o, v, p);
            if constexpr (DBG) {
                const int64_t i = w.rb * 16 + Form::row(w.lane, o), j = w.cb * 16 + (w.lane & 15);
                if (i < a.M && j < a.N)
                    a.dbgD[((int64_t)t * a.M + i) * a.N + j] += v;
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

// Register-resident fold of the whole-triangle kernel.  There beta = 7 and
// the band starts at t = 0, so diagonal t lands at bit 7 e, e = S-1-t, which
// is column e / 4 (weight 2^(28 (e / 4))) shifted left by the static amount
// 7 (e mod 4).  One depth chunk adds less than 2^31 (1 + 2^7 + 2^14 + 2^21)
// < 2^53 to a column; after every chunk the columns are carried back to 28
// bits.  The top column takes only carries and is the signed one.
// x[4 r + o] holds output o of the lane in row block rb0 + r.
template <int S, int R, bool DBG>
__device__ __forceinline__ void tri_fold(const v4i (&acc)[R][S], int64_t (&x)[4 * R][Tri<S>::kCols],
                                         const GemmArgs& a, int64_t rb0, int64_t cb, int lane)
{
#pragma unroll
    for (int g = 0; g < S; ++g) {
        const int e = S - 1 - g;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                x[4 * r + o][e >> 2] += (int64_t)acc[r][g][o] * ((int64_t)1 << (7 * (e & 3)));
                if constexpr (DBG) {
                    const int64_t i = (rb0 + r) * 16 + FormI8::row(lane, o), j = cb * 16 + (lane & 15);
                    if (i < a.M && j < a.N)
                        a.dbgD[((int64_t)g * a.M + i) * a.N + j] += acc[r][g][o];
                }
            }
    }
#pragma unroll
    for (int n = 0; n < 4 * R; ++n)
        carry28(x[n]);
}

// Greedy renormalisation of the lane's 4 R outputs, their steps interleaved.
template <int S, int R>
__device__ __forceinline__ void tri_outputs(int64_t (&x)[4 * R][Tri<S>::kCols], const GemmArgs& a,
                                            int64_t rb0, int64_t cb, int lane)
{
    constexpr int NL = Tri<S>::kLimbs, NO = 4 * R;
    uint32_t L[NO][NL];
    double sgn[NO], *out[NO];
    int scale[NO];
    bool ok[NO];
#pragma unroll
    for (int n = 0; n < NO; ++n) {
        const int64_t i = (rb0 + n / 4) * 16 + FormI8::row(lane, n % 4), j = cb * 16 + (lane & 15);
        ok[n] = i < a.M && j < a.N;
        scale[n] = ok[n] ? a.E[i] + a.F[j] - 7 * (S + 1) : 0;
        out[n] = a.C + (ok[n] ? i * a.ldc + j : 0);
        sgn[n] = to_limbs(x[n], L[n]) ? -1.0 : 1.0;
    }
    for (int t = 0; t < a.m; ++t) {
#pragma unroll
        for (int n = 0; n < NO; ++n) {
            const double wv = rn_next(L[n], sgn[n], scale[n]);
            if (ok[n])
                out[n][t * a.psc] = wv;
        }
    }
}

// Load lead of the triangle kernels' A fragments, in matrix instructions.
constexpr int kLeadA = 48;

// Whole-triangle INT8 contraction, S <= 32 diagonals in one band, one row
// block per wave (32 x 32 workgroup tile), any number of exactness chunks.
template <int S, bool DBG>
__global__ __launch_bounds__(256, 1) void k_tri_i8(GemmArgs a)
{
    const WaveTile w(a, 1);
    const uint64_t bytes = (uint64_t)a.nkc * S * 1024;   // one row block of fragments
    const FragStream LA[1] = {frag_stream((const char*)a.A + w.rb * bytes, bytes, w.lane)};
    const FragStream LB = frag_stream((const char*)a.B + w.cb * bytes, bytes, w.lane);
    int64_t x[4][Tri<S>::kCols];
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
        for (int j = 0; j < Tri<S>::kCols; ++j)
            x[o][j] = 0;
    for (int64_t c0 = 0; c0 < a.nkc; c0 += a.kcc) {
        v4i acc[1][S];
#pragma unroll
        for (int g = 0; g < S; ++g)
            acc[0][g] = FormI8::zero();
        tri_run_i8<S, 1, kLeadA>(acc, LA, LB, c0, min(c0 + a.kcc, a.nkc));
        tri_fold<S, 1, DBG>(acc, x, a, w.rb, w.cb, w.lane);
    }
    tri_outputs<S, 1>(x, a, w.rb, w.cb, w.lane);
}

// The same with two row blocks per wave (64 x 32 workgroup tile), which
// share the B window: half the B loads per matrix instruction.  The whole
// depth is one exactness chunk, so the fold columns exist only after the
// contraction.  A row block past the digit array (M padded to 32 rows) reads
// through an empty descriptor: zeros.
template <int S>
__global__ __launch_bounds__(256, 1) void k_tri2_i8(GemmArgs a)
{
    const WaveTile w(a, 2);
    const uint64_t bytes = (uint64_t)a.nkc * S * 1024;
    const int64_t nrb = 2 * ((a.M + kTile - 1) / kTile);
    FragStream LA[2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
        LA[r] = frag_stream((const char*)a.A + (w.rb + r) * bytes, w.rb + r < nrb ? bytes : 0,
                            w.lane);
    const FragStream LB = frag_stream((const char*)a.B + w.cb * bytes, bytes, w.lane);
    v4i acc[2][S];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int g = 0; g < S; ++g)
            acc[r][g] = FormI8::zero();
    tri_run_i8<S, 2, kLeadA>(acc, LA, LB, 0, a.nkc);
    int64_t x[8][Tri<S>::kCols];
#pragma unroll
    for (int n = 0; n < 8; ++n)
#pragma unroll
        for (int j = 0; j < Tri<S>::kCols; ++j)
            x[n][j] = 0;
    tri_fold<S, 2, false>(acc, x, a, w.rb, w.cb, w.lane);
    tri_outputs<S, 2>(x, a, w.rb, w.cb, w.lane);
}

// lds_fold: the kernel keeps its fold columns in LDS (4 waves x ncol x 256)
template <class Kernel>
hipError_t launch_kernel(Kernel k, const GemmArgs& a, hipStream_t st, bool lds_fold = true,
                         int tile_rows = kTile)
{
    const size_t lds = lds_fold ? (size_t)4 * a.ncol * 256 * sizeof(int64_t) : 0;
    if (lds) {
        const hipError_t e = hipFuncSetAttribute(
            (const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    const int64_t tiles = ((a.N + kTile - 1) / kTile) * ((a.M + tile_rows - 1) / tile_rows);
    hipLaunchKernelGGL(k, dim3((unsigned)tiles), dim3(256), lds, st, a);
    return hipGetLastError();
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

template <int S>
struct DispatchTri {
    static hipError_t run(const GemmArgs& a, hipStream_t st)
    {
        if (a.S == S)
            return a.dbgD ? launch_kernel(k_tri_i8<S, true>, a, st, false)
                          : launch_kernel(k_tri_i8<S, false>, a, st, false);
        return DispatchTri<S - 1>::run(a, st);
    }
};
template <>
struct DispatchTri<0> {
    static hipError_t run(const GemmArgs&, hipStream_t) { return hipErrorInvalidValue; }
};

template <int S>
struct DispatchTri2 {
    static hipError_t run(const GemmArgs& a, hipStream_t st)
    {
        if (a.S == S)
            return launch_kernel(k_tri2_i8<S>, a, st, false, 2 * kTile);
        return DispatchTri2<S - 1>::run(a, st);
    }
};
template <>
struct DispatchTri2<0> {
    static hipError_t run(const GemmArgs&, hipStream_t) { return hipErrorInvalidValue; }
};

// min over the outputs of P_ij = sum_k qA_ik qB_kj, depth up to 2^11 depth
// fragments (INT32 exact: one fragment adds below 64 * 127^2 < 2^20): a wave
// computes a 64 x 64 block (4 x 4 fragments), a workgroup 128 x 128.  The
// fragments of the next kMagDepth depth steps are in flight while the
// current one multiplies.  Row or column blocks past the padded arrays read
// through empty descriptors (zeros; those outputs are not counted).
constexpr int kMagDepth = 4;

__global__ __launch_bounds__(256) void k_mag_min_short(const v4i* __restrict__ qA,
                                                       const v4i* __restrict__ qB, int64_t M,
                                                       int64_t N, int64_t nkc,
                                                       unsigned long long* minP)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t rb0 = ((int64_t)blockIdx.y * 2 + (wave >> 1)) * 4;
    const int64_t cb0 = ((int64_t)blockIdx.x * 2 + (wave & 1)) * 4;
    const int64_t nrb = 2 * ((M + kTile - 1) / kTile), ncb = 2 * ((N + kTile - 1) / kTile);
    const uint64_t bytes = (uint64_t)nkc * 1024;
    FragStream SA[4], SB[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        SA[x] = frag_stream((const char*)qA + (rb0 + x) * bytes, rb0 + x < nrb ? bytes : 0, lane);
        SB[x] = frag_stream((const char*)qB + (cb0 + x) * bytes, cb0 + x < ncb ? bytes : 0, lane);
    }
    v4i acc[4][4], pa[kMagDepth][4], pb[kMagDepth][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
            acc[x][y] = v4i{0, 0, 0, 0};
#pragma unroll
    for (int d = 0; d < kMagDepth; ++d)
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            pa[d][x] = SA[x](d * 1024u);
            pb[d][x] = SB[x](d * 1024u);
        }
    for (int64_t kc = 0; kc < nkc; kc += kMagDepth) {
#pragma unroll
        for (int d = 0; d < kMagDepth; ++d) {
            // depth steps past nkc read zeros and add nothing
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_i32_16x16x64_i8(pa[d][x], pb[d][y], acc[x][y],
                                                                      0, 0, 0);
            const uint32_t nxt = (uint32_t)(kc + d + kMagDepth) * 1024u;
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                pa[d][x] = SA[x](nxt);
                pb[d][x] = SB[x](nxt);
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
                                                 int64_t nkc, unsigned long long* minP)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t rb0 = ((int64_t)blockIdx.y * 2 + (wave >> 1)) * 4;
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

// Diagonal sums t0 .. t0+G-1 of the 16 pairs of row block blockIdx.y over the
// depth fragments [c0, c0 + range), range within one exactness chunk.  The
// partial sums are added into D with 64-bit integer atomics: integer
// addition is associative, so D does not depend on their order.
template <class Form, int G>
__global__ __launch_bounds__(64) void k_dot_band(DotArgs a)
{
    typedef typename Form::frag Frag;
    typedef typename Form::acc Acc;
    const int lane = threadIdx.x;
    const int64_t rb = blockIdx.y;
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
            dim3 grid((unsigned)((a.nkc + a.range - 1) / a.range), (unsigned)((a.batch + 15) / 16),
                      (unsigned)a.nbands);
            hipLaunchKernelGGL((k_dot_band<Form, G>), grid, dim3(64), 0, st, a);
            return hipGetLastError();
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
    dim3 grid((unsigned)((N + 127) / 128), (unsigned)((M + 127) / 128));
    if (nkc <= 2048)
        hipLaunchKernelGGL(k_mag_min_short, grid, dim3(256), 0, st, (const v4i*)qA, (const v4i*)qB,
                           M, N, nkc, minP);
    else
        hipLaunchKernelGGL(k_mag_min, grid, dim3(256), 0, st, (const v4i*)qA, (const v4i*)qB, M, N,
                           nkc, minP);
    return hipGetLastError();
}

hipError_t launch_gemm_i8(const GemmArgs& a, hipStream_t st)
{
    // the triangle kernel's register fold holds |X| / 2^(28 ceil(S/4)) < K 2^9
    // in its signed top column
    if (a.nbands == 1 && a.S <= kTriMaxI8 && a.nkc * kKcI8 < ((int64_t)1 << 48)) {
        // one exactness chunk: two row blocks per wave (no debug dump there)
        if (a.kcc >= a.nkc && !a.dbgD)
            return DispatchTri2<kTriMaxI8>::run(a, st);
        return DispatchTri<kTriMaxI8>::run(a, st);
    }
    return Dispatch<FormI8, kGmaxI8>::run(a, st);
}

hipError_t launch_gemm_f64(const GemmArgs& a, hipStream_t st)
{
    return Dispatch<FormF64, kGmaxF64>::run(a, st);
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
        const hipError_t e = hipFuncSetAttribute((const void*)k_dot_final,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
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

}  // namespace mdg
