// Exponent alignment and split of m-double operands into integer slices.
//
// Shared exponent (the paper assumes one exponent for all doubles, Section
// 2; here one per row of A and per column of B): E_r is the largest frexp
// exponent (2^(e-1) <= |x| < 2^e) of the leading words of row r, zero words
// skipped, and 0 for an all-zero row.  Nonoverlapping words keep every
// entry of the row below 2^E_r in magnitude.
//
// Split (the paper's quarters, Section 2 and Figure 1, with beta bits in
// place of 13): digit s of an entry is
//   d_s = sum_w sgn(w) * (floor(|w| * 2^(beta (s+1) - E_r)) mod 2^beta),
// i.e. each word is cut on the beta-bit grid that starts at 2^E_r and
// truncated toward zero below 2^(E_r - beta S).  Because the words' bits are
// disjoint, |d_s| <= 2^beta - 1 (INT8: beta = 7 fits int8).
//
// The split works a limb at a time: a limb is a run of D = floor(63/beta)
// digits, W = D beta bits wide.  For limb j the positive words and the
// negative words are each gathered into one W-bit integer (their bits are
// disjoint, so OR adds them), and digit D j + i is the difference of the
// i-th beta-bit fields of the two.
//
// Balanced INT8 digits (an encoding of the same truncation that uses all
// 256 int8 values): the grid starts at 2^(E_r + 2) (the exponent array then
// holds E_r + 2), beta = 8, and the truncated integer
// X = sum_w sgn(w) floor(|w| 2^(8 S - E_r - 2)) is written as
// X = sum_s d_s 256^(S-1-s) with d_s in [-128, 127].  |X| < 2^(8S-2), inside
// what S such digits reach.
#include "mdgemm_internal.h"
#include "split.h"
#include "ldslimbs.h"

#include <climits>

namespace mdg {
namespace {

__global__ void k_fill_zero(double* C, int m, int64_t M, int64_t N, int64_t ldc, int64_t psc)
{
    const int64_t n = (int64_t)m * M * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t w = e / (M * N), r = e % (M * N);
        C[w * psc + (r / N) * ldc + (r % N)] = 0.0;
    }
}

// stats: [0] span max of A, [1] span max of B, [2..3] (as one uint64) the
// minimum magnitude product, started at its largest value
__global__ void k_exp_init(int32_t* hi, int32_t* lo, int64_t R, int32_t* stats)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < R) {
        hi[r] = INT_MIN;
        lo[r] = INT_MAX;
    }
    if (r < 2 && stats)
        stats[r] = 0;
    if (r == 0 && stats)
        *reinterpret_cast<unsigned long long*>(stats + 2) = ~0ull;
    if (r < 4 && stats)   // largest and smallest shared exponents of A, then B
        stats[4 + r] = (r & 1) ? INT_MAX : INT_MIN;
}

// Block: 16 rows x `depth` (256, more only where the grid's second
// dimension would exceed 65535 blocks), 256 threads, 16 threads per row
// (short blocks: many waves in flight, each with its loads unrolled).  Each row's
// threads reduce with wavefront shuffles: in row order (the depth
// contiguous) they are 16 adjacent lanes (xor 1, 2, 4, 8); in column order
// (rows_fast: the rows contiguous, as for the columns of B) they are lanes
// 16 apart in each of the four waves (xor 16, 32), and every wave adds its
// partial row result by atomics.
constexpr int kExpRows = 16, kExpDepth = 256;
constexpr int64_t kMaxGridY = 65535;   // blocks on a launch's second grid dimension

__device__ __forceinline__ void exp_partial_block(const Operand& op, int32_t* hi, int32_t* lo, int rows_fast,
                                                  int64_t depth, int64_t bx, int64_t by)
{
    const int t = threadIdx.x;
    const int tr = rows_fast ? (t & 15) : (t >> 4);
    const int tk = rows_fast ? (t >> 4) : (t & 15);
    const int64_t r = bx * kExpRows + tr;
    const int64_t k0 = by * depth;
    int h = INT_MIN, l = INT_MAX;
    if (r < op.R) {
        const double* p = op.p + r * op.sr;
        const int64_t kend = min(k0 + depth, op.K);
#pragma unroll 4
        for (int64_t k = k0 + tk; k < kend; k += 16) {
            const double x = p[k * op.sk];
            if (x != 0.0) {
                const int e = frexp_exponent(x);
                h = max(h, e);
                l = min(l, e);
            }
        }
    }
    bool lead;
    if (rows_fast) {
        for (int o = 16; o < 64; o <<= 1) {
            h = max(h, __shfl_xor(h, o));
            l = min(l, __shfl_xor(l, o));
        }
        lead = (t & 63) < 16;
    } else {
        for (int o = 1; o < 16; o <<= 1) {
            h = max(h, __shfl_xor(h, o));
            l = min(l, __shfl_xor(l, o));
        }
        lead = tk == 0;
    }
    if (lead && r < op.R && h != INT_MIN) {
        atomicMax(hi + r, h);
        atomicMin(lo + r, l);
    }
}

__global__ __launch_bounds__(256) void k_exp_partial(Operand op, int32_t* hi, int32_t* lo,
                                                     int rows_fast, int64_t depth)
{
    exp_partial_block(op, hi, lo, rows_fast, depth, blockIdx.x, blockIdx.y);
}

// E[r] = the shared exponent plus eoff (the digit grid's start); the debug
// dump and the spans take the shared exponent itself.  ext (optional):
// ext[0] and ext[1] take the largest and smallest shared exponent of the
// rows with a nonzero leading word (wavefront-reduced, one atomic pair per
// wave).
__device__ __forceinline__ void exp_final_rows(const int32_t* hi, const int32_t* lo, int64_t R, int32_t* E,
                                               int32_t* span_max, int32_t* ext, int32_t* dbgE, int eoff,
                                               int64_t r)
{
    const int h = r < R ? hi[r] : INT_MIN;
    const int e = h == INT_MIN ? 0 : h;
    int span = h == INT_MIN ? 0 : h - lo[r];
    int emax = h, emin = h == INT_MIN ? INT_MAX : h;
    if (r < R) {
        E[r] = e + eoff;
        if (dbgE)
            dbgE[r] = e;
    }
    for (int o = 1; o < 64; o <<= 1) {
        span = max(span, __shfl_xor(span, o));
        emax = max(emax, __shfl_xor(emax, o));
        emin = min(emin, __shfl_xor(emin, o));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(span_max, span);
        if (ext && emax != INT_MIN) {
            atomicMax(ext, emax);
            atomicMin(ext + 1, emin);
        }
    }
}

__global__ void k_exp_final(const int32_t* hi, const int32_t* lo, int64_t R, int32_t* E,
                            int32_t* span_max, int32_t* ext, int32_t* dbgE, int eoff)
{
    exp_final_rows(hi, lo, R, E, span_max, ext, dbgE, eoff, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Input preconditions of one entry (flags: 1 a word not finite, 2 not
// weakly nonoverlapping, 4 a nonzero leading word outside [2^-900, 2^900)).
// Weak nonoverlap: the highest set bit of every nonzero word lies below the
// lowest set bit of the nonzero word before it, and no nonzero word follows
// a zero one.
template <int MW>
__device__ __forceinline__ int entry_flags(const Operand& op, int64_t r, int64_t k)
{
    int f = 0, prev_low = 0;
    bool have_prev = false, seen_zero = false;
#pragma unroll
    for (int w = 0; w < MW; ++w) {
        const uint64_t b = (uint64_t)__double_as_longlong(op.p[w * op.ps + r * op.sr + k * op.sk]);
        const int eb = (int)((b >> 52) & 0x7ff);
        const uint64_t f52 = b & ((1ull << 52) - 1);
        if (eb == 0x7ff) {
            f |= 1;
            continue;
        }
        if (eb == 0 && f52 == 0) {
            seen_zero = true;
            continue;
        }
        const uint64_t mant = eb ? (f52 | (1ull << 52)) : f52;
        const int ex = eb ? eb - 1075 : -1074;                // |x| = mant 2^ex
        const int low = ex + __builtin_ctzll(mant);
        const int high = ex + 63 - __builtin_clzll(mant);
        if (seen_zero || (have_prev && !(high < prev_low)))
            f |= 2;
        if (w == 0 && !(high >= -900 && high < 900))      // 2^-900 <= |x| < 2^900
            f |= 4;
        prev_low = low;
        have_prev = true;
    }
    return (f & 1) ? 1 : f;
}

// OR of the flags of every entry into *flags; entries in the order of the
// contiguous dimension.
template <int MW>
__global__ __launch_bounds__(256) void k_validate(Operand op, int rows_fast, int32_t* flags)
{
    const int64_t n = op.R * op.K;
    int f = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = rows_fast ? e % op.R : e / op.K;
        const int64_t k = rows_fast ? e / op.R : e % op.K;
        f |= entry_flags<MW>(op, r, k);
    }
    if (f)
        atomicOr(flags, f);
}

// Store of EPT consecutive digit bytes.
template <int EPT> struct Bytes;
template <> struct Bytes<4> { typedef uint32_t type; };
template <> struct Bytes<2> { typedef uint16_t type; };
template <> struct Bytes<1> { typedef uint8_t type; };

// INT8 split: a fragment is 1 KB; the 256 threads of a block write 256 EPT
// bytes of it, EPT bytes each (4 / EPT blocks per fragment): thread T of
// part p covers fragment bytes [EPT T', EPT T' + EPT), T' = T + 256 p, i.e.
// lane L = EPT T' / 16 (row L % 16) at depths 16 (L / 16) + (EPT T') % 16 + q.
// With more words per entry, fewer entries per thread keep the decoded words
// in registers.
template <int MW, int EPT, bool DBG>
__global__ __launch_bounds__(256) void k_split_i8(Operand op, const int32_t* E, int S,
                                                  int64_t nkc, int8_t* out, int32_t* dbg, int64_t rb0)
{
    constexpr int beta = 7, D = 9, W = 63, parts = 4 / EPT;
    typedef typename Bytes<EPT>::type Store;
    const int64_t rb = rb0 + blockIdx.y, kc = blockIdx.x / parts;
    const int byte0 = EPT * ((int)threadIdx.x + 256 * (int)(blockIdx.x % parts));
    const int L = byte0 >> 4;                 // fragment lane
    const int64_t r = rb * kRowBlock + (L & 15);
    const int64_t kbase = kc * kKcI8 + 16 * (L >> 4) + (byte0 & 15);
    const bool row_ok = r < op.R;
    const int Er = row_ok ? E[r] : 0;

    uint64_t mant[EPT][MW];
    int sh0[EPT][MW];
    bool neg[EPT][MW];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int64_t k = kbase + q;
        const bool ok = row_ok && k < op.K;
#pragma unroll
        for (int w = 0; w < MW; ++w) {
            const double x = ok ? op.p[w * op.ps + r * op.sr + k * op.sk] : 0.0;
            int ex;
            neg[q][w] = decode(x, mant[q][w], ex);
            sh0[q][w] = ex - Er;
        }
    }
    const uint64_t wmask = (1ull << W) - 1;
    Store* o = reinterpret_cast<Store*>(out + ((rb * nkc + kc) * (int64_t)S) * 1024 + byte0);
    const int nl = (S + D - 1) / D;
    for (int j = 0; j < nl; ++j) {
        uint64_t P[EPT], N[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q)
            limb_pair<MW>(mant[q], sh0[q], neg[q], W * (j + 1), wmask, P[q], N[q]);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int s = D * j + i;
            if (s >= S)
                break;
            const int rs = W - beta * (i + 1);
            uint32_t packed = 0;
            int dv[EPT];
#pragma unroll
            for (int q = 0; q < EPT; ++q) {
                dv[q] = (int)((P[q] >> rs) & 127) - (int)((N[q] >> rs) & 127);
                packed |= ((uint32_t)(dv[q] & 0xff)) << (8 * q);
            }
            o[(int64_t)s * (1024 / EPT)] = (Store)packed;
            if (DBG && row_ok) {
#pragma unroll
                for (int q = 0; q < EPT; ++q)
                    if (kbase + q < op.K)
                        dbg[((int64_t)s * op.R + r) * op.K + kbase + q] = dv[q];
            }
        }
    }
}

// Balanced INT8 split, same threads and stores as k_split_i8.  Limbs of
// D = 7 digits (56 bits) go from the least significant end: limb j holds
// digits [S - 7 (j+1), S - 7 j) (the top limb may reach below s = 0, where
// the digits are zero).  Its positive and negative words are gathered as in
// the sign-magnitude split, V = P - N + carry from the limb below, and with
// the bias 0x80..80 (7 bytes) U = V + bias: byte i of U mod 2^56, top bit
// flipped, is the digit 128 below it, d_(S - 7 j - 1 - i), and U >> 56 (in
// {-1, 0, 1}) is carried up.
template <int MW, int EPT, bool DBG>
__global__ __launch_bounds__(256) void k_split_i8bal(Operand op, const int32_t* E, int S,
                                                     int64_t nkc, int8_t* out, int32_t* dbg, int64_t rb0)
{
    constexpr int D = 7, W = 56, parts = 4 / EPT;
    constexpr int64_t kBias = 0x80808080808080LL;
    typedef typename Bytes<EPT>::type Store;
    const int64_t rb = rb0 + blockIdx.y, kc = blockIdx.x / parts;
    const int byte0 = EPT * ((int)threadIdx.x + 256 * (int)(blockIdx.x % parts));
    const int L = byte0 >> 4;                 // fragment lane
    const int64_t r = rb * kRowBlock + (L & 15);
    const int64_t kbase = kc * kKcI8 + 16 * (L >> 4) + (byte0 & 15);
    const bool row_ok = r < op.R;
    const int Er = row_ok ? E[r] : 0;

    uint64_t mant[EPT][MW];
    int sh0[EPT][MW];
    bool neg[EPT][MW];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int64_t k = kbase + q;
        const bool ok = row_ok && k < op.K;
#pragma unroll
        for (int w = 0; w < MW; ++w) {
            const double x = ok ? op.p[w * op.ps + r * op.sr + k * op.sk] : 0.0;
            int ex;
            neg[q][w] = decode(x, mant[q][w], ex);
            sh0[q][w] = ex - Er;
        }
    }
    const uint64_t wmask = (1ull << W) - 1;
    Store* o = reinterpret_cast<Store*>(out + ((rb * nkc + kc) * (int64_t)S) * 1024 + byte0);
    int64_t carry[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q)
        carry[q] = 0;
    const int nl = (S + D - 1) / D;
    for (int j = 0; j < nl; ++j) {
        const int s_end = S - D * j;
        uint64_t U[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            uint64_t P, N;
            limb_pair<MW>(mant[q], sh0[q], neg[q], 8 * s_end, wmask, P, N);
            const int64_t u = (int64_t)P - (int64_t)N + carry[q] + kBias;
            carry[q] = u >> W;
            U[q] = (uint64_t)u;
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int s = s_end - 1 - i;
            if (s < 0)
                break;
            uint32_t packed = 0;
#pragma unroll
            for (int q = 0; q < EPT; ++q)
                packed |= (((uint32_t)(U[q] >> (8 * i)) & 0xffu) ^ 0x80u) << (8 * q);
            o[(int64_t)s * (1024 / EPT)] = (Store)packed;
            if (DBG && row_ok) {
#pragma unroll
                for (int q = 0; q < EPT; ++q)
                    if (kbase + q < op.K)
                        dbg[((int64_t)s * op.R + r) * op.K + kbase + q] =
                            (int)((U[q] >> (8 * i)) & 0xffu) - 128;
            }
        }
    }
}

// Magnitude digits for the ratio certificate: q = floor(|a^(0)| 2^(7 - E_r)),
// in [0, 127] because |a^(0)| < 2^E_r; one slice in INT8 fragment order.
// Nonoverlapping words give |a| >= |a^(0)| (1 - 2^-52) >= q 2^(E_r - 7) (1 - 2^-52).
// E holds E_r + eoff.
__device__ __forceinline__ void split_mag_block(const Operand& op, const int32_t* E, int eoff, int64_t nkc,
                                                int8_t* out, int64_t rb, int64_t kc)
{
    const int T = threadIdx.x;
    const int L = T >> 2;
    const int64_t r = rb * kRowBlock + (L & 15);
    const int64_t kbase = kc * kKcI8 + 16 * (L >> 4) + 4 * (T & 3);
    const bool row_ok = r < op.R;
    const int Er = row_ok ? E[r] - eoff : 0;
    uint32_t packed = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t k = kbase + q;
        const double x = (row_ok && k < op.K) ? op.p[r * op.sr + k * op.sk] : 0.0;
        uint64_t mant;
        int ex;
        decode(x, mant, ex);
        const uint64_t v = field(mant, ex + 7 - Er, 127);
        packed |= (uint32_t)v << (8 * q);
    }
    reinterpret_cast<uint32_t*>(out)[(rb * nkc + kc) * 256 + T] = packed;
}


// The exponent pass and the magnitude split of both operands of a product,
// one launch per step instead of two (blockIdx.z: 0 for A, 1 for B; the
// grid covers the larger operand, and each side's blocks past its own rows
// do nothing): small products are bound by their launches.
__global__ void k_exp_init2(ExpSide a, ExpSide b, int32_t* stats)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < a.op.R) {
        a.hi[r] = INT_MIN;
        a.lo[r] = INT_MAX;
    } else if (r < a.op.R + b.op.R) {
        b.hi[r - a.op.R] = INT_MIN;
        b.lo[r - a.op.R] = INT_MAX;
    }
    if (r < 2)
        stats[r] = 0;
    if (r == 0)
        *reinterpret_cast<unsigned long long*>(stats + 2) = ~0ull;
    if (r < 4)   // largest and smallest shared exponents of A, then B
        stats[4 + r] = (r & 1) ? INT_MAX : INT_MIN;
}

__global__ __launch_bounds__(256) void k_exp_partial2(ExpSide a, ExpSide b, int64_t depth)
{
    if (blockIdx.z == 0)
        exp_partial_block(a.op, a.hi, a.lo, a.rows_fast, depth, blockIdx.x, blockIdx.y);
    else
        exp_partial_block(b.op, b.hi, b.lo, b.rows_fast, depth, blockIdx.x, blockIdx.y);
}

__global__ void k_exp_final2(ExpSide a, ExpSide b, int eoff)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.z == 0)
        exp_final_rows(a.hi, a.lo, a.op.R, a.E, a.span_max, a.ext, a.dbgE, eoff, r);
    else
        exp_final_rows(b.hi, b.lo, b.op.R, b.E, b.span_max, b.ext, b.dbgE, eoff, r);
}

__global__ __launch_bounds__(256) void k_split_mag2(ExpSide a, ExpSide b, int eoff, int64_t nkc, int64_t rb0)
{
    const int64_t rb = rb0 + blockIdx.y;
    if (blockIdx.z == 0) {
        if (rb < a.nrb)
            split_mag_block(a.op, a.E, eoff, nkc, a.q, rb, blockIdx.x);
    } else if (rb < b.nrb) {
        split_mag_block(b.op, b.E, eoff, nkc, b.q, rb, blockIdx.x);
    }
}

// Store of EPT consecutive digit doubles.
template <int EPT> struct Doubles;
template <> struct Doubles<4> { typedef double4 type; };
template <> struct Doubles<2> { typedef double2 type; };
template <> struct Doubles<1> { typedef double type; };

template <int EPT>
__device__ __forceinline__ typename Doubles<EPT>::type pack_doubles(const double (&v)[EPT]);
template <>
__device__ __forceinline__ double4 pack_doubles<4>(const double (&v)[4])
{
    return double4{v[0], v[1], v[2], v[3]};
}
template <>
__device__ __forceinline__ double2 pack_doubles<2>(const double (&v)[2])
{
    return double2{v[0], v[1]};
}
template <>
__device__ __forceinline__ double pack_doubles<1>(const double (&v)[1])
{
    return v[0];
}

// FP64 split: a fragment is 64 lanes x 4 doubles (lane l holds row l%16 at
// depths 4q + l/16); a block of 256 threads writes EPT fragments, EPT
// consecutive doubles per thread: thread u of a fragment covers doubles
// [EPT u, EPT u + EPT), i.e. lane EPT u / 4, q from (EPT u) % 4.
template <int MW, int EPT, bool DBG>
__global__ __launch_bounds__(256) void k_split_f64(Operand op, const int32_t* E, int S, int beta,
                                                   int64_t nrb, int64_t nkc, double* out,
                                                   int32_t* dbg)
{
    constexpr int TPF = 256 / EPT;            // threads per fragment
    typedef typename Doubles<EPT>::type Store;
    const int u = threadIdx.x % TPF;
    const int64_t frag = (int64_t)blockIdx.x * EPT + threadIdx.x / TPF;
    if (frag >= nrb * nkc)
        return;
    const int d0 = EPT * u;                   // first double of this thread
    const int lane = d0 >> 2, q0 = d0 & 3;
    const int64_t rb = frag / nkc, kc = frag % nkc;
    const int64_t r = rb * kRowBlock + (lane & 15);
    const bool row_ok = r < op.R;
    const int Er = row_ok ? E[r] : 0;
    const int D = 63 / beta, W = D * beta;

    uint64_t mant[EPT][MW];
    int sh0[EPT][MW];
    bool neg[EPT][MW];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int64_t k = kc * kKcF64 + 4 * (q0 + q) + (lane >> 4);
        const bool ok = row_ok && k < op.K;
#pragma unroll
        for (int w = 0; w < MW; ++w) {
            const double x = ok ? op.p[w * op.ps + r * op.sr + k * op.sk] : 0.0;
            int ex;
            neg[q][w] = decode(x, mant[q][w], ex);
            sh0[q][w] = ex - Er;
        }
    }
    const uint64_t wmask = (1ull << W) - 1, dmask = (1ull << beta) - 1;
    Store* o = reinterpret_cast<Store*>(out + ((rb * nkc + kc) * (int64_t)S) * 256 + d0);
    const int nl = (S + D - 1) / D;
    for (int j = 0; j < nl; ++j) {
        uint64_t P[EPT], N[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q)
            limb_pair<MW>(mant[q], sh0[q], neg[q], W * (j + 1), wmask, P[q], N[q]);
        for (int i = 0; i < D; ++i) {
            const int s = D * j + i;
            if (s >= S)
                break;
            const int rs = W - beta * (i + 1);
            double dv[EPT];
#pragma unroll
            for (int q = 0; q < EPT; ++q)
                dv[q] = (double)((int64_t)((P[q] >> rs) & dmask) - (int64_t)((N[q] >> rs) & dmask));
            o[(int64_t)s * TPF] = pack_doubles<EPT>(dv);
            if (DBG && row_ok) {
#pragma unroll
                for (int q = 0; q < EPT; ++q) {
                    const int64_t k = kc * kKcF64 + 4 * (q0 + q) + (lane >> 4);
                    if (k < op.K)
                        dbg[((int64_t)s * op.R + r) * op.K + k] = (int32_t)dv[q];
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_fill_zero(double* C, int m, int64_t M, int64_t N, int64_t ldc, int64_t psc,
                            hipStream_t st)
{
    const int64_t n = (int64_t)m * M * N;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st,
                       C, m, M, N, ldc, psc);
    return hipGetLastError();
}

hipError_t launch_exp_init(int32_t* hi, int32_t* lo, int64_t R, int32_t* stats, hipStream_t st)
{
    const int64_t blocks = std::max<int64_t>((R + 255) / 256, 1);
    hipLaunchKernelGGL(k_exp_init, dim3((unsigned)blocks), dim3(256), 0, st, hi, lo, R, stats);
    return hipGetLastError();
}

hipError_t launch_exp_partial(const Operand& op, int32_t* hi, int32_t* lo, hipStream_t st)
{
    const int rows_fast = (op.sr == 1 && op.sk != 1) ? 1 : 0;
    int64_t depth = kExpDepth;
    while ((op.K + depth - 1) / depth > kMaxGridY)
        depth *= 2;
    const int64_t gx = (op.R + kExpRows - 1) / kExpRows;
    if (gx > 0x7fffffff)
        return hipErrorInvalidValue;
    dim3 grid((unsigned)gx, (unsigned)((op.K + depth - 1) / depth));
    hipLaunchKernelGGL(k_exp_partial, grid, dim3(256), 0, st, op, hi, lo, rows_fast, depth);
    return hipGetLastError();
}

hipError_t launch_exp_final(const int32_t* hi, const int32_t* lo, int64_t R, int32_t* E,
                            int32_t* span_max, int32_t* ext, int32_t* dbgE, int eoff, hipStream_t st)
{
    const int64_t blocks = std::max<int64_t>((R + 255) / 256, 1);
    hipLaunchKernelGGL(k_exp_final, dim3((unsigned)blocks), dim3(256), 0, st, hi, lo, R, E,
                       span_max, ext, dbgE, eoff);
    return hipGetLastError();
}

hipError_t launch_exp_pass2(const ExpSide& a, const ExpSide& b, int32_t* stats, int eoff, hipStream_t st)
{
    if (a.op.K != b.op.K)
        return hipErrorInvalidValue;
    const int64_t R = std::max(a.op.R, b.op.R);
    hipLaunchKernelGGL(k_exp_init2, dim3((unsigned)std::max<int64_t>((a.op.R + b.op.R + 255) / 256, 1)), dim3(256),
                       0, st, a, b, stats);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (a.op.K > 0) {
        int64_t depth = kExpDepth;
        while ((a.op.K + depth - 1) / depth > kMaxGridY)
            depth *= 2;
        const int64_t gx = std::max<int64_t>((R + kExpRows - 1) / kExpRows, 1);
        if (gx > 0x7fffffff)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_exp_partial2, dim3((unsigned)gx, (unsigned)((a.op.K + depth - 1) / depth), 2),
                           dim3(256), 0, st, a, b, depth);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_exp_final2, dim3((unsigned)std::max<int64_t>((R + 255) / 256, 1), 1, 2), dim3(256), 0, st,
                       a, b, eoff);
    return hipGetLastError();
}

hipError_t launch_split_mag2(const ExpSide& a, const ExpSide& b, int eoff, int64_t nkc, hipStream_t st)
{
    if (nkc > 0x7fffffff)
        return hipErrorInvalidValue;
    const int64_t nrb = std::max(a.nrb, b.nrb);
    for (int64_t y0 = 0; y0 < nrb; y0 += kMaxGridY) {
        const dim3 grid((unsigned)nkc, (unsigned)std::min<int64_t>(nrb - y0, kMaxGridY), 2);
        hipLaunchKernelGGL(k_split_mag2, grid, dim3(256), 0, st, a, b, eoff, nkc, y0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// Caller-given shared exponents: E[r] (the data's own + eoff) becomes
// Ein[r] + eoff when Ein[r] lies in [own, kExpMax]; otherwise E[r] stays and
// bit 8 is set in *flags (a coarser grid keeps every word below 2^E; a
// finer one would not).  A row with no nonzero leading word (hi[r] at its
// initial INT_MIN) splits into zero digits on every grid, so any Ein[r] in
// [-kExpMax, kExpMax] is taken for it: E = 0 is only the all-zero
// convention, not a bound on the grid.
constexpr int kExpMax = 1100;

__global__ void k_exp_set(const int32_t* Ein, const int32_t* hi, int64_t R, int eoff, int32_t* E,
                          int32_t* flags)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R)
        return;
    const int own = E[r] - eoff, want = Ein[r];
    const int lowest = hi[r] == INT_MIN ? -kExpMax : own;
    if (want >= lowest && want <= kExpMax)
        E[r] = want + eoff;
    else
        atomicOr(flags, 8);
}

hipError_t launch_exp_set(const int32_t* Ein, const int32_t* hi, int64_t R, int eoff, int32_t* E,
                          int32_t* flags, hipStream_t st)
{
    const int64_t blocks = std::max<int64_t>((R + 255) / 256, 1);
    hipLaunchKernelGGL(k_exp_set, dim3((unsigned)blocks), dim3(256), 0, st, Ein, hi, R, eoff, E, flags);
    return hipGetLastError();
}

// Entries per thread of the splits: fewer when an entry has more words.
// INT8 split by word placement (the digits of split.h), m <= 4: the same
// threads, entries and stores as k_split_i8 / k_split_i8bal with four
// entries per thread, the four entries of a thread being the four bytes of
// each digit word.  Each word's truncated significand is placed at its bit
// position in the entry's integer (two LDS adds into at most two limbs)
// instead of being cut at every limb, about 40% fewer instructions per
// entry.  Digits in a container of SC >= S (the low SC - S zero); digit s
// of the entry is container digit s, most significant first.
template <int MW, int SC, bool BAL, bool DBG>
__global__ __launch_bounds__(256) void k_split_place(Operand op, const int32_t* E, int S, int64_t nkc,
                                                     int8_t* out, int32_t* dbg, int64_t rb0)
{
    constexpr int bits = BAL ? 8 : 7;
    constexpr int NS = store_limbs<SC, BAL>();
    __shared__ uint64_t limbs[4][NS][64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t rb = rb0 + blockIdx.y, kc = blockIdx.x;
    const int byte0 = 4 * t;
    const int L = byte0 >> 4;                 // fragment lane
    const int64_t r = rb * kRowBlock + (L & 15);
    const int64_t kbase = kc * kKcI8 + 16 * (L >> 4) + (byte0 & 15);
    const bool row_ok = r < op.R;
    const int Er = row_ok ? E[r] : 0;
    const int kn = Er + 1075 - bits * S, pad = bits * (SC - S);

    double x[4][MW];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t k = kbase + q;
        const bool ok = row_ok && k < op.K;
#pragma unroll
        for (int w = 0; w < MW; ++w)
            x[q][w] = ok ? op.p[w * op.ps + r * op.sr + k * op.sk] : 0.0;
    }
    LdsLimbs Ls{&limbs[wave][0][lane]};
#pragma unroll
    for (int i = 0; i < NS; ++i)
        Ls.col[i * 64] = 0;
    uint32_t xs[SC];
#pragma unroll
    for (int s = 0; s < SC; ++s)
        xs[s] = 0;
    unroll<4>([&](auto QQ) {
        constexpr int q = decltype(QQ)::value;
        if constexpr (BAL)
            digits_bal<q, MW, SC>(x[q], kn, pad, xs, Ls);
        else
            digits_sm<q, MW, SC>(x[q], kn, pad, xs, Ls);
    });
    uint32_t* o = reinterpret_cast<uint32_t*>(out + ((rb * nkc + kc) * (int64_t)S) * 1024 + byte0);
#pragma unroll
    for (int s = 0; s < SC; ++s) {
        if (s < S) {
            const uint32_t v = BAL ? xs[s] ^ 0x80808080u : xs[s];
            o[(int64_t)s * 256] = v;
            if (DBG && row_ok) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (kbase + q < op.K)
                        dbg[((int64_t)s * op.R + r) * op.K + kbase + q] = (int)(int8_t)(v >> (8 * q));
            }
        }
    }
}

// the container for S: the smallest multiple of 8 from 8 to 48 holding it
template <int MW, int SC, bool BAL>
hipError_t split_place_sc(const Operand& op, const int32_t* E, int S, int64_t nkc, int8_t* out, int32_t* dbg,
                          dim3 grid, int64_t y0, hipStream_t st)
{
    if constexpr (SC <= 48) {
        if (S > SC)
            return split_place_sc<MW, SC + 8, BAL>(op, E, S, nkc, out, dbg, grid, y0, st);
        if (dbg)
            hipLaunchKernelGGL((k_split_place<MW, SC, BAL, true>), grid, dim3(256), 0, st, op, E, S, nkc, out, dbg, y0);
        else
            hipLaunchKernelGGL((k_split_place<MW, SC, BAL, false>), grid, dim3(256), 0, st, op, E, S, nkc, out, dbg, y0);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

constexpr int split_ept(int m) { return m <= 4 ? 4 : (m == 8 ? 2 : 1); }

template <int MW>
hipError_t split_i8_m(const Operand& op, const int32_t* E, int S, int64_t nrb, int64_t nkc,
                      int8_t* out, int32_t* dbg, bool balanced, hipStream_t st)
{
    constexpr int EPT = split_ept(MW);
    if (nkc * (4 / EPT) > 0x7fffffff)
        return hipErrorInvalidValue;
    // word placement where a container holds S (m <= 4, S <= 48)
    constexpr bool kPlace = MW <= 4;
    // row blocks on the grid's second dimension, at most kMaxGridY per launch
    for (int64_t y0 = 0; y0 < nrb; y0 += kMaxGridY) {
        const dim3 grid((unsigned)(nkc * (4 / EPT)), (unsigned)std::min<int64_t>(nrb - y0, kMaxGridY));
        if (kPlace && S >= 1 && S <= 48) {
            const hipError_t e = balanced ? split_place_sc<MW, 8, true>(op, E, S, nkc, out, dbg, grid, y0, st)
                                          : split_place_sc<MW, 8, false>(op, E, S, nkc, out, dbg, grid, y0, st);
            if (e != hipSuccess)
                return e;
            continue;
        }
        if (balanced) {
            if (dbg)
                hipLaunchKernelGGL((k_split_i8bal<MW, EPT, true>), grid, dim3(256), 0, st, op, E, S, nkc, out, dbg, y0);
            else
                hipLaunchKernelGGL((k_split_i8bal<MW, EPT, false>), grid, dim3(256), 0, st, op, E, S, nkc, out, dbg, y0);
        } else if (dbg) {
            hipLaunchKernelGGL((k_split_i8<MW, EPT, true>), grid, dim3(256), 0, st, op, E, S, nkc, out, dbg, y0);
        } else {
            hipLaunchKernelGGL((k_split_i8<MW, EPT, false>), grid, dim3(256), 0, st, op, E, S, nkc, out, dbg, y0);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_split_i8(const Operand& op, int m, const int32_t* E, int S, int64_t nrb,
                           int64_t nkc, int8_t* out, int32_t* dbg, bool balanced, hipStream_t st)
{
    switch (m) {
    case 1: return split_i8_m<1>(op, E, S, nrb, nkc, out, dbg, balanced, st);
    case 2: return split_i8_m<2>(op, E, S, nrb, nkc, out, dbg, balanced, st);
    case 4: return split_i8_m<4>(op, E, S, nrb, nkc, out, dbg, balanced, st);
    case 8: return split_i8_m<8>(op, E, S, nrb, nkc, out, dbg, balanced, st);
    case 16: return split_i8_m<16>(op, E, S, nrb, nkc, out, dbg, balanced, st);
    default: return hipErrorInvalidValue;
    }
}

template <int MW>
hipError_t validate_m(const Operand& op, int32_t* flags, hipStream_t st)
{
    const int rows_fast = (op.sr == 1 && op.sk != 1) ? 1 : 0;
    const int64_t n = op.R * op.K;
    const int64_t blocks = std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 16384);
    hipLaunchKernelGGL((k_validate<MW>), dim3((unsigned)blocks), dim3(256), 0, st, op, rows_fast, flags);
    return hipGetLastError();
}

hipError_t launch_validate(const Operand& op, int m, int32_t* flags, hipStream_t st)
{
    switch (m) {
    case 1: return validate_m<1>(op, flags, st);
    case 2: return validate_m<2>(op, flags, st);
    case 4: return validate_m<4>(op, flags, st);
    case 8: return validate_m<8>(op, flags, st);
    case 16: return validate_m<16>(op, flags, st);
    default: return hipErrorInvalidValue;
    }
}

template <int MW>
hipError_t split_f64_m(const Operand& op, const int32_t* E, int S, int beta, int64_t nrb,
                       int64_t nkc, double* out, int32_t* dbg, hipStream_t st)
{
    constexpr int EPT = split_ept(MW);
    const int64_t blocks = (nrb * nkc + EPT - 1) / EPT;
    if (dbg)
        hipLaunchKernelGGL((k_split_f64<MW, EPT, true>), dim3((unsigned)blocks), dim3(256), 0, st, op, E,
                           S, beta, nrb, nkc, out, dbg);
    else
        hipLaunchKernelGGL((k_split_f64<MW, EPT, false>), dim3((unsigned)blocks), dim3(256), 0, st, op,
                           E, S, beta, nrb, nkc, out, dbg);
    return hipGetLastError();
}

hipError_t launch_split_f64(const Operand& op, int m, const int32_t* E, int S, int beta,
                            int64_t nrb, int64_t nkc, double* out, int32_t* dbg, hipStream_t st)
{
    switch (m) {
    case 1: return split_f64_m<1>(op, E, S, beta, nrb, nkc, out, dbg, st);
    case 2: return split_f64_m<2>(op, E, S, beta, nrb, nkc, out, dbg, st);
    case 4: return split_f64_m<4>(op, E, S, beta, nrb, nkc, out, dbg, st);
    case 8: return split_f64_m<8>(op, E, S, beta, nrb, nkc, out, dbg, st);
    case 16: return split_f64_m<16>(op, E, S, beta, nrb, nkc, out, dbg, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mdg
