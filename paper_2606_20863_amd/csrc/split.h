// Word decoding and digit production shared by the splits: the slices of an
// m-double entry on its row's grid are cut word by word (the paper's
// quarters, Section 2), each word's bits being a field of its significand
// shifted to the grid.
//
// Everything here is plain integer code, also built for the host (with the
// device annotations defined away and the byte-permute builtin emulated) to
// check it against the oracle on the CPU.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace mdg {
namespace {

// |x| = mant * 2^ex with mant < 2^53; returns true if x < 0
__device__ __forceinline__ bool decode(double x, uint64_t& mant, int& ex)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const int eb = (int)((b >> 52) & 0x7ff);
    const uint64_t f = b & ((1ull << 52) - 1);
    mant = eb ? (f | (1ull << 52)) : f;
    ex = eb ? eb - 1075 : -1074;
    return (b >> 63) != 0;
}

// e with 2^(e-1) <= |x| < 2^e, x nonzero and finite
__device__ __forceinline__ int frexp_exponent(double x)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const int eb = (int)((b >> 52) & 0x7ff);
    if (eb)
        return eb - 1022;
    const uint64_t f = b & ((1ull << 52) - 1);
    return (64 - __builtin_clzll(f)) - 1074;
}

// floor(mant * 2^sh) mod 2^W, W <= 63, mant < 2^53; branch-free (clamped
// shift counts and selects), as the word offsets differ from lane to lane
__device__ __forceinline__ uint64_t field(uint64_t mant, int sh, uint64_t wmask)
{
    const uint64_t up = mant << (sh & 63);                     // used for 0 <= sh < 63
    const uint64_t down = mant >> (sh < -63 ? 63 : -sh & 63);   // used for sh < 0
    const uint64_t v = sh >= 63 ? 0 : (sh >= 0 ? up : down);
    return v & wmask;
}

// Gather limb j (digits [D j, D j + D)) of the positive and the negative
// words of one entry.
template <int MW>
__device__ __forceinline__ void limb_pair(const uint64_t (&mant)[MW], const int (&sh0)[MW],
                                          const bool (&neg)[MW], int shift, uint64_t wmask,
                                          uint64_t& P, uint64_t& N)
{
    P = 0;
    N = 0;
#pragma unroll
    for (int w = 0; w < MW; ++w) {
        const uint64_t v = field(mant[w], sh0[w] + shift, wmask);
        N |= neg[w] ? v : 0;
        P |= neg[w] ? 0 : v;
    }
}

// magnitude digit of the ratio certificate: floor(|x| 2^(7 - Er)) in [0, 127]
// (|x| < 2^Er); branch-free, from the same decoding as place_word, which the
// compiler shares with the word's placement
__device__ __forceinline__ uint32_t mag_digit(double x, int Er)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t bh = (uint32_t)(b >> 32);
    const int eb = (int)(bh >> 20) & 0x7ff;
    const uint32_t hid = eb < 1 ? 0u : 1u;
    const uint64_t mant = ((uint64_t)((bh & 0xfffffu) | (hid << 20)) << 32) | (uint32_t)b;
    const int e1 = eb > 1 ? eb : 1;                 // |x| = mant 2^(e1 - 1075)
    const int t = Er + 1068 - e1;                   // floor(|x| 2^(7 - Er)) = mant >> t
    const uint64_t down = mant >> (t > 63 ? 63 : (t < 0 ? 0 : t));
    const uint64_t up = mant << (t < -63 ? 63 : (t > 0 ? 0 : -t));   // t < 0: tiny Er, subnormal x
    return (uint32_t)(t >= 0 ? down : up) & 127u;
}

// The words in registers at this point of the program: an empty volatile
// statement that takes and gives back every one.  Volatile statements and
// loads keep their order, so a cut pinned this way is done before the loads
// that follow it are issued (else the cuts may sink below every load of
// the step, and all their words are live at once).
template <int SC>
__device__ __forceinline__ void pin(uint32_t (&xs)[SC], uint32_t& mx)
{
#pragma unroll
    for (int s = 0; s < SC; ++s)
        asm volatile("" : "+v"(xs[s]));
    asm volatile("" : "+v"(mx));
}

// ---------------------------------------------------------------------------
// Digits by word placement.
//
// An entry's truncated integer on its grid (unit 2^(Eg - nbits), nbits =
// digit bits times S) is X = sum_w sgn(w) v_w, v_w = floor(|w| 2^(nbits -
// Eg)).  A word's v_w is a run of at most 53 bits starting at bit P_w of X,
// so it meets at most two W-bit limbs (W >= 53): place_word gives the limb
// index j and the two parts, and each limb adds the parts that fall into it
// (two compares and selects per limb and word, instead of cutting every
// word at every limb).  X is kept in a container of SC >= S digits, shifted
// up by SC - S digits (pad = digit bits times SC - S): the low SC - S
// digits are zero, and digit s of the entry is digit s of the container,
// most significant first.

struct Placed {
    uint64_t lo;   // bits [0, W) of limb j
    int64_t hi;    // added to limb j + 1
    int j;
};

// kn = Eg + 1075 - nbits (minus the bit index, in X, of the unit of a word
// whose biased exponent is 1).  SIGNED: the parts carry the word's sign (lo
// the low W bits of sgn v 2^o in two's complement, hi the rest, arithmetic);
// else they are the magnitude's and neg tells the sign.
template <int W, bool SIGNED>
__device__ __forceinline__ Placed place_word(double x, int kn, int pad, bool& neg)
{
    static_assert(W >= 53 && W <= 63, "a significand meets at most two limbs");
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t bh = (uint32_t)(b >> 32);
    const int eb = (int)(bh >> 20) & 0x7ff;
    const uint32_t hid = eb < 1 ? 0u : 1u;          // the hidden bit: 0 for subnormals
    const uint64_t mant = ((uint64_t)((bh & 0xfffffu) | (hid << 20)) << 32) | (uint32_t)b;
    const int e1 = eb > 1 ? eb : 1;                 // |x| = mant 2^(e1 - 1075)
    const int np = kn - e1;                         // the unit of mant sits at bit -np of X
    const int t = np < 0 ? 0 : (np > 63 ? 63 : np);
    const uint64_t v = mant >> t;                   // truncated toward zero below the grid
    const uint32_t P = (uint32_t)((np < 0 ? -np : 0) + pad);
    Placed r;
    // floor(P / W) as a 24-bit product and shift: exact for P < 2^10
    // (within the digits of any container here, P < 8 * 64 + 64)
    constexpr uint32_t kMagic = (65536u + W - 1) / W;
    r.j = (int)(__umul24(P, kMagic) >> 16);
    const int o = (int)P - W * r.j;
    neg = (b >> 63) != 0;
    if (SIGNED) {
        // sgn v without a compare: (v ^ s) - s with s = 0 or all ones
        const uint64_t sm = (uint64_t)((int64_t)b >> 63);
        const int64_t sv = (int64_t)((v ^ sm) + (sm & 1));
        r.lo = ((uint64_t)sv << o) & ((1ull << W) - 1);
        r.hi = sv >> (W - o);
    } else {
        r.lo = (v << o) & ((1ull << W) - 1);
        r.hi = (int64_t)(v >> (W - o));
    }
    return r;
}

// dst with byte Q replaced by byte K of src
template <int Q, int K>
__device__ __forceinline__ uint32_t byte_insert(uint32_t dst, uint32_t src)
{
    static_assert(Q >= 0 && Q < 4 && K >= 0 && K < 4, "bytes of 32-bit words");
    constexpr uint32_t sel = ((Q == 0 ? 4 + K : 0) << 0) | ((Q == 1 ? 4 + K : 1) << 8) |
                             ((Q == 2 ? 4 + K : 2) << 16) | ((Q == 3 ? 4 + K : 3) << 24);
    // bytes 0-3 of the selection are dst's, 4-7 src's
    return __builtin_amdgcn_perm(src, dst, sel);
}

// f(integral_constant<int, I>) for I = 0 .. N-1, each I a compile-time index
template <int I, int N>
struct Unroll {
    template <class F>
    static __device__ __forceinline__ void run(F& f)
    {
        if constexpr (I < N) {
            f(std::integral_constant<int, I>{});
            Unroll<I + 1, N>::run(f);
        }
    }
};

template <int N, class F>
__device__ __forceinline__ void unroll(F&& f)
{
    Unroll<0, N>::run(f);
}

// The limbs of an entry live in a store indexed at run time (LDS on the
// device: a word's limb index differs from lane to lane, and selects over
// every limb would cost more than the word itself).  The store adds into
// limb i with add(i, v), reads and clears it with take(i), and has one
// spare limb above the last, written and never read (the carry part of a
// word in the top limb, which lies above every digit).

// Balanced 8-bit digits (grid Eg = shared exponent + 2, kn = Eg + 1075 -
// 8 S, pad = 8 (SC - S)) of one entry into byte Q of xs[0 .. SC): limbs of
// 56 bits, least significant first; with the bias 0x80..80 (7 bytes) each
// limb plus the carry from below, U = V + carry + bias, holds in byte k
// (top bit flipped) the digit of container position 7 i + k, and U >> 56 is
// carried up.  The caller flips the top bits of all four bytes afterwards
// (xs[s] ^= 0x80808080).  The store's limbs start and end at zero.
template <int SC>
constexpr int bal_limbs()
{
    return (SC + 6) / 7;
}

template <int Q, int MW, int SC, class Limbs>
__device__ __forceinline__ void digits_bal(const double (&x)[MW], int kn, int pad, uint32_t (&xs)[SC], Limbs& L)
{
    constexpr int NL = bal_limbs<SC>();
    constexpr int64_t kBias = 0x80808080808080LL;
#pragma unroll
    for (int w = 0; w < MW; ++w) {
        bool neg;
        const Placed p = place_word<56, true>(x[w], kn, pad, neg);
        const int j = p.j < NL - 1 ? p.j : NL - 1;
        L.add(j, p.lo);
        L.add(j + 1, (uint64_t)p.hi);
    }
    int64_t carry = 0;
    unroll<NL>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const int64_t u = (int64_t)L.take(i) + carry + kBias;
        carry = u >> 56;
        const uint32_t l32 = (uint32_t)u, h32 = (uint32_t)((uint64_t)u >> 32);
        unroll<7>([&](auto K) {
            constexpr int k = decltype(K)::value, c = 7 * i + k;
            if constexpr (c < SC)
                xs[SC - 1 - c] = byte_insert<Q, k & 3>(xs[SC - 1 - c], k < 4 ? l32 : h32);
        });
    });
}

// Sign-magnitude 7-bit digits (grid Eg = shared exponent, kn = Eg + 1075 -
// 7 S, pad = 7 (SC - S)) of one entry into byte Q of xs[0 .. SC): the
// positive words gathered in limbs 0 .. NL-1 of 63 bits (nine fields), the
// negative ones in limbs NL+1 .. 2NL, digit = field of the positives minus
// field of the negatives (limbs NL and 2NL+1 are the spare ones).
template <int SC>
constexpr int sm_limbs()
{
    return (SC + 8) / 9;
}

template <int Q, int MW, int SC, class Limbs>
__device__ __forceinline__ void digits_sm(const double (&x)[MW], int kn, int pad, uint32_t (&xs)[SC], Limbs& L)
{
    constexpr int NL = sm_limbs<SC>();
#pragma unroll
    for (int w = 0; w < MW; ++w) {
        bool neg;
        const Placed p = place_word<63, false>(x[w], kn, pad, neg);
        const int j = (p.j < NL - 1 ? p.j : NL - 1) + (neg ? NL + 1 : 0);
        L.add(j, p.lo);
        L.add(j + 1, (uint64_t)p.hi);
    }
    unroll<NL>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const uint64_t P = L.take(i), N = L.take(NL + 1 + i);
        unroll<9>([&](auto K) {
            constexpr int k = decltype(K)::value, c = 9 * i + k;
            if constexpr (c < SC) {
                const int d = (int)((P >> (7 * k)) & 127) - (int)((N >> (7 * k)) & 127);
                xs[SC - 1 - c] = byte_insert<Q, 0>(xs[SC - 1 - c], (uint32_t)d);
            }
        });
    });
}

// limbs a store needs (spare limbs included)
template <int SC, bool BAL>
constexpr int store_limbs()
{
    return BAL ? bal_limbs<SC>() + 1 : 2 * sm_limbs<SC>() + 2;
}

}  // namespace
}  // namespace mdg
