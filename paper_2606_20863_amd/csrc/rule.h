// The slice-count rule (error budget) and the certificates it takes, for
// the host (parameter choice before the launches) and the device (the
// certificate of a call that runs on a caller's slice-count hint without
// waiting for the data's exponents).
//
// Budget (paper Section 2 splits each double into bit fields and sums the
// parts exactly; here the truncation of the split and the dropped digit
// pairs s + u >= S are the only errors before the one rounding): with 2^G
// bounding N_ij 2^(E_i + F_j) / (|A||B|)_ij, sign-magnitude digits of beta
// bits meet 2^-T when beta S >= T + G + ceil(log2(S + 2)) + 1, balanced
// 8-bit digits when 8 S >= T + G + ceil(log2(S + 3)) + 3.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mdg {

// smallest b with 2^b >= n (0 for n <= 1)
__host__ __device__ inline int rule_ceil_log2(int64_t n)
{
    return n <= 1 ? 0 : 64 - __builtin_clzll((unsigned long long)(n - 1));
}

// The searches below start at a lower bound of the answer (the log term is
// at least 1), so that they take a few steps: the device runs them in one
// thread.

// smallest S with beta S >= T + G + ceil(log2(S + 2)) + 1
__host__ __device__ inline int rule_slice_count(int beta, int T, int G)
{
    const int64_t need0 = (int64_t)T + G + 2;
    int S = need0 > beta ? (int)((need0 - 1) / beta) : 1;
    while ((int64_t)beta * S < (int64_t)T + G + rule_ceil_log2(S + 2) + 1)
        ++S;
    return S;
}

// balanced digits: smallest S with 8 S >= T + G + ceil(log2(S + 3)) + 3
__host__ __device__ inline int rule_slice_count_balanced(int T, int G)
{
    const int64_t need0 = (int64_t)T + G + 5;
    int S = need0 > 8 ? (int)((need0 - 1) / 8) : 1;
    while ((int64_t)8 * S < (int64_t)T + G + rule_ceil_log2(S + 3) + 3)
        ++S;
    return S;
}

// Bands of at most gmax diagonals, all of one width: S rounds up to
// nb * ceil(S / nb) with nb = ceil(S / gmax); S <= single stays one band.
__host__ __device__ inline void rule_band_round(int Smin, int gmax, int single, int& S, int& band)
{
    if (Smin <= single) {
        S = band = Smin;
        return;
    }
    const int nb = (Smin + gmax - 1) / gmax;
    band = (Smin + nb - 1) / nb;
    S = nb * band;
}

// Magnitude certificate.  With q = floor(|a^(0)| 2^(7-E_i)) and strongly
// nonoverlapping words, |a_ik||b_kj| >= (1 - 2^-51) 2^(E_i+F_j-14) qA_ik qB_kj,
// so N_ij 2^(E_i+F_j) / (|A||B|)_ij <= K 2^14 / ((1 - 2^-51) minP).  Returns the
// smallest G >= 0 with minP 2^G >= K 2^14 + 1 (which covers the 1 - 2^-51
// factor for K < 2^36), or -1 when minP is 0 (no certificate).
__host__ __device__ inline int rule_rho_exponent(uint64_t minP, int64_t K)
{
    if (minP == 0 || minP == ~0ull)
        return -1;
    const unsigned __int128 target = ((unsigned __int128)K << 14) + 1;
    // minP 2^g < target for every g below bitlen(target) - bitlen(minP) - 1
    const int lt = 128 - (int)(target >> 64 ? __builtin_clzll((unsigned long long)(target >> 64))
                                            : 64 + __builtin_clzll((unsigned long long)target));
    const int lm = 64 - __builtin_clzll(minP);
    int g = lt - lm - 1 > 0 ? lt - lm - 1 : 0;
    while (((unsigned __int128)minP << g) < target)
        ++g;
    return g;
}

// Certified log2 of the largest relative error against (|A||B|)_ij for S
// slices of beta bits (balanced: 8-bit digits) under the ratio bound 2^G,
// the final rounding into m words included.
__host__ __device__ inline double rule_log2_bound(bool balanced, int G, int beta, int S, int m)
{
    const double lb = balanced ? (double)(G + 2 - 8 * S) + log2((double)S + 3.0)
                               : (double)(G - beta * S) + log2((double)S + 2.0);
    return log2(exp2(lb) + exp2(-53.0 * m + 0.1));
}

// Double range: the fold of an entry is below K 2^(E_i + F_j) in magnitude,
// which stays finite when E_i + F_j + ceil(log2 K) <= 1023; the greedy
// rounding errs by at most 2^-(53 m) of the fold plus 2^-1075 once a word
// falls below the normal range, which stays within 2^-(T+2) of
// (|A||B|)_ij >= 2^(E_i + F_j - G) when E_i + F_j >= G + T - 1073.  Emax and
// Emin are the largest and smallest shared exponents over the rows of op(A)
// with a nonzero leading word (Fmax, Fmin over the columns of op(B)).
__host__ __device__ inline bool rule_in_range(int Emax, int Emin, int Fmax, int Fmin, int64_t K, int G,
                                              int T)
{
    if (Emax < Emin || Fmax < Fmin)   // an operand with no nonzero word: C = 0
        return true;
    return (int64_t)Emax + Fmax + rule_ceil_log2(K) <= 1023 && (int64_t)Emin + Fmin >= (int64_t)G + T - 1073;
}

}  // namespace mdg
