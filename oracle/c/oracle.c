/*
 * Exact CPU oracle for the m-double matrix product, plain C with OpenMP.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, __graft_entry__.smoke() and the
 * CPU leg of bench.py (cpu_baseline and the sampled error check); never by
 * the product path, and sharing no code with it.
 *
 * Two layers, both exact:
 *
 *  - exact layer: C*_ij = sum_k a_ik b_kj with every word decoded exactly,
 *    accumulated in a fixed-point superaccumulator that spans every product
 *    of two doubles; rounded greedily to nearest into m words.  Also
 *    (|A||B|)_ij and the error of a given m-double result.
 *  - method layer: the error-free summation of the paper (Section 2) for
 *    chosen entries: shared exponents (max frexp exponent of the leading
 *    word per row of A / column of B), per-word truncated sign-magnitude
 *    digits of width beta, the diagonal sums D_t = sum_{s+u=t} sum_k
 *    dA_s dB_u for t < S (the paper's convolution sums), their exact fold
 *    sum_t D_t 2^(E_i+F_j-beta(t+2)), and greedy round-to-nearest.
 *
 * Readings of the paper (it fixes none of these): shared exponent per row /
 * column, truncation toward zero per word, the triangle s+u <= S-1, one exact
 * fold followed by one rounding.
 *
 * Matrices are component planes: A[w*M*K + i*K + k], B[w*K*N + k*N + j].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Superaccumulator: limb i holds a signed 64-bit count of units of
 * 2^(32 i + ACC_LOW); between normalisations limbs are carry-save.  Every
 * product of two finite doubles lies in [2^-2148, 2^2048). */
#define ACC_LOW (-2240)
#define ACC_LIMBS 144

typedef struct {
    int64_t l[ACC_LIMBS];
    int64_t adds;
} acc_t;

static void acc_clear(acc_t *a) { memset(a, 0, sizeof(*a)); }

static void acc_normalize(acc_t *a)
{
    for (int i = 0; i < ACC_LIMBS - 1; ++i) {
        int64_t carry = a->l[i] >> 32; /* floor division by 2^32 */
        a->l[i] -= carry * ((int64_t)1 << 32);
        a->l[i + 1] += carry;
    }
    a->adds = 0;
}

/* add sign * v * 2^e, with v < 2^128 */
static void acc_add_u128(acc_t *a, unsigned __int128 v, int e, int neg)
{
    if (v == 0)
        return;
    int pos = e - ACC_LOW;
    int q = pos >> 5, r = pos & 31;
    for (int c = 0; c < 4 && v != 0; ++c) {
        uint64_t chunk = (uint64_t)(v & 0xffffffffu);
        v >>= 32;
        uint64_t x = chunk << r; /* < 2^63 */
        int64_t lo = (int64_t)(x & 0xffffffffu), hi = (int64_t)(x >> 32);
        if (neg) {
            a->l[q + c] -= lo;
            a->l[q + c + 1] -= hi;
        } else {
            a->l[q + c] += lo;
            a->l[q + c + 1] += hi;
        }
    }
    if (++a->adds >= (1 << 26))
        acc_normalize(a);
}

/* |x| = mant * 2^ex exactly, mant < 2^53; returns the sign bit */
static int decode(double x, uint64_t *mant, int *ex)
{
    uint64_t bits;
    memcpy(&bits, &x, 8);
    int eb = (int)((bits >> 52) & 0x7ff);
    uint64_t frac = bits & ((1ull << 52) - 1);
    if (eb == 0) {
        *mant = frac;
        *ex = -1074;
    } else {
        *mant = frac | (1ull << 52);
        *ex = eb - 1075;
    }
    return (int)(bits >> 63);
}

static void acc_add_double(acc_t *a, double x, int negate)
{
    uint64_t mt;
    int ex;
    int s = decode(x, &mt, &ex);
    acc_add_u128(a, mt, ex, s ^ negate);
}

/* add x*y, negated if `flip` */
static void acc_add_product(acc_t *a, double x, double y, int flip)
{
    uint64_t mx, my;
    int ex, ey;
    int sx = decode(x, &mx, &ex), sy = decode(y, &my, &ey);
    acc_add_u128(a, (unsigned __int128)mx * my, ex + ey, sx ^ sy ^ flip);
}

static void acc_add_int64(acc_t *a, int64_t v, int e)
{
    if (v < 0)
        acc_add_u128(a, (unsigned __int128)(-(__int128)v), e, 1);
    else
        acc_add_u128(a, (unsigned __int128)v, e, 0);
}

/* value of bit `pos` (global bit index from limb 0) of a normalized,
 * nonnegative accumulator */
static int acc_bit(const acc_t *a, int pos)
{
    return (int)((a->l[pos >> 5] >> (pos & 31)) & 1);
}

/* Round the (normalized) accumulator to the nearest double, ties to even. */
static double acc_round(acc_t *a)
{
    acc_normalize(a);
    int neg = a->l[ACC_LIMBS - 1] < 0;
    acc_t mag = *a;
    if (neg) {
        for (int i = 0; i < ACC_LIMBS; ++i)
            mag.l[i] = -mag.l[i];
        acc_normalize(&mag);
    }
    int top = -1;
    for (int i = ACC_LIMBS - 1; i >= 0; --i) {
        if (mag.l[i] != 0) {
            top = 32 * i + 31 - __builtin_clzll((unsigned long long)mag.l[i] << 32);
            break;
        }
    }
    if (top < 0)
        return 0.0;
    int unit = top - 52;
    int umin = -1074 - ACC_LOW;
    if (unit < umin)
        unit = umin;
    uint64_t n = 0;
    for (int p = top; p >= unit; --p)
        n = (n << 1) | (uint64_t)acc_bit(&mag, p);
    int round_bit = unit > 0 ? acc_bit(&mag, unit - 1) : 0;
    int sticky = 0;
    for (int p = unit - 2; p >= 0 && !sticky; --p) {
        if ((p & 31) == 31 && mag.l[p >> 5] == 0) {
            p -= 31;
            continue;
        }
        sticky = acc_bit(&mag, p);
    }
    if (round_bit && (sticky || (n & 1)))
        n += 1;
    double w = ldexp((double)n, unit + ACC_LOW);
    return neg ? -w : w;
}

/* greedy round-to-nearest renormalisation into m words */
static void acc_renorm(acc_t *a, int m, double *out, int64_t stride)
{
    for (int t = 0; t < m; ++t) {
        double w = acc_round(a);
        out[t * stride] = w;
        if (w != 0.0)
            acc_add_double(a, w, 1);
    }
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Exact layer for a list of entries (ii[e], jj[e]).
 * Crn[e*m + t]: greedy RN words of C*; absab[e]: RN of (|A||B|)_ij;
 * if Cq != NULL (Cq[e*m + t], an m-double result to check), err[e] is
 * RN(C*_ij - sum_t Cq[e*m+t]).
 */
int orc_exact_entries(int m, int64_t M, int64_t N, int64_t K, const double *A, const double *B,
                      int64_t nent, const int64_t *ii, const int64_t *jj, const double *Cq,
                      double *Crn, double *absab, double *err)
{
    if (m < 1 || M < 0 || N < 0 || K < 0)
        return 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t e = 0; e < nent; ++e) {
        int64_t i = ii[e], j = jj[e];
        acc_t *acc = (acc_t *)malloc(sizeof(acc_t));
        acc_t *aab = (acc_t *)malloc(sizeof(acc_t));
        acc_clear(acc);
        acc_clear(aab);
        for (int64_t k = 0; k < K; ++k) {
            /* nonoverlapping words: the sign of an entry is that of its
             * leading word, so |a||b| = sgn(a0) sgn(b0) sum_{w,u} a_w b_u */
            int flip = signbit(A[i * K + k]) != signbit(B[k * N + j]);
            for (int w = 0; w < m; ++w) {
                double a = A[(int64_t)w * M * K + i * K + k];
                if (a == 0.0)
                    continue;
                for (int u = 0; u < m; ++u) {
                    double b = B[(int64_t)u * K * N + k * N + j];
                    if (b == 0.0)
                        continue;
                    acc_add_product(acc, a, b, 0);
                    acc_add_product(aab, a, b, flip);
                }
            }
        }
        if (Crn) {
            acc_t tmp = *acc;
            acc_renorm(&tmp, m, Crn + e * m, 1);
        }
        if (absab)
            absab[e] = acc_round(aab);
        if (Cq && err) {
            for (int t = 0; t < m; ++t)
                acc_add_double(acc, Cq[e * m + t], 1);
            err[e] = acc_round(acc);
        }
        free(acc);
        free(aab);
    }
    return 0;
}

/* frexp exponent of a nonzero double: 2^(e-1) <= |x| < 2^e */
static int frexp_exp(double x)
{
    int e;
    frexp(x, &e);
    return e;
}

/*
 * Shared exponent and span of R rows of leading words: element (r, k) at
 * lead[r*stride_r + k*stride_k].  E[r] = max frexp exponent over nonzero
 * entries (0 if none); span[r] = E[r] - min exponent (0 if none).
 */
int orc_exponents(int64_t R, int64_t K, const double *lead, int64_t stride_r, int64_t stride_k,
                  int32_t *E, int32_t *span)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < R; ++r) {
        int hi = 0, lo = 0, any = 0;
        for (int64_t k = 0; k < K; ++k) {
            double x = lead[r * stride_r + k * stride_k];
            if (x == 0.0)
                continue;
            int e = frexp_exp(x);
            if (!any || e > hi)
                hi = e;
            if (!any || e < lo)
                lo = e;
            any = 1;
        }
        E[r] = any ? hi : 0;
        if (span)
            span[r] = any ? hi - lo : 0;
    }
    return 0;
}

/* digits d_0..d_{S-1} of one entry (words x[w*wstride]) aligned to 2^E */
static void split_entry(int m, const double *x, int64_t wstride, int E, int beta, int S, int32_t *d)
{
    uint64_t mask = (1ull << beta) - 1;
    for (int s = 0; s < S; ++s)
        d[s] = 0;
    for (int w = 0; w < m; ++w) {
        double v = x[w * wstride];
        if (v == 0.0)
            continue;
        uint64_t mt;
        int ex;
        int neg = decode(v, &mt, &ex);
        for (int s = 0; s < S; ++s) {
            int sh = ex + beta * (s + 1) - E;
            uint64_t f;
            if (sh >= 0)
                f = sh >= beta ? 0 : ((mt << sh) & mask);
            else
                f = -sh >= 64 ? 0 : ((mt >> -sh) & mask);
            d[s] += neg ? -(int32_t)f : (int32_t)f;
        }
    }
}

/*
 * Balanced base-256 digits of the integer sum_s d[s] 256^(S-1-s) (any signs,
 * d[0] most significant): each digit plus the carry from below becomes its
 * centred remainder in [-128, 127], the rest is carried up.  Returns the
 * carry out of the top digit (0 when S balanced digits reach the integer).
 */
static int recode_balanced(int32_t *d, int S)
{
    int carry = 0;
    for (int s = S - 1; s >= 0; --s) {
        int v = d[s] + carry;
        int r = ((v + 128) % 256 + 256) % 256 - 128;
        d[s] = r;
        carry = (v - r) / 256;
    }
    return carry;
}

/*
 * Method layer for the entries rows x cols.
 * E[i] (M) and F[j] (N) are computed over full rows / columns and returned.
 * D[(a*ncols + b)*S + t] = D_t of entry (rows[a], cols[b]);
 * C[(a*ncols + b)*m + w] = greedy RN of the fold.
 * balanced: the balanced 8-bit digits (beta = 8): each entry truncated on
 * the grid that starts at 2^(E+2) and recoded into digits in [-128, 127];
 * the fold then takes E+2 and F+2.
 */
int orc_method_entries(int m, int64_t M, int64_t N, int64_t K, const double *A, const double *B,
                       int beta, int S, int balanced, int64_t nrows, const int64_t *rows,
                       int64_t ncols, const int64_t *cols, int32_t *E, int32_t *F, int64_t *D,
                       double *C)
{
    if (m < 1 || beta < 1 || beta > 30 || S < 1 || (balanced && beta != 8))
        return 1;
    const int h = balanced ? 2 : 0;
    int bad = 0;
    orc_exponents(M, K, A, K, 1, E, NULL);
    orc_exponents(N, K, B, 1, N, F, NULL);
    int32_t *dA = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nrows * K * S + 1));
    int32_t *dB = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncols * K * S + 1));
    if (!dA || !dB) {
        free(dA);
        free(dB);
        return 2;
    }
#pragma omp parallel for schedule(static) reduction(|: bad)
    for (int64_t a = 0; a < nrows; ++a)
        for (int64_t k = 0; k < K; ++k) {
            int32_t *d = dA + (a * K + k) * S;
            split_entry(m, A + rows[a] * K + k, M * K, E[rows[a]] + h, beta, S, d);
            if (balanced)
                bad |= recode_balanced(d, S) != 0;
        }
#pragma omp parallel for schedule(static) reduction(|: bad)
    for (int64_t b = 0; b < ncols; ++b)
        for (int64_t k = 0; k < K; ++k) {
            int32_t *d = dB + (b * K + k) * S;
            split_entry(m, B + k * N + cols[b], K * N, F[cols[b]] + h, beta, S, d);
            if (balanced)
                bad |= recode_balanced(d, S) != 0;
        }
    if (bad) {
        free(dA);
        free(dB);
        return 3;
    }
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int64_t a = 0; a < nrows; ++a) {
        for (int64_t b = 0; b < ncols; ++b) {
            int64_t *Dt = D + (a * ncols + b) * S;
            for (int t = 0; t < S; ++t) {
                int64_t sum = 0;
                for (int s = 0; s <= t; ++s) {
                    const int32_t *pa = dA + a * K * S + s;
                    const int32_t *pb = dB + b * K * S + (t - s);
                    for (int64_t k = 0; k < K; ++k)
                        sum += (int64_t)pa[k * S] * pb[k * S];
                }
                Dt[t] = sum;
            }
            acc_t *acc = (acc_t *)malloc(sizeof(acc_t));
            acc_clear(acc);
            int ef = E[rows[a]] + F[cols[b]] + 2 * h;
            for (int t = 0; t < S; ++t)
                acc_add_int64(acc, Dt[t], ef - beta * (t + 2));
            acc_renorm(acc, m, C + (a * ncols + b) * m, 1);
            free(acc);
        }
    }
    free(dA);
    free(dB);
    return 0;
}
