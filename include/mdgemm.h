/*
 * mdgemm: m-double matrix product by error-free summation on one MI355X.
 *
 * An m-double is an unevaluated sum of m nonoverlapping doubles (paper,
 * Section 1).  C = A B is computed the way the paper computes m-double inner
 * products (Section 2, Figure 1, and the convolutions of the Conclusions):
 *
 *   1. every row i of A and every column j of B gets a shared exponent E_i,
 *      F_j (the largest exponent of its leading words);
 *   2. every entry is split into S signed integer slices (digits) of beta
 *      bits on the grid that starts at that exponent, the paper's "quarters";
 *   3. the diagonal sums D_t = sum_{s+u=t} sum_k dA_{ik,s} dB_{kj,u},
 *      t = 0..S-1, the paper's convolution sums s_i, run as exact slice
 *      matrix products on the matrix cores;
 *   4. sum_t D_t 2^(E_i + F_j - beta (t+2)) is folded exactly and rounded
 *      once, greedily to nearest, into m nonoverlapping output words
 *      (postponed renormalisation, Conclusions).
 *
 * Three slice forms:
 *   MD_FORM_FP64: digits of up to 24 bits held in doubles, FP64 matrix-core
 *                 products, exact while every partial sum stays below 2^53;
 *   MD_FORM_INT8: 7-bit sign-magnitude digits in int8, INT8 matrix-core
 *                 products with INT32 accumulation, exact while every
 *                 partial sum stays below 2^31;
 *   MD_FORM_INT8_BAL: the same truncation on the 8-bit grid that starts at
 *                 2^(E_i + 2), the truncated integer written in base 256
 *                 with balanced digits in [-128, 127] (all int8 values, so
 *                 8 bits per slice: fewer slices for the same T); the fold
 *                 then takes E_i + F_j + 4.  Not in the paper, whose
 *                 quarters are sign-magnitude bit fields.
 * S and beta are chosen per call from the target accuracy 2^-T (T = 50 m)
 * relative to (|A||B|)_ij.  The contraction is cut into depth chunks so that
 * every accumulation stays exact.
 *
 * Data layout: component planes.  Word w of entry (r, c) of a matrix X is at
 * X[w * plane_stride + r * ld + c]; all pointers are DEVICE pointers to
 * doubles; the words of an entry must be nonoverlapping (decreasing, with
 * disjoint bit ranges; zero words only at the tail) and finite, and a
 * nonzero leading word must lie in [2^-900, 2^900).  These preconditions are
 * checked only when opts->validate is set (MD_EINPUT otherwise undetected:
 * outputs of inputs that break them are unspecified).
 *
 * Every call is ordered on `stream` (a hipStream_t; NULL = the null stream).
 * Choosing S from the data needs the exponent spans on the host, so the
 * call synchronises `stream` once after the exponent step unless
 * opts->force_S is set, or opts->s_hint with opts->cert: then the call runs
 * on the hinted S and the device checks the data's certificate into
 * *opts->cert without waiting.  Errors of argument checking are returned
 * before any work is queued; device faults surface at the next
 * synchronisation.
 *
 * Range: the 2^-T bound needs every product inside the double range, which
 * the rule checks from the shared exponents (E_i + F_j + ceil(log2 K) <=
 * 1023 and E_i + F_j >= G + T - 1073 over the rows and columns with a
 * nonzero leading word); where it fails the call still returns the rounded
 * words, and md_info.input_flags bit 16 (MD_CERT_RANGE in a certificate)
 * reports that no bound is certified.
 *
 * All entry points are thread-safe; calls on different streams may run
 * concurrently.  The library allocates its scratch memory with
 * hipMallocAsync on `stream` and frees it on the same stream, unless the
 * caller passes a workspace.
 */
#ifndef MDGEMM_H
#define MDGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define MD_OK 0
#define MD_EINVAL_M 1      /* m not in {1, 2, 4, 8, 16} */
#define MD_EINVAL_DIM 2    /* negative size, bad leading dimension or stride, overflow */
#define MD_ENULL 3         /* NULL data pointer with a nonzero size */
#define MD_EALIAS 4        /* an output overlaps an input (C and A or B) or another output */
#define MD_ENOMEM 5        /* scratch allocation failed, or the given workspace is too small */
#define MD_EHIP 6          /* a HIP runtime call failed; md_last_hip_error() has the code */
#define MD_EINVAL_OPT 7    /* unknown form or rule, or forced S / beta out of range */
#define MD_ERANGE 8        /* no exact slice parameters exist for this size and target */
#define MD_EINPUT 9        /* validation mode: an input entry breaks the preconditions;
                              md_gemm_fixed: a given shared exponent was not taken */

/* slice forms */
#define MD_FORM_FP64 0
#define MD_FORM_INT8 1
#define MD_FORM_INT8_BAL 2

/* slice-count rules: both bound 2^G >= max_ij N_ij 2^(E_i+F_j) / (|A||B|)_ij,
 * N_ij the number of k with a_ik b_kj != 0; S is the smallest count with
 * beta S >= T + G + ceil(log2(S+2)) + 1, for the balanced digits with
 * 8 S >= T + G + ceil(log2(S+3)) + 3 (rounded up to equal bands).  The
 * certificates assume strongly nonoverlapping words, |w_{t+1}| <= ulp(w_t)/2. */
#define MD_S_RHO 0         /* default: the smaller of the span bound and a magnitude bound
                              from one extra INT8 product of 7-bit leading-word magnitudes */
#define MD_S_SPAN 1        /* span bound only: G = span_A + span_B + 2 */

/* Result of a call: the parameters the library chose. */
typedef struct md_info {
    int S;              /* slices per entry */
    int beta;           /* slice width in bits */
    int kc;             /* depth of one exact accumulation chunk */
    int band;           /* diagonals per band of the slice contraction */
    int span_A;         /* max over rows of A of (E_i - smallest exponent) */
    int span_B;         /* same over the columns of B */
    int G;              /* log2 of the certified ratio bound used by the rule */
    int G_span;         /* span bound: span_A + span_B + 2 */
    int G_rho;          /* magnitude bound (-1: not computed or not certifiable) */
    int target_bits;    /* T */
    double log2_bound;  /* certified log2 of the max relative error vs (|A||B|)_ij
                           (+inf: none; 0 with a forced S; NaN with a hint: see md_cert) */
    int input_flags;    /* validation mode: OR over the entries of 1 (a word not finite),
                           2 (not weakly nonoverlapping), 4 (leading word out of range);
                           md_gemm_fixed: 8 (a given shared exponent not taken);
                           the rule: 16 (a product may leave the double range, no bound) */
} md_info;

/* Certificate of a call run on a slice-count hint (md_opts.s_hint), written
 * on the device in stream order into caller-owned device memory: the rule's
 * certificates for this call's data, checked against the hinted S. */
typedef struct md_cert {
    int32_t flags;      /* MD_CERT_SMALL | MD_CERT_RANGE, 0 when the hint meets 2^-T */
    int32_t S_min;      /* S the rule would take for this data (same form and beta) */
    int32_t S;          /* S used (the hint) */
    int32_t G;          /* certified ratio exponent (the smaller of G_span and G_rho) */
    int32_t G_span;
    int32_t G_rho;      /* -1: not computed (MD_S_SPAN) or not certifiable */
    double log2_bound;  /* certified log2 relative error of the S used (+inf: none) */
} md_cert;
#define MD_CERT_SMALL 1 /* the hint is below S_min: 2^-T is not certified, log2_bound is */
#define MD_CERT_RANGE 2 /* a product may leave the double range: no bound */

/* Debug dump (small shapes): every non-NULL pointer is a device buffer the
 * caller owns, of at least the size shown; the library writes it during the
 * call.  digits_A, digits_B and D are sized by S, so they need a forced S
 * (opts->force_S; MD_EINVAL_OPT otherwise). */
typedef struct md_debug {
    int32_t *E;         /* [M]      shared exponents of the rows of op(A) (the balanced
                                    digits' grid starts 2 above) */
    int32_t *F;         /* [N]      shared exponents of the columns of op(B) */
    int32_t *digits_A;  /* [S][M][K] digits of op(A) */
    int32_t *digits_B;  /* [S][N][K] digits of op(B), by column */
    int64_t *D;         /* [S][M][N] diagonal sums D_t */
} md_debug;

typedef struct md_opts {
    int form;              /* MD_FORM_FP64 (default), MD_FORM_INT8 or MD_FORM_INT8_BAL */
    int s_rule;            /* MD_S_RHO (default) or MD_S_SPAN */
    int target_bits;       /* 0: T = 50 m */
    int force_S;           /* > 0: use this S (and force_beta) instead of the rule */
    int force_beta;        /* with force_S: slice width (INT8: 7; INT8_BAL: 8; FP64: 8..24) */
    void *workspace;       /* optional device scratch; NULL: allocate per call */
    size_t workspace_bytes;
    md_debug *dbg;         /* optional debug dump */
    md_info *info;         /* optional: receives the chosen parameters */
    void *ev_gemm_begin;   /* optional hipEvent_t pair (caller-owned), recorded on */
    void *ev_gemm_end;     /*   `stream` right before / after the slice contraction */
    int validate;          /* nonzero: check the input preconditions first (one read of
                              the inputs and one synchronisation); MD_EINPUT, with C
                              untouched and md_info.input_flags set, if any fails */
    int32_t *exp_flags;    /* md_gemm_fixed with given E or F: optional device int32 into
                              which bit 8 is ORed (never cleared) when a given exponent is
                              not taken, instead of a synchronisation and MD_EINPUT */
    int s_hint;            /* > 0 (force_S = 0): run on this S (FP64: with force_beta)
                              without waiting for the rule, e.g. the previous call's S;
                              needs cert */
    md_cert *cert;         /* with s_hint: device record of the data's certificate */
} md_opts;

/*
 * C = A B for m-double matrices, the plain FP64-slice form: the paper's
 * error-free summation of m-double inner products (Section 2: split every
 * double into bit fields, add the parts exactly, fuse once; Figure 1) for
 * every entry, its convolution sums run as slice matrix products
 * (Conclusions).
 *   m: words per entry, 1, 2, 4, 8 or 16.
 *   A: m planes of M x K, row-major, dense (lda = K, plane stride M K).
 *   B: m planes of K x N, row-major, dense.
 *   C: m planes of M x N, row-major, dense; fully overwritten; must not
 *      overlap A or B.
 *   stream: hipStream_t.
 * M = 0 or N = 0 is a no-op; K = 0 writes zeros.
 */
int md_gemm(int m, int64_t M, int64_t N, int64_t K, const double *A, const double *B, double *C,
            void *stream);

/*
 * C = op(A) op(B) with strides and options: md_gemm's computation (Section
 * 2, Figure 1, Conclusions) in any of the three slice forms.
 *   op(A) is M x K: element (i, k) at A[i*lda + k] (transA = 0) or
 *   A[k*lda + i] (transA = 1), word w at + w*plane_stride_A.
 *   op(B) is K x N: element (k, j) at B[k*ldb + j] (transB = 0) or
 *   B[j*ldb + k] (transB = 1), word w at + w*plane_stride_B.
 *   C: element (i, j) word w at C[w*plane_stride_C + i*ldc + j].
 *   opts may be NULL (FP64 form, MD_S_RHO rule, T = 50 m).
 * Graph capture: with opts->force_S (or opts->s_hint and opts->cert) set,
 * opts->validate and opts->dbg clear and a workspace of at least
 * md_gemm_workspace_size bytes, the call only launches kernels on `stream`
 * (no allocation, copy, memset or synchronisation), so it can be captured
 * into a HIP graph and replayed.
 * Replays reuse the workspace: replays (or calls) that share one must not
 * run concurrently.
 */
int md_gemm_ex(int m, int transA, int transB, int64_t M, int64_t N, int64_t K, const double *A,
               int64_t lda, int64_t plane_stride_A, const double *B, int64_t ldb,
               int64_t plane_stride_B, double *C, int64_t ldc, int64_t plane_stride_C,
               const md_opts *opts, void *stream);

/*
 * md_gemm_ex for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same arguments and results as md_gemm_ex, but its scratch is a
 * library-owned array of MD_NOALLOC_SCRATCH_BYTES bytes in each device's
 * global memory (held until the process ends), so the call makes no
 * allocation or free of any kind.
 *   opts->workspace must be NULL (MD_EINVAL_OPT otherwise).
 *   A call whose scratch (md_gemm_workspace_size for its form and S) would
 *   exceed the array returns MD_ENOMEM with C untouched; with the slice
 *   rule this is known only after the exponent step has run on the stream.
 * The array keeps the last call's contents; no step reads scratch it has
 * not written in the same call.  All calls on one device share the array:
 * calls that overlap in time on one device (different streams or host
 * threads without ordering) race and give undefined results; calls on one
 * stream are ordered.  Graph capture as md_gemm_ex (forced S or a hint),
 * with no workspace needed.
 */
#define MD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int md_gemm_ex_noalloc(int m, int transA, int transB, int64_t M, int64_t N, int64_t K, const double *A,
                       int64_t lda, int64_t plane_stride_A, const double *B, int64_t ldb,
                       int64_t plane_stride_B, double *C, int64_t ldc, int64_t plane_stride_C,
                       const md_opts *opts, void *stream);

/*
 * Batched inner products of m-double vectors, the paper's experiment
 * (Section 3, Table 2): out_b = sum_k x_bk y_bk for b = 0..batch-1.  The
 * same four steps as md_gemm_ex with one row of X and one column (a row of
 * Y) per product: every vector gets a shared exponent, every pair's digits
 * are contracted on the matrix cores, and every sum is folded exactly and
 * rounded once into m words.
 *   m: 1, 2, 4, 8 or 16 words per entry.
 *   X: word w of element k of vector b at X[w*plane_stride_X + b*ldx + k]
 *      (ldx >= n); Y likewise with ldy, plane_stride_Y.
 *   out: word w of product b at out[w*plane_stride_out + b]
 *      (plane_stride_out >= batch when m > 1); fully overwritten; must not
 *      overlap X or Y.
 *   opts as for md_gemm_ex (NULL: FP64 form, MD_S_RHO rule, T = 50 m),
 *   except that dbg must be NULL; ev_gemm_begin / ev_gemm_end bracket the
 *   contraction and the fold.  Guarantee: md_gemm_ex's, with (|A||B|)_ij
 *   read as sum_k |x_bk| |y_bk|.
 * batch = 0 is a no-op; n = 0 writes zeros.  Return codes as md_gemm_ex.
 */
int md_dot_ex(int m, int64_t batch, int64_t n, const double *X, int64_t ldx,
              int64_t plane_stride_X, const double *Y, int64_t ldy, int64_t plane_stride_Y,
              double *out, int64_t plane_stride_out, const md_opts *opts, void *stream);

/* md_dot_ex on dense planes (ldx = ldy = n, plane strides batch n and
 * batch), the plain FP64-slice form. */
int md_dot(int m, int64_t batch, int64_t n, const double *X, const double *Y, double *out,
           void *stream);

/*
 * The comparison baseline (paper, Section 1, Table 1, and the "ordinary"
 * columns of Table 2): C = A B in ordinary m-double arithmetic, every
 * multiplication and addition renormalised to m words, each entry
 * accumulated over k in increasing order from zero.  m = 1 (plain double
 * arithmetic), 2 (accurate double-double addition, Dekker-product
 * multiplication), 4 (quad-double operations grouped by order, one
 * renormalisation each) or 8 (floating-point expansion arithmetic as in
 * CAMPARY, the paper's reference for any length: addition by merging the
 * words by magnitude, multiplication by the product of expansions
 * truncated at order 8, both renormalised by VecSum and VecSumErrBranch);
 * no fused multiply-add.  Not error-free: the error grows with K.  Dense
 * planes as md_gemm; C must not overlap A or B.  M = 0 or N = 0 is a no-op;
 * K = 0 writes zeros.  Return codes as md_gemm (MD_EINVAL_M for other m).
 */
int md_gemm_ordinary(int m, int64_t M, int64_t N, int64_t K, const double *A, const double *B,
                     double *C, void *stream);

/*
 * Batched inner products in ordinary m-double arithmetic (the "ordinary"
 * side of the paper's experiment, Section 3, Table 2): out_b = sum_k
 * x_bk y_bk with md_gemm_ordinary's operations, m = 1, 2, 4 or 8, and
 * m = 16 (the octo-double expansion arithmetic on 16 words).  Order:
 * 64 partial sums per pair, sum l accumulating add(acc, mul(x_k, y_k)) over
 * k = l, l + 64, l + 128, .. from zero, then pairwise, sum l < h taking
 * add(sum_l, sum_(l+h)) for h = 32, 16, .., 1.  Dense planes as md_dot (X
 * and Y: word w of element k of vector b at [w batch n + b n + k]; out:
 * [w batch + b]); out must not overlap X or Y.  batch = 0 is a no-op;
 * n = 0 writes zeros.  Return codes as md_dot (MD_EINVAL_M for other m).
 */
int md_dot_ordinary(int m, int64_t batch, int64_t n, const double *X, const double *Y, double *out,
                    void *stream);

/*
 * Exact fixed-point results (paper, Section 1: multiword integers; the
 * splitting of Section 2).  The product's exact sum before its one
 * rounding is an integer X_ij at a power-of-two scale:
 *   X_ij = sum_t D_t 2^(beta (S-1-t)),  C~_ij = X_ij 2^scale_ij,
 *   scale_ij = E_i + F_j + 2h - beta (S+1)  (h = 2 for MD_FORM_INT8_BAL, else 0).
 * When every depth block of a product is split on the same shared
 * exponents (those of the full rows of A and columns of B, md_exponents),
 * the blocks' integers add up exactly to the whole product's (md_fixed_add),
 * and md_fixed_round of the sum returns what md_gemm_ex returns for the
 * whole product with the same form, S and beta: a depth-split product
 * (across streams or devices) reduced without any intermediate rounding.
 *
 * Integer layout: limb planes.  Limb k (32-bit two's complement, least
 * significant first) of entry e is X[k * count + e]; for an M x N result
 * count = M N and e = i N + j.  All pointers are device pointers.
 */

/* Limbs that hold X for any product of depth up to K with this beta and S
 * (|X| < K 2^(beta (S+1) + 1)), or -1 if beta is not in [1, 24], S not in
 * [1, 512] or K < 0.  Host only. */
int md_fixed_limbs(int beta, int S, int64_t K);

/*
 * Shared exponents of the rows of A (M x K, row-major, leading dimension
 * lda >= K; leading words only, plane 0) into E[M], and of the columns of B
 * (K x N, row-major, ldb >= N) into F[N]: the largest frexp exponent of
 * the nonzero leading words, 0 for an all-zero row or column (or K = 0).
 * E or F may be NULL to skip that operand.  Returns MD_OK, MD_EINVAL_DIM,
 * MD_ENULL, MD_ENOMEM or MD_EHIP.
 */
int md_exponents(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda, const double *B,
                 int64_t ldb, int32_t *E, int32_t *F, void *stream);

/*
 * X (nlimb limb planes of M N entries) and scale[M N] (int32) of the exact
 * product A B, m-double planes as md_gemm_ex without transposition: A is
 * m planes of M x K (leading dimension lda, plane stride plane_stride_A),
 * B m planes of K x N (ldb, plane_stride_B) -- so a depth block of larger
 * matrices is addressed in place.
 *   opts:  required, with force_S and force_beta set (the slices are fixed
 *          by the caller so that every block shares them); form as
 *          md_gemm_ex; dbg must be NULL; workspace, if given, serves the
 *          product's own scratch and, on the paths that capture the
 *          diagonal sums (below), also those sums (S M N int64) and the
 *          rounded words they produce on the way (m M N doubles).
 *   E, F:  shared exponents of the rows of A and columns of B (device, M and
 *          N int32) or NULL for the data's own.  Each given one must be at
 *          least the data's own (any value from -1100 for a row or column
 *          whose leading words are all zero in this block: its digits are
 *          zero on every grid) and at most 1100; otherwise the call
 *          returns MD_EINPUT with md_info.input_flags bit 8 (if opts->info),
 *          X and scale unspecified.  Given E or F make the call synchronise
 *          `stream` once to check them, unless opts->exp_flags is set: then
 *          bit 8 is ORed into that device word on the stream (one word can
 *          collect every block of a split) and the call does not wait.
 *   nlimb: at least md_fixed_limbs(force_beta, force_S, K), at most 80
 *          (MD_ERANGE otherwise).
 * X and scale must not overlap each other (MD_EALIAS).  K must be at least
 * 1 (MD_EINVAL_DIM); M = 0 or N = 0 is a no-op.  The INT8 forms whose
 * whole depth is one exactness chunk, and every banded contraction, write
 * the integers from their own epilogue at the product's speed; the other
 * cases (FP64 bands folded in LDS, INT8 triangles over several chunks)
 * capture the S M N int64 diagonal sums in scratch and fold them after.
 */
int md_gemm_fixed(int m, int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                  int64_t plane_stride_A, const double *B, int64_t ldb, int64_t plane_stride_B,
                  const int32_t *E, const int32_t *F, int32_t *X, int nlimb, int32_t *scale,
                  const md_opts *opts, void *stream);

/* Z = X + Y modulo 2^(32 nlimb) for count entries of nlimb limb planes
 * each (Z may be X or Y).  Both must be at the same scale (same E, F, S,
 * beta); md_fixed_limbs of the total depth keeps the sum in range.
 * nlimb in [1, 80] (MD_ERANGE otherwise). */
int md_fixed_add(int64_t count, int nlimb, const int32_t *X, const int32_t *Y, int32_t *Z,
                 void *stream);

/* C = X 2^scale rounded greedily to nearest into m nonoverlapping words
 * (word w of entry e at C[w * plane_stride_C + e], plane_stride_C >= count),
 * the product's own final rounding.  m in {1, 2, 4, 8, 16}; nlimb in
 * [1, 80]; C must not overlap X or scale (MD_EALIAS). */
int md_fixed_round(int m, int64_t count, int nlimb, const int32_t *X, const int32_t *scale, double *C,
                   int64_t plane_stride_C, void *stream);

/*
 * Parameter rule alone (host only, no device work): (beta, S, kc, band) for
 * a form, contraction depth K, target T and ratio-bound exponent G.
 * Returns MD_OK, MD_EINVAL_OPT or MD_ERANGE.
 */
int md_choose_params(int form, int64_t K, int T, int G, int *beta, int *S, int *kc, int *band);

/* Scratch bytes an md_gemm_ex call with these sizes, form and S needs (the
 * workspace that lets a call allocate nothing). */
size_t md_gemm_workspace_size(int form, int64_t M, int64_t N, int64_t K, int S);

/* The same (the name of earlier versions). */
size_t md_workspace_size(int form, int64_t M, int64_t N, int64_t K, int S);

/* Scratch bytes an md_dot_ex call with batch pairs of length n and slice
 * count S needs (with a forced S and this workspace the call, like
 * md_gemm_ex, only launches kernels and can be captured into a HIP graph). */
size_t md_dot_workspace_size(int form, int64_t batch, int64_t n, int S);

/* Text of a return code (static storage). */
const char *md_strerror(int code);

/* hipError_t of the last MD_EHIP on this thread (0 if none). */
int md_last_hip_error(void);

/* Library version: major * 10000 + minor * 100 + patch. */
int md_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MDGEMM_H */
