// Internal interfaces of the m-double product library (not installed).
//
// Tiled slice layout ("fragments").  An operand op(X) has R rows (rows of A,
// or columns of B) and depth K.  Rows are grouped in blocks of 16, depth in
// chunks of KC (64 for INT8, 16 for FP64).  For row block rb, depth chunk kc
// and slice s, one fragment holds the 16 x KC digits in the order one
// wavefront hands them to the matrix cores:
//
//   INT8 (v_mfma_i32_16x16x64_i8): 64 lanes x 16 bytes; lane l holds row
//     rb*16 + l%16, depth kc*64 + 16*(l/16) + b in byte b.
//   FP64 (v_mfma_f64_16x16x4f64, four steps): 64 lanes x 4 doubles; lane l
//     holds row rb*16 + l%16, depth kc*16 + 4*q + l/16 in double q, and step q
//     of the matrix-core product uses double q of both operands.
//
// Fragment (rb, kc, s) starts at element ((rb * nkc + kc) * S + s) * 64 lanes,
// so the S slices of one depth chunk are adjacent.  Rows beyond R and depth
// beyond K hold zero digits.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mdg {

constexpr int kRowBlock = 16;   // rows per fragment
constexpr int kKcI8 = 64;       // depth per INT8 fragment
constexpr int kKcF64 = 16;      // depth per FP64 fragment
constexpr int kTile = 32;       // rows and columns per workgroup (2 x 2 waves)
constexpr int kTriMaxI8 = 32;   // INT8: up to this many diagonals in one band (whole triangle)
constexpr int kGmaxI8 = 16;     // INT8: widest band when S needs several bands
constexpr int kGmaxF64 = 16;    // widest band of diagonals, FP64 form
constexpr int kDuoMin = 36;     // INT8: S in [kDuoMin, kDuoMax], a multiple of 4, may run as two
constexpr int kDuoMax = 64;     //   bands of S/2 diagonals over the whole depth (one exactness chunk)

// S and band of the two-band INT8 contraction
inline bool duo_shape(int S, int band)
{
    return S % 4 == 0 && S >= kDuoMin && S <= kDuoMax && 2 * band == S;
}

// element (r, k), word w of an operand: p[w * ps + r * sr + k * sk]
struct Operand {
    const double* p;
    int64_t ps, sr, sk;
    int64_t R, K;
};

struct GemmArgs {
    const void* A;          // tiled digits of op(A)
    const void* B;          // tiled digits of op(B)^T (rows = columns of op(B))
    const int32_t* E;       // [M]
    const int32_t* F;       // [N]
    double* C;
    int64_t ldc, psc;
    int64_t M, N;
    int64_t nkc;            // depth chunks
    int64_t kcc;            // depth chunks per exact accumulation chunk
    int S, beta, band, nbands, m;
    int ncol;               // 32-bit columns of the exact fold accumulator
    int64_t* dbgD;          // optional [S][M][N]
    // Diagonal-sum buffer: when set, the banded kernels add their diagonal
    // sums here instead of folding in LDS (the first exactness chunk masks
    // the old contents to zero; every slot belongs to one band, so it needs
    // no clearing), and launch_gemm_final folds and rounds afterwards.  Tile-private layout: wave w of workgroup
    // tile (ty, tx) (gx = ceil(N/32) tiles per row, tiles of 32 gR rows)
    // keeps per diagonal t its 64 lanes x 4 gR consecutive int64, slot
    // r*4 + o holding output o of the lane in its row block r:
    //   ((((ty gx + tx) 4 + w) S + t) 64 + lane) 4 gR + r*4 + o.
    int64_t* gD;
    int gR;                 // row blocks per wave of that layout (1 or 2)
    int gI8;                // accumulator rows as in the INT8 (1) or FP64 (0) matrix cores
    // Fixed-point output (optional): the whole-triangle fixed-point kernels
    // and the buffer fold write the exact integers X (fixNL two's complement
    // 32-bit limb planes of M N entries, least significant first) and their
    // scales E_i + F_j - beta (S+1) instead of rounded words.
    int32_t* fixX;
    int32_t* fixScale;
    int fixNL;
};

// int64 elements of the diagonal-sum buffer for an M x N product
inline int64_t gd_elements(int64_t M, int64_t N, int S, int gR)
{
    const int64_t gy = (M + 32 * gR - 1) / (32 * gR), gx = (N + 31) / 32;
    return gy * gx * 4 * (int64_t)S * 64 * 4 * gR;
}

// Raise the kernel's dynamic LDS limit to at least `bytes` on the current
// device (once per kernel and device: later launches, also under stream
// capture, make no runtime call)
hipError_t ensure_dynamic_lds(const void* kernel, size_t bytes);

hipError_t launch_fill_zero(double* C, int m, int64_t M, int64_t N, int64_t ldc, int64_t psc,
                            hipStream_t st);

// Statistics of a call (int32 words, reset by launch_exp_init with stats):
// [0], [1] the span maxima of A and B; [2..3] the smallest magnitude
// product (uint64, starts at UINT64_MAX); [4], [5] the largest and
// smallest shared exponent of A's rows with a nonzero leading word, [6],
// [7] those of B's columns.
constexpr int kStatWords = 8;
hipError_t launch_exp_init(int32_t* hi, int32_t* lo, int64_t R, int32_t* stats, hipStream_t st);
hipError_t launch_exp_partial(const Operand& op, int32_t* hi, int32_t* lo, hipStream_t st);
// Both operands of a product at once: the exponent pass (as launch_exp_init,
// launch_exp_partial and launch_exp_final on each, stats laid out as they
// fill it: span maxima in words 0 and 1, extreme shared exponents of A in 4
// and 5, of B in 6 and 7) and the magnitude split (one INT8 slice of
// leading-word magnitudes on the shared-exponent grids, the ratio
// certificate's), in half the launches.
struct ExpSide {
    Operand op;
    int32_t *hi, *lo;        // working maxima and minima, op.R each
    int32_t* E;              // shared exponent + eoff per row
    int32_t* dbgE;           // optional
    int32_t *span_max, *ext;
    int rows_fast;           // rows contiguous (op.sr == 1 and op.sk != 1)
    int64_t nrb;             // row blocks of the magnitude split
    int8_t* q;               // magnitude digits
};
hipError_t launch_exp_pass2(const ExpSide& a, const ExpSide& b, int32_t* stats, int eoff, hipStream_t st);
hipError_t launch_split_mag2(const ExpSide& a, const ExpSide& b, int eoff, int64_t nkc, hipStream_t st);
// E[r] = shared exponent + eoff (2 for the balanced INT8 digits, else 0);
// dbgE gets the shared exponent itself; ext (optional) the largest and
// smallest shared exponent of the rows with a nonzero leading word
hipError_t launch_exp_final(const int32_t* hi, const int32_t* lo, int64_t R, int32_t* E,
                            int32_t* span_max, int32_t* ext, int32_t* dbgE, int eoff, hipStream_t st);
// Certificate of a call run on a slice-count hint: from stats (complete on
// the stream), writes an md_cert record to cert (device).  beta, S, band:
// the parameters used; T the target, m the words, K the depth.  With ph,
// stats are first made from the per-pair exponents and magnitude products
// of whole-pair inner products (LaneDotArgs::ph, pm; pm null: no magnitude
// certificate), every word written; a null cert then only makes stats.
hipError_t launch_cert(const int32_t* stats, int form, int64_t K, int T, int m, int beta, int S,
                       void* cert, hipStream_t st, const int32_t* ph = nullptr,
                       const unsigned long long* pm = nullptr, int64_t batch = 0);

// E[r] = Ein[r] + eoff where Ein[r] is at least the shared exponent (E[r] -
// eoff; -1100 for a row whose leading words are all zero, hi[r] = INT_MIN
// from the exponent pass) and at most 1100; else E[r] is kept and
// *flags |= 8
hipError_t launch_exp_set(const int32_t* Ein, const int32_t* hi, int64_t R, int eoff, int32_t* E,
                          int32_t* flags, hipStream_t st);

// INT8 digits: 7-bit sign-magnitude, or balanced 8-bit (E then holds the
// shared exponent + 2)
hipError_t launch_split_i8(const Operand& op, int m, const int32_t* E, int S, int64_t nrb,
                           int64_t nkc, int8_t* out, int32_t* dbg, bool balanced, hipStream_t st);
// OR of the input-precondition flags of every entry of op into *flags
// (1 not finite, 2 not weakly nonoverlapping, 4 leading word out of range)
hipError_t launch_validate(const Operand& op, int m, int32_t* flags, hipStream_t st);
hipError_t launch_split_f64(const Operand& op, int m, const int32_t* E, int S, int beta,
                            int64_t nrb, int64_t nkc, double* out, int32_t* dbg, hipStream_t st);

hipError_t launch_gemm_i8(const GemmArgs& a, hipStream_t st);
// minP[0] = min over (i < M, j < N) of sum_k qA_ik qB_kj (must start at
// UINT64_MAX); qA, qB from launch_split_mag2, nkc depth fragments each.
hipError_t launch_mag_min(const void* qA, const void* qB, int64_t M, int64_t N, int64_t nkc,
                          unsigned long long* minP, hipStream_t st);
hipError_t launch_gemm_f64(const GemmArgs& a, hipStream_t st);
// exact fold and rounding of every output from a.gD (one thread per entry)
hipError_t launch_gemm_final(const GemmArgs& a, hipStream_t st);
// whole-triangle INT8 kernels, by digit width (7 or 8 bits) and range of S
// (one translation unit each)
hipError_t launch_tri_s1_22(const GemmArgs& a, hipStream_t st);
hipError_t launch_tri_s23_28(const GemmArgs& a, hipStream_t st);
hipError_t launch_tri_s29_32(const GemmArgs& a, hipStream_t st);
hipError_t launch_tri8_s1_22(const GemmArgs& a, hipStream_t st);
hipError_t launch_tri8_s23_28(const GemmArgs& a, hipStream_t st);
hipError_t launch_tri8_s29_32(const GemmArgs& a, hipStream_t st);
// whole-triangle kernels with the A fragments shared through LDS (one
// exactness chunk, no debug dump or fixed-point output), for the (S, beta)
// of trid_shape
bool trid_shape(int S, int beta);
hipError_t launch_trid(const GemmArgs& a, hipStream_t st);
// two-band kernels (duo_shape, one exactness chunk, no debug dump or
// fixed-point output), by digit width and range of S
hipError_t launch_duo_s36_48(const GemmArgs& a, hipStream_t st);
hipError_t launch_duo_s52_64(const GemmArgs& a, hipStream_t st);
hipError_t launch_duo8_s36_48(const GemmArgs& a, hipStream_t st);
hipError_t launch_duo8_s52_64(const GemmArgs& a, hipStream_t st);
// their fixed-point variants (a.fixX set, one exactness chunk)
hipError_t launch_trifix_s1_22(const GemmArgs& a, hipStream_t st);
hipError_t launch_trifix_s23_32(const GemmArgs& a, hipStream_t st);
hipError_t launch_trifix8_s1_22(const GemmArgs& a, hipStream_t st);
hipError_t launch_trifix8_s23_32(const GemmArgs& a, hipStream_t st);

// Batched inner products out_b = sum_k x_bk y_bk: both operands are split
// with the vectors as rows (fragment layout of op(A)), so block rb of 16
// pairs multiplies row block rb of X with row block rb of Y and keeps the
// diagonal of each 16 x 16 slice product.
struct DotArgs {
    const void* X;       // digit fragments of X (rows = vectors)
    const void* Y;       // digit fragments of Y
    int64_t* D;          // S x batch diagonal sums, zeroed before the launch
    int64_t batch, nkc;  // pairs, depth fragments
    int64_t range;       // depth fragments per workgroup (within one exactness chunk)
    int S, band, nbands;
};
hipError_t launch_dot_diag(const DotArgs& a, int form_int8, hipStream_t st);

// Batched INT8 inner products with the digits cut in registers and
// multiplied lane-wise (no digit planes): one workgroup of 64 nw threads per
// pair and depth range [y chunk, (y+1) chunk); containers of SC digits (a
// multiple of 8, S <= SC, within lane_sc_range(m)).
struct LaneDotArgs {
    const double* X;       // pair b, entry k, word w at X[w psx + b ldx + k]
    int64_t ldx, psx;
    const double* Y;
    int64_t ldy, psy;
    int64_t batch, n;
    int64_t b0;            // first pair of a launch (set by the launcher)
    int64_t chunk;         // depth per workgroup
    const int32_t* E;      // grid exponents (shared exponent + eoff) of the
    const int32_t* F;      //   exponent pass, unless whole-pair mode
    int32_t* ph;           // whole-pair mode: per pair, the largest and smallest frexp
                           //   exponent of x's leading words, then of y's (4 planes of
                           //   batch; INT_MIN / INT_MAX for none), for launch_cert
    unsigned long long* pm;  // whole-pair mode with mag: per pair, sum_k qx_k qy_k
    int64_t* D;            // [S][batch] diagonal sums (several chunks per pair)
    double* out;           // one chunk per pair: out_b, word t at out[t pso + b]
    int64_t pso;
    int S, eoff;
    int full;              // whole-pair mode: chunk >= n, exponents found here
    int mag;               // whole-pair mode: also the magnitude certificate
    int atomic;            // several chunks per pair: add into a zeroed D, no rounding
};
// The slice rule's statistics pass of batched inner products, one
// workgroup per pair: E, F (shared exponents plus eoff), the per-pair
// leading exponents ph (as LaneDotArgs::ph) and, with pm, the magnitude
// products; launch_cert with ph (and no record) reduces them to stats.
hipError_t launch_dot_pre(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t batch, int64_t n,
                          int eoff, int32_t* E, int32_t* F, int32_t* ph, unsigned long long* pm, hipStream_t st);
// SC range of the lane kernels for m words (0, 0 if none)
void lane_sc_range(int m, int& lo, int& hi);
// steps of 4 entries per lane whose int32 diagonal sums stay exact
int64_t lane_steps_limit(int SC);
hipError_t launch_dot_lane(const LaneDotArgs& a, int m, int SC, bool balanced, int nw, int64_t nch,
                           hipStream_t st);
hipError_t launch_dot_lane_m1(const LaneDotArgs& a, int SC, bool balanced, int nw, int64_t nch, hipStream_t st);
hipError_t launch_dot_lane_m2(const LaneDotArgs& a, int SC, bool balanced, int nw, int64_t nch, hipStream_t st);
hipError_t launch_dot_lane_m4(const LaneDotArgs& a, int SC, bool balanced, int nw, int64_t nch, hipStream_t st);
// The matrix-core kernels of batched inner products (digit positions on
// the tile rows, entries on the depth; m = 8 and 16): SC range for m words (0, 0
// if none), the depth a workgroup may take, and the launch (grid batch x
// nch of two-wave workgroups; LaneDotArgs as for the lane kernels).
void mma_sc_range(int m, int& lo, int& hi);
int64_t mma_depth_limit();
hipError_t launch_dot_mma(const LaneDotArgs& a, int m, int SC, bool balanced, int64_t nch, hipStream_t st);
hipError_t launch_dot_mma_m8(const LaneDotArgs& a, int SC, bool balanced, int64_t nch, hipStream_t st);
hipError_t launch_dot_mma_m16(const LaneDotArgs& a, int SC, bool balanced, int64_t nch, hipStream_t st);
hipError_t launch_fill_zero_i64(int64_t* p, int64_t n, hipStream_t st);
// out_b (m words, plane stride pso) from the diagonal sums: exact fold and
// greedy rounding, ncol 32-bit fold columns per pair
hipError_t launch_dot_final(const int64_t* D, const int32_t* E, const int32_t* F, int64_t batch,
                            int S, int beta, int ncol, int m, double* out, int64_t pso,
                            hipStream_t st);
// Fixed-point results.  X [nlimb][M N] (two's complement 32-bit limbs,
// least significant first) and scale [M N] of sum_t D_t 2^(beta (S-1-t)),
// D [S][M N]; scale = E_i + F_j + 2 eoff - beta (S+1); ncol: the fold width
// in 32-bit columns (registers); E, F unshifted.
hipError_t launch_fixed_from_D(const int64_t* D, int S, int beta, int64_t M, int64_t N,
                               const int32_t* E, const int32_t* F, int eoff, int ncol, int32_t* X,
                               int nlimb, int32_t* scale, hipStream_t st);
// Z = X + Y mod 2^(32 nlimb), limb planes of count entries
hipError_t launch_fixed_add(int64_t count, int nlimb, const int32_t* X, const int32_t* Y, int32_t* Z,
                            hipStream_t st);
// greedy round to nearest of X 2^scale into m words (plane stride psc)
hipError_t launch_fixed_round(int m, int64_t count, int nlimb, const int32_t* X, const int32_t* scale,
                              double* C, int64_t psc, hipStream_t st);

// ordinary m-double product (m = 1, 2, 4, 8) of dense planes
hipError_t launch_ordinary(int m, const double* A, const double* B, double* C, int64_t M,
                           int64_t N, int64_t K, hipStream_t st);
// batched ordinary inner products (m = 1, 2, 4, 8, 16): dense planes X, Y
// of batch x n, out with plane stride pso; one wave per pair
hipError_t launch_ordinary_dot(int m, const double* X, const double* Y, double* out, int64_t pso,
                               int64_t batch, int64_t n, hipStream_t st);
// the same for m = 16 (a unit of its own)
hipError_t launch_ordinary_dot16(const double* X, const double* Y, double* out, int64_t pso, int64_t batch,
                                 int64_t n, hipStream_t st);
// min over pairs of sum_k qX_bk qY_bk into *minP (atomic min)
hipError_t launch_mag_min_diag(const void* qX, const void* qY, int64_t batch, int64_t nkc,
                               unsigned long long* minP, hipStream_t st);

}  // namespace mdg
