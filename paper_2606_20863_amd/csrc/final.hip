// Exact fold and rounding of every output from the diagonal-sum buffer that
// the banded kernels fill (INT8 beyond 32 diagonals; FP64 where the LDS fold
// does not fit): X = sum_t D_t 2^(beta (S-1-t)), then greedy round to
// nearest of X 2^(E_i + F_j - beta (S+1)) into m words.
#include "mdgemm_internal.h"
#include "renorm.h"

namespace mdg {
namespace {

constexpr int kRing = 8;   // diagonal sums in flight per thread

// One thread per slot of the buffer's layout, so that the reads of each
// diagonal are contiguous across the block: block (tile, wave, h) takes
// slots [256 h, 256 h + 256) of that wave (gR = 2 has two such halves),
// thread u lane u / 4gR, row block r and accumulator element o from
// u mod 4gR.  The entry follows from the matrix cores' row mapping (INT8:
// row 4 (lane/16) + o; FP64: row 4 o + lane/16); slots of padded rows or
// columns are read but not written.
//
// The fold runs from the least significant end: D_t sits at bit
// beta (S-1-t), so taking t = S-1, S-2, .. the positions rise; a signed
// 128-bit window holds the part of X from bit 32 k up, and when the next
// sum starts at or above bit 32 (k+1), the window's low 32 bits are limb k.
// NL 32-bit limbs (NL >= the fold width, so the window ends as the sign)
// stay in registers: the limb index is the unrolled loop's; the diagonal
// index is a runtime count, served from a ring of prefetched sums.  Then the
// magnitude is rounded greedily, word by word (the triangle kernels'
// register renormalisation).  With a debug buffer the sums are also written
// there as [S][M][N].  FIX: the folded integer itself (two's complement
// limbs, the window's sign past NL) and its scale go to a.fixX and
// a.fixScale instead of rounded words.
template <int NL, bool FIX>
__global__ __launch_bounds__(256) void k_gemm_final(GemmArgs a)
{
    const int R = a.gR;
    const int64_t gx = (a.N + kTile - 1) / kTile;
    const int64_t blk = blockIdx.x;
    const int h = (int)(blk % R);
    const int wave = (int)((blk / R) % 4);
    const int64_t tile = blk / (4 * R);
    const int64_t ty = tile / gx, tx = tile % gx;
    const int u = h * 256 + (int)threadIdx.x;
    const int lane = u / (4 * R), slot = u % (4 * R);
    const int r = slot / 4, o = slot % 4;
    const int i16 = a.gI8 ? 4 * (lane / 16) + o : 4 * o + lane / 16;
    const int64_t i = ty * (kTile * R) + (wave >> 1) * (16 * R) + r * 16 + i16;
    const int64_t j = tx * kTile + (wave & 1) * 16 + (lane & 15);
    const bool ok = i < a.M && j < a.N;
    const int64_t stride = 256 * (int64_t)R;   // between diagonals
    const int64_t* src = a.gD + (tile * 4 + wave) * (int64_t)a.S * stride + u;

    int64_t ring[kRing];
#pragma unroll
    for (int q = 0; q < kRing; ++q) {
        const int tq = a.S - 1 - q;
        const int64_t v = src[(int64_t)max(tq, 0) * stride];
        ring[q] = tq >= 0 ? v : 0;
    }
    uint32_t L[NL];
    __int128 win = 0;
    int t = a.S - 1, p = 0;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        while (t >= 0 && p < 32 * (k + 1)) {
            const int64_t v = ring[0];
#pragma unroll
            for (int q = 0; q + 1 < kRing; ++q)
                ring[q] = ring[q + 1];
            const int tn = t - kRing;
            const int64_t ld = src[(int64_t)max(tn, 0) * stride];
            ring[kRing - 1] = tn >= 0 ? ld : 0;
            win += (__int128)v << (p - 32 * k);
            if (a.dbgD && ok)
                a.dbgD[((int64_t)t * a.M + i) * a.N + j] = v;
            --t;
            p += a.beta;
        }
        L[k] = (uint32_t)(uint64_t)win;
        win >>= 32;
    }
    if constexpr (FIX) {
        if (!ok)
            return;
        const int64_t count = a.M * a.N, e = i * a.N + j;
        for (int k = 0; k < a.fixNL; ++k) {
            uint32_t v = win < 0 ? 0xffffffffu : 0u;
#pragma unroll
            for (int q = 0; q < NL; ++q)
                v = q == k ? L[q] : v;
            a.fixX[(int64_t)k * count + e] = (int32_t)v;
        }
        a.fixScale[e] = a.E[i] + a.F[j] - a.beta * (a.S + 1);
        return;
    }
    // magnitude (two's complement negation when X < 0)
    const bool neg = win < 0;
    uint64_t cy = 1;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const uint64_t v = (uint64_t)(~L[k]) + cy;
        cy = v >> 32;
        L[k] = neg ? (uint32_t)v : L[k];
    }
    double sgn = neg ? -1.0 : 1.0;
    int scale = ok ? a.E[i] + a.F[j] - a.beta * (a.S + 1) : 0;
    double* out = a.C + (ok ? i * a.ldc + j : 0);
    for (int w = 0; w < a.m; ++w) {
        const double wv = rn_next(L, sgn, scale);
        if (ok)
            out[w * a.psc] = wv;
    }
}

template <int NL>
hipError_t launch_final(const GemmArgs& a, unsigned blocks, hipStream_t st)
{
    if (a.fixX)
        hipLaunchKernelGGL((k_gemm_final<NL, true>), dim3(blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_gemm_final<NL, false>), dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_final(const GemmArgs& a, hipStream_t st)
{
    // one block per (tile, wave, half of the wave's slots)
    const int64_t gy = (a.M + kTile * a.gR - 1) / (kTile * a.gR), gx = (a.N + kTile - 1) / kTile;
    const int64_t blocks = gy * gx * 4 * a.gR;
    if (blocks > 0x7fffffff)
        return hipErrorInvalidValue;
    // limbs: the fold width a.ncol (32-bit columns, with margin) rounded up
    const unsigned b = (unsigned)blocks;
    if (a.ncol <= 8) return launch_final<8>(a, b, st);
    if (a.ncol <= 12) return launch_final<12>(a, b, st);
    if (a.ncol <= 16) return launch_final<16>(a, b, st);
    if (a.ncol <= 20) return launch_final<20>(a, b, st);
    if (a.ncol <= 24) return launch_final<24>(a, b, st);
    if (a.ncol <= 32) return launch_final<32>(a, b, st);
    if (a.ncol <= 40) return launch_final<40>(a, b, st);
    if (a.ncol <= 48) return launch_final<48>(a, b, st);
    if (a.ncol <= 64) return launch_final<64>(a, b, st);
    if (a.ncol <= 80) return launch_final<80>(a, b, st);
    return hipErrorInvalidValue;
}

}  // namespace mdg
