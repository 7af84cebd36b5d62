// C ABI of the m-double product library: argument checking, parameter rule,
// scratch memory and the launch sequence on the caller's stream.
#include "../../include/mdgemm.h"
#include "mdgemm_internal.h"
#include "rule.h"

#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>

using namespace mdg;

namespace mdg {

namespace {
std::mutex g_attr_mu;
struct AttrSet {
    int dev;
    const void* kernel;
    size_t bytes;
};
AttrSet g_attr[256];
int g_nattr = 0;
}  // namespace

hipError_t ensure_dynamic_lds(const void* kernel, size_t bytes)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    std::lock_guard<std::mutex> lk(g_attr_mu);
    int slot = -1;
    for (int q = 0; q < g_nattr; ++q)
        if (g_attr[q].dev == dev && g_attr[q].kernel == kernel) {
            if (g_attr[q].bytes >= bytes)
                return hipSuccess;
            slot = q;
        }
    if ((e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess)
        return e;
    if (slot < 0 && g_nattr < 256)
        slot = g_nattr++;
    if (slot >= 0)
        g_attr[slot] = AttrSet{dev, kernel, bytes};
    return hipSuccess;
}

}  // namespace mdg

namespace {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e)
{
    g_last_hip = (int)e;
    return MD_EHIP;
}

int ceil_log2(int64_t n) { return rule_ceil_log2(n); }

bool is_i8(int form) { return form == MD_FORM_INT8 || form == MD_FORM_INT8_BAL; }

// the digit grid of a row starts at 2^(E + grid_offset)
int grid_offset(int form) { return form == MD_FORM_INT8_BAL ? 2 : 0; }

// largest digit magnitude
int64_t digit_max(int form, int beta)
{
    return form == MD_FORM_INT8_BAL ? 128 : ((int64_t)1 << beta) - 1;
}

void band_round(int Smin, int gmax, int single, int& S, int& band)
{
    rule_band_round(Smin, gmax, single, S, band);
}

// Largest multiple of gran with S * kc * dmax^2 < limit (dmax the largest
// digit magnitude), capped at K rounded up to gran.
int64_t chunk_depth(int S, int64_t dmax, int64_t K, int64_t limit, int gran)
{
    const int64_t per = (int64_t)S * dmax * dmax;
    int64_t kc = ((limit - 1) / per) / gran * gran;
    const int64_t kfull = (std::max<int64_t>(K, 1) + gran - 1) / gran * gran;
    return std::min(kc, kfull);
}

// The two-band INT8 contraction takes S (a multiple of 4 in [36, 64]) when
// its whole depth is one exactness chunk.
bool duo_fits(int S, int64_t dmax, int64_t K)
{
    if (S % 4 || S < kDuoMin || S > kDuoMax)
        return false;
    const int64_t kfull = (std::max<int64_t>(K, 1) + kKcI8 - 1) / kKcI8 * kKcI8;
    return chunk_depth(S, dmax, K, (int64_t)1 << 31, kKcI8) >= kfull;
}

// INT8 slices: S = the budget's Smin up to 32 (one triangle); above that
// Smin rounded up to a multiple of 4 (at least 36) in two bands of S/2 when
// one exactness chunk holds the depth (and duo: the caller's kernels take
// two bands), else equal bands of at most 16.
int choose_i8(int Smin, int64_t dmax, int64_t K, bool duo, int& S, int64_t& kc, int& band)
{
    const int S4 = std::max(kDuoMin, (Smin + 3) / 4 * 4);
    if (duo && Smin > kTriMaxI8 && duo_fits(S4, dmax, K)) {
        S = S4;
        band = S4 / 2;
    } else {
        band_round(Smin, kGmaxI8, kTriMaxI8, S, band);
    }
    kc = chunk_depth(S, dmax, K, (int64_t)1 << 31, kKcI8);
    return kc > 0 ? MD_OK : MD_ERANGE;
}

int choose(int form, int64_t K, int T, int G, int& beta, int& S, int64_t& kc, int& band, bool duo = true)
{
    if (T < 1 || G < 0 || K < 0)
        return MD_EINVAL_OPT;
    if (form == MD_FORM_INT8) {
        beta = 7;
        return choose_i8(rule_slice_count(7, T, G), 127, K, duo, S, kc, band);
    }
    if (form == MD_FORM_INT8_BAL) {
        beta = 8;
        return choose_i8(rule_slice_count_balanced(T, G), 128, K, duo, S, kc, band);
    }
    if (form == MD_FORM_FP64) {
        bool found = false;
        for (int b = 8; b <= 24; ++b) {
            int s, bd;
            band_round(rule_slice_count(b, T, G), kGmaxF64, 0, s, bd);
            const int64_t k = chunk_depth(s, ((int64_t)1 << b) - 1, K, (int64_t)1 << 53, kKcF64);
            if (k <= 0)
                continue;
            if (!found || s < S || (s == S && k > kc)) {
                found = true;
                beta = b;
                S = s;
                kc = k;
                band = bd;
            }
        }
        return found ? MD_OK : MD_ERANGE;
    }
    return MD_EINVAL_OPT;
}

// 32-bit columns of the exact fold: X < K 2^(beta (S+1) + 1), plus carries
int fold_columns(int beta, int S, int64_t Kp)
{
    return (beta * (S + 1) + ceil_log2(std::max<int64_t>(Kp, 1)) + 2 + 31) / 32 + 3;
}

int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

// The [S][M][N] diagonal-sum buffer: the banded INT8 kernels always use it
// (two row blocks per wave), the FP64 bands when their LDS fold (4 waves x
// ncol x 256 int64) exceeds the 160 KB of LDS; the whole-triangle INT8
// kernels fold in registers.
bool needs_global_fold(int form, int band, int S, int ncol)
{
    if (is_i8(form))
        return !(band == S && S <= kTriMaxI8) && !duo_shape(S, band);
    return (size_t)4 * ncol * 256 * sizeof(int64_t) > 160 * 1024;
}

struct Span {
    uintptr_t lo, hi;  // [lo, hi) in bytes; empty if lo == hi
};

Span extent(const double* p, int m, int64_t R, int64_t Cc, int64_t ld_r, int64_t ld_c, int64_t ps)
{
    if (R == 0 || Cc == 0)
        return {0, 0};
    const int64_t last = (int64_t)(m - 1) * ps + (R - 1) * ld_r + (Cc - 1) * ld_c;
    const uintptr_t lo = (uintptr_t)p;
    return {lo, lo + (uintptr_t)(last + 1) * sizeof(double)};
}

bool overlap(Span a, Span b) { return a.lo < a.hi && b.lo < b.hi && a.lo < b.hi && b.lo < a.hi; }

bool mul_ok(int64_t a, int64_t b) { return a == 0 || b <= INT64_MAX / a; }

std::mutex g_pool_mu;
hipMemPool_t g_pool[64];
bool g_pool_init[64];

// Scratch of md_gemm_ex_noalloc: one array in every device's global memory,
// held until the process ends.  Host code takes its device address from
// hipGetSymbolAddress (once per device, with that device current) and
// passes that address on; the array's name itself is only a host-side
// stand-in.
static __device__ __align__(256) char noalloc_scratch[MD_NOALLOC_SCRATCH_BYTES];
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[64];

int noalloc_scratch_address(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e);
    if (dev < 0 || dev >= 64)
        return MD_EINVAL_OPT;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (e != hipSuccess)
            return hip_fail(e);
        g_noalloc_ptr[dev] = p;
    }
    *out = g_noalloc_ptr[dev];
    return MD_OK;
}

int get_pool(hipMemPool_t& pool)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e);
    if (dev < 0 || dev >= 64)
        return MD_EINVAL_OPT;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (!g_pool_init[dev]) {
        hipMemPoolProps props;
        memset(&props, 0, sizeof(props));
        props.allocType = hipMemAllocationTypePinned;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        e = hipMemPoolCreate(&g_pool[dev], &props);
        if (e != hipSuccess)
            return hip_fail(e);
        uint64_t keep = UINT64_MAX;
        e = hipMemPoolSetAttribute(g_pool[dev], hipMemPoolAttrReleaseThreshold, &keep);
        if (e != hipSuccess)
            return hip_fail(e);
        g_pool_init[dev] = true;
    }
    pool = g_pool[dev];
    return MD_OK;
}

// Scratch: either the caller's workspace (bump allocation) or pool memory.
struct Scratch {
    char* user = nullptr;
    size_t user_bytes = 0, used = 0;
    hipStream_t st = nullptr;
    void* owned[8] = {};
    int nowned = 0;

    int get(size_t bytes, void** out)
    {
        bytes = (bytes + 255) / 256 * 256;
        if (user) {
            if (used + bytes > user_bytes)
                return MD_ENOMEM;
            *out = user + used;
            used += bytes;
            return MD_OK;
        }
        hipMemPool_t pool;
        int rc = get_pool(pool);
        if (rc)
            return rc;
        hipError_t e = hipMallocFromPoolAsync(out, std::max<size_t>(bytes, 256), pool, st);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return MD_ENOMEM;
        }
        if (nowned == 8) {
            (void)hipFreeAsync(*out, st);
            return MD_ENOMEM;
        }
        owned[nowned++] = *out;
        return MD_OK;
    }
    ~Scratch()
    {
        for (int i = 0; i < nowned; ++i)
            (void)hipFreeAsync(owned[i], st);
    }
};

// Validation mode: the OR of the precondition flags of both operands, on
// the host (one synchronisation).  Returns MD_OK, MD_EINPUT or an error.
int validate_inputs(Scratch& scr, const Operand& a, const Operand& b, int m, md_info* info,
                    hipStream_t st)
{
    void* p;
    int rc = scr.get(256, &p);
    if (rc)
        return rc;
    int32_t* flags = (int32_t*)p;
    hipError_t e;
    if ((e = launch_fill_zero_i64((int64_t*)flags, 1, st)) != hipSuccess) return hip_fail(e);
    if ((e = launch_validate(a, m, flags, st)) != hipSuccess) return hip_fail(e);
    if ((e = launch_validate(b, m, flags, st)) != hipSuccess) return hip_fail(e);
    int32_t h = 0;
    if ((e = hipMemcpyAsync(&h, flags, sizeof(h), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(e);
    if ((e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(e);
    if (info)
        info->input_flags = h;
    return h ? MD_EINPUT : MD_OK;
}

size_t digits_bytes(int form, int64_t R, int64_t K, int S)
{
    const int64_t Rp = round_up(std::max<int64_t>(R, 1), kTile);
    if (is_i8(form))
        return (size_t)S * Rp * round_up(std::max<int64_t>(K, 1), kKcI8);
    return (size_t)S * Rp * round_up(std::max<int64_t>(K, 1), kKcF64) * sizeof(double);
}

size_t small_bytes(int64_t M, int64_t N)
{
    return (size_t)(3 * round_up(M + 64, 64) + 3 * round_up(N + 64, 64) + 64) * sizeof(int32_t) + 7 * 256;
}


// Slice parameters of a call and what the rule certified.
struct Choice {
    int beta = 0, S = 0, band = 0;
    int64_t kc = 0;
    int G = -1, G_span = -1, G_rho = -1, span_A = -1, span_B = -1;
    int flags = 0;              // md_info.input_flags bits of the rule (16: range)
    double log2_bound = 0.0;
};

// Option checks of the slice parameters (before any device work).  A given
// S splits into equal bands of at most 16 diagonals, or (duo: the call may
// use the two-band INT8 kernel) into two bands of S/2 over one exactness
// chunk of depth K.
int check_slice_opts(const md_opts& o, int64_t K, bool duo)
{
    if (o.force_S < 0 || o.force_S > 512 || o.s_hint < 0 || o.s_hint > 512)
        return MD_EINVAL_OPT;
    const int S = o.force_S > 0 ? o.force_S : o.s_hint;
    if (S == 0)
        return MD_OK;
    if (o.force_S == 0 && !o.cert)
        return MD_EINVAL_OPT;   // a hint needs the device record of its certificate
    // a given S must split into equal bands
    int s2, band;
    band_round(S, is_i8(o.form) ? kGmaxI8 : kGmaxF64, is_i8(o.form) ? kTriMaxI8 : 0, s2, band);
    if (s2 != S && !(duo && is_i8(o.form) && duo_fits(S, digit_max(o.form, o.form == MD_FORM_INT8 ? 7 : 8), K)))
        return MD_EINVAL_OPT;
    const int need = o.form == MD_FORM_INT8 ? 7 : o.form == MD_FORM_INT8_BAL ? 8 : 0;
    if (need)
        return o.force_beta == need || (o.force_S == 0 && o.force_beta == 0) ? MD_OK : MD_EINVAL_OPT;
    return o.force_beta >= 1 && o.force_beta <= 24 ? MD_OK : MD_EINVAL_OPT;
}

// Forced S (opts->force_S): no device reads.  Hint (opts->s_hint): the same
// parameters, and the certificate of the data is checked on the device into
// *opts->cert after the statistics (no wait).  Otherwise the rule: one copy
// of the statistics to the host and one synchronisation.  stats: the
// call's statistics (kStatWords), complete in stream order.
int choose_slices(const md_opts& o, int m, int64_t K, int T, const int32_t* stats, hipStream_t st, Choice& c,
                  bool duo, bool defer_cert = false)
{
    const int Sgiven = o.force_S > 0 ? o.force_S : o.s_hint;
    hipError_t e;
    if (Sgiven > 0) {
        c.beta = o.form == MD_FORM_INT8 ? 7 : o.form == MD_FORM_INT8_BAL ? 8 : o.force_beta;
        const int gmax = is_i8(o.form) ? kGmaxI8 : kGmaxF64;
        const int single = is_i8(o.form) ? kTriMaxI8 : 0;
        int s2;
        band_round(Sgiven, gmax, single, s2, c.band);
        if (duo && is_i8(o.form) && Sgiven > kTriMaxI8 && duo_fits(Sgiven, digit_max(o.form, c.beta), K))
            c.band = Sgiven / 2;   // two bands over the whole depth
        else if (s2 != Sgiven)
            return MD_EINVAL_OPT;   // a given S must split into equal bands
        c.S = Sgiven;
        c.kc = chunk_depth(c.S, digit_max(o.form, c.beta), K,
                           is_i8(o.form) ? ((int64_t)1 << 31) : ((int64_t)1 << 53), is_i8(o.form) ? kKcI8 : kKcF64);
        if (c.kc <= 0)
            return MD_ERANGE;
        if (o.force_S > 0)
            return MD_OK;
        c.log2_bound = __builtin_nan("");
        if (defer_cert)
            return MD_OK;   // the caller certifies once the statistics are made
        if ((e = launch_cert(stats, o.form, K, T, m, c.beta, c.S, o.cert, st)) != hipSuccess)
            return hip_fail(e);
        return MD_OK;
    }
    // the statistics into pinned host memory (one small buffer per host
    // thread, portable across devices, allocated at its first rule call and
    // never released): no staging copy on the way
    static thread_local int32_t* pinned = nullptr;
    if (!pinned && (e = hipHostMalloc((void**)&pinned, kStatWords * sizeof(int32_t), hipHostMallocPortable)) != hipSuccess) {
        pinned = nullptr;
        return hip_fail(e);
    }
    if ((e = hipMemcpyAsync(pinned, stats, kStatWords * sizeof(int32_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(e);
    if ((e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(e);
    int32_t h[kStatWords];
    memcpy(h, pinned, sizeof(h));
    c.span_A = h[0];
    c.span_B = h[1];
    c.G_span = h[0] + h[1] + 2;
    c.G = c.G_span;
    if (o.s_rule == MD_S_RHO) {
        uint64_t minP;
        memcpy(&minP, h + 2, sizeof(minP));
        c.G_rho = rule_rho_exponent(minP, K);
        if (c.G_rho >= 0 && c.G_rho < c.G)
            c.G = c.G_rho;
    }
    const int rc = choose(o.form, K, T, c.G, c.beta, c.S, c.kc, c.band, duo);
    if (rc)
        return rc;
    c.log2_bound = rule_log2_bound(o.form == MD_FORM_INT8_BAL, c.G, c.beta, c.S, m);
    if (!rule_in_range(h[4], h[5], h[6], h[7], K, c.G, T)) {
        c.flags |= 16;
        c.log2_bound = __builtin_inf();
    }
    return MD_OK;
}

void fill_info(md_info* in, const Choice& c, int T, bool validated)
{
    in->S = c.S;
    in->beta = c.beta;
    in->kc = (int)std::min<int64_t>(c.kc, INT_MAX);
    in->band = c.band;
    in->span_A = c.span_A;
    in->span_B = c.span_B;
    in->G = c.G;
    in->G_span = c.G_span;
    in->G_rho = c.G_rho;
    in->target_bits = T;
    in->log2_bound = c.log2_bound;
    in->input_flags = validated ? in->input_flags | c.flags : c.flags;
}

}  // namespace

extern "C" {

const char* md_strerror(int code)
{
    switch (code) {
    case MD_OK: return "success";
    case MD_EINVAL_M: return "m must be 1, 2, 4, 8 or 16";
    case MD_EINVAL_DIM: return "invalid size, leading dimension or plane stride";
    case MD_ENULL: return "NULL data pointer";
    case MD_EALIAS: return "an output overlaps an input or another output";
    case MD_ENOMEM: return "scratch allocation failed or workspace too small";
    case MD_EHIP: return "HIP runtime error (see md_last_hip_error)";
    case MD_EINVAL_OPT: return "invalid option";
    case MD_ERANGE: return "no exact slice parameters for this size and target";
    case MD_EINPUT: return "an input breaks the preconditions (validation mode) or a given shared exponent was not taken";
    default: return "unknown error";
    }
}

int md_last_hip_error(void) { return g_last_hip; }

int md_version(void) { return 30000; }

int md_choose_params(int form, int64_t K, int T, int G, int* beta, int* S, int* kc, int* band)
{
    int b = 0, s = 0, bd = 0;
    int64_t k = 0;
    const int rc = choose(form, K, T, G, b, s, k, bd);
    if (rc == MD_OK) {
        if (beta) *beta = b;
        if (S) *S = s;
        if (kc) *kc = (int)std::min<int64_t>(k, INT_MAX);
        if (band) *band = bd;
    }
    return rc;
}

// Launch shape of the lane-wise INT8 inner products for S slices, if a lane
// kernel holds S: containers of SC digits, 64 nw threads per workgroup,
// depth ranges of `chunk` entries (nch per pair), each within the steps
// whose int32 sums stay exact, and about 1024 workgroups where the pairs
// are few.
struct LanePlan {
    int SC = 0, nw = 0;
    int64_t chunk = 0, nch = 0;
    bool mma = false;   // the matrix-core kernel (digit positions on the tile rows)
};

// Batched inner products on the matrix cores for m = 8 and 16 (the lane
// kernels' S (S+1) / 2 byte products per four entries outweigh the cut
// there; at m <= 4 the lane kernels are faster): two-wave workgroups of 128
// entries per round, about 1024 workgroups or one per pair, at most
// mma_depth_limit() entries each.
bool plan_mma(int form, int m, int S, int64_t batch, int64_t n, LanePlan& p)
{
    if (!is_i8(form) || n <= 0 || (m != 8 && m != 16))
        return false;
    int lo, hi;
    mma_sc_range(m, lo, hi);
    const int SC = (S + 15) / 16 * 16;
    if (lo == 0 || SC < lo || SC > hi)
        return false;
    p.SC = SC;
    p.nw = 2;
    p.mma = true;
    constexpr int64_t round = 128;
    const int64_t cap = mma_depth_limit();
    const int64_t spread = std::min<int64_t>((1024 + batch - 1) / batch, (n + 4 * round - 1) / (4 * round));
    const int64_t nch = std::max<int64_t>({(n + cap - 1) / cap, spread, 1});
    p.chunk = round_up((n + nch - 1) / nch, round);
    p.nch = (n + p.chunk - 1) / p.chunk;
    return p.nch <= 65535;
}

bool plan_lane(int form, int m, int S, int64_t batch, int64_t n, LanePlan& p)
{
    if (plan_mma(form, m, S, batch, n, p))
        return true;
    if (!is_i8(form) || n <= 0)
        return false;
    int lo, hi;
    lane_sc_range(m, lo, hi);
    const int SC = (S + 7) / 8 * 8;
    if (lo == 0 || SC < lo || SC > hi)
        return false;
    p.SC = SC;
    // many pairs: two waves per pair, else (and for single words, whose
    // light steps leave the exponent scan more exposed) four
    p.nw = batch >= 512 && m > 1 ? 2 : 4;
    const int64_t stepw = 256 * p.nw;
    const int64_t cap = stepw * lane_steps_limit(SC);
    const int64_t spread = std::min<int64_t>((1024 + batch - 1) / batch, (n + 4 * stepw - 1) / (4 * stepw));
    const int64_t nch = std::max<int64_t>({(n + cap - 1) / cap, spread, 1});
    p.chunk = round_up((n + nch - 1) / nch, stepw);
    p.nch = (n + p.chunk - 1) / p.chunk;
    return p.nch <= 65535;
}

hipError_t launch_planned_dot(const LaneDotArgs& la, int m, const LanePlan& lp, bool balanced, hipStream_t st)
{
    if (lp.mma)
        return launch_dot_mma(la, m, lp.SC, balanced, lp.nch, st);
    return launch_dot_lane(la, m, lp.SC, balanced, lp.nw, lp.nch, st);
}

size_t md_dot_workspace_size(int form, int64_t batch, int64_t n, int S)
{
    // exponents and statistics, the two magnitude slices (slice rule), the
    // two digit planes (the FP64 form; INT8 cuts digits in registers where a
    // lane kernel holds S), the S x batch diagonal sums and the per-pair
    // statistics of whole-pair calls
    return small_bytes(batch, batch) + 2 * digits_bytes(MD_FORM_INT8, batch, n, 1) +
           2 * digits_bytes(form, batch, n, S) + (size_t)S * batch * sizeof(int64_t) +
           (size_t)batch * 24 + 4096;
}

size_t md_gemm_workspace_size(int form, int64_t M, int64_t N, int64_t K, int S)
{
    size_t bytes = small_bytes(M, N) + digits_bytes(MD_FORM_INT8, M, K, 1) +
                   digits_bytes(MD_FORM_INT8, N, K, 1) + digits_bytes(form, M, K, S) +
                   digits_bytes(form, N, K, S) + 4096;
    // the diagonal-sum buffer where the LDS fold does not fit (widest FP64
    // digits as the bound)
    const int kcg = is_i8(form) ? kKcI8 : kKcF64;
    const int ncol = fold_columns(is_i8(form) ? 8 : 24, S, round_up(std::max<int64_t>(K, 1), kcg));
    const bool global = is_i8(form) ? S > kTriMaxI8
                                    : (size_t)4 * ncol * 256 * sizeof(int64_t) > 160 * 1024;
    if (global)
        bytes += (size_t)gd_elements(M, N, S, is_i8(form) ? 2 : 1) * sizeof(int64_t) + 256;
    return bytes;
}

size_t md_workspace_size(int form, int64_t M, int64_t N, int64_t K, int S)
{
    return md_gemm_workspace_size(form, M, N, K, S);
}

}  // extern "C"

namespace {

// Exact fixed-point output of a product: nlimb limb planes X and scale.
struct FixedOut {
    int32_t* X;
    int32_t* scale;
    int nlimb;
};

// md_gemm_ex; E_in / F_in (optional, device, M and N entries): shared
// exponents that replace those of op(A)'s rows and op(B)'s columns (a
// forced S is then required: the rule's certificates hold for the data's
// own exponents only).  An override below the data's own exponent, or above
// 1100, is not taken: bit 8 goes into *exp_flags (device, zeroed by the
// caller) and the data's own exponent stays.  fx (optional): write the exact
// integers instead of C (C is then ignored): the whole-triangle INT8 kernels
// with one exactness chunk and the buffer fold write them directly; the other
// paths capture the diagonal sums in an [S][M][N] buffer and fold them after.
int gemm_impl(int m, int transA, int transB, int64_t M, int64_t N, int64_t K, const double* A,
              int64_t lda, int64_t plane_stride_A, const double* B, int64_t ldb,
              int64_t plane_stride_B, double* C, int64_t ldc, int64_t plane_stride_C,
              const md_opts* opts, void* stream, const int32_t* E_in, const int32_t* F_in,
              int32_t* exp_flags, const FixedOut* fx, bool noalloc = false)
{
    g_last_hip = 0;
    if (m != 1 && m != 2 && m != 4 && m != 8 && m != 16)
        return MD_EINVAL_M;
    if (M < 0 || N < 0 || K < 0)
        return MD_EINVAL_DIM;
    md_opts o;
    memset(&o, 0, sizeof(o));
    if (opts)
        o = *opts;
    if (o.form != MD_FORM_FP64 && !is_i8(o.form))
        return MD_EINVAL_OPT;
    if (o.s_rule != MD_S_SPAN && o.s_rule != MD_S_RHO)
        return MD_EINVAL_OPT;
    if (M == 0 || N == 0)
        return MD_OK;
    if ((!C && !fx) || (K > 0 && (!A || !B)))
        return MD_ENULL;
    if (fx && (K == 0 || !fx->X || !fx->scale))
        return MD_EINVAL_DIM;
    // leading dimensions and plane strides
    if (!fx && (ldc < N || plane_stride_C < 1))
        return MD_EINVAL_DIM;
    if (K > 0) {
        if (lda < (transA ? M : K) || ldb < (transB ? K : N) || plane_stride_A < 1 || plane_stride_B < 1)
            return MD_EINVAL_DIM;
    }
    if (!mul_ok(M, std::max<int64_t>(fx ? N : ldc, 1)) || !mul_ok(std::max<int64_t>(M, K), std::max<int64_t>(lda, 1)) ||
        !mul_ok(std::max<int64_t>(K, N), std::max<int64_t>(ldb, 1)) || M > (INT64_C(1) << 40) ||
        N > (INT64_C(1) << 40) || K > (INT64_C(1) << 40))
        return MD_EINVAL_DIM;
    const Span sc = fx ? Span{0, 0} : extent(C, m, M, N, ldc, 1, plane_stride_C);
    if (K > 0) {
        const Span sa = transA ? extent(A, m, K, M, lda, 1, plane_stride_A) : extent(A, m, M, K, lda, 1, plane_stride_A);
        const Span sb = transB ? extent(B, m, N, K, ldb, 1, plane_stride_B) : extent(B, m, K, N, ldb, 1, plane_stride_B);
        if (overlap(sc, sa) || overlap(sc, sb))
            return MD_EALIAS;
    }
    const int T = o.target_bits > 0 ? o.target_bits : 50 * m;
    // the two-band kernel writes neither the diagonal-sum dump nor integers
    const bool duo = !fx && !(o.dbg && o.dbg->D);
    if (check_slice_opts(o, K, duo) != MD_OK)
        return MD_EINVAL_OPT;
    if ((E_in || F_in) && (o.force_S == 0 || !exp_flags))
        return MD_EINVAL_OPT;
    // the dumps sized by S need S fixed before the call
    if (o.dbg && (o.dbg->digits_A || o.dbg->digits_B || o.dbg->D) && o.force_S == 0)
        return MD_EINVAL_OPT;

    hipStream_t st = (hipStream_t)stream;
    if (K == 0) {
        hipError_t e = launch_fill_zero(C, m, M, N, ldc, plane_stride_C, st);
        if (e != hipSuccess)
            return hip_fail(e);
        if (o.info) {
            memset(o.info, 0, sizeof(*o.info));
            o.info->target_bits = T;
            o.info->log2_bound = -1.0 / 0.0;
        }
        return MD_OK;
    }

    Operand opA{A, plane_stride_A, transA ? 1 : lda, transA ? lda : 1, M, K};
    Operand opB{B, plane_stride_B, transB ? ldb : 1, transB ? 1 : ldb, N, K};

    Scratch scr;
    scr.st = st;
    if (noalloc) {
        // md_gemm_ex_noalloc: the library's fixed array, never the pool
        void* p = nullptr;
        const int rc = noalloc_scratch_address(&p);
        if (rc)
            return rc;
        scr.user = (char*)p;
        scr.user_bytes = MD_NOALLOC_SCRATCH_BYTES;
    } else if (o.workspace) {
        scr.user = (char*)o.workspace;
        scr.user_bytes = o.workspace_bytes;
    }
    if (o.validate) {
        const int rc = validate_inputs(scr, opA, opB, m, o.info, st);
        if (rc)
            return rc;
    }
    int32_t *hiA, *loA, *hiB, *loB, *E, *F, *stats;
    {
        void* p;
        int rc = scr.get(small_bytes(M, N), &p);
        if (rc)
            return rc;
        int32_t* q = (int32_t*)p;
        const int64_t Ma = round_up(M + 64, 64), Na = round_up(N + 64, 64);
        hiA = q; q += Ma;
        loA = q; q += Ma;
        E = q; q += Ma;
        hiB = q; q += Na;
        loB = q; q += Na;
        F = q; q += Na;
        stats = q;
    }
    md_debug* dbg = o.dbg;
    hipError_t e;
    const int eoff = grid_offset(o.form);
    // the exponent pass of both operands, one launch per step
    ExpSide sa{opA, hiA, loA, E, dbg ? dbg->E : nullptr, stats, stats + 4, (opA.sr == 1 && opA.sk != 1) ? 1 : 0,
               round_up(M, kTile) / kRowBlock, nullptr};
    ExpSide sb{opB, hiB, loB, F, dbg ? dbg->F : nullptr, stats + 1, stats + 6, (opB.sr == 1 && opB.sk != 1) ? 1 : 0,
               round_up(N, kTile) / kRowBlock, nullptr};
    if ((e = launch_exp_pass2(sa, sb, stats, eoff, st)) != hipSuccess)
        return hip_fail(e);
    if (E_in && (e = launch_exp_set(E_in, hiA, M, eoff, E, exp_flags, st)) != hipSuccess) return hip_fail(e);
    if (F_in && (e = launch_exp_set(F_in, hiB, N, eoff, F, exp_flags, st)) != hipSuccess) return hip_fail(e);

    const bool use_rho = o.force_S == 0 && o.s_rule == MD_S_RHO;
    if (use_rho) {
        // magnitude certificate: min_ij sum_k qA_ik qB_kj, q the 7-bit
        // leading-word magnitudes on the shared-exponent grid
        const int64_t nkm = (K + kKcI8 - 1) / kKcI8;
        void *qA, *qB;
        int rc = scr.get(digits_bytes(MD_FORM_INT8, M, K, 1), &qA);
        if (rc)
            return rc;
        rc = scr.get(digits_bytes(MD_FORM_INT8, N, K, 1), &qB);
        if (rc)
            return rc;
        sa.q = (int8_t*)qA;
        sb.q = (int8_t*)qB;
        if ((e = launch_split_mag2(sa, sb, eoff, nkm, st)) != hipSuccess)
            return hip_fail(e);
        if ((e = launch_mag_min(qA, qB, M, N, nkm, (unsigned long long*)(stats + 2), st)) != hipSuccess)
            return hip_fail(e);
    }
    Choice ch;
    {
        const int rc = choose_slices(o, m, K, T, stats, st, ch, duo);
        if (rc)
            return rc;
    }
    const int beta = ch.beta, S = ch.S, band = ch.band;
    const int64_t kc = ch.kc;
    const int kcg = is_i8(o.form) ? kKcI8 : kKcF64;
    const int64_t nkc = (K + kcg - 1) / kcg;
    const int64_t Mp = round_up(M, kTile), Np = round_up(N, kTile);
    const int ncol = fold_columns(beta, S, nkc * kcg);
    // the banded kernels fold in LDS when 4 waves' columns fit, else they
    // add their diagonal sums into a [S][M][N] buffer that a second kernel
    // folds and rounds (one entry per thread); the whole-triangle INT8
    // kernels fold in registers
    const bool global_fold = needs_global_fold(o.form, band, S, ncol);
    if ((size_t)ncol * 256 * sizeof(int64_t) > 160 * 1024)
        return MD_ERANGE;

    const int64_t kcc = std::max<int64_t>(kc / kcg, 1);
    int64_t* fixD = nullptr;
    md_debug fixdbg;
    if (fx) {
        const bool tri2 = is_i8(o.form) && band == S && S <= kTriMaxI8 && kcc >= nkc;
        if (!global_fold && !tri2) {
            // no direct fixed-point epilogue on this path: capture the
            // diagonal sums (the debug dump's route) and fold them after
            void *pD, *pC;
            int rc = scr.get((size_t)(M * N) * S * sizeof(int64_t), &pD);
            if (!rc)
                rc = scr.get((size_t)(M * N) * m * sizeof(double), &pC);
            if (rc)
                return rc;
            memset(&fixdbg, 0, sizeof(fixdbg));
            fixdbg.D = fixD = (int64_t*)pD;
            dbg = &fixdbg;
            C = (double*)pC;
            ldc = N;
            plane_stride_C = M * N;
        }
    }

    void *dA, *dB;
    int rc = scr.get(digits_bytes(o.form, M, K, S), &dA);
    if (rc)
        return rc;
    rc = scr.get(digits_bytes(o.form, N, K, S), &dB);
    if (rc)
        return rc;

    if (is_i8(o.form)) {
        const bool bal = o.form == MD_FORM_INT8_BAL;
        if ((e = launch_split_i8(opA, m, E, S, Mp / kRowBlock, nkc, (int8_t*)dA, dbg ? dbg->digits_A : nullptr, bal, st)) != hipSuccess)
            return hip_fail(e);
        if ((e = launch_split_i8(opB, m, F, S, Np / kRowBlock, nkc, (int8_t*)dB, dbg ? dbg->digits_B : nullptr, bal, st)) != hipSuccess)
            return hip_fail(e);
    } else {
        if ((e = launch_split_f64(opA, m, E, S, beta, Mp / kRowBlock, nkc, (double*)dA, dbg ? dbg->digits_A : nullptr, st)) != hipSuccess)
            return hip_fail(e);
        if ((e = launch_split_f64(opB, m, F, S, beta, Np / kRowBlock, nkc, (double*)dB, dbg ? dbg->digits_B : nullptr, st)) != hipSuccess)
            return hip_fail(e);
    }
    if (dbg && dbg->D) {
        if ((e = launch_fill_zero((double*)dbg->D, S, M, N, N, M * N, st)) != hipSuccess)
            return hip_fail(e);
    }
    int64_t* gD = nullptr;
    const int gR = is_i8(o.form) ? 2 : 1;   // row blocks per wave of the banded kernels
    if (global_fold) {
        // every slot is written by the first exactness chunk of its band:
        // no clearing
        const int64_t n = gd_elements(M, N, S, gR);
        void* p;
        if ((rc = scr.get((size_t)n * sizeof(int64_t), &p)))
            return rc;
        gD = (int64_t*)p;
    }
    GemmArgs ga;
    ga.A = dA;
    ga.B = dB;
    ga.E = E;
    ga.F = F;
    ga.C = C;
    ga.ldc = ldc;
    ga.psc = plane_stride_C;
    ga.M = M;
    ga.N = N;
    ga.nkc = nkc;
    ga.kcc = kcc;
    ga.S = S;
    ga.beta = beta;
    ga.band = band;
    ga.nbands = S / band;
    ga.m = m;
    ga.ncol = ncol;
    ga.dbgD = dbg ? dbg->D : nullptr;   // with the sum buffer, the final kernel fills it
    ga.gD = gD;
    ga.gR = gR;
    ga.gI8 = is_i8(o.form);
    ga.fixX = fx && !fixD ? fx->X : nullptr;
    ga.fixScale = fx && !fixD ? fx->scale : nullptr;
    ga.fixNL = fx ? fx->nlimb : 0;
    if (o.ev_gemm_begin && (e = hipEventRecord((hipEvent_t)o.ev_gemm_begin, st)) != hipSuccess)
        return hip_fail(e);
    e = is_i8(o.form) ? launch_gemm_i8(ga, st) : launch_gemm_f64(ga, st);
    if (e != hipSuccess)
        return hip_fail(e);
    if (global_fold && (e = launch_gemm_final(ga, st)) != hipSuccess)
        return hip_fail(e);
    // E and F hold the grid starts (shared exponent + offset): no offset here
    if (fixD && (e = launch_fixed_from_D(fixD, S, beta, M, N, E, F, 0, ncol, fx->X, fx->nlimb, fx->scale,
                                         st)) != hipSuccess)
        return hip_fail(e);
    if (o.ev_gemm_end && (e = hipEventRecord((hipEvent_t)o.ev_gemm_end, st)) != hipSuccess)
        return hip_fail(e);

    if (o.info)
        fill_info(o.info, ch, T, o.validate != 0);
    return MD_OK;
}

}  // namespace

extern "C" {

int md_gemm_ex(int m, int transA, int transB, int64_t M, int64_t N, int64_t K, const double* A,
               int64_t lda, int64_t plane_stride_A, const double* B, int64_t ldb,
               int64_t plane_stride_B, double* C, int64_t ldc, int64_t plane_stride_C,
               const md_opts* opts, void* stream)
{
    return gemm_impl(m, transA, transB, M, N, K, A, lda, plane_stride_A, B, ldb, plane_stride_B, C, ldc,
                     plane_stride_C, opts, stream, nullptr, nullptr, nullptr, nullptr);
}

int md_gemm_ex_noalloc(int m, int transA, int transB, int64_t M, int64_t N, int64_t K, const double* A,
                       int64_t lda, int64_t plane_stride_A, const double* B, int64_t ldb,
                       int64_t plane_stride_B, double* C, int64_t ldc, int64_t plane_stride_C,
                       const md_opts* opts, void* stream)
{
    g_last_hip = 0;
    if (opts && (opts->workspace || opts->workspace_bytes))
        return MD_EINVAL_OPT;   // the scratch is the library's own array
    return gemm_impl(m, transA, transB, M, N, K, A, lda, plane_stride_A, B, ldb, plane_stride_B, C, ldc,
                     plane_stride_C, opts, stream, nullptr, nullptr, nullptr, nullptr, true);
}

int md_dot_ex(int m, int64_t batch, int64_t n, const double* X, int64_t ldx, int64_t plane_stride_X,
              const double* Y, int64_t ldy, int64_t plane_stride_Y, double* out,
              int64_t plane_stride_out, const md_opts* opts, void* stream)
{
    g_last_hip = 0;
    if (m != 1 && m != 2 && m != 4 && m != 8 && m != 16)
        return MD_EINVAL_M;
    if (batch < 0 || n < 0)
        return MD_EINVAL_DIM;
    md_opts o;
    memset(&o, 0, sizeof(o));
    if (opts)
        o = *opts;
    if (o.form != MD_FORM_FP64 && !is_i8(o.form))
        return MD_EINVAL_OPT;
    if (o.s_rule != MD_S_SPAN && o.s_rule != MD_S_RHO)
        return MD_EINVAL_OPT;
    if (o.dbg)
        return MD_EINVAL_OPT;
    if (batch == 0)
        return MD_OK;
    if (!out || (n > 0 && (!X || !Y)))
        return MD_ENULL;
    if (m > 1 && plane_stride_out < batch)
        return MD_EINVAL_DIM;
    if (n > 0 && (ldx < n || ldy < n || plane_stride_X < 1 || plane_stride_Y < 1))
        return MD_EINVAL_DIM;
    if (!mul_ok(batch, std::max<int64_t>(ldx, 1)) || !mul_ok(batch, std::max<int64_t>(ldy, 1)) ||
        !mul_ok(m, std::max<int64_t>(plane_stride_out, 1)) || batch > (INT64_C(1) << 40) ||
        n > (INT64_C(1) << 40))
        return MD_EINVAL_DIM;
    const Span so = extent(out, m, 1, batch, 0, 1, std::max<int64_t>(plane_stride_out, 1));
    if (n > 0) {
        const Span sx = extent(X, m, batch, n, ldx, 1, plane_stride_X);
        const Span sy = extent(Y, m, batch, n, ldy, 1, plane_stride_Y);
        if (overlap(so, sx) || overlap(so, sy))
            return MD_EALIAS;
    }
    const int T = o.target_bits > 0 ? o.target_bits : 50 * m;
    if (check_slice_opts(o, n, false) != MD_OK)
        return MD_EINVAL_OPT;

    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (n == 0) {
        if ((e = launch_fill_zero(out, m, 1, batch, batch, std::max<int64_t>(plane_stride_out, 1), st)) !=
            hipSuccess)
            return hip_fail(e);
        if (o.info) {
            memset(o.info, 0, sizeof(*o.info));
            o.info->target_bits = T;
            o.info->log2_bound = -1.0 / 0.0;
        }
        return MD_OK;
    }

    // both operands with the vectors as rows
    Operand opX{X, plane_stride_X, ldx, 1, batch, n};
    Operand opY{Y, plane_stride_Y, ldy, 1, batch, n};

    Scratch scr;
    scr.st = st;
    if (o.workspace) {
        scr.user = (char*)o.workspace;
        scr.user_bytes = o.workspace_bytes;
    }
    if (o.validate) {
        const int rc = validate_inputs(scr, opX, opY, m, o.info, st);
        if (rc)
            return rc;
    }
    int32_t *hiX, *loX, *hiY, *loY, *E, *F, *stats;
    {
        void* p;
        int rc = scr.get(small_bytes(batch, batch), &p);
        if (rc)
            return rc;
        int32_t* q = (int32_t*)p;
        const int64_t Ba = round_up(batch + 64, 64);
        hiX = q; q += Ba;
        loX = q; q += Ba;
        E = q; q += Ba;
        hiY = q; q += Ba;
        loY = q; q += Ba;
        F = q; q += Ba;
        stats = q;
    }
    const int eoff = grid_offset(o.form);
    const bool use_rho = o.force_S == 0 && o.s_rule == MD_S_RHO;
    const int Sgiven = o.force_S > 0 ? o.force_S : o.s_hint;
    LanePlan lp;

    // A given S whose lane kernel takes each pair in one workgroup: that
    // kernel finds the exponents and the statistics itself, and the
    // certificate follows it.
    if (Sgiven > 0 && plan_lane(o.form, m, Sgiven, batch, n, lp) && lp.nch == 1) {
        Choice ch;
        int rc = choose_slices(o, m, n, T, stats, st, ch, false, true);
        if (rc)
            return rc;
        void* pp;
        rc = scr.get((size_t)batch * (4 * sizeof(int32_t) + sizeof(unsigned long long)), &pp);
        if (rc)
            return rc;
        unsigned long long* pm = (unsigned long long*)pp;
        int32_t* ph = (int32_t*)(pm + batch);
        LaneDotArgs la{opX.p, ldx, plane_stride_X, opY.p, ldy, plane_stride_Y, batch, n, 0, lp.chunk,
                       nullptr, nullptr, ph, pm, nullptr, out, std::max<int64_t>(plane_stride_out, 1),
                       ch.S, eoff, 1, use_rho ? 1 : 0, 0};
        if (o.ev_gemm_begin && (e = hipEventRecord((hipEvent_t)o.ev_gemm_begin, st)) != hipSuccess)
            return hip_fail(e);
        if ((e = launch_planned_dot(la, m, lp, o.form == MD_FORM_INT8_BAL, st)) != hipSuccess)
            return hip_fail(e);
        if (o.ev_gemm_end && (e = hipEventRecord((hipEvent_t)o.ev_gemm_end, st)) != hipSuccess)
            return hip_fail(e);
        if (o.force_S == 0 && (e = launch_cert(stats, o.form, n, T, m, ch.beta, ch.S, o.cert, st, ph,
                                               use_rho ? pm : nullptr, batch)) != hipSuccess)
            return hip_fail(e);
        if (o.info)
            fill_info(o.info, ch, T, o.validate != 0);
        return MD_OK;
    }

    const int64_t nrb = round_up(batch, kTile) / kRowBlock;
    if (is_i8(o.form) && (m <= 8 || m == 16) && (batch >= 64 || n <= 16384)) {
        // INT8 digits: exponents and magnitude products in one pass per pair
        void* pp;
        int rc = scr.get((size_t)batch * (4 * sizeof(int32_t) + sizeof(unsigned long long)), &pp);
        if (rc)
            return rc;
        unsigned long long* pm = (unsigned long long*)pp;
        int32_t* ph = (int32_t*)(pm + batch);
        if ((e = launch_dot_pre(opX.p, ldx, opY.p, ldy, batch, n, eoff, E, F, ph, use_rho ? pm : nullptr, st)) !=
            hipSuccess)
            return hip_fail(e);
        if ((e = launch_cert(stats, o.form, n, T, m, 0, 0, nullptr, st, ph, use_rho ? pm : nullptr, batch)) !=
            hipSuccess)
            return hip_fail(e);
    } else {
        ExpSide sx{opX, hiX, loX, E, nullptr, stats, stats + 4, (opX.sr == 1 && opX.sk != 1) ? 1 : 0, nrb, nullptr};
        ExpSide sy{opY, hiY, loY, F, nullptr, stats + 1, stats + 6, (opY.sr == 1 && opY.sk != 1) ? 1 : 0, nrb, nullptr};
        if ((e = launch_exp_pass2(sx, sy, stats, eoff, st)) != hipSuccess)
            return hip_fail(e);

        if (use_rho) {
            // magnitude certificate over the pairs: min_b sum_k qX_bk qY_bk
            const int64_t nkm = (n + kKcI8 - 1) / kKcI8;
            void *qX, *qY;
            int rc = scr.get(digits_bytes(MD_FORM_INT8, batch, n, 1), &qX);
            if (rc)
                return rc;
            rc = scr.get(digits_bytes(MD_FORM_INT8, batch, n, 1), &qY);
            if (rc)
                return rc;
            sx.q = (int8_t*)qX;
            sy.q = (int8_t*)qY;
            if ((e = launch_split_mag2(sx, sy, eoff, nkm, st)) != hipSuccess)
                return hip_fail(e);
            if ((e = launch_mag_min_diag(qX, qY, batch, nkm, (unsigned long long*)(stats + 2), st)) != hipSuccess)
                return hip_fail(e);
        }
    }
    Choice ch;
    {
        const int rc = choose_slices(o, m, n, T, stats, st, ch, false);
        if (rc)
            return rc;
    }
    const int beta = ch.beta, S = ch.S, band = ch.band;
    const int64_t kc = ch.kc;
    const int kcg = is_i8(o.form) ? kKcI8 : kKcF64;
    const int64_t nkc = (n + kcg - 1) / kcg;
    const int ncol = fold_columns(beta, S, nkc * kcg);
    if ((size_t)ncol * 256 * sizeof(int64_t) > 160 * 1024)
        return MD_ERANGE;

    void* Dp;
    int rc = scr.get((size_t)S * batch * sizeof(int64_t), &Dp);
    if (rc)
        return rc;
    if (plan_lane(o.form, m, S, batch, n, lp)) {
        // INT8 digits cut in registers, no digit planes
        if (lp.nch > 1 && (e = launch_fill_zero_i64((int64_t*)Dp, (int64_t)S * batch, st)) != hipSuccess)
            return hip_fail(e);
        LaneDotArgs la{opX.p, ldx, plane_stride_X, opY.p, ldy, plane_stride_Y, batch, n, 0, lp.chunk,
                       E, F, nullptr, nullptr, (int64_t*)Dp, out, std::max<int64_t>(plane_stride_out, 1),
                       S, eoff, 0, 0, lp.nch > 1 ? 1 : 0};
        if (o.ev_gemm_begin && (e = hipEventRecord((hipEvent_t)o.ev_gemm_begin, st)) != hipSuccess)
            return hip_fail(e);
        if ((e = launch_planned_dot(la, m, lp, o.form == MD_FORM_INT8_BAL, st)) != hipSuccess)
            return hip_fail(e);
        if (lp.nch == 1) {
            // the lane kernel rounded every pair itself
            if (o.ev_gemm_end && (e = hipEventRecord((hipEvent_t)o.ev_gemm_end, st)) != hipSuccess)
                return hip_fail(e);
            if (o.info)
                fill_info(o.info, ch, T, o.validate != 0);
            return MD_OK;
        }
    } else {
        void *dX, *dY;
        rc = scr.get(digits_bytes(o.form, batch, n, S), &dX);
        if (rc)
            return rc;
        rc = scr.get(digits_bytes(o.form, batch, n, S), &dY);
        if (rc)
            return rc;
        if (is_i8(o.form)) {
            const bool bal = o.form == MD_FORM_INT8_BAL;
            if ((e = launch_split_i8(opX, m, E, S, nrb, nkc, (int8_t*)dX, nullptr, bal, st)) != hipSuccess)
                return hip_fail(e);
            if ((e = launch_split_i8(opY, m, F, S, nrb, nkc, (int8_t*)dY, nullptr, bal, st)) != hipSuccess)
                return hip_fail(e);
        } else {
            if ((e = launch_split_f64(opX, m, E, S, beta, nrb, nkc, (double*)dX, nullptr, st)) != hipSuccess)
                return hip_fail(e);
            if ((e = launch_split_f64(opY, m, F, S, beta, nrb, nkc, (double*)dY, nullptr, st)) != hipSuccess)
                return hip_fail(e);
        }
        if ((e = launch_fill_zero_i64((int64_t*)Dp, (int64_t)S * batch, st)) != hipSuccess)
            return hip_fail(e);

        DotArgs da;
        da.X = dX;
        da.Y = dY;
        da.D = (int64_t*)Dp;
        da.batch = batch;
        da.nkc = nkc;
        da.S = S;
        da.band = band;
        da.nbands = S / band;
        // depth fragments per workgroup: within one exactness chunk, and short
        // enough that about 2048 workgroups share the depth
        {
            const int64_t kcc = std::max<int64_t>(kc / kcg, 1);
            const int64_t units = ((batch + 15) / 16) * da.nbands;
            const int64_t want = (nkc * units + 2047) / 2048;
            da.range = std::max<int64_t>(1, std::min<int64_t>(kcc, want));
        }
        if (o.ev_gemm_begin && (e = hipEventRecord((hipEvent_t)o.ev_gemm_begin, st)) != hipSuccess)
            return hip_fail(e);
        if ((e = launch_dot_diag(da, is_i8(o.form), st)) != hipSuccess)
            return hip_fail(e);
    }
    if ((e = launch_dot_final((const int64_t*)Dp, E, F, batch, S, beta, ncol, m, out,
                              std::max<int64_t>(plane_stride_out, 1), st)) != hipSuccess)
        return hip_fail(e);
    if (o.ev_gemm_end && (e = hipEventRecord((hipEvent_t)o.ev_gemm_end, st)) != hipSuccess)
        return hip_fail(e);

    if (o.info)
        fill_info(o.info, ch, T, o.validate != 0);
    return MD_OK;
}

int md_dot(int m, int64_t batch, int64_t n, const double* X, const double* Y, double* out, void* stream)
{
    return md_dot_ex(m, batch, n, X, n, batch * n, Y, n, batch * n, out, batch, nullptr, stream);
}

int md_gemm_ordinary(int m, int64_t M, int64_t N, int64_t K, const double* A, const double* B,
                     double* C, void* stream)
{
    g_last_hip = 0;
    if (m != 1 && m != 2 && m != 4 && m != 8)
        return MD_EINVAL_M;
    if (M < 0 || N < 0 || K < 0)
        return MD_EINVAL_DIM;
    if (M == 0 || N == 0)
        return MD_OK;
    if (!C || (K > 0 && (!A || !B)))
        return MD_ENULL;
    if (!mul_ok(M, N) || !mul_ok(M, std::max<int64_t>(K, 1)) || !mul_ok(K, N) ||
        M > (INT64_C(1) << 40) || N > (INT64_C(1) << 40) || K > (INT64_C(1) << 40) ||
        ((M + 15) / 16) * ((N + 15) / 16) > (INT64_C(1) << 24))   // grid of 256-thread tiles
        return MD_EINVAL_DIM;
    const Span sc = extent(C, m, M, N, N, 1, M * N);
    if (K > 0 && (overlap(sc, extent(A, m, M, K, K, 1, M * K)) || overlap(sc, extent(B, m, K, N, N, 1, K * N))))
        return MD_EALIAS;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = K == 0 ? launch_fill_zero(C, m, M, N, N, M * N, st) : launch_ordinary(m, A, B, C, M, N, K, st);
    return e == hipSuccess ? MD_OK : hip_fail(e);
}

int md_dot_ordinary(int m, int64_t batch, int64_t n, const double* X, const double* Y, double* out,
                    void* stream)
{
    g_last_hip = 0;
    if (m != 1 && m != 2 && m != 4 && m != 8 && m != 16)
        return MD_EINVAL_M;
    if (batch < 0 || n < 0 || batch > (INT64_C(1) << 40) || n > (INT64_C(1) << 40) || !mul_ok(batch, n))
        return MD_EINVAL_DIM;
    if (batch == 0)
        return MD_OK;
    if (!out || (n > 0 && (!X || !Y)))
        return MD_ENULL;
    const Span so = extent(out, m, 1, batch, 0, 1, batch);
    if (n > 0 && (overlap(so, extent(X, m, batch, n, n, 1, batch * n)) || overlap(so, extent(Y, m, batch, n, n, 1, batch * n))))
        return MD_EALIAS;
    hipStream_t st = (hipStream_t)stream;
    const hipError_t e = n == 0 ? launch_fill_zero(out, m, 1, batch, batch, batch, st)
                                : launch_ordinary_dot(m, X, Y, out, batch, batch, n, st);
    return e == hipSuccess ? MD_OK : hip_fail(e);
}

int md_gemm(int m, int64_t M, int64_t N, int64_t K, const double* A, const double* B, double* C,
            void* stream)
{
    return md_gemm_ex(m, 0, 0, M, N, K, A, K, M * K, B, N, K * N, C, N, M * N, nullptr, stream);
}

int md_fixed_limbs(int beta, int S, int64_t K)
{
    if (beta < 1 || beta > 24 || S < 1 || S > 512 || K < 0)
        return -1;
    // |X| < K 2^(beta (S+1) + 1): two's complement with one bit to spare
    return (beta * (S + 1) + ceil_log2(std::max<int64_t>(K, 1)) + 3 + 31) / 32;
}

int md_exponents(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B,
                 int64_t ldb, int32_t* E, int32_t* F, void* stream)
{
    g_last_hip = 0;
    if (M < 0 || N < 0 || K < 0 || M > (INT64_C(1) << 40) || N > (INT64_C(1) << 40) ||
        K > (INT64_C(1) << 40))
        return MD_EINVAL_DIM;
    const bool doE = E && M > 0, doF = F && N > 0;
    if (!doE && !doF)
        return MD_OK;
    if ((doE && K > 0 && !A) || (doF && K > 0 && !B))
        return MD_ENULL;
    if ((doE && K > 0 && (lda < K || !mul_ok(M, lda))) || (doF && K > 0 && (ldb < N || !mul_ok(K, ldb))))
        return MD_EINVAL_DIM;
    hipStream_t st = (hipStream_t)stream;
    Scratch scr;
    scr.st = st;
    void* p;
    int rc = scr.get(small_bytes(M, N), &p);
    if (rc)
        return rc;
    int32_t* q = (int32_t*)p;
    int32_t* stats = q;
    q += 64;
    hipError_t e;
    if (doE) {
        int32_t *hi = q, *lo = q + round_up(M + 64, 64);
        const Operand op{A, 1, lda, 1, M, K};
        if ((e = launch_exp_init(hi, lo, M, stats, st)) != hipSuccess) return hip_fail(e);
        if (K > 0 && (e = launch_exp_partial(op, hi, lo, st)) != hipSuccess) return hip_fail(e);
        if ((e = launch_exp_final(hi, lo, M, E, stats, nullptr, nullptr, 0, st)) != hipSuccess) return hip_fail(e);
        q = lo + round_up(M + 64, 64);
    }
    if (doF) {
        int32_t *hi = q, *lo = q + round_up(N + 64, 64);
        const Operand op{B, 1, 1, ldb, N, K};
        if ((e = launch_exp_init(hi, lo, N, stats, st)) != hipSuccess) return hip_fail(e);
        if (K > 0 && (e = launch_exp_partial(op, hi, lo, st)) != hipSuccess) return hip_fail(e);
        if ((e = launch_exp_final(hi, lo, N, F, stats + 1, nullptr, nullptr, 0, st)) != hipSuccess) return hip_fail(e);
    }
    return MD_OK;
}

int md_gemm_fixed(int m, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                  int64_t plane_stride_A, const double* B, int64_t ldb, int64_t plane_stride_B,
                  const int32_t* E, const int32_t* F, int32_t* X, int nlimb, int32_t* scale,
                  const md_opts* opts, void* stream)
{
    g_last_hip = 0;
    if (m != 1 && m != 2 && m != 4 && m != 8 && m != 16)
        return MD_EINVAL_M;
    if (!opts || opts->force_S <= 0 || opts->dbg)
        return MD_EINVAL_OPT;
    if (M < 0 || N < 0 || K < 1)
        return MD_EINVAL_DIM;
    if (M == 0 || N == 0)
        return MD_OK;
    if (!A || !B || !X || !scale)
        return MD_ENULL;
    const int S = opts->force_S, beta = opts->force_beta;
    const int need = md_fixed_limbs(beta, S, K);
    if (need < 0)
        return MD_EINVAL_OPT;
    if (nlimb < need || nlimb > 80)
        return MD_ERANGE;
    if (!mul_ok(M, N) || !mul_ok(M * N, (int64_t)S * 8) || !mul_ok(M * N, (int64_t)nlimb * 4) ||
        !mul_ok(M * N, (int64_t)m * 8) || M * N > (INT64_C(1) << 40))
        return MD_EINVAL_DIM;
    const uintptr_t x0 = (uintptr_t)X, x1 = x0 + (uintptr_t)(M * N * nlimb) * 4;
    const uintptr_t s0 = (uintptr_t)scale, s1 = s0 + (uintptr_t)(M * N) * 4;
    if (x0 < s1 && s0 < x1)
        return MD_EALIAS;

    hipStream_t st = (hipStream_t)stream;
    Scratch scr;
    scr.st = st;
    int32_t* flags = opts->exp_flags;   // bit 8: an exponent override not taken
    const bool wait = (E || F) && !flags;
    hipError_t e;
    if (wait) {
        void* p;
        const int rc = scr.get(sizeof(int64_t), &p);
        if (rc)
            return rc;
        flags = (int32_t*)p;
        if ((e = launch_fill_zero_i64((int64_t*)flags, 1, st)) != hipSuccess)
            return hip_fail(e);
    }
    md_opts o = *opts;
    const FixedOut fo{X, scale, nlimb};
    const int rc = gemm_impl(m, 0, 0, M, N, K, A, lda, plane_stride_A, B, ldb, plane_stride_B, nullptr, 0, 0,
                             &o, stream, E, F, flags, &fo);
    if (rc)
        return rc;
    if (wait) {
        int32_t fl = 0;
        if ((e = hipMemcpyAsync(&fl, flags, sizeof(fl), hipMemcpyDeviceToHost, st)) != hipSuccess)
            return hip_fail(e);
        if ((e = hipStreamSynchronize(st)) != hipSuccess)
            return hip_fail(e);
        if (fl) {
            if (opts->info)
                opts->info->input_flags = fl;
            return MD_EINPUT;
        }
    }
    return MD_OK;
}

int md_fixed_add(int64_t count, int nlimb, const int32_t* X, const int32_t* Y, int32_t* Z, void* stream)
{
    g_last_hip = 0;
    if (count < 0 || nlimb < 1 || nlimb > 80 || count > (INT64_C(1) << 40))
        return count < 0 || count > (INT64_C(1) << 40) ? MD_EINVAL_DIM : MD_ERANGE;
    if (count == 0)
        return MD_OK;
    if (!X || !Y || !Z)
        return MD_ENULL;
    const hipError_t e = launch_fixed_add(count, nlimb, X, Y, Z, (hipStream_t)stream);
    return e == hipSuccess ? MD_OK : hip_fail(e);
}

int md_fixed_round(int m, int64_t count, int nlimb, const int32_t* X, const int32_t* scale, double* C,
                   int64_t plane_stride_C, void* stream)
{
    g_last_hip = 0;
    if (m != 1 && m != 2 && m != 4 && m != 8 && m != 16)
        return MD_EINVAL_M;
    if (count < 0 || count > (INT64_C(1) << 40))
        return MD_EINVAL_DIM;
    if (nlimb < 1 || nlimb > 80)
        return MD_ERANGE;
    if (count == 0)
        return MD_OK;
    if (!X || !scale || !C)
        return MD_ENULL;
    if (plane_stride_C < count || !mul_ok(plane_stride_C, (int64_t)m * 8))
        return MD_EINVAL_DIM;
    const Span sc = extent(C, m, 1, count, count, 1, plane_stride_C);
    const uintptr_t x0 = (uintptr_t)X, x1 = x0 + (uintptr_t)(count * nlimb) * 4;
    const uintptr_t s0 = (uintptr_t)scale, s1 = s0 + (uintptr_t)count * 4;
    if (overlap(sc, Span{x0, x1}) || overlap(sc, Span{s0, s1}))
        return MD_EALIAS;
    const hipError_t e = launch_fixed_round(m, count, nlimb, X, scale, C, plane_stride_C, (hipStream_t)stream);
    return e == hipSuccess ? MD_OK : hip_fail(e);
}

}  // extern "C"
