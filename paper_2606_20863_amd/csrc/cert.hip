// Certificate of a call that runs on a caller's slice-count hint: the
// slice-count rule of the host, evaluated on the device from the call's
// statistics (exponent spans, smallest magnitude product, extreme shared
// exponents), so that the call queues its kernels without waiting for them.
#include "../../include/mdgemm.h"
#include "mdgemm_internal.h"
#include "rule.h"

#include <climits>

namespace mdg {
namespace {

// The call statistics as the certificate reads them (kStatWords layout).
struct CallStats {
    int span_a, span_b;
    uint64_t minP;
    int emax, emin, fmax, fmin;
};

constexpr int kCertThreads = 256;

// max / min over the lanes of a wave
__device__ __forceinline__ void wave_reduce(int (&v)[6], unsigned long long& mn)
{
    for (int o = 1; o < 64; o <<= 1) {
        v[0] = max(v[0], __shfl_xor(v[0], o));
        v[1] = max(v[1], __shfl_xor(v[1], o));
        v[2] = max(v[2], __shfl_xor(v[2], o));
        v[3] = min(v[3], __shfl_xor(v[3], o));
        v[4] = max(v[4], __shfl_xor(v[4], o));
        v[5] = min(v[5], __shfl_xor(v[5], o));
        const unsigned long long u = __shfl_xor(mn, o);
        mn = u < mn ? u : mn;
    }
}

// Span maxima, extreme shared exponents and the smallest magnitude product
// over the pairs of whole-pair inner products (what the exponent pass and
// the magnitude kernels would leave): every thread of the workgroup
// reduces its pairs, then the waves', all in shuffles; thread 0 gets them
// and also stores them in stats.
__device__ CallStats pair_stats(const int32_t* ph, const unsigned long long* pm, int64_t batch, int32_t* stats)
{
    constexpr int NW = kCertThreads / 64;
    __shared__ int32_t xs[NW][6];
    __shared__ unsigned long long xm[NW];
    int v[6] = {0, 0, INT_MIN, INT_MAX, INT_MIN, INT_MAX};   // spans, extremes of x, of y
    unsigned long long mn = ~0ull;
    // unrolled: a thread's loads of several pairs in flight together
#pragma unroll 4
    for (int64_t b = threadIdx.x; b < batch; b += kCertThreads) {
        const int hx = ph[b], lx = ph[batch + b], hy = ph[2 * batch + b], ly = ph[3 * batch + b];
        if (hx != INT_MIN) {
            v[0] = max(v[0], hx - lx);
            v[2] = max(v[2], hx);
            v[3] = min(v[3], hx);
        }
        if (hy != INT_MIN) {
            v[1] = max(v[1], hy - ly);
            v[4] = max(v[4], hy);
            v[5] = min(v[5], hy);
        }
        if (pm && pm[b] < mn)
            mn = pm[b];
    }
    wave_reduce(v, mn);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        for (int i = 0; i < 6; ++i)
            xs[w][i] = v[i];
        xm[w] = mn;
    }
    __syncthreads();
    CallStats c{};
    if (w == 0) {
        const bool in = lane < NW;
        for (int i = 0; i < 6; ++i)
            v[i] = in ? xs[lane][i] : ((i == 3 || i == 5) ? INT_MAX : (i >= 2 ? INT_MIN : 0));
        mn = in ? xm[lane] : ~0ull;
        wave_reduce(v, mn);
        c = CallStats{v[0], v[1], mn, v[2], v[3], v[4], v[5]};
        if (lane == 0) {
            stats[0] = v[0];
            stats[1] = v[1];
            __builtin_memcpy(stats + 2, &mn, sizeof(mn));   // UINT64_MAX: not computed
            stats[4] = v[2];
            stats[5] = v[3];
            stats[6] = v[4];
            stats[7] = v[5];
        }
    }
    return c;
}

__global__ __launch_bounds__(kCertThreads) void k_cert(int32_t* stats, int form, int64_t K, int T, int m,
                                                       int beta, int S, md_cert* cert, const int32_t* ph,
                                                       const unsigned long long* pm, int64_t batch)
{
    CallStats c;
    if (ph) {
        c = pair_stats(ph, pm, batch, stats);
    } else if (threadIdx.x == 0) {
        c.span_a = stats[0];
        c.span_b = stats[1];
        __builtin_memcpy(&c.minP, stats + 2, sizeof(c.minP));
        c.emax = stats[4];
        c.emin = stats[5];
        c.fmax = stats[6];
        c.fmin = stats[7];
    }
    if (threadIdx.x != 0 || !cert)
        return;
    const int G_span = c.span_a + c.span_b + 2;
    const int G_rho = rule_rho_exponent(c.minP, K);   // -1: not computed or not certifiable
    const int G = G_rho >= 0 && G_rho < G_span ? G_rho : G_span;
    const bool bal = form == MD_FORM_INT8_BAL;
    const int need = bal ? rule_slice_count_balanced(T, G) : rule_slice_count(form == MD_FORM_INT8 ? 7 : beta, T, G);
    int S_min, band;
    if (form == MD_FORM_FP64)
        rule_band_round(need, kGmaxF64, 0, S_min, band);
    else
        rule_band_round(need, kGmaxI8, kTriMaxI8, S_min, band);
    int flags = S < need ? MD_CERT_SMALL : 0;
    double bound = rule_log2_bound(bal, G, beta, S, m);
    if (!rule_in_range(c.emax, c.emin, c.fmax, c.fmin, K, G, T)) {
        flags |= MD_CERT_RANGE;
        bound = __builtin_inf();
    }
    cert->flags = flags;
    cert->S_min = S_min;
    cert->S = S;
    cert->G = G;
    cert->G_span = G_span;
    cert->G_rho = G_rho;
    cert->log2_bound = bound;
}

}  // namespace

hipError_t launch_cert(const int32_t* stats, int form, int64_t K, int T, int m, int beta, int S, void* cert,
                       hipStream_t st, const int32_t* ph, const unsigned long long* pm, int64_t batch)
{
    hipLaunchKernelGGL(k_cert, dim3(1), dim3(kCertThreads), 0, st, const_cast<int32_t*>(stats), form, K, T, m, beta, S,
                       (md_cert*)cert, ph, pm, batch);
    return hipGetLastError();
}

}  // namespace mdg
