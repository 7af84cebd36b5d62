// Certificate of a call that runs on a caller's slice-count hint: the
// slice-count rule of the host, evaluated on the device from the call's
// statistics (exponent spans, smallest magnitude product, extreme shared
// exponents), so that the call queues its kernels without waiting for them.
#include "../../include/mdgemm.h"
#include "mdgemm_internal.h"
#include "rule.h"

namespace mdg {
namespace {

__global__ void k_cert(const int32_t* stats, int form, int64_t K, int T, int m, int beta, int S,
                       md_cert* cert)
{
    if (threadIdx.x != 0)
        return;
    const int G_span = stats[0] + stats[1] + 2;
    uint64_t minP;
    __builtin_memcpy(&minP, stats + 2, sizeof(minP));
    const int G_rho = rule_rho_exponent(minP, K);   // -1: not computed or not certifiable
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
    if (!rule_in_range(stats[4], stats[5], stats[6], stats[7], K, G, T)) {
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
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_cert, dim3(1), dim3(64), 0, st, stats, form, K, T, m, beta, S, (md_cert*)cert);
    return hipGetLastError();
}

}  // namespace mdg
