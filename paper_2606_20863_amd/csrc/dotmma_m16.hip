// Matrix-core INT8 inner-product kernels for m = 16 words, containers of 80 .. 128 digits.
#include "dotmma.h"

namespace mdg {

hipError_t launch_dot_mma_m16(const LaneDotArgs& a, int SC, bool balanced, int64_t nch, hipStream_t st)
{
    return DispatchMma<16, 128, 80>::run(a, SC, balanced, nch, st);
}

}  // namespace mdg
