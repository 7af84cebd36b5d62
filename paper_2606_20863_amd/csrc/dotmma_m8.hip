// Matrix-core INT8 inner-product kernels for m = 8 words, containers of 32 .. 64 digits.
#include "dotmma.h"

namespace mdg {

hipError_t launch_dot_mma_m8(const LaneDotArgs& a, int SC, bool balanced, int64_t nch, hipStream_t st)
{
    return DispatchMma<8, 64, 32>::run(a, SC, balanced, nch, st);
}

}  // namespace mdg
