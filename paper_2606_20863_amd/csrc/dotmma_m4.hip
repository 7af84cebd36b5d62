// Matrix-core INT8 inner-product kernels for m = 4 words, containers of 16 .. 48 digits.
#include "dotmma.h"

namespace mdg {

hipError_t launch_dot_mma_m4(const LaneDotArgs& a, int SC, bool balanced, int64_t nch, hipStream_t st)
{
    return DispatchMma<4, 48, 16>::run(a, SC, balanced, nch, st);
}

}  // namespace mdg
