// Whole-triangle INT8 contraction with the A fragments shared through LDS
// (direct-to-LDS loads), for the slice counts it is built for.
#include "trid.h"

namespace mdg {

bool trid_shape(int S, int beta)
{
    return beta == 8 && S == 27;
}

hipError_t launch_trid(const GemmArgs& a, hipStream_t st)
{
    if (a.beta == 8 && a.S == 27)
        return launch_kernel(k_tri2d_i8<27, 8, 9>, a, st, false, 2 * kTile);
    return hipErrorInvalidValue;
}

}  // namespace mdg
