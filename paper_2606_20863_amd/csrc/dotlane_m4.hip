// Lane-wise INT8 inner-product kernels for m = 4 words, containers of 8 .. 48 digits.
#include "dotlane.h"

namespace mdg {

hipError_t launch_dot_lane_m4(const LaneDotArgs& a, int SC, bool balanced, int nw, int64_t nch, hipStream_t st)
{
    return DispatchLane<4, 48, 8>::run(a, SC, balanced, nw, nch, st);
}

}  // namespace mdg
