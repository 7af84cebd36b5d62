// Lane-wise INT8 inner-product kernels for m = 8 words, containers of 24 .. 64 digits.
#include "dotlane.h"

namespace mdg {

hipError_t launch_dot_lane_m8(const LaneDotArgs& a, int SC, bool balanced, int nw, int64_t nch, hipStream_t st)
{
    return DispatchLane<8, 64, 24>::run(a, SC, balanced, nw, nch, st);
}

}  // namespace mdg
