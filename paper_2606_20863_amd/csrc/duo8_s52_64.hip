// Two-band INT8 slice contraction kernels for S = 52, 56, .., 64, balanced 8-bit digits.
#include "duo.h"

namespace mdg {

hipError_t launch_duo8_s52_64(const GemmArgs& a, hipStream_t st)
{
    return DispatchDuoRange<64, 52, 8>::run(a, st);
}

}  // namespace mdg
