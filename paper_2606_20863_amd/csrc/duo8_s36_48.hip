// Two-band INT8 slice contraction kernels for S = 36, 40, .., 48, balanced 8-bit digits.
#include "duo.h"

namespace mdg {

hipError_t launch_duo8_s36_48(const GemmArgs& a, hipStream_t st)
{
    return DispatchDuoRange<48, 36, 8>::run(a, st);
}

}  // namespace mdg
