// Two-band INT8 slice contraction kernels for S = 52, 56, .., 64, 7-bit sign-magnitude digits.
#include "duo.h"

namespace mdg {

hipError_t launch_duo_s52_64(const GemmArgs& a, hipStream_t st)
{
    return DispatchDuoRange<64, 52, 7>::run(a, st);
}

}  // namespace mdg
