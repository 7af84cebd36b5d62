// Two-band INT8 slice contraction kernels for S = 36, 40, .., 48, 7-bit sign-magnitude digits.
#include "duo.h"

namespace mdg {

hipError_t launch_duo_s36_48(const GemmArgs& a, hipStream_t st)
{
    return DispatchDuoRange<48, 36, 7>::run(a, st);
}

}  // namespace mdg
