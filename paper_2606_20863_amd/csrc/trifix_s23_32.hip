// Whole-triangle INT8 slice contraction kernels returning exact fixed-point
// integers, S = 23..32, 7-bit sign-magnitude digits.
#include "tri.h"

namespace mdg {

hipError_t launch_trifix_s23_32(const GemmArgs& a, hipStream_t st)
{
    return DispatchTriFixRange<32, 23, 7>::run(a, st);
}

}  // namespace mdg
