// Whole-triangle INT8 slice contraction kernels returning exact fixed-point
// integers, S = 1..22, 7-bit sign-magnitude digits.
#include "tri.h"

namespace mdg {

hipError_t launch_trifix_s1_22(const GemmArgs& a, hipStream_t st)
{
    return DispatchTriFixRange<22, 1, 7>::run(a, st);
}

}  // namespace mdg
