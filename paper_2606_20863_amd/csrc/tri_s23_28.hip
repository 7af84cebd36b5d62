// Whole-triangle INT8 slice contraction kernels for S = 23..28, 7-bit
// sign-magnitude digits.
#include "tri.h"

namespace mdg {

hipError_t launch_tri_s23_28(const GemmArgs& a, hipStream_t st)
{
    return DispatchTriRange<28, 23, 7>::run(a, st);
}

}  // namespace mdg
