// Whole-triangle INT8 slice contraction kernels for S = 29..32, 7-bit
// sign-magnitude digits.
#include "tri.h"

namespace mdg {

hipError_t launch_tri_s29_32(const GemmArgs& a, hipStream_t st)
{
    return DispatchTriRange<32, 29, 7>::run(a, st);
}

}  // namespace mdg
