// Whole-triangle INT8 slice contraction kernels for S = 23..28, balanced
// 8-bit digits.
#include "tri.h"

namespace mdg {

hipError_t launch_tri8_s23_28(const GemmArgs& a, hipStream_t st)
{
    return DispatchTriRange<28, 23, 8>::run(a, st);
}

}  // namespace mdg
