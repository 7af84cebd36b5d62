// Whole-triangle INT8 slice contraction kernels for S = 29..32, balanced
// 8-bit digits.
#include "tri.h"

namespace mdg {

hipError_t launch_tri8_s29_32(const GemmArgs& a, hipStream_t st)
{
    return DispatchTriRange<32, 29, 8>::run(a, st);
}

}  // namespace mdg
