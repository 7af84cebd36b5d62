// Whole-triangle INT8 slice contraction kernels returning exact fixed-point
// integers, S = 1..22, balanced 8-bit digits.
#include "tri.h"

namespace mdg {

hipError_t launch_trifix8_s1_22(const GemmArgs& a, hipStream_t st)
{
    return DispatchTriFixRange<22, 1, 8>::run(a, st);
}

}  // namespace mdg
