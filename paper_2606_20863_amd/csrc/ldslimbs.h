// The limb store of the word-placement digit split on the device: a lane's
// column of its wave's limb array in LDS (limb i of lane l at [i][l]: the
// 64 lanes' 8-byte limbs side by side, so the reads, the clears and the adds
// of one limb index meet no bank twice; the adds land on limbs that differ
// from lane to lane).  Only the lane itself touches its column, so no
// barrier is needed; LDS operations of a wave complete in order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mdg {
namespace {

struct LdsLimbs {
    uint64_t* col;
    __device__ __forceinline__ void add(int i, uint64_t v)
    {
        atomicAdd(reinterpret_cast<unsigned long long*>(col + i * 64), (unsigned long long)v);
    }
    __device__ __forceinline__ uint64_t take(int i)
    {
        const uint64_t v = col[i * 64];
        col[i * 64] = 0;
        return v;
    }
};

}  // namespace
}  // namespace mdg
