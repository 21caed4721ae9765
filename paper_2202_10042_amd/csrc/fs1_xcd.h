// fs1_xcd.h -- workgroup placement over the accelerator complex dies.
//
// The device dispatches the workgroups of a launch to its 8 XCDs round-robin
// (workgroup b to XCD b mod 8), and each XCD has its own L2.  Work items that
// share cache lines (adjacent lines of a strided grid axis, consecutive chunks
// of one batched instance) hit one L2 only if they run on one XCD, so the
// launches below take their work item from xcd_contiguous(b, nb): a bijection
// of [0, nb) that gives every XCD a contiguous range of items, taken in order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fs1 {

constexpr uint32_t kXcds = 8;

__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t nb) {
  const uint32_t per = nb / kXcds, rem = nb % kXcds, x = b % kXcds;
  return x * per + min(x, rem) + b / kXcds;
}

}  // namespace fs1
