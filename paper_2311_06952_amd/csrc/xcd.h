// xcd.h -- block order by XCD.  MI355X hands the blocks of a launch to its 8
// XCDs round-robin in launch order (block b runs on XCD b % 8), and each XCD
// has its own L2.  A kernel that launches a multiple of 8 blocks and works as
// block xcd_order(b, g) of its work list gives each XCD one contiguous range
// of that list, so that work items that read the same data (the chunks of one
// feature) share an L2.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mh {

__device__ __forceinline__ uint32_t xcd_order(uint32_t b, uint32_t g) {
  return (b & 7u) * (g >> 3) + (b >> 3);
}
// The grid for `blocks` work items: a multiple of 8 (the blocks past the list
// return at once).
inline uint32_t xcd_grid(uint32_t blocks) { return (blocks + 7u) & ~7u; }

}  // namespace mh
