// Work-group numbering for launches whose neighbouring blocks should share
// an L2: work-groups are dispatched to the 8 XCDs round-robin in launch order
// (x fastest), each XCD with its own L2.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wh {

// Grid for nblk logical blocks: a multiple of 8 work-groups (whole rounds over
// the XCDs), one row of up to 2^24 of them (a launch dimension holds at most
// 2^32 work-items, and rows here are at most 64 work-items wide), rows of
// 2^16 beyond that.
inline dim3 xcd_grid(int64_t nblk) {
  const int64_t padded = (nblk + 7) / 8 * 8;
  if (padded <= (int64_t(1) << 24)) return dim3((unsigned)padded);
  return dim3(1u << 16, (unsigned)((padded + (1 << 16) - 1) >> 16));
}

// Logical block of the work-group with linear launch index L in a grid of
// `total` work-groups made by xcd_grid: XCD x (= L mod 8) takes the logical
// blocks x * total/8 .. (x + 1) * total/8 - 1, in launch order.  Values of
// nblk and above are padding.
__host__ __device__ inline int64_t xcd_block(int64_t L, int64_t total) { return (L % 8) * (total / 8) + L / 8; }

}  // namespace wh
