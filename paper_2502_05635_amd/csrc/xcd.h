// Workgroup placement on the 8 XCDs of the chip, each with its own L2.
#pragma once

#include <hip/hip_runtime.h>

namespace tdg {

constexpr int XCDS = 8;

// Workgroups are handed to the XCDs in turn (workgroup i, counted x fastest
// over the grid, to XCD i % 8).  This maps i to a logical index so that each
// XCD takes one contiguous range of logical indices, in order: blocks whose
// logical indices are close then share an L2.  A bijection on [0, count).
__device__ inline int xcd_block(int i, int count) {
  const int q = count / XCDS, r = count % XCDS, x = i % XCDS, l = i / XCDS;
  return x < r ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// The (x, y, z) block of a 3-D grid that the running workgroup takes, so that
// blocks adjacent in x (then y, then z) run on one XCD.
__device__ inline void xcd_block3(int& bx, int& by, int& bz) {
  const int gx = gridDim.x, gy = gridDim.y;
  const int i = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int l = xcd_block(i, gx * gy * gridDim.z);
  bx = l % gx;
  by = (l / gx) % gy;
  bz = l / (gx * gy);
}

}  // namespace tdg
