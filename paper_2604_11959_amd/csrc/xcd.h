// Work-list launches spread over the XCDs of the chip.
//
// The dispatcher hands workgroup b (linear id) to XCD b % 8, and each XCD
// has its own L2.  The passes over the general range and the redistribution
// walk lists in column order and gather from their neighbours in the list
// (lateral neighbours a few hundred entries away).  With the plain mapping,
// consecutive blocks land on different XCDs and every XCD pulls most of the
// gathered arrays through its L2.  Here the x extent of the grid is rounded
// up to a multiple of 8 and block x works on block (x % 8) * (extent / 8) +
// x / 8 of the list: each XCD walks its own contiguous eighth, whose
// gathers stay within it (plus a thin margin) and hit that XCD's L2.  For a
// grid with a y extent the linear id is x + y * extent, so x % 8 still names
// the XCD.  The blocks past the end of the list exit through the callers'
// bounds checks.
#pragma once

#include <hip/hip_runtime.h>

namespace ebs {

constexpr int kXcds = 8;

// grid x extent for nblk blocks of work: a multiple of the XCD count
inline unsigned xcd_grid(long long nblk) {
    return (unsigned)((nblk + kXcds - 1) / kXcds * kXcds);
}

// the block of the work list this block takes (grid x extent from xcd_grid)
__device__ inline int xcd_block() {
    const int per = (int)gridDim.x / kXcds;
    return ((int)blockIdx.x % kXcds) * per + (int)blockIdx.x / kXcds;
}

}  // namespace ebs
