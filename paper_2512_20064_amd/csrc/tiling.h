// Tile scheduling shared by the contraction kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace mps {

// Workgroup b -> output tile (tm, tn over the concatenated column tiles of all
// problems of the launch).  Workgroups are dealt round-robin to the 8 XCDs of
// an MI355X, so each XCD first gets a contiguous run of tile indices.  Inside
// that run tiles go in groups of group_m row blocks, column-major within a
// group: the workgroups resident on one XCD at a time then cover a few row
// blocks by several column tiles, and both operands are reused from that
// XCD's L2 instead of re-streaming the whole site tensor for every row block.
__device__ inline bool map_tile(int b, int tiles_m, int tn_total, int per_xcd, int group_m, int& tm, int& tn) {
  const int t = (b & 7) * per_xcd + (b >> 3);
  if (t >= tiles_m * tn_total) return false;
  if (group_m <= 1) {
    tm = t / tn_total;
    tn = t - tm * tn_total;
    return true;
  }
  const int g = t / (group_m * tn_total);
  const int r = t - g * group_m * tn_total;
  const int rows_in = min(group_m, tiles_m - g * group_m);
  tn = r / rows_in;
  tm = g * group_m + (r - tn * rows_in);
  return true;
}

// Problem p with tn_start[p] <= tn < tn_start[p + 1] (tn_start[0] = 0).
__device__ inline int find_problem(const int* tn_start, int nprob, int tn) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tn_start[mid] <= tn) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace mps
