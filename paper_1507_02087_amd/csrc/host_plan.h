// Host-side planning of the square launches (internal): the padded row
// stride of an iterate, the order of the upper tiles of a tile grid, and the
// division of a launch group's tiles into workgroups (with K-split tail
// tiles). Pure host code with no GPU calls, built on its own with the
// sanitizers in the host checks of the test suite.
#pragma once

#include <stdint.h>

#include <vector>

#include "sp2_device.h"

namespace sp2 {

int64_t row_stride(int64_t np);

void append_tile_list(int nt, std::vector<int2>& out);

// Work plan of one launch group.
struct Plan {
  std::vector<WorkItem> items;   // one per workgroup
  std::vector<TailItem> tails;
  int split = 1;
};

Plan make_plan(const std::vector<int>& slots, const std::vector<int>& owner,
               const std::vector<int>& nk, int concurrency, int tail_split);

}  // namespace sp2
