// Square kernels of the B3 family: every configuration of the
// family in every mode, and the persistent batch kernel where compiled.
#include "square_impl.h"

namespace sp2 {

hipError_t launch_square_b3(int id, const SquareArgs& a, int grid, hipStream_t s) {
  switch (id) {
    case 6: return launch_cfg<B3_128_2x2>(a, grid, s);
    case 7: return launch_cfg<B3_256_2x2>(a, grid, s);
    case 8: return launch_cfg<B3_256_2x4>(a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

int persist_grid_b3(int id, bool stretch, int num_cus) {
  switch (id) {
    case 6: return persist_grid_cfg<B3_128_2x2>(stretch, num_cus);
    default: return 0;
  }
}

hipError_t launch_persist_b3(int id, const SquareArgs& a, const PQueue& q, int grid,
                             hipStream_t s) {
  switch (id) {
    case 6: return launch_persist_cfg<B3_128_2x2>(a, q, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sp2
