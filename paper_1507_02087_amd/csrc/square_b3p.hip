// Square kernels of the B3P family: every configuration of the
// family in every mode, and the persistent batch kernel where compiled.
#include "square_impl.h"

namespace sp2 {

hipError_t launch_square_b3p(int id, const SquareArgs& a, int grid, hipStream_t s) {
  switch (id) {
    case 12: return launch_cfg<B3P_256_2x4>(a, grid, s);
    case 13: return launch_cfg<B3P_256_2x4_32>(a, grid, s);
    case 14: return launch_cfg<B3P_128_2x2>(a, grid, s);
    case 16: return launch_cfg<B3P_256_4x4_32>(a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

int persist_grid_b3p(int id, bool stretch, int num_cus) {
  switch (id) {
    case 14: return persist_grid_cfg<B3P_128_2x2>(stretch, num_cus);
    default: return 0;
  }
}

hipError_t launch_persist_b3p(int id, const SquareArgs& a, const PQueue& q, int grid,
                              hipStream_t s) {
  switch (id) {
    case 14: return launch_persist_cfg<B3P_128_2x2>(a, q, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sp2
