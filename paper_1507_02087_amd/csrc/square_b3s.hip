// Square kernels of the B3S family: every configuration of the
// family in every mode, and the persistent batch kernel where compiled.
#include "square_impl.h"

namespace sp2 {

hipError_t launch_square_b3s(int id, const SquareArgs& a, int grid, hipStream_t s) {
  switch (id) {
    case 9: return launch_cfg<B3S_256_2x4>(a, grid, s);
    case 10: return launch_cfg<B3S_256_2x4_16>(a, grid, s);
    case 11: return launch_cfg<B3S_128_2x2>(a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

int persist_grid_b3s(int id, bool stretch, int num_cus) {
  switch (id) {
    case 11: return persist_grid_cfg<B3S_128_2x2>(stretch, num_cus);
    default: return 0;
  }
}

hipError_t launch_persist_b3s(int id, const SquareArgs& a, const PQueue& q, int grid,
                              hipStream_t s) {
  switch (id) {
    case 11: return launch_persist_cfg<B3S_128_2x2>(a, q, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sp2
