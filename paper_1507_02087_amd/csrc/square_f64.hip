// Square kernels of the F64 family: every configuration of the
// family in every mode, and the persistent batch kernel where compiled.
#include "square_impl.h"

namespace sp2 {

hipError_t launch_square_f64(int id, const SquareArgs& a, int grid, hipStream_t s) {
  switch (id) {
    case 0: return launch_cfg<F64_128_2x4>(a, grid, s);
    case 1: return launch_cfg<F64_128_2x2>(a, grid, s);
    case 2: return launch_cfg<F64_64_2x2>(a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

int persist_grid_f64(int id, bool stretch, int num_cus) {
  switch (id) {
    case 0: return persist_grid_cfg<F64_128_2x4>(stretch, num_cus);
    case 2: return persist_grid_cfg<F64_64_2x2>(stretch, num_cus);
    default: return 0;
  }
}

hipError_t launch_persist_f64(int id, const SquareArgs& a, const PQueue& q, int grid,
                              hipStream_t s) {
  switch (id) {
    case 0: return launch_persist_cfg<F64_128_2x4>(a, q, grid, s);
    case 2: return launch_persist_cfg<F64_64_2x2>(a, q, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sp2
