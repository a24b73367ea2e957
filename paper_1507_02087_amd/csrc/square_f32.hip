// Square kernels of the F32 family: every configuration of the
// family in every mode, and the persistent batch kernel where compiled.
#include "square_impl.h"

namespace sp2 {

hipError_t launch_square_f32(int id, const SquareArgs& a, int grid, hipStream_t s) {
  switch (id) {
    case 3: return launch_cfg<F32_128_2x2>(a, grid, s);
    case 4: return launch_cfg<F32_128_2x4>(a, grid, s);
    case 5: return launch_cfg<F32_256_2x2>(a, grid, s);
    case 15: return launch_cfg<F32_256_2x4>(a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

int persist_grid_f32(int id, bool stretch, int num_cus) {
  switch (id) {
    case 3: return persist_grid_cfg<F32_128_2x2>(stretch, num_cus);
    case 4: return persist_grid_cfg<F32_128_2x4>(stretch, num_cus);
    default: return 0;
  }
}

hipError_t launch_persist_f32(int id, const SquareArgs& a, const PQueue& q, int grid,
                              hipStream_t s) {
  switch (id) {
    case 3: return launch_persist_cfg<F32_128_2x2>(a, q, grid, s);
    case 4: return launch_persist_cfg<F32_128_2x4>(a, q, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sp2
