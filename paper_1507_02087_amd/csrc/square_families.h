// Per-family entry points of the square kernels (internal): each kernel
// family's configurations are instantiated in a translation unit of their
// own (square_<family>.hip); square_dense.hip dispatches by configuration.
#pragma once

#include "sp2_device.h"

namespace sp2 {

hipError_t launch_square_f64(int id, const SquareArgs& a, int grid, hipStream_t s);
int persist_grid_f64(int id, bool stretch, int num_cus);
hipError_t launch_persist_f64(int id, const SquareArgs& a, const PQueue& q, int grid,
                            hipStream_t s);
hipError_t launch_square_f32(int id, const SquareArgs& a, int grid, hipStream_t s);
int persist_grid_f32(int id, bool stretch, int num_cus);
hipError_t launch_persist_f32(int id, const SquareArgs& a, const PQueue& q, int grid,
                            hipStream_t s);
hipError_t launch_square_b3(int id, const SquareArgs& a, int grid, hipStream_t s);
int persist_grid_b3(int id, bool stretch, int num_cus);
hipError_t launch_persist_b3(int id, const SquareArgs& a, const PQueue& q, int grid,
                            hipStream_t s);
hipError_t launch_square_b3s(int id, const SquareArgs& a, int grid, hipStream_t s);
int persist_grid_b3s(int id, bool stretch, int num_cus);
hipError_t launch_persist_b3s(int id, const SquareArgs& a, const PQueue& q, int grid,
                            hipStream_t s);
hipError_t launch_square_b3p(int id, const SquareArgs& a, int grid, hipStream_t s);
int persist_grid_b3p(int id, bool stretch, int num_cus);
hipError_t launch_persist_b3p(int id, const SquareArgs& a, const PQueue& q, int grid,
                            hipStream_t s);

}  // namespace sp2
