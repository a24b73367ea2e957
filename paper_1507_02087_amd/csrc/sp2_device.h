// Internal declarations shared by the HIP kernels and the host driver of the
// SP2 library. Not part of the public ABI (include/sp2.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sp2 {

// Largest number of squares a run may compute (public SP2_MAX_ITER_LIMIT).
constexpr int kMaxIter = 200;

// Per-run state kept in device memory. The finalize kernel is its only
// writer during a run; the square kernels read `done` and the polynomial of
// their step from it. Index conventions follow Alg. 2: p[i] is the
// polynomial that produced X~_i (p[0] unused), v[k] = ||X~_k - X~_k^2||_F,
// t1[k] = Tr X~_k, t2[k] = Tr X~_k^2, r[k] the observed order at step k.
struct DevState {
  int32_t done;      // 0 while running, 1 once the outcome is fixed
  int32_t status;    // sp2_status of the outcome
  int32_t n;         // index of the returned iterate X~_n
  int32_t squares;   // squares whose partial sums were finalised
  int8_t p[kMaxIter + 2];
  double v[kMaxIter + 1];
  double t1[kMaxIter + 2];
  double t2[kMaxIter + 2];
  double r[kMaxIter + 1];
};

// Mirror of the outcome fields in host-coherent pinned memory, written by
// the finalize kernel with system-scope stores so that the host can see the
// stop without copying device memory.
struct HostMirror {
  int32_t done;
  int32_t status;
  int32_t n;
  int32_t squares;
};

// Parameters of the scalar stop/branch logic (Alg. 2).
struct StopParams {
  double n_occ;      // number of occupied states
  double n;          // matrix dimension (divergence test Tr X^2 > Tr X + n)
  int32_t branch;    // 0 = trace-nearest, 1 = literal Tr X > n_occ
  int32_t max_iter;  // squares allowed
};

// Host-side launchers (implemented in the .hip files).
hipError_t launch_state_reset(DevState* st, hipStream_t s);
hipError_t launch_f0(const double* F, int64_t ldf, int n, int np, double lmax,
                     double width, double tau, void* X0, bool fp64_store,
                     double* part, int rows_per_block, hipStream_t s);
hipError_t launch_finalize(const double* part, int count, DevState* st,
                           HostMirror* mirror, int iter, StopParams prm,
                           hipStream_t s);
hipError_t launch_fill(void* X, bool fp64_store, int n, int np, int identity,
                       hipStream_t s);
hipError_t launch_copy_out(const void* X, bool fp64_store, int n, int ldx,
                           void* D, int64_t ldd, bool out_fp64,
                           hipStream_t s);

// One symmetric square step: reads X~_{iter-1} from X, writes X~_iter to Y
// (upper tiles and their mirrors), one FP64 partial triple per tile.
struct SquareArgs {
  const void* X;
  void* Y;
  int ld;              // padded dimension (multiple of the tile edge)
  const int2* tiles;   // upper-triangle tile coordinates, XCD-grouped order
  int ntiles;
  int per_xcd;         // ceil(ntiles / 8)
  const DevState* st;
  int iter;
  double* part;        // 3 doubles per tile: ||X - S||_F^2, Tr, ||X_new||_F^2
  double tau;
};

hipError_t launch_square_f64(const SquareArgs& a, int tile, hipStream_t s);
hipError_t launch_square_f32(const SquareArgs& a, int tile, hipStream_t s);
hipError_t launch_square_bf16x3(const SquareArgs& a, int tile, hipStream_t s);
bool square_tile_supported(int precision, int tile);

}  // namespace sp2
