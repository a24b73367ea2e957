// End eigenvalues of the small symmetric tridiagonal matrices that the
// Lanczos estimates of the mixed and the spectral norm build (sec. 2).
// Internal to the library; every thread of a 256-thread workgroup calls
// these together.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace sp2 {

constexpr int kTridiagThreads = 256;

// Number of eigenvalues of the symmetric tridiagonal matrix (diagonal a,
// off-diagonal b, order m) below x: Sturm count of the LDL^T pivots.
__device__ __forceinline__ int sturm_below(const double* a, const double* b,
                                           int m, double x) {
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < m; ++i) {
    const double bb = (i > 0) ? b[i - 1] * b[i - 1] : 0.0;
    d = (a[i] - x) - ((i > 0) ? bb / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++cnt;
  }
  return cnt;
}

// Eigenvalue number `rank` (1 = smallest, m = largest) of the tridiagonal
// (a, b) of order m by multisection: every thread counts at one point of the
// current bracket, and the bracket shrinks to the two points around the
// eigenvalue; five rounds of 256 points narrow a Gershgorin bracket by 256^5.
// `hits` is an LDS array of 256 ints.
__device__ inline double tridiag_eig(const double* a, const double* b, int m,
                                     int rank, int* hits) {
  double lo = a[0], hi = a[0];
  for (int i = 0; i < m; ++i) {
    const double r = ((i > 0) ? fabs(b[i - 1]) : 0.0) +
                     ((i + 1 < m) ? fabs(b[i]) : 0.0);
    lo = fmin(lo, a[i] - r);
    hi = fmax(hi, a[i] + r);
  }
  for (int round = 0; round < 5; ++round) {
    const double h = (hi - lo) / kTridiagThreads;
    const double x = lo + h * (threadIdx.x + 1);
    // hits[t] = 1 when at least `rank` eigenvalues lie below the point x_t
    __syncthreads();
    hits[threadIdx.x] = (sturm_below(a, b, m, x) >= rank) ? 1 : 0;
    __syncthreads();
    int first = kTridiagThreads - 1;   // smallest such t
    for (int t = 0; t < kTridiagThreads; ++t)
      if (hits[t]) {
        first = t;
        break;
      }
    hi = lo + h * (first + 1);
    lo = lo + h * first;
  }
  return 0.5 * (lo + hi);
}

}  // namespace sp2
