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
// `hits` is an LDS array of (at least) 4 ints.
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
    // smallest t whose point x_t has at least `rank` eigenvalues below it
    // (the last point if none): the lowest set lane of each wave's ballot,
    // then the minimum over the waves
    const bool hit = sturm_below(a, b, m, x) >= rank;
    const unsigned long long mask = __ballot(hit);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();   // hits may still be read from the previous round
    if (lane == 0)
      hits[wave] = mask ? wave * 64 + __ffsll(static_cast<long long>(mask)) - 1
                        : kTridiagThreads - 1;
    __syncthreads();
    int first = hits[0];
    for (int w = 1; w < kTridiagThreads / 64; ++w) first = min(first, hits[w]);
    hi = lo + h * (first + 1);
    lo = lo + h * first;
  }
  return 0.5 * (lo + hi);
}

// Both end eigenvalues of the tridiagonal (a, b) of order m at once: the
// first two waves bisect for the smallest, the last two for the largest,
// 128 points each per round; six rounds narrow each Gershgorin bracket by
// 128^6. `hits` is an LDS array of 4 ints.
__device__ inline void tridiag_ends(const double* a, const double* b, int m,
                                    int* hits, double* bottom, double* top) {
  double lo = a[0], hi = a[0];
  for (int i = 0; i < m; ++i) {
    const double r = ((i > 0) ? fabs(b[i - 1]) : 0.0) +
                     ((i + 1 < m) ? fabs(b[i]) : 0.0);
    lo = fmin(lo, a[i] - r);
    hi = fmax(hi, a[i] + r);
  }
  constexpr int kHalf = kTridiagThreads / 2;
  const int half = threadIdx.x / kHalf, t = threadIdx.x % kHalf;
  const int rank = half ? m : 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int round = 0; round < 6; ++round) {
    const double h = (hi - lo) / kHalf;
    const double x = lo + h * (t + 1);
    const bool hit = sturm_below(a, b, m, x) >= rank;
    const unsigned long long mask = __ballot(hit);
    __syncthreads();   // hits may still be read from the previous round
    if (lane == 0)
      hits[wave] = mask ? (wave & 1) * 64 + __ffsll(static_cast<long long>(mask)) - 1
                        : kHalf - 1;
    __syncthreads();
    const int first = min(hits[2 * half], hits[2 * half + 1]);
    hi = lo + h * (first + 1);
    lo = lo + h * first;
  }
  const double mid = 0.5 * (lo + hi);
  // hand each half's result to every thread through two LDS doubles
  __shared__ double ends[2];
  if (t == 0) ends[half] = mid;
  __syncthreads();
  *bottom = ends[0];
  *top = ends[1];
  __syncthreads();
}

}  // namespace sp2
