// Spectral norm of E = X~ - X~^2, the error e_i of Alg. 2 (sec. 2), for
// every running instance of a batch, by Lanczos with full
// reorthogonalisation in FP64.
//
// E is applied through two products with the stored iterate,
// E q = X~ q - X~ (X~ q), so E itself is never formed and the estimate is the
// norm of the idempotency error of the iterate as stored, evaluated in FP64
// whatever the working precision of the squares. E is symmetric but not
// semidefinite (eigenvalues of X~ outside [0, 1] give negative
// eigenvalues of E), so the estimate is the larger magnitude of the two end
// Ritz values.
//
// One cooperative launch per step runs the Lanczos processes of all
// instances in lockstep: the rows of every instance are cut into chunks of
// kSpecRows rows, each workgroup owns a fixed set of chunks, and grid-wide
// barriers separate the phases of one Lanczos step:
//   P1  beta_{j-1} = ||w||, q_j = w / beta_{j-1}, y = X~ q_j; the workgroup
//       owning an instance's first chunk also updates that instance's
//       estimate from the tridiagonal T_j and decides whether it is final
//   P2  w = y - X~ y (= E q_j), first Gram-Schmidt pass: dots q_l . w
//   P3  w -= sum_l c_l q_l, second pass: dots
//   P4  w -= sum_l c'_l q_l, ||w||^2 per chunk
// An instance is final when its estimate changes by less than 1e-12
// relative, when w vanishes (an invariant subspace), or after kLanczosMax
// steps (or n). Every sum over chunks is taken in one fixed order, so every
// workgroup derives the same scalars and the result does not depend on the
// grid.
#include <hip/hip_cooperative_groups.h>
#include <math.h>

#include "sp2_device.h"
#include "tridiag.h"

namespace sp2 {

namespace {

namespace cg = cooperative_groups;

constexpr int kThreads = kTridiagThreads;
constexpr int kWaves = kThreads / 64;
constexpr int kRowsPerWave = kSpecRows / kWaves;
constexpr double kSpecTol = 1e-12;
static_assert(kSpecRows == 32, "one row per lane of a half wave");
static_assert(kLanczosMax == 64, "one coefficient per lane of a wave");

__device__ __forceinline__ double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Sum over each 32-lane half of the wave (every lane receives its half's).
__device__ __forceinline__ double half_sum(double x) {
  for (int off = 16; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Sum over the workgroup, returned to every thread (fixed order).
__device__ __forceinline__ double block_sum(double x, double* red) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = x;
  __syncthreads();
  double t = red[0];
  for (int w = 1; w < kWaves; ++w) t += red[w];
  return t;
}

// Entry `row` of the start vector: SplitMix64's output for the row index,
// mapped to [-1, 1). A fixed pseudo-random vector has a component along
// every eigenvector of E except by accident.
__device__ __forceinline__ double start_entry(int row) {
  uint64_t z = static_cast<uint64_t>(row) * 0x9E3779B97F4A7C15ull +
               0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return static_cast<double>(z >> 11) * 0x1.0p-52 - 1.0;
}

// Phase separator: every workgroup's global stores are made visible to the
// whole device (agent-scope release), the grid meets, and each workgroup
// drops its stale cached copies (agent-scope acquire).
__device__ __forceinline__ void grid_barrier(cg::grid_group& g) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  g.sync();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  __device__ static __forceinline__ void load(const float* p, double* x) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    x[0] = v.x;
    x[1] = v.y;
    x[2] = v.z;
    x[3] = v.w;
  }
};
template <>
struct Vec4<double> {
  __device__ static __forceinline__ void load(const double* p, double* x) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    x[0] = a.x;
    x[1] = a.y;
    x[2] = b.x;
    x[3] = b.y;
  }
};

// out[r] = s * sum_c X[row0 + r][c] v[c] for the kSpecRows rows of one chunk
// (0 for rows >= n), FP64 accumulation. Wave w handles rows
// row0 + w * kRowsPerWave ..; lanes walk the row in groups of 4 columns, so
// a wave reads each row as contiguous 1 KiB (FP32) or 2 KiB (FP64) runs.
// v is zero past n; the iterate's padding columns are zero as well.
template <typename T>
__device__ __forceinline__ void chunk_matvec(const T* __restrict__ X, int ld,
                                             int n, int ldq, int row0,
                                             const double* __restrict__ v,
                                             double s, double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = row0 + wave * kRowsPerWave;
  const int nr = min(kRowsPerWave, n - r0);   // rows of this wave inside n
  double acc[kRowsPerWave];
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) acc[r] = 0.0;
  if (nr == kRowsPerWave) {
    for (int col = lane * 4; col < ldq; col += 256) {
      const double2 va = *reinterpret_cast<const double2*>(v + col);
      const double2 vb = *reinterpret_cast<const double2*>(v + col + 2);
      double x[kRowsPerWave][4];
#pragma unroll
      for (int r = 0; r < kRowsPerWave; ++r)
        Vec4<T>::load(X + static_cast<size_t>(r0 + r) * ld + col, x[r]);
#pragma unroll
      for (int r = 0; r < kRowsPerWave; ++r) {
        acc[r] = fma(x[r][0], va.x, acc[r]);
        acc[r] = fma(x[r][1], va.y, acc[r]);
        acc[r] = fma(x[r][2], vb.x, acc[r]);
        acc[r] = fma(x[r][3], vb.y, acc[r]);
      }
    }
  } else if (nr > 0) {
    for (int col = lane * 4; col < ldq; col += 256) {
      const double2 va = *reinterpret_cast<const double2*>(v + col);
      const double2 vb = *reinterpret_cast<const double2*>(v + col + 2);
      for (int r = 0; r < nr; ++r) {
        double x[4];
        Vec4<T>::load(X + static_cast<size_t>(r0 + r) * ld + col, x);
        acc[r] = fma(x[0], va.x, acc[r]);
        acc[r] = fma(x[1], va.y, acc[r]);
        acc[r] = fma(x[2], vb.x, acc[r]);
        acc[r] = fma(x[3], vb.y, acc[r]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) {
    const double t = wave_sum(acc[r]);
    if (lane == 0) out[wave * kRowsPerWave + r] = (r < nr) ? t * s : 0.0;
  }
}

// part[l] = sum over the chunk's rows of Q[l][row] * wl[row - row0] for
// l = 0..j: each 32-lane half of a wave takes one l at a time.
__device__ __forceinline__ void chunk_dots(const double* __restrict__ Q,
                                           int ldq, int row0,
                                           const double* wl, int j,
                                           double* __restrict__ part) {
  const int g = threadIdx.x >> 5, t = threadIdx.x & 31;
  const double wt = wl[t];
  for (int l0 = 0; l0 <= j; l0 += kThreads / 32) {
    const int l = l0 + g;
    double d = (l <= j) ? Q[static_cast<size_t>(l) * ldq + row0 + t] * wt : 0.0;
    d = half_sum(d);
    if (t == 0 && l <= j) part[l] = d;
  }
}

// coef[l] = sum over the instance's chunks, in chunk order, of
// part[q * kLanczosMax + l], l = 0..j. The four waves sum interleaved
// quarters of the chunks; the quarters are added in wave order.
__device__ __forceinline__ void sum_over_chunks(const double* __restrict__ part,
                                                int nch, int j, double* coef,
                                                double (*quarter)[kLanczosMax]) {
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double s = 0.0;
  if (l <= j)
    for (int q = wave; q < nch; q += kWaves) s += part[q * kLanczosMax + l];
  __syncthreads();
  quarter[wave][l] = s;
  __syncthreads();
  if (threadIdx.x <= j) {
    double t = quarter[0][threadIdx.x];
    for (int w = 1; w < kWaves; ++w) t += quarter[w][threadIdx.x];
    coef[threadIdx.x] = t;
  }
  __syncthreads();
}

// Whether the workgroup skips a chunk of instance `in`: the instance has
// stopped, or its estimate is final. One thread reads the flags and shares
// them through LDS, so the whole workgroup takes the same branch even while
// another workgroup is setting the instance's final flag (phase P1).
__device__ __forceinline__ bool skip_chunk(const Instance& in, int* flag) {
  __syncthreads();   // flag may still be read for the previous chunk
  if (threadIdx.x == 0) {
    int sk = in.st->done ? 1 : 0;
    if (!sk) {
      const SpecView v = spec_view(in.sp, in.n);
      sk = (__hip_atomic_load(&v.misc[1], __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT) != 0.0)
               ? 1
               : 0;
    }
    *flag = sk;
  }
  __syncthreads();
  return *flag != 0;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void spectral_kernel(SpecArgs a) {
  cg::grid_group grid = cg::this_grid();
  __shared__ double coef[kLanczosMax];
  __shared__ double quarter[kWaves][kLanczosMax];
  __shared__ double rowv[kSpecRows];
  __shared__ double tta[kLanczosMax], ttb[kLanczosMax];
  __shared__ double red[kWaves];
  __shared__ int hits[kThreads];
  __shared__ int skip;
  const int G = static_cast<int>(gridDim.x);
  const int iter = a.iter;

  // Instances still running; their done flags do not change during the
  // launch, so every workgroup counts the same number and takes the same
  // path through the barriers below.
  double act_d = 0.0;
  for (int q = threadIdx.x; q < a.count; q += kThreads)
    act_d += a.inst[q].st->done ? 0.0 : 1.0;
  const int act = static_cast<int>(block_sum(act_d, red));
  if (act == 0) return;

  // start vector, unnormalised, in w
  for (int c = blockIdx.x; c < a.nchunks; c += G) {
    const int2 ch = a.chunks[c];
    const Instance& in = a.inst[ch.x];
    if (in.st->done) continue;
    const SpecView v = spec_view(in.sp, in.n);
    const int lc = c - in.sp_ch0;
    double x = 0.0;
    if (threadIdx.x < kSpecRows) {
      const int row = ch.y + threadIdx.x;
      x = (row < in.n) ? start_entry(row) : 0.0;
      v.w[row] = x;
    }
    const double s2 = block_sum(x * x, red);
    if (threadIdx.x == 0) {
      v.nrm[lc] = s2;
      if (lc == 0) {
        v.misc[0] = 0.0;
        v.misc[1] = 0.0;
      }
    }
  }
  grid_barrier(grid);

  for (int j = 0;; ++j) {
    // P1
    for (int c = blockIdx.x; c < a.nchunks; c += G) {
      const int2 ch = a.chunks[c];
      const Instance& in = a.inst[ch.x];
      if (skip_chunk(in, &skip)) continue;
      const SpecView v = spec_view(in.sp, in.n);
      const int lc = c - in.sp_ch0;
      double s2 = 0.0;
      for (int q = threadIdx.x; q < in.sp_nch; q += kThreads) s2 += v.nrm[q];
      const double beta = sqrt(block_sum(s2, red));
      if (lc == 0 && j >= 1) {
        // estimate from T_j: alpha_0..alpha_{j-1}, beta_0..beta_{j-2}
        const double prev = v.misc[0];   // read before thread 0 rewrites it
        for (int q = threadIdx.x; q < j; q += kThreads) {
          tta[q] = v.ta[q];
          ttb[q] = (q + 1 < j) ? v.tb[q] : 0.0;
        }
        __syncthreads();
        const double top = tridiag_eig(tta, ttb, j, j, hits);
        const double bot = tridiag_eig(tta, ttb, j, 1, hits);
        const double theta = fmax(fabs(top), fabs(bot));
        const bool fin = !(beta > 1e-14 * theta) || !isfinite(beta) ||
                         (j >= 2 && fabs(theta - prev) <= kSpecTol * theta) ||
                         j == kLanczosMax || j == in.n;
        if (threadIdx.x == 0) {
          v.tb[j - 1] = beta;
          if (fin) {
            in.st->m[iter - 1] = theta;
            __hip_atomic_store(&v.misc[1], 1.0, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(a.ndone, 1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
          } else {
            v.misc[0] = theta;
          }
        }
        __syncthreads();
        if (fin) continue;
      }
      if (j == kLanczosMax) continue;   // every instance is final now
      const double inv = (beta > 0.0) ? 1.0 / beta : 0.0;
      if (threadIdx.x < kSpecRows) {
        const int row = ch.y + threadIdx.x;
        v.Q[static_cast<size_t>(j) * spec_ldq(in.n) + row] = v.w[row] * inv;
      }
      const void* Xv = in.X[(iter - 1) & 1];
      chunk_matvec<T>(static_cast<const T*>(Xv), in.ld, in.n, spec_ldq(in.n),
                      ch.y, v.w, inv, rowv);
      __syncthreads();
      if (threadIdx.x < kSpecRows) v.y[ch.y + threadIdx.x] = rowv[threadIdx.x];
      __syncthreads();
    }
    grid_barrier(grid);
    const int fin_cnt = __hip_atomic_load(a.ndone, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    if (fin_cnt >= act) break;

    // P2: w = y - X~ y, first pass of dots
    for (int c = blockIdx.x; c < a.nchunks; c += G) {
      const int2 ch = a.chunks[c];
      const Instance& in = a.inst[ch.x];
      if (skip_chunk(in, &skip)) continue;
      const SpecView v = spec_view(in.sp, in.n);
      const int lc = c - in.sp_ch0;
      const int ldq = spec_ldq(in.n);
      const void* Xv = in.X[(iter - 1) & 1];
      chunk_matvec<T>(static_cast<const T*>(Xv), in.ld, in.n, ldq, ch.y, v.y,
                      1.0, rowv);
      __syncthreads();
      if (threadIdx.x < kSpecRows) {
        const int row = ch.y + threadIdx.x;
        const double wv = v.y[row] - rowv[threadIdx.x];
        v.w[row] = wv;
        rowv[threadIdx.x] = wv;
      }
      __syncthreads();
      chunk_dots(v.Q, ldq, ch.y, rowv, j, v.c1 + lc * kLanczosMax);
      __syncthreads();
    }
    grid_barrier(grid);

    // P3: w -= sum_l c_l q_l, second pass of dots; alpha_j = c_j + c'_j
    for (int c = blockIdx.x; c < a.nchunks; c += G) {
      const int2 ch = a.chunks[c];
      const Instance& in = a.inst[ch.x];
      if (skip_chunk(in, &skip)) continue;
      const SpecView v = spec_view(in.sp, in.n);
      const int lc = c - in.sp_ch0;
      const int ldq = spec_ldq(in.n);
      sum_over_chunks(v.c1, in.sp_nch, j, coef, quarter);
      if (lc == 0 && threadIdx.x == 0) v.ta[j] = coef[j];
      if (threadIdx.x < kSpecRows) {
        const int row = ch.y + threadIdx.x;
        double x = v.w[row];
        for (int l = 0; l <= j; ++l)
          x -= coef[l] * v.Q[static_cast<size_t>(l) * ldq + row];
        v.w[row] = x;
        rowv[threadIdx.x] = x;
      }
      __syncthreads();
      chunk_dots(v.Q, ldq, ch.y, rowv, j, v.c2 + lc * kLanczosMax);
      __syncthreads();
    }
    grid_barrier(grid);

    // P4: w -= sum_l c'_l q_l, ||w||^2 per chunk
    for (int c = blockIdx.x; c < a.nchunks; c += G) {
      const int2 ch = a.chunks[c];
      const Instance& in = a.inst[ch.x];
      if (skip_chunk(in, &skip)) continue;
      const SpecView v = spec_view(in.sp, in.n);
      const int lc = c - in.sp_ch0;
      const int ldq = spec_ldq(in.n);
      sum_over_chunks(v.c2, in.sp_nch, j, coef, quarter);
      if (lc == 0 && threadIdx.x == 0) v.ta[j] += coef[j];
      double x = 0.0;
      if (threadIdx.x < kSpecRows) {
        const int row = ch.y + threadIdx.x;
        x = v.w[row];
        for (int l = 0; l <= j; ++l)
          x -= coef[l] * v.Q[static_cast<size_t>(l) * ldq + row];
        v.w[row] = x;
      }
      const double s2 = block_sum(x * x, red);
      if (threadIdx.x == 0) v.nrm[lc] = s2;
    }
    grid_barrier(grid);
  }
}

}  // namespace

int spectral_max_grid(bool fp64_store, int num_cus) {
  int per_cu = 0;
  const hipError_t e =
      fp64_store ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                       &per_cu, spectral_kernel<double>, kThreads, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                       &per_cu, spectral_kernel<float>, kThreads, 0);
  if (e != hipSuccess || per_cu < 1) return 0;
  return per_cu * num_cus;
}

hipError_t launch_spectral(const SpecArgs& a, bool fp64_store, int grid,
                           hipStream_t s) {
  SpecArgs arg = a;
  void* params[] = {&arg};
  const void* fn = fp64_store
                       ? reinterpret_cast<const void*>(&spectral_kernel<double>)
                       : reinterpret_cast<const void*>(&spectral_kernel<float>);
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kThreads), params, 0,
                                    s);
}

}  // namespace sp2
