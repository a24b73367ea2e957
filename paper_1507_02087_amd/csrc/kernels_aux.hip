// Auxiliary kernels of the SP2 path: the affine start X_0 with its FP64
// traces, the scalar finalize/stop step, and small fill/copy kernels.
#include <math.h>

#include "sp2_device.h"

namespace sp2 {

namespace {

constexpr int kThreads = 256;

// C of Alg. 2: the smallest constant with r_k >= 2 in exact arithmetic over
// two alternating SP2 steps, (71 + 17 sqrt 17) / 32.
__device__ __forceinline__ double c_sp2() {
  return (71.0 + 17.0 * sqrt(17.0)) / 32.0;
}
// q~ of sec. 2.
constexpr double kQTilde = 1.8;

__device__ __forceinline__ double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Fixed-order block reduction of three doubles (deterministic).
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c,
                                           double (*sh)[3]) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wave][0] = a;
    sh[wave][1] = b;
    sh[wave][2] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = sh[0][0];
    b = sh[0][1];
    c = sh[0][2];
    for (int w = 1; w < kThreads / 64; ++w) {
      a += sh[w][0];
      b += sh[w][1];
      c += sh[w][2];
    }
  }
}

__global__ __launch_bounds__(kThreads) void state_reset_kernel(DevState* st) {
  // Clears the whole state with vector stores; one block.
  int32_t* w = reinterpret_cast<int32_t*>(st);
  const int words = static_cast<int>(sizeof(DevState) / sizeof(int32_t));
  for (int i = threadIdx.x; i < words; i += kThreads) w[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) st->p[0] = -1;
}

// X_0 = (lambda_max I - F) / (lambda_max - lambda_min) in FP64 (Alg. 2),
// truncated (|x| < tau -> 0, sec. 5), rounded to the storage type, with the
// padding region set to zero. Each block handles `rows` consecutive rows of
// the padded matrix and writes one partial triple (0, Tr, sum x^2).
template <typename T>
__global__ __launch_bounds__(kThreads) void f0_kernel(
    const double* __restrict__ F, int64_t ldf, int n, int np, double lmax,
    double width, double tau, T* __restrict__ X, double* __restrict__ part,
    int rows) {
  __shared__ double sh[kThreads / 64][3];
  double t1 = 0.0, t2 = 0.0;
  const int r0 = blockIdx.x * rows;
  for (int rr = 0; rr < rows; ++rr) {
    const int i = r0 + rr;
    const double* Fi = F + static_cast<int64_t>(i) * ldf;
    T* Xi = X + static_cast<int64_t>(i) * np;
    for (int j = threadIdx.x; j < np; j += kThreads) {
      double x = 0.0;
      if (i < n && j < n) {
        const double f = Fi[j];
        x = ((i == j) ? lmax - f : -f) / width;
        if (fabs(x) < tau) x = 0.0;
      }
      const T xs = static_cast<T>(x);
      const double xd = static_cast<double>(xs);
      Xi[j] = xs;
      t2 += xd * xd;
      if (i == j) t1 += xd;
    }
  }
  double v = 0.0;
  block_sum3(v, t1, t2, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x + 0] = 0.0;
    part[3 * blockIdx.x + 1] = t1;
    part[3 * blockIdx.x + 2] = t2;
  }
}

__device__ __forceinline__ void publish(DevState* st, HostMirror* m,
                                        int status, int n) {
  st->status = status;
  st->n = n;
  st->done = 1;
  if (m) {
    __hip_atomic_store(&m->status, status, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&m->n, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&m->squares, st->squares, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&m->done, 1, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Sums the partial triples of step `iter` in a fixed order and applies the
// scalar part of Alg. 2 on one thread:
//   iter == 0: Tr X~_0, Tr X~_0^2; divergence check; choose p_1.
//   iter >= 1: v_{iter-1} from the square of X~_{iter-1}; Tr/Tr^2 of X~_iter;
//     stop test at k = iter - 1; divergence; max_iter; choose p_{iter+1}.
__global__ __launch_bounds__(kThreads) void finalize_kernel(
    const double* __restrict__ part, int count, DevState* st,
    HostMirror* mirror, int iter, StopParams prm) {
  __shared__ double sh[kThreads / 64][3];
  if (st->done) return;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < count; i += kThreads) {
    a += part[3 * i + 0];
    b += part[3 * i + 1];
    c += part[3 * i + 2];
  }
  block_sum3(a, b, c, sh);
  if (threadIdx.x != 0) return;

  const double t1 = b, t2 = c;
  st->t1[iter] = t1;
  st->t2[iter] = t2;
  if (iter == 0) {
    if (!isfinite(t1) || !isfinite(t2)) {
      publish(st, mirror, /*DIVERGED*/ 5, 0);
      return;
    }
  } else {
    const int k = iter - 1;
    const double vk = sqrt(a);
    st->v[k] = vk;
    st->squares = iter;
    double r = NAN;
    if (k >= 2) {
      const double vkm2 = st->v[k - 2];
      if (vkm2 > 0.0 && vkm2 < 1.0 && vk > 0.0)
        r = log(vk / c_sp2()) / log(vkm2);   // observed order (sec. 2)
    }
    st->r[k] = r;
    if (!isfinite(vk)) {
      publish(st, mirror, 5, k);
      return;
    }
    if (vk == 0.0) {                          // exactly idempotent
      publish(st, mirror, 0, k);
      return;
    }
    if (k >= 2 && st->p[k] != st->p[k - 1] && !isnan(r) && r < kQTilde) {
      publish(st, mirror, 0, k);              // Alg. 2 stop
      return;
    }
    if (!isfinite(t1) || !isfinite(t2) || t2 > t1 + prm.n) {
      publish(st, mirror, 5, iter);
      return;
    }
    if (iter >= prm.max_iter) {
      publish(st, mirror, /*NOT_CONVERGED*/ 4, iter);
      return;
    }
  }
  // Polynomial of the next step from the traces of X~_iter (Alg. 2 branch).
  int pn;
  if (prm.branch == 1) {
    pn = (t1 > prm.n_occ) ? 1 : 0;
  } else {
    pn = (fabs(t2 - prm.n_occ) < fabs(2.0 * t1 - t2 - prm.n_occ)) ? 1 : 0;
  }
  st->p[iter + 1] = static_cast<int8_t>(pn);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void fill_kernel(T* X, int n, int np,
                                                        int identity) {
  const int64_t total = static_cast<int64_t>(np) * np;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
       e < total; e += static_cast<int64_t>(gridDim.x) * kThreads) {
    const int i = static_cast<int>(e / np), j = static_cast<int>(e % np);
    X[e] = (identity && i == j && i < n) ? T(1) : T(0);
  }
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kThreads) void copy_out_kernel(
    const Tin* __restrict__ X, int n, int ldx, Tout* __restrict__ D,
    int64_t ldd) {
  const int64_t total = static_cast<int64_t>(n) * n;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
       e < total; e += static_cast<int64_t>(gridDim.x) * kThreads) {
    const int64_t i = e / n, j = e % n;
    D[i * ldd + j] = static_cast<Tout>(X[i * ldx + j]);
  }
}

int grid_for(int64_t total) {
  int64_t g = (total + kThreads - 1) / kThreads;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return static_cast<int>(g);
}

}  // namespace

hipError_t launch_state_reset(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(state_reset_kernel, dim3(1), dim3(kThreads), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_f0(const double* F, int64_t ldf, int n, int np, double lmax,
                     double width, double tau, void* X0, bool fp64_store,
                     double* part, int rows_per_block, hipStream_t s) {
  const int blocks = np / rows_per_block;
  if (fp64_store)
    hipLaunchKernelGGL(f0_kernel<double>, dim3(blocks), dim3(kThreads), 0, s,
                       F, ldf, n, np, lmax, width, tau,
                       static_cast<double*>(X0), part, rows_per_block);
  else
    hipLaunchKernelGGL(f0_kernel<float>, dim3(blocks), dim3(kThreads), 0, s,
                       F, ldf, n, np, lmax, width, tau,
                       static_cast<float*>(X0), part, rows_per_block);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* part, int count, DevState* st,
                           HostMirror* mirror, int iter, StopParams prm,
                           hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kThreads), 0, s, part,
                     count, st, mirror, iter, prm);
  return hipGetLastError();
}

hipError_t launch_fill(void* X, bool fp64_store, int n, int np, int identity,
                       hipStream_t s) {
  const int g = grid_for(static_cast<int64_t>(np) * np);
  if (fp64_store)
    hipLaunchKernelGGL(fill_kernel<double>, dim3(g), dim3(kThreads), 0, s,
                       static_cast<double*>(X), n, np, identity);
  else
    hipLaunchKernelGGL(fill_kernel<float>, dim3(g), dim3(kThreads), 0, s,
                       static_cast<float*>(X), n, np, identity);
  return hipGetLastError();
}

hipError_t launch_copy_out(const void* X, bool fp64_store, int n, int ldx,
                           void* D, int64_t ldd, bool out_fp64,
                           hipStream_t s) {
  const int g = grid_for(static_cast<int64_t>(n) * n);
  if (fp64_store) {
    hipLaunchKernelGGL((copy_out_kernel<double, double>), dim3(g),
                       dim3(kThreads), 0, s, static_cast<const double*>(X), n,
                       ldx, static_cast<double*>(D), ldd);
  } else if (out_fp64) {
    hipLaunchKernelGGL((copy_out_kernel<float, double>), dim3(g),
                       dim3(kThreads), 0, s, static_cast<const float*>(X), n,
                       ldx, static_cast<double*>(D), ldd);
  } else {
    hipLaunchKernelGGL((copy_out_kernel<float, float>), dim3(g),
                       dim3(kThreads), 0, s, static_cast<const float*>(X), n,
                       ldx, static_cast<float*>(D), ldd);
  }
  return hipGetLastError();
}

}  // namespace sp2
