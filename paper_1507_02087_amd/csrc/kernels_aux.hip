// Auxiliary kernels of the SP2 path: the affine start X_0 with its FP64
// traces, the scalar finalize/stop step, and small fill/copy kernels.
#include <math.h>

#include "finalize_logic.h"
#include "sp2_device.h"
#include "tridiag.h"

namespace sp2 {

namespace {

constexpr int kThreads = 256;


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

// Clears the states of `count` instances and the batch's done counter.
__global__ __launch_bounds__(kThreads) void state_reset_kernel(
    DevState* st, int count, int32_t* ndone, int32_t* zero, int nzero) {
  DevState* me = st + blockIdx.x;
  int32_t* w = reinterpret_cast<int32_t*>(me);
  const int words = static_cast<int>(sizeof(DevState) / sizeof(int32_t));
  for (int i = threadIdx.x; i < words; i += kThreads) w[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    me->p[0] = -1;
    me->alpha[0] = 1.0;
    if (blockIdx.x == 0) *ndone = 0;
  }
  if (blockIdx.x == 0 && zero)
    for (int i = threadIdx.x; i < nzero; i += kThreads) zero[i] = 0;
}

// X_0 = (lambda_max I - F) / (lambda_max - lambda_min) in FP64 (Alg. 2),
// truncated (|x| < tau -> 0, sec. 5), rounded to the storage type, with the
// padding region set to zero; X_0 = 0 or I when n_occ is 0 or n. With a
// stretch on step 1 the buffer receives a X~_0 + c I (OpMap). Each block
// handles kF0Rows rows of one instance and writes one partial triple
// (0, Tr, sum x^2) of X~_0.
template <typename T>
__global__ __launch_bounds__(kThreads) void f0_kernel(
    const Instance* __restrict__ insts, const F0Item* __restrict__ items,
    double* __restrict__ part) {
  __shared__ double sh[kThreads / 64][3];
  const F0Item it = items[blockIdx.x];
  const Instance& in = insts[it.inst];
  const int n = in.n, ld = in.ld;   // row stride (padded width)
  const int n_occ = static_cast<int>(in.prm.n_occ);
  const int trivial = (n_occ == 0) ? 1 : (n_occ == n ? 2 : 0);
  T* X = static_cast<T*>(in.X[0]);
  __bf16* XH = static_cast<__bf16*>(in.XH[0]);
  __bf16* XL = static_cast<__bf16*>(in.XL[0]);
  // stored: the matrix step 1 squares, a X~_0 + c I (OpMap; X~_0 itself
  // without a stretch and for n_occ = 0 or n)
  const OpMap m1 = step_map(in, 1);
  const bool stretch = !trivial && (m1.a != 1.0 || m1.c != 0.0);
  double t1 = 0.0, t2 = 0.0;
  for (int rr = 0; rr < kF0Rows; ++rr) {
    const int i = it.row0 + rr;
    const double* Fi = in.F + static_cast<int64_t>(i) * in.ldf;
    T* Xi = X + static_cast<int64_t>(i) * ld;
    for (int j = threadIdx.x; j < ld; j += kThreads) {
      double x = 0.0;
      if (i < n && j < n) {
        if (trivial) {
          x = (trivial == 2 && i == j) ? 1.0 : 0.0;
        } else {
          const double f = Fi[j];
          x = ((i == j) ? in.lmax - f : -f) / in.width;
          if (fabs(x) < in.tau) x = 0.0;
        }
      }
      const T xt = static_cast<T>(x);
      const double xd = static_cast<double>(xt);
      const T xs = stretch ? static_cast<T>(__builtin_fma(
                                 m1.a, xd, (i == j && i < n) ? m1.c : 0.0))
                           : xt;
      Xi[j] = xs;
      if (XH) {
        const float xf = static_cast<float>(xs);
        const __bf16 hb = static_cast<__bf16>(xf);
        const size_t o = static_cast<size_t>(i) * ld + j;
        XH[o] = hb;
        XL[o] = static_cast<__bf16>(xf - static_cast<float>(hb));
      }
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

// Sum over the workgroup, returned to every thread (fixed order).
__device__ __forceinline__ double block_sum_all(double x, double* red) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();   // red may still be read from a previous call
  if (lane == 0) red[wave] = x;
  __syncthreads();
  double t = red[0];
  for (int w = 1; w < kThreads / 64; ++w) t += red[w];
  return t;
}

constexpr int kMaxBlockRows = 2048;   // n / 32 for n <= 65536

constexpr int kLanczos = kLanczosMax;  // Krylov dimension cap
constexpr double kLanczosTol = 1e-12; // relative change of the top Ritz value

// Mixed norm of X~_{iter-1} - S (sec. 2): the spectral norm of the
// symmetric, nonnegative matrix M of block Frobenius norms that the step's
// epilogues wrote, i.e. its largest eigenvalue, by Lanczos from the
// normalised all-ones vector with full reorthogonalisation (classical
// Gram-Schmidt, twice), in FP64. The Lanczos basis lives in the instance's
// scratch (kLanczos x nbk doubles); w is an LDS vector of nbk doubles, c an
// LDS array of kLanczos doubles. Every thread of the workgroup takes part
// and receives the result.
__device__ double mixed_norm(const Instance& in, int iter, double* w,
                             double* c, double* ta, double* tb, int* hits,
                             double* red, int* steps) {
  const int nb = in.nbk;
  const bool sparse = (in.brp[0] != nullptr);
  const int32_t* rp = sparse ? in.brp[iter & 1] : nullptr;
  const int32_t* col = sparse ? in.bcol[iter & 1] : nullptr;
  double* Q = in.lz;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double q0 = 1.0 / sqrt(static_cast<double>(nb));
  for (int i = threadIdx.x; i < nb; i += kThreads) Q[i] = q0;
  double theta = 0.0;
  int m = 0;
  for (int j = 0; j < kLanczos; ++j) {
    __syncthreads();   // Q row j complete
    const double* qj = Q + static_cast<size_t>(j) * nb;
    for (int i = threadIdx.x; i < nb; i += kThreads) {
      double acc = 0.0;
      if (sparse) {
#pragma unroll 4
        for (int q = rp[i]; q < rp[i + 1]; ++q)
          acc += static_cast<double>(in.blk[q]) * qj[col[q]];
      } else {
        // M is symmetric: walk column i so that neighbouring threads read
        // neighbouring addresses; the loads of 16 rows go out together
#pragma unroll 16
        for (int l = 0; l < nb; ++l)
          acc += static_cast<double>(in.blk[static_cast<size_t>(l) * nb + i]) *
                 qj[l];
      }
      w[i] = acc;
    }
    // w -= sum_l (q_l . w) q_l over l = 0..j, twice; the first pass's
    // coefficient for l = j is alpha_j = q_j . M q_j
    for (int pass = 0; pass < 2; ++pass) {
      __syncthreads();
      for (int l = wave; l <= j; l += kThreads / 64) {
        const double* ql = Q + static_cast<size_t>(l) * nb;
        double d = 0.0;
        for (int i = lane; i < nb; i += 64) d += ql[i] * w[i];
        d = wave_sum(d);
        if (lane == 0) c[l] = d;
      }
      __syncthreads();
      if (pass == 0 && threadIdx.x == 0) ta[j] = c[j];
      for (int i = threadIdx.x; i < nb; i += kThreads) {
        double x = w[i];
#pragma unroll 8
        for (int l = 0; l <= j; ++l) x -= c[l] * Q[static_cast<size_t>(l) * nb + i];
        w[i] = x;
      }
    }
    double ww = 0.0;
    for (int i = threadIdx.x; i < nb; i += kThreads) ww += w[i] * w[i];
    ww = block_sum_all(ww, red);
    const double beta = sqrt(ww);
    m = j + 1;
    const double prev = theta;
    theta = tridiag_eig(ta, tb, m, m, hits);   // the top eigenvalue
    // an invariant subspace (beta ~ 0), convergence, or the last step
    if (!(beta > 1e-14 * fabs(theta)) || !isfinite(beta) ||
        (j > 0 && fabs(theta - prev) <= kLanczosTol * fabs(theta)) ||
        j + 1 == kLanczos || j + 1 == nb)
      break;
    __syncthreads();
    if (threadIdx.x == 0) tb[j] = beta;
    double* qn = Q + static_cast<size_t>(j + 1) * nb;
    for (int i = threadIdx.x; i < nb; i += kThreads) qn[i] = w[i] / beta;
  }
  *steps = m;
  return theta;
}

// One block per instance: sums the instance's partial triples of step
// `iter` in a fixed order and applies the scalar part of Alg. 2 (Alg. 4
// with a schedule) on one thread:
//   iter == 0: Tr X~_0, Tr X~_0^2; divergence check; choose p_1 (an
//     instance with n_occ = 0 or n stops here with n = 0).
//   iter >= 1: v_{iter-1} from the square of X~_{iter-1}; Tr/Tr^2 of X~_iter;
//     stop test at k = iter - 1 (from k = 2, or from n_min with a schedule;
//     a schedule also ends at k = n_max); divergence; max_iter; choose
//     p_{iter+1} and its stretch.
__global__ __launch_bounds__(kThreads) void finalize_kernel(
    const Instance* __restrict__ insts, int count,
    const double* __restrict__ part, const double* __restrict__ part_f0,
    int32_t* ndone, HostMirror* mirror, int iter) {
  __shared__ double sh[kThreads / 64][3];
  const Instance& in = insts[blockIdx.x];
  DevState* st = in.st;
  if (st->done) return;
  const double* pp = (iter == 0) ? part_f0 + 3 * in.f0blk0 : part + 3 * in.tile0;
  const int cnt = (iter == 0) ? in.nf0blk : in.ntiles;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < cnt; i += kThreads) {
    a += pp[3 * i + 0];
    b += pp[3 * i + 1];
    c += pp[3 * i + 2];
  }
  block_sum3(a, b, c, sh);
  const StopParams& prm = in.prm;
  double mk = 0.0;
  int mk_steps = 0;
  if (iter >= 1 && prm.norm == 1) {
    __shared__ double wv[kMaxBlockRows], cf[kLanczos], ta[kLanczos],
        tb[kLanczos], red[kThreads / 64];
    __shared__ int hits[kThreads];
    mk = mixed_norm(in, iter, wv, cf, ta, tb, hits, red, &mk_steps);
  }
  if (threadIdx.x != 0) return;
  finalize_scalar(in, iter, a, b, c, mk, mk_steps, ndone, count, mirror);
}

// D = (X - c I) / a (OpMap m; a = 1, c = 0 copies exactly).
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kThreads) void copy_out_kernel(
    const Tin* __restrict__ X, int n, int ldx, OpMap m, Tout* __restrict__ D,
    int64_t ldd) {
  const int64_t total = static_cast<int64_t>(n) * n;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
       e < total; e += static_cast<int64_t>(gridDim.x) * kThreads) {
    const int64_t i = e / n, j = e % n;
    const double x = static_cast<double>(X[i * ldx + j]);
    D[i * ldd + j] = static_cast<Tout>((x - (i == j ? m.c : 0.0)) / m.a);
  }
}

// D = (X - c I) / a for a symmetric X of which only the upper triangle is
// current: block (bi, bj) of 32 x 32 with bi <= bj reads the upper tile
// through LDS and writes it and its transpose, both as rows (coalesced).
// Blocks with bi > bj have nothing to do.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kThreads) void copy_out_sym_kernel(
    const Tin* __restrict__ X, int n, int ldx, OpMap m, Tout* __restrict__ D,
    int64_t ldd) {
  constexpr int B = 32;
  __shared__ Tin t[B][B + 1];
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bi > bj) return;
  const int i0 = bi * B, j0 = bj * B;
  for (int e = threadIdx.x; e < B * B; e += kThreads) {
    const int r = e / B, c = e % B;
    const int i = i0 + r, j = j0 + c;
    if (i < n && j < n) t[r][c] = X[static_cast<int64_t>(i) * ldx + j];
  }
  __syncthreads();
  auto val = [&](Tin x, bool diag) {
    return static_cast<Tout>((static_cast<double>(x) - (diag ? m.c : 0.0)) / m.a);
  };
  for (int e = threadIdx.x; e < B * B; e += kThreads) {
    const int r = e / B, c = e % B;
    const int i = i0 + r, j = j0 + c;
    if (i < n && j < n) {
      // on a diagonal tile the lower part comes from the transposed position
      const Tin x = (bi == bj && r > c) ? t[c][r] : t[r][c];
      D[static_cast<int64_t>(i) * ldd + j] = val(x, i == j);
    }
  }
  if (bi == bj) return;
  // the transpose: row j0 + r of D receives column r of the tile
  for (int e = threadIdx.x; e < B * B; e += kThreads) {
    const int r = e / B, c = e % B;
    const int i = j0 + r, j = i0 + c;
    if (i < n && j < n)
      D[static_cast<int64_t>(i) * ldd + j] = val(t[c][r], false);
  }
}

int grid_for(int64_t total) {
  int64_t g = (total + kThreads - 1) / kThreads;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return static_cast<int>(g);
}

}  // namespace

hipError_t launch_state_reset(DevState* st, int count, int32_t* ndone,
                              int32_t* zero, int nzero, hipStream_t s) {
  hipLaunchKernelGGL(state_reset_kernel, dim3(count), dim3(kThreads), 0, s, st,
                     count, ndone, zero, nzero);
  return hipGetLastError();
}

hipError_t launch_f0(const Instance* inst, const F0Item* items, int nitems,
                     bool fp64_store, double* part_f0, hipStream_t s) {
  if (fp64_store)
    hipLaunchKernelGGL(f0_kernel<double>, dim3(nitems), dim3(kThreads), 0, s,
                       inst, items, part_f0);
  else
    hipLaunchKernelGGL(f0_kernel<float>, dim3(nitems), dim3(kThreads), 0, s,
                       inst, items, part_f0);
  return hipGetLastError();
}

hipError_t launch_finalize(const Instance* inst, int count,
                           const double* part, const double* part_f0,
                           int32_t* ndone, HostMirror* mirror, int iter,
                           hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(count), dim3(kThreads), 0, s, inst,
                     count, part, part_f0, ndone, mirror, iter);
  return hipGetLastError();
}

hipError_t launch_copy_out(const void* X, bool fp64_store, int n, int ldx,
                           void* D, int64_t ldd, bool out_fp64, bool symmetric,
                           OpMap m, hipStream_t s) {
  if (symmetric) {
    const int nb = (n + 31) / 32;
    const dim3 grid(nb, nb);
    if (fp64_store)
      hipLaunchKernelGGL((copy_out_sym_kernel<double, double>), grid,
                         dim3(kThreads), 0, s, static_cast<const double*>(X), n,
                         ldx, m, static_cast<double*>(D), ldd);
    else if (out_fp64)
      hipLaunchKernelGGL((copy_out_sym_kernel<float, double>), grid,
                         dim3(kThreads), 0, s, static_cast<const float*>(X), n,
                         ldx, m, static_cast<double*>(D), ldd);
    else
      hipLaunchKernelGGL((copy_out_sym_kernel<float, float>), grid,
                         dim3(kThreads), 0, s, static_cast<const float*>(X), n,
                         ldx, m, static_cast<float*>(D), ldd);
    return hipGetLastError();
  }
  const int g = grid_for(static_cast<int64_t>(n) * n);
  if (fp64_store) {
    hipLaunchKernelGGL((copy_out_kernel<double, double>), dim3(g),
                       dim3(kThreads), 0, s, static_cast<const double*>(X), n,
                       ldx, m, static_cast<double*>(D), ldd);
  } else if (out_fp64) {
    hipLaunchKernelGGL((copy_out_kernel<float, double>), dim3(g),
                       dim3(kThreads), 0, s, static_cast<const float*>(X), n,
                       ldx, m, static_cast<double*>(D), ldd);
  } else {
    hipLaunchKernelGGL((copy_out_kernel<float, float>), dim3(g),
                       dim3(kThreads), 0, s, static_cast<const float*>(X), n,
                       ldx, m, static_cast<float*>(D), ldd);
  }
  return hipGetLastError();
}

}  // namespace sp2
