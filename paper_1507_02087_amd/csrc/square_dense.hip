// Fused symmetric square of the SP2 recursion on gfx950 matrix cores.
//
// One launch computes S = X X for a symmetric X (Alg. 2: the one matrix
// product of every SP2 step). Because X is symmetric, S_ij = sum_k X_ik X_jk:
// both operands are row panels of X, contiguous along k, and only the upper
// triangle of macro tiles (I <= J) is computed; each tile is also stored
// transposed. The epilogue of each tile fuses the rest of the step:
//   d = X_old - S            (FP64)  -> sum d^2 = ||X~_{i-1} - X~_{i-1}^2||_F^2
//   X_new = S or 2 X_old - S  (Alg. 2, polynomial p_i read from device state)
//   |X_new| < tau -> 0        (truncation E_i, sec. 5)
//   Tr X_new and sum X_new^2  (FP64; traces for the next polynomial choice)
// Off-diagonal tiles count twice in the sums. In diagonal tiles only the
// upper triangle (row <= col) is used and mirrored, so every iterate is
// exactly symmetric.
//
// Each workgroup (4 waves) owns a BM x BM macro tile; the K loop stages
// BM x BK slices of the two row panels through double-buffered LDS with a
// register prefetch of the next slice. Within a wave the k index assigned to
// (MFMA substep, lane group) is permuted so that every lane reads a
// contiguous run of k from LDS; both operands use the same permutation, so
// the sum over k is unchanged.
//
// Workgroup -> tile mapping is XCD aware: dispatch places workgroup b on XCD
// b mod 8, and XCD x processes the contiguous chunk x of a tile list ordered
// by groups of neighbouring tiles, which keeps the row panels those tiles
// share resident in that XCD's L2.
#include "sp2_device.h"

namespace sp2 {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

struct Sums {
  double v = 0.0, t1 = 0.0, t2 = 0.0;
};

__device__ __forceinline__ double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Writes the tile's three partial sums in a fixed order (deterministic).
__device__ __forceinline__ void store_partials(Sums s, double* part, int slot) {
  __shared__ double sh[kThreads / 64][3];
  s.v = wave_sum(s.v);
  s.t1 = wave_sum(s.t1);
  s.t2 = wave_sum(s.t2);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wave][0] = s.v;
    sh[wave][1] = s.t1;
    sh[wave][2] = s.t2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = sh[0][0], b = sh[0][1], c = sh[0][2];
    for (int w = 1; w < kThreads / 64; ++w) {
      a += sh[w][0];
      b += sh[w][1];
      c += sh[w][2];
    }
    part[3 * slot + 0] = a;
    part[3 * slot + 1] = b;
    part[3 * slot + 2] = c;
  }
}

// The per-element part of the epilogue. w is the multiplicity of the element
// in the full symmetric matrix (2 off the diagonal, 1 on it).
// The truncation test compares the stored value in FP64.
template <typename T>
__device__ __forceinline__ T epilogue_elem(T s, T xo, int p, double tau,
                                           double w, bool on_diag, Sums& acc) {
  const double d = static_cast<double>(xo) - static_cast<double>(s);
  acc.v += w * (d * d);
  T xn = p ? s : T(2) * xo - s;
  double xd = static_cast<double>(xn);
  if (fabs(xd) < tau) {
    xn = T(0);
    xd = 0.0;
  }
  acc.t2 += w * (xd * xd);
  if (on_diag) acc.t1 += xd;
  return xn;
}

__device__ __forceinline__ int tile_slot(int per_xcd) {
  return static_cast<int>(blockIdx.x % 8u) * per_xcd +
         static_cast<int>(blockIdx.x / 8u);
}

// ---------------------------------------------------------------- FP32
// 128 x 128 macro tile, BK = 32, waves in 2 x 2, each wave 64 x 64 made of
// 2 x 2 blocks of v_mfma_f32_32x32x2_f32. Lane l of a 32x32 block supplies
// A[row = l % 32][kk = l / 32] and B[kk = l / 32][col = l % 32]; accumulator
// register j of lane l holds row 8 (j/4) + 4 (l/32) + j%4, column l % 32.
namespace f32 {
constexpr int BM = 128, BK = 32, LDK = BK + 4;
}

__global__ __launch_bounds__(kThreads) void square_f32_kernel(SquareArgs a) {
  using namespace f32;
  __shared__ __attribute__((aligned(16))) float As[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) float Bs[2][BM][LDK];
  if (a.st->done) return;
  const int slot = tile_slot(a.per_xcd);
  if (slot >= a.ntiles) return;
  const int2 tt = a.tiles[slot];
  const int I = tt.x, J = tt.y;
  const int p = a.st->p[a.iter];
  const int ld = a.ld;
  const float* __restrict__ X = static_cast<const float*>(a.X);
  float* __restrict__ Y = static_cast<float*>(a.Y);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int r = lane & 31, h = lane >> 5;
  const float* Ap = X + static_cast<size_t>(I * BM) * ld;
  const float* Bp = X + static_cast<size_t>(J * BM) * ld;
  const int lr = tid >> 3, lc = (tid & 7) * 4;

  floatx4 ra[4], rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ra[q] = *reinterpret_cast<const floatx4*>(
          Ap + static_cast<size_t>(lr + 32 * q) * ld + k0 + lc);
      rb[q] = *reinterpret_cast<const floatx4*>(
          Bp + static_cast<size_t>(lr + 32 * q) * ld + k0 + lc);
    }
  };
  auto sstore = [&](int b) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      *reinterpret_cast<floatx4*>(&As[b][lr + 32 * q][lc]) = ra[q];
      *reinterpret_cast<floatx4*>(&Bs[b][lr + 32 * q][lc]) = rb[q];
    }
  };

  floatx16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx16{};

  const int nk = ld / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int b = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
    floatx4 af[2][4], bfr[2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        af[m][q] = *reinterpret_cast<const floatx4*>(
            &As[b][wm + m * 32 + r][h * 16 + q * 4]);
        bfr[m][q] = *reinterpret_cast<const floatx4*>(
            &Bs[b][wn + m * 32 + r][h * 16 + q * 4]);
      }
#pragma unroll
    for (int s = 0; s < 16; ++s)
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
          acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(
              af[m][s >> 2][s & 3], bfr[n][s >> 2][s & 3], acc[m][n], 0, 0, 0);
    if (kt + 1 < nk) sstore(b ^ 1);
    __syncthreads();
  }

  // Epilogue.
  Sums sums;
  const double tau = a.tau;
  const bool diag_tile = (I == J);
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      const int gc = J * BM + wn + n * 32 + r;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int gr0 = I * BM + wm + m * 32 + 8 * jj + 4 * h;
        floatx4 out;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int gr = gr0 + e;
          const size_t idx = static_cast<size_t>(gr) * ld + gc;
          const float s = acc[m][n][jj * 4 + e];
          if (!diag_tile) {
            out[e] = epilogue_elem<float>(s, X[idx], p, tau, 2.0, false, sums);
            Y[idx] = out[e];
          } else if (gr <= gc) {
            const bool on = (gr == gc);
            const float xn = epilogue_elem<float>(s, X[idx], p, tau,
                                                  on ? 1.0 : 2.0, on, sums);
            Y[idx] = xn;
            if (!on) Y[static_cast<size_t>(gc) * ld + gr] = xn;
          }
        }
        if (!diag_tile)
          *reinterpret_cast<floatx4*>(Y + static_cast<size_t>(gc) * ld + gr0) =
              out;
      }
    }
  store_partials(sums, a.part, slot);
}

// ---------------------------------------------------------------- BF16x3
// Same tiling as FP32 with v_mfma_f32_32x32x16_bf16. Each FP32 element of X
// is split while it is staged into LDS: H = bf16(x), L = bf16(x - H), both
// rounded to nearest even; the tile accumulates H H + H L + L H in FP32
// (the L L term is below FP32 rounding of the result and is dropped).
// Lane l supplies 8 consecutive k of A[row = l % 32] and B[col = l % 32].
namespace b3 {
constexpr int BM = 128, BK = 32, LDK = BK + 8;
}

__device__ __forceinline__ void split_bf16(floatx4 x, bf16x4& hi, bf16x4& lo) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const __bf16 hb = static_cast<__bf16>(x[e]);
    hi[e] = hb;
    lo[e] = static_cast<__bf16>(x[e] - static_cast<float>(hb));
  }
}

__global__ __launch_bounds__(kThreads) void square_bf16x3_kernel(SquareArgs a) {
  using namespace b3;
  __shared__ __attribute__((aligned(16))) __bf16 AH[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 AL[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 BH[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 BL[2][BM][LDK];
  if (a.st->done) return;
  const int slot = tile_slot(a.per_xcd);
  if (slot >= a.ntiles) return;
  const int2 tt = a.tiles[slot];
  const int I = tt.x, J = tt.y;
  const int p = a.st->p[a.iter];
  const int ld = a.ld;
  const float* __restrict__ X = static_cast<const float*>(a.X);
  float* __restrict__ Y = static_cast<float*>(a.Y);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int r = lane & 31, h = lane >> 5;
  const float* Ap = X + static_cast<size_t>(I * BM) * ld;
  const float* Bp = X + static_cast<size_t>(J * BM) * ld;
  const int lr = tid >> 3, lc = (tid & 7) * 4;

  floatx4 ra[4], rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ra[q] = *reinterpret_cast<const floatx4*>(
          Ap + static_cast<size_t>(lr + 32 * q) * ld + k0 + lc);
      rb[q] = *reinterpret_cast<const floatx4*>(
          Bp + static_cast<size_t>(lr + 32 * q) * ld + k0 + lc);
    }
  };
  auto sstore = [&](int b) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      bf16x4 hi, lo;
      split_bf16(ra[q], hi, lo);
      *reinterpret_cast<bf16x4*>(&AH[b][lr + 32 * q][lc]) = hi;
      *reinterpret_cast<bf16x4*>(&AL[b][lr + 32 * q][lc]) = lo;
      split_bf16(rb[q], hi, lo);
      *reinterpret_cast<bf16x4*>(&BH[b][lr + 32 * q][lc]) = hi;
      *reinterpret_cast<bf16x4*>(&BL[b][lr + 32 * q][lc]) = lo;
    }
  };

  floatx16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx16{};

  const int nk = ld / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int b = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
    // 16 consecutive k per lane (two substeps of 8).
    bf16x8 ah[2][2], al[2][2], bh[2][2], bl[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        ah[m][s] = *reinterpret_cast<const bf16x8*>(
            &AH[b][wm + m * 32 + r][h * 16 + s * 8]);
        al[m][s] = *reinterpret_cast<const bf16x8*>(
            &AL[b][wm + m * 32 + r][h * 16 + s * 8]);
        bh[m][s] = *reinterpret_cast<const bf16x8*>(
            &BH[b][wn + m * 32 + r][h * 16 + s * 8]);
        bl[m][s] = *reinterpret_cast<const bf16x8*>(
            &BL[b][wn + m * 32 + r][h * 16 + s * 8]);
      }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              ah[m][s], bh[n][s], acc[m][n], 0, 0, 0);
          acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              ah[m][s], bl[n][s], acc[m][n], 0, 0, 0);
          acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              al[m][s], bh[n][s], acc[m][n], 0, 0, 0);
        }
    if (kt + 1 < nk) sstore(b ^ 1);
    __syncthreads();
  }

  Sums sums;
  const double tau = a.tau;
  const bool diag_tile = (I == J);
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      const int gc = J * BM + wn + n * 32 + r;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int gr0 = I * BM + wm + m * 32 + 8 * jj + 4 * h;
        floatx4 out;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int gr = gr0 + e;
          const size_t idx = static_cast<size_t>(gr) * ld + gc;
          const float s = acc[m][n][jj * 4 + e];
          if (!diag_tile) {
            out[e] = epilogue_elem<float>(s, X[idx], p, tau, 2.0, false, sums);
            Y[idx] = out[e];
          } else if (gr <= gc) {
            const bool on = (gr == gc);
            const float xn = epilogue_elem<float>(s, X[idx], p, tau,
                                                  on ? 1.0 : 2.0, on, sums);
            Y[idx] = xn;
            if (!on) Y[static_cast<size_t>(gc) * ld + gr] = xn;
          }
        }
        if (!diag_tile)
          *reinterpret_cast<floatx4*>(Y + static_cast<size_t>(gc) * ld + gr0) =
              out;
      }
    }
  store_partials(sums, a.part, slot);
}

// ---------------------------------------------------------------- FP64
// 128 x 128 macro tile, BK = 16, waves in 2 x 2, each wave 64 x 64 made of
// 4 x 4 blocks of v_mfma_f64_16x16x4_f64. Lane l of a 16x16 block supplies
// A[row = l % 16][kk = l / 16] and B[kk = l / 16][col = l % 16]; accumulator
// register j of lane l holds row 4 (l/16) + j, column l % 16.
namespace f64 {
constexpr int BM = 128, BK = 16, LDK = BK + 2;
}

__global__ __launch_bounds__(kThreads) void square_f64_kernel(SquareArgs a) {
  using namespace f64;
  __shared__ __attribute__((aligned(16))) double As[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) double Bs[2][BM][LDK];
  if (a.st->done) return;
  const int slot = tile_slot(a.per_xcd);
  if (slot >= a.ntiles) return;
  const int2 tt = a.tiles[slot];
  const int I = tt.x, J = tt.y;
  const int p = a.st->p[a.iter];
  const int ld = a.ld;
  const double* __restrict__ X = static_cast<const double*>(a.X);
  double* __restrict__ Y = static_cast<double*>(a.Y);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int r = lane & 15, g = lane >> 4;
  const double* Ap = X + static_cast<size_t>(I * BM) * ld;
  const double* Bp = X + static_cast<size_t>(J * BM) * ld;
  const int lr = tid >> 3, lc = (tid & 7) * 2;

  double2 ra[4], rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ra[q] = *reinterpret_cast<const double2*>(
          Ap + static_cast<size_t>(lr + 32 * q) * ld + k0 + lc);
      rb[q] = *reinterpret_cast<const double2*>(
          Bp + static_cast<size_t>(lr + 32 * q) * ld + k0 + lc);
    }
  };
  auto sstore = [&](int b) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      *reinterpret_cast<double2*>(&As[b][lr + 32 * q][lc]) = ra[q];
      *reinterpret_cast<double2*>(&Bs[b][lr + 32 * q][lc]) = rb[q];
    }
  };

  doublex4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = doublex4{};

  const int nk = ld / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int b = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
    double af[4][4], bfr[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const double2 a0 = *reinterpret_cast<const double2*>(
          &As[b][wm + m * 16 + r][g * 4]);
      const double2 a1 = *reinterpret_cast<const double2*>(
          &As[b][wm + m * 16 + r][g * 4 + 2]);
      af[m][0] = a0.x; af[m][1] = a0.y; af[m][2] = a1.x; af[m][3] = a1.y;
      const double2 b0 = *reinterpret_cast<const double2*>(
          &Bs[b][wn + m * 16 + r][g * 4]);
      const double2 b1 = *reinterpret_cast<const double2*>(
          &Bs[b][wn + m * 16 + r][g * 4 + 2]);
      bfr[m][0] = b0.x; bfr[m][1] = b0.y; bfr[m][2] = b1.x; bfr[m][3] = b1.y;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n)
          acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(
              af[m][s], bfr[n][s], acc[m][n], 0, 0, 0);
    if (kt + 1 < nk) sstore(b ^ 1);
    __syncthreads();
  }

  Sums sums;
  const double tau = a.tau;
  const bool diag_tile = (I == J);
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int gc = J * BM + wn + n * 16 + r;
      const int gr0 = I * BM + wm + m * 16 + 4 * g;
      double out[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gr = gr0 + e;
        const size_t idx = static_cast<size_t>(gr) * ld + gc;
        const double s = acc[m][n][e];
        if (!diag_tile) {
          out[e] = epilogue_elem<double>(s, X[idx], p, tau, 2.0, false, sums);
          Y[idx] = out[e];
        } else if (gr <= gc) {
          const bool on = (gr == gc);
          const double xn = epilogue_elem<double>(s, X[idx], p, tau,
                                                  on ? 1.0 : 2.0, on, sums);
          Y[idx] = xn;
          if (!on) Y[static_cast<size_t>(gc) * ld + gr] = xn;
        }
      }
      if (!diag_tile) {
        double* dst = Y + static_cast<size_t>(gc) * ld + gr0;
        *reinterpret_cast<double2*>(dst) = double2{out[0], out[1]};
        *reinterpret_cast<double2*>(dst + 2) = double2{out[2], out[3]};
      }
    }
  store_partials(sums, a.part, slot);
}

int grid_of(const SquareArgs& a) { return 8 * a.per_xcd; }

}  // namespace

bool square_tile_supported(int precision, int tile) {
  (void)precision;
  return tile == 128;
}

hipError_t launch_square_f64(const SquareArgs& a, int tile, hipStream_t s) {
  if (tile != f64::BM) return hipErrorInvalidValue;
  hipLaunchKernelGGL(square_f64_kernel, dim3(grid_of(a)), dim3(kThreads), 0, s,
                     a);
  return hipGetLastError();
}

hipError_t launch_square_f32(const SquareArgs& a, int tile, hipStream_t s) {
  if (tile != f32::BM) return hipErrorInvalidValue;
  hipLaunchKernelGGL(square_f32_kernel, dim3(grid_of(a)), dim3(kThreads), 0, s,
                     a);
  return hipGetLastError();
}

hipError_t launch_square_bf16x3(const SquareArgs& a, int tile, hipStream_t s) {
  if (tile != b3::BM) return hipErrorInvalidValue;
  hipLaunchKernelGGL(square_bf16x3_kernel, dim3(grid_of(a)), dim3(kThreads), 0,
                     s, a);
  return hipGetLastError();
}

}  // namespace sp2
