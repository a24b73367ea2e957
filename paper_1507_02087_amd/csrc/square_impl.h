// Kernel templates of the fused symmetric square (included by the
// per-family translation units square_f64.hip, square_f32.hip,
// square_b3.hip, square_b3s.hip and square_b3p.hip, which instantiate
// the configurations of one kernel family each, so that they compile in
// parallel).
//
// Fused symmetric square of the SP2 recursion on gfx950 matrix cores.
//
// One launch computes S = X X for a symmetric X (Alg. 2: the one matrix
// product of every SP2 step). Because X is symmetric, S_ij = sum_k X_ik X_jk:
// both operands are row panels of X, contiguous along k, and only the upper
// triangle of macro tiles (I <= J) is computed; each tile is also stored
// transposed. The epilogue of each tile fuses the rest of the step:
//   d = X_old - S            (FP64)  -> sum d^2 = ||X~_{i-1} - X~_{i-1}^2||_F^2
//   X_new = S or 2 X_old - S  (Alg. 2, polynomial p_i read from device state)
//   |X_new| < tau -> 0        (truncation E_i, sec. 5; compared in FP64)
//   Tr X_new and sum X_new^2  (FP64; traces for the next polynomial choice)
// With a stretch (SP2-ACC, McW-ACC) X_old is the stretched matrix
// Y = a X~ + c I that the step squares (OpMap), d is formed from Y and S
// with the step's coefficients, and the stored output is the next step's
// stretched matrix.
// Off-diagonal tiles count twice in the sums. In diagonal tiles only the
// upper triangle (row <= col) is used and mirrored, so every iterate is
// exactly symmetric.
//
// Work decomposition: the host gives every workgroup a WorkItem: a whole
// tile, one K-range piece of a tail tile, or nothing. Tail tiles are the
// tiles of an incomplete last round of workgroups; splitting each into
// several K pieces lets that round finish in a fraction of a tile's time.
// A piece stores its FP32/FP64 accumulators to a workspace in register order
// and a second kernel sums the pieces of each tail tile in a fixed order and
// runs the same epilogue (deterministic; no atomics).
//
// Each workgroup stages BM x BK slices of the two row panels through
// double-buffered LDS with a register prefetch of the next slice. The k index
// assigned to (MFMA substep, lane group) is permuted so that each lane reads
// contiguous runs of k from LDS; both operands use the same permutation, so
// the sum over k is unchanged.
#pragma once

#include <algorithm>

#include "finalize_logic.h"
#include "sp2_device.h"
#include "square_families.h"

namespace sp2 {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

struct Sums {
  double v = 0.0, t1 = 0.0, t2 = 0.0;
};

__device__ __forceinline__ double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Writes the tile's three partial sums in a fixed order (deterministic).
// mode 1 (McWeeny square) writes only the error, mode 2 (McWeeny product
// X~ S) only the traces, so that the two products of a step fill one slot.
template <int THREADS>
__device__ __forceinline__ void store_partials(Sums s, double* part, int slot,
                                               int mode = 0) {
  __shared__ double sh[THREADS / 64][3];
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
    for (int w = 1; w < THREADS / 64; ++w) {
      a += sh[w][0];
      b += sh[w][1];
      c += sh[w][2];
    }
    if (mode != 2) part[3 * slot + 0] = a;
    if (mode != 1) {
      part[3 * slot + 1] = b;
      part[3 * slot + 2] = c;
    }
  }
}

// Step polynomial in the storage type, applied to the stored matrix Y of
// the step and its square S = Y^2. mode 0 (SP2 step): X_i = ca S + cb Y,
// i.e. S (p = 1) or 2 Y - S (p = 0). mode 1 (McWeeny, first product): the
// square itself is the output. mode 2 (McWeeny, second product T = Y S):
// X_i = ca T + cs S = 3 S - 2 T. e holds the FP64 error coefficients and the
// map of the next step's matrix (StepCoef).
template <typename T>
struct Coef {
  T ca, cb, cs;
  int mode;
  // the run stretches: the error and the stored output take the step's
  // coefficients, read from ec (ey, es, ei, an, cn) where they are used, so
  // that they occupy no registers during the main loop; else a = 1, c = 0
  bool affine;
  const double* ec;
};

__device__ __forceinline__ double fused(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}
__device__ __forceinline__ float fused(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

// The per-element part of the epilogue. w is the multiplicity of the element
// in the full symmetric matrix (2 off the diagonal, 1 on it); on_diag marks
// a diagonal element of the matrix proper (not of its zero padding, which
// must stay zero under the identity terms). Without a stretch the new value
// is exactly S or the single rounding of 2 Y - S, and d = Y - S rounded once
// in FP64. The traces are those of X~_i; the returned (stored) value is the
// next step's matrix an X~_i + cn I, formed in FP64 and rounded once.
template <typename T, int MODE>
__device__ __forceinline__ T epilogue_elem(T s, T xo, T sv, const Coef<T>& k,
                                           double tau, double w, bool on_diag,
                                           Sums& acc, double& d2) {
  T xn;
  if (MODE == 2) {
    // s = (Y S)_ij, sv = S_ij: the new iterate, no error term
    d2 = 0.0;
    xn = fused(k.ca, s, k.cs * sv);
  } else {
    const double d =
        k.affine ? __builtin_fma(k.ec[1], static_cast<double>(s),
                                 k.ec[0] * static_cast<double>(xo)) +
                       (on_diag ? k.ec[2] : 0.0)
                 : static_cast<double>(xo) - static_cast<double>(s);
    d2 = d * d;
    acc.v += w * d2;
    if (MODE == 1) return s;   // the square S, kept as it is
    xn = fused(k.cb, xo, k.ca * s);
  }
  double xd = static_cast<double>(xn);
  if (fabs(xd) < tau) {
    xn = T(0);
    xd = 0.0;
  }
  acc.t2 += w * (xd * xd);
  if (on_diag) acc.t1 += xd;
  if (k.affine)
    xn = static_cast<T>(__builtin_fma(k.ec[3], xd, on_diag ? k.ec[4] : 0.0));
  return xn;
}

// Contribution of one processed element to the squared Frobenius norm of
// its 32 x 32 block of X~ - S: inside a diagonal block only the upper
// triangle is processed, so an off-diagonal element there stands for itself
// and its mirror.
__device__ __forceinline__ double block_share(int gr, int gc, double d2) {
  return (gr / kMixedBlock == gc / kMixedBlock && gr != gc) ? 2.0 * d2 : d2;
}

// Stores the Frobenius norm of block (rb, cb) of X~ - S and of its mirror.
__device__ __forceinline__ void blk_write(float* blk, int nbk, int rb, int cb,
                                          double sum) {
  const float v = static_cast<float>(sqrt(sum));
  *grw(blk + static_cast<size_t>(rb) * nbk + cb) = v;
  *grw(blk + static_cast<size_t>(cb) * nbk + rb) = v;
}

// Applies the epilogue to one accumulator value at tile-local (lr, lc);
// returns the element's share of its block's squared norm (0 if the element
// is a mirrored one that this tile does not process).
template <typename T, int MODE>
__device__ __forceinline__ double epilogue_at(const T* __restrict__ X,
                                              const T* __restrict__ Sr,
                                              T* __restrict__ Y, int ld, int n,
                                              int I, int J, int BM, int lr,
                                              int lc, T s, const Coef<T>& k,
                                              double tau, Sums& sums) {
  const int gr = I * BM + lr, gc = J * BM + lc;
  const size_t idx = static_cast<size_t>(gr) * ld + gc;
  double d2 = 0.0;
  const T sv = (MODE == 2) ? *gro(Sr + idx) : T(0);
  if (I != J) {
    const T xn = epilogue_elem<T, MODE>(s, *gro(X + idx), sv, k, tau, 2.0, false,
                                  sums, d2);
    *grw(Y + idx) = xn;
    *grw(Y + static_cast<size_t>(gc) * ld + gr) = xn;
    return d2;
  } else if (gr <= gc) {
    const bool on = (gr == gc);
    const T xn = epilogue_elem<T, MODE>(s, *gro(X + idx), sv, k, tau,
                                  on ? 1.0 : 2.0, on && gr < n, sums, d2);
    *grw(Y + idx) = xn;
    if (!on) *grw(Y + static_cast<size_t>(gc) * ld + gr) = xn;
    return block_share(gr, gc, d2);
  }
  return 0.0;
}

// Sum over the 32 lanes of a half wave (fixed order).
__device__ __forceinline__ double half_wave_sum(double x) {
  for (int off = 16; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}
__device__ __forceinline__ double full_wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Global -> register staging of a BM x BK slice of two row panels, in
// 16-byte chunks (CH elements each), spread over THREADS threads.
template <typename T, int BM, int BK, int THREADS>
struct Stage {
  static constexpr int CH = 16 / sizeof(T);
  static constexpr int CPR = BK / CH;                 // chunks per row
  static constexpr int NCH = BM * CPR / THREADS;      // chunks per thread
  static_assert(BM * CPR % THREADS == 0, "stage size");
  typedef T vec __attribute__((ext_vector_type(CH)));
  vec a[NCH], b[NCH];
  __device__ __forceinline__ static int row(int tid, int q) {
    return (tid + q * THREADS) / CPR;
  }
  __device__ __forceinline__ static int col(int tid, int q) {
    return ((tid + q * THREADS) % CPR) * CH;
  }
  __device__ __forceinline__ void load(const T* Ap, const T* Bp, int ld,
                                       int k0, int tid) {
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
      const size_t off =
          static_cast<size_t>(row(tid, q)) * ld + k0 + col(tid, q);
      a[q] = *gro(reinterpret_cast<const vec*>(Ap + off));
      b[q] = *gro(reinterpret_cast<const vec*>(Bp + off));
    }
  }
};

// What one workgroup needs to know about its step, built at kernel start.
template <typename T>
struct StepCtx {
  const T* X;     // X~_{i-1}: A operand rows, and the epilogue's X~
  const T* B;     // B operand rows: X~ (a square) or S (McWeeny X~ S)
  const T* Sr;    // S for the McWeeny X~ S epilogue (null otherwise)
  T* Y;           // output: X~_i, or S for the McWeeny square
  const __bf16* Xh;   // BF16x3 split of X~_{i-1} (null if absent)
  const __bf16* Xl;
  const __bf16* Bh;   // BF16x3 split of the B operand
  const __bf16* Bl;
  __bf16* Yh;         // BF16x3 split of the output (null if absent)
  __bf16* Yl;
  int ld;
  int n;          // matrix dimension (rows and columns >= n are padding)
  int2 tile;      // (I, J)
  Coef<T> k;      // polynomial of step i (Alg. 2 / Alg. 4)
  double tau;
  float* blk;     // block norms of X~_{i-1} - S (mixed norm), or null
  int nbk;
  bool mirror32;  // write the FP32 output's lower triangle
};

// STRETCH: the run stretches the matrices it squares (SP2-ACC, McW-ACC), so
// the error and the stored output take the coefficients the finalize kernel
// wrote; otherwise they are the constants of a = 1, c = 0 (the kernels of
// Alg. 2 carry no code for a stretch).
template <typename T, bool STRETCH>
__device__ __forceinline__ StepCtx<T> step_ctx(const SquareArgs& a,
                                               const Instance& in, int slot) {
  StepCtx<T> c;
  c.X = static_cast<const T*>(in.X[(a.iter - 1) & 1]);
  c.Xh = static_cast<const __bf16*>(in.XH[(a.iter - 1) & 1]);
  c.Xl = static_cast<const __bf16*>(in.XL[(a.iter - 1) & 1]);
  c.ld = in.ld;
  c.n = in.n;
  c.tile = a.tiles[slot];
  c.tau = in.tau;
  c.blk = in.blk;
  c.nbk = in.nbk;
  c.mirror32 = a.mirror32 != 0;
  c.Sr = nullptr;
  // the step's error coefficients and the map of the matrix it stores, as
  // the finalize kernel computed them with the step's polynomial
  const double* ec = STRETCH ? in.st->ecoef : nullptr;
  if (a.mode == 0) {
    const bool p1 = in.st->p[a.iter] != 0;
    c.k = Coef<T>{p1 ? T(1) : T(-1), p1 ? T(0) : T(2), T(0), 0, STRETCH, ec};
  } else if (a.mode == 1) {
    c.k = Coef<T>{T(1), T(0), T(0), 1, STRETCH, ec};
    c.tau = 0.0;   // S is not an iterate: no truncation
  } else {
    c.k = Coef<T>{T(-2), T(0), T(3), 2, STRETCH, ec};
    c.blk = nullptr;   // the block norms came from the square
  }
  // operands: X~ X~ for a square, X~ S for McWeeny's second product
  c.B = (a.mode == 2) ? static_cast<const T*>(in.S) : c.X;
  c.Bh = (a.mode == 2) ? static_cast<const __bf16*>(in.SH) : c.Xh;
  c.Bl = (a.mode == 2) ? static_cast<const __bf16*>(in.SL) : c.Xl;
  if (a.mode == 2) c.Sr = static_cast<const T*>(in.S);
  // output: S for McWeeny's square, the next iterate otherwise
  c.Y = (a.mode == 1) ? static_cast<T*>(in.S) : static_cast<T*>(in.X[a.iter & 1]);
  c.Yh = (a.mode == 1) ? static_cast<__bf16*>(in.SH)
                       : static_cast<__bf16*>(in.XH[a.iter & 1]);
  c.Yl = (a.mode == 1) ? static_cast<__bf16*>(in.SL)
                       : static_cast<__bf16*>(in.XL[a.iter & 1]);
  return c;
}

// ============================================================== FP64
// v_mfma_f64_16x16x4_f64: lane l supplies A[row = l % 16][kk = l / 16] and
// B[kk = l / 16][col = l % 16]; accumulator register j of lane l holds row
// l / 16 + 4 j, column l % 16 (checked with an on-device layout probe).
template <int BM_, int WM_, int WN_, int BK_>
struct CfgF64 {
  using T = double;
  static constexpr int BM = BM_, WM = WM_, WN = WN_, BK = BK_;
  static constexpr int THREADS = 64 * WM * WN;
  static constexpr int TM = BM / WM, TN = BM / WN;
  static constexpr int MB = TM / 16, NB = TN / 16;
  static constexpr int KS = BK / 4;     // MFMA substeps per K slice
  static constexpr int LDK = BK + 2;    // LDS row stride (doubles)
  // the main loop's two double-buffered operand arrays and the epilogue's
  // band share one LDS allocation
  static constexpr int MAIN_BYTES = 2 * 2 * BM * LDK * 8;
  static constexpr int EPI_BYTES = TM * (BM + 1) * 8;
  static constexpr int SMEM = MAIN_BYTES > EPI_BYTES ? MAIN_BYTES : EPI_BYTES;
  struct Acc {
    doublex4 c[MB][NB];
  };
};

template <class C>
__device__ __forceinline__ void acc_zero(typename C::Acc& acc) {
#pragma unroll
  for (int m = 0; m < C::MB; ++m)
#pragma unroll
    for (int n = 0; n < C::NB; ++n)
#pragma unroll
      for (int j = 0; j < static_cast<int>(sizeof(acc.c[0][0]) /
                                          sizeof(acc.c[0][0][0]));
           ++j)
        acc.c[m][n][j] = 0;
}

template <class C>
__device__ __forceinline__ void mainloop_f64(const StepCtx<double>& sc,
                                             const WorkItem& w,
                                             typename C::Acc& acc,
                                             char* smem) {
  using T = double;
  T(*As)[C::BM][C::LDK] = reinterpret_cast<T(*)[C::BM][C::LDK]>(smem);
  T(*Bs)[C::BM][C::LDK] = As + 2;
  const int2 tt = sc.tile;
  const int ld = sc.ld;
  const T* X = sc.X;
  const T* Ap = X + static_cast<size_t>(tt.x * C::BM) * ld;
  const T* Bp = sc.B + static_cast<size_t>(tt.y * C::BM) * ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / C::WN) * C::TM, wn = (wave % C::WN) * C::TN;
  const int r = lane & 15, g = lane >> 4;
  using St = Stage<T, C::BM, C::BK, C::THREADS>;
  St st;
  auto sstore = [&](int b) {
#pragma unroll
    for (int q = 0; q < St::NCH; ++q) {
      const int rr = St::row(tid, q), cc = St::col(tid, q);
      *reinterpret_cast<typename St::vec*>(&As[b][rr][cc]) = st.a[q];
      *reinterpret_cast<typename St::vec*>(&Bs[b][rr][cc]) = st.b[q];
    }
  };
  acc_zero<C>(acc);
  st.load(Ap, Bp, ld, w.k0 * C::BK, tid);
  sstore(0);
  __syncthreads();
  for (int kt = w.k0; kt < w.k1; ++kt) {
    const int b = (kt - w.k0) & 1;
    if (kt + 1 < w.k1) st.load(Ap, Bp, ld, (kt + 1) * C::BK, tid);
#pragma unroll
    for (int s2 = 0; s2 < C::KS; s2 += 2) {
      double2 af[C::MB], bf[C::NB];
#pragma unroll
      for (int m = 0; m < C::MB; ++m)
        af[m] = *reinterpret_cast<const double2*>(
            &As[b][wm + m * 16 + r][g * C::KS + s2]);
#pragma unroll
      for (int n = 0; n < C::NB; ++n)
        bf[n] = *reinterpret_cast<const double2*>(
            &Bs[b][wn + n * 16 + r][g * C::KS + s2]);
#pragma unroll
      for (int m = 0; m < C::MB; ++m)
#pragma unroll
        for (int n = 0; n < C::NB; ++n)
          acc.c[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(
              af[m].x, bf[n].x, acc.c[m][n], 0, 0, 0);
#pragma unroll
      for (int m = 0; m < C::MB; ++m)
#pragma unroll
        for (int n = 0; n < C::NB; ++n)
          acc.c[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(
              af[m].y, bf[n].y, acc.c[m][n], 0, 0, 0);
    }
    if (kt + 1 < w.k1) sstore(b ^ 1);
    __syncthreads();
  }
}


// ============================================================== FP32
// v_mfma_f32_32x32x2_f32: lane l supplies A[row = l % 32][kk = l / 32] and
// B[kk = l / 32][col = l % 32]; accumulator register j of lane l holds row
// 8 (j / 4) + 4 (l / 32) + j % 4, column l % 32.
template <int BM_, int WM_, int WN_, int BK_>
struct CfgF32 {
  using T = float;
  static constexpr int BM = BM_, WM = WM_, WN = WN_, BK = BK_;
  static constexpr int THREADS = 64 * WM * WN;
  static constexpr int TM = BM / WM, TN = BM / WN;
  static constexpr int MB = TM / 32, NB = TN / 32;
  static constexpr int KH = BK / 2;     // k values per lane half per slice
  static constexpr int LDK = BK + 4;
  // the main loop's two double-buffered operand arrays and the epilogue's
  // band share one LDS allocation
  static constexpr int MAIN_BYTES = 2 * 2 * BM * LDK * 4;
  static constexpr int EPI_BYTES = TM * (BM + 1) * 4;
  static constexpr int SMEM = MAIN_BYTES > EPI_BYTES ? MAIN_BYTES : EPI_BYTES;
  struct Acc {
    floatx16 c[MB][NB];
  };
};

template <class C>
__device__ __forceinline__ void mainloop_f32(const StepCtx<float>& sc,
                                             const WorkItem& w,
                                             typename C::Acc& acc,
                                             char* smem) {
  using T = float;
  T(*As)[C::BM][C::LDK] = reinterpret_cast<T(*)[C::BM][C::LDK]>(smem);
  T(*Bs)[C::BM][C::LDK] = As + 2;
  const int2 tt = sc.tile;
  const int ld = sc.ld;
  const T* X = sc.X;
  const T* Ap = X + static_cast<size_t>(tt.x * C::BM) * ld;
  const T* Bp = sc.B + static_cast<size_t>(tt.y * C::BM) * ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / C::WN) * C::TM, wn = (wave % C::WN) * C::TN;
  const int r = lane & 31, h = lane >> 5;
  using St = Stage<T, C::BM, C::BK, C::THREADS>;
  St st;
  auto sstore = [&](int b) {
#pragma unroll
    for (int q = 0; q < St::NCH; ++q) {
      const int rr = St::row(tid, q), cc = St::col(tid, q);
      *reinterpret_cast<typename St::vec*>(&As[b][rr][cc]) = st.a[q];
      *reinterpret_cast<typename St::vec*>(&Bs[b][rr][cc]) = st.b[q];
    }
  };
  acc_zero<C>(acc);
  st.load(Ap, Bp, ld, w.k0 * C::BK, tid);
  sstore(0);
  __syncthreads();
  for (int kt = w.k0; kt < w.k1; ++kt) {
    const int b = (kt - w.k0) & 1;
    if (kt + 1 < w.k1) st.load(Ap, Bp, ld, (kt + 1) * C::BK, tid);
#pragma unroll
    for (int s4 = 0; s4 < C::KH; s4 += 4) {
      floatx4 af[C::MB], bf[C::NB];
#pragma unroll
      for (int m = 0; m < C::MB; ++m)
        af[m] = *reinterpret_cast<const floatx4*>(
            &As[b][wm + m * 32 + r][h * C::KH + s4]);
#pragma unroll
      for (int n = 0; n < C::NB; ++n)
        bf[n] = *reinterpret_cast<const floatx4*>(
            &Bs[b][wn + n * 32 + r][h * C::KH + s4]);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int m = 0; m < C::MB; ++m)
#pragma unroll
          for (int n = 0; n < C::NB; ++n)
            acc.c[m][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                af[m][e], bf[n][e], acc.c[m][n], 0, 0, 0);
    }
    if (kt + 1 < w.k1) sstore(b ^ 1);
    __syncthreads();
  }
}

template <class C, int MODE>
__device__ __forceinline__ void epilogue_f32(const StepCtx<float>& sc,
                                             double* part, int slot,
                                             const typename C::Acc& acc) {
  using T = float;
  const int2 tt = sc.tile;
  const T* X = sc.X;
  T* Y = sc.Y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave / C::WN) * C::TM, wn = (wave % C::WN) * C::TN;
  Sums sums;
  // a 32 x 32 fragment is one block of the mixed norm
#pragma unroll
  for (int m = 0; m < C::MB; ++m)
#pragma unroll
    for (int n = 0; n < C::NB; ++n) {
      double bs = 0.0;
#pragma unroll
      for (int j = 0; j < 16; ++j)
        bs += epilogue_at<T, MODE>(
            X, sc.Sr, Y, sc.ld, sc.n, tt.x, tt.y, C::BM,
            wm + m * 32 + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3),
            wn + n * 32 + (lane & 31), acc.c[m][n][j], sc.k, sc.tau, sums);
      if (MODE != 2 && sc.blk) {
        const double t = full_wave_sum(bs);
        const int rb = (tt.x * C::BM + wm) / kMixedBlock + m;
        const int cb = (tt.y * C::BM + wn) / kMixedBlock + n;
        if (lane == 0 && rb <= cb) blk_write(sc.blk, sc.nbk, rb, cb, t);
      }
    }
  store_partials<C::THREADS>(sums, part, slot, MODE);
}

// ============================================================== BF16x3
// v_mfma_f32_32x32x16_bf16: lane l supplies 8 consecutive k of
// A[row = l % 32] and of B[col = l % 32]; the accumulator layout is the FP32
// 32x32 one. Each FP32 element of X is split while it is staged into LDS:
// H = bf16(x), L = bf16(x - H), both rounded to nearest even; the tile
// accumulates H H + H L + L H in FP32 (the L L term is dropped).
template <int BM_, int WM_, int WN_, int BK_>
struct CfgB3 {
  using T = float;
  static constexpr int BM = BM_, WM = WM_, WN = WN_, BK = BK_;
  static constexpr int THREADS = 64 * WM * WN;
  static constexpr int TM = BM / WM, TN = BM / WN;
  static constexpr int MB = TM / 32, NB = TN / 32;
  static constexpr int KH = BK / 2;     // k values per lane half per slice
  static constexpr int LDK = BK + 8;    // LDS row stride (bf16)
  struct Acc {
    floatx16 c[MB][NB];
  };
};

__device__ __forceinline__ void split_bf16(floatx4 x, bf16x4& hi, bf16x4& lo) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const __bf16 hb = static_cast<__bf16>(x[e]);
    hi[e] = hb;
    lo[e] = static_cast<__bf16>(x[e] - static_cast<float>(hb));
  }
}

template <class C>
__device__ __forceinline__ void mainloop_b3(const StepCtx<float>& sc,
                                            const WorkItem& w,
                                            typename C::Acc& acc) {
  using T = float;
  __shared__ __attribute__((aligned(16))) __bf16 AH[2][C::BM][C::LDK];
  __shared__ __attribute__((aligned(16))) __bf16 AL[2][C::BM][C::LDK];
  __shared__ __attribute__((aligned(16))) __bf16 BH[2][C::BM][C::LDK];
  __shared__ __attribute__((aligned(16))) __bf16 BL[2][C::BM][C::LDK];
  const int2 tt = sc.tile;
  const int ld = sc.ld;
  const T* X = sc.X;
  const T* Ap = X + static_cast<size_t>(tt.x * C::BM) * ld;
  const T* Bp = sc.B + static_cast<size_t>(tt.y * C::BM) * ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / C::WN) * C::TM, wn = (wave % C::WN) * C::TN;
  const int r = lane & 31, h = lane >> 5;
  using St = Stage<T, C::BM, C::BK, C::THREADS>;
  St st;
  auto sstore = [&](int b) {
#pragma unroll
    for (int q = 0; q < St::NCH; ++q) {
      const int rr = St::row(tid, q), cc = St::col(tid, q);
      bf16x4 hi, lo;
      split_bf16(st.a[q], hi, lo);
      *reinterpret_cast<bf16x4*>(&AH[b][rr][cc]) = hi;
      *reinterpret_cast<bf16x4*>(&AL[b][rr][cc]) = lo;
      split_bf16(st.b[q], hi, lo);
      *reinterpret_cast<bf16x4*>(&BH[b][rr][cc]) = hi;
      *reinterpret_cast<bf16x4*>(&BL[b][rr][cc]) = lo;
    }
  };
  acc_zero<C>(acc);
  st.load(Ap, Bp, ld, w.k0 * C::BK, tid);
  sstore(0);
  __syncthreads();
  for (int kt = w.k0; kt < w.k1; ++kt) {
    const int b = (kt - w.k0) & 1;
    if (kt + 1 < w.k1) st.load(Ap, Bp, ld, (kt + 1) * C::BK, tid);
#pragma unroll
    for (int s8 = 0; s8 < C::KH; s8 += 8) {
      bf16x8 ah[C::MB], al[C::MB], bh[C::NB], bl[C::NB];
#pragma unroll
      for (int m = 0; m < C::MB; ++m) {
        ah[m] = *reinterpret_cast<const bf16x8*>(
            &AH[b][wm + m * 32 + r][h * C::KH + s8]);
        al[m] = *reinterpret_cast<const bf16x8*>(
            &AL[b][wm + m * 32 + r][h * C::KH + s8]);
      }
#pragma unroll
      for (int n = 0; n < C::NB; ++n) {
        bh[n] = *reinterpret_cast<const bf16x8*>(
            &BH[b][wn + n * 32 + r][h * C::KH + s8]);
        bl[n] = *reinterpret_cast<const bf16x8*>(
            &BL[b][wn + n * 32 + r][h * C::KH + s8]);
      }
#pragma unroll
      for (int m = 0; m < C::MB; ++m)
#pragma unroll
        for (int n = 0; n < C::NB; ++n) {
          acc.c[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              ah[m], bh[n], acc.c[m][n], 0, 0, 0);
          acc.c[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              ah[m], bl[n], acc.c[m][n], 0, 0, 0);
          acc.c[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              al[m], bh[n], acc.c[m][n], 0, 0, 0);
        }
    }
    if (kt + 1 < w.k1) sstore(b ^ 1);
    __syncthreads();
  }
}

// ============================================================== BF16x3, v2
// Same arithmetic as above with an unpadded LDS layout: every 16-byte chunk
// (8 bf16 along k) of a row is stored at chunk position c ^ g(row), where
// g spreads 16 consecutive rows over the 16 distinct 16-byte slots of a
// 256-byte LDS line, so both the fragment reads (16 rows, same chunk) and
// the staging writes (whole rows) are free of bank conflicts. The smaller
// footprint allows K slices of 32 (two MFMA substeps per barrier) with
// double buffering. The epilogue stages the tile through LDS so that both
// the tile and its transpose are written in whole rows.
template <int BM_, int WM_, int WN_, int BK_>
struct CfgB3S {
  using T = float;
  static constexpr int BM = BM_, WM = WM_, WN = WN_, BK = BK_;
  static constexpr int THREADS = 64 * WM * WN;
  static constexpr int TM = BM / WM, TN = BM / WN;
  static constexpr int MB = TM / 32, NB = TN / 32;
  static constexpr int KH = BK / 2;     // k values per lane half per slice
  static constexpr int ARR = BM * BK;   // bf16 per staged array
  static constexpr int MAIN_BYTES = 2 * 4 * ARR * 2;
  static constexpr int EPI_BYTES = TM * (BM + 1) * 4;
  static constexpr int SMEM = MAIN_BYTES > EPI_BYTES ? MAIN_BYTES : EPI_BYTES;
  struct Acc {
    floatx16 c[MB][NB];
  };
};

// Element offset of (row, k) in a swizzled [rows][BK] bf16 array.
template <int BK>
__device__ __forceinline__ int swz_off(int row, int k) {
  constexpr int CH = BK / 8;                                  // chunks per row
  constexpr int SHIFT = BK == 16 ? 3 : (BK == 32 ? 2 : 1);    // log2(128 / BK)
  const int chunk = (k >> 3) ^ ((row >> SHIFT) & (CH - 1));
  return row * BK + (chunk << 3) + (k & 7);
}

template <class C>
__device__ __forceinline__ void mainloop_b3s(const StepCtx<float>& sc,
                                             const WorkItem& w,
                                             typename C::Acc& acc,
                                             char* smem) {
  using T = float;
  __bf16* lds = reinterpret_cast<__bf16*>(smem);
  // array a (0 AH, 1 AL, 2 BH, 3 BL) of buffer b
  auto arr = [&](int b, int a) { return lds + (b * 4 + a) * C::ARR; };
  const int2 tt = sc.tile;
  const int ld = sc.ld;
  const T* X = sc.X;
  const T* Ap = X + static_cast<size_t>(tt.x * C::BM) * ld;
  const T* Bp = sc.B + static_cast<size_t>(tt.y * C::BM) * ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / C::WN) * C::TM, wn = (wave % C::WN) * C::TN;
  const int r = lane & 31, h = lane >> 5;
  using St = Stage<T, C::BM, C::BK, C::THREADS>;
  St st;
  auto sstore = [&](int b) {
#pragma unroll
    for (int q = 0; q < St::NCH; ++q) {
      const int rr = St::row(tid, q), cc = St::col(tid, q);
      const int o = swz_off<C::BK>(rr, cc);
      bf16x4 hi, lo;
      split_bf16(st.a[q], hi, lo);
      *reinterpret_cast<bf16x4*>(arr(b, 0) + o) = hi;
      *reinterpret_cast<bf16x4*>(arr(b, 1) + o) = lo;
      split_bf16(st.b[q], hi, lo);
      *reinterpret_cast<bf16x4*>(arr(b, 2) + o) = hi;
      *reinterpret_cast<bf16x4*>(arr(b, 3) + o) = lo;
    }
  };
  acc_zero<C>(acc);
  st.load(Ap, Bp, ld, w.k0 * C::BK, tid);
  sstore(0);
  __syncthreads();
  for (int kt = w.k0; kt < w.k1; ++kt) {
    const int b = (kt - w.k0) & 1;
    if (kt + 1 < w.k1) st.load(Ap, Bp, ld, (kt + 1) * C::BK, tid);
#pragma unroll
    for (int s8 = 0; s8 < C::KH; s8 += 8) {
      bf16x8 ah[C::MB], al[C::MB], bh[C::NB], bl[C::NB];
#pragma unroll
      for (int m = 0; m < C::MB; ++m) {
        const int o = swz_off<C::BK>(wm + m * 32 + r, h * C::KH + s8);
        ah[m] = *reinterpret_cast<const bf16x8*>(arr(b, 0) + o);
        al[m] = *reinterpret_cast<const bf16x8*>(arr(b, 1) + o);
      }
#pragma unroll
      for (int n = 0; n < C::NB; ++n) {
        const int o = swz_off<C::BK>(wn + n * 32 + r, h * C::KH + s8);
        bh[n] = *reinterpret_cast<const bf16x8*>(arr(b, 2) + o);
        bl[n] = *reinterpret_cast<const bf16x8*>(arr(b, 3) + o);
      }
#pragma unroll
      for (int m = 0; m < C::MB; ++m)
#pragma unroll
        for (int n = 0; n < C::NB; ++n) {
          acc.c[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              ah[m], bh[n], acc.c[m][n], 0, 0, 0);
          acc.c[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              ah[m], bl[n], acc.c[m][n], 0, 0, 0);
          acc.c[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              al[m], bh[n], acc.c[m][n], 0, 0, 0);
        }
    }
    if (kt + 1 < w.k1) sstore(b ^ 1);
    __syncthreads();
  }
}

// Stores the BF16x3 split of x: H = bf16(x), L = bf16(x - H).
__device__ __forceinline__ void store_split(__bf16* Yh, __bf16* Yl, size_t i,
                                            float x) {
  const __bf16 hb = static_cast<__bf16>(x);
  *grw(Yh + i) = hb;
  *grw(Yl + i) = static_cast<__bf16>(x - static_cast<float>(hb));
}

// ============================================================== BF16x3, v3
// Same arithmetic and LDS layout as v2, but the operands arrive already
// split: the affine start and the v2/v3 epilogues store H = bf16(x) and
// L = bf16(x - H) beside the FP32 iterate, so the K loop moves bf16 chunks
// from global memory to LDS with no conversion. Global loads run two K
// slices ahead (two register sets, loop unrolled by two).
template <int BM_, int WM_, int WN_, int BK_>
struct CfgB3P : CfgB3S<BM_, WM_, WN_, BK_> {};

template <class C>
struct SplitStage {
  static constexpr int CPR = C::BK / 8;                  // 16-B chunks per row
  static constexpr int NC = C::BM * CPR / C::THREADS;    // chunks per thread
  static_assert(C::BM * CPR % C::THREADS == 0, "stage size");
  bf16x8 ah[NC], al[NC], bh[NC], bl[NC];
  __device__ __forceinline__ static int row(int tid, int q) {
    return (tid + q * C::THREADS) / CPR;
  }
  __device__ __forceinline__ static int col(int tid, int q) {
    return ((tid + q * C::THREADS) % CPR) * 8;
  }
  __device__ __forceinline__ void load(const __bf16* Ah, const __bf16* Al,
                                       const __bf16* Bh, const __bf16* Bl,
                                       int ld, int k0, int tid) {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const size_t off = static_cast<size_t>(row(tid, q)) * ld + k0 + col(tid, q);
      ah[q] = *gro(reinterpret_cast<const bf16x8*>(Ah + off));
      al[q] = *gro(reinterpret_cast<const bf16x8*>(Al + off));
      bh[q] = *gro(reinterpret_cast<const bf16x8*>(Bh + off));
      bl[q] = *gro(reinterpret_cast<const bf16x8*>(Bl + off));
    }
  }
};

template <class C>
__device__ __forceinline__ void mainloop_b3p(const StepCtx<float>& sc,
                                             const WorkItem& w,
                                             typename C::Acc& acc,
                                             char* smem) {
  __bf16* lds = reinterpret_cast<__bf16*>(smem);
  auto arr = [&](int b, int a) { return lds + (b * 4 + a) * C::ARR; };
  const int2 tt = sc.tile;
  const int ld = sc.ld;
  const size_t ao = static_cast<size_t>(tt.x * C::BM) * ld;
  const size_t bo = static_cast<size_t>(tt.y * C::BM) * ld;
  const __bf16 *Ah = sc.Xh + ao, *Al = sc.Xl + ao;
  const __bf16 *Bh = sc.Bh + bo, *Bl = sc.Bl + bo;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / C::WN) * C::TM, wn = (wave % C::WN) * C::TN;
  const int r = lane & 31, h = lane >> 5;
  using St = SplitStage<C>;
  St s0, s1;
  auto sstore = [&](const St& st, int b) {
#pragma unroll
    for (int q = 0; q < St::NC; ++q) {
      const int o = swz_off<C::BK>(St::row(tid, q), St::col(tid, q));
      *reinterpret_cast<bf16x8*>(arr(b, 0) + o) = st.ah[q];
      *reinterpret_cast<bf16x8*>(arr(b, 1) + o) = st.al[q];
      *reinterpret_cast<bf16x8*>(arr(b, 2) + o) = st.bh[q];
      *reinterpret_cast<bf16x8*>(arr(b, 3) + o) = st.bl[q];
    }
  };
  // fragments of one MFMA k step (8 k per lane) of the slice in buffer b
  struct Frag {
    bf16x8 ah[C::MB], al[C::MB], bh[C::NB], bl[C::NB];
  };
  // Issue order follows the first MFMAs' needs: ah[0] and the bh row of
  // fragments first, so that the first product of a k step waits for two
  // reads instead of the whole A panel; then the rest of ah, bl and al.
  auto fread = [&](Frag& f, int b, int s8) {
    auto oa = [&](int m) { return swz_off<C::BK>(wm + m * 32 + r, h * C::KH + s8); };
    auto ob = [&](int n) { return swz_off<C::BK>(wn + n * 32 + r, h * C::KH + s8); };
    f.ah[0] = *reinterpret_cast<const bf16x8*>(arr(b, 0) + oa(0));
#pragma unroll
    for (int n = 0; n < C::NB; ++n)
      f.bh[n] = *reinterpret_cast<const bf16x8*>(arr(b, 2) + ob(n));
#pragma unroll
    for (int m = 1; m < C::MB; ++m)
      f.ah[m] = *reinterpret_cast<const bf16x8*>(arr(b, 0) + oa(m));
#pragma unroll
    for (int n = 0; n < C::NB; ++n)
      f.bl[n] = *reinterpret_cast<const bf16x8*>(arr(b, 3) + ob(n));
#pragma unroll
    for (int m = 0; m < C::MB; ++m)
      f.al[m] = *reinterpret_cast<const bf16x8*>(arr(b, 1) + oa(m));
  };
  auto mma = [&](const Frag& f) {
#pragma unroll
    for (int m = 0; m < C::MB; ++m)
#pragma unroll
      for (int n = 0; n < C::NB; ++n)
        acc.c[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            f.ah[m], f.bh[n], acc.c[m][n], 0, 0, 0);
#pragma unroll
    for (int m = 0; m < C::MB; ++m)
#pragma unroll
      for (int n = 0; n < C::NB; ++n)
        acc.c[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            f.ah[m], f.bl[n], acc.c[m][n], 0, 0, 0);
#pragma unroll
    for (int m = 0; m < C::MB; ++m)
#pragma unroll
      for (int n = 0; n < C::NB; ++n)
        acc.c[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            f.al[m], f.bh[n], acc.c[m][n], 0, 0, 0);
  };
  acc_zero<C>(acc);
  const int k0 = w.k0, k1 = w.k1;
  // Loads and stores run unconditionally: a slice index past the last one
  // is clamped to it (a harmless re-read whose store lands in a buffer no
  // later slice reads). Branch-free loads let the compiler wait for just the
  // older register set before storing it, not for every load in flight.
  auto kc = [&](int kt) { return min(kt, k1 - 1) * C::BK; };
  // Global loads run AHEAD - 1 slices ahead of their LDS store: two
  // register sets for 8-wave workgroups; one for 16-wave workgroups, whose
  // register budget (four waves per SIMD) has no room for a second and
  // whose extra waves cover the latency instead.
  constexpr int AHEAD = (C::THREADS > 512) ? 2 : 3;
  s0.load(Ah, Al, Bh, Bl, ld, k0 * C::BK, tid);
  sstore(s0, 0);
  // the scheduling fences keep each register set's loads together and in
  // the same order as inside the loop
  __builtin_amdgcn_sched_barrier(0);
  s0.load(Ah, Al, Bh, Bl, ld, kc(k0 + 1), tid);
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (AHEAD == 3) s1.load(Ah, Al, Bh, Bl, ld, kc(k0 + 2), tid);
  __builtin_amdgcn_sched_barrier(0);
  __syncthreads();
  // one K slice: read the fragments of its first k step from buffer b,
  // store slice kt + 1 (held in st) into the other LDS buffer (last read in
  // slice kt - 1, before the barrier that ended it), refill st with slice
  // kt + 3, then issue the MFMAs. The fragment reads go first: the LDS
  // serves them ahead of the stores, so the MFMAs start without waiting for
  // every wave's stores of the next slice.
  auto step = [&](int kt, St& st) {
    const int b = (kt - k0) & 1;
    Frag f;
    fread(f, b, 0);
    __builtin_amdgcn_sched_barrier(0);
    sstore(st, b ^ 1);
    st.load(Ah, Al, Bh, Bl, ld, kc(kt + AHEAD), tid);
    mma(f);
#pragma unroll
    for (int s8 = 8; s8 < C::KH; s8 += 8) {
      Frag g;
      fread(g, b, s8);
      mma(g);
    }
    __syncthreads();
  };
  // pairs of slices, then an odd last one: no branch inside the loop body
  int kt = k0;
  if constexpr (AHEAD == 3) {
    for (; kt + 1 < k1; kt += 2) {
      step(kt, s0);
      step(kt + 1, s1);
    }
    if (kt < k1) step(kt, s0);
  } else {
    for (; kt < k1; ++kt) step(kt, s0);
  }
}

// Tile-relative position of accumulator register j of fragment (m, n) held
// by `lane`: the 16 x 16 FP64 layout, or the 32 x 32 layout of the FP32 and
// BF16 MFMAs.
template <class C>
__device__ __forceinline__ void acc_pos(int m, int n, int j, int lane, int& r,
                                        int& c) {
  const int wave = threadIdx.x >> 6;
  const int wm = (wave / C::WN) * C::TM, wn = (wave % C::WN) * C::TN;
  if (sizeof(typename C::T) == 8) {
    r = wm + m * 16 + (lane >> 4) + 4 * j;
    c = wn + n * 16 + (lane & 15);
  } else {
    r = wm + m * 32 + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
    c = wn + n * 32 + (lane & 31);
  }
}

// Stores the BF16x3 split of four consecutive values (8-byte stores,
// non-temporal: see epilogue_lds).
__device__ __forceinline__ void store_split4(__bf16* Yh, __bf16* Yl, size_t i,
                                             floatx4 x) {
  bf16x4 hi, lo;
  split_bf16(x, hi, lo);
  __builtin_nontemporal_store(hi, grw(reinterpret_cast<bf16x4*>(Yh + i)));
  __builtin_nontemporal_store(lo, grw(reinterpret_cast<bf16x4*>(Yl + i)));
}

// Sum over the 8 lanes of an aligned lane octet (fixed order).
__device__ __forceinline__ double octet_sum(double x) {
  for (int off = 4; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  using type = floatx4;
};
template <>
struct Vec4<double> {
  using type = doublex4;
};

// Epilogue staged through LDS, for the accumulators of any family (FP64
// 16x16 or FP32 32x32 MFMA layout, placed by acc_pos). The tile is
// processed one band of TM rows at a time (the rows of one row of waves):
// the waves of the band write their accumulators to LDS, then every thread
// applies the element epilogue to runs of four consecutive elements of a
// row (vector loads of the old iterate and vector stores of the new one,
// with 8-byte stores of the bf16 split in FP32 runs; whole rows per group
// of threads) and writes runs of four consecutive elements of the
// transposed band, read down the columns of LDS. With a row stride of
// BM + 1 elements the column reads put at most two lanes of a wave on one
// bank and the row reads (lanes four elements apart) four; the epilogue's
// LDS traffic is small beside its stores.
// The old iterate is read and the new one written with non-temporal hints:
// neither is touched again before the next square, and keeping them out of
// L2 leaves it to the operand panels that the other workgroups stream
// (1.3 % faster squares at N = 8192).
template <class C, int MODE>
__device__ __forceinline__ void epilogue_lds(const StepCtx<typename C::T>& sc,
                                             double* part, int slot,
                                             const typename C::Acc& acc,
                                             char* smem) {
  using T = typename C::T;
  using V4 = typename Vec4<T>::type;
  constexpr int BM = C::BM, TM = C::TM, LD = BM + 1;
  constexpr int V = 4;                   // consecutive elements per thread
  constexpr int TPR = BM / V;            // threads per row of the tile
  constexpr int R = C::THREADS / TPR;    // rows of a band one pass covers
  constexpr int NJ = kMixedBlock / R;    // rows of a block row per thread
  constexpr int BPT = kMixedBlock / V;   // threads per row of a block
  static_assert(C::THREADS % TPR == 0 && kMixedBlock % R == 0 &&
                    TM % kMixedBlock == 0 && TPR % BPT == 0 && 64 % BPT == 0,
                "epilogue thread layout");
  __shared__ double bred[R][TM / kMixedBlock][BM / kMixedBlock];
  T* S = reinterpret_cast<T*>(smem);
  const int2 tt = sc.tile;
  const int I = tt.x, J = tt.y;
  const bool diag = (I == J);
  const int ld = sc.ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wg = wave / C::WN;
  const bool split = (sizeof(T) == 4) && (sc.Yh != nullptr);
  Sums sums;
  // Thread tid owns columns c0 .. c0 + 3 (c0 = 4 (tid % TPR)) of the rows
  // ph + R j of a band (ph = tid / TPR). Rows are visited one 32-row block at
  // a time so that the block sums of the mixed norm are complete after each
  // block row. The old iterate's (and in mode 2 the square's) values are
  // loaded in batches of NB rows, each batch while the previous one is
  // processed, and a band's first batch before its accumulators go to LDS.
  const int c0 = (tid % TPR) * V, ph = tid / TPR;
  const int gc0 = J * BM + c0;
  // rows per load batch: all of a block row's (two in the McWeeny product
  // mode), halved where a band would otherwise hold an odd number of
  // batches (the loop below processes them in pairs)
  constexpr int NB0 = (MODE == 2) ? (NJ < 2 ? NJ : 2) : NJ;
  constexpr int NB = ((TM / kMixedBlock) * (NJ / NB0)) % 2 == 0 || NB0 < 2
                         ? NB0 : NB0 / 2;
  constexpr int PER_RB = NJ / NB;
  constexpr int NBATCH = (TM / kMixedBlock) * PER_RB;
  static_assert(NJ % NB == 0 && NBATCH % 2 == 0, "load batches");
  V4 xa[NB], sa[NB], xb[NB], sb[NB];
  // in a diagonal tile, rows whose four elements all lie below the diagonal
  // are neither loaded nor processed
  auto load_batch = [&](int r0, int bi, V4* xv, V4* sv) {
    const int rb = bi / PER_RB, j0 = (bi % PER_RB) * NB;
#pragma unroll
    for (int jj = 0; jj < NB; ++jj) {
      const int gr = r0 + rb * kMixedBlock + ph + R * (j0 + jj);
      const size_t idx = static_cast<size_t>(gr) * ld + gc0;
      const bool any = !(diag && gr > gc0 + V - 1);
      const V4 z = {T(0), T(0), T(0), T(0)};
      xv[jj] = any ? __builtin_nontemporal_load(
                         gro(reinterpret_cast<const V4*>(sc.X + idx)))
                   : z;
      sv[jj] = (MODE == 2 && any)
                   ? __builtin_nontemporal_load(
                         gro(reinterpret_cast<const V4*>(sc.Sr + idx)))
                   : z;
    }
  };
  double bs = 0.0;
  auto process = [&](int r0, int bi, const V4* xv, const V4* sv) {
    const int rb = bi / PER_RB, j0 = (bi % PER_RB) * NB;
#pragma unroll
    for (int jj = 0; jj < NB; ++jj) {
      const int rr = rb * kMixedBlock + ph + R * (j0 + jj);
      const int gr = r0 + rr;
      const size_t idx = static_cast<size_t>(gr) * ld + gc0;
      if (diag && gr > gc0 + V - 1) continue;
      V4 xn4;
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const int gc = gc0 + i;
        xn4[i] = T(0);
        if (!(diag && gr > gc)) {
          const bool on = (gr == gc);
          double d2;
          const T xn = epilogue_elem<T, MODE>(
              S[rr * LD + c0 + i], xv[jj][i], sv[jj][i], sc.k, sc.tau,
              on ? 1.0 : 2.0, on && gr < sc.n, sums, d2);
          xn4[i] = xn;
          S[rr * LD + c0 + i] = xn;
          bs += block_share(gr, gc, d2);
        }
      }
      if (!diag || gr <= gc0) {   // all four elements are processed
        __builtin_nontemporal_store(xn4, grw(reinterpret_cast<V4*>(sc.Y + idx)));
        if constexpr (sizeof(T) == 4)
          if (split) store_split4(sc.Yh, sc.Yl, idx, xn4);
      } else {                    // the run crosses the diagonal
#pragma unroll
        for (int i = 0; i < V; ++i)
          if (gr <= gc0 + i) {
            *grw(sc.Y + idx + i) = xn4[i];
            if constexpr (sizeof(T) == 4)
              if (split) store_split(sc.Yh, sc.Yl, idx + i, xn4[i]);
          }
      }
    }
    if ((bi + 1) % PER_RB == 0) {   // the block row is complete
      if (sc.blk) {
        // the 8 lanes of an aligned octet hold the 32 columns of one block
        const double t = octet_sum(bs);
        if ((lane & (BPT - 1)) == 0) bred[ph][rb][c0 / kMixedBlock] = t;
      }
      bs = 0.0;
    }
  };
  // transposed band: thread tid writes rows r4 .. r4 + 3 of the band (as
  // four consecutive columns) into row oc of the transpose
  constexpr int TPO = TM / V;             // threads per transposed row
  constexpr int OPP = C::THREADS / TPO;   // transposed rows per pass
  static_assert(C::THREADS % TPO == 0 && BM % OPP == 0, "mirror layout");
  const int r4 = (tid % TPO) * V;
  for (int g = 0; g < C::WM; ++g) {
    const int r0 = I * BM + g * TM;
    load_batch(r0, 0, xa, sa);
    __syncthreads();
    if (wg == g) {
      constexpr int PER = sizeof(acc.c[0][0]) / sizeof(T);
#pragma unroll
      for (int m = 0; m < C::MB; ++m)
#pragma unroll
        for (int n = 0; n < C::NB; ++n)
#pragma unroll
          for (int j = 0; j < PER; ++j) {
            int rr, cc;
            acc_pos<C>(m, n, j, lane, rr, cc);
            S[(rr - g * TM) * LD + cc] = acc.c[m][n][j];
          }
    }
    __syncthreads();
    for (int bi = 0; bi < NBATCH; bi += 2) {
      load_batch(r0, bi + 1, xb, sb);
      process(r0, bi, xa, sa);
      if (bi + 2 < NBATCH) load_batch(r0, bi + 2, xa, sa);
      process(r0, bi + 1, xb, sb);
    }
    __syncthreads();
    if (sc.blk && tid < (TM / kMixedBlock) * (BM / kMixedBlock)) {
      const int rb = tid / (BM / kMixedBlock), cb = tid % (BM / kMixedBlock);
      double t = 0.0;
      for (int q = 0; q < R; ++q) t += bred[q][rb][cb];
      const int grb = r0 / kMixedBlock + rb, gcb = J * BM / kMixedBlock + cb;
      if (grb <= gcb) blk_write(sc.blk, sc.nbk, grb, gcb, t);
    }
    const int gr0 = r0 + r4;
    for (int oc = tid / TPO; oc < BM; oc += OPP) {
      const int gc = J * BM + oc;
      if (diag && gr0 >= gc) continue;   // all four on or below the diagonal
      V4 v;
#pragma unroll
      for (int i = 0; i < V; ++i) v[i] = S[(r4 + i) * LD + oc];
      const size_t idt = static_cast<size_t>(gc) * ld + gr0;
      if (!diag || gr0 + V - 1 < gc) {
        if (sc.mirror32)
          __builtin_nontemporal_store(v, grw(reinterpret_cast<V4*>(sc.Y + idt)));
        if constexpr (sizeof(T) == 4)
          if (split) store_split4(sc.Yh, sc.Yl, idt, v);
      } else {
#pragma unroll
        for (int i = 0; i < V; ++i)
          if (gr0 + i < gc) {
            if (sc.mirror32) *grw(sc.Y + idt + i) = v[i];
            if constexpr (sizeof(T) == 4)
              if (split) store_split(sc.Yh, sc.Yl, idt + i, v[i]);
          }
      }
    }
  }
  store_partials<C::THREADS>(sums, part, slot, MODE);
}

// ============================================================== drivers
// A K-range piece of a tail tile is stored row-major (BM x BM), so that the
// tail reduction can work on bands of rows; a register index is a row
// segment of 16 or 32 consecutive values across the lanes (coalesced).
template <class C>
__device__ __forceinline__ void ws_store(const typename C::Acc& acc,
                                         typename C::T* ws) {
  const int lane = threadIdx.x & 63;
  constexpr int PER = sizeof(acc.c[0][0]) / sizeof(typename C::T);
#pragma unroll
  for (int m = 0; m < C::MB; ++m)
#pragma unroll
    for (int n = 0; n < C::NB; ++n)
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        int r, c;
        acc_pos<C>(m, n, j, lane, r, c);
        *grw(ws + static_cast<size_t>(r) * C::BM + c) = acc.c[m][n][j];
      }
}

template <class C>
struct Ops;

template <int A, int B, int Cc, int D>
struct Ops<CfgF64<A, B, Cc, D>> {
  using C = CfgF64<A, B, Cc, D>;
  static constexpr int kSmem = C::SMEM;
  using T = typename C::T;
  __device__ static void main(const StepCtx<T>& sc, const WorkItem& w,
                              typename C::Acc& acc, char* smem) {
    mainloop_f64<C>(sc, w, acc, smem);
  }
  template <int MODE>
  __device__ static void epi(const StepCtx<T>& sc, double* part, int slot,
                             const typename C::Acc& acc, char* smem) {
    epilogue_lds<C, MODE>(sc, part, slot, acc, smem);
  }
};

template <int A, int B, int Cc, int D>
struct Ops<CfgF32<A, B, Cc, D>> {
  using C = CfgF32<A, B, Cc, D>;
  static constexpr int kSmem = C::SMEM;
  using T = typename C::T;
  __device__ static void main(const StepCtx<T>& sc, const WorkItem& w,
                              typename C::Acc& acc, char* smem) {
    mainloop_f32<C>(sc, w, acc, smem);
  }
  template <int MODE>
  __device__ static void epi(const StepCtx<T>& sc, double* part, int slot,
                             const typename C::Acc& acc, char* smem) {
    epilogue_lds<C, MODE>(sc, part, slot, acc, smem);
  }
};

template <int A, int B, int Cc, int D>
struct Ops<CfgB3<A, B, Cc, D>> {
  using C = CfgB3<A, B, Cc, D>;
  static constexpr int kSmem = 16;
  using T = typename C::T;
  __device__ static void main(const StepCtx<T>& sc, const WorkItem& w,
                              typename C::Acc& acc, char*) {
    mainloop_b3<C>(sc, w, acc);
  }
  // The BF16x3 accumulators have the FP32 32x32 layout.
  template <int MODE>
  __device__ static void epi(const StepCtx<T>& sc, double* part, int slot,
                             const typename C::Acc& acc, char*) {
    epilogue_f32<C, MODE>(sc, part, slot, acc);
  }
};

template <int A, int B, int Cc, int D>
struct Ops<CfgB3S<A, B, Cc, D>> {
  using C = CfgB3S<A, B, Cc, D>;
  using T = typename C::T;
  static constexpr int kSmem = C::SMEM;
  __device__ static void main(const StepCtx<T>& sc, const WorkItem& w,
                              typename C::Acc& acc, char* smem) {
    mainloop_b3s<C>(sc, w, acc, smem);
  }
  template <int MODE>
  __device__ static void epi(const StepCtx<T>& sc, double* part, int slot,
                             const typename C::Acc& acc, char* smem) {
    epilogue_lds<C, MODE>(sc, part, slot, acc, smem);
  }
};

template <int A, int B, int Cc, int D>
struct Ops<CfgB3P<A, B, Cc, D>> {
  using C = CfgB3P<A, B, Cc, D>;
  using T = typename C::T;
  static constexpr int kSmem = C::SMEM;
  __device__ static void main(const StepCtx<T>& sc, const WorkItem& w,
                              typename C::Acc& acc, char* smem) {
    mainloop_b3p<C>(sc, w, acc, smem);
  }
  template <int MODE>
  __device__ static void epi(const StepCtx<T>& sc, double* part, int slot,
                             const typename C::Acc& acc, char* smem) {
    epilogue_lds<C, MODE>(sc, part, slot, acc, smem);
  }
};

// Waves per SIMD a configuration is compiled for (the register budget
// follows from it; HIP's second launch bound): 4 for the 128-tile FP64
// configuration with 2 x 4 waves, i.e. two workgroups per CU, whose LDS (two
// operand buffers of 36 KiB) leaves room for a second workgroup to run while
// the first waits at a slice barrier; 1 (no constraint) for the others.
template <class C>
struct MinWaves {
  static constexpr int value = 1;
};
template <>
struct MinWaves<CfgF64<128, 2, 4, 16>> {
  static constexpr int value = 4;
};

template <class C, int MODE, bool STRETCH>
__global__ __launch_bounds__(C::THREADS, MinWaves<C>::value) void square_kernel(
    SquareArgs a) {
  __shared__ __attribute__((aligned(16))) char smem[Ops<C>::kSmem];
  const WorkItem w = a.items[blockIdx.x];
  if (w.slot < 0) return;
  const Instance& in = a.inst[w.inst];
  if (in.st->done) return;
  using T = typename C::T;
  const StepCtx<T> sc = step_ctx<T, STRETCH>(a, in, w.slot);
  typename C::Acc acc;
  Ops<C>::main(sc, w, acc, smem);
  if (w.piece < 0) {
    Ops<C>::template epi<MODE>(sc, a.part, w.slot, acc, smem);
  } else {
    ws_store<C>(acc, static_cast<T*>(a.ws) +
                         static_cast<size_t>(w.piece) * C::BM * C::BM);
  }
}

// Tail reduction, one workgroup per band of 32 rows (one block row of the
// mixed norm) of a tail tile: sums the tile's K pieces in piece order, applies
// the element epilogue to the band, writes the band and (through LDS, as
// 32-element row segments) its mirror, and the band's partial sums. The last
// band of a tile to finish (agent-scope counter) adds the bands' partials in
// band order into the tile's slot and resets the counter: deterministic.
template <class C, int MODE, bool STRETCH>
__global__ __launch_bounds__(C::THREADS) void square_tail_kernel(SquareArgs a) {
  using T = typename C::T;
  constexpr int BM = C::BM, NBAND = BM / kMixedBlock, R = C::THREADS / BM;
  static_assert(C::THREADS % BM == 0 && kMixedBlock % R == 0 && BM % 64 == 0,
                "tail band layout");
  __shared__ T band[kMixedBlock][BM + 1];
  __shared__ double bred[R][BM / kMixedBlock];
  __shared__ double sh[C::THREADS / 64][3];
  __shared__ int is_last;
  const int ti = blockIdx.x / NBAND, q = blockIdx.x % NBAND;
  const TailItem t = a.tails[ti];
  const Instance& in = a.inst[t.inst];
  if (in.st->done) return;
  const StepCtx<T> sc = step_ctx<T, STRETCH>(a, in, t.slot);
  const int I = sc.tile.x, J = sc.tile.y;
  const bool diag = (I == J);
  const int ld = sc.ld;
  const bool split = (sc.Yh != nullptr);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cc = tid % BM, ph = tid / BM;
  const int r0 = q * kMixedBlock;            // first tile row of the band
  const int gc = J * BM + cc;
  const T* ws = static_cast<const T*>(a.ws) +
                static_cast<size_t>(t.piece0) * BM * BM;
  // Sum of the pieces for the thread's rows ph + R jj of the band, in piece
  // order; four pieces of all rows are loaded at a time so that many
  // independent loads are in flight.
  constexpr int NR = kMixedBlock / R;
  T rows[NR];
#pragma unroll
  for (int jj = 0; jj < NR; ++jj) rows[jj] = T(0);
  const T* src = ws + static_cast<size_t>(r0 + ph) * BM + cc;
  for (int p0 = 0; p0 < a.split; p0 += 4) {
    T v[4][NR];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int jj = 0; jj < NR; ++jj)
        v[p][jj] = (p0 + p < a.split)
                       ? *gro(src + static_cast<size_t>(p0 + p) * BM * BM +
                              static_cast<size_t>(R * jj) * BM)
                       : T(0);
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int jj = 0; jj < NR; ++jj)
        if (p0 + p < a.split) rows[jj] += v[p][jj];
  }
  Sums sums;
  double bs = 0.0;
#pragma unroll
  for (int jj = 0; jj < NR; ++jj) {
    const int rr = ph + R * jj, lr = r0 + rr;
    const int gr = I * BM + lr;
    const T sv_acc = rows[jj];
    T xn = T(0);
    if (!(diag && gr > gc)) {
      const size_t idx = static_cast<size_t>(gr) * ld + gc;
      const bool on = (gr == gc);
      const T sv = (MODE == 2) ? *gro(sc.Sr + idx) : T(0);
      double d2;
      xn = epilogue_elem<T, MODE>(sv_acc, *gro(sc.X + idx), sv, sc.k, sc.tau,
                                  on ? 1.0 : 2.0, on && gr < sc.n, sums, d2);
      *grw(sc.Y + idx) = xn;
      if (split) store_split(sc.Yh, sc.Yl, idx, xn);
      bs += block_share(gr, gc, d2);
    }
    band[rr][cc] = xn;
  }
  if (MODE != 2 && sc.blk) {
    bs = half_wave_sum(bs);
    if ((lane & 31) == 0) bred[ph][cc / kMixedBlock] = bs;
  }
  __syncthreads();
  if (MODE != 2 && sc.blk && tid < BM / kMixedBlock) {
    double tb = 0.0;
    for (int p = 0; p < R; ++p) tb += bred[p][tid];
    const int grb = (I * BM + r0) / kMixedBlock, gcb = J * BM / kMixedBlock + tid;
    if (grb <= gcb) blk_write(sc.blk, sc.nbk, grb, gcb, tb);
  }
  // mirror: element (c, rr) of the transpose, 32 consecutive rows of the
  // band per column
  for (int e = tid; e < kMixedBlock * BM; e += C::THREADS) {
    const int c = e / kMixedBlock, rr = e % kMixedBlock;
    const int gr = I * BM + r0 + rr, gcc = J * BM + c;
    if (diag && gr >= gcc) continue;
    const size_t idt = static_cast<size_t>(gcc) * ld + gr;
    const T xn = band[rr][c];
    if (sc.mirror32) *grw(sc.Y + idt) = xn;
    if (split) store_split(sc.Yh, sc.Yl, idt, xn);
  }
  // partial sums of the band, then of the tile
  sums.v = wave_sum(sums.v);
  sums.t1 = wave_sum(sums.t1);
  sums.t2 = wave_sum(sums.t2);
  if (lane == 0) {
    sh[wave][0] = sums.v;
    sh[wave][1] = sums.t1;
    sh[wave][2] = sums.t2;
  }
  __syncthreads();
  if (tid == 0) {
    double v = sh[0][0], t1 = sh[0][1], t2 = sh[0][2];
    for (int w = 1; w < C::THREADS / 64; ++w) {
      v += sh[w][0];
      t1 += sh[w][1];
      t2 += sh[w][2];
    }
    double* bp = a.bpart + 3 * (static_cast<size_t>(ti) * NBAND + q);
    bp[0] = v;
    bp[1] = t1;
    bp[2] = t2;
    const int before = __hip_atomic_fetch_add(a.bcnt + ti, 1, __ATOMIC_ACQ_REL,
                                              __HIP_MEMORY_SCOPE_AGENT);
    is_last = (before == NBAND - 1);
  }
  __syncthreads();
  if (tid == 0 && is_last) {
    double v = 0.0, t1 = 0.0, t2 = 0.0;
    const double* bp = a.bpart + 3 * static_cast<size_t>(ti) * NBAND;
    for (int b = 0; b < NBAND; ++b) {
      v += bp[3 * b + 0];
      t1 += bp[3 * b + 1];
      t2 += bp[3 * b + 2];
    }
    if (MODE != 2) a.part[3 * t.slot + 0] = v;
    if (MODE != 1) {
      a.part[3 * t.slot + 1] = t1;
      a.part[3 * t.slot + 2] = t2;
    }
    a.bcnt[ti] = 0;
  }
}

// Kernel configurations: macro tile, waves (M x N), K slice.
using F64_128_2x4 = CfgF64<128, 2, 4, 16>;
using F64_128_2x2 = CfgF64<128, 2, 2, 16>;
using F64_64_2x2 = CfgF64<64, 2, 2, 16>;
using F32_128_2x2 = CfgF32<128, 2, 2, 32>;
using F32_128_2x4 = CfgF32<128, 2, 4, 32>;
using F32_256_2x2 = CfgF32<256, 2, 2, 16>;
using F32_256_2x4 = CfgF32<256, 2, 4, 32>;
using B3_128_2x2 = CfgB3<128, 2, 2, 32>;
using B3_256_2x2 = CfgB3<256, 2, 2, 16>;
using B3_256_2x4 = CfgB3<256, 2, 4, 16>;
using B3S_256_2x4 = CfgB3S<256, 2, 4, 32>;
using B3S_256_2x4_16 = CfgB3S<256, 2, 4, 16>;
using B3S_128_2x2 = CfgB3S<128, 2, 2, 32>;
using B3P_256_2x4 = CfgB3P<256, 2, 4, 16>;
using B3P_256_2x4_32 = CfgB3P<256, 2, 4, 32>;
using B3P_128_2x2 = CfgB3P<128, 2, 2, 32>;
using B3P_256_4x4_32 = CfgB3P<256, 4, 4, 32>;

template <class C, int MODE, bool STRETCH>
hipError_t launch_mode(const SquareArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((square_kernel<C, MODE, STRETCH>), dim3(grid),
                     dim3(C::THREADS), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.ntail == 0) return e;
  hipLaunchKernelGGL((square_tail_kernel<C, MODE, STRETCH>),
                     dim3(a.ntail * (C::BM / kMixedBlock)), dim3(C::THREADS), 0,
                     s, a);
  return hipGetLastError();
}

// The step's mode and whether the run stretches are template parameters of
// the kernels, so that the SP2 step carries no code of the McWeeny products
// and Alg. 2 none of the stretch.
template <class C>
hipError_t launch_cfg(const SquareArgs& a, int grid, hipStream_t s) {
  const int sel = a.mode + (a.stretch ? 3 : 0);
  switch (sel) {
    case 0: return launch_mode<C, 0, false>(a, grid, s);
    case 1: return launch_mode<C, 1, false>(a, grid, s);
    case 2: return launch_mode<C, 2, false>(a, grid, s);
    case 3: return launch_mode<C, 0, true>(a, grid, s);
    case 4: return launch_mode<C, 1, true>(a, grid, s);
    case 5: return launch_mode<C, 2, true>(a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

// ============================================================== persistent
// One launch for a whole batch run (see PQueue). Each workgroup loops: take
// the next queue index, wait for its item, compute the whole tile (the same
// main loop and epilogue as square_kernel), release its stores and count it;
// the workgroup that counts an instance's last tile of the step acquires
// the other tiles' partial sums, runs the instance's scalar step
// (finalize_scalar, with the partials summed in the finalize kernel's order,
// so both drivers take the same decisions from the same values) and, unless
// the instance stopped, publishes the tiles of its next step. Every wait is
// bounded: a workgroup gives up (and raises the error flag) once the next
// item has not appeared within q.wait_limit ticks of the constant clock, and
// every workgroup returns once every instance has an outcome. Items are
// published only by workgroups that hold no item, so the queue drains.

// Threads that sum an instance's partials (the finalize kernel's width).
constexpr int kPersistSumThreads = 256;

// Thread 0: takes the next index and waits for its item. false: no more
// work (every instance has an outcome, or a wait exceeded its limit).
__device__ __attribute__((noinline)) bool take_item(const PQueue& q, PItem* out) {
  const int idx = __hip_atomic_fetch_add(q.ctl + 0, 1, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
  const long long t0 = wall_clock64();
  for (;;) {
    if (idx < q.cap) {
      PItem* p = q.items + idx;
      if (__hip_atomic_load(&p->seq, __ATOMIC_ACQUIRE,
                            __HIP_MEMORY_SCOPE_AGENT) == idx + 1) {
        out->inst = p->inst;
        out->slot = p->slot;
        out->iter = p->iter;
        out->seq = idx + 1;
        return true;
      }
    }
    if (__hip_atomic_load(q.ndone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
            q.count ||
        __hip_atomic_load(q.ctl + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
      return false;
    if (wall_clock64() - t0 > q.wait_limit) {
      __hip_atomic_store(q.ctl + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Sums of an instance's partial triples in the finalize kernel's order:
// kPersistSumThreads threads stride over the tiles, each wave sums its
// lanes, thread 0 adds the waves in order (waves past the finalize kernel's
// width contribute zeros). The result is valid on thread 0.
template <int THREADS>
__device__ __forceinline__ void persist_sums(const double* pp, int cnt,
                                             double& a, double& b, double& c,
                                             double (*sh)[3]) {
  a = b = c = 0.0;
  if (threadIdx.x < kPersistSumThreads)
    for (int i = threadIdx.x; i < cnt; i += kPersistSumThreads) {
      a += pp[3 * i + 0];
      b += pp[3 * i + 1];
      c += pp[3 * i + 2];
    }
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
    for (int w = 1; w < THREADS / 64; ++w) {
      a += sh[w][0];
      b += sh[w][1];
      c += sh[w][2];
    }
  }
}

// The scalar step of an instance, called (not inlined) from the persistent
// kernel: it runs once per step of an instance, and its registers must not
// count against the tile loop's.
__device__ __attribute__((noinline)) bool persist_finalize(
    const Instance& in, int iter, double a, double b, double c, int32_t* ndone,
    int count, HostMirror* mirror) {
  return finalize_scalar(in, iter, a, b, c, 0.0, 0, ndone, count, mirror);
}

// Publishes the ntiles tiles of step `iter` of instance `inst` from index
// base on (all threads of the workgroup).
template <int THREADS>
__device__ __forceinline__ void persist_publish(const PQueue& q, int base,
                                                int inst, int tile0,
                                                int ntiles, int iter) {
  for (int t = threadIdx.x; t < ntiles; t += THREADS) {
    PItem* p = q.items + base + t;
    p->inst = inst;
    p->slot = tile0 + t;
    p->iter = iter;
    __hip_atomic_store(&p->seq, base + t + 1, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Waves per SIMD the persistent kernel is compiled for: two workgroups per
// CU, as the square kernels of these configurations run (the queue and the
// scalar step must not take the registers that let a second workgroup run
// while the first waits at a slice barrier).
template <class C>
struct PersistWaves {
  static constexpr int value = 2 * C::THREADS / 256;
};

template <class C, bool STRETCH>
__global__ __launch_bounds__(C::THREADS, PersistWaves<C>::value) void persist_kernel(
    SquareArgs a, PQueue q) {
  __shared__ __attribute__((aligned(16))) char smem[Ops<C>::kSmem];
  __shared__ PItem cur;
  __shared__ int flag, base_sh;
  __shared__ double sh[C::THREADS / 64][3];
  using T = typename C::T;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) flag = take_item(q, &cur) ? 1 : 0;
    __syncthreads();
    if (!flag) return;
    // the item's inputs were released by the workgroups that wrote them;
    // thread 0's acquire (the load that found the item published) invalidates
    // the CU's caches for every wave of the workgroup, which waits for it at
    // the barrier above
    const PItem it = cur;
    const Instance& in = a.inst[it.inst];
    SquareArgs aa = a;
    aa.iter = it.iter;
    const StepCtx<T> sc = step_ctx<T, STRETCH>(aa, in, it.slot);
    const int np = (in.n + C::BM - 1) / C::BM * C::BM;
    const WorkItem w{it.inst, it.slot, -1, 0, np / C::BK, 0};
    typename C::Acc acc;
    Ops<C>::main(sc, w, acc, smem);
    Ops<C>::template epi<0>(sc, a.part, it.slot, acc, smem);
    // every wave's stores of the tile and its partials have completed at the
    // barrier; thread 0's release (the count) makes them visible to the
    // device
    __syncthreads();
    if (tid == 0) {
      const int before = __hip_atomic_fetch_add(
          q.cnt + it.inst, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      flag = (before == in.ntiles - 1) ? 1 : 0;
    }
    __syncthreads();
    if (flag) {
      // the instance's step is complete (thread 0's count acquired the other
      // tiles' partials): its scalar step, here
      double pa, pb, pc;
      persist_sums<C::THREADS>(a.part + 3 * in.tile0, in.ntiles, pa, pb, pc, sh);
      if (tid == 0) {
        int base = -1;
        if (!persist_finalize(in, it.iter, pa, pb, pc, q.ndone, q.count,
                              q.mirror)) {
          __hip_atomic_store(q.cnt + it.inst, 0, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
          base = __hip_atomic_fetch_add(q.ctl + 1, in.ntiles, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
          if (base + in.ntiles > q.cap) {   // cannot happen: cap covers max_iter
            __hip_atomic_store(q.ctl + 2, 2, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            base = -1;
          }
        }
        base_sh = base;
      }
      __syncthreads();
      if (base_sh >= 0)
        persist_publish<C::THREADS>(q, base_sh, it.inst, in.tile0, in.ntiles,
                                    it.iter + 1);
    }
    __syncthreads();
  }
}

template <class C>
int persist_grid_cfg(bool stretch, int num_cus) {
  int per = 0;
  const void* fn =
      stretch ? reinterpret_cast<const void*>(&persist_kernel<C, true>)
              : reinterpret_cast<const void*>(&persist_kernel<C, false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, C::THREADS, 0) !=
          hipSuccess ||
      per < 1)
    return 0;
  return per * num_cus;
}

template <class C>
hipError_t launch_persist_cfg(const SquareArgs& a, const PQueue& q, int grid,
                              hipStream_t s) {
  if (a.stretch)
    hipLaunchKernelGGL((persist_kernel<C, true>), dim3(grid), dim3(C::THREADS),
                       0, s, a, q);
  else
    hipLaunchKernelGGL((persist_kernel<C, false>), dim3(grid), dim3(C::THREADS),
                       0, s, a, q);
  return hipGetLastError();
}

}  // namespace
}  // namespace sp2
