// Spectral norm of E = X~ - X~^2, the error e_i of Alg. 2 (sec. 2), for
// every running instance of a batch (dense) or of a block-sparse run, by
// Lanczos in FP64.
//
// E is applied through two products with the stored iterate,
// E q = X~ q - X~ (X~ q), so E itself is never formed and the estimate is the
// norm of the idempotency error of the iterate as stored, evaluated in FP64
// whatever the working precision of the squares. E is symmetric but not
// semidefinite (eigenvalues of X~ outside [0, 1] give negative eigenvalues
// of E), so the estimate is the larger magnitude of the two end Ritz values.
//
// The three-term Lanczos recurrence without reorthogonalisation: loss of
// orthogonality only repeats Ritz values that have converged, and the end
// Ritz values stay inside the spectrum, so the estimate of an extreme
// eigenvalue is unaffected. Step j (q_{-1} = 0, alpha_{-1} = 0, w_{-1} = a
// fixed start vector):
//   u_j = w_{j-1} - alpha_{j-1} q_{j-1},  beta_{j-1} = ||u_j||,
//   q_j = u_j / beta_{j-1},  w_j = E q_j - beta_{j-1} q_{j-1},
//   alpha_j = q_j . w_j.
// The product X~ u_j is formed before beta_{j-1} is known and scaled after
// (it is linear), so a step needs two grid-wide barriers while every
// coefficient is an exact inner product.
//
// One cooperative launch per step runs the Lanczos processes of all
// instances in lockstep: the rows of every instance are cut into chunks of
// kSpecRows rows, each workgroup owns a fixed set of chunks, and the two
// phases of a step are
//   P1  alpha_{j-1} from the partials; u_j for the chunk's rows and its
//       squared norm; y = X~ u_j (u_j formed while it is staged)
//   P2  beta_{j-1}; q_j; w_j = y / beta - X~ (y / beta) - beta q_{j-1} for the
//       chunk's rows; partial q_j . w_j. The designated workgroup of an
//       instance updates its estimate from T_j (alpha_0..alpha_{j-1},
//       beta_0..beta_{j-2}) and decides whether it is final.
// An instance is final when its estimate changes by less than 1e-12
// relative, when beta_{j-1} vanishes (an invariant subspace), or at
// kLanczosMax (or n) steps. Every sum over chunks is taken in one fixed
// order, so every workgroup derives the same scalars and the result does not
// depend on the grid. Workgroup b owns chunks b, b + G, ...; the designated
// workgroup of an instance is a workgroup without chunks when the grid has
// one to spare (so that the small eigenvalue problem runs beside the
// products instead of after them), else the owner of its first chunk.
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
static_assert(kSpecRows % kWaves == 0 && kSpecRows <= 64, "rows per wave");

__device__ __forceinline__ double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
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

// Native vector types (HIP's float4/double2 are classes whose copies go
// through generic references, which would turn the loads below into flat
// loads).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// Raw row segment of 4 entries as loaded (converted to FP64 at use), and
// how many 256-column steps a wave keeps in flight.
template <typename T>
struct Seg;
template <>
struct Seg<float> {
  using V = f32x4;
  static constexpr int kSteps = 4;
};
template <>
struct Seg<double> {
  using V = f64x4;
  static constexpr int kSteps = 2;
};

template <typename V>
__device__ __forceinline__ double dot4(const V& x, const f64x2& a,
                                       const f64x2& b, double acc) {
  acc = fma(static_cast<double>(x.x), a.x, acc);
  acc = fma(static_cast<double>(x.y), a.y, acc);
  acc = fma(static_cast<double>(x.z), b.x, acc);
  acc = fma(static_cast<double>(x.w), b.y, acc);
  return acc;
}

// Loads through pointers cast to the global (1) or LDS (3) address space:
// the pointers here come from tables in memory or pass through structs, and
// generic (flat) loads would share the LDS wait counter, so that every read
// of the staged vector would also wait for the row loads in flight.
template <typename V, typename T>
__device__ __forceinline__ V gload(const T* p) {
  return *(const __attribute__((address_space(1))) V*)(p);
}
__device__ __forceinline__ f64x2 lload(const double* p) {
  return *(const __attribute__((address_space(3))) f64x2*)(p);
}

// Sources of the product's input vector, four entries from column `col`:
// a vector staged in LDS, a vector in global memory, or (w - alpha q) * s
// formed from two global vectors.
struct SrcLds {
  const double* v;
  __device__ __forceinline__ void get(int col, f64x2& a, f64x2& b) const {
    a = lload(v + col);
    b = lload(v + col + 2);
  }
  __device__ __forceinline__ double get1(int col) const {
    return *(const __attribute__((address_space(3))) double*)(v + col);
  }
};
struct SrcPlain {
  const double* v;
  __device__ __forceinline__ void get(int col, f64x2& a, f64x2& b) const {
    a = gload<f64x2>(v + col);
    b = gload<f64x2>(v + col + 2);
  }
  __device__ __forceinline__ double get1(int col) const { return gload<double>(v + col); }
};
struct SrcComb {
  const double* w;
  const double* q;
  double alpha, s;
  __device__ __forceinline__ void get(int col, f64x2& a, f64x2& b) const {
    const f64x2 wa = gload<f64x2>(w + col);
    const f64x2 wb = gload<f64x2>(w + col + 2);
    const f64x2 qa = gload<f64x2>(q + col);
    const f64x2 qb = gload<f64x2>(q + col + 2);
    a = (wa - alpha * qa) * s;
    b = (wb - alpha * qb) * s;
  }
  __device__ __forceinline__ double get1(int col) const {
    return (gload<double>(w + col) - alpha * gload<double>(q + col)) * s;
  }
};

// out[r] = sum_c X[row0 + r][c] v[c] for the kSpecRows rows of one chunk
// (0 for rows >= n), FP64 accumulation in column order. Wave w handles rows
// row0 + w * kRowsPerWave ..; lanes walk the row in groups of 4 columns, so
// a wave reads each row as contiguous 1 KiB (FP32) or 2 KiB (FP64) runs, and
// every lane issues the loads of Seg<T>::kSteps column steps of all its rows
// before it uses any. v is zero past n; the iterate's padding columns are
// zero as well.
template <typename T, typename Src>
__device__ __forceinline__ void chunk_matvec(const T* __restrict__ X, int ld,
                                             int n, int ldq, int row0,
                                             const Src& src, double* out) {
  using V = typename Seg<T>::V;
  constexpr int U = Seg<T>::kSteps;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = row0 + wave * kRowsPerWave;
  const int nr = min(kRowsPerWave, n - r0);   // rows of this wave inside n
  double acc[kRowsPerWave];
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) acc[r] = 0.0;
  if (nr == kRowsPerWave) {
    for (int c0 = lane * 4; c0 < ldq; c0 += 256 * U) {
      V x[U][kRowsPerWave];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int col = c0 + 256 * u;
#pragma unroll
        for (int r = 0; r < kRowsPerWave; ++r)
          x[u][r] = (col < ldq)
                        ? gload<V>(X + static_cast<size_t>(r0 + r) * ld + col)
                        : V{0, 0, 0, 0};
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int col = c0 + 256 * u;
        if (col < ldq) {
          f64x2 va, vb;
          src.get(col, va, vb);
#pragma unroll
          for (int r = 0; r < kRowsPerWave; ++r)
            acc[r] = dot4(x[u][r], va, vb, acc[r]);
        }
      }
    }
  } else if (nr > 0) {
    for (int col = lane * 4; col < ldq; col += 256) {
      f64x2 va, vb;
      src.get(col, va, vb);
      for (int r = 0; r < nr; ++r) {
        const V x = gload<V>(X + static_cast<size_t>(r0 + r) * ld + col);
        acc[r] = dot4(x, va, vb, acc[r]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) {
    const double t = wave_sum(acc[r]);
    if (lane == 0) out[wave * kRowsPerWave + r] = (r < nr) ? t : 0.0;
  }
}

// The same product for a block-sparse instance (the chunk is one block row
// I = row0 / 32 of the iterate in buffer k): out[r] = sum over the flagged
// blocks (I, K) of sum_c X_IK[r][c] v[32 K + c], FP64 accumulation in block
// order. Lane (h, c) takes column c of the rows of its half h; the block
// columns of the row are read once into lanes and broadcast.
template <typename Src>
__device__ __forceinline__ void chunk_matvec_bsr(const Instance& in, int k,
                                                 int row0, const Src& src,
                                                 double* out) {
  static_assert(kSpecRows == kBsrBlock, "one block row per chunk");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 31, h = lane >> 5;
  const int I = row0 / kBsrBlock;
  const int32_t* rp = in.brp[k];
  const int q0 = rp[I], q1 = rp[I + 1];
  double acc[kRowsPerWave];
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) acc[r] = 0.0;
  for (int b0 = q0; b0 < q1; b0 += 64) {
    const int qb = b0 + lane;
    const int kc = (qb < q1 && in.bflag[k][qb] != 0) ? in.bcol[k][qb] : -1;
    const int nb = min(64, q1 - b0);
#pragma unroll 4
    for (int t = 0; t < nb; ++t) {
      const int K = __builtin_amdgcn_readlane(kc, t);
      if (K < 0) continue;
      const double vk = src.get1(K * kBsrBlock + c);
      const float* blk = in.bval[k] + static_cast<size_t>(b0 + t) * kBsrBlock * kBsrBlock;
#pragma unroll
      for (int r = 0; r < kRowsPerWave; r += 2) {
        const int rr = r + h;
        acc[rr] = fma(static_cast<double>(gload<float>(blk + blk_off(wave * kRowsPerWave + rr, c))),
                      vk, acc[rr]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) {
    // rows of the other half contribute zero from this lane
    const double t = wave_sum(((r & 1) == h) ? acc[r] : 0.0);
    if (lane == 0) out[wave * kRowsPerWave + r] = (row0 + wave * kRowsPerWave + r < in.n) ? t : 0.0;
  }
}

// vs[i] = (w[i] - alpha q[i]) * s for i < ldq (q may be null: vs = w * s):
// each thread takes four entries per segment and issues the loads of eight
// segments before it uses any.
template <bool kWithQ>
__device__ __forceinline__ void stage(double* vs, const double* w,
                                      const double* q, double alpha, double s,
                                      int ldq) {
  constexpr int kSeg = 8;
  for (int i0 = threadIdx.x * 4; i0 < ldq; i0 += kThreads * 4 * kSeg) {
    f64x4 wv[kSeg], qv[kSeg];
#pragma unroll
    for (int k = 0; k < kSeg; ++k) {
      const int i = i0 + k * kThreads * 4;
      wv[k] = (i < ldq) ? gload<f64x4>(w + i) : f64x4{0, 0, 0, 0};
      qv[k] = (kWithQ && i < ldq) ? gload<f64x4>(q + i) : f64x4{0, 0, 0, 0};
    }
#pragma unroll
    for (int k = 0; k < kSeg; ++k) {
      const int i = i0 + k * kThreads * 4;
      if (i < ldq)
        *(__attribute__((address_space(3))) f64x4*)(vs + i) =
            (wv[k] - alpha * qv[k]) * s;
    }
  }
}

// Whether the workgroup skips instance `in`: the instance has stopped, or
// its estimate is final. One thread reads the flags and shares them through
// LDS, so the whole workgroup takes the same branch even while another
// workgroup is setting the instance's final flag (phase P1).
__device__ __forceinline__ bool skip_instance(const Instance& in, int* flag) {
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

// Sum over the instance's nch chunks of part[q], in a fixed order, returned
// to every thread.
__device__ __forceinline__ double chunk_sum(const double* part, int nch,
                                           double* red) {
  double s = 0.0;
  for (int q = threadIdx.x; q < nch; q += kThreads) s += part[q];
  return block_sum(s, red);
}

// The designated workgroup's part of P2 for one instance at step j >= 1:
// record alpha_{j-1} and beta_{j-1}, update the estimate from T_j and decide
// whether it is final.
__device__ void decide(const Instance& in, int j, int iter, double alpha,
                       double beta, int32_t* ndone, double* tta, double* ttb,
                       int* hits) {
  const SpecView v = spec_view(in.sp, in.n);
  const double prev = v.misc[0];   // read before thread 0 rewrites it
  // T_j: alpha_0..alpha_{j-1}, beta_0..beta_{j-2}
  __syncthreads();   // tta/ttb may still be read for another instance
  for (int q = threadIdx.x; q < j - 1; q += kThreads) {
    tta[q] = v.ta[q];
    ttb[q] = v.tb[q];
  }
  if (threadIdx.x == 0) {
    tta[j - 1] = alpha;
    ttb[j - 1] = 0.0;
  }
  __syncthreads();
  double bot, top;
  tridiag_ends(tta, ttb, j, hits, &bot, &top);
  const double theta = fmax(fabs(top), fabs(bot));
  const bool fin = !(beta > 1e-14 * theta) || !isfinite(beta) ||
                   (j >= 2 && fabs(theta - prev) <= kSpecTol * theta) ||
                   j == kLanczosMax || j == in.n;
  if (threadIdx.x == 0) {
    v.ta[j - 1] = alpha;
    v.tb[j - 1] = beta;
    if (fin) {
      in.st->m[iter - 1] = theta;
      in.st->krylov[iter - 1] = j;
      __hip_atomic_store(&v.misc[1], 1.0, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(ndone, 1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    } else {
      v.misc[0] = theta;
    }
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kThreads, 2) void spectral_kernel(SpecArgs a) {
  cg::grid_group grid = cg::this_grid();
  extern __shared__ __align__(16) double vs[];   // staged input vector
  __shared__ double rowv[kSpecRows];
  __shared__ double tta[kLanczosMax], ttb[kLanczosMax];
  __shared__ double red[kWaves];
  __shared__ int hits[kWaves];
  __shared__ int skip;
  const int G = static_cast<int>(gridDim.x);
  const int iter = a.iter;
  int32_t* const ndone = a.ctl;
  // workgroups without chunks, which take the designated parts
  const int spare = G - a.nchunks;

  // Instances still running; their done flags do not change during the
  // launch, so every workgroup counts the same number and takes the same
  // path through the barriers below.
  double act_d = 0.0;
  for (int q = threadIdx.x; q < a.count; q += kThreads)
    act_d += a.inst[q].st->done ? 0.0 : 1.0;
  const int act = static_cast<int>(block_sum(act_d, red));
  if (act == 0) return;

  // P0: the start vector in w, q_{-1} = 0, and alpha-partials 0 for the
  // parity of step -1
  for (int c = blockIdx.x; c < a.nchunks; c += G) {
    const int2 ch = a.chunks[c];
    const Instance& in = a.inst[ch.x];
    if (in.st->done) continue;
    const SpecView v = spec_view(in.sp, in.n);
    const int ldq = spec_ldq(in.n), nch = ldq / kSpecRows;
    const int lc = c - in.sp_ch0;
    if (threadIdx.x < kSpecRows) {
      const int row = ch.y + threadIdx.x;
      v.w[row] = (row < in.n) ? start_entry(row) : 0.0;
      v.q[row] = 0.0;
      v.q[ldq + row] = 0.0;
    }
    if (threadIdx.x == 0) {
      v.part[nch + lc] = 0.0;
      if (lc == 0) {
        v.misc[0] = 0.0;
        v.misc[1] = 0.0;
      }
    }
  }
  grid.sync();

  for (int j = 0;; ++j) {
    const int pj = j & 1, pp = pj ^ 1;   // slots of q_j and q_{j-1}
    // P1: u_j = w - alpha_{j-1} q_{j-1} (into q_j's slot), ||u_j||^2 per
    // chunk, y = X~ u_j
    int staged = -1;
    for (int c = blockIdx.x; c < a.nchunks; c += G) {
      const int2 ch = a.chunks[c];
      const Instance& in = a.inst[ch.x];
      if (skip_instance(in, &skip)) continue;
      const SpecView v = spec_view(in.sp, in.n);
      const int ldq = spec_ldq(in.n), nch = ldq / kSpecRows;
      const int lc = c - in.sp_ch0;
      const double alpha = chunk_sum(v.part + pp * nch, nch, red);
      const double* qp = v.q + pp * ldq;
      double u = 0.0;
      if (threadIdx.x < kSpecRows) {
        const int row = ch.y + threadIdx.x;
        u = v.w[row] - alpha * qp[row];
        v.q[pj * ldq + row] = u;
      }
      const double uu = block_sum(u * u, red);
      if (threadIdx.x == 0) v.nu[lc] = uu;
      if (j == kLanczosMax) continue;   // only beta_{j-1} is still needed
      const T* X = static_cast<const T*>(in.X[(iter - 1) & 1]);
      const bool bsr = (in.bval[0] != nullptr);
      if (ldq <= a.vec_cap) {
        if (staged != ch.x) {
          __syncthreads();   // vs may still be read for the previous chunk
          stage<true>(vs, v.w, qp, alpha, 1.0, ldq);
          __syncthreads();
          staged = ch.x;
        }
        if (bsr)
          chunk_matvec_bsr(in, (iter - 1) & 1, ch.y, SrcLds{vs}, rowv);
        else
          chunk_matvec<T>(X, in.ld, in.n, ldq, ch.y, SrcLds{vs}, rowv);
      } else if (bsr) {
        chunk_matvec_bsr(in, (iter - 1) & 1, ch.y, SrcComb{v.w, qp, alpha, 1.0}, rowv);
      } else {
        chunk_matvec<T>(X, in.ld, in.n, ldq, ch.y,
                        SrcComb{v.w, qp, alpha, 1.0}, rowv);
      }
      __syncthreads();
      // the buffer holds Y = a X~ + c I (OpMap): X~ u = (Y u - c u) / a
      if (threadIdx.x < kSpecRows) {
        const OpMap m = op_map(in.prm.method, in.st->p[iter], in.st->alpha[iter]);
        v.y[ch.y + threadIdx.x] = (rowv[threadIdx.x] - m.c * u) / m.a;
      }
    }
    grid.sync();

    // P2, designated parts: on the spare workgroups, else on the owner of
    // the instance's first chunk
    auto designated = [&](const Instance& in) {
      const SpecView v = spec_view(in.sp, in.n);
      const int nch = spec_ldq(in.n) / kSpecRows;
      const double alpha = chunk_sum(v.part + pp * nch, nch, red);
      const double beta = sqrt(chunk_sum(v.nu, nch, red));
      decide(in, j, iter, alpha, beta, ndone, tta, ttb, hits);
    };
    if (spare > 0 && j >= 1) {
      for (int i = static_cast<int>(blockIdx.x) - a.nchunks;
           i >= 0 && i < a.count; i += spare) {
        const Instance& in = a.inst[i];
        if (in.sp_nch == 0 || skip_instance(in, &skip)) continue;
        designated(in);
      }
    }
    // P2, chunks: q_j = u_j / beta_{j-1}; w = X~ q_j - X~ X~ q_j -
    // beta_{j-1} q_{j-1}; partial q_j . w
    staged = -1;
    for (int c = blockIdx.x; c < a.nchunks; c += G) {
      const int2 ch = a.chunks[c];
      const Instance& in = a.inst[ch.x];
      if (skip_instance(in, &skip)) continue;
      if (spare <= 0 && j >= 1 && c == in.sp_ch0) designated(in);
      if (j == kLanczosMax) continue;   // every instance is final now
      const SpecView v = spec_view(in.sp, in.n);
      const int ldq = spec_ldq(in.n), nch = ldq / kSpecRows;
      const int lc = c - in.sp_ch0;
      const double beta = sqrt(chunk_sum(v.nu, nch, red));
      const double inv = (beta > 0.0) ? 1.0 / beta : 0.0;
      const T* X = static_cast<const T*>(in.X[(iter - 1) & 1]);
      const bool bsr = (in.bval[0] != nullptr);
      if (ldq <= a.vec_cap) {
        if (staged != ch.x) {
          __syncthreads();
          stage<false>(vs, v.y, nullptr, 0.0, inv, ldq);
          __syncthreads();
          staged = ch.x;
        }
        if (bsr)
          chunk_matvec_bsr(in, (iter - 1) & 1, ch.y, SrcLds{vs}, rowv);
        else
          chunk_matvec<T>(X, in.ld, in.n, ldq, ch.y, SrcLds{vs}, rowv);
      } else {
        // X~ (y / beta) = (X~ y) / beta
        if (bsr)
          chunk_matvec_bsr(in, (iter - 1) & 1, ch.y, SrcPlain{v.y}, rowv);
        else
          chunk_matvec<T>(X, in.ld, in.n, ldq, ch.y, SrcPlain{v.y}, rowv);
        __syncthreads();
        if (threadIdx.x < kSpecRows) rowv[threadIdx.x] *= inv;
      }
      __syncthreads();
      double qw = 0.0;
      if (threadIdx.x < kSpecRows) {
        const int row = ch.y + threadIdx.x;
        const double q = v.q[pj * ldq + row] * inv;
        // X~ (X~ q_j) from Y (X~ q_j) = rowv (see P1)
        const OpMap m = op_map(in.prm.method, in.st->p[iter], in.st->alpha[iter]);
        const double xxq = (rowv[threadIdx.x] - m.c * v.y[row] * inv) / m.a;
        const double x = v.y[row] * inv - xxq - beta * v.q[pp * ldq + row];
        v.q[pj * ldq + row] = q;
        v.w[row] = x;
        qw = q * x;
      }
      qw = block_sum(qw, red);
      if (threadIdx.x == 0) v.part[pj * nch + lc] = qw;
    }
    grid.sync();
    const int fin_cnt = __hip_atomic_load(ndone, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    if (fin_cnt >= act) break;
  }
}

template <typename T>
int max_grid(int num_cus, int vec_cap) {
  int per_cu = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, spectral_kernel<T>, kThreads, vec_cap * sizeof(double));
  if (e != hipSuccess || per_cu < 1) return 0;
  return per_cu * num_cus;
}

}  // namespace

int spectral_max_grid(bool fp64_store, int num_cus, int vec_cap) {
  return fp64_store ? max_grid<double>(num_cus, vec_cap)
                    : max_grid<float>(num_cus, vec_cap);
}

hipError_t launch_spectral(const SpecArgs& a, bool fp64_store, int grid,
                           hipStream_t s) {
  SpecArgs arg = a;
  void* params[] = {&arg};
  const void* fn = fp64_store
                       ? reinterpret_cast<const void*>(&spectral_kernel<double>)
                       : reinterpret_cast<const void*>(&spectral_kernel<float>);
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kThreads), params,
                                    a.vec_cap * sizeof(double), s);
}

}  // namespace sp2
