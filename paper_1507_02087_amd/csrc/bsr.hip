// Block-sparse SP2 step for matrices with decaying entries (the sparse
// setting of sec. 5 and sec. 6, where truncation E_i keeps the iterates
// sparse). Storage: block-sparse rows (BSR) with 32 x 32 FP32 blocks, both
// triangles stored (exactly symmetric), column indices sorted per row, and
// a per-block flag that is 1 when the block holds a nonzero after
// truncation.
//
// One step, X~_{i-1} (pattern P, some blocks flagged zero) -> X~_i:
//   1. index the nonzero blocks P' of X~_{i-1} per row (one workgroup);
//   2. symbolic product: the pattern Q = P' P' + P' per block row from an
//      LDS bitmap over the block columns, an exclusive scan of the row
//      counts, and a fill of the sorted column indices;
//   3. numeric: one wave per upper block (I, J) of Q, S_IJ = sum over
//      K in P'(I) and P'(J) of X_IK X_JK^T (X_KJ = X_JK^T by symmetry) on
//      v_mfma_f32_32x32x2_f32, then the same fused epilogue as the dense
//      square (error, polynomial, truncation, FP64 traces) and the mirrored
//      store of the transposed block; persistent waves walk the blocks with
//      a fixed stride, so the partial sums are deterministic.
// Blocks that truncation empties stay in Q with flag 0 and are dropped by
// the next step's index, so values are never compacted.
#include "sp2_device.h"

namespace sp2 {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int BS = 32;            // block edge
constexpr int BE = BS * BS;       // elements per block
constexpr int kScanThreads = 1024;

__device__ __forceinline__ double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Exclusive scan of cnt[0..n) into out[0..n] (out[n] = total) by one block
// of kScanThreads threads; n <= 2 * kScanThreads.
__device__ void block_exclusive_scan(const int32_t* cnt, int n, int32_t* out,
                                     int32_t* sh) {
  const int t = threadIdx.x;
  const int a = (2 * t < n) ? cnt[2 * t] : 0;
  const int b = (2 * t + 1 < n) ? cnt[2 * t + 1] : 0;
  sh[t] = a + b;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const int v = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  const int excl = sh[t] - (a + b);
  if (2 * t < n) out[2 * t] = excl;
  if (2 * t + 1 < n) out[2 * t + 1] = excl + a;
  if (t == kScanThreads - 1) out[n] = sh[t];
}

// (1) Index of the nonzero blocks of M, per row, in column order.
__global__ __launch_bounds__(kScanThreads) void bsr_index_kernel(
    BsrMat M, int nb, BsrIndex idx, const DevState* st, BsrCounters* ctr,
    int iter) {
  __shared__ int32_t cnt[2 * kScanThreads];
  __shared__ int32_t sh[kScanThreads];
  if (st && st->done) return;
  for (int r = threadIdx.x; r < nb; r += kScanThreads) {
    int c = 0;
    for (int q = M.row_ptr[r]; q < M.row_ptr[r + 1]; ++q) c += M.flag[q] ? 1 : 0;
    cnt[r] = c;
  }
  __syncthreads();
  block_exclusive_scan(cnt, nb, idx.ptr, sh);
  __syncthreads();
  if (iter > 0 && threadIdx.x == 0) ctr->nonzero[iter] = idx.ptr[nb];
  for (int r = threadIdx.x; r < nb; r += kScanThreads) {
    int o = idx.ptr[r];
    for (int q = M.row_ptr[r]; q < M.row_ptr[r + 1]; ++q)
      if (M.flag[q]) {
        idx.col[o] = M.col[q];
        idx.pos[o] = q;
        ++o;
      }
  }
}

// (2a) Row bitmaps of Q = P' P' + P' + diag and their popcounts.
__global__ __launch_bounds__(256) void bsr_symbolic_count_kernel(
    BsrIndex idx, int nb, int nbw, uint32_t* bitmap, int32_t* qcnt,
    const DevState* st) {
  __shared__ uint32_t bm[kMaxBlockCols / 32];
  __shared__ int32_t red[4];
  if (st->done) return;
  const int I = blockIdx.x;
  for (int w = threadIdx.x; w < nbw; w += 256) bm[w] = 0;
  __syncthreads();
  const int b0 = idx.ptr[I], b1 = idx.ptr[I + 1];
  // the diagonal block is always kept: the identity term of a stretched
  // step (Alg. 4) writes it even where the iterate's block is empty
  if (threadIdx.x == 0) atomicOr(&bm[I >> 5], 1u << (I & 31));
  for (int a = b0; a < b1; ++a) {
    const int K = idx.col[a];
    if (threadIdx.x == 0) atomicOr(&bm[K >> 5], 1u << (K & 31));
    for (int q = idx.ptr[K] + threadIdx.x; q < idx.ptr[K + 1]; q += 256) {
      const int J = idx.col[q];
      atomicOr(&bm[J >> 5], 1u << (J & 31));
    }
  }
  __syncthreads();
  int c = 0;
  for (int w = threadIdx.x; w < nbw; w += 256) {
    bitmap[static_cast<size_t>(I) * nbw + w] = bm[w];
    c += __popc(bm[w]);
  }
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) qcnt[I] = red[0] + red[1] + red[2] + red[3];
}

// (2b) Row pointers of Q; flags an overflow when Q exceeds the capacity.
__global__ __launch_bounds__(kScanThreads) void bsr_symbolic_scan_kernel(
    const int32_t* qcnt, int nb, int32_t* row_ptr, int32_t cap,
    BsrCounters* ctr, const DevState* st, int iter) {
  __shared__ int32_t cnt[2 * kScanThreads];
  __shared__ int32_t sh[kScanThreads];
  if (st->done) return;
  for (int r = threadIdx.x; r < nb; r += kScanThreads) cnt[r] = qcnt[r];
  __syncthreads();
  block_exclusive_scan(cnt, nb, row_ptr, sh);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int total = row_ptr[nb];
    ctr->nnzb = total;
    ctr->stored[iter] = total;
    if (total > cap) ctr->overflow = 1;
  }
}

// (2c) Sorted column indices (and block rows) of Q from the bitmaps.
__global__ __launch_bounds__(64) void bsr_symbolic_fill_kernel(
    const uint32_t* bitmap, int nb, int nbw, BsrMat Q, const BsrCounters* ctr,
    const DevState* st) {
  if (st->done || ctr->overflow) return;
  const int I = blockIdx.x;
  int base = Q.row_ptr[I];
  for (int w0 = 0; w0 < nbw; w0 += 64) {
    const int w = w0 + threadIdx.x;
    const uint32_t bits = (w < nbw) ? bitmap[static_cast<size_t>(I) * nbw + w] : 0u;
    int c = __popc(bits);
    // inclusive prefix over the wave
    int incl = c;
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (threadIdx.x >= off) incl += v;
    }
    int o = base + incl - c;
    uint32_t b = bits;
    while (b) {
      const int bit = __ffs(b) - 1;
      b &= b - 1;
      Q.col[o] = 32 * w + bit;
      Q.brow[o] = I;
      ++o;
    }
    base += __shfl(incl, 63, 64);
  }
}

// Position of column c in the sorted list col[lo..hi), or -1.
__device__ __forceinline__ int find_col(const int32_t* col, int lo, int hi,
                                        int c) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int v = col[mid];
    if (v == c) return mid;
    if (v < c) lo = mid + 1;
    else hi = mid;
  }
  return -1;
}

// (3) Numeric product and fused epilogue. Persistent: wave g of G handles
// blocks g, g + G, ... of Q (upper ones only).
__global__ __launch_bounds__(256) void bsr_numeric_kernel(
    BsrMat A, BsrIndex idx, BsrMat B, BsrCounters* ctr,
    const Instance* inst, int iter, int n, double* part) {
  __shared__ double sh[4][3];
  const Instance& in = inst[0];
  const DevState* st = in.st;
  if (st->done) return;
  if (ctr->overflow) {
    // No product this step: non-finite partial sums make the finalize step
    // stop the run; the host reports the reason from the counters.
    if (threadIdx.x == 0) {
      part[3 * blockIdx.x + 0] = NAN;
      part[3 * blockIdx.x + 1] = NAN;
      part[3 * blockIdx.x + 2] = NAN;
    }
    return;
  }
  // the step squares the stored Y = a X~ + c I (OpMap); X_i = S or 2 Y - S,
  // the error of X~ from Y and S, and the stored output is the next step's
  // matrix an X~_i + cn I
  const bool p1 = st->p[iter] != 0;
  const StepCoef k{st->ecoef[0], st->ecoef[1], st->ecoef[2], st->ecoef[3],
                   st->ecoef[4]};
  const bool stretch = st->stretch != 0;
  const float ka = p1 ? 1.f : -1.f, kb = p1 ? 0.f : 2.f;
  const double tau = in.tau;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 31, h = lane >> 5;
  const int total = ctr->nnzb;
  const int G = gridDim.x * 4;
  double sv = 0.0, st1 = 0.0, st2 = 0.0;
  unsigned long long nprod = 0;
  for (int q = blockIdx.x * 4 + wave; q < total; q += G) {
    const int I = B.brow[q], J = B.col[q];
    if (J < I) continue;
    // S_IJ = sum_K X_IK X_JK^T over K in P'(I) and P'(J), in K order.
    floatx16 acc;
    for (int j = 0; j < 16; ++j) acc[j] = 0.f;
    const int i0 = idx.ptr[I], i1 = idx.ptr[I + 1];
    const int j0 = idx.ptr[J], j1 = idx.ptr[J + 1];
    for (int c0 = i0; c0 < i1; c0 += 64) {
      int posI = -1, posJ = -1;
      if (c0 + lane < i1) {
        const int K = idx.col[c0 + lane];
        const int m = find_col(idx.col, j0, j1, K);
        if (m >= 0) {
          posI = idx.pos[c0 + lane];
          posJ = idx.pos[m];
        }
      }
      unsigned long long mask = __ballot(posI >= 0);
      nprod += __popcll(mask);
      while (mask) {
        const int src = __ffsll(static_cast<long long>(mask)) - 1;
        mask &= mask - 1;
        const int pa = __shfl(posI, src, 64), pb = __shfl(posJ, src, 64);
        const float* ab = A.val + static_cast<size_t>(pa) * BE + r * BS + h * 16;
        const float* bb = A.val + static_cast<size_t>(pb) * BE + r * BS + h * 16;
        floatx4 af[4], bf[4];
        for (int u = 0; u < 4; ++u) {
          af[u] = *gro(reinterpret_cast<const floatx4*>(ab + 4 * u));
          bf[u] = *gro(reinterpret_cast<const floatx4*>(bb + 4 * u));
        }
        for (int s = 0; s < 16; ++s)
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(af[s >> 2][s & 3],
                                                     bf[s >> 2][s & 3], acc,
                                                     0, 0, 0);
      }
    }
    // Epilogue. Old block X_IJ (zero if absent or emptied).
    const int po = find_col(idx.col, i0, i1, J);
    const float* old = (po >= 0) ? A.val + static_cast<size_t>(idx.pos[po]) * BE
                                 : nullptr;
    const int qT = (I == J) ? q : find_col(B.col, B.row_ptr[J], B.row_ptr[J + 1], I);
    if (qT < 0) {
      // (J, I) missing: the pattern is not symmetric (F was not).
      if (lane == 0) atomicOr(&ctr->overflow, 2);
      continue;
    }
    float* out = B.val + static_cast<size_t>(q) * BE;
    float* outT = B.val + static_cast<size_t>(qT) * BE;
    bool nz = false;
    double bsq = 0.0;   // squared Frobenius norm of this block of X~ - S
    for (int j = 0; j < 16; ++j) {
      const int m = 8 * (j >> 2) + 4 * h + (j & 3);   // row in the block
      const int c = r;                                // column in the block
      if (I == J && m > c) continue;
      const float s = acc[j];
      const float xo = old ? *gro(old + m * BS + c) : 0.f;
      // identity terms only inside the matrix proper
      const bool on = (I == J && m == c && I * BS + m < n);
      const double d = __builtin_fma(k.es, static_cast<double>(s),
                                     k.ey * static_cast<double>(xo)) +
                       (on ? k.ei : 0.0);
      const double w = (I == J && m == c) ? 1.0 : 2.0;
      sv += w * d * d;
      bsq += (I == J) ? w * d * d : d * d;
      float xn = __builtin_fmaf(kb, xo, ka * s);
      double xd = static_cast<double>(xn);
      if (fabs(xd) < tau) {
        xn = 0.f;
        xd = 0.0;
      }
      st2 += w * xd * xd;
      if (I == J && m == c) st1 += xd;
      nz = nz || (xn != 0.f);
      if (stretch) xn = static_cast<float>(__builtin_fma(k.an, xd, on ? k.cn : 0.0));
      *grw(out + m * BS + c) = xn;
      if (!(I == J && m == c)) *grw(outT + c * BS + m) = xn;
    }
    const int any = __any(nz) ? 1 : 0;
    if (lane == 0) {
      B.flag[q] = any;
      B.flag[qT] = any;
    }
    if (in.blk) {
      // mixed norm: one value per block of the output pattern
      bsq = wave_sum(bsq);
      if (lane == 0) {
        const float bn = static_cast<float>(sqrt(bsq));
        *grw(in.blk + q) = bn;
        *grw(in.blk + qT) = bn;
      }
    }
  }
  sv = wave_sum(sv);
  st1 = wave_sum(st1);
  st2 = wave_sum(st2);
  if (lane == 0) {
    sh[wave][0] = sv;
    sh[wave][1] = st1;
    sh[wave][2] = st2;
  }
  __syncthreads();
  if (lane == 0 && nprod) atomicAdd(&ctr->products[iter], nprod);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x + 0] = sh[0][0] + sh[1][0] + sh[2][0] + sh[3][0];
    part[3 * blockIdx.x + 1] = sh[0][1] + sh[1][1] + sh[2][1] + sh[3][1];
    part[3 * blockIdx.x + 2] = sh[0][2] + sh[1][2] + sh[2][2] + sh[3][2];
  }
}

// Affine start on the input pattern: X_0 = (lambda_max I - F)/width in FP64,
// truncated, rounded to FP32; one block of X per workgroup, which also
// writes its FP64 partial traces.
__global__ __launch_bounds__(256) void bsr_f0_kernel(
    const double* __restrict__ F, BsrMat X, const Instance* inst, int n,
    double* part) {
  __shared__ double sh[4][2];
  __shared__ int anyz[4];
  const Instance& in = inst[0];
  const int q = blockIdx.x;
  const int I = X.brow[q], J = X.col[q];
  const int n_occ = static_cast<int>(in.prm.n_occ);
  const int trivial = (n_occ == 0) ? 1 : (n_occ == n ? 2 : 0);
  const OpMap m1 = step_map(in, 1);
  const bool stretch = (m1.a != 1.0 || m1.c != 0.0);
  double t1 = 0.0, t2 = 0.0;
  bool nz = false;
  for (int e = threadIdx.x; e < BE; e += 256) {
    const int m = e / BS, c = e % BS;
    const int gi = I * BS + m, gj = J * BS + c;
    double x = 0.0;
    if (gi < n && gj < n) {
      if (trivial) {
        x = (trivial == 2 && gi == gj) ? 1.0 : 0.0;
      } else {
        const double f = F[static_cast<size_t>(q) * BE + e];
        x = ((gi == gj) ? in.lmax - f : -f) / in.width;
        if (fabs(x) < in.tau) x = 0.0;
      }
    }
    const float xs = static_cast<float>(x);
    const double xd = static_cast<double>(xs);
    // stored: the matrix of step 1 (a X~_0 + c I with a stretch)
    X.val[static_cast<size_t>(q) * BE + e] =
        (stretch && !trivial)
            ? static_cast<float>(__builtin_fma(m1.a, xd,
                                               (gi == gj && gi < n) ? m1.c : 0.0))
            : xs;
    t2 += xd * xd;
    if (gi == gj) t1 += xd;
    nz = nz || (xs != 0.f);
  }
  t1 = wave_sum(t1);
  t2 = wave_sum(t2);
  const int any = __any(nz) ? 1 : 0;
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[wave][0] = t1;
    sh[wave][1] = t2;
    anyz[wave] = any;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[3 * q + 0] = 0.0;
    part[3 * q + 1] = sh[0][0] + sh[1][0] + sh[2][0] + sh[3][0];
    part[3 * q + 2] = sh[0][1] + sh[1][1] + sh[2][1] + sh[3][1];
    X.flag[q] = anyz[0] | anyz[1] | anyz[2] | anyz[3];
  }
}

__global__ void bsr_reset_kernel(BsrCounters* ctr) {
  int32_t* w = reinterpret_cast<int32_t*>(ctr);
  const int words = static_cast<int>(sizeof(BsrCounters) / sizeof(int32_t));
  for (int i = threadIdx.x; i < words; i += blockDim.x) w[i] = 0;
}

// Gathers the blocks listed by idx.pos into a compact array (FP64 or FP32),
// as (x - c [diagonal]) / a: the returned iterate from its stored matrix.
template <typename To>
__global__ __launch_bounds__(256) void bsr_gather_kernel(
    const float* __restrict__ val, const int32_t* __restrict__ brow,
    const int32_t* __restrict__ bcol, const int32_t* __restrict__ pos, int cnt,
    int n, OpMap m, To* __restrict__ out) {
  for (int b = blockIdx.x; b < cnt; b += gridDim.x) {
    const int p = pos[b];
    const float* src = val + static_cast<size_t>(p) * BE;
    const bool dblk = (brow[p] == bcol[p]);
    for (int e = threadIdx.x; e < BE; e += 256) {
      const int i = e / BS, j = e % BS;
      const bool on = dblk && i == j && brow[p] * BS + i < n;
      out[static_cast<size_t>(b) * BE + e] = static_cast<To>(
          (static_cast<double>(src[e]) - (on ? m.c : 0.0)) / m.a);
    }
  }
}

// Expands the nonzero blocks into a dense n x n matrix (zero elsewhere),
// as (x - c [diagonal]) / a.
template <typename To>
__global__ __launch_bounds__(256) void bsr_to_dense_kernel(
    const float* __restrict__ val, BsrIndex idx, int nb, int n, OpMap m,
    To* __restrict__ D, int64_t ldd) {
  const int I = blockIdx.x;
  for (int b = idx.ptr[I]; b < idx.ptr[I + 1]; ++b) {
    const int J = idx.col[b];
    const float* src = val + static_cast<size_t>(idx.pos[b]) * BE;
    for (int e = threadIdx.x; e < BE; e += 256) {
      const int gi = I * BS + e / BS, gj = J * BS + e % BS;
      if (gi < n && gj < n)
        D[gi * ldd + gj] = static_cast<To>(
            (static_cast<double>(src[e]) - (gi == gj ? m.c : 0.0)) / m.a);
    }
  }
  (void)nb;
}

}  // namespace

hipError_t launch_bsr_reset(BsrCounters* ctr, hipStream_t s) {
  hipLaunchKernelGGL(bsr_reset_kernel, dim3(1), dim3(64), 0, s, ctr);
  return hipGetLastError();
}

hipError_t launch_bsr_index(const BsrMat& M, int nb, const BsrIndex& idx,
                            const DevState* st, BsrCounters* ctr, int iter,
                            hipStream_t s) {
  hipLaunchKernelGGL(bsr_index_kernel, dim3(1), dim3(kScanThreads), 0, s, M,
                     nb, idx, st, ctr, iter);
  return hipGetLastError();
}

hipError_t launch_bsr_symbolic(const BsrIndex& idx, int nb, uint32_t* bitmap,
                               int32_t* qcnt, const BsrMat& Q, int32_t cap,
                               BsrCounters* ctr, const DevState* st, int iter,
                               hipStream_t s) {
  const int nbw = (nb + 31) / 32;
  hipLaunchKernelGGL(bsr_symbolic_count_kernel, dim3(nb), dim3(256), 0, s, idx,
                     nb, nbw, bitmap, qcnt, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bsr_symbolic_scan_kernel, dim3(1), dim3(kScanThreads), 0,
                     s, qcnt, nb, Q.row_ptr, cap, ctr, st, iter);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bsr_symbolic_fill_kernel, dim3(nb), dim3(64), 0, s,
                     bitmap, nb, nbw, Q, ctr, st);
  return hipGetLastError();
}

hipError_t launch_bsr_numeric(const BsrMat& A, const BsrIndex& idx,
                              const BsrMat& B, BsrCounters* ctr,
                              const Instance* inst, int iter, int n,
                              double* part, int grid, hipStream_t s) {
  hipLaunchKernelGGL(bsr_numeric_kernel, dim3(grid), dim3(256), 0, s, A, idx,
                     B, ctr, inst, iter, n, part);
  return hipGetLastError();
}

hipError_t launch_bsr_f0(const double* F, const BsrMat& X, int nnzb,
                         const Instance* inst, int n, double* part,
                         hipStream_t s) {
  hipLaunchKernelGGL(bsr_f0_kernel, dim3(nnzb), dim3(256), 0, s, F, X, inst, n,
                     part);
  return hipGetLastError();
}

hipError_t launch_bsr_gather(const BsrMat& M, const int32_t* pos, int cnt,
                             int n, OpMap m, void* out, bool fp64,
                             hipStream_t s) {
  const int g = cnt < 4096 ? (cnt > 0 ? cnt : 1) : 4096;
  if (fp64)
    hipLaunchKernelGGL(bsr_gather_kernel<double>, dim3(g), dim3(256), 0, s,
                       M.val, M.brow, M.col, pos, cnt, n, m,
                       static_cast<double*>(out));
  else
    hipLaunchKernelGGL(bsr_gather_kernel<float>, dim3(g), dim3(256), 0, s,
                       M.val, M.brow, M.col, pos, cnt, n, m,
                       static_cast<float*>(out));
  return hipGetLastError();
}

hipError_t launch_bsr_to_dense(const float* val, const BsrIndex& idx, int nb,
                               int n, OpMap m, void* D, int64_t ldd, bool fp64,
                               hipStream_t s) {
  if (fp64)
    hipLaunchKernelGGL(bsr_to_dense_kernel<double>, dim3(nb), dim3(256), 0, s,
                       val, idx, nb, n, m, static_cast<double*>(D), ldd);
  else
    hipLaunchKernelGGL(bsr_to_dense_kernel<float>, dim3(nb), dim3(256), 0, s,
                       val, idx, nb, n, m, static_cast<float*>(D), ldd);
  return hipGetLastError();
}

}  // namespace sp2
