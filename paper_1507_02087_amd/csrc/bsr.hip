// Block-sparse SP2 step for matrices with decaying entries (the sparse
// setting of sec. 5 and sec. 6, where truncation E_i keeps the iterates
// sparse). Storage: block-sparse rows (BSR) with 32 x 32 FP32 blocks, both
// triangles stored (exactly symmetric), column indices sorted per row, and
// a per-block flag that is 1 when the stored block (the operand of the next
// square, a X~ + c I under a stretch) holds a nonzero after truncation.
//
// One step, X~_{i-1} (pattern P, some blocks flagged zero) -> X~_i:
//   1. symbolic product: the pattern Q = P' P' + P' + diag (P': the flagged
//      blocks) per block row from an LDS bitmap over the block columns, then
//      a fill of the row starts, the sorted column indices and the list of
//      upper blocks (I, J >= I) with the position of each one's transpose;
//   2. numeric: one wave per upper block (I, J) of Q, S_IJ = sum over
//      K in P'(I) and P'(J) of X_IK X_JK^T (X_KJ = X_JK^T by symmetry) on
//      v_mfma_f32_32x32x2_f32, then the same fused epilogue as the dense
//      square (error, polynomial, truncation, FP64 traces) and the store of
//      the block and of its transpose; each wave takes a fixed set of
//      blocks, so the partial sums are deterministic.
// Elements of a block are stored in the MFMA operand order of blk_off, so
// that every load of a block row's operand reads contiguous memory.
// Blocks that truncation empties stay in Q with flag 0 and are skipped by
// the next step, so values are never compacted. The index kernel (nonzero
// blocks per row, in column order) serves the extraction of the result.
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

// Index of the flagged blocks of M, per row, in column order (for the
// extraction of the result).
__global__ __launch_bounds__(kScanThreads) void bsr_index_kernel(
    BsrMat M, int nb, BsrIndex idx) {
  __shared__ int32_t cnt[2 * kScanThreads];
  __shared__ int32_t sh[kScanThreads];
  for (int r = threadIdx.x; r < nb; r += kScanThreads) {
    int c = 0;
    for (int q = M.row_ptr[r]; q < M.row_ptr[r + 1]; ++q) c += M.flag[q] ? 1 : 0;
    cnt[r] = c;
  }
  __syncthreads();
  block_exclusive_scan(cnt, nb, idx.ptr, sh);
  __syncthreads();

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

// (2a) Row bitmaps of Q = P' P' + P' + diag (P': the flagged blocks of the
// iterate), the prefix popcounts of their words, and the counts of all and
// of upper (J >= I) blocks per row. The workgroup first reads the column K
// and the extent of row K of every flagged block of row I (one thread
// each), then each wave ORs the flagged columns of its share of those rows
// into the LDS bitmap. Also counts the flagged blocks (statistics).
constexpr int kCountThreads = 256;

__global__ __launch_bounds__(kCountThreads) void bsr_symbolic_count_kernel(
    BsrMat A, int nb, int nbw, BsrSymbolic sym, BsrCounters* ctr,
    const DevState* st, int iter) {
  __shared__ uint32_t bm[kMaxBlockCols / 32];
  __shared__ int32_t rk0[kCountThreads], pfx[kCountThreads + 1];
  __shared__ int32_t wsum[kCountThreads / 64];
  if (st->done) return;
  const int I = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  for (int w = t; w < nbw; w += kCountThreads) bm[w] = 0;
  const int b0 = A.row_ptr[I], b1 = A.row_ptr[I + 1];
  __syncthreads();
  // the diagonal block is always kept: the identity term of a stretched
  // step (Alg. 4) writes it even where the iterate's block is empty
  if (t == 0) atomicOr(&bm[I >> 5], 1u << (I & 31));
  int nonzero = 0;
  for (int a0 = b0; a0 < b1; a0 += kCountThreads) {
    // thread t: flagged block a0 + t of row I, its column K and the extent
    // of row K; then the (row, entry) pairs of all those rows are walked as
    // one flat range, one pair per thread, found through the prefix sums of
    // the row lengths
    const int na = min(kCountThreads, b1 - a0);
    int len = 0;
    bool nz = false;
    if (t < na && A.flag[a0 + t]) {
      const int K = A.col[a0 + t];
      atomicOr(&bm[K >> 5], 1u << (K & 31));
      const int r0 = A.row_ptr[K];
      rk0[t] = r0;
      len = A.row_ptr[K + 1] - r0;
      nz = true;
    }
    int incl = len;
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    nonzero += __syncthreads_count(nz);
    int base = 0;
    for (int w = 0; w < wave; ++w) base += wsum[w];
    pfx[t + 1] = base + incl;
    if (t == 0) pfx[0] = 0;
    __syncthreads();
    const int total = pfx[na];
    for (int p = t; p < total; p += kCountThreads) {
      // largest a with pfx[a] <= p (rows of length 0 are skipped over)
      int lo = 0, hi = na;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pfx[mid] <= p) lo = mid;
        else hi = mid;
      }
      const int q = rk0[lo] + (p - pfx[lo]);
      if (A.flag[q]) {
        const int J = A.col[q];
        atomicOr(&bm[J >> 5], 1u << (J & 31));
      }
    }
    __syncthreads();
  }
  if (t == 0) sym.nzrow[I] = nonzero;
  if (wave == 0) {
    // nbw <= 64: one word per lane
    const int w = lane;
    const uint32_t bits = (w < nbw) ? bm[w] : 0u;
    const int c = __popc(bits);
    int incl = c;
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    if (w < nbw) {
      sym.bitmap[static_cast<size_t>(I) * nbw + w] = bits;
      sym.wpre[static_cast<size_t>(I) * nbw + w] = incl - c;
    }
    const int wi = I >> 5;
    const uint32_t um = (w > wi) ? ~0u : (w == wi ? (~0u << (I & 31)) : 0u);
    int u = __popc(bits & um);
    for (int off = 32; off > 0; off >>= 1) u += __shfl_xor(u, off, 64);
    if (lane == 63) sym.qcnt[I] = incl;
    if (lane == 0) sym.ucnt[I] = u;
  }
}

// (2b) Sorted column indices (and block rows) of Q from the bitmaps, and the
// upper work list: for each block (I, J >= I) its position, the position of
// (J, I) (start of row J plus the rank of I among the columns of row J, from
// J's bitmap word and its prefix popcount), I and J. One wave per row. The
// row starts of Q are exclusive sums of the row counts; every workgroup
// forms them itself in LDS (integer sums, exact in any order) rather than
// waiting for a separate scan launch, and so also knows the totals: a
// pattern over capacity stops every workgroup before it writes anything.
// Workgroup 0 records the totals and the statistics for the host.
static_assert(kMaxBlockCols <= 64 * 32, "a row's bitmap is at most one word per lane");
__global__ __launch_bounds__(64) void bsr_symbolic_fill_kernel(
    BsrSymbolic sym, int nb, int nbw, BsrMat Q, int32_t cap, BsrCounters* ctr,
    const DevState* st, int iter) {
  __shared__ int32_t cols[kMaxBlockCols];
  __shared__ int32_t pre[kMaxBlockCols + 1];
  if (st->done) return;
  const int I = blockIdx.x;
  const int lane = threadIdx.x;
  // this row's bitmap words (nbw <= 64: one per lane) and the prefix
  // popcount at the diagonal's word, loaded with the row counts below
  const int wi = I >> 5;
  const uint32_t* brow_bits = sym.bitmap + static_cast<size_t>(I) * nbw;
  const uint32_t bits = (lane < nbw) ? brow_bits[lane] : 0u;
  const int wpre_i = sym.wpre[static_cast<size_t>(I) * nbw + wi];
  // exclusive prefix sums of the stored blocks per row (pre) and the upper
  // blocks before row I (u0): lane l takes rows l * per .. l * per + per - 1
  // (all its loads in flight at once), then one scan over the lanes' sums
  constexpr int kPer = kMaxBlockCols / 64;
  const int per = (nb + 63) / 64;
  const int r0 = lane * per;
  int v[kPer];
  int sum = 0, ub = 0, ut = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int r = r0 + k;
    const bool ok = k < per && r < nb;
    v[k] = ok ? sym.qcnt[r] : 0;
    const int uc = ok ? sym.ucnt[r] : 0;
    sum += v[k];
    ut += uc;
    ub += (ok && r < I) ? uc : 0;
  }
  int incl = sum;
  for (int off = 1; off < 64; off <<= 1) {
    const int x = __shfl_up(incl, off, 64);
    if (lane >= off) incl += x;
  }
  int run = incl - sum;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int r = r0 + k;
    if (k < per && r < nb) pre[r] = run;
    run += v[k];
  }
  const int base = __shfl(incl, 63, 64);
  for (int off = 32; off > 0; off >>= 1) {
    ub += __shfl_xor(ub, off, 64);
    ut += __shfl_xor(ut, off, 64);
  }
  const int total = base;
  if (lane == 0) pre[nb] = total;
  __syncthreads();
  if (total > cap) {
    if (I == 0 && lane == 0) atomicOr(&ctr->overflow, 1);
    return;
  }
  if (I == 0) {
    // flagged blocks of the iterate (statistics)
    int nz = 0;
    for (int r = lane; r < nb; r += 64) nz += sym.nzrow[r];
    for (int off = 32; off > 0; off >>= 1) nz += __shfl_xor(nz, off, 64);
    if (lane == 0) {
      ctr->nnzb = total;
      ctr->nupper = ut;
      ctr->stored[iter] = total;
      ctr->nonzero[iter] = nz;
      Q.row_ptr[nb] = total;
    }
  }
  const int row0 = pre[I];
  if (lane == 0) Q.row_ptr[I] = row0;
  int count;
  {
    const int c = __popc(bits);
    int ic = c;
    for (int off = 1; off < 64; off <<= 1) {
      const int x = __shfl_up(ic, off, 64);
      if (lane >= off) ic += x;
    }
    int o = ic - c;
    uint32_t b = bits;
    while (b) {
      const int bit = __ffs(b) - 1;
      b &= b - 1;
      const int J = 32 * lane + bit;
      cols[o] = J;
      Q.col[row0 + o] = J;
      Q.brow[row0 + o] = I;
      ++o;
    }
    count = __shfl(ic, 63, 64);
  }
  __syncthreads();
  const uint32_t low = (1u << (I & 31)) - 1u;
  // columns before the diagonal block, which is always present
  const int first = wpre_i + __popc(static_cast<uint32_t>(__shfl(static_cast<int>(bits), wi, 64)) & low);
  const int u0 = ub;
  for (int t = first + lane; t < count; t += 64) {
    const int J = cols[t];
    const int q = row0 + t;
    int qT = q;
    if (J != I) {
      const uint32_t wj = sym.bitmap[static_cast<size_t>(J) * nbw + wi];
      if (!((wj >> (I & 31)) & 1u)) {
        // (J, I) missing: the pattern is not symmetric (F was not)
        atomicOr(&ctr->overflow, 2);
        continue;
      }
      qT = pre[J] + sym.wpre[static_cast<size_t>(J) * nbw + wi] + __popc(wj & low);
    }
    BsrWork wk;
    wk.q = q;
    wk.qT = qT;
    wk.I = I;
    wk.J = J;
    sym.work[u0 + t - first] = wk;
  }
}

// (3) Numeric product and fused epilogue, one upper output block (I, J) of
// the work list per wave at a time. Workgroup b runs on XCD b % 8 (the grid
// is a multiple of 8); XCD x takes the x-th contiguous eighth of the work
// list (ordered by block row), so the blocks that neighbouring rows share
// stay in its L2, and each of its workgroups a contiguous share of that;
// wave w of a workgroup takes blocks w, w + 4, w + 8, ... of its share.
// Every lane adds its elements' partial sums over the wave's blocks, then
// the wave and the workgroup add theirs in a fixed order, so the sums do
// not depend on timing.
// Per block: the flagged columns K of rows I and J (one per lane, both rows
// loaded at once), the common ones found by comparing each of row I's
// columns with every column of row J (broadcast lane by lane), then the
// products X_IK X_JK^T with the operands of the next product loaded during
// the current one's MFMAs. The old block is read as its stored transpose
// X_JI (rows of X_JI are columns of X_IJ, which is what each lane's
// accumulator holds) into registers while the products run. The work
// entry of the wave's next block is loaded at the start of this one, its
// row extents during this one's epilogue.
__device__ __forceinline__ void load_block_frag(const float* val, int p, int lane,
                                                floatx4 (&f)[4]) {
  const float* b = val + static_cast<size_t>(p) * BE + 4 * lane;
  for (int u = 0; u < 4; ++u) f[u] = *gro(reinterpret_cast<const floatx4*>(b + 256 * u));
}

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Row stride of the LDS tile that transposes an output block: 36 floats keep
// every 16-byte row segment aligned, and the 16 lanes of a quarter-wave read
// rows m at 36 m, which fall on 16 distinct groups of four of the 64 banks.
constexpr int kTileLd = 36;

__global__ __launch_bounds__(256, 4) void bsr_numeric_kernel(
    BsrMat A, BsrMat B, const BsrWork* __restrict__ work, uint32_t* prod_wg,
    BsrCounters* ctr, const Instance* inst, int iter, int n, double* part) {
  __shared__ double wsum[4][3];
  __shared__ unsigned long long shp[4];
  // per wave: the output block, row-major with rows padded to 36 floats, to
  // turn the accumulator's columns into the storage order's rows
  __shared__ __attribute__((aligned(16))) float tile[4][BS * kTileLd];
  // The instance and its state are read as scalars through the constant
  // address space (neither changes during the launch). Through generic
  // pointers they would be FLAT loads, and while one of those is pending the
  // compiler cannot count vector loads in order, so every wait in the
  // product loop below would wait for all loads in flight.
  const auto* in = cro(inst);
  const auto* st = cro(in->st);
  if (st->done) return;
  if (ctr->overflow) {
    // No product this step: non-finite partial sums make the finalize step
    // stop the run; the host reports the reason from the counters.
    if (threadIdx.x == 0) {
      part[3 * blockIdx.x + 0] = NAN;
      part[3 * blockIdx.x + 1] = NAN;
      part[3 * blockIdx.x + 2] = NAN;
      prod_wg[static_cast<size_t>(iter) * gridDim.x + blockIdx.x] = 0;
    }
    return;
  }
  const int lane = threadIdx.x & 63;
  const int wave = uni(threadIdx.x >> 6);
  // The step squares the stored Y = a X~ + c I (OpMap); X_i = S or 2 Y - S,
  // the error of X~ from Y and S, and the stored output is the next step's
  // matrix an X~_i + cn I. These and the truncation threshold are read once.
  const bool p1 = st->p[iter] != 0;
  const StepCoef k{st->ecoef[0], st->ecoef[1], st->ecoef[2], st->ecoef[3],
                   st->ecoef[4]};
  const bool stretch = st->stretch != 0;
  const float ka = p1 ? 1.f : -1.f, kb = p1 ? 0.f : 2.f;
  const double tau = in->tau;
  // the largest float below tau: for a float x, |x| < tau <=> |x| <= tf
  float tf = static_cast<float>(tau);
  if (tf > 0.f && static_cast<double>(tf) >= tau) tf = __int_as_float(__float_as_int(tf) - 1);
  float* const blk = in->blk;
  const int total = ctr->nupper;
  const int nx = (gridDim.x % 8 == 0) ? 8 : 1;
  const int x = blockIdx.x % nx;
  const int gx = gridDim.x / nx, lb = blockIdx.x / nx;
  const int u_lo = static_cast<int>(static_cast<int64_t>(total) * x / nx);
  const int u_hi = static_cast<int>(static_cast<int64_t>(total) * (x + 1) / nx);
  const int w_lo = u_lo + static_cast<int>(static_cast<int64_t>(u_hi - u_lo) * lb / gx);
  const int w_hi = u_lo + static_cast<int>(static_cast<int64_t>(u_hi - u_lo) * (lb + 1) / gx);
  double sv = 0.0, st1 = 0.0, st2 = 0.0;   // this lane's partial sums
  unsigned long long nprod = 0;
  // the lane's entry of a row chunk: its column if flagged, else `none`.
  // Lanes past the row read position 0 (always valid) and discard it, so the
  // loads need no branch and the two rows' loads are all in flight at once.
  auto first_cols = [&](int lo, int hi, int none) {
    const bool ok = lo + lane < hi;
    const int i = ok ? lo + lane : 0;
    const int f = A.flag[i];
    const int c = A.col[i];
    return (ok && f != 0) ? c : none;
  };
  // work list and row pointers of the old iterate: read-only here, read as
  // scalars (so their waits do not include the vector stores in flight)
  const auto* wl = cro(work);
  const auto* rp = cro(A.row_ptr);
  auto work_at = [&](int i) {
    return BsrWork{wl[i].q, wl[i].qT, wl[i].I, wl[i].J};
  };
  int u = w_lo + wave;
  BsrWork wk{0, 0, 0, 0};
  int i0 = 0, i1 = 0, j0 = 0, j1 = 0;
  if (u < w_hi) {
    wk = work_at(u);
    i0 = rp[wk.I];
    i1 = rp[wk.I + 1];
    j0 = rp[wk.J];
    j1 = rp[wk.J + 1];
  }
  for (; u < w_hi; u += 4) {
    // The lane's row and half, made opaque per block so that the compiler
    // does not hoist the 16 elements' lane masks and addresses out of the
    // loop (they would not fit in registers).
    int lr = lane;
    asm volatile("" : "+v"(lr));
    const int r = lr & 31, h = lr >> 5;
    // wave-uniform values (kept in scalar registers)
    const int q = uni(wk.q), qT = uni(wk.qT), I = uni(wk.I), J = uni(wk.J);
    const int ri0 = uni(i0), ri1 = uni(i1), rj0 = uni(j0), rj1 = uni(j1);
    const bool diag = (I == J);
    const int un = u + 4;
    BsrWork wn{0, 0, 0, 0};
    if (un < w_hi) wn = work_at(un);
    // first 64 flagged columns of both rows
    const int KI0 = first_cols(ri0, ri1, -1);
    const int KJ0 = first_cols(rj0, rj1, -2);
    // the old block's transpose X_JI, if row J holds it flagged
    int po = -1;
    for (int d0 = rj0; d0 < rj1; d0 += 64) {
      const int KJ = (d0 == rj0) ? KJ0 : first_cols(d0, rj1, -2);
      const unsigned long long mo = __ballot(KJ == I);
      if (mo) {
        po = __builtin_amdgcn_readlane(d0 + lane, __ffsll(static_cast<long long>(mo)) - 1);
        break;
      }
    }
    // the old block's elements of this lane: X_IJ[m][r] = X_JI[r][m] for
    // m = 8 a + 4 h + e are four consecutive floats of the stored X_JI per a
    // (one coalesced 16-byte load each), in flight during the products
    floatx4 xo4[4];
    if (po >= 0) {
      const float* ob = A.val + static_cast<size_t>(po) * BE;
      for (int a = 0; a < 4; ++a)
        xo4[a] = *gro(reinterpret_cast<const floatx4*>(ob + ((2 * a + h) & 3) * 256 +
                                                       (r + 32 * (a >> 1)) * 4));
    } else {
      for (int a = 0; a < 4; ++a) xo4[a] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    floatx16 acc;
    for (int j = 0; j < 16; ++j) acc[j] = 0.f;
    for (int c0 = ri0; c0 < ri1; c0 += 64) {
      const int K = (c0 == ri0) ? KI0 : first_cols(c0, ri1, -1);
      const bool vi = K >= 0;
      const int pI = c0 + lane;
      int pJ = -1;
      for (int d0 = rj0; d0 < rj1; d0 += 64) {
        const int KJ = (d0 == rj0) ? KJ0 : first_cols(d0, rj1, -2);
        const int PJ = d0 + lane;
        const int m = min(64, rj1 - d0);
        for (int t = 0; t < m; ++t) {
          const int kt = __builtin_amdgcn_readlane(KJ, t);
          const int pt = __builtin_amdgcn_readlane(PJ, t);
          if (K == kt) pJ = pt;
        }
      }
      unsigned long long mask = __ballot(vi && pJ >= 0);
      const int np = __popcll(mask);
      nprod += np;
      if (!np) continue;
      // Products in mask order, in pairs, through two operand sets: while
      // one set's MFMAs run, the other set's loads are in flight. Every pair
      // but the last is a loop iteration that also loads the next pair;
      // loads past the last product repeat its blocks. With a single exit
      // from the loop and the same loads outstanding on every path, each
      // wait covers only the set it uses. (The empty asm with a memory
      // clobber keeps each set's loads where they are issued, and the
      // scheduling barrier keeps the other set's MFMAs after them.)
      int src = __ffsll(static_cast<long long>(mask)) - 1;
      auto next_src = [&]() {
        if (mask) {
          src = __ffsll(static_cast<long long>(mask)) - 1;
          mask &= mask - 1;
        }
        return src;
      };
      auto load_pair = [&](int sl, floatx4 (&xa)[4], floatx4 (&xb)[4]) {
        load_block_frag(A.val, __builtin_amdgcn_readlane(pI, sl), lr, xa);
        load_block_frag(A.val, __builtin_amdgcn_readlane(pJ, sl), lr, xb);
      };
      auto mfma16 = [&](const floatx4 (&xa)[4], const floatx4 (&xb)[4]) {
        for (int s = 0; s < 16; ++s)
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(xa[s >> 2][s & 3], xb[s >> 2][s & 3],
                                                     acc, 0, 0, 0);
      };
      floatx4 fa[4], fb[4], ga[4], gb[4];
      load_pair(next_src(), fa, fb);
      load_pair(next_src(), ga, gb);
      asm volatile("" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
      const int pairs = (np + 1) >> 1;
      for (int pp = 1; pp < pairs; ++pp) {
        mfma16(fa, fb);
        load_pair(next_src(), fa, fb);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        mfma16(ga, gb);
        load_pair(next_src(), ga, gb);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
      }
      mfma16(fa, fb);
      if (!(np & 1)) mfma16(ga, gb);
    }
    // acc[j] is element (m, r) of S_IJ, m = 8 (j/4) + 4 h + j%4
    float xo[16];
    for (int a = 0; a < 4; ++a)
      for (int e = 0; e < 4; ++e) xo[4 * a + e] = xo4[a][e];
    // the next block's row extents load during this epilogue
    int ni0 = 0, ni1 = 0, nj0 = 0, nj1 = 0;
    if (un < w_hi) {
      ni0 = rp[wn.I];
      ni1 = rp[wn.I + 1];
      nj0 = rp[wn.J];
      nj1 = rp[wn.J + 1];
    }
    float* out = B.val + static_cast<size_t>(q) * BE;
    float* outT = B.val + static_cast<size_t>(qT) * BE;
    float* const tl = &tile[wave][0];
    bool nz = false;
    double bsq = 0.0;   // squared Frobenius norm of this block of X~ - S
    float xs[16];
    if (!diag) {
      // off the diagonal: every element counts twice (the block and its
      // transpose), no identity terms; |x| < tau tested as |x| <= tf
      double e2 = 0.0, x2 = 0.0;
      for (int j = 0; j < 16; ++j) {
        const float s = acc[j];
        const double d = __builtin_fma(k.es, static_cast<double>(s),
                                       k.ey * static_cast<double>(xo[j]));
        e2 = __builtin_fma(d, d, e2);
        float xn = __builtin_fmaf(kb, xo[j], ka * s);
        if (!(__builtin_fabsf(xn) > tf)) xn = 0.f;
        const double xd = static_cast<double>(xn);
        x2 = __builtin_fma(xd, xd, x2);
        if (stretch) xn = static_cast<float>(k.an * xd);
        nz = nz || (xn != 0.f);   // the stored block, the next step's operand
        xs[j] = xn;
      }
      sv += 2.0 * e2;
      st2 += 2.0 * x2;
      bsq = e2;
      // the transposed block: elements (r, m) for four consecutive m are
      // consecutive in storage
      for (int a = 0; a < 4; ++a) {
        floatx4 v4;
        for (int e = 0; e < 4; ++e) v4[e] = xs[4 * a + e];
        *grw(reinterpret_cast<floatx4*>(outT + ((2 * a + h) & 3) * 256 + (r + 32 * (a >> 1)) * 4)) = v4;
      }
      // the block itself through the tile: element (m, r) at m * 36 + r
      for (int j = 0; j < 16; ++j) tl[(8 * (j >> 2) + 4 * h + (j & 3)) * kTileLd + r] = xs[j];
    } else {
      for (int j = 0; j < 16; ++j) {
        const int m = 8 * (j >> 2) + 4 * h + (j & 3);   // row in the block
        const int c = r;                                // column in the block
        xs[j] = 0.f;
        if (m > c) continue;
        const float s = acc[j];
        // identity terms only inside the matrix proper
        const bool on = (m == c && I * BS + m < n);
        const double d = __builtin_fma(k.es, static_cast<double>(s),
                                       k.ey * static_cast<double>(xo[j])) +
                         (on ? k.ei : 0.0);
        const double w = (m == c) ? 1.0 : 2.0;
        sv += w * d * d;
        bsq += w * d * d;
        float xn = __builtin_fmaf(kb, xo[j], ka * s);
        double xd = static_cast<double>(xn);
        if (fabs(xd) < tau) {
          xn = 0.f;
          xd = 0.0;
        }
        st2 += w * xd * xd;
        if (m == c) st1 += xd;
        if (stretch) xn = static_cast<float>(__builtin_fma(k.an, xd, on ? k.cn : 0.0));
        nz = nz || (xn != 0.f);   // the stored block, the next step's operand
        xs[j] = xn;
      }
      // upper elements and their mirror images, through the tile
      for (int j = 0; j < 16; ++j) {
        const int m = 8 * (j >> 2) + 4 * h + (j & 3);
        if (m <= r) tl[m * kTileLd + r] = xs[j];
        if (m < r) tl[r * kTileLd + m] = xs[j];
      }
    }
    // Storage panel u of the block is one contiguous 1 KiB: lane l = m + 32 g
    // writes row m, columns 16 g + 4 u .. + 3 (a 16-byte read of the tile).
    {
      const int m = lr & 31, g = lr >> 5;
      for (int u4 = 0; u4 < 4; ++u4) {
        const floatx4 v = *reinterpret_cast<const floatx4*>(tl + m * kTileLd + 16 * g + 4 * u4);
        *grw(reinterpret_cast<floatx4*>(out + 256 * u4 + 4 * lr)) = v;
      }
    }
    const int any = __any(nz) ? 1 : 0;
    if (lane == 0) {
      B.flag[q] = any;
      B.flag[qT] = any;
    }
    if (blk) {
      // mixed norm: one value per block of the output pattern
      bsq = wave_sum(bsq);
      if (lane == 0) {
        const float bn = static_cast<float>(sqrt(bsq));
        *grw(blk + q) = bn;
        *grw(blk + qT) = bn;
      }
    }
    wk = wn;
    i0 = ni0;
    i1 = ni1;
    j0 = nj0;
    j1 = nj1;
  }
  sv = wave_sum(sv);
  st1 = wave_sum(st1);
  st2 = wave_sum(st2);
  if (lane == 0) {
    wsum[wave][0] = sv;
    wsum[wave][1] = st1;
    wsum[wave][2] = st2;
    shp[wave] = nprod;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    prod_wg[static_cast<size_t>(iter) * gridDim.x + blockIdx.x] =
        static_cast<uint32_t>(shp[0] + shp[1] + shp[2] + shp[3]);
    for (int v = 0; v < 3; ++v)
      part[3 * blockIdx.x + v] = ((wsum[0][v] + wsum[1][v]) + wsum[2][v]) + wsum[3][v];
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
    // stored: the matrix of step 1 (a X~_0 + c I with a stretch); the flag
    // describes the stored block
    const float xst =
        (stretch && !trivial)
            ? static_cast<float>(__builtin_fma(m1.a, xd,
                                               (gi == gj && gi < n) ? m1.c : 0.0))
            : xs;
    X.val[static_cast<size_t>(q) * BE + blk_off(m, c)] = xst;
    t2 += xd * xd;
    if (gi == gj) t1 += xd;
    nz = nz || (xst != 0.f);
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
          (static_cast<double>(src[blk_off(i, j)]) - (on ? m.c : 0.0)) / m.a);
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
            (static_cast<double>(src[blk_off(e / BS, e % BS)]) - (gi == gj ? m.c : 0.0)) /
            m.a);
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
                            hipStream_t s) {
  hipLaunchKernelGGL(bsr_index_kernel, dim3(1), dim3(kScanThreads), 0, s, M,
                     nb, idx);
  return hipGetLastError();
}

hipError_t launch_bsr_symbolic(const BsrMat& A, int nb,
                               const BsrSymbolic& sym, const BsrMat& Q,
                               int32_t cap, BsrCounters* ctr,
                               const DevState* st, int iter, hipStream_t s) {
  const int nbw = (nb + 31) / 32;
  hipLaunchKernelGGL(bsr_symbolic_count_kernel, dim3(nb), dim3(kCountThreads),
                     0, s, A, nb, nbw, sym, ctr, st, iter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bsr_symbolic_fill_kernel, dim3(nb), dim3(64), 0, s, sym,
                     nb, nbw, Q, cap, ctr, st, iter);
  return hipGetLastError();
}

hipError_t launch_bsr_numeric(const BsrMat& A, const BsrMat& B,
                              const BsrSymbolic& sym, BsrCounters* ctr,
                              const Instance* inst, int iter, int n,
                              double* part, int grid, hipStream_t s) {
  hipLaunchKernelGGL(bsr_numeric_kernel, dim3(grid), dim3(256), 0, s, A, B,
                     sym.work, sym.prod_wg, ctr, inst, iter, n, part);
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
