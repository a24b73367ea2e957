// Internal declarations shared by the HIP kernels and the host driver of the
// SP2 library. Not part of the public ABI (include/sp2.h is).
//
// Every run is a batch of independent instances (a single dense run is a
// batch of one). Each instance has its own iterate buffers, device state,
// polynomial choices and stop; all instances advance one step per launch
// sequence, and kernels of an instance that has stopped return at once.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sp2 {

// Pointers into global memory as the kernels use them. Addresses that the
// kernels read from tables in memory are generic to the compiler, which
// then emits flat loads and stores; flat accesses are tracked together with
// LDS accesses, so waiting for an LDS read would also wait for every global
// prefetch in flight. Casting to the global address space gives global
// loads and stores with their own counter.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gro(
    const T* p) {
  return (const __attribute__((address_space(1))) T*)(p);
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* grw(T* p) {
  return (__attribute__((address_space(1))) T*)(p);
}
// Read-only data that no thread writes during the launch, read through the
// constant address space: uniform reads become scalar loads.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* cro(const T* p) {
  return (const __attribute__((address_space(4))) T*)(p);
}

// Largest number of squares one run may compute (public SP2_MAX_ITER_LIMIT).
constexpr int kMaxIter = 200;
// Rows of X_0 per workgroup of the affine-start kernel.
constexpr int kF0Rows = 8;

// Per-instance state kept in device memory. The finalize kernel is its only
// writer during a run; the square kernels read `done` and the polynomial of
// their step from it. Index conventions follow Alg. 2: p[i] is the
// polynomial that produced X~_i (p[0] unused), alpha[i] its stretch (1 in
// Alg. 2, Alg. 4's alpha_i with a schedule), v[k] = ||X~_k - X~_k^2||_F,
// t1[k] = Tr X~_k, t2[k] = Tr X~_k^2, r[k] the observed order at step k.
struct DevState {
  int32_t done;      // 0 while running, 1 once the outcome is fixed
  int32_t status;    // sp2_status of the outcome
  int32_t n;         // index of the returned iterate X~_n
  int32_t squares;   // squares whose partial sums were finalised
  int8_t p[kMaxIter + 2];
  double alpha[kMaxIter + 2];
  double v[kMaxIter + 1];
  // ||X~_k - X~_k^2|| in the norm the stop reads when it is not the
  // Frobenius norm: the mixed norm, or the spectral norm of Alg. 2
  double m[kMaxIter + 1];
  int32_t krylov[kMaxIter + 1];   // Lanczos steps behind m[k]
  double t1[kMaxIter + 2];
  double t2[kMaxIter + 2];
  double r[kMaxIter + 1];
  // epilogue coefficients (StepCoef: ey, es, ei, an, cn) of the next step to
  // run, written by the finalize kernel when it chooses that step's
  // polynomial, and whether that step's output is stretched (an != 1 or
  // cn != 0); precomputed so that the square kernels load them as scalars
  double ecoef[5];
  int32_t stretch;
  int32_t pad;
};

// Outcome of the whole batch, in host-coherent pinned memory, written by the
// finalize kernel with system-scope stores so that the host can see that
// every instance has stopped without copying device memory.
struct HostMirror {
  int32_t all_done;
  int32_t pad[3];
};

// Parameters of the scalar stop/branch logic (Alg. 2; Alg. 4 when a
// schedule is set).
struct StopParams {
  double n_occ;      // number of occupied states
  double n;          // matrix dimension (divergence test Tr X^2 > Tr X + n)
  int32_t branch;    // 0 = trace-nearest, 1 = literal Tr X > n_occ
  int32_t max_iter;  // squares allowed
  int32_t n_min;     // schedule: first step where the stop is tested
  int32_t n_max;     // schedule length; 0 = no schedule (Alg. 2 branch)
  int32_t norm;      // error fed to the stop: 0 Frobenius, 1 mixed, 2 spectral
  int32_t method;    // 0 SP2 (Alg. 2, or Alg. 4 with a schedule), 1 McWeeny
  // McWeeny: first step whose error the stop tests, and the number of steps
  // with a stretch in the table sched_alpha (alpha = 1 after them)
  int32_t mw_first;
  int32_t mw_len;
};

// Edge of the blocks of the mixed norm (the block size of sec. 6), and the
// largest Krylov dimension used to find its spectral norm.
constexpr int kMixedBlock = 32;
constexpr int kLanczosMax = 64;

// Spectral norm of X~ - X~^2 (Alg. 2's e_i) by Lanczos: rows of X~ per work
// chunk, and the per-instance scratch of the process (FP64). ldq is the
// dimension rounded up to whole chunks; vectors are zero past n.
constexpr int kSpecRows = 32;
struct SpecView {
  double* q;      // 2 x ldq: the last two Lanczos vectors (q_j in slot j % 2)
  double* y;      // ldq: X~ u_j (u_j = beta_{j-1} q_j, not yet normalised)
  double* w;      // ldq: E q_j - beta_{j-1} q_{j-1}
  double* part;   // 2 x nch: per chunk q_j . w, by parity of j
  double* nu;     // nch: per chunk u_j . u_j
  double* ta;     // kLanczosMax: diagonal alpha_j of the Lanczos tridiagonal
  double* tb;     // kLanczosMax: off-diagonal beta_j
  double* misc;   // [0] previous estimate, [1] nonzero once final
};
__host__ __device__ __forceinline__ int spec_ldq(int n) {
  return (n + kSpecRows - 1) / kSpecRows * kSpecRows;
}
__host__ __device__ __forceinline__ size_t spec_doubles(int n) {
  const size_t ldq = static_cast<size_t>(spec_ldq(n));
  const size_t nch = ldq / kSpecRows;
  const size_t d = 4 * ldq + 3 * nch + 2 * kLanczosMax + 4;
  return (d + 31) / 32 * 32;   // 256-byte aligned blocks
}
__host__ __device__ __forceinline__ SpecView spec_view(double* base, int n) {
  const size_t ldq = static_cast<size_t>(spec_ldq(n));
  const size_t nch = ldq / kSpecRows;
  SpecView v;
  v.q = base;
  v.y = v.q + 2 * ldq;
  v.w = v.y + ldq;
  v.part = v.w + ldq;
  v.nu = v.part + 2 * nch;
  v.ta = v.nu + nch;
  v.tb = v.ta + kLanczosMax;
  v.misc = v.tb + kLanczosMax;
  return v;
}

// The matrix a step squares (Alg. 4; X_s of Alg. McW-ACC, sec. 3). The
// buffer that feeds step i holds Y_i = a X~_{i-1} + c I rather than X~_{i-1}:
//   SP2, p_i = 1:  ((1 - a) I + a X~)^2  ->  c = 1 - a,  X_i = Y^2
//   SP2, p_i = 0:  2 a X~ - (a X~)^2      ->  c = 0,      X_i = 2 Y - Y^2
//   McWeeny:       X_s = a (X~ - I/2) + I/2 -> c = (1 - a)/2, X_i = 3 Y^2 - 2 Y^3
// so every step applies the plain polynomial to the square of the stored
// matrix, whose rounding is not scaled by the stretch. Alg. 2 (and every
// step with the stretch off) has a = 1, c = 0: the buffer holds X~ itself.
struct OpMap {
  double a, c;
};
__host__ __device__ __forceinline__ OpMap op_map(int method, int p, double a) {
  if (method == 1) return OpMap{a, 0.5 * (1.0 - a)};
  return OpMap{a, p ? 1.0 - a : 0.0};
}

// Coefficients of one step's epilogue in terms of the stored Y = a X~ + c I
// and its square S = Y^2 (FP64):
//   error of X~:   X~ - X~^2 = ey Y + es S + ei I, i.e.
//                  ((a + 2c) Y - S - c (a + c) I) / a^2
//   next operand:  Y' = an X~_i + cn I  (the map of the following step)
struct StepCoef {
  double ey, es, ei;
  double an, cn;
};
__host__ __device__ __forceinline__ StepCoef step_coef(OpMap m, OpMap next) {
  const double ia2 = 1.0 / (m.a * m.a);
  return StepCoef{(m.a + 2.0 * m.c) * ia2, -ia2, -m.c * (m.a + m.c) * ia2,
                  next.a, next.c};
}

// One instance as the kernels see it.
struct Instance {
  void* X[2];          // iterate buffers (step i reads X[(i-1)&1])
  // BF16x3 only: the iterate split as H = bf16(x), L = bf16(x - H), same
  // layout as X, written by the affine start and by the epilogues of the
  // kernel families that read them (null otherwise)
  void* XH[2];
  void* XL[2];
  // McWeeny only: the square S = X~^2 of the step (same layout as X) and
  // its BF16x3 split (null otherwise)
  void* S;
  void* SH;
  void* SL;
  const double* F;     // input, FP64, row-major
  int64_t ldf;
  int n;               // matrix dimension
  int ld;              // row stride of the iterate buffers: the padded
                       // dimension (multiple of the tile edge) or more
  int tile0, ntiles;   // range of this instance in the tile table
  int f0blk0, nf0blk;  // range of its affine-start blocks
  DevState* st;
  double lmax, width;  // lambda_max, lambda_max - lambda_min
  double tau;          // truncation threshold (0 = off)
  StopParams prm;
  // schedule of Alg. 3, entries 1..prm.n_max (null without a schedule); for
  // McW-ACC sched_alpha holds the stretches of steps 1..prm.mw_len
  const int8_t* sched_p;
  const double* sched_alpha;
  // Mixed norm (null unless prm.norm == 1): Frobenius norms of the 32 x 32
  // blocks of X~_{i-1} - S, written by the step's epilogues. Dense: an
  // nbk x nbk row-major matrix (nbk = ld / 32). Block-sparse: one value per
  // block of the step's output pattern, whose row pointers and columns are
  // brp/bcol[i & 1] (nbk block rows).
  float* blk;
  double* lz;        // Lanczos basis of the mixed norm: 64 x nbk doubles
  int nbk;
  int pad_blk;
  const int32_t* brp[2];
  const int32_t* bcol[2];
  // Block-sparse instance (null for dense ones): flags and 32 x 32 FP32
  // values of the two iterate buffers, whose row pointers and columns are
  // brp/bcol (step i reads buffer (i-1)&1)
  const int32_t* bflag[2];
  const float* bval[2];
  // Spectral norm (null unless prm.norm == 2): Lanczos scratch (spec_view)
  // and the instance's range in the chunk table of the spectral launch
  double* sp;
  int sp_ch0, sp_nch;
};

// The map of step i from the schedule tables alone (no device state): the
// SP2-ACC schedule of Alg. 3 for steps 1..n_max, the McW-ACC stretches for
// steps 1..mw_len, else a = 1, c = 0 (Alg. 2, and after a schedule).
__device__ __forceinline__ OpMap step_map(const Instance& in, int i) {
  if (in.prm.method == 1)
    return op_map(1, 1, (i >= 1 && i <= in.prm.mw_len) ? in.sched_alpha[i] : 1.0);
  if (in.prm.n_max > 0 && i >= 1 && i <= in.prm.n_max)
    return op_map(0, in.sched_p[i], in.sched_alpha[i]);
  return OpMap{1.0, 0.0};
}

// One unit of work of a square launch, given per workgroup by the host:
// inst/slot = instance and global tile index (slot -1: idle), piece =
// workspace index of a K-range piece of a tail tile (-1: whole tile),
// K slices [k0, k1).
struct WorkItem {
  int32_t inst;
  int32_t slot;
  int32_t piece;
  int32_t k0;
  int32_t k1;
  int32_t pad;
};

// A tile whose K range was split into pieces; pieces piece0 .. piece0+split-1.
struct TailItem {
  int32_t inst;
  int32_t slot;
  int32_t piece0;
  int32_t pad;
};

// One workgroup of the affine start: instance and first row.
struct F0Item {
  int32_t inst;
  int32_t row0;
};

// Alg. 3 on the host: fills p[i-1], alpha[i-1] for steps i = 1..n_max
// (arrays of at least `cap` entries, or null) and returns 0, or -1 for
// bounds out of order / overlapping, -2 for a schedule longer than `cap` or
// kMaxIter steps.
int acc_schedule(double lmin, double lmax, double homo_out, double homo_in,
                 double lumo_in, double lumo_out, bool accelerate, int cap,
                 int* n_min, int* n_max, int8_t* p, double* alpha);

// A compiled square-kernel configuration.
struct KernelConfig {
  int precision;   // sp2_precision
  int bm;          // macro tile edge
  int wm, wn;      // waves along M and N
  int bk;          // K slice staged per LDS buffer
  int threads;     // workgroup size
  int occupancy;   // workgroups per CU the configuration is built for
  const char* name;  // family, tile, waves and K slice, e.g. "B3P_256_2x4_32"
  // 1: the main loop reads only the bf16 split of the iterate, so the FP32
  // iterate's lower triangle is not read by the next square
  int presplit;
};

// Arguments of one square step of one launch group (instances sharing a
// kernel configuration).
struct SquareArgs {
  const Instance* inst;
  const int2* tiles;          // tile table (I, J), I <= J, per instance
  const WorkItem* items;      // one per workgroup of the main launch
  const TailItem* tails;      // one per workgroup of the tail launch
  void* ws;                   // tail-piece accumulators (FP32 or FP64)
  int ntail;                  // tail tiles (0: no tail launch)
  int split;                  // pieces per tail tile
  int iter;                   // step i: X~_{i-1} -> X~_i
  int mode;                   // 0 SP2 step; McWeeny: 1 S = X~^2, 2 T = X~ S
  // 1: the run stretches the matrices it squares (SP2-ACC schedule or
  // McW-ACC): the kernels read the step's coefficients from the state
  int stretch;
  // 1: the epilogues write the mirror (lower triangle) of the FP32 output;
  // 0: only its bf16 split (configurations with presplit operands, when
  // nothing else reads the FP32 lower triangle during the run)
  int mirror32;
  double* part;   // 3 doubles per tile (global slot): ||X - S||_F^2, Tr, sum x^2
  double* bpart;  // 3 doubles per band of 32 rows of every tail tile
  int* bcnt;      // per tail tile: bands finished (0 between launches)
};

// Persistent batch: one launch runs every step of every instance. Work
// items (instance, tile, step) sit in a queue in device memory; a workgroup
// takes the next index, waits until that item is published, computes the
// tile, and the workgroup that finishes the last tile of an instance's step
// runs that instance's scalar step and publishes the tiles of its next step.
struct PItem {
  int32_t inst;
  int32_t slot;   // global tile index
  int32_t iter;   // step i: X~_{i-1} -> X~_i
  int32_t seq;    // index + 1 once the item is published (0 before)
};
struct PQueue {
  PItem* items;
  int32_t cap;          // items available (every step of every instance)
  int32_t count;        // instances
  int32_t* ctl;         // [0] next index to take, [1] next index to publish,
                        // [2] nonzero once a wait exceeded its limit
  int32_t* cnt;         // per instance: tiles of its current step finished
  int32_t* ndone;       // instances with an outcome
  HostMirror* mirror;
  long long wait_limit; // constant-clock ticks a workgroup waits for an item
};
// Configurations (0-based ids) the persistent kernel is compiled for.
bool persist_supported(int cfg);
// Workgroups of the persistent kernel that fit on the device at once.
int persist_grid(int cfg, bool stretch, int num_cus);
// Clears the queue and publishes step 1 of every instance still running
// after the affine start's finalize.
hipError_t launch_persist_seed(const Instance* inst, int count, const PQueue& q,
                               hipStream_t s);
hipError_t launch_persist(int cfg, const SquareArgs& a, const PQueue& q,
                          int grid, hipStream_t s);

// Arguments of one spectral-norm launch: every running instance with a
// chunk table entry (instance, first row) per kSpecRows rows.
struct SpecArgs {
  const Instance* inst;
  const int2* chunks;
  int nchunks;
  int count;          // instances of the batch
  int iter;           // step i: the norm of X~_{i-1}, written to m[i-1]
  int vec_cap;        // doubles of dynamic LDS for the product's input vector
  // kSpecCtl counters, zero at launch: [0] instances whose estimate is
  // final
  int32_t* ctl;
};
constexpr int kSpecCtl = 1;
// Largest input vector (doubles) staged in LDS; longer rows read it from
// global memory.
constexpr int kSpecLdsVec = 8192;

// Host-side launchers (implemented in the .hip files).
// Clears the states and the batch's done counter; `zero` (may be null)
// names `nzero` further counters to clear.
hipError_t launch_state_reset(DevState* st, int count, int32_t* ndone,
                              int32_t* zero, int nzero, hipStream_t s);
// One cooperative launch of `grid` workgroups (at most spectral_max_grid)
// with a.vec_cap doubles of dynamic LDS.
hipError_t launch_spectral(const SpecArgs& a, bool fp64_store, int grid,
                           hipStream_t s);
// Workgroups of the spectral kernel that fit on the device at once with
// vec_cap doubles of dynamic LDS each.
int spectral_max_grid(bool fp64_store, int num_cus, int vec_cap);
hipError_t launch_f0(const Instance* inst, const F0Item* items, int nitems,
                     bool fp64_store, double* part_f0, hipStream_t s);
hipError_t launch_finalize(const Instance* inst, int count,
                           const double* part, const double* part_f0,
                           int32_t* ndone, HostMirror* mirror, int iter,
                           hipStream_t s);
// symmetric = true rebuilds the lower triangle from the upper one (for
// iterates whose FP32 mirror was not written).
// D = (X - c I) / a (a = 1, c = 0 copies): the returned iterate X~_n from
// its buffer, which holds the operand a X~_n + c I of the following step.
hipError_t launch_copy_out(const void* X, bool fp64_store, int n, int ldx,
                           void* D, int64_t ldd, bool out_fp64, bool symmetric,
                           OpMap m, hipStream_t s);

// ---- Block-sparse (BSR, 32 x 32 FP32 blocks) path.
constexpr int kBsrBlock = 32;
constexpr int kMaxBlockCols = 2048;   // block rows/columns: n <= 65536

// One block-sparse iterate: both triangles stored, columns sorted per row.
// Storage order of the 1024 elements of a block: four panels of 256 floats;
// panel u holds, for each of the 64 (row m, half g) pairs in the order
// m + 32 g, the four columns 16 g + 4 u .. 16 g + 4 u + 3. Lane l = m + 32 g
// of a wave thus reads the 16 elements of its row and half as four 16-byte
// loads at u * 256 + 4 l, each instruction one contiguous 1 KiB, which is
// the operand layout of the 32 x 32 x 2 MFMA over a block row.
__host__ __device__ constexpr int blk_off(int m, int c) {
  return ((c & 15) >> 2) * 256 + (m + 32 * (c >> 4)) * 4 + (c & 3);
}

struct BsrMat {
  int32_t* row_ptr;   // nb + 1
  int32_t* col;       // capacity
  int32_t* brow;      // capacity: block row of each stored block
  float* val;         // capacity * 32 * 32, element (m, c) at blk_off(m, c)
  int32_t* flag;      // capacity: 1 if the block holds a nonzero
};

// Nonzero blocks of an iterate, per row: columns and storage positions.
struct BsrIndex {
  int32_t* ptr;       // nb + 1
  int32_t* col;
  int32_t* pos;
};

// One upper block (J >= I) of the pattern being built: its storage position,
// the position of its transpose (J, I), and its block row and column.
struct BsrWork {
  int32_t q, qT, I, J;
};

// Symbolic product buffers: per block row, the bitmap of the pattern's
// columns, the exclusive prefix of the bitmap words' popcounts, the counts
// of all and of upper blocks, and the row pointers of the upper work list.
struct BsrSymbolic {
  uint32_t* bitmap;   // nb x nbw
  int32_t* wpre;      // nb x nbw
  int32_t* qcnt;      // nb
  int32_t* ucnt;      // nb
  int32_t* nzrow;     // nb: flagged blocks per row of the iterate
  BsrWork* work;      // capacity
  // block products of each numeric workgroup per step ((kMaxIter + 2) x
  // grid), summed on the host after the run (no same-address atomics)
  uint32_t* prod_wg;
};

struct BsrCounters {
  int32_t nnzb;       // stored blocks of the pattern being built
  int32_t overflow;   // 1: capacity exceeded; 2: pattern not symmetric
  int32_t nupper;     // upper blocks of that pattern (work list length)
  int32_t pad;
  // per step i: blocks of the pattern of X~_i, flagged blocks of X~_{i-1},
  // and block products X_IK X_JK^T computed (filled in on the host from
  // BsrSymbolic::prod_wg)
  int32_t stored[kMaxIter + 2];
  int32_t nonzero[kMaxIter + 2];
  unsigned long long products[kMaxIter + 2];
};

hipError_t launch_bsr_reset(BsrCounters* ctr, hipStream_t s);
// Index of the flagged blocks of M per row (extraction of the result).
hipError_t launch_bsr_index(const BsrMat& M, int nb, const BsrIndex& idx,
                            hipStream_t s);
// Symbolic product of step iter from the flagged blocks of A: the pattern Q
// and the upper work list; counts A's flagged blocks in ctr->nonzero[iter].
hipError_t launch_bsr_symbolic(const BsrMat& A, int nb,
                               const BsrSymbolic& sym, const BsrMat& Q,
                               int32_t cap, BsrCounters* ctr,
                               const DevState* st, int iter, hipStream_t s);
hipError_t launch_bsr_numeric(const BsrMat& A, const BsrMat& B,
                              const BsrSymbolic& sym, BsrCounters* ctr,
                              const Instance* inst, int iter, int n,
                              double* part, int grid, hipStream_t s);
hipError_t launch_bsr_f0(const double* F, const BsrMat& X, int nnzb,
                         const Instance* inst, int n, double* part,
                         hipStream_t s);
// The returned block-sparse iterate as (x - c [diagonal]) / a from its
// stored matrix (OpMap m of the following step).
hipError_t launch_bsr_gather(const BsrMat& M, const int32_t* pos, int cnt,
                             int n, OpMap m, void* out, bool fp64,
                             hipStream_t s);
hipError_t launch_bsr_to_dense(const float* val, const BsrIndex& idx, int nb,
                               int n, OpMap m, void* D, int64_t ldd, bool fp64,
                               hipStream_t s);

int kernel_config_count();
const KernelConfig* kernel_config(int id);   // id in [0, count)
// Launches the main square kernel of configuration `id` with `grid`
// workgroups, then (if a.ntail > 0) the tail reduction kernel.
hipError_t launch_square(int id, const SquareArgs& a, int grid, hipStream_t s);

}  // namespace sp2
