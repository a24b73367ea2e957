// Host driver and C ABI of the SP2 library (see include/sp2.h).
//
// Every run is a batch of instances (sp2_init_dense prepares a batch of
// one). A run is a stream-ordered sequence of kernels:
//   state reset -> f0 (X_0 and its traces, all instances) -> finalize(0)
//   -> for i = 1, 2, ...: square(i) per launch group -> finalize(i)
// A launch group is the set of instances that share a square-kernel
// configuration. The polynomial choices, the stop tests and the outcomes
// live in device memory (one DevState per instance); the finalize kernel
// counts stopped instances and tells the host, through host-coherent pinned
// memory, when all have stopped. The host keeps up to kLookahead steps
// queued ahead of the step whose outcome it last observed, so the device
// never waits on the host; steps queued after the stop return at once
// because every kernel first reads its instance's done flag.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/sp2.h"
#include "host_plan.h"
#include "sp2_device.h"

using sp2::DevState;
using sp2::HostMirror;
using sp2::Instance;
using sp2::Plan;
using sp2::append_tile_list;
using sp2::make_plan;
using sp2::row_stride;

namespace {

constexpr int kLookahead = 3;
constexpr int kRing = 8;

// Instance as the host keeps it.
struct HostInst {
  const double* F = nullptr;
  int64_t n = 0, ldf = 0, n_occ = 0, np = 0;
  int64_t ld = 0;              // row stride of the iterate buffers (>= np)
  double lmin = 0.0, lmax = 0.0;
  int cfg = 0;                 // 0-based kernel configuration id
  size_t xoff = 0;             // element offset in the iterate pools
  bool trivial = false;        // n_occ == 0 or n_occ == n
};


// Instances sharing one kernel configuration, with their work plan.
struct Group {
  int cfg = 0;
  int grid = 0;
  int ntail = 0, split = 1;
  sp2::WorkItem* items = nullptr;   // device
  sp2::TailItem* tails = nullptr;   // device
  size_t items_cap = 0, tails_cap = 0;
};

}  // namespace

struct sp2_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int num_cus = 256;

  // configuration table: (precision, n_max, 0-based config id)
  struct TableEntry {
    int precision;
    int64_t n_max;
    int cfg;
  };
  std::vector<TableEntry> table;

  // problem
  sp2_options opt{};
  bool fp64_store = true;
  std::vector<HostInst> hi;
  std::vector<Group> groups;

  // device workspaces
  void* pool[2] = {nullptr, nullptr};
  size_t pool_cap[2] = {0, 0};
  void* split_pool[4] = {nullptr, nullptr, nullptr, nullptr};   // H0 L0 H1 L1
  size_t split_cap[4] = {0, 0, 0, 0};
  // McWeeny: the square S of every instance, and its split (BF16x3)
  void* s_pool = nullptr;
  size_t s_pool_cap = 0;
  void* s_split[2] = {nullptr, nullptr};
  size_t s_split_cap[2] = {0, 0};
  bool mcweeny = false;
  // some instance's schedule stretches a step (alpha != 1): the square
  // kernels with the stretch coefficients run
  bool stretch = false;
  Instance* d_inst = nullptr;
  size_t d_inst_cap = 0;
  std::vector<Instance> h_inst;    // host copy of the instance table
  void* d_sched = nullptr;         // SP2-ACC schedules: alphas, then p's
  size_t d_sched_cap = 0;
  // host copies of the schedule tables (kMaxIter + 2 entries per instance):
  // SP2-ACC's p and alpha, or McW-ACC's alpha
  std::vector<double> h_sched_alpha;
  std::vector<int8_t> h_sched_p;
  float* d_blk = nullptr;          // block norms of the mixed norm
  size_t d_blk_cap = 0;
  double* d_lz = nullptr;          // Lanczos bases of the mixed norm
  size_t d_lz_cap = 0;
  // spectral norm: Lanczos scratch of every instance, the chunk table of the
  // spectral launch, and one counter of final estimates per step
  double* d_spec = nullptr;
  size_t d_spec_cap = 0;
  int2* d_spec_chunks = nullptr;
  size_t d_spec_chunks_cap = 0;
  int32_t* d_spec_ctl = nullptr;
  size_t d_spec_ctl_cap = 0;
  int spec_nchunks = 0;
  int spec_grid = 0;
  int spec_vec_cap = 0;
  DevState* d_st = nullptr;
  size_t d_st_cap = 0;
  int2* d_tiles = nullptr;
  size_t d_tiles_cap = 0;
  double* d_part = nullptr;
  size_t d_part_cap = 0;
  double* d_part_f0 = nullptr;
  size_t d_part_f0_cap = 0;
  sp2::F0Item* d_f0 = nullptr;
  size_t d_f0_cap = 0;
  int nf0 = 0;
  void* d_ws = nullptr;
  size_t d_ws_cap = 0;
  double* d_bpart = nullptr;       // tail bands' partial sums
  size_t d_bpart_cap = 0;
  int* d_bcnt = nullptr;           // tail tiles' band counters
  size_t d_bcnt_cap = 0;
  int32_t* d_ndone = nullptr;
  HostMirror* mirror = nullptr;
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
  hipEvent_t ev_ring[kRing] = {};
  std::vector<hipEvent_t> ev_sq;   // pairs around each step's squares
  std::vector<float> square_ms;
  std::vector<hipEvent_t> ev_nm;   // pairs around each step's spectral launch
  std::vector<float> norm_ms;
  bool timed = false;

  // block-sparse mode
  bool bsr = false;
  struct {
    int64_t n = 0;
    int nb = 0, nnzb_in = 0, cap = 0, grid = 0;
    const double* F = nullptr;
    sp2::BsrMat m[2] = {};
    sp2::BsrIndex idx = {};
    sp2::BsrSymbolic sym = {};
    sp2::BsrCounters* ctr = nullptr;
    sp2::BsrCounters host_ctr = {};   // counters of the last run
    size_t bytes = 0;              // bytes of the allocation below
    void* mem = nullptr;           // one allocation holding all of the above
  } b;

  // persistent driver (SP2_LAUNCH_PERSISTENT): the configuration every
  // instance uses, the queue, and the captured graph of a run
  bool persistent = false;
  int pcfg = 0;
  int pgrid = 0;
  sp2::PItem* d_pitems = nullptr;
  size_t d_pitems_cap = 0;
  int32_t pitems = 0;
  int32_t* d_pctl = nullptr;       // 4 counters
  size_t d_pctl_cap = 0;
  int32_t* d_pcnt = nullptr;       // per instance
  size_t d_pcnt_cap = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  long long wall_khz = 100000;     // rate of the kernels' constant clock
  long long wait_ms = 2000;        // longest wait of a workgroup for an item

  // Workspace arena of the no-allocation entry point (null for contexts made
  // by sp2_create): every workspace is carved from it instead of allocated.
  char* arena = nullptr;
  size_t arena_cap = 0, arena_off = 0;

  // outcome
  bool inited = false, ran = false;
  double run_ms = 0.0;
  int32_t steps = 0;               // squares of the longest instance
  std::vector<DevState> host_state;
};

namespace {

// Device memory for a workspace of at least `bytes`. A context made by
// sp2_create allocates with hipMalloc and replaces a buffer only when a
// larger one is needed; a context of the no-allocation entry point carves
// every workspace from its arena (256-byte aligned) and reports
// hipErrorOutOfMemory when the arena is full.
template <typename P>
hipError_t grow(sp2_ctx c, P*& ptr, size_t& cap, size_t bytes, hipStream_t s) {
  if (bytes <= cap) return hipSuccess;
  if (c->arena) {
    const size_t off = (c->arena_off + 255) / 256 * 256;
    if (bytes > c->arena_cap || off > c->arena_cap - bytes)
      return hipErrorOutOfMemory;
    ptr = reinterpret_cast<P*>(c->arena + off);
    cap = bytes;
    c->arena_off = off + bytes;
    return hipSuccess;
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  cap = 0;
  e = hipMalloc(reinterpret_cast<void**>(&ptr), bytes);
  if (e == hipSuccess) cap = bytes;
  return e;
}

sp2_status fail(sp2_ctx c, sp2_status s, const char* what, hipError_t e) {
  if (c) {
    c->err = what;
    if (e != hipSuccess) {
      c->err += ": ";
      c->err += hipGetErrorString(e);
    }
  }
  return s;
}

#define SP2_HIP(ctx, call)                                            \
  do {                                                                \
    hipError_t e_ = (call);                                           \
    if (e_ != hipSuccess) {                                           \
      return fail((ctx), e_ == hipErrorOutOfMemory ? SP2_OUT_OF_MEMORY \
                                                   : SP2_HIP_ERROR,   \
                  #call, e_);                                         \
    }                                                                 \
  } while (0)

// Library choice of square-kernel configuration (0-based id) for one
// instance of dimension n, from timings of every configuration on MI355X
// at n = 4096 and 8192 (128 x 128 tiles with 2 x 4 waves for FP64/FP32;
// for BF16x3 the swizzled 256 x 256 tile with 2 x 4 waves at n = 8192 and
// the swizzled 128 x 128 tile below). An autotuned table installed with
// sp2_set_kernel_table takes precedence.
int default_config(int precision, int64_t n) {
  switch (precision) {
    case SP2_FP64: return n >= 1024 ? 0 : 2;
    case SP2_FP32: return n >= 1024 ? 4 : 3;
    default: return n >= 6144 ? 13 : 11;
  }
}

sp2_status ensure_events(sp2_ctx c) {
  if (c->ev_start) return SP2_OK;
  SP2_HIP(c, hipEventCreate(&c->ev_start));
  SP2_HIP(c, hipEventCreate(&c->ev_stop));
  for (int i = 0; i < kRing; ++i)
    SP2_HIP(c, hipEventCreateWithFlags(&c->ev_ring[i], hipEventDisableTiming));
  return SP2_OK;
}

sp2_status validate_options(sp2_ctx c, sp2_options& opt) {
  if (opt.max_iter == 0) opt.max_iter = 100;
  if (opt.precision < SP2_FP64 || opt.precision > SP2_BF16X3)
    return fail(c, SP2_INVALID_ARG, "unknown precision", hipSuccess);
  if (opt.branch != SP2_BRANCH_NEAREST && opt.branch != SP2_BRANCH_LITERAL)
    return fail(c, SP2_INVALID_ARG, "unknown branch rule", hipSuccess);
  if (!(opt.trunc_tau >= 0.0) || !isfinite(opt.trunc_tau))
    return fail(c, SP2_INVALID_ARG, "trunc_tau must be finite and >= 0",
                hipSuccess);
  if (opt.max_iter < 1 || opt.max_iter > SP2_MAX_ITER_LIMIT)
    return fail(c, SP2_INVALID_ARG, "max_iter outside [1, SP2_MAX_ITER_LIMIT]",
                hipSuccess);
  if (opt.kernel_config != 0) {
    const sp2::KernelConfig* kc = sp2::kernel_config(opt.kernel_config - 1);
    if (!kc || kc->precision != opt.precision)
      return fail(c, SP2_INVALID_ARG,
                  "kernel_config unknown or of another precision", hipSuccess);
  }
  if (opt.tail_split < 0 || opt.tail_split > 64)
    return fail(c, SP2_INVALID_ARG, "tail_split outside [0, 64]", hipSuccess);
  if (opt.norm != SP2_NORM_FROBENIUS && opt.norm != SP2_NORM_MIXED &&
      opt.norm != SP2_NORM_SPECTRAL)
    return fail(c, SP2_INVALID_ARG, "unknown norm", hipSuccess);
  if (opt.launch < SP2_LAUNCH_AUTO || opt.launch > SP2_LAUNCH_PERSISTENT)
    return fail(c, SP2_INVALID_ARG, "unknown launch mode", hipSuccess);
  if (opt.launch == SP2_LAUNCH_PERSISTENT && opt.norm != SP2_NORM_FROBENIUS)
    return fail(c, SP2_INVALID_ARG,
                "the persistent launch supports the Frobenius norm only",
                hipSuccess);
  return SP2_OK;
}

sp2_status validate_instance(sp2_ctx c, const double* F, int64_t n, int64_t ldf,
                             double lmin, double lmax, int64_t n_occ) {
  if (!F) return fail(c, SP2_INVALID_ARG, "F_dev is NULL", hipSuccess);
  if (n <= 0 || n > 65536)
    return fail(c, SP2_INVALID_ARG, "n must be in [1, 65536]", hipSuccess);
  if (ldf < n) return fail(c, SP2_INVALID_ARG, "ldf < n", hipSuccess);
  if (n_occ < 0 || n_occ > n)
    return fail(c, SP2_INVALID_ARG, "n_occ outside [0, n]", hipSuccess);
  if (!isfinite(lmin) || !isfinite(lmax) || !(lmax > lmin) ||
      !isfinite(lmax - lmin))
    return fail(c, SP2_INVALID_ARG,
                "spectral bounds must be finite with lambda_max > lambda_min",
                hipSuccess);
  return SP2_OK;
}

// Drops the captured run of the persistent driver (its kernel arguments
// name workspaces that a new init may replace).
void release_graph(sp2_ctx c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
}

void release_groups(sp2_ctx c) {
  for (Group& g : c->groups) {
    if (c->arena) continue;   // carved from the arena
    if (g.items) (void)hipFree(g.items);
    if (g.tails) (void)hipFree(g.tails);
  }
  c->groups.clear();
}

// Builds the instance table, tile table, launch groups and their plans, and
// (re)allocates every workspace. Instances come in c->hi.
sp2_status setup(sp2_ctx c) {
  const int count = static_cast<int>(c->hi.size());
  const size_t esz = c->fp64_store ? 8 : 4;
  hipStream_t s = c->stream;
  release_graph(c);
  // configurations, padding, pool offsets
  auto choose = [&](int64_t n) {
    int cfg = c->opt.kernel_config ? c->opt.kernel_config - 1
                                   : default_config(c->opt.precision, n);
    if (!c->opt.kernel_config)
      for (const auto& e : c->table)
        if (e.precision == c->opt.precision && n <= e.n_max) {
          cfg = e.cfg;
          break;
        }
    return cfg;
  };
  // the persistent driver runs every instance with one configuration: the
  // choice for the largest instance when the persistent kernel is compiled
  // for it, else the 64/128-tile default of the precision
  c->persistent =
      !c->arena && c->opt.norm == SP2_NORM_FROBENIUS &&
      (c->opt.launch == SP2_LAUNCH_PERSISTENT ||
       (c->opt.launch == SP2_LAUNCH_AUTO && count > 1));
  if (c->persistent) {
    int64_t nmax = 0;
    for (const HostInst& h : c->hi) nmax = std::max(nmax, h.n);
    int cfg = choose(nmax);
    if (!sp2::persist_supported(cfg)) {
      if (c->opt.kernel_config)
        return fail(c, SP2_INVALID_ARG,
                    "kernel_config is not one the persistent launch is "
                    "compiled for", hipSuccess);
      cfg = c->opt.precision == SP2_FP64 ? 2 : (c->opt.precision == SP2_FP32 ? 4 : 11);
    }
    c->pcfg = cfg;
  }
  size_t pool_elems = 0;
  for (HostInst& h : c->hi) {
    h.cfg = c->persistent ? c->pcfg : choose(h.n);
    const int bm = sp2::kernel_config(h.cfg)->bm;
    h.np = ((h.n + bm - 1) / bm) * bm;
    h.ld = row_stride(h.np);
    h.xoff = pool_elems;
    pool_elems += static_cast<size_t>(h.np) * h.ld;
    pool_elems = (pool_elems + 63) / 64 * 64;   // 256-byte aligned starts
    h.trivial = (h.n_occ == 0 || h.n_occ == h.n);
  }
  for (int q = 0; q < 2; ++q)
    SP2_HIP(c, grow(c, c->pool[q], c->pool_cap[q], pool_elems * esz, s));
  const bool split = (c->opt.precision == SP2_BF16X3);
  if (split)
    for (int q = 0; q < 4; ++q)
      SP2_HIP(c, grow(c, c->split_pool[q], c->split_cap[q], pool_elems * 2, s));

  // block norms of the mixed norm: an (np/32)^2 matrix per instance
  const bool mixed = (c->opt.norm == SP2_NORM_MIXED);
  std::vector<size_t> blk_off(count, 0), lz_off(count, 0);
  size_t blk_elems = 0, lz_elems = 0;
  for (int b = 0; b < count; ++b) {
    blk_off[b] = blk_elems;
    lz_off[b] = lz_elems;
    const size_t nbk = static_cast<size_t>(c->hi[b].np / sp2::kMixedBlock);
    if (mixed) {
      blk_elems += (nbk * nbk + 63) / 64 * 64;
      lz_elems += sp2::kLanczosMax * nbk;
    }
  }
  if (mixed) {
    SP2_HIP(c, grow(c, c->d_blk, c->d_blk_cap, blk_elems * sizeof(float), s));
    SP2_HIP(c, grow(c, c->d_lz, c->d_lz_cap, lz_elems * sizeof(double), s));
  }

  // spectral norm: Lanczos scratch per instance and the chunk table (rows
  // of the non-trivial instances in chunks of kSpecRows)
  const bool spectral = (c->opt.norm == SP2_NORM_SPECTRAL);
  std::vector<size_t> sp_off(count, 0);
  std::vector<int2> chunks;
  std::vector<int> sp_ch0(count, 0), sp_nch(count, 0);
  if (spectral) {
    size_t sp_elems = 0;
    for (int b = 0; b < count; ++b) {
      const HostInst& h = c->hi[b];
      sp_off[b] = sp_elems;
      sp_elems += sp2::spec_doubles(static_cast<int>(h.n));
      if (h.trivial) continue;
      sp_ch0[b] = static_cast<int>(chunks.size());
      for (int r = 0; r < h.n; r += sp2::kSpecRows) chunks.push_back(int2{b, r});
      sp_nch[b] = static_cast<int>(chunks.size()) - sp_ch0[b];
    }
    SP2_HIP(c, grow(c, c->d_spec, c->d_spec_cap, sp_elems * sizeof(double), s));
    SP2_HIP(c, grow(c, c->d_spec_chunks, c->d_spec_chunks_cap,
                    std::max<size_t>(1, chunks.size()) * sizeof(int2), s));
    SP2_HIP(c, grow(c, c->d_spec_ctl, c->d_spec_ctl_cap,
                    (sp2::kMaxIter + 2) * sp2::kSpecCtl * sizeof(int32_t), s));
    if (!chunks.empty())
      SP2_HIP(c, hipMemcpyAsync(c->d_spec_chunks, chunks.data(),
                                chunks.size() * sizeof(int2),
                                hipMemcpyHostToDevice, s));
    // the product's input vector is staged in LDS for rows of up to
    // kSpecLdsVec entries
    int max_ldq = 0;
    for (int b = 0; b < count; ++b)
      if (!c->hi[b].trivial)
        max_ldq = std::max(max_ldq, sp2::spec_ldq(static_cast<int>(c->hi[b].n)));
    c->spec_vec_cap = std::min(max_ldq, sp2::kSpecLdsVec);
    const int gmax =
        sp2::spectral_max_grid(c->fp64_store, c->num_cus, c->spec_vec_cap);
    if (gmax < 1)
      return fail(c, SP2_HIP_ERROR, "spectral kernel: no co-resident grid",
                  hipGetLastError());
    // one workgroup per chunk, plus spare workgroups (one per instance at
    // most) that take the small eigenvalue problems off the products' path
    int active = 0;
    for (int b = 0; b < count; ++b) active += c->hi[b].trivial ? 0 : 1;
    c->spec_grid = std::min<int>(gmax, static_cast<int>(chunks.size()) + active);
  }
  c->spec_nchunks = static_cast<int>(chunks.size());

  // instance table, tiles and affine-start blocks
  SP2_HIP(c, grow(c, c->d_st, c->d_st_cap, count * sizeof(DevState), s));
  std::vector<int2> tiles;
  std::vector<Instance> inst(count);
  std::vector<sp2::F0Item> f0;
  for (int b = 0; b < count; ++b) {
    const HostInst& h = c->hi[b];
    const int bm = sp2::kernel_config(h.cfg)->bm;
    Instance& in = inst[b];
    in.X[0] = static_cast<char*>(c->pool[0]) + h.xoff * esz;
    in.X[1] = static_cast<char*>(c->pool[1]) + h.xoff * esz;
    for (int q = 0; q < 2; ++q) {
      in.XH[q] = split ? static_cast<char*>(c->split_pool[2 * q]) + h.xoff * 2
                       : nullptr;
      in.XL[q] = split ? static_cast<char*>(c->split_pool[2 * q + 1]) + h.xoff * 2
                       : nullptr;
    }
    in.F = h.F;
    in.ldf = h.ldf;
    in.n = static_cast<int>(h.n);
    in.ld = static_cast<int>(h.ld);
    in.tile0 = static_cast<int>(tiles.size());
    append_tile_list(static_cast<int>(h.np / bm), tiles);
    in.ntiles = static_cast<int>(tiles.size()) - in.tile0;
    in.f0blk0 = static_cast<int>(f0.size());
    for (int r = 0; r < h.np; r += sp2::kF0Rows)
      f0.push_back(sp2::F0Item{b, r});
    in.nf0blk = static_cast<int>(f0.size()) - in.f0blk0;
    in.st = c->d_st + b;
    in.lmax = h.lmax;
    in.width = h.lmax - h.lmin;
    in.tau = c->opt.trunc_tau;
    in.prm.n_occ = static_cast<double>(h.n_occ);
    in.prm.n = static_cast<double>(h.n);
    in.prm.branch = c->opt.branch;
    in.prm.max_iter = c->opt.max_iter;
    in.prm.norm = c->opt.norm;
    in.nbk = static_cast<int>(h.np / sp2::kMixedBlock);
    in.blk = mixed ? c->d_blk + blk_off[b] : nullptr;
    in.lz = mixed ? c->d_lz + lz_off[b] : nullptr;
    in.sp = spectral ? c->d_spec + sp_off[b] : nullptr;
    in.sp_ch0 = sp_ch0[b];
    in.sp_nch = sp_nch[b];
  }

  // launch groups: one per configuration in use (trivial instances stop
  // before any square and get no work)
  release_groups(c);
  std::vector<int> cfgs;
  for (const HostInst& h : c->hi)
    if (!h.trivial && std::find(cfgs.begin(), cfgs.end(), h.cfg) == cfgs.end())
      cfgs.push_back(h.cfg);
  size_t ws_elems = 0, max_tail = 0, max_bands = 0;
  for (int cfg : cfgs) {
    const sp2::KernelConfig* kc = sp2::kernel_config(cfg);
    std::vector<int> slots, owner, nk;
    for (int b = 0; b < count; ++b) {
      if (c->hi[b].cfg != cfg || c->hi[b].trivial) continue;
      for (int t = 0; t < inst[b].ntiles; ++t) {
        slots.push_back(inst[b].tile0 + t);
        owner.push_back(b);
        nk.push_back(static_cast<int>(c->hi[b].np / kc->bk));
      }
    }
    Plan pl = make_plan(slots, owner, nk, c->num_cus * kc->occupancy,
                        c->opt.tail_split);
    Group g;
    g.cfg = cfg;
    g.grid = static_cast<int>(pl.items.size());
    g.ntail = static_cast<int>(pl.tails.size());
    g.split = pl.split;
    // Groups run one after another on the stream, so they share one
    // workspace sized for the largest.
    ws_elems = std::max(ws_elems, static_cast<size_t>(g.ntail) * g.split *
                                      kc->bm * kc->bm);
    max_tail = std::max(max_tail, static_cast<size_t>(g.ntail));
    max_bands = std::max(max_bands, static_cast<size_t>(g.ntail) *
                                        (kc->bm / sp2::kMixedBlock));
    c->groups.push_back(g);
    Group& gg = c->groups.back();
    SP2_HIP(c, grow(c, gg.items, gg.items_cap,
                    pl.items.size() * sizeof(sp2::WorkItem), s));
    SP2_HIP(c, hipMemcpyAsync(gg.items, pl.items.data(),
                              pl.items.size() * sizeof(sp2::WorkItem),
                              hipMemcpyHostToDevice, s));
    if (!pl.tails.empty()) {
      SP2_HIP(c, grow(c, gg.tails, gg.tails_cap,
                      pl.tails.size() * sizeof(sp2::TailItem), s));
      SP2_HIP(c, hipMemcpyAsync(gg.tails, pl.tails.data(),
                                pl.tails.size() * sizeof(sp2::TailItem),
                                hipMemcpyHostToDevice, s));
    }
    // the copies read host vectors that go out of scope: finish them now
    SP2_HIP(c, hipStreamSynchronize(s));
  }
  if (ws_elems) SP2_HIP(c, grow(c, c->d_ws, c->d_ws_cap, ws_elems * esz, s));
  if (max_tail) {
    // the counters start at zero and every tail launch leaves them at zero
    SP2_HIP(c, grow(c, c->d_bpart, c->d_bpart_cap,
                    max_bands * 3 * sizeof(double), s));
    const size_t old_cap = c->d_bcnt_cap;
    SP2_HIP(c, grow(c, c->d_bcnt, c->d_bcnt_cap, max_tail * sizeof(int), s));
    if (c->d_bcnt_cap != old_cap || old_cap == 0)
      SP2_HIP(c, hipMemsetAsync(c->d_bcnt, 0, c->d_bcnt_cap, s));
  }
  SP2_HIP(c, grow(c, c->d_inst, c->d_inst_cap, count * sizeof(Instance), s));
  SP2_HIP(c, grow(c, c->d_tiles, c->d_tiles_cap,
                  std::max<size_t>(1, tiles.size()) * sizeof(int2), s));
  SP2_HIP(c, grow(c, c->d_part, c->d_part_cap,
                  std::max<size_t>(1, tiles.size()) * 3 * sizeof(double), s));
  SP2_HIP(c, grow(c, c->d_part_f0, c->d_part_f0_cap,
                  f0.size() * 3 * sizeof(double), s));
  SP2_HIP(c, grow(c, c->d_f0, c->d_f0_cap, f0.size() * sizeof(sp2::F0Item), s));
  SP2_HIP(c, hipMemcpyAsync(c->d_inst, inst.data(), count * sizeof(Instance),
                            hipMemcpyHostToDevice, s));
  c->h_inst = inst;
  c->mcweeny = false;
  c->stretch = false;
  if (!tiles.empty())
    SP2_HIP(c, hipMemcpyAsync(c->d_tiles, tiles.data(),
                              tiles.size() * sizeof(int2),
                              hipMemcpyHostToDevice, s));
  SP2_HIP(c, hipMemcpyAsync(c->d_f0, f0.data(), f0.size() * sizeof(sp2::F0Item),
                            hipMemcpyHostToDevice, s));
  SP2_HIP(c, hipStreamSynchronize(s));
  c->nf0 = static_cast<int>(f0.size());
  if (c->persistent) {
    // every step of every instance can be queued once
    size_t cap = 1;
    for (int b = 0; b < count; ++b)
      if (!c->hi[b].trivial)
        cap += static_cast<size_t>(inst[b].ntiles) * c->opt.max_iter;
    if (cap > static_cast<size_t>(INT32_MAX))
      return fail(c, SP2_INVALID_ARG, "batch too large for the persistent launch",
                  hipSuccess);
    c->pitems = static_cast<int32_t>(cap);
    SP2_HIP(c, grow(c, c->d_pitems, c->d_pitems_cap, cap * sizeof(sp2::PItem), s));
    SP2_HIP(c, grow(c, c->d_pctl, c->d_pctl_cap, 4 * sizeof(int32_t), s));
    SP2_HIP(c, grow(c, c->d_pcnt, c->d_pcnt_cap, count * sizeof(int32_t), s));
  }
  return SP2_OK;
}

// The persistent driver's run, captured once (after every init, and after
// a change of the stretch) on a private stream into a graph that every run
// launches on the context's stream: the state reset, the affine start and
// its scalar step, the queue seeding and the persistent kernel. Errors
// inside the capture end it before returning.
sp2_status capture_persistent(sp2_ctx c) {
  const int count = static_cast<int>(c->hi.size());
  if (!c->cap_stream)
    SP2_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  const int grid = sp2::persist_grid(c->pcfg, c->stretch, c->num_cus);
  if (grid < 1)
    return fail(c, SP2_HIP_ERROR, "persistent kernel: no resident workgroup",
                hipGetLastError());
  c->pgrid = grid;
  sp2::SquareArgs a{};
  a.inst = c->d_inst;
  a.tiles = c->d_tiles;
  a.part = c->d_part;
  a.iter = 1;
  a.mode = 0;
  a.stretch = c->stretch ? 1 : 0;
  a.split = 1;
  a.mirror32 = sp2::kernel_config(c->pcfg)->presplit ? 0 : 1;
  sp2::PQueue q{};
  q.items = c->d_pitems;
  q.cap = c->pitems;
  q.count = count;
  q.ctl = c->d_pctl;
  q.cnt = c->d_pcnt;
  q.ndone = c->d_ndone;
  q.mirror = c->mirror;
  q.wait_limit = c->wait_ms * c->wall_khz;
  hipStream_t cs = c->cap_stream;
  SP2_HIP(c, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  hipError_t e = sp2::launch_state_reset(c->d_st, count, c->d_ndone, nullptr, 0, cs);
  if (e == hipSuccess)
    e = sp2::launch_f0(c->d_inst, c->d_f0, c->nf0, c->fp64_store, c->d_part_f0, cs);
  if (e == hipSuccess)
    e = sp2::launch_finalize(c->d_inst, count, c->d_part, c->d_part_f0,
                             c->d_ndone, c->mirror, 0, cs);
  if (e == hipSuccess) e = sp2::launch_persist_seed(c->d_inst, count, q, cs);
  if (e == hipSuccess) e = sp2::launch_persist(c->pcfg, a, q, grid, cs);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(cs, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(c, SP2_HIP_ERROR, "capturing the persistent run",
                e != hipSuccess ? e : e2);
  }
  c->graph = g;
  SP2_HIP(c, hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
  return SP2_OK;
}

// One run of the persistent driver: the captured graph on the context's
// stream, then the outcome of every instance.
sp2_status run_persistent(sp2_ctx c) {
  const int count = static_cast<int>(c->hi.size());
  hipStream_t s = c->stream;
  if (!c->gexec) {
    const sp2_status st = capture_persistent(c);
    if (st != SP2_OK) return st;
  }
  c->mirror->all_done = 0;
  __atomic_thread_fence(__ATOMIC_SEQ_CST);
  c->timed = false;
  c->square_ms.clear();
  c->norm_ms.clear();
  SP2_HIP(c, hipEventRecord(c->ev_start, s));
  SP2_HIP(c, hipGraphLaunch(c->gexec, s));
  SP2_HIP(c, hipEventRecord(c->ev_stop, s));
  SP2_HIP(c, hipEventSynchronize(c->ev_stop));
  float ms = 0.f;
  SP2_HIP(c, hipEventElapsedTime(&ms, c->ev_start, c->ev_stop));
  int32_t ctl[4] = {0, 0, 0, 0};
  SP2_HIP(c, hipMemcpyAsync(ctl, c->d_pctl, sizeof(ctl), hipMemcpyDeviceToHost, s));
  c->host_state.resize(count);
  SP2_HIP(c, hipMemcpyAsync(c->host_state.data(), c->d_st,
                            count * sizeof(DevState), hipMemcpyDeviceToHost, s));
  SP2_HIP(c, hipStreamSynchronize(s));
  if (ctl[2] != 0)
    return fail(c, SP2_HIP_ERROR,
                "persistent run: a workgroup waited for a queue item longer "
                "than its limit", hipSuccess);
  int32_t steps = 0;
  for (const DevState& h : c->host_state) {
    if (!h.done)
      return fail(c, SP2_BAD_STATE, "run ended without an outcome", hipSuccess);
    steps = std::max(steps, h.squares);
  }
  c->steps = steps;
  c->run_ms = ms;
  c->ran = true;
  return SP2_OK;
}

// Steps enqueued between two looks at the done counter by a context of the
// no-allocation entry point (it has no pinned mirror and no events).
constexpr int kNoAllocChunk = 4;

sp2_status run_batch(sp2_ctx c) {
  SP2_HIP(c, hipSetDevice(c->device));
  if (c->persistent && !c->mcweeny && !c->bsr) return run_persistent(c);
  hipStream_t s = c->stream;
  const int count = static_cast<int>(c->hi.size());
  const bool noalloc = (c->arena != nullptr);
  if (!noalloc) {
    c->mirror->all_done = 0;
    __atomic_thread_fence(__ATOMIC_SEQ_CST);
  }
  const bool timing = c->opt.kernel_timing != 0 && !noalloc;
  if (timing && c->ev_sq.empty()) {
    c->ev_sq.assign(2 * (SP2_MAX_ITER_LIMIT + 1), nullptr);
    for (hipEvent_t& e : c->ev_sq) SP2_HIP(c, hipEventCreate(&e));
  }
  c->timed = false;
  c->square_ms.clear();
  c->norm_ms.clear();

  if (!noalloc) SP2_HIP(c, hipEventRecord(c->ev_start, s));
  const bool spectral = (c->opt.norm == SP2_NORM_SPECTRAL) && c->spec_nchunks > 0;
  if (timing && spectral && c->ev_nm.empty()) {
    c->ev_nm.assign(2 * (SP2_MAX_ITER_LIMIT + 1), nullptr);
    for (hipEvent_t& e : c->ev_nm) SP2_HIP(c, hipEventCreate(&e));
  }
  SP2_HIP(c, sp2::launch_state_reset(c->d_st, count, c->d_ndone,
                                     spectral ? c->d_spec_ctl : nullptr,
                                     (sp2::kMaxIter + 2) * sp2::kSpecCtl, s));
  if (c->bsr) {
    SP2_HIP(c, sp2::launch_bsr_reset(c->b.ctr, s));
    SP2_HIP(c, sp2::launch_bsr_f0(c->b.F, c->b.m[0], c->b.nnzb_in, c->d_inst,
                                  static_cast<int>(c->b.n), c->d_part_f0, s));
  } else {
    SP2_HIP(c, sp2::launch_f0(c->d_inst, c->d_f0, c->nf0, c->fp64_store,
                              c->d_part_f0, s));
  }
  HostMirror* mirror = noalloc ? nullptr : c->mirror;
  SP2_HIP(c, sp2::launch_finalize(c->d_inst, count, c->d_part, c->d_part_f0,
                                  c->d_ndone, mirror, 0, s));
  if (!noalloc) SP2_HIP(c, hipEventRecord(c->ev_ring[0], s));

  sp2::SquareArgs a;
  a.mode = 0;
  a.stretch = c->stretch ? 1 : 0;
  a.mirror32 = 1;
  a.inst = c->d_inst;
  a.tiles = c->d_tiles;
  a.ws = c->d_ws;
  a.part = c->d_part;
  a.bpart = c->d_bpart;
  a.bcnt = c->d_bcnt;
  int last = 0;
  const bool any_work = c->bsr || !c->groups.empty();
  for (int i = 1; i <= c->opt.max_iter && any_work; ++i) {
    if (noalloc) {
      // every kNoAllocChunk steps: wait for the queued steps and read the
      // number of instances with an outcome
      if (i > 1 && (i - 1) % kNoAllocChunk == 0) {
        int32_t nd = 0;
        SP2_HIP(c, hipMemcpyAsync(&nd, c->d_ndone, sizeof(nd),
                                  hipMemcpyDeviceToHost, s));
        SP2_HIP(c, hipStreamSynchronize(s));
        if (nd >= count) break;
      }
    } else {
      if (i > kLookahead)
        SP2_HIP(c, hipEventSynchronize(c->ev_ring[(i - kLookahead) % kRing]));
      if (__atomic_load_n(&c->mirror->all_done, __ATOMIC_ACQUIRE)) break;
    }
    a.iter = i;
    if (timing) SP2_HIP(c, hipEventRecord(c->ev_sq[2 * i], s));
    if (c->bsr) {
      const sp2::BsrMat& cur = c->b.m[(i - 1) & 1];
      const sp2::BsrMat& nxt = c->b.m[i & 1];
      SP2_HIP(c, sp2::launch_bsr_symbolic(cur, c->b.nb, c->b.sym, nxt,
                                          c->b.cap, c->b.ctr, c->d_st, i, s));
      SP2_HIP(c, sp2::launch_bsr_numeric(cur, nxt, c->b.sym, c->b.ctr,
                                         c->d_inst, i,
                                         static_cast<int>(c->b.n), c->d_part,
                                         c->b.grid, s));
    }
    // one square per group (Alg. 2 / Alg. 4); McWeeny: the square S of
    // every group, then X~ S of every group (the groups share the workspace)
    const int nmodes = c->mcweeny ? 2 : 1;
    for (int mi = 0; mi < nmodes; ++mi) {
      a.mode = c->mcweeny ? mi + 1 : 0;
      for (const Group& g : c->groups) {
        a.mirror32 = (!sp2::kernel_config(g.cfg)->presplit ||
                      c->opt.norm == SP2_NORM_SPECTRAL)
                         ? 1
                         : 0;
        a.items = g.items;
        a.tails = g.tails;
        a.ntail = g.ntail;
        a.split = g.split;
        SP2_HIP(c, sp2::launch_square(g.cfg, a, g.grid, s));
      }
    }
    if (timing) SP2_HIP(c, hipEventRecord(c->ev_sq[2 * i + 1], s));
    if (spectral) {
      // e_{i-1} in the spectral norm, from X~_{i-1} (the squares' input)
      if (timing) SP2_HIP(c, hipEventRecord(c->ev_nm[2 * i], s));
      sp2::SpecArgs sa;
      sa.inst = c->d_inst;
      sa.chunks = c->d_spec_chunks;
      sa.nchunks = c->spec_nchunks;
      sa.count = count;
      sa.iter = i;
      sa.vec_cap = c->spec_vec_cap;
      sa.ctl = c->d_spec_ctl + sp2::kSpecCtl * i;
      SP2_HIP(c, sp2::launch_spectral(sa, c->fp64_store, c->spec_grid, s));
      if (timing) SP2_HIP(c, hipEventRecord(c->ev_nm[2 * i + 1], s));
    }
    SP2_HIP(c, sp2::launch_finalize(c->d_inst, count, c->d_part, c->d_part_f0,
                                    c->d_ndone, mirror, i, s));
    if (!noalloc) SP2_HIP(c, hipEventRecord(c->ev_ring[i % kRing], s));
    last = i;
  }
  float ms = 0.f;
  if (!noalloc) {
    SP2_HIP(c, hipEventRecord(c->ev_stop, s));
    SP2_HIP(c, hipEventSynchronize(c->ev_stop));
    SP2_HIP(c, hipEventElapsedTime(&ms, c->ev_start, c->ev_stop));
  }
  c->host_state.resize(count);
  SP2_HIP(c, hipMemcpyAsync(c->host_state.data(), c->d_st,
                            count * sizeof(DevState), hipMemcpyDeviceToHost,
                            s));
  SP2_HIP(c, hipStreamSynchronize(s));
  int32_t steps = 0;
  for (const DevState& h : c->host_state) {
    if (!h.done)
      return fail(c, SP2_BAD_STATE, "run ended without an outcome", hipSuccess);
    steps = std::max(steps, h.squares);
  }
  c->steps = steps;
  c->run_ms = ms;
  if (c->bsr) {
    sp2::BsrCounters& ctr = c->b.host_ctr;
    SP2_HIP(c, hipMemcpy(&ctr, c->b.ctr, sizeof(ctr), hipMemcpyDeviceToHost));
    // block products per step: the numeric workgroups' counts, summed here
    const int nst = std::min(steps, c->opt.max_iter);
    if (nst > 0) {
      std::vector<uint32_t> pw(static_cast<size_t>(nst + 1) * c->b.grid);
      SP2_HIP(c, hipMemcpy(pw.data(), c->b.sym.prod_wg, pw.size() * sizeof(uint32_t),
                           hipMemcpyDeviceToHost));
      for (int i = 1; i <= nst; ++i) {
        unsigned long long t = 0;
        for (int b = 0; b < c->b.grid; ++b) t += pw[static_cast<size_t>(i) * c->b.grid + b];
        ctr.products[i] = t;
      }
    }
    if (ctr.overflow & 1)
      return fail(c, SP2_OUT_OF_MEMORY,
                  "block-sparse iterate exceeded the block capacity", hipSuccess);
    if (ctr.overflow & 2)
      return fail(c, SP2_INVALID_ARG,
                  "block pattern lost its symmetry: F is not symmetric",
                  hipSuccess);
  }
  if (timing) {
    for (int i = 1; i <= std::min(steps, last); ++i) {
      float t = 0.f;
      SP2_HIP(c, hipEventElapsedTime(&t, c->ev_sq[2 * i], c->ev_sq[2 * i + 1]));
      c->square_ms.push_back(t);
      if (spectral) {
        SP2_HIP(c, hipEventElapsedTime(&t, c->ev_nm[2 * i], c->ev_nm[2 * i + 1]));
        c->norm_ms.push_back(t);
      }
    }
    c->timed = true;
  }
  c->ran = true;
  return SP2_OK;
}

// Index of the flagged blocks of the returned block-sparse iterate.
sp2_status bsr_result_index(sp2_ctx c, int64_t* nnzb) {
  const sp2::BsrMat& m = c->b.m[c->host_state[0].n & 1];
  SP2_HIP(c, sp2::launch_bsr_index(m, c->b.nb, c->b.idx, c->stream));
  int32_t cnt = 0;
  SP2_HIP(c, hipMemcpyAsync(&cnt, c->b.idx.ptr + c->b.nb, sizeof(int32_t),
                            hipMemcpyDeviceToHost, c->stream));
  SP2_HIP(c, hipStreamSynchronize(c->stream));
  *nnzb = cnt;
  return SP2_OK;
}

// Map of the matrix stored for the returned iterate X~_n of instance idx:
// its buffer holds the operand of step n + 1 (OpMap; the identity without
// a stretch and for n_occ = 0 or n).
sp2::OpMap result_map(const sp2_ctx c, int idx) {
  const sp2::OpMap id{1.0, 0.0};
  if (c->hi[idx].trivial || c->h_inst.empty()) return id;
  const sp2::StopParams& prm = c->h_inst[idx].prm;
  const int i = c->host_state[idx].n + 1;
  const size_t o = static_cast<size_t>(idx) * (sp2::kMaxIter + 2) + i;
  if (prm.method == 1)
    return sp2::op_map(1, 1, (i <= prm.mw_len) ? c->h_sched_alpha[o] : 1.0);
  if (prm.n_max > 0 && i <= prm.n_max)
    return sp2::op_map(0, c->h_sched_p[o], c->h_sched_alpha[o]);
  return id;
}

sp2_status copy_density(sp2_ctx c, int idx, void* D_dev, int64_t ldd,
                        int32_t as_fp64) {
  if (c->bsr) {
    if (!D_dev || ldd < c->b.n)
      return fail(c, SP2_INVALID_ARG, "D_dev NULL or ldd < n", hipSuccess);
    SP2_HIP(c, hipSetDevice(c->device));
    int64_t nnzb = 0;
    sp2_status st = bsr_result_index(c, &nnzb);
    if (st != SP2_OK) return st;
    const size_t es = as_fp64 ? 8 : 4;
    SP2_HIP(c, hipMemset2DAsync(D_dev, ldd * es, 0, c->b.n * es, c->b.n,
                                c->stream));
    const sp2::BsrMat& m = c->b.m[c->host_state[0].n & 1];
    SP2_HIP(c, sp2::launch_bsr_to_dense(m.val, c->b.idx, c->b.nb,
                                        static_cast<int>(c->b.n),
                                        result_map(c, 0), D_dev, ldd,
                                        as_fp64 != 0, c->stream));
    SP2_HIP(c, hipStreamSynchronize(c->stream));
    return SP2_OK;
  }
  const HostInst& h = c->hi[idx];
  if (!D_dev || ldd < h.n)
    return fail(c, SP2_INVALID_ARG, "D_dev NULL or ldd < n", hipSuccess);
  const DevState& st = c->host_state[idx];
  const size_t esz = c->fp64_store ? 8 : 4;
  const void* X = static_cast<const char*>(c->pool[st.n & 1]) + h.xoff * esz;
  SP2_HIP(c, hipSetDevice(c->device));
  // configurations with presplit operands leave the FP32 iterate's lower
  // triangle unwritten unless the spectral norm reads it
  const bool sym = sp2::kernel_config(h.cfg)->presplit &&
                   c->opt.norm != SP2_NORM_SPECTRAL;
  SP2_HIP(c, sp2::launch_copy_out(X, c->fp64_store, static_cast<int>(h.n),
                                  static_cast<int>(h.ld), D_dev, ldd,
                                  as_fp64 != 0, sym, result_map(c, idx),
                                  c->stream));
  SP2_HIP(c, hipStreamSynchronize(c->stream));
  return SP2_OK;
}

void fill_history(const sp2_ctx c, int idx, int32_t cap, int32_t* len,
                  double* v, double* t1, double* t2, int8_t* p, double* r) {
  const DevState& h = c->host_state[idx];
  const bool trivial = c->hi[idx].trivial;
  const int nv = trivial ? 0 : h.squares;
  if (len) *len = nv;
  // Traces exist for X~_0 .. X~_m where m is the last iterate formed.
  const int nt = trivial ? 0 : nv + 1;
  for (int k = 0; k < cap; ++k) {
    if (v) v[k] = k < nv ? h.v[k] : NAN;
    if (r) r[k] = k < nv ? h.r[k] : NAN;
    if (t1) t1[k] = k < nt ? h.t1[k] : NAN;
    if (t2) t2[k] = k < nt ? h.t2[k] : NAN;
    if (p) p[k] = k < nt ? (k == 0 ? -1 : h.p[k]) : -1;
  }
}

// Scratch of the no-allocation entry point: one array per device, holding
// every workspace of a dense run (iterates, bf16 split, partial sums, work
// plan, state). Host code uses only the device address that
// hipGetSymbolAddress returns for it on each device, never the array's name.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
char* g_scratch_ptr[kScratchDevices] = {};
std::mutex g_scratch_mu;

// The scratch array's address on `device` (which must be current), looked
// up once per device.
sp2_status scratch_on_device(int device, char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return SP2_HIP_ERROR;
    g_scratch_ptr[device] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return SP2_OK;
}

}  // namespace

extern "C" {

void sp2_default_options(sp2_options* opt) {
  if (!opt) return;
  opt->precision = SP2_FP64;
  opt->branch = SP2_BRANCH_NEAREST;
  opt->trunc_tau = 0.0;
  opt->max_iter = 100;
  opt->kernel_config = 0;
  opt->tail_split = 0;
  opt->kernel_timing = 0;
  opt->norm = SP2_NORM_FROBENIUS;
  opt->launch = SP2_LAUNCH_AUTO;
}

const char* sp2_status_string(sp2_status s) {
  switch (s) {
    case SP2_OK: return "SP2_OK";
    case SP2_INVALID_ARG: return "SP2_INVALID_ARG";
    case SP2_OUT_OF_MEMORY: return "SP2_OUT_OF_MEMORY";
    case SP2_HIP_ERROR: return "SP2_HIP_ERROR";
    case SP2_NOT_CONVERGED: return "SP2_NOT_CONVERGED";
    case SP2_DIVERGED: return "SP2_DIVERGED";
    case SP2_BAD_STATE: return "SP2_BAD_STATE";
  }
  return "SP2_UNKNOWN_STATUS";
}

const char* sp2_last_error(sp2_ctx ctx) { return ctx ? ctx->err.c_str() : ""; }

int32_t sp2_kernel_config_count(void) { return sp2::kernel_config_count(); }

sp2_status sp2_set_kernel_table(sp2_ctx c, int32_t count,
                                const int32_t* precision, const int64_t* n_max,
                                const int32_t* config_id) {
  if (!c || count < 0) return SP2_INVALID_ARG;
  if (count > 0 && (!precision || !n_max || !config_id))
    return fail(c, SP2_INVALID_ARG, "NULL table array", hipSuccess);
  std::vector<sp2_ctx_s::TableEntry> t;
  for (int e = 0; e < count; ++e) {
    const sp2::KernelConfig* kc = sp2::kernel_config(config_id[e] - 1);
    if (!kc || kc->precision != precision[e])
      return fail(c, SP2_INVALID_ARG,
                  "table entry names an unknown configuration or one of "
                  "another precision", hipSuccess);
    t.push_back({precision[e], n_max[e], config_id[e] - 1});
  }
  c->table = std::move(t);
  return SP2_OK;
}

sp2_status sp2_kernel_config_info(int32_t id, int32_t* precision,
                                  int32_t* tile, int32_t* waves_m,
                                  int32_t* waves_n, int32_t* k_slice) {
  const sp2::KernelConfig* k = sp2::kernel_config(id - 1);
  if (!k) return SP2_INVALID_ARG;
  if (precision) *precision = k->precision;
  if (tile) *tile = k->bm;
  if (waves_m) *waves_m = k->wm;
  if (waves_n) *waves_n = k->wn;
  if (k_slice) *k_slice = k->bk;
  return SP2_OK;
}

const char* sp2_kernel_config_name(int32_t id) {
  const sp2::KernelConfig* k = sp2::kernel_config(id - 1);
  return k ? k->name : nullptr;
}

sp2_status sp2_create(sp2_ctx* out, int device, void* hip_stream) {
  if (!out) return SP2_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return SP2_INVALID_ARG;
  sp2_ctx c = new (std::nothrow) sp2_ctx_s();
  if (!c) return SP2_OUT_OF_MEMORY;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipMalloc(&c->d_ndone, 256);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&c->mirror), sizeof(HostMirror),
                      hipHostMallocCoherent | hipHostMallocMapped);
  if (e != hipSuccess) {
    sp2_destroy(c);
    return e == hipErrorOutOfMemory ? SP2_OUT_OF_MEMORY : SP2_HIP_ERROR;
  }
  memset(c->mirror, 0, sizeof(HostMirror));
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) ==
          hipSuccess && khz > 0)
    c->wall_khz = khz;
  // SP2_PERSIST_WAIT_MS: longest wait of a persistent workgroup for a queue
  // item before the run gives up (milliseconds; default 2000)
  if (const char* w = getenv("SP2_PERSIST_WAIT_MS")) {
    char* end = nullptr;
    const long long v = strtoll(w, &end, 10);
    if (end != w && v >= 0) c->wait_ms = v;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess &&
      prop.multiProcessorCount > 0)
    c->num_cus = prop.multiProcessorCount;
  if (ensure_events(c) != SP2_OK) {
    sp2_destroy(c);
    return SP2_HIP_ERROR;
  }
  *out = c;
  return SP2_OK;
}

sp2_status sp2_destroy(sp2_ctx c) {
  if (!c) return SP2_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  auto rel = [](void* p) {
    if (p) (void)hipFree(p);
  };
  rel(c->pool[0]);
  rel(c->pool[1]);
  for (void* p : c->split_pool) rel(p);
  rel(c->d_inst);
  rel(c->d_sched);
  rel(c->d_blk);
  rel(c->d_lz);
  rel(c->d_spec);
  rel(c->d_spec_chunks);
  rel(c->d_spec_ctl);
  rel(c->s_pool);
  rel(c->s_split[0]);
  rel(c->s_split[1]);
  rel(c->d_st);
  rel(c->d_tiles);
  rel(c->d_part);
  rel(c->d_part_f0);
  rel(c->d_f0);
  rel(c->d_ws);
  rel(c->d_bpart);
  rel(c->d_bcnt);
  rel(c->d_ndone);
  rel(c->b.mem);
  rel(c->d_pitems);
  rel(c->d_pctl);
  rel(c->d_pcnt);
  release_graph(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  release_groups(c);
  if (c->mirror) (void)hipHostFree(c->mirror);
  if (c->ev_start) (void)hipEventDestroy(c->ev_start);
  if (c->ev_stop) (void)hipEventDestroy(c->ev_stop);
  for (hipEvent_t e : c->ev_ring)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ev_sq)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ev_nm)
    if (e) (void)hipEventDestroy(e);
  delete c;
  return SP2_OK;
}

sp2_status sp2_batch_init(sp2_ctx c, int32_t count, const double* const* F_dev,
                          const int64_t* n, const int64_t* ldf,
                          const double* lambda_min, const double* lambda_max,
                          const int64_t* n_occ, const sp2_options* opt_in) {
  if (!c) return SP2_INVALID_ARG;
  c->err.clear();
  c->inited = false;
  c->ran = false;
  if (count < 1 || count > 65536 || !F_dev || !n || !ldf || !lambda_min ||
      !lambda_max || !n_occ)
    return fail(c, SP2_INVALID_ARG, "count outside [1, 65536] or NULL array",
                hipSuccess);
  sp2_options opt;
  if (opt_in) {
    opt = *opt_in;
  } else {
    sp2_default_options(&opt);
  }
  sp2_status st = validate_options(c, opt);
  if (st != SP2_OK) return st;
  std::vector<HostInst> hi(count);
  for (int b = 0; b < count; ++b) {
    st = validate_instance(c, F_dev[b], n[b], ldf[b], lambda_min[b],
                           lambda_max[b], n_occ[b]);
    if (st != SP2_OK) {
      c->err += " (instance " + std::to_string(b) + ")";
      return st;
    }
    hi[b].F = F_dev[b];
    hi[b].n = n[b];
    hi[b].ldf = ldf[b];
    hi[b].lmin = lambda_min[b];
    hi[b].lmax = lambda_max[b];
    hi[b].n_occ = n_occ[b];
  }
  SP2_HIP(c, hipSetDevice(c->device));
  c->bsr = false;
  c->opt = opt;
  c->fp64_store = (opt.precision == SP2_FP64);
  c->hi = std::move(hi);
  st = setup(c);
  if (st != SP2_OK) return st;
  c->inited = true;
  return SP2_OK;
}

sp2_status sp2_init_bsr(sp2_ctx c, int64_t n, int32_t block, int64_t nnzb,
                        const int32_t* row_ptr_dev, const int32_t* col_idx_dev,
                        const double* blocks_dev, double lambda_min,
                        double lambda_max, int64_t n_occ,
                        const sp2_options* opt_in) {
  if (!c) return SP2_INVALID_ARG;
  c->err.clear();
  c->inited = false;
  c->ran = false;
  sp2_options opt;
  if (opt_in) {
    opt = *opt_in;
  } else {
    sp2_default_options(&opt);
    opt.precision = SP2_FP32;
  }
  sp2_status st = validate_options(c, opt);
  if (st != SP2_OK) return st;
  if (opt.precision != SP2_FP32)
    return fail(c, SP2_INVALID_ARG, "block-sparse runs use SP2_FP32",
                hipSuccess);
  if (block != sp2::kBsrBlock)
    return fail(c, SP2_INVALID_ARG, "block must be 32", hipSuccess);
  if (n <= 0 || n > static_cast<int64_t>(sp2::kMaxBlockCols) * sp2::kBsrBlock)
    return fail(c, SP2_INVALID_ARG, "n must be in [1, 65536]", hipSuccess);
  if (!row_ptr_dev || !col_idx_dev || !blocks_dev || nnzb <= 0)
    return fail(c, SP2_INVALID_ARG, "NULL array or nnzb <= 0", hipSuccess);
  if (n_occ < 0 || n_occ > n)
    return fail(c, SP2_INVALID_ARG, "n_occ outside [0, n]", hipSuccess);
  if (!isfinite(lambda_min) || !isfinite(lambda_max) ||
      !(lambda_max > lambda_min) || !isfinite(lambda_max - lambda_min))
    return fail(c, SP2_INVALID_ARG,
                "spectral bounds must be finite with lambda_max > lambda_min",
                hipSuccess);
  const int nb = static_cast<int>((n + sp2::kBsrBlock - 1) / sp2::kBsrBlock);
  if (nnzb > static_cast<int64_t>(nb) * nb)
    return fail(c, SP2_INVALID_ARG, "nnzb exceeds nb * nb", hipSuccess);
  SP2_HIP(c, hipSetDevice(c->device));
  // Validate the pattern on the host: sorted unique columns, every diagonal
  // block present, and a symmetric pattern.
  std::vector<int32_t> rp(nb + 1), ci(nnzb);
  SP2_HIP(c, hipMemcpy(rp.data(), row_ptr_dev, (nb + 1) * sizeof(int32_t),
                       hipMemcpyDeviceToHost));
  SP2_HIP(c, hipMemcpy(ci.data(), col_idx_dev, nnzb * sizeof(int32_t),
                       hipMemcpyDeviceToHost));
  if (rp[0] != 0 || rp[nb] != nnzb)
    return fail(c, SP2_INVALID_ARG, "row_ptr must start at 0 and end at nnzb",
                hipSuccess);
  std::vector<int32_t> brow(nnzb);
  for (int r = 0; r < nb; ++r) {
    if (rp[r + 1] < rp[r])
      return fail(c, SP2_INVALID_ARG, "row_ptr not monotone", hipSuccess);
    bool diag = false;
    for (int q = rp[r]; q < rp[r + 1]; ++q) {
      if (ci[q] < 0 || ci[q] >= nb || (q > rp[r] && ci[q] <= ci[q - 1]))
        return fail(c, SP2_INVALID_ARG,
                    "column indices out of range or not sorted and unique",
                    hipSuccess);
      diag = diag || ci[q] == r;
      brow[q] = r;
    }
    if (!diag)
      return fail(c, SP2_INVALID_ARG, "every diagonal block must be stored",
                  hipSuccess);
  }
  for (int r = 0; r < nb; ++r)
    for (int q = rp[r]; q < rp[r + 1]; ++q) {
      const int cc = ci[q];
      if (!std::binary_search(ci.begin() + rp[cc], ci.begin() + rp[cc + 1], r))
        return fail(c, SP2_INVALID_ARG, "block pattern is not symmetric",
                    hipSuccess);
    }
  // Capacity for the fill of the iterates.
  const int64_t cap64 = std::min<int64_t>(static_cast<int64_t>(nb) * nb,
                                          16 * nnzb + 64 * nb);
  const int cap = static_cast<int>(cap64);
  const int nbw = (nb + 31) / 32;
  const int grid = 4 * c->num_cus;
  // One allocation, carved into aligned pieces.
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  size_t o_m[2][5];
  for (int k = 0; k < 2; ++k) {
    o_m[k][0] = take((nb + 1) * sizeof(int32_t));
    o_m[k][1] = take(cap * sizeof(int32_t));
    o_m[k][2] = take(cap * sizeof(int32_t));
    o_m[k][3] = take(static_cast<size_t>(cap) * 1024 * sizeof(float));
    o_m[k][4] = take(cap * sizeof(int32_t));
  }
  const size_t o_ip = take((nb + 1) * sizeof(int32_t));
  const size_t o_ic = take(cap * sizeof(int32_t));
  const size_t o_is = take(cap * sizeof(int32_t));
  const size_t o_bm = take(static_cast<size_t>(nb) * nbw * sizeof(uint32_t));
  const size_t o_wp = take(static_cast<size_t>(nb) * nbw * sizeof(int32_t));
  const size_t o_qc = take(nb * sizeof(int32_t));
  const size_t o_uc = take(nb * sizeof(int32_t));
  const size_t o_nz = take(nb * sizeof(int32_t));
  const size_t o_pw = take(static_cast<size_t>(sp2::kMaxIter + 2) * grid * sizeof(uint32_t));
  const size_t o_wk = take(static_cast<size_t>(cap) * sizeof(sp2::BsrWork));
  const size_t o_ct = take(sizeof(sp2::BsrCounters));
  if (off > c->b.bytes) {
    SP2_HIP(c, hipStreamSynchronize(c->stream));
    if (c->b.mem) (void)hipFree(c->b.mem);
    c->b.mem = nullptr;
    c->b.bytes = 0;
    SP2_HIP(c, hipMalloc(&c->b.mem, off));
    c->b.bytes = off;
  }
  char* base = static_cast<char*>(c->b.mem);
  for (int k = 0; k < 2; ++k) {
    c->b.m[k].row_ptr = reinterpret_cast<int32_t*>(base + o_m[k][0]);
    c->b.m[k].col = reinterpret_cast<int32_t*>(base + o_m[k][1]);
    c->b.m[k].brow = reinterpret_cast<int32_t*>(base + o_m[k][2]);
    c->b.m[k].val = reinterpret_cast<float*>(base + o_m[k][3]);
    c->b.m[k].flag = reinterpret_cast<int32_t*>(base + o_m[k][4]);
  }
  c->b.idx.ptr = reinterpret_cast<int32_t*>(base + o_ip);
  c->b.idx.col = reinterpret_cast<int32_t*>(base + o_ic);
  c->b.idx.pos = reinterpret_cast<int32_t*>(base + o_is);
  c->b.sym.bitmap = reinterpret_cast<uint32_t*>(base + o_bm);
  c->b.sym.wpre = reinterpret_cast<int32_t*>(base + o_wp);
  c->b.sym.qcnt = reinterpret_cast<int32_t*>(base + o_qc);
  c->b.sym.ucnt = reinterpret_cast<int32_t*>(base + o_uc);
  c->b.sym.nzrow = reinterpret_cast<int32_t*>(base + o_nz);
  c->b.sym.prod_wg = reinterpret_cast<uint32_t*>(base + o_pw);
  c->b.sym.work = reinterpret_cast<sp2::BsrWork*>(base + o_wk);
  c->b.ctr = reinterpret_cast<sp2::BsrCounters*>(base + o_ct);
  c->b.n = n;
  c->b.nb = nb;
  c->b.nnzb_in = static_cast<int>(nnzb);
  c->b.cap = cap;
  c->b.grid = grid;
  c->b.F = blocks_dev;
  hipStream_t s = c->stream;
  // the input pattern becomes the pattern of X_0
  SP2_HIP(c, hipMemcpyAsync(c->b.m[0].row_ptr, rp.data(),
                            (nb + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
  SP2_HIP(c, hipMemcpyAsync(c->b.m[0].col, ci.data(), nnzb * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
  SP2_HIP(c, hipMemcpyAsync(c->b.m[0].brow, brow.data(),
                            nnzb * sizeof(int32_t), hipMemcpyHostToDevice, s));
  // instance table of one entry: partial sums of the numeric kernel (one
  // triple per workgroup) and of the affine start (one per block)
  Instance in{};
  SP2_HIP(c, grow(c, c->d_st, c->d_st_cap, sizeof(DevState), s));
  in.n = static_cast<int>(n);
  in.tile0 = 0;
  in.ntiles = grid;
  in.f0blk0 = 0;
  in.nf0blk = static_cast<int>(nnzb);
  in.st = c->d_st;
  in.lmax = lambda_max;
  in.width = lambda_max - lambda_min;
  in.tau = opt.trunc_tau;
  in.prm.n_occ = static_cast<double>(n_occ);
  in.prm.n = static_cast<double>(n);
  in.prm.branch = opt.branch;
  in.prm.max_iter = opt.max_iter;
  in.prm.norm = opt.norm;
  in.nbk = nb;
  for (int k = 0; k < 2; ++k) {
    in.brp[k] = c->b.m[k].row_ptr;
    in.bcol[k] = c->b.m[k].col;
    in.bflag[k] = c->b.m[k].flag;
    in.bval[k] = c->b.m[k].val;
  }
  if (opt.norm == SP2_NORM_MIXED) {
    // one block norm per block of the output pattern
    SP2_HIP(c, grow(c, c->d_blk, c->d_blk_cap,
                    static_cast<size_t>(cap) * sizeof(float), s));
    in.blk = c->d_blk;
    SP2_HIP(c, grow(c, c->d_lz, c->d_lz_cap,
                    static_cast<size_t>(sp2::kLanczosMax) * nb * sizeof(double),
                    s));
    in.lz = c->d_lz;
  }
  c->spec_nchunks = 0;
  if (opt.norm == SP2_NORM_SPECTRAL && n_occ != 0 && n_occ != n) {
    // Lanczos scratch and one chunk (one block row) per 32 rows; the
    // product's input vector is staged in LDS up to kSpecLdsVec entries
    std::vector<int2> chunks;
    for (int r = 0; r < n; r += sp2::kSpecRows) chunks.push_back(int2{0, r});
    SP2_HIP(c, grow(c, c->d_spec, c->d_spec_cap,
                    sp2::spec_doubles(static_cast<int>(n)) * sizeof(double), s));
    SP2_HIP(c, grow(c, c->d_spec_chunks, c->d_spec_chunks_cap,
                    chunks.size() * sizeof(int2), s));
    SP2_HIP(c, grow(c, c->d_spec_ctl, c->d_spec_ctl_cap,
                    (sp2::kMaxIter + 2) * sp2::kSpecCtl * sizeof(int32_t), s));
    SP2_HIP(c, hipMemcpyAsync(c->d_spec_chunks, chunks.data(),
                              chunks.size() * sizeof(int2),
                              hipMemcpyHostToDevice, s));
    c->spec_vec_cap = std::min(sp2::spec_ldq(static_cast<int>(n)), sp2::kSpecLdsVec);
    const int gmax = sp2::spectral_max_grid(false, c->num_cus, c->spec_vec_cap);
    if (gmax < 1)
      return fail(c, SP2_HIP_ERROR, "spectral kernel: no co-resident grid",
                  hipGetLastError());
    c->spec_grid = std::min<int>(gmax, static_cast<int>(chunks.size()) + 1);
    c->spec_nchunks = static_cast<int>(chunks.size());
    in.sp = c->d_spec;
    in.sp_ch0 = 0;
    in.sp_nch = c->spec_nchunks;
  }
  SP2_HIP(c, grow(c, c->d_inst, c->d_inst_cap, sizeof(Instance), s));
  SP2_HIP(c, grow(c, c->d_part, c->d_part_cap, grid * 3 * sizeof(double), s));
  SP2_HIP(c, grow(c, c->d_part_f0, c->d_part_f0_cap, nnzb * 3 * sizeof(double), s));
  SP2_HIP(c, hipMemcpyAsync(c->d_inst, &in, sizeof(Instance),
                            hipMemcpyHostToDevice, s));
  SP2_HIP(c, hipStreamSynchronize(s));
  c->h_inst.assign(1, in);
  c->mcweeny = false;
  c->stretch = false;
  release_groups(c);
  HostInst h;
  h.F = nullptr;
  h.n = n;
  h.n_occ = n_occ;
  h.lmin = lambda_min;
  h.lmax = lambda_max;
  h.trivial = (n_occ == 0 || n_occ == n);
  c->hi.assign(1, h);
  c->opt = opt;
  c->fp64_store = false;
  c->bsr = true;
  c->inited = true;
  return SP2_OK;
}

sp2_status sp2_get_bsr_nnzb(sp2_ctx c, int64_t* nnzb) {
  if (!c || !nnzb) return SP2_INVALID_ARG;
  if (!c->ran || !c->bsr)
    return fail(c, SP2_BAD_STATE, "no completed block-sparse run", hipSuccess);
  SP2_HIP(c, hipSetDevice(c->device));
  return bsr_result_index(c, nnzb);
}

sp2_status sp2_get_bsr(sp2_ctx c, int32_t* row_ptr_dev, int32_t* col_idx_dev,
                       void* blocks_dev, int32_t as_fp64) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->ran || !c->bsr)
    return fail(c, SP2_BAD_STATE, "no completed block-sparse run", hipSuccess);
  if (!row_ptr_dev || !col_idx_dev || !blocks_dev)
    return fail(c, SP2_INVALID_ARG, "NULL output array", hipSuccess);
  SP2_HIP(c, hipSetDevice(c->device));
  int64_t nnzb = 0;
  sp2_status st = bsr_result_index(c, &nnzb);
  if (st != SP2_OK) return st;
  hipStream_t s = c->stream;
  SP2_HIP(c, hipMemcpyAsync(row_ptr_dev, c->b.idx.ptr,
                            (c->b.nb + 1) * sizeof(int32_t),
                            hipMemcpyDeviceToDevice, s));
  if (nnzb > 0) {
    SP2_HIP(c, hipMemcpyAsync(col_idx_dev, c->b.idx.col,
                              nnzb * sizeof(int32_t), hipMemcpyDeviceToDevice,
                              s));
    const sp2::BsrMat& m = c->b.m[c->host_state[0].n & 1];
    SP2_HIP(c, sp2::launch_bsr_gather(m, c->b.idx.pos, static_cast<int>(nnzb),
                                      static_cast<int>(c->b.n), result_map(c, 0),
                                      blocks_dev, as_fp64 != 0, s));
  }
  SP2_HIP(c, hipStreamSynchronize(s));
  return SP2_OK;
}

sp2_status sp2_get_bsr_stats(sp2_ctx c, int32_t cap, int32_t* len,
                             int64_t* stored, int64_t* nonzero,
                             int64_t* products) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->ran || !c->bsr)
    return fail(c, SP2_BAD_STATE, "no completed block-sparse run", hipSuccess);
  const sp2::BsrCounters& h = c->b.host_ctr;
  const int m = c->hi[0].trivial ? 0 : c->host_state[0].squares;
  if (len) *len = m;
  for (int i = 0; i < cap && i < m; ++i) {
    if (stored) stored[i] = h.stored[i + 1];
    if (nonzero) nonzero[i] = h.nonzero[i + 1];
    if (products) products[i] = static_cast<int64_t>(h.products[i + 1]);
  }
  return SP2_OK;
}

sp2_status sp2_init_dense(sp2_ctx c, const double* F_dev, int64_t n,
                          int64_t ldf, double lambda_min, double lambda_max,
                          int64_t n_occ, const sp2_options* opt) {
  return sp2_batch_init(c, 1, &F_dev, &n, &ldf, &lambda_min, &lambda_max,
                        &n_occ, opt);
}

sp2_status sp2_batch_run(sp2_ctx c) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->inited) return fail(c, SP2_BAD_STATE, "run before init", hipSuccess);
  c->err.clear();
  c->ran = false;
  return run_batch(c);
}

sp2_status sp2_run(sp2_ctx c) {
  sp2_status st = sp2_batch_run(c);
  if (st != SP2_OK) return st;
  return static_cast<sp2_status>(c->host_state[0].status);
}

sp2_status sp2_batch_get(sp2_ctx c, int32_t idx, void* D_dev, int64_t ldd,
                         int32_t as_fp64, int32_t* n_iter, int32_t* n_squares,
                         int32_t* status) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->ran) return fail(c, SP2_BAD_STATE, "no completed run", hipSuccess);
  if (idx < 0 || idx >= static_cast<int32_t>(c->hi.size()))
    return fail(c, SP2_INVALID_ARG, "instance index out of range", hipSuccess);
  const DevState& h = c->host_state[idx];
  if (n_iter) *n_iter = h.n;
  if (n_squares) *n_squares = c->hi[idx].trivial ? 0 : h.squares;
  if (status) *status = h.status;
  if (D_dev) return copy_density(c, idx, D_dev, ldd, as_fp64);
  return SP2_OK;
}

sp2_status sp2_batch_get_history(sp2_ctx c, int32_t idx, int32_t cap,
                                 int32_t* len, double* v, double* t1,
                                 double* t2, int8_t* p, double* r) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->ran) return SP2_BAD_STATE;
  if (cap < 0 || idx < 0 || idx >= static_cast<int32_t>(c->hi.size()))
    return SP2_INVALID_ARG;
  fill_history(c, idx, cap, len, v, t1, t2, p, r);
  return SP2_OK;
}

sp2_status sp2_get_density(sp2_ctx c, void* D_dev, int64_t ldd,
                           int32_t as_fp64) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->ran) return fail(c, SP2_BAD_STATE, "no completed run", hipSuccess);
  return copy_density(c, 0, D_dev, ldd, as_fp64);
}

sp2_status sp2_get_info(sp2_ctx c, int32_t* n_iter, int32_t* n_squares,
                        double* run_ms) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->ran) return SP2_BAD_STATE;
  const DevState& h = c->host_state[0];
  if (n_iter) *n_iter = h.n;
  if (n_squares) *n_squares = c->hi[0].trivial ? 0 : h.squares;
  if (run_ms) *run_ms = c->run_ms;
  return SP2_OK;
}

sp2_status sp2_set_mcweeny(sp2_ctx c, int32_t count, const double* mu,
                           const double* xi) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->inited)
    return fail(c, SP2_BAD_STATE, "no instances: call an init first",
                hipSuccess);
  if (c->bsr)
    return fail(c, SP2_INVALID_ARG,
                "McWeeny needs a general product; not available for "
                "block-sparse contexts",
                hipSuccess);
  if (count != static_cast<int32_t>(c->hi.size()) || !mu)
    return fail(c, SP2_INVALID_ARG,
                "count must equal the number of instances; mu must be given",
                hipSuccess);
  if (c->h_inst.size() && c->h_inst[0].prm.n_max > 0)
    return fail(c, SP2_INVALID_ARG,
                "an SP2-ACC schedule is set: re-initialise first", hipSuccess);
  if (c->opt.launch == SP2_LAUNCH_PERSISTENT)
    return fail(c, SP2_INVALID_ARG,
                "McWeeny runs are driven by a launch sequence per step, not "
                "by the persistent launch", hipSuccess);
  for (int b = 0; b < count; ++b) {
    const HostInst& h = c->hi[b];
    const double gam = 2.0 * std::max(h.lmax - mu[b], mu[b] - h.lmin);
    const bool ok_mu = isfinite(mu[b]) && mu[b] >= h.lmin && mu[b] <= h.lmax;
    const bool ok_xi = !xi || (isfinite(xi[b]) && xi[b] > 0.0 && xi[b] <= gam);
    if (!ok_mu || !ok_xi || !(gam > 0.0)) {
      c->err = "instance " + std::to_string(b) +
               ": mu outside [lambda_min, lambda_max] or xi outside (0, gamma]";
      return SP2_INVALID_ARG;
    }
  }
  SP2_HIP(c, hipSetDevice(c->device));
  hipStream_t s = c->stream;
  size_t pool_elems = 0;
  for (const HostInst& h : c->hi)
    pool_elems = std::max(pool_elems,
                          h.xoff + static_cast<size_t>(h.np) * h.ld);
  const size_t esz = c->fp64_store ? 8 : 4;
  SP2_HIP(c, grow(c, c->s_pool, c->s_pool_cap, pool_elems * esz, s));
  const bool split = (c->opt.precision == SP2_BF16X3);
  if (split)
    for (int q = 0; q < 2; ++q)
      SP2_HIP(c, grow(c, c->s_split[q], c->s_split_cap[q], pool_elems * 2, s));
  // McW-ACC (sec. 3): the stretch of every step from the scalar recursion
  // beta_i = p_mw(alpha_i (beta_{i-1} - 1/2) + 1/2), beta_0 = (1 - xi /
  // gamma) / 2, alpha_i = 3 / sqrt(12 beta^2 - 18 beta + 9); with the
  // Frobenius or the mixed norm the stretch is switched off once beta < 0.01
  // and the stop is tested from the step after (reading R24); with the
  // spectral norm the stretch stays on and every step is tested.
  const int L = sp2::kMaxIter + 2;
  std::vector<double> alpha(static_cast<size_t>(count) * L, 1.0);
  std::vector<int> mw_len(count, 0), mw_first(count, 1);
  const bool spectral = (c->opt.norm == SP2_NORM_SPECTRAL);
  for (int b = 0; b < count && xi; ++b) {
    const HostInst& h = c->hi[b];
    const double gam = 2.0 * std::max(h.lmax - mu[b], mu[b] - h.lmin);
    double beta = 0.5 * (1.0 - xi[b] / gam);
    mw_first[b] = sp2::kMaxIter + 2;   // until the stretch is switched off
    for (int i = 1; i <= sp2::kMaxIter + 1; ++i) {
      if (!spectral && beta < 0.01) {
        mw_first[b] = i + 1;
        break;
      }
      const double a = 3.0 / sqrt(12.0 * beta * beta - 18.0 * beta + 9.0);
      alpha[static_cast<size_t>(b) * L + i] = a;
      mw_len[b] = i;
      const double bs = a * (beta - 0.5) + 0.5;
      beta = 3.0 * bs * bs - 2.0 * bs * bs * bs;
    }
    if (spectral) mw_first[b] = 1;
  }
  const size_t abytes = alpha.size() * sizeof(double);
  SP2_HIP(c, grow(c, c->d_sched, c->d_sched_cap, abytes, s));
  SP2_HIP(c, hipMemcpyAsync(c->d_sched, alpha.data(), abytes,
                            hipMemcpyHostToDevice, s));
  c->h_sched_alpha = alpha;
  c->h_sched_p.assign(alpha.size(), 1);
  c->stretch = std::any_of(alpha.begin(), alpha.end(),
                           [](double x) { return x != 1.0; });
  release_graph(c);
  for (int b = 0; b < count; ++b) {
    const HostInst& h = c->hi[b];
    Instance& in = c->h_inst[b];
    const double gam = 2.0 * std::max(h.lmax - mu[b], mu[b] - h.lmin);
    // X_0 = (mu I - F) / gamma + I / 2 = ((mu + gamma / 2) I - F) / gamma
    in.lmax = mu[b] + 0.5 * gam;
    in.width = gam;
    in.S = static_cast<char*>(c->s_pool) + h.xoff * esz;
    in.SH = split ? static_cast<char*>(c->s_split[0]) + h.xoff * 2 : nullptr;
    in.SL = split ? static_cast<char*>(c->s_split[1]) + h.xoff * 2 : nullptr;
    in.prm.method = 1;
    in.prm.mw_first = mw_first[b];
    in.prm.mw_len = mw_len[b];
    in.sched_alpha = static_cast<const double*>(c->d_sched) +
                     static_cast<size_t>(b) * L;
  }
  SP2_HIP(c, hipMemcpyAsync(c->d_inst, c->h_inst.data(),
                            count * sizeof(Instance), hipMemcpyHostToDevice, s));
  SP2_HIP(c, hipStreamSynchronize(s));
  c->mcweeny = true;
  return SP2_OK;
}

sp2_status sp2_get_mixed_history(sp2_ctx c, int32_t index, int32_t cap,
                                 int32_t* len, double* m) {
  if (!c) return SP2_INVALID_ARG;
  if (c->ran && c->opt.norm != SP2_NORM_MIXED)
    return fail(c, SP2_BAD_STATE, "the last run did not use the mixed norm",
                hipSuccess);
  return sp2_get_norm_history(c, index, cap, len, m, nullptr);
}

sp2_status sp2_get_norm_history(sp2_ctx c, int32_t index, int32_t cap,
                                int32_t* len, double* m, int32_t* krylov) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->ran || c->opt.norm == SP2_NORM_FROBENIUS)
    return fail(c, SP2_BAD_STATE,
                "no completed run with the mixed or the spectral norm",
                hipSuccess);
  if (index < 0 || index >= static_cast<int32_t>(c->host_state.size()) ||
      cap < 0)
    return fail(c, SP2_INVALID_ARG, "index or cap out of range", hipSuccess);
  const DevState& h = c->host_state[index];
  const int cnt = c->hi[index].trivial ? 0 : h.squares;
  if (len) *len = cnt;
  if (m)
    for (int k = 0; k < cnt && k < cap; ++k) m[k] = h.m[k];
  if (krylov)
    for (int k = 0; k < cnt && k < cap; ++k) krylov[k] = h.krylov[k];
  return SP2_OK;
}

sp2_status sp2_set_homo_lumo(sp2_ctx c, int32_t count, const double* homo_out,
                             const double* homo_in, const double* lumo_in,
                             const double* lumo_out, int32_t accelerate) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->inited)
    return fail(c, SP2_BAD_STATE, "no instances: call an init first",
                hipSuccess);
  if (count != static_cast<int32_t>(c->hi.size()) ||
      count != static_cast<int32_t>(c->h_inst.size()))
    return fail(c, SP2_INVALID_ARG,
                "count must equal the number of instances of the last init",
                hipSuccess);
  if (!homo_out || !homo_in || !lumo_in || !lumo_out)
    return fail(c, SP2_INVALID_ARG, "NULL bound array", hipSuccess);
  if (c->mcweeny)
    return fail(c, SP2_INVALID_ARG,
                "the context runs McWeeny: re-initialise first", hipSuccess);
  SP2_HIP(c, hipSetDevice(c->device));
  const int L = sp2::kMaxIter + 2;   // entries 1..n_max are used
  std::vector<double> alpha(static_cast<size_t>(count) * L, 1.0);
  std::vector<int8_t> pol(static_cast<size_t>(count) * L, 0);
  std::vector<int> nmin(count, 0), nmax(count, 0);
  for (int b = 0; b < count; ++b) {
    const HostInst& h = c->hi[b];
    if (h.trivial) continue;   // stops before any square; no homo/lumo
    const size_t o = static_cast<size_t>(b) * L + 1;
    const int rc = sp2::acc_schedule(h.lmin, h.lmax, homo_out[b], homo_in[b],
                                     lumo_in[b], lumo_out[b], accelerate != 0,
                                     sp2::kMaxIter, &nmin[b], &nmax[b],
                                     pol.data() + o, alpha.data() + o);
    if (rc != 0) {
      c->err = "instance " + std::to_string(b) +
               (rc == -1 ? ": homo/lumo bounds not finite, out of order or "
                           "overlapping"
                         : ": schedule longer than SP2_MAX_ITER_LIMIT steps");
      return SP2_INVALID_ARG;
    }
  }
  hipStream_t s = c->stream;
  const size_t abytes = alpha.size() * sizeof(double);
  SP2_HIP(c, grow(c, c->d_sched, c->d_sched_cap, abytes + pol.size(), s));
  c->h_sched_alpha = alpha;
  c->h_sched_p = pol;
  c->stretch = std::any_of(alpha.begin(), alpha.end(),
                           [](double x) { return x != 1.0; });
  release_graph(c);
  double* d_alpha = static_cast<double*>(c->d_sched);
  int8_t* d_pol = reinterpret_cast<int8_t*>(static_cast<char*>(c->d_sched) + abytes);
  SP2_HIP(c, hipMemcpyAsync(d_alpha, alpha.data(), abytes,
                            hipMemcpyHostToDevice, s));
  SP2_HIP(c, hipMemcpyAsync(d_pol, pol.data(), pol.size(),
                            hipMemcpyHostToDevice, s));
  for (int b = 0; b < count; ++b) {
    Instance& in = c->h_inst[b];
    in.prm.n_min = nmin[b];
    in.prm.n_max = nmax[b];
    in.sched_alpha = nmax[b] ? d_alpha + static_cast<size_t>(b) * L : nullptr;
    in.sched_p = nmax[b] ? d_pol + static_cast<size_t>(b) * L : nullptr;
  }
  SP2_HIP(c, hipMemcpyAsync(c->d_inst, c->h_inst.data(),
                            count * sizeof(Instance), hipMemcpyHostToDevice, s));
  // the copies read host vectors that go out of scope
  SP2_HIP(c, hipStreamSynchronize(s));
  return SP2_OK;
}

sp2_status sp2_get_config(sp2_ctx c, int32_t index, int32_t* config_id) {
  if (!c || !config_id) return SP2_INVALID_ARG;
  if (!c->inited) return SP2_BAD_STATE;
  if (index < 0 || index >= static_cast<int32_t>(c->hi.size()))
    return SP2_INVALID_ARG;
  const HostInst& h = c->hi[index];
  *config_id = (c->bsr || h.trivial) ? 0 : h.cfg + 1;
  return SP2_OK;
}

sp2_status sp2_batch_get_run_time(sp2_ctx c, double* run_ms, int32_t* steps) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->ran) return SP2_BAD_STATE;
  if (run_ms) *run_ms = c->run_ms;
  if (steps) *steps = c->steps;
  return SP2_OK;
}

sp2_status sp2_get_kernel_times(sp2_ctx c, int32_t cap, int32_t* len,
                                float* ms) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->ran || !c->timed) return SP2_BAD_STATE;
  const int m = static_cast<int>(c->square_ms.size());
  if (len) *len = m;
  if (ms)
    for (int i = 0; i < cap && i < m; ++i) ms[i] = c->square_ms[i];
  return SP2_OK;
}

sp2_status sp2_get_norm_times(sp2_ctx c, int32_t cap, int32_t* len,
                              float* ms) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->ran || !c->timed || c->opt.norm != SP2_NORM_SPECTRAL)
    return SP2_BAD_STATE;
  const int m = static_cast<int>(c->norm_ms.size());
  if (len) *len = m;
  if (ms)
    for (int i = 0; i < cap && i < m; ++i) ms[i] = c->norm_ms[i];
  return SP2_OK;
}

sp2_status sp2_get_history(sp2_ctx c, int32_t cap, int32_t* len, double* v,
                           double* t1, double* t2, int8_t* p, double* r) {
  return sp2_batch_get_history(c, 0, cap, len, v, t1, t2, p, r);
}

sp2_status sp2_run_dense_noalloc(int device, void* hip_stream,
                                 const double* F_dev, int64_t n, int64_t ldf,
                                 double lambda_min, double lambda_max,
                                 int64_t n_occ, const sp2_options* opt_in,
                                 void* D_dev, int64_t ldd, int32_t as_fp64,
                                 int32_t cap, double* v, int32_t* n_iter,
                                 int32_t* n_squares) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev ||
      device >= kScratchDevices)
    return SP2_INVALID_ARG;
  sp2_ctx_s ctx;
  sp2_ctx c = &ctx;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  sp2_options opt;
  if (opt_in) {
    opt = *opt_in;
  } else {
    sp2_default_options(&opt);
  }
  sp2_status st = validate_options(c, opt);
  if (st != SP2_OK) return st;
  if (opt.norm != SP2_NORM_FROBENIUS || opt.tail_split > 1 ||
      opt.kernel_timing != 0 || cap < 0 || (cap > 0 && !v))
    return SP2_INVALID_ARG;
  opt.tail_split = 1;   // whole tiles only: no tail workspace
  st = validate_instance(c, F_dev, n, ldf, lambda_min, lambda_max, n_occ);
  if (st != SP2_OK) return st;
  if (!D_dev || ldd < n) return SP2_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return SP2_HIP_ERROR;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                            device) == hipSuccess && cus > 0)
    c->num_cus = cus;
  st = scratch_on_device(device, &c->arena);
  if (st != SP2_OK) return st;
  c->arena_cap = kScratchBytes;
  size_t nd_cap = 0;
  if (grow(c, c->d_ndone, nd_cap, 256, c->stream) != hipSuccess)
    return SP2_INVALID_ARG;
  HostInst h;
  h.F = F_dev;
  h.n = n;
  h.ldf = ldf;
  h.lmin = lambda_min;
  h.lmax = lambda_max;
  h.n_occ = n_occ;
  c->hi.assign(1, h);
  c->bsr = false;
  c->opt = opt;
  c->fp64_store = (opt.precision == SP2_FP64);
  st = setup(c);
  // workspaces that do not fit the scratch: the input is too large
  if (st == SP2_OUT_OF_MEMORY) return SP2_INVALID_ARG;
  if (st != SP2_OK) return st;
  c->inited = true;
  st = run_batch(c);
  if (st != SP2_OK) return st;
  st = copy_density(c, 0, D_dev, ldd, as_fp64);
  if (st != SP2_OK) return st;
  const DevState& hs = c->host_state[0];
  const int sq = c->hi[0].trivial ? 0 : hs.squares;
  if (n_iter) *n_iter = hs.n;
  if (n_squares) *n_squares = sq;
  for (int k = 0; k < cap; ++k) v[k] = k < sq ? hs.v[k] : NAN;
  return static_cast<sp2_status>(hs.status);
}

}  // extern "C"
