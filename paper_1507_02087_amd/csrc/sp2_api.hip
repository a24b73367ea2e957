// Host driver and C ABI of the SP2 library (see include/sp2.h).
//
// A run is a stream-ordered sequence of kernels:
//   state reset -> f0 (X_0 and its traces) -> finalize(0)
//   -> for i = 1, 2, ...: square(i) -> finalize(i)
// The polynomial choice, the stop test and the outcome live in device memory
// (DevState); the finalize kernel also mirrors the outcome into host-coherent
// pinned memory. The host keeps up to kLookahead steps queued ahead of the
// step whose outcome it last observed, so the device never waits on the host;
// steps queued after the stop return at once because every kernel first
// reads the device-side done flag.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/sp2.h"
#include "sp2_device.h"

using sp2::DevState;
using sp2::HostMirror;

namespace {

constexpr int kLookahead = 3;
constexpr int kRing = 8;
constexpr int kF0Rows = 8;

}  // namespace

struct sp2_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;

  // problem
  const double* F = nullptr;
  int64_t n = 0, ldf = 0, n_occ = 0, np = 0;
  double lmin = 0.0, lmax = 0.0;
  sp2_options opt{};
  int tile = 128;
  bool fp64_store = true;

  // workspaces
  void* X[2] = {nullptr, nullptr};
  size_t x_bytes = 0;
  double* part = nullptr;
  size_t part_count = 0;
  int2* tiles = nullptr;
  size_t tiles_cap = 0;
  int ntiles = 0;
  int per_xcd = 0;
  DevState* st = nullptr;
  HostMirror* mirror = nullptr;
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
  hipEvent_t ev_ring[kRing] = {};
  std::vector<hipEvent_t> ev_sq;   // pairs around each square when timing
  std::vector<float> square_ms;
  bool timed = false;

  // outcome
  bool inited = false, ran = false;
  sp2_status last = SP2_BAD_STATE;
  int32_t n_iter = 0, n_squares = 0;
  double run_ms = 0.0;
  int result_buf = 0;
  DevState host_state{};
  bool trivial = false;  // n_occ == 0 or n_occ == n
};

namespace {

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

int default_tile(int precision, int64_t n) {
  (void)precision;
  (void)n;
  return 128;
}

// Upper-triangle tiles (I <= J) of an nt x nt tile grid, ordered by groups of
// G x G neighbouring tiles so that consecutive list entries share row panels.
std::vector<int2> build_tile_list(int nt) {
  const int G = 4;
  std::vector<int2> out;
  out.reserve(static_cast<size_t>(nt) * (nt + 1) / 2);
  for (int gi = 0; gi < nt; gi += G)
    for (int gj = gi; gj < nt; gj += G)
      for (int i = gi; i < gi + G && i < nt; ++i)
        for (int j = gj; j < gj + G && j < nt; ++j)
          if (i <= j) out.push_back(make_int2(i, j));
  return out;
}

sp2_status ensure_events(sp2_ctx c) {
  if (c->ev_start) return SP2_OK;
  SP2_HIP(c, hipEventCreate(&c->ev_start));
  SP2_HIP(c, hipEventCreate(&c->ev_stop));
  for (int i = 0; i < kRing; ++i)
    SP2_HIP(c, hipEventCreateWithFlags(&c->ev_ring[i], hipEventDisableTiming));
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
  opt->tile = 0;
  opt->kernel_timing = 0;
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

int32_t sp2_tile_supported(int32_t precision, int32_t tile) {
  if (precision < SP2_FP64 || precision > SP2_BF16X3) return 0;
  return sp2::square_tile_supported(precision, tile) ? 1 : 0;
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
  if (e == hipSuccess) e = hipMalloc(&c->st, sizeof(DevState));
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&c->mirror), sizeof(HostMirror),
                      hipHostMallocCoherent | hipHostMallocMapped);
  if (e != hipSuccess) {
    sp2_destroy(c);
    return e == hipErrorOutOfMemory ? SP2_OUT_OF_MEMORY : SP2_HIP_ERROR;
  }
  memset(c->mirror, 0, sizeof(HostMirror));
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
  for (void* p : c->X)
    if (p) (void)hipFree(p);
  if (c->part) (void)hipFree(c->part);
  if (c->tiles) (void)hipFree(c->tiles);
  if (c->st) (void)hipFree(c->st);
  if (c->mirror) (void)hipHostFree(c->mirror);
  if (c->ev_start) (void)hipEventDestroy(c->ev_start);
  if (c->ev_stop) (void)hipEventDestroy(c->ev_stop);
  for (hipEvent_t e : c->ev_ring)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ev_sq)
    if (e) (void)hipEventDestroy(e);
  delete c;
  return SP2_OK;
}

sp2_status sp2_init_dense(sp2_ctx c, const double* F_dev, int64_t n,
                          int64_t ldf, double lambda_min, double lambda_max,
                          int64_t n_occ, const sp2_options* opt_in) {
  if (!c) return SP2_INVALID_ARG;
  c->err.clear();
  c->inited = false;
  c->ran = false;
  sp2_options opt;
  if (opt_in) {
    opt = *opt_in;
  } else {
    sp2_default_options(&opt);
  }
  if (opt.max_iter == 0) opt.max_iter = 100;
  if (!F_dev) return fail(c, SP2_INVALID_ARG, "F_dev is NULL", hipSuccess);
  if (n <= 0 || n > 65536)
    return fail(c, SP2_INVALID_ARG, "n must be in [1, 65536]", hipSuccess);
  if (ldf < n) return fail(c, SP2_INVALID_ARG, "ldf < n", hipSuccess);
  if (n_occ < 0 || n_occ > n)
    return fail(c, SP2_INVALID_ARG, "n_occ outside [0, n]", hipSuccess);
  if (!isfinite(lambda_min) || !isfinite(lambda_max) ||
      !(lambda_max > lambda_min) || !isfinite(lambda_max - lambda_min))
    return fail(c, SP2_INVALID_ARG,
                "spectral bounds must be finite with lambda_max > lambda_min",
                hipSuccess);
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
  int tile = opt.tile ? opt.tile : default_tile(opt.precision, n);
  if (!sp2::square_tile_supported(opt.precision, tile))
    return fail(c, SP2_INVALID_ARG, "unsupported tile", hipSuccess);

  SP2_HIP(c, hipSetDevice(c->device));
  const int64_t np = ((n + tile - 1) / tile) * tile;
  const bool fp64 = (opt.precision == SP2_FP64);
  const size_t xb = static_cast<size_t>(np) * np * (fp64 ? 8 : 4);
  if (xb > c->x_bytes) {
    SP2_HIP(c, hipStreamSynchronize(c->stream));
    for (void*& p : c->X) {
      if (p) (void)hipFree(p);
      p = nullptr;
    }
    c->x_bytes = 0;
    for (void*& p : c->X) SP2_HIP(c, hipMalloc(&p, xb));
    c->x_bytes = xb;
  }
  const int nt = static_cast<int>(np / tile);
  std::vector<int2> tl = build_tile_list(nt);
  const size_t f0_blocks = static_cast<size_t>(np / kF0Rows);
  const size_t need_part = std::max(tl.size(), f0_blocks);
  if (need_part > c->part_count) {
    SP2_HIP(c, hipStreamSynchronize(c->stream));
    if (c->part) (void)hipFree(c->part);
    c->part = nullptr;
    c->part_count = 0;
    SP2_HIP(c, hipMalloc(&c->part, need_part * 3 * sizeof(double)));
    c->part_count = need_part;
  }
  if (tl.size() > c->tiles_cap) {
    SP2_HIP(c, hipStreamSynchronize(c->stream));
    if (c->tiles) (void)hipFree(c->tiles);
    c->tiles = nullptr;
    c->tiles_cap = 0;
    SP2_HIP(c, hipMalloc(&c->tiles, tl.size() * sizeof(int2)));
    c->tiles_cap = tl.size();
  }
  SP2_HIP(c, hipMemcpyAsync(c->tiles, tl.data(), tl.size() * sizeof(int2),
                            hipMemcpyHostToDevice, c->stream));
  SP2_HIP(c, hipStreamSynchronize(c->stream));
  c->ntiles = static_cast<int>(tl.size());
  c->per_xcd = (c->ntiles + 7) / 8;
  c->F = F_dev;
  c->n = n;
  c->ldf = ldf;
  c->n_occ = n_occ;
  c->np = np;
  c->lmin = lambda_min;
  c->lmax = lambda_max;
  c->opt = opt;
  c->tile = tile;
  c->fp64_store = fp64;
  c->inited = true;
  return SP2_OK;
}

sp2_status sp2_run(sp2_ctx c) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->inited) return fail(c, SP2_BAD_STATE, "sp2_run before init", hipSuccess);
  c->err.clear();
  c->ran = false;
  SP2_HIP(c, hipSetDevice(c->device));
  hipStream_t s = c->stream;
  const int n = static_cast<int>(c->n), np = static_cast<int>(c->np);

  c->trivial = (c->n_occ == 0 || c->n_occ == c->n);
  SP2_HIP(c, hipEventRecord(c->ev_start, s));
  SP2_HIP(c, sp2::launch_state_reset(c->st, s));
  if (c->trivial) {
    SP2_HIP(c, sp2::launch_fill(c->X[0], c->fp64_store, n, np,
                                c->n_occ == c->n ? 1 : 0, s));
    SP2_HIP(c, hipEventRecord(c->ev_stop, s));
    SP2_HIP(c, hipEventSynchronize(c->ev_stop));
    float ms = 0.f;
    SP2_HIP(c, hipEventElapsedTime(&ms, c->ev_start, c->ev_stop));
    memset(&c->host_state, 0, sizeof(DevState));
    c->host_state.p[0] = -1;
    c->result_buf = 0;
    c->n_iter = 0;
    c->n_squares = 0;
    c->run_ms = ms;
    c->last = SP2_OK;
    c->ran = true;
    return SP2_OK;
  }

  c->mirror->done = 0;
  c->mirror->status = 0;
  c->mirror->n = 0;
  c->mirror->squares = 0;
  __atomic_thread_fence(__ATOMIC_SEQ_CST);

  sp2::StopParams prm;
  prm.n_occ = static_cast<double>(c->n_occ);
  prm.n = static_cast<double>(c->n);
  prm.branch = c->opt.branch;
  prm.max_iter = c->opt.max_iter;

  SP2_HIP(c, sp2::launch_f0(c->F, c->ldf, n, np, c->lmax, c->lmax - c->lmin,
                            c->opt.trunc_tau, c->X[0], c->fp64_store, c->part,
                            kF0Rows, s));
  SP2_HIP(c, sp2::launch_finalize(c->part, np / kF0Rows, c->st, c->mirror, 0,
                                  prm, s));
  SP2_HIP(c, hipEventRecord(c->ev_ring[0], s));

  const bool timing = c->opt.kernel_timing != 0;
  if (timing && c->ev_sq.empty()) {
    c->ev_sq.assign(2 * (SP2_MAX_ITER_LIMIT + 1), nullptr);
    for (hipEvent_t& e : c->ev_sq) SP2_HIP(c, hipEventCreate(&e));
  }
  c->timed = false;
  c->square_ms.clear();

  sp2::SquareArgs a;
  a.ld = np;
  a.tiles = c->tiles;
  a.ntiles = c->ntiles;
  a.per_xcd = c->per_xcd;
  a.st = c->st;
  a.part = c->part;
  a.tau = c->opt.trunc_tau;
  for (int i = 1; i <= c->opt.max_iter; ++i) {
    if (i > kLookahead) {
      SP2_HIP(c, hipEventSynchronize(c->ev_ring[(i - kLookahead) % kRing]));
      if (__atomic_load_n(&c->mirror->done, __ATOMIC_ACQUIRE)) break;
    }
    a.X = c->X[(i - 1) & 1];
    a.Y = c->X[i & 1];
    a.iter = i;
    if (timing) SP2_HIP(c, hipEventRecord(c->ev_sq[2 * i], s));
    hipError_t e;
    switch (c->opt.precision) {
      case SP2_FP64: e = sp2::launch_square_f64(a, c->tile, s); break;
      case SP2_FP32: e = sp2::launch_square_f32(a, c->tile, s); break;
      default: e = sp2::launch_square_bf16x3(a, c->tile, s); break;
    }
    SP2_HIP(c, e);
    if (timing) SP2_HIP(c, hipEventRecord(c->ev_sq[2 * i + 1], s));
    SP2_HIP(c, sp2::launch_finalize(c->part, c->ntiles, c->st, c->mirror, i,
                                    prm, s));
    SP2_HIP(c, hipEventRecord(c->ev_ring[i % kRing], s));
  }
  SP2_HIP(c, hipEventRecord(c->ev_stop, s));
  SP2_HIP(c, hipEventSynchronize(c->ev_stop));
  float ms = 0.f;
  SP2_HIP(c, hipEventElapsedTime(&ms, c->ev_start, c->ev_stop));
  SP2_HIP(c, hipMemcpyAsync(&c->host_state, c->st, sizeof(DevState),
                            hipMemcpyDeviceToHost, s));
  SP2_HIP(c, hipStreamSynchronize(s));
  const DevState& h = c->host_state;
  if (!h.done)
    return fail(c, SP2_BAD_STATE, "run ended without an outcome", hipSuccess);
  c->run_ms = ms;
  c->n_iter = h.n;
  c->n_squares = h.squares;
  c->result_buf = h.n & 1;
  c->last = static_cast<sp2_status>(h.status);
  if (timing) {
    for (int i = 1; i <= h.squares; ++i) {
      float t = 0.f;
      SP2_HIP(c, hipEventElapsedTime(&t, c->ev_sq[2 * i], c->ev_sq[2 * i + 1]));
      c->square_ms.push_back(t);
    }
    c->timed = true;
  }
  c->ran = true;
  return c->last;
}

sp2_status sp2_get_density(sp2_ctx c, void* D_dev, int64_t ldd,
                           int32_t as_fp64) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->ran) return fail(c, SP2_BAD_STATE, "no completed run", hipSuccess);
  if (!D_dev || ldd < c->n)
    return fail(c, SP2_INVALID_ARG, "D_dev NULL or ldd < n", hipSuccess);
  SP2_HIP(c, hipSetDevice(c->device));
  SP2_HIP(c, sp2::launch_copy_out(c->X[c->result_buf], c->fp64_store,
                                  static_cast<int>(c->n),
                                  static_cast<int>(c->np), D_dev, ldd,
                                  as_fp64 != 0, c->stream));
  SP2_HIP(c, hipStreamSynchronize(c->stream));
  return SP2_OK;
}

sp2_status sp2_get_info(sp2_ctx c, int32_t* n_iter, int32_t* n_squares,
                        double* run_ms) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->ran) return SP2_BAD_STATE;
  if (n_iter) *n_iter = c->n_iter;
  if (n_squares) *n_squares = c->n_squares;
  if (run_ms) *run_ms = c->run_ms;
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

sp2_status sp2_get_history(sp2_ctx c, int32_t cap, int32_t* len, double* v,
                           double* t1, double* t2, int8_t* p, double* r) {
  if (!c) return SP2_INVALID_ARG;
  if (!c->ran) return SP2_BAD_STATE;
  if (cap < 0) return SP2_INVALID_ARG;
  const DevState& h = c->host_state;
  const int nv = c->n_squares;
  if (len) *len = nv;
  // Traces exist for X~_0 .. X~_m where m is the last iterate formed.
  int nt = c->trivial ? 0 : nv + 1;
  if (!c->trivial && h.status == SP2_DIVERGED && h.n == 0 && nv == 0) nt = 1;
  for (int k = 0; k < cap; ++k) {
    if (v) v[k] = k < nv ? h.v[k] : NAN;
    if (r) r[k] = k < nv ? h.r[k] : NAN;
    if (t1) t1[k] = k < nt ? h.t1[k] : NAN;
    if (t2) t2[k] = k < nt ? h.t2[k] : NAN;
    if (p) p[k] = k < nt ? (k == 0 ? -1 : h.p[k]) : -1;
  }
  return SP2_OK;
}

}  // extern "C"
