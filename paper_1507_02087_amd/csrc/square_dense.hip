// Fused symmetric square of the SP2 recursion on gfx950 matrix cores:
// the table of compiled configurations and the dispatch to the per-family
// translation units (kernels in square_impl.h), and the queue kernels of
// the persistent batch driver.
#include "square_impl.h"

namespace sp2 {
namespace {

template <class C>
struct Presplit {
  static constexpr int value = 0;
};
template <int A, int B, int Cc, int D>
struct Presplit<CfgB3P<A, B, Cc, D>> {
  static constexpr int value = 1;
};


template <class C>
constexpr KernelConfig describe(int precision, int occupancy,
                                const char* name) {
  return KernelConfig{precision, C::BM, C::WM,     C::WN,
                      C::BK,     C::THREADS, occupancy, name,
                      Presplit<C>::value};
}
#define SP2_DESCRIBE(C, prec, occ) describe<C>(prec, occ, #C)

// Occupancy = workgroups per CU that the configuration's LDS and registers
// allow; the host uses it to size the split of tail tiles.
const KernelConfig kConfigs[] = {
    SP2_DESCRIBE(F64_128_2x4, 0, 2), SP2_DESCRIBE(F64_128_2x2, 0, 1),
    SP2_DESCRIBE(F64_64_2x2, 0, 2),  SP2_DESCRIBE(F32_128_2x2, 1, 2),
    SP2_DESCRIBE(F32_128_2x4, 1, 1), SP2_DESCRIBE(F32_256_2x2, 1, 1),
    SP2_DESCRIBE(B3_128_2x2, 2, 1),  SP2_DESCRIBE(B3_256_2x2, 2, 1),
    SP2_DESCRIBE(B3_256_2x4, 2, 1),  SP2_DESCRIBE(B3S_256_2x4, 2, 1),
    SP2_DESCRIBE(B3S_256_2x4_16, 2, 1), SP2_DESCRIBE(B3S_128_2x2, 2, 2),
    SP2_DESCRIBE(B3P_256_2x4, 2, 1), SP2_DESCRIBE(B3P_256_2x4_32, 2, 1),
    SP2_DESCRIBE(B3P_128_2x2, 2, 2), SP2_DESCRIBE(F32_256_2x4, 1, 1),
    SP2_DESCRIBE(B3P_256_4x4_32, 2, 1),
};
constexpr int kNumConfigs = sizeof(kConfigs) / sizeof(kConfigs[0]);


// One workgroup per instance after the affine start's finalize: publishes
// step 1 of every instance still running. The queue was cleared before.
__global__ __launch_bounds__(256) void persist_seed_kernel(
    const Instance* __restrict__ insts, PQueue q) {
  __shared__ int base_sh;
  const Instance& in = insts[blockIdx.x];
  if (threadIdx.x == 0) {
    int base = -1;
    if (!in.st->done && in.ntiles > 0) {
      base = __hip_atomic_fetch_add(q.ctl + 1, in.ntiles, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
      if (base + in.ntiles > q.cap) base = -1;
    }
    base_sh = base;
  }
  __syncthreads();
  if (base_sh >= 0)
    persist_publish<256>(q, base_sh, blockIdx.x, in.tile0, in.ntiles, 1);
}

__global__ __launch_bounds__(256) void persist_clear_kernel(PQueue q) {
  const int g = blockIdx.x * 256 + threadIdx.x, stride = gridDim.x * 256;
  for (int i = g; i < q.cap; i += stride) q.items[i].seq = 0;
  for (int i = g; i < q.count; i += stride) q.cnt[i] = 0;
  if (g < 3) q.ctl[g] = 0;
}

}  // namespace

int kernel_config_count() { return kNumConfigs; }

const KernelConfig* kernel_config(int id) {
  return (id >= 0 && id < kNumConfigs) ? &kConfigs[id] : nullptr;
}

// The persistent kernel is compiled for the configurations a batch of
// instances of up to a few thousand rows uses: 64- and 128-tiles.
bool persist_supported(int cfg) {
  return cfg == 0 || cfg == 2 || cfg == 3 || cfg == 4 || cfg == 6 || cfg == 11 ||
         cfg == 14;
}

int persist_grid(int cfg, bool stretch, int num_cus) {
  switch (cfg) {
    case 0: return persist_grid_f64(cfg, stretch, num_cus);
    case 2: return persist_grid_f64(cfg, stretch, num_cus);
    case 3: return persist_grid_f32(cfg, stretch, num_cus);
    case 4: return persist_grid_f32(cfg, stretch, num_cus);
    case 6: return persist_grid_b3(cfg, stretch, num_cus);
    case 11: return persist_grid_b3s(cfg, stretch, num_cus);
    case 14: return persist_grid_b3p(cfg, stretch, num_cus);
    default: return 0;
  }
}

hipError_t launch_persist(int cfg, const SquareArgs& a, const PQueue& q,
                          int grid, hipStream_t s) {
  switch (cfg) {
    case 0: return launch_persist_f64(cfg, a, q, grid, s);
    case 2: return launch_persist_f64(cfg, a, q, grid, s);
    case 3: return launch_persist_f32(cfg, a, q, grid, s);
    case 4: return launch_persist_f32(cfg, a, q, grid, s);
    case 6: return launch_persist_b3(cfg, a, q, grid, s);
    case 11: return launch_persist_b3s(cfg, a, q, grid, s);
    case 14: return launch_persist_b3p(cfg, a, q, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_persist_seed(const Instance* inst, int count, const PQueue& q,
                               hipStream_t s) {
  const int g = std::max(1, std::min(1024, (q.cap + 255) / 256));
  hipLaunchKernelGGL(persist_clear_kernel, dim3(g), dim3(256), 0, s, q);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(persist_seed_kernel, dim3(count), dim3(256), 0, s, inst, q);
  return hipGetLastError();
}

hipError_t launch_square(int id, const SquareArgs& a, int grid, hipStream_t s) {
  switch (id) {
    case 0: return launch_square_f64(id, a, grid, s);
    case 1: return launch_square_f64(id, a, grid, s);
    case 2: return launch_square_f64(id, a, grid, s);
    case 3: return launch_square_f32(id, a, grid, s);
    case 4: return launch_square_f32(id, a, grid, s);
    case 5: return launch_square_f32(id, a, grid, s);
    case 6: return launch_square_b3(id, a, grid, s);
    case 7: return launch_square_b3(id, a, grid, s);
    case 8: return launch_square_b3(id, a, grid, s);
    case 9: return launch_square_b3s(id, a, grid, s);
    case 10: return launch_square_b3s(id, a, grid, s);
    case 11: return launch_square_b3s(id, a, grid, s);
    case 12: return launch_square_b3p(id, a, grid, s);
    case 13: return launch_square_b3p(id, a, grid, s);
    case 14: return launch_square_b3p(id, a, grid, s);
    case 15: return launch_square_f32(id, a, grid, s);
    case 16: return launch_square_b3p(id, a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sp2
