// hk_grid.hpp -- grid-wide barrier for the persistent batched solvers.
//
// The persistent kernels are launched cooperatively (every workgroup
// resident), so a counter barrier cannot deadlock on scheduling.  The
// barrier still has a time limit: a workgroup that waits longer than
// kSpinLimitTicks sets an abort flag and every workgroup leaves the kernel
// at its next barrier, so a broken launch ends instead of hanging.
//
// barrier_last(): the workgroup that arrives last runs a callback (the
// second stage of the reductions and the per-system scalar updates) before
// releasing the others, which then read the published values.
#pragma once

#include "hk_common.hpp"

namespace hk {

struct GridBar {
  unsigned count;
  unsigned gen;
  int abort;
  int pad;
};

// 100 MHz constant clock: 4e8 ticks = 4 s.
constexpr unsigned long long kSpinLimitTicks = 400000000ull;

__device__ __forceinline__ unsigned ld_acquire_u32(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_acquire_i32(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Returns true if the kernel must stop (abort raised by some workgroup).
// All threads of the block must call it; the result is uniform in the block.
template <class F>
__device__ __forceinline__ bool barrier_last(GridBar* bar, F&& on_last) {
  __shared__ int s_last;
  __shared__ int s_stop;
  __shared__ unsigned s_gen;
  __syncthreads();
  if (threadIdx.x == 0) {
    s_gen = ld_acquire_u32(&bar->gen);
    __threadfence();
    const unsigned a = atomicAdd(&bar->count, 1u);
    s_last = (a == gridDim.x - 1);
  }
  __syncthreads();
  if (s_last) {
    __threadfence();
    on_last();
    __syncthreads();
    if (threadIdx.x == 0) {
      atomicExch(&bar->count, 0u);
      __threadfence();
      atomicAdd(&bar->gen, 1u);
    }
  } else if (threadIdx.x == 0) {
    const unsigned long long t0 = wall_clock64();
    while (ld_acquire_u32(&bar->gen) == s_gen) {
      __builtin_amdgcn_s_sleep(2);
      if (ld_acquire_i32(&bar->abort)) break;
      if (wall_clock64() - t0 > kSpinLimitTicks) {
        atomicExch(&bar->abort, 1);
        break;
      }
    }
  }
  if (threadIdx.x == 0) s_stop = ld_acquire_i32(&bar->abort);
  __syncthreads();
  __threadfence();
  return s_stop != 0;
}

}  // namespace hk
