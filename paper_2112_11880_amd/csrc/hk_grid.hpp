// hk_grid.hpp -- grid-wide barrier for the persistent batched solvers.
//
// The persistent kernels are launched cooperatively (every workgroup
// resident), so a barrier cannot deadlock on scheduling.  The barrier is a
// flag array: each workgroup publishes the barrier's epoch in its own word
// (after a release fence for the data it wrote), workgroup 0 waits until
// every word shows the epoch, runs a callback (the second stage of the
// reductions and the per-system scalar updates), then publishes the epoch in
// a release word that the other workgroups wait on.  A single shared counter
// incremented by every workgroup cost ~136 us per barrier on MI355X (256
// serialised device-scope atomics); flags in separate words cost a few
// round trips.
//
// Only thread 0 of a workgroup fences; the workgroup barrier that follows
// orders the other threads after it (the usual grid-sync pattern).  On
// gfx950 an agent-scope acquire fence invalidates caches, and executing it in
// all 16 waves of a 1024-thread workgroup made one barrier cost ~63 us (one
// wave: a few us).  Each fence is one-sided: a release (L2 write-back) before
// a flag is published, an acquire (L2 invalidate) after one is observed.
// Two-sided fences at both points cost ~25 us more per solver iteration
// (5 barriers) on MI355X.
//
// Every wait has a time limit: a workgroup that waits longer than the
// barrier's spin_limit (kSpinLimitTicks unless the host sets another) raises
// an abort flag and every workgroup leaves the kernel at its next barrier,
// so a broken launch ends instead of hanging.
#pragma once

#include <cstdlib>

#include "hk_common.hpp"

namespace hk {

constexpr int kBarMaxBlocks = 1024;

struct GridBar {
  unsigned release;      // last epoch released by workgroup 0
  int abort;
  unsigned long long spin_limit;  // wall-clock ticks a wait may take before it aborts
  // optional: stamps[e] = wall clock (100 MHz ticks) when every workgroup had
  // arrived at barrier e, for e < nstamps (null: none)
  double* stamps;
  unsigned long long nstamps;
  // per-XCD-group sums of barrier_reduce: kXcds x 4 x 64 doubles (null if unused)
  double* gpart;
  unsigned pad[54];      // keep release/abort on their own 256-byte line
  unsigned arrive[kBarMaxBlocks];  // last epoch each workgroup arrived at
  unsigned garrive[kXcds];         // last epoch each group's sums were published at
};

// 100 MHz constant clock: 4e8 ticks = 4 s.
constexpr unsigned long long kSpinLimitTicks = 400000000ull;

__device__ __forceinline__ unsigned ld_relaxed_u32(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_relaxed_i32(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed_u32(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits (one thread) until *p >= e; false on abort or time-out (which raises abort).
__device__ __forceinline__ bool wait_epoch(const unsigned* p, unsigned e, GridBar* bar) {
  const unsigned long long t0 = wall_clock64();
  const unsigned long long limit = bar->spin_limit;
  while (ld_relaxed_u32(p) < e) {
    __builtin_amdgcn_s_sleep(1);
    if (ld_relaxed_i32(&bar->abort)) return false;
    if (wall_clock64() - t0 > limit) {
      atomicExch(&bar->abort, 1);
      return false;
    }
  }
  return true;
}

// Grid barrier; on_last() runs in workgroup 0 (all its threads) once every
// workgroup has arrived.  `epoch` is the caller's per-workgroup counter
// (start at 0; the barrier memory must be zeroed before the launch).
// Returns true if the kernel must stop (abort raised somewhere).  All
// threads of every workgroup must call it.
template <class F>
__device__ __forceinline__ bool barrier_last(GridBar* bar, unsigned& epoch, F&& on_last) {
  __shared__ int s_stop;
  const unsigned e = ++epoch;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this workgroup's writes before its flag
    st_relaxed_u32(&bar->arrive[blockIdx.x], e);
  }
  if (blockIdx.x == 0) {
    bool ok = true;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) ok = wait_epoch(&bar->arrive[b], e, bar) && ok;
    if (!ok) atomicExch(&bar->abort, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
      s_stop = ld_relaxed_i32(&bar->abort);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every workgroup's writes
      if (bar->stamps && e < bar->nstamps) bar->stamps[e] = (double)wall_clock64();
    }
    __syncthreads();
    if (!s_stop) on_last();
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the callback's writes before the epoch
      st_relaxed_u32(&bar->release, e);
    }
  } else if (threadIdx.x == 0) {
    (void)wait_epoch(&bar->release, e, bar);
  }
  if (threadIdx.x == 0) {
    s_stop = ld_relaxed_i32(&bar->abort);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // workgroup 0's release, and through it every arrival
  }
  __syncthreads();
  return s_stop != 0;
}

// Host: the spin limit of a launch, kSpinLimitTicks unless the environment
// variable HK_BARRIER_SPIN_TICKS holds a positive count (tests use a tiny
// one to drive the abort path).
inline unsigned long long barrier_spin_limit() {
  const char* v = getenv("HK_BARRIER_SPIN_TICKS");
  if (v) {
    const unsigned long long t = strtoull(v, nullptr, 10);
    if (t > 0) return t;
  }
  return kSpinLimitTicks;
}

}  // namespace hk
