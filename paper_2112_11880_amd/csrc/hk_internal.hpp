// hk_internal.hpp -- host-side plumbing shared by the libhk translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/hk.h"

namespace hk {

// Thread-local text of the last failure, returned by hk_last_error().
void set_error_text(const char* fmt, ...);
const char* error_text();

#define HK_FAIL(code, ...)              \
  do {                                  \
    ::hk::set_error_text(__VA_ARGS__);  \
    return (code);                      \
  } while (0)

#define HK_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      HK_FAIL(HK_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
              __LINE__);                                                              \
  } while (0)

#define HK_CHECK_LAUNCH() HK_HIP(hipGetLastError())

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Per-(device, stream) scratch for the partial sums of the BLAS-1
// reductions.  Grows on demand; lives until the process ends.
struct ReduceScratch {
  void* partials = nullptr;
  size_t bytes = 0;
};
int reduce_scratch(hipStream_t s, size_t bytes, ReduceScratch** out);

// Launch shape of a CSR product: lanes per row, rows per lane group, grid.
struct SpmvPlan {
  int L = 16;
  int U = 2;
  int grid = 0;     // workgroups per launch (0: one per tile)
  int tuned = 0;    // 1 if chosen by timing on the device
  int nw = 0;       // row-block fused solver kernels: waves per workgroup (0: the fewest that fit)
  int pairs = 0;    // row-block fused solver kernels: paired-entry layout (16-bit column stream only)
};

}  // namespace hk

// The opaque matrix handle.
struct hk_csr_s {
  int64_t n = 0, nnz = 0;
  const int32_t* rowptr = nullptr;
  const int32_t* col = nullptr;
  const void* val = nullptr;
  // 16-bit column offsets from each row's 64-aligned base (owned; null when
  // an offset exceeds 32767 or HK_INT32_COLS was given): the column stream
  // of the row-block products, nnz entries plus one zero padding entry
  int16_t* col16 = nullptr;
  int dtype = HK_C128;
  int device = 0;
  int max_row = 0;         // longest row (host copy, from the validation pass)
  hk::SpmvPlan plan;
  // solver workspace (device), allocated on first solve, freed by destroy
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // complex64 copy of the values for the mixed-precision solve, and the
  // launch shape tuned for it (when the handle was tuned)
  void* val32 = nullptr;
  hk::SpmvPlan plan32;
  void* ws32 = nullptr;
  size_t ws32_bytes = 0;
  // launch shapes of the solver's fused SpMV+dot kernels, tuned on the
  // first solve of a tuned handle ([0] complex128, [1] complex64)
  hk::SpmvPlan dot_plan[2];
  // pinned host words the solver reads its status through
  int* pinned = nullptr;
};

namespace hk {
int spmv_tiles(const hk_csr_s* A, int L, int U);
// Times every launch shape of the CSR product on A (its dtype and values)
// and stores the fastest in A->plan (cached per matrix shape and dtype).
int spmv_autotune(hk_csr_s* A, hipStream_t s);
int default_grid(int ntiles);
}
