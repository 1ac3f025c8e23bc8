// hk_spmv.hip -- CSR matrix handles, the CSR product and its launch-shape tuner.
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "hk_internal.hpp"
#include "hk_spmv.hpp"

namespace hk {

// ----------------------------------------------------------------- kernels

// MODE 0: y = alpha*A*x + beta*y (beta_zero: y not read)
// MODE 1: y = b - A*x
template <int L, int U, class V, int MODE>
__global__ __launch_bounds__(kBlock) void k_spmv(int n, int ntiles, const int* __restrict__ rowptr,
                                                 const int* __restrict__ col,
                                                 const V* __restrict__ val, const V* __restrict__ x,
                                                 V* __restrict__ y, const V* __restrict__ b,
                                                 V alpha, V beta, int beta_zero) {
  constexpr int RT = (kBlock / L) * U;
  const int g = threadIdx.x / L, lane = threadIdx.x & (L - 1);
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int r0 = t * RT + g * U;
    V acc[U];
    csr_rows<L, U, V>(r0, n, rowptr, col, val, x, acc);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = r0 + u;
      if (lane == u && r < n) {
        V out;
        if (MODE == 1) {
          out = csub(b[r], acc[u]);
        } else {
          out = cmul(alpha, acc[u]);
          if (!beta_zero) out = cfma(beta, y[r], out);
        }
        stnt(y + r, out);
      }
    }
  }
}

// Row-block variant: R rows per wave, a tile is kRbWaves * R rows.
template <int R, class V, int MODE, class CI>
__global__ __launch_bounds__(kRbThreads) void k_spmv_rb(int n, int ntiles, const int* __restrict__ rowptr,
                                                        const CI* __restrict__ col,
                                                        const V* __restrict__ val, const V* __restrict__ x,
                                                        V* __restrict__ y, const V* __restrict__ b,
                                                        V alpha, V beta, int beta_zero) {
  constexpr int CH = RbCh<R, V>::v;
  __shared__ V lds[kRbWaves * CH * kWave];
  V* buf = lds + (threadIdx.x / kWave) * CH * kWave;
  const int l = threadIdx.x & (kWave - 1);
  for (int tb = blockIdx.x; tb < ntiles; tb += gridDim.x) {
    const int t = R == 32   ? tile_of<kSpmvTileChunk>(tb, ntiles)
                  : R == 16 ? tile_of<kSpmvTileChunk16>(tb, ntiles)
                            : tile_of(tb, ntiles);
    const int r0 = t * (kRbWaves * R) + (threadIdx.x / kWave) * R;
    const V acc = csr_block_rows<R, CH, V, CI>(r0, n, rowptr, col, val, x, buf);
    const int r = r0 + l;
    if (l < R && r < n) {
      V out;
      if (MODE == 1) {
        out = csub(b[r], acc);
      } else {
        out = cmul(alpha, acc);
        if (!beta_zero) out = cfma(beta, y[r], out);
      }
      // a non-temporal store keeps y out of the L2, which holds the x
      // window: 107.6 -> 99.6 us per product on the 1.8M-row system
      stnt(y + r, out);
    }
  }
}

// Structure check of a CSR matrix.  flags[0] |= 1 on any violation,
// flags[1] = longest row, flags[2] = largest |col - (row & ~63)|.
__global__ void k_csr_check(int n, int nnz, const int* __restrict__ rowptr,
                            const int* __restrict__ col, int* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = rowptr[i], e = rowptr[i + 1];
  int bad = 0, far = 0;
  if (i == 0 && s != 0) bad = 1;
  if (i == n - 1 && e != nnz) bad = 1;
  if (e < s || s < 0 || e > nnz) bad = 1;
  if (!bad) {
    const int base = i & ~63;
    int prev = -1;
    for (int p = s; p < e; ++p) {
      const int c = col[p];
      if (c < 0 || c >= n || c <= prev) { bad = 1; break; }
      prev = c;
      far = max(far, abs(c - base));
    }
  }
  if (bad) atomicOr(&flags[0], 1);
  if (!bad) {
    atomicMax(&flags[1], e - s);
    atomicMax(&flags[2], far);
  }
}

// col16[p] = col[p] - (row & ~63) for every entry (offsets checked to fit).
__global__ void k_col16(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                        int16_t* __restrict__ col16) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int base = i & ~63;
  for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) col16[p] = (int16_t)(col[p] - base);
}

// ------------------------------------------------------------- dispatch

// Row u of a lane group is written by lane u of the group, so U <= L.
// L == 64 selects the row-block scheme, U = rows per wave.
static bool valid_shape(int L, int U) {
  if (L == kRowBlockL) return U == 16 || U == 32 || U == 64;
  return (L == 4 || L == 8 || L == 16 || L == 32) && (U == 1 || U == 2 || U == 4 || U == 8) && U <= L;
}

template <class V, int MODE>
static hipError_t launch_spmv_t(const hk_csr_s* A, const SpmvPlan& p, const V* x, V* y, const V* b,
                                V alpha, V beta, int beta_zero, hipStream_t s) {
  if (!valid_shape(p.L, p.U)) return hipErrorInvalidValue;
  const int ntiles = spmv_tiles(A, p.L, p.U);
  const int grid = p.grid > 0 ? (p.grid < ntiles ? p.grid : ntiles) : ntiles;
  if (ntiles == 0) return hipSuccess;
  const int n = (int)A->n;
  const V* val = static_cast<const V*>(A->val);
#define HK_SPMV_CASE(LL, UU)                                                                   \
  if (p.L == LL && p.U == UU) {                                                                \
    hipLaunchKernelGGL((k_spmv<LL, UU, V, MODE>), dim3(grid), dim3(kBlock), 0, s, n, ntiles,   \
                       A->rowptr, A->col, val, x, y, b, alpha, beta, beta_zero);               \
    return hipGetLastError();                                                                  \
  }
  HK_SPMV_CASE(4, 1) HK_SPMV_CASE(4, 2) HK_SPMV_CASE(4, 4)
  HK_SPMV_CASE(8, 1) HK_SPMV_CASE(8, 2) HK_SPMV_CASE(8, 4) HK_SPMV_CASE(8, 8)
  HK_SPMV_CASE(16, 1) HK_SPMV_CASE(16, 2) HK_SPMV_CASE(16, 4) HK_SPMV_CASE(16, 8)
  HK_SPMV_CASE(32, 1) HK_SPMV_CASE(32, 2) HK_SPMV_CASE(32, 4) HK_SPMV_CASE(32, 8)
#undef HK_SPMV_CASE
#define HK_RB_CASE(RR)                                                                          \
  if (p.L == kRowBlockL && p.U == RR) {                                                         \
    if (A->col16)                                                                               \
      hipLaunchKernelGGL((k_spmv_rb<RR, V, MODE, short>), dim3(grid), dim3(kRbThreads), 0, s, n, \
                         ntiles, A->rowptr, (const short*)A->col16, val, x, y, b, alpha, beta,   \
                         beta_zero);                                                            \
    else                                                                                        \
      hipLaunchKernelGGL((k_spmv_rb<RR, V, MODE, int>), dim3(grid), dim3(kRbThreads), 0, s, n,   \
                         ntiles, A->rowptr, A->col, val, x, y, b, alpha, beta, beta_zero);      \
    return hipGetLastError();                                                                   \
  }
  HK_RB_CASE(16) HK_RB_CASE(32) HK_RB_CASE(64)
#undef HK_RB_CASE
  return hipErrorInvalidValue;
}

int spmv_tiles(const hk_csr_s* A, int L, int U) {
  const long long rt = L == kRowBlockL ? (long long)kRbWaves * U : (long long)(kBlock / L) * U;
  return (int)((A->n + rt - 1) / rt);
}

int default_grid(int ntiles) { return ntiles; }



// Shape of an untuned handle: row blocks of the most rows whose mean entry
// count fits one pass of the wave (512 complex128 or 1024 complex64
// entries), which every FE matrix measured here preferred; 32-lane groups
// when even 16 rows overflow a pass.
static SpmvPlan heuristic_plan(const hk_csr_s* A) {
  SpmvPlan p;
  const double mean = A->n > 0 ? (double)A->nnz / (double)A->n : 0.0;
  const double pass = A->dtype == HK_C128 ? RbCh<64, double2>::v * kWave : RbCh<64, float2>::v * kWave;
  if (16 * mean > pass) {
    p.L = 32;
    p.U = 2;
  } else {
    p.L = kRowBlockL;
    p.U = 64 * mean <= pass ? 64 : 32 * mean <= pass ? 32 : 16;
  }
  p.grid = 0;
  p.tuned = 0;
  return p;
}

// Time every launch shape on this matrix (hipEvents on the caller's
// stream), keep the fastest.  Results are cached per (n, nnz, longest row,
// dtype, column stream) for the life of the process.
int spmv_autotune(hk_csr_s* A, hipStream_t s) {
  static std::mutex mu;
  static std::map<std::tuple<int64_t, int64_t, int, int, int, bool>, SpmvPlan> cache;
  int dev = 0;
  HK_HIP(hipGetDevice(&dev));
  auto key = std::make_tuple(A->n, A->nnz, A->max_row, A->dtype, dev, A->col16 != nullptr);
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) { A->plan = it->second; return HK_OK; }
  }
  const size_t vb = (A->dtype == HK_C128 ? 16 : 8) * (size_t)A->n;
  void *x = nullptr, *y = nullptr;
  if (hipMalloc(&x, vb) != hipSuccess) HK_FAIL(HK_ENOMEM, "autotune: hipMalloc failed");
  if (hipMalloc(&y, vb) != hipSuccess) { (void)hipFree(x); HK_FAIL(HK_ENOMEM, "autotune: hipMalloc failed"); }
  HK_HIP(hipMemsetAsync(x, 0, vb, s));
  hipEvent_t e0, e1;
  HK_HIP(hipEventCreate(&e0));
  HK_HIP(hipEventCreate(&e1));
  SpmvPlan best = heuristic_plan(A);
  float best_ms = 1e30f;
  const int Ls[] = {4, 8, 16, 32, kRowBlockL};
  const int Us[] = {1, 2, 4, 8, 16, 32, 64};
  const int grids[] = {0, 2048};
  int rc = HK_OK;
  for (int L : Ls) {
    if (L > 2 * A->max_row + 4 && L != 4 && L != kRowBlockL) continue;
    for (int U : Us) {
      if (!valid_shape(L, U)) continue;
      for (int gsel : grids) {
        SpmvPlan p;
        p.L = L; p.U = U; p.grid = gsel; p.tuned = 1;
        hipError_t err = hipSuccess;
        const int reps = 6;
        for (int it = 0; it < reps + 2 && err == hipSuccess; ++it) {
          if (it == 2) err = hipEventRecord(e0, s);
          if (err != hipSuccess) break;
          if (A->dtype == HK_C128)
            err = launch_spmv_t<double2, 0>(A, p, (const double2*)x, (double2*)y, nullptr,
                                            make_double2(1, 0), make_double2(0, 0), 1, s);
          else
            err = launch_spmv_t<float2, 0>(A, p, (const float2*)x, (float2*)y, nullptr,
                                           make_float2(1, 0), make_float2(0, 0), 1, s);
        }
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err != hipSuccess) {
          set_error_text("autotune: %s", hipGetErrorString(err));
          rc = HK_EHIP;
          break;
        }
        if (ms < best_ms) { best_ms = ms; best = p; }
      }
      if (rc != HK_OK) break;
    }
    if (rc != HK_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(x);
  (void)hipFree(y);
  if (rc != HK_OK) return rc;
  A->plan = best;
  std::lock_guard<std::mutex> lock(mu);
  cache[key] = best;
  return HK_OK;
}

int spmv_dispatch(const hk_csr_s* A, const void* x, void* y, const void* b, const void* alpha,
                  const void* beta, int mode, hipStream_t s) {
  hipError_t err;
  if (A->dtype == HK_C128) {
    double2 a = make_double2(1, 0), bt = make_double2(0, 0);
    int bz = 1;
    if (alpha) a = make_double2(((const double*)alpha)[0], ((const double*)alpha)[1]);
    if (beta) {
      bt = make_double2(((const double*)beta)[0], ((const double*)beta)[1]);
      bz = (bt.x == 0.0 && bt.y == 0.0);
    }
    err = mode == 1 ? launch_spmv_t<double2, 1>(A, A->plan, (const double2*)x, (double2*)y,
                                                (const double2*)b, a, bt, 1, s)
                    : launch_spmv_t<double2, 0>(A, A->plan, (const double2*)x, (double2*)y,
                                                nullptr, a, bt, bz, s);
  } else {
    float2 a = make_float2(1, 0), bt = make_float2(0, 0);
    int bz = 1;
    if (alpha) a = make_float2(((const float*)alpha)[0], ((const float*)alpha)[1]);
    if (beta) {
      bt = make_float2(((const float*)beta)[0], ((const float*)beta)[1]);
      bz = (bt.x == 0.0f && bt.y == 0.0f);
    }
    err = mode == 1 ? launch_spmv_t<float2, 1>(A, A->plan, (const float2*)x, (float2*)y,
                                               (const float2*)b, a, bt, 1, s)
                    : launch_spmv_t<float2, 0>(A, A->plan, (const float2*)x, (float2*)y, nullptr,
                                               a, bt, bz, s);
  }
  if (err != hipSuccess) HK_FAIL(HK_EHIP, "spmv launch: %s", hipGetErrorString(err));
  return HK_OK;
}

}  // namespace hk

using namespace hk;

extern "C" int hk_csr_create(hk_csr* out, int64_t n, int64_t nnz, const int32_t* d_rowptr,
                             const int32_t* d_col, const void* d_val, int dtype, int flags,
                             void* stream) {
  if (!out) HK_FAIL(HK_EINVAL, "hk_csr_create: out is NULL");
  *out = nullptr;
  if (n <= 0 || nnz < 0) HK_FAIL(HK_EINVAL, "hk_csr_create: n=%lld nnz=%lld", (long long)n, (long long)nnz);
  if (n >= (1ll << 31) - 1 || nnz >= (1ll << 31) - 1)
    HK_FAIL(HK_EINVAL, "hk_csr_create: n and nnz must fit int32 indices");
  if (!d_rowptr || (nnz > 0 && (!d_col || !d_val)))
    HK_FAIL(HK_EINVAL, "hk_csr_create: null device pointer");
  if (dtype != HK_C128 && dtype != HK_C64) HK_FAIL(HK_EINVAL, "hk_csr_create: bad dtype %d", dtype);
  hipStream_t s = as_stream(stream);
  int device = 0;
  HK_HIP(hipGetDevice(&device));
  hk_csr_s* A = new hk_csr_s();
  A->n = n; A->nnz = nnz; A->rowptr = d_rowptr; A->col = d_col; A->val = d_val; A->dtype = dtype;
  A->device = device;
  int* flags_d = nullptr;
  if (hipMalloc(&flags_d, 3 * sizeof(int)) != hipSuccess) {
    delete A;
    HK_FAIL(HK_ENOMEM, "hk_csr_create: hipMalloc failed");
  }
  int h[3] = {0, 0, 0};
  hipError_t err = hipMemsetAsync(flags_d, 0, 3 * sizeof(int), s);
  if (err == hipSuccess) {
    hipLaunchKernelGGL(k_csr_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (int)n,
                       (int)nnz, d_rowptr, d_col, flags_d);
    err = hipGetLastError();
  }
  if (err == hipSuccess) err = hipMemcpyAsync(h, flags_d, sizeof(h), hipMemcpyDeviceToHost, s);
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  (void)hipFree(flags_d);
  if (err != hipSuccess) {
    delete A;
    HK_FAIL(HK_EHIP, "hk_csr_create: %s", hipGetErrorString(err));
  }
  if (h[0]) {
    delete A;
    HK_FAIL(HK_EINVAL, "hk_csr_create: malformed CSR (rowptr/col out of range or unsorted)");
  }
  A->max_row = h[1];
  if (!(flags & HK_INT32_COLS) && nnz > 0 && h[2] <= 32767) {
    if (hipMalloc(&A->col16, 2 * ((size_t)nnz + 1)) != hipSuccess) {
      delete A;
      HK_FAIL(HK_ENOMEM, "hk_csr_create: hipMalloc failed");
    }
    err = hipMemsetAsync(A->col16 + nnz, 0, 2, s);
    if (err == hipSuccess) {
      hipLaunchKernelGGL(k_col16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (int)n, d_rowptr,
                         d_col, A->col16);
      err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (err != hipSuccess) {
      (void)hipFree(A->col16);
      delete A;
      HK_FAIL(HK_EHIP, "hk_csr_create: %s", hipGetErrorString(err));
    }
  }
  A->plan = heuristic_plan(A);
  if (flags & HK_AUTOTUNE) {
    int rc = spmv_autotune(A, s);
    if (rc != HK_OK) {
      (void)hk_csr_destroy(A);
      return rc;
    }
  }
  *out = A;
  return HK_OK;
}

extern "C" int hk_csr_destroy(hk_csr A) {
  if (!A) return HK_OK;
  int rc = HK_OK;
  if (A->ws || A->ws32 || A->val32 || A->col16) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(A->device);
    if (hipDeviceSynchronize() != hipSuccess) rc = HK_EHIP;
    if (A->ws) (void)hipFree(A->ws);
    if (A->ws32) (void)hipFree(A->ws32);
    if (A->val32) (void)hipFree(A->val32);
    if (A->col16) (void)hipFree(A->col16);
    (void)hipSetDevice(cur);
  }
  if (A->pinned) (void)hipHostFree(A->pinned);
  delete A;
  if (rc != HK_OK) HK_FAIL(rc, "hk_csr_destroy: device synchronisation failed");
  return HK_OK;
}

extern "C" int hk_csr_plan(hk_csr A, int32_t* L, int32_t* U, int32_t* grid, int32_t* tuned) {
  if (!A) HK_FAIL(HK_EINVAL, "hk_csr_plan: NULL handle");
  if (L) *L = A->plan.L;
  if (U) *U = A->plan.U;
  if (grid) *grid = A->plan.grid;
  if (tuned) *tuned = A->plan.tuned;
  return HK_OK;
}

extern "C" int hk_csr_info(hk_csr A, int64_t* n, int64_t* nnz, int32_t* max_row, int32_t* col_bytes) {
  if (!A) HK_FAIL(HK_EINVAL, "hk_csr_info: NULL handle");
  if (n) *n = A->n;
  if (nnz) *nnz = A->nnz;
  if (max_row) *max_row = A->max_row;
  if (col_bytes) *col_bytes = A->col16 ? 2 : 4;
  return HK_OK;
}

extern "C" int hk_csr_set_plan(hk_csr A, int32_t L, int32_t U, int32_t grid) {
  if (!A) HK_FAIL(HK_EINVAL, "hk_csr_set_plan: NULL handle");
  if (!valid_shape(L, U) || grid < 0) HK_FAIL(HK_EINVAL, "hk_csr_set_plan: bad shape L=%d U=%d grid=%d", L, U, grid);
  A->plan.L = L; A->plan.U = U; A->plan.grid = grid; A->plan.tuned = 0;
  A->dot_plan[0] = A->dot_plan[1] = SpmvPlan{};  // the solvers' products follow the new shape
  return HK_OK;
}

extern "C" int hk_csr_set_solver_plan(hk_csr A, int32_t rows_per_wave, int32_t waves, int32_t grid,
                                      int32_t paired) {
  if (!A) HK_FAIL(HK_EINVAL, "hk_csr_set_solver_plan: NULL handle");
  if (!(rows_per_wave == 16 || rows_per_wave == 32 || rows_per_wave == 64) ||
      !(waves == 2 || waves == 4 || waves == 8) || grid < 0 || (paired != 0 && paired != 1))
    HK_FAIL(HK_EINVAL, "hk_csr_set_solver_plan: bad shape rows_per_wave=%d waves=%d grid=%d paired=%d",
            rows_per_wave, waves, grid, paired);
  if (paired && !A->col16)
    HK_FAIL(HK_EINVAL, "hk_csr_set_solver_plan: the paired layout needs the 16-bit column stream");
  SpmvPlan p;
  p.L = kRowBlockL; p.U = rows_per_wave; p.nw = waves; p.grid = grid; p.pairs = paired; p.tuned = 2;
  A->dot_plan[0] = A->dot_plan[1] = p;
  return HK_OK;
}

extern "C" int hk_spmv(hk_csr A, const void* alpha, const void* d_x, const void* beta, void* d_y,
                       void* stream) {
  if (!A || !alpha || !d_x || !d_y) HK_FAIL(HK_EINVAL, "hk_spmv: null argument");
  if (d_x == d_y) HK_FAIL(HK_EINVAL, "hk_spmv: x and y must not overlap");
  return spmv_dispatch(A, d_x, d_y, nullptr, alpha, beta, 0, as_stream(stream));
}

extern "C" int hk_residual(hk_csr A, const void* d_b, const void* d_x, void* d_r, void* stream) {
  if (!A || !d_b || !d_x || !d_r) HK_FAIL(HK_EINVAL, "hk_residual: null argument");
  if (d_x == d_r) HK_FAIL(HK_EINVAL, "hk_residual: x and r must not overlap");
  return spmv_dispatch(A, d_x, d_r, d_b, nullptr, nullptr, 1, as_stream(stream));
}
