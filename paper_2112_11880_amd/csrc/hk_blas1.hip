// hk_blas1.hip -- complex128 BLAS-1 of the paper's Section 3 on gfx950.
//
// Element-wise kernels (scal, axpy, element-wise product, assign) move one
// 16-byte complex per lane per vector.  Dots and the norm follow the
// paper's two-task scheme (element-wise product, then sum): each workgroup
// reduces a contiguous chunk (wave butterfly, then across its 4 waves) into
// one partial, and a one-workgroup kernel sums the partials in a fixed order
// and writes the result to device memory, so no host copy is needed and the
// result is bitwise reproducible.
#include <mutex>

#include "hk_common.hpp"
#include "hk_internal.hpp"

namespace hk {

constexpr int kRedMaxBlocks = 4096;
// Vectors of at least this many elements (64 MiB of complex128) are streamed
// with non-temporal loads and stores: they do not fit the last-level cache
// with their operands, and the hint measured 80.1 -> 74.0 us for zdotc and
// 114.9 -> 102.6 us for zaxpy at 14M elements.  Smaller vectors keep plain
// accesses (at 648,849 elements zaxpy took 8.1 us plain, 9.7 us
// non-temporal).
constexpr int64_t kNtMinElems = int64_t(1) << 22;
template <bool NT> __device__ __forceinline__ double2 ld(const double2* p) { return NT ? ldnt(p) : *p; }
template <bool NT> __device__ __forceinline__ void st(double2* p, double2 v) {
  if (NT) stnt(p, v);
  else *p = v;
}
// largest n of the allocation-free dot (the index arithmetic is int64; this
// bound keeps chunk * workgroups far from overflow)
constexpr int64_t kNoAllocMaxN = int64_t(1) << 40;

// workgroups of a reduction over n elements: at least 8 elements per thread,
// at most kRedMaxBlocks workgroups (each then walks a longer chunk)
static int reduce_blocks(int64_t n) {
  int64_t b = (n + kBlock * 8 - 1) / (kBlock * 8);
  if (b < 1) b = 1;
  return (int)(b > kRedMaxBlocks ? kRedMaxBlocks : b);
}

// First stage. KIND 0: x^H y, 1: x^T y, 2: ||x||^2.  Each workgroup reduces
// a contiguous chunk, 4 independent loads per vector in flight per thread.
// Chunks are whole multiples of 64 elements, so every wave's 1 KB load
// covers 8 whole 128-byte lines of an aligned vector (with chunks of n / nb
// elements the 14M-element dot read 1.039x its bytes, lines at chunk and
// load boundaries fetched twice; the trailing workgroups may get no
// elements).
template <int KIND, bool NT>
__global__ __launch_bounds__(kBlock) void k_reduce(int64_t n, const double2* __restrict__ x,
                                                   const double2* __restrict__ y, double* partials) {
  __shared__ double lds[2 * (kBlock / kWave)];
  const int nb = gridDim.x;
  const int lb = xcd_block(blockIdx.x, nb);
  const int64_t chunk = ((n + nb - 1) / nb + 63) & ~int64_t(63);
  const int64_t i0 = (int64_t)lb * chunk;
  const int64_t i1 = i0 + chunk < n ? i0 + chunk : n;
  double2 acc = make_double2(0.0, 0.0);
  int64_t i = i0 + threadIdx.x;
  for (; i + 3 * kBlock < i1; i += 4 * kBlock) {
    double2 a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = ld<NT>(x + i + u * kBlock);
      if (KIND != 2) b[u] = ld<NT>(y + i + u * kBlock);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (KIND == 0) acc = cfmac(a[u], b[u], acc);
      else if (KIND == 1) acc = cfma(a[u], b[u], acc);
      else acc.x = fma(a[u].x, a[u].x, fma(a[u].y, a[u].y, acc.x));
    }
  }
  for (; i < i1; i += kBlock) {
    const double2 a = ld<NT>(x + i);
    if (KIND == 0) acc = cfmac(a, ld<NT>(y + i), acc);
    else if (KIND == 1) acc = cfma(a, ld<NT>(y + i), acc);
    else acc.x = fma(a.x, a.x, fma(a.y, a.y, acc.x));
  }
  constexpr int NV = KIND == 2 ? 1 : 2;
  double v[NV];
  v[0] = acc.x;
  if (NV == 2) v[NV - 1] = acc.y;
  block_sum<NV>(v, lds);
  store_block_partials<NV>(v, partials);
}

// Second stage (one workgroup of BS threads): the result, written to device
// memory.
template <int KIND, int BS>
__global__ __launch_bounds__(BS) void k_reduce_fin(const double* partials, int nb, double* out) {
  constexpr int NV = KIND == 2 ? 1 : 2;
  __shared__ double lds[NV * (BS / kWave)];
  double tot[NV];
  final_sum<NV, double, BS>(partials, nb, tot, lds);
  if (threadIdx.x == 0) {
    if (KIND == 2) out[0] = sqrt(tot[0]);
    else { out[0] = tot[0]; out[NV - 1] = tot[NV - 1]; }
  }
}

template <bool NT>
__global__ void k_axpy(int64_t n, double2 a, const double2* __restrict__ x, double2* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) st<NT>(y + i, cfma(a, ld<NT>(x + i), ld<NT>(y + i)));
}
template <bool NT>
__global__ void k_scal(int64_t n, double2 a, double2* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) st<NT>(x + i, cmul(a, ld<NT>(x + i)));
}
template <bool NT>
__global__ void k_axmy(int64_t n, const double2* __restrict__ x, double2* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) st<NT>(y + i, cmul(ld<NT>(x + i), ld<NT>(y + i)));
}
template <bool NT>
__global__ void k_copy(int64_t n, const double2* __restrict__ x, double2* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) st<NT>(y + i, ld<NT>(x + i));
}
__global__ void k_conj(int64_t n, const double2* x, double2* y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = cconj(x[i]);
}

static dim3 ew_grid(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

// res[0 .. count) = 0 (the value of an empty sum; a kernel rather than a
// memset so the call stays capturable in a graph)
__global__ void k_zero_res(double* res, int count) {
  if ((int)threadIdx.x < count) res[threadIdx.x] = 0.0;
}

// The two stages of a reduction over n > 0 elements, partials in `partials`
// (room for 2 reduce_blocks(n) doubles).
template <int KIND>
static int launch_reduce(int64_t n, const void* x, const void* y, void* res, hipStream_t s, double* partials) {
  const int nb = reduce_blocks(n);
  if (n >= kNtMinElems)
    hipLaunchKernelGGL((k_reduce<KIND, true>), dim3(nb), dim3(kBlock), 0, s, n, (const double2*)x,
                       (const double2*)y, partials);
  else
    hipLaunchKernelGGL((k_reduce<KIND, false>), dim3(nb), dim3(kBlock), 0, s, n, (const double2*)x,
                       (const double2*)y, partials);
  HK_CHECK_LAUNCH();
  if (nb <= kFinSmallNb)
    hipLaunchKernelGGL((k_reduce_fin<KIND, kFinBlockSmall>), dim3(1), dim3(kFinBlockSmall), 0, s,
                       (const double*)partials, nb, (double*)res);
  else
    hipLaunchKernelGGL((k_reduce_fin<KIND, kFinBlock>), dim3(1), dim3(kFinBlock), 0, s,
                       (const double*)partials, nb, (double*)res);
  HK_CHECK_LAUNCH();
  return HK_OK;
}

template <int KIND>
static int reduce(int64_t n, const void* x, const void* y, void* res, void* stream, const char* who) {
  if (n < 0 || !res || (n > 0 && (!x || (KIND != 2 && !y))))
    HK_FAIL(HK_EINVAL, "%s: bad argument (n=%lld)", who, (long long)n);
  hipStream_t s = as_stream(stream);
  if (n == 0) {
    hipLaunchKernelGGL(k_zero_res, dim3(1), dim3(64), 0, s, (double*)res, KIND == 2 ? 1 : 2);
    HK_CHECK_LAUNCH();
    return HK_OK;
  }
  ReduceScratch* rs = nullptr;
  int rc = reduce_scratch(s, sizeof(double) * 2 * reduce_blocks(n), &rs);
  if (rc != HK_OK) return rc;
  return launch_reduce<KIND>(n, x, y, res, s, (double*)rs->partials);
}

// ------------------------------------------- allocation-free zdotc scratch
//
// The partials of hk_zdotc_noalloc live in this file-scope device array (one
// copy per GPU, held until the process ends): two doubles for each of at
// most kRedMaxBlocks workgroups, 64 KiB.  Every first-stage workgroup writes
// its partial before the finalize reads it, so nothing needs clearing
// between calls.  The array's name is only a host-side stand-in; kernels get
// its device address, looked up once per device.
constexpr int kNoAllocPartials = 2 * kRedMaxBlocks;
static __device__ __align__(256) double scratch[kNoAllocPartials];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on first use).
static int noalloc_scratch(double** out) {
  int dev = 0;
  HK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) HK_FAIL(HK_EINVAL, "hk_zdotc_noalloc: device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      HK_FAIL(HK_EHIP, "hk_zdotc_noalloc: hipGetSymbolAddress(scratch) on device %d: %s", dev,
              hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return HK_OK;
}

}  // namespace hk

using namespace hk;

extern "C" int hk_zdotc(int64_t n, const void* x, const void* y, void* res, void* stream) {
  return reduce<0>(n, x, y, res, stream, "hk_zdotc");
}
extern "C" int hk_zdotc_noalloc(int64_t n, const void* x, const void* y, void* res, void* stream) {
  if (n < 0 || !res || (n > 0 && (!x || !y)))
    HK_FAIL(HK_EINVAL, "hk_zdotc_noalloc: bad argument (n=%lld)", (long long)n);
  if (n > kNoAllocMaxN)
    HK_FAIL(HK_EINVAL, "hk_zdotc_noalloc: n=%lld above the limit %lld", (long long)n, (long long)kNoAllocMaxN);
  hipStream_t s = as_stream(stream);
  if (n == 0) {
    hipLaunchKernelGGL(k_zero_res, dim3(1), dim3(64), 0, s, (double*)res, 2);
    HK_CHECK_LAUNCH();
    return HK_OK;
  }
  if (2 * reduce_blocks(n) > kNoAllocPartials)
    HK_FAIL(HK_EINVAL, "hk_zdotc_noalloc: %d partials exceed the scratch of %d", 2 * reduce_blocks(n),
            kNoAllocPartials);
  double* partials = nullptr;
  const int rc = noalloc_scratch(&partials);
  if (rc != HK_OK) return rc;
  return launch_reduce<0>(n, x, y, res, s, partials);
}
extern "C" int hk_zdotu(int64_t n, const void* x, const void* y, void* res, void* stream) {
  return reduce<1>(n, x, y, res, stream, "hk_zdotu");
}
extern "C" int hk_dznrm2(int64_t n, const void* x, double* res, void* stream) {
  return reduce<2>(n, x, nullptr, res, stream, "hk_dznrm2");
}

extern "C" int hk_zaxpy(int64_t n, const double* alpha, const void* x, void* y, void* stream) {
  if (n < 0 || !alpha || (n > 0 && (!x || !y))) HK_FAIL(HK_EINVAL, "hk_zaxpy: bad argument");
  if (n == 0) return HK_OK;
  hipLaunchKernelGGL(n >= kNtMinElems ? k_axpy<true> : k_axpy<false>, ew_grid(n), dim3(kBlock), 0,
                     as_stream(stream), n, make_double2(alpha[0], alpha[1]), (const double2*)x, (double2*)y);
  HK_CHECK_LAUNCH();
  return HK_OK;
}
extern "C" int hk_zscal(int64_t n, const double* alpha, void* x, void* stream) {
  if (n < 0 || !alpha || (n > 0 && !x)) HK_FAIL(HK_EINVAL, "hk_zscal: bad argument");
  if (n == 0) return HK_OK;
  hipLaunchKernelGGL(n >= kNtMinElems ? k_scal<true> : k_scal<false>, ew_grid(n), dim3(kBlock), 0,
                     as_stream(stream), n, make_double2(alpha[0], alpha[1]), (double2*)x);
  HK_CHECK_LAUNCH();
  return HK_OK;
}
extern "C" int hk_zaxmy(int64_t n, const void* x, void* y, void* stream) {
  if (n < 0 || (n > 0 && (!x || !y))) HK_FAIL(HK_EINVAL, "hk_zaxmy: bad argument");
  if (n == 0) return HK_OK;
  hipLaunchKernelGGL(n >= kNtMinElems ? k_axmy<true> : k_axmy<false>, ew_grid(n), dim3(kBlock), 0,
                     as_stream(stream), n, (const double2*)x, (double2*)y);
  HK_CHECK_LAUNCH();
  return HK_OK;
}
extern "C" int hk_zcopy(int64_t n, const void* x, void* y, void* stream) {
  if (n < 0 || (n > 0 && (!x || !y))) HK_FAIL(HK_EINVAL, "hk_zcopy: bad argument");
  if (n == 0) return HK_OK;
  hipLaunchKernelGGL(n >= kNtMinElems ? k_copy<true> : k_copy<false>, ew_grid(n), dim3(kBlock), 0,
                     as_stream(stream), n, (const double2*)x, (double2*)y);
  HK_CHECK_LAUNCH();
  return HK_OK;
}
extern "C" int hk_zconj(int64_t n, const void* x, void* y, void* stream) {
  if (n < 0 || (n > 0 && (!x || !y))) HK_FAIL(HK_EINVAL, "hk_zconj: bad argument");
  if (n == 0) return HK_OK;
  hipLaunchKernelGGL(k_conj, ew_grid(n), dim3(kBlock), 0, as_stream(stream), n, (const double2*)x,
                     (double2*)y);
  HK_CHECK_LAUNCH();
  return HK_OK;
}
