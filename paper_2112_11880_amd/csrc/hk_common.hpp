// hk_common.hpp -- device helpers shared by the HIP kernels of libhk (gfx950).
//
// Complex values are stored interleaved (re, im) as double2 / float2, the
// layout of the paper's complex<T> structure (Section 3: a pair of reals with
// the usual complex operations).  Reductions are deterministic: every sum is
// taken in an order fixed by the launch shape, never by atomics on values.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hk {

constexpr int kWave = 64;      // CDNA wavefront
constexpr int kBlock = 256;    // threads per workgroup (4 waves)
constexpr int kXcds = 8;       // MI355X: 8 XCDs, workgroup b runs on XCD b % 8

// ------------------------------------------------------------ complex ops
template <class R> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <class R> using cplx = typename cvec<R>::type;

template <class V> __device__ __forceinline__ V cmake(decltype(V::x) re, decltype(V::x) im) {
  V v; v.x = re; v.y = im; return v;
}
template <class V> __device__ __forceinline__ V czero() { return cmake<V>(0, 0); }
template <class V> __device__ __forceinline__ V cadd(V a, V b) { return cmake<V>(a.x + b.x, a.y + b.y); }
template <class V> __device__ __forceinline__ V csub(V a, V b) { return cmake<V>(a.x - b.x, a.y - b.y); }
template <class V> __device__ __forceinline__ V cmul(V a, V b) {
  return cmake<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc + a * b
template <class V> __device__ __forceinline__ V cfma(V a, V b, V acc) {
  acc.x = fma(a.x, b.x, acc.x); acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y); acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// acc + conj(a) * b
template <class V> __device__ __forceinline__ V cfmac(V a, V b, V acc) {
  acc.x = fma(a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
template <class V> __device__ __forceinline__ V cconj(V a) { return cmake<V>(a.x, -a.y); }
template <class V> __device__ __forceinline__ decltype(V::x) cabs2(V a) { return a.x * a.x + a.y * a.y; }
// a / b by Smith's method (R. L. Smith, CACM 5(8), 1962): divide through by
// the larger component of b so |b|^2 is never formed.  Forming |b|^2
// underflows in float once |b| < 1e-19, which the BiCGStab scalars reach.
template <class V> __device__ __forceinline__ V cdiv(V a, V b) {
  if (fabs(b.x) >= fabs(b.y)) {
    const auto r = b.y / b.x;
    const auto d = b.x + b.y * r;
    return cmake<V>((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  const auto r = b.x / b.y;
  const auto d = b.x * r + b.y;
  return cmake<V>((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
template <class V> __device__ __forceinline__ bool cfinite(V a) {
  return isfinite(a.x) && isfinite(a.y);
}

// ------------------------------------------------- non-temporal access
// Loads and stores that hint the caches not to keep the line: for streams
// read or written once (matrix entries, results, vectors larger than the
// last-level cache).
typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf2 __attribute__((ext_vector_type(2)));

template <class V> struct native;
template <> struct native<double2> { using type = nd2; };
template <> struct native<float2> { using type = nf2; };

template <class V> __device__ __forceinline__ V ldnt(const V* p) {
  using N = typename native<V>::type;
  N v = __builtin_nontemporal_load(reinterpret_cast<const N*>(p));
  return cmake<V>(v.x, v.y);
}
// Non-temporal store of one complex value (a result written once and not
// read again by the same kernel).
template <class V> __device__ __forceinline__ void stnt(V* p, V v) {
  using N = typename native<V>::type;
  N o;
  o.x = v.x;
  o.y = v.y;
  __builtin_nontemporal_store(o, reinterpret_cast<N*>(p));
}
__device__ __forceinline__ int ldnt(const int* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ int ldnt(const short* p) { return (int)__builtin_nontemporal_load(p); }

__device__ __forceinline__ double2 to_c128(float2 a) { return make_double2(a.x, a.y); }
__device__ __forceinline__ float2 to_c64(double2 a) { return make_float2((float)a.x, (float)a.y); }

// ------------------------------------------------------- launch geometry
// Logical block id such that each XCD gets one contiguous range of ids, so
// neighbouring rows (which share x gathers) meet in the same L2.
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
  int x = b % kXcds, i = b / kXcds;
  int q = nblocks / kXcds, r = nblocks % kXcds;
  return x * q + (x < r ? x : r) + i;
}

// ------------------------------------------------------------ reductions
template <class T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int m = kWave / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}
// Sum over aligned groups of L lanes; every lane of the group gets the sum.
template <int L, class T> __device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int m = L / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

// Block-wide sum of NV values per thread over a workgroup of NW waves
// (blockDim.x == NW * 64); the result is valid in thread 0.  Order:
// butterfly within each wave, then waves 0..NW-1.
template <int NV, class T, int NW = kBlock / kWave>
__device__ __forceinline__ void block_sum(T (&v)[NV], T* lds /*[NV*NW]*/) {
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[k * NW + w] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      T s = lds[k * NW];
      for (int j = 1; j < NW; ++j) s += lds[k * NW + j];
      v[k] = s;
    }
  }
}

// First stage of a two-stage reduction: thread 0 stores the block's NV
// totals at partials[k * gridDim.x + blockIdx.x].  No fence or atomic: the
// second stage runs in a later kernel on the same stream, and the kernel
// boundary makes these stores visible.  (A per-workgroup release fence here
// costs an L2 write-back on gfx950 and made reduction kernels 4-6x slower.)
template <int NV, class T>
__device__ __forceinline__ void store_block_partials(const T (&v)[NV], T* partials) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) partials[k * gridDim.x + blockIdx.x] = v[k];
  }
}

constexpr int kFinBlock = 1024;  // threads of a second-stage (finalize) kernel
// Finalize kernels over at most this many partials run with kFinBlockSmall
// threads: on a 4,913-row system a BiCGStab iteration (three finalize
// kernels) took 28.5 us instead of 31 us, while over the 7,094 partials of
// the 1.8M-row system the 1024-thread kernels stay faster.
constexpr int kFinBlockSmall = 256;
constexpr int kFinSmallNb = 1024;

// Second stage, run by one workgroup of BS threads: out[k] (valid in thread
// 0) = sum over nb partials, each thread summing a strided subset in index
// order, then a fixed tree over the waves.  A thread issues the loads of up
// to kFinUnroll of its partials (all NV components) before adding, so the
// load latency is paid once per kFinUnroll*BS partials rather than once per
// partial.
constexpr int kFinUnroll = 8;
template <int NV, class T, int BS = kFinBlock>
__device__ __forceinline__ void final_sum(const T* partials, int nb, T (&out)[NV], T* lds /*[NV*BS/64]*/) {
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  constexpr int W = BS / kWave;
  T s[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) s[k] = 0;
  for (int j0 = threadIdx.x; j0 < nb; j0 += kFinUnroll * BS) {
    T v[NV][kFinUnroll];
#pragma unroll
    for (int u = 0; u < kFinUnroll; ++u) {
      const int j = j0 + u * BS;
#pragma unroll
      for (int k = 0; k < NV; ++k) v[k][u] = j < nb ? partials[k * nb + j] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kFinUnroll; ++u)
#pragma unroll
      for (int k = 0; k < NV; ++k) s[k] += v[k][u];
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const T t = wave_sum(s[k]);
    if (lane == 0) lds[k * W + w] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      T s = lds[k * W];
      for (int j = 1; j < W; ++j) s += lds[k * W + j];
      out[k] = s;
    }
  }
}

}  // namespace hk
