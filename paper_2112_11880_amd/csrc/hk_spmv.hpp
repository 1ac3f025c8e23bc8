// hk_spmv.hpp -- CSR row kernels for gfx950 (complex128 / complex64).
//
// The paper calls the CSR sparse matrix-vector product the most time
// consuming operation of a Krylov iteration and organises threads on the
// grid per matrix (Section 3, Table 8).  Here a row is owned by a group of
// L lanes of a 64-wide wave (L in {4, 8, 16, 32}); each lane streams
// (col, val) pairs of its row -- one 16-byte value load per lane, so a
// 16-lane group reads a row's values as one contiguous run -- gathers x, and
// the group reduces with cross-lane shuffles.  A group handles U consecutive
// rows with all loads issued before the multiply-adds, to keep enough bytes
// in flight per wave.  Matrix streams use non-temporal loads so they do not
// evict the x window from L2.  A workgroup of 256 threads covers
// (256/L)*U consecutive rows ("tile"); a launch of G workgroups walks the
// tiles with a grid stride, in launch order.
// The row-block scheme (csr_block_rows) instead gives a whole wave a block
// of 16-64 rows and streams the block's entries with all lanes.
#pragma once

#include "hk_common.hpp"

namespace hk {


// Column stream of the row-block products.  A matrix whose every entry lies
// within 32767 columns of its row's 64-aligned base (row & ~63) -- a banded
// FE matrix, for one -- is streamed as 16-bit offsets from that base, 2 bytes
// per entry instead of 4; otherwise as the int32 indices themselves.  Every
// row of a row block (16, 32 or 64 rows starting at a multiple of the block
// size) has the same base, so a lane decodes any entry of its block without
// knowing the entry's row.
__device__ __forceinline__ int col_at(const int* col, int p, int) { return ldnt(col + p); }
__device__ __forceinline__ int col_at(const short* col, int p, int base) { return base + ldnt(col + p); }

// Row sums of rows r0 .. r0+U-1 (rows >= n give 0), U <= L.  Every lane of
// the L-lane group returns the full sums; callers write row u from lane u.  Within a row, lane j accumulates
// entries j, j+L, j+2L, ...; the group total is a fixed butterfly.
// All loads are issued unconditionally from in-bounds indices (a lane past
// the end of its row re-reads the row's last entry and contributes zero),
// so the compiler keeps the U rows' loads in flight together instead of
// branching around each one.
template <int L, int U, class V>
__device__ __forceinline__ void csr_rows(int r0, int n, const int* __restrict__ rowptr,
                                         const int* __restrict__ col, const V* __restrict__ val,
                                         const V* __restrict__ x, V (&acc)[U]) {
  const int lane = threadIdx.x & (L - 1);
  int s[U], e[U];
  int len = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int r = r0 + u;
    const int rc = r < n ? r : n - 1;
    const int a = rowptr[rc], b = rowptr[rc + 1];
    s[u] = r < n ? a : 0;
    e[u] = r < n ? b : 0;
    len = max(len, e[u] - s[u]);
    acc[u] = czero<V>();
  }
  for (int k = 0; k < len; k += L) {
    int c[U];
    V a[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = s[u] + k + lane;
      ok[u] = p < e[u];
      // len > 0 here, so the matrix has entries and index 0 is valid
      const int pc = ok[u] ? p : (e[u] > 0 ? e[u] - 1 : 0);
      c[u] = ldnt(col + pc);
      a[u] = ldnt(val + pc);
    }
    V xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const V av = ok[u] ? a[u] : czero<V>();
      acc[u] = cfma(av, xv[u], acc[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    acc[u].x = group_sum<L>(acc[u].x);
    acc[u].y = group_sum<L>(acc[u].y);
  }
}

// Row sums of a row block from the products parked in LDS.  The 64 lanes
// are dealt S = 64/R per row: lane l sums the entries e = q, q + S, q + 2S,
// ... (q = l % S) of row r0 + l/S that this pass holds, so a row's chain of
// LDS reads is 1/S of its length.  rs and re are the row's entry range (of
// row r0 + l/S in lane l), buf holds entries [c0, cend).
template <int R, class V>
__device__ __forceinline__ void block_row_sums(V& acc, const V* buf, int rs, int re, int c0, int cend) {
  constexpr int S = kWave / R;
  const int q = S > 1 ? (int)(threadIdx.x & (S - 1)) : 0;
  const int lo = (rs > c0 ? rs : c0) + q, hi = re < cend ? re : cend;
  for (int e = lo; e < hi; e += S) acc = cadd(acc, buf[e - c0]);
}

// Lane l < R: the sum of row r0 + l, from the S lanes that summed its parts
// (block_row_sums); other lanes: unspecified.
template <int R, class V>
__device__ __forceinline__ V block_row_total(V acc) {
  constexpr int S = kWave / R;
  if constexpr (S == 1) {
    return acc;
  } else {
#pragma unroll
    for (int m = S / 2; m >= 1; m >>= 1) {
      acc.x += __shfl_xor(acc.x, m, kWave);
      acc.y += __shfl_xor(acc.y, m, kWave);
    }
    const int src = ((int)(threadIdx.x & (kWave - 1)) * S) & (kWave - 1);
    return cmake<V>(__shfl(acc.x, src, kWave), __shfl(acc.y, src, kWave));
  }
}

// Row-block CSR: one wave per R consecutive rows r0 .. r0+R-1 (R in
// {16, 32, 64}, r0 a multiple of R); col is either column stream (col_at).
// The wave streams the rows' entries with all 64 lanes -- entry e of a pass
// goes to lane e % 64, CH entries per lane per pass, every column and value
// load issued before any gather -- parks the products in its LDS slice
// buf[CH*64], then the 64/R lanes of each row sum interleaved parts of its
// products and combine them by a butterfly (block_row_sums,
// block_row_total).  On the 86^3 Q1 system (27 entries per row, 16-row
// blocks) this cut the product from 68.3 to 65.6 us against one lane
// summing each row in entry order.  Rows of any length are handled by
// passes over the block's entry range, the first starting at the 128-byte
// line of values that holds the block's first entry (the pass count is
// uniform across the wave).
// Returns the sum of row r0 + lane for lanes < R with r0 + lane < n, zero
// otherwise.  All 64 lanes must call it.
template <int R, int CH, class V, class CI>
__device__ __forceinline__ V csr_block_rows(int r0, int n, const int* __restrict__ rowptr,
                                            const CI* __restrict__ col, const V* __restrict__ val,
                                            const V* __restrict__ x, V* buf) {
  static_assert(R == 16 || R == 32 || R == 64, "rows per wave");
  const int l = threadIdx.x & (kWave - 1);
  const int base = r0 & ~63;
  // lane l <= R holds rowptr[r0 + l] (clamped to n): lane R the block's end
  const int li = l < R ? l : R;
  const int rs = rowptr[r0 + li < n ? r0 + li : n];
  int rend;
  if constexpr (R == kWave) rend = rowptr[r0 + kWave < n ? r0 + kWave : n];
  else rend = __shfl(rs, R, kWave);
  const int nxt = __shfl(rs, (l + 1) & (kWave - 1), kWave);
  const int re = l < kWave - 1 ? nxt : rend;
  // passes start at a 128-byte line of values (up to AL - 1 entries before
  // the block's first, loaded and never summed), so each 64-entry value load
  // covers whole lines; from the block's first entry a complex128 load
  // straddled 9 lines, and under non-temporal streaming a line two loads
  // share can be fetched twice
  constexpr int AL = 128 / (int)sizeof(V);
  const int s0 = __shfl(rs, 0, kWave) & ~(AL - 1);
  // entry range of the row this lane sums (row r0 + l / S)
  constexpr int S = kWave / R;
  const int rsum = S > 1 ? __shfl(rs, l / S, kWave) : (l < R ? rs : 0);
  const int resum = S > 1 ? __shfl(re, l / S, kWave) : (l < R ? re : 0);
  V acc = czero<V>();
  for (int c0 = s0; c0 < rend; c0 += CH * kWave) {
    const int cend = c0 + CH * kWave < rend ? c0 + CH * kWave : rend;
    int c[CH];
    V a[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int e = c0 + l + kWave * k;
      const int p = e < cend ? e : cend - 1;
      c[k] = col_at(col, p, base);
      // an entry before the block decodes a 16-bit offset with this block's base
      if constexpr (sizeof(CI) == 2) c[k] = min(max(c[k], 0), n - 1);
      a[k] = ldnt(val + p);
    }
    V xv[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) xv[k] = x[c[k]];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int e = c0 + l + kWave * k;
      if (e < cend) buf[e - c0] = cmul(a[k], xv[k]);
    }
    // LDS accesses of one wave complete in issue order; the barrier keeps the
    // compiler from moving the reads above the writes (and the next pass's
    // writes above these reads)
    __builtin_amdgcn_wave_barrier();
    block_row_sums<R>(acc, buf, rsum, resum, c0, cend);
    __builtin_amdgcn_wave_barrier();
  }
  return block_row_total<R>(acc);
}

// Paired layout of the same product for the 16-bit column stream: lane l
// takes entries c0 + 2l + 128k and the next one, with one 4-byte load for
// both column offsets and one load of both values (16 bytes for complex64),
// half the load instructions of the lane-per-entry layout.  Passes start
// at even entries, so the first pass may load the entry before the block
// and the last may load the entry after the end of the matrix: `val` and
// `col` must hold one padding entry after the last, and any entry outside
// the block decodes with the block's base, so every decoded column is
// clamped to [0, n).  Row sums are formed as in csr_block_rows.
template <class V> struct pair_of;
template <> struct pair_of<float2> { typedef float type __attribute__((ext_vector_type(4))); };

template <int R, int CH, class V>
__device__ __forceinline__ V csr_block_rows_pairs(int r0, int n, const int* __restrict__ rowptr,
                                                  const short* __restrict__ col, const V* __restrict__ val,
                                                  const V* __restrict__ x, V* buf) {
  static_assert(R == 16 || R == 32 || R == 64, "rows per wave");
  static_assert(CH % 2 == 0, "pairs");
  const int l = threadIdx.x & (kWave - 1);
  const int base = r0 & ~63;
  const int li = l < R ? l : R;
  const int rs = rowptr[r0 + li < n ? r0 + li : n];
  int rend;
  if constexpr (R == kWave) rend = rowptr[r0 + kWave < n ? r0 + kWave : n];
  else rend = __shfl(rs, R, kWave);
  const int nxt = __shfl(rs, (l + 1) & (kWave - 1), kWave);
  const int re = l < kWave - 1 ? nxt : rend;
  const int s0 = __shfl(rs, 0, kWave) & ~1;
  constexpr int S = kWave / R;
  const int rsum = S > 1 ? __shfl(rs, l / S, kWave) : (l < R ? rs : 0);
  const int resum = S > 1 ? __shfl(re, l / S, kWave) : (l < R ? re : 0);
  V acc = czero<V>();
  for (int c0 = s0; c0 < rend; c0 += CH * kWave) {
    const int cend = c0 + CH * kWave < rend ? c0 + CH * kWave : rend;
    int c[CH];
    V a[CH];
#pragma unroll
    for (int k = 0; k < CH / 2; ++k) {
      const int e = c0 + 2 * l + 2 * kWave * k;
      const int p = e < cend ? e : ((cend - 1) & ~1);  // even, in [c0, cend)
      const int pr = __builtin_nontemporal_load(reinterpret_cast<const int*>(col + p));
      c[2 * k] = min(max(base + (int)(short)(pr & 0xffff), 0), n - 1);
      c[2 * k + 1] = min(max(base + (pr >> 16), 0), n - 1);
      if constexpr (sizeof(V) == 8) {
        const auto v = __builtin_nontemporal_load(reinterpret_cast<const typename pair_of<V>::type*>(val + p));
        a[2 * k] = cmake<V>(v.x, v.y);
        a[2 * k + 1] = cmake<V>(v.z, v.w);
      } else {
        a[2 * k] = ldnt(val + p);
        a[2 * k + 1] = ldnt(val + p + 1);
      }
    }
    V xv[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) xv[k] = x[c[k]];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int e = c0 + 2 * l + 2 * kWave * (k / 2) + (k & 1);
      if (e < cend) buf[e - c0] = cmul(a[k], xv[k]);
    }
    __builtin_amdgcn_wave_barrier();
    block_row_sums<R>(acc, buf, rsum, resum, c0, cend);
    __builtin_amdgcn_wave_barrier();
  }
  return block_row_total<R>(acc);
}

// Row-block tile of virtual block b: within every run of 8*CHUNK
// consecutive tiles, XCD x (virtual blocks b with b % 8 == x) takes the x-th
// chunk of CHUNK tiles, so neighbouring tiles -- which gather the same x
// entries -- share an L2 while the chip still advances as one front.  A
// trailing partial run keeps the identity order.  For the fused solver
// products chunks of 8 measured ~2 us faster per product than chunks of 1,
// 32 or 128 on the 1.8M-row system; the plain product with 32 rows per wave
// and 16-bit columns measured 94.4 us with chunks of 512 tiles against 95.9
// us with 8 (and 95.1-96.4 us with 128, 256, 1024 or 2048), so it uses 512;
// with 64 rows per wave 512 was no better.  With 16 rows per wave (the Q1
// hexahedral product, 27-entry rows) chunks of 32 tiles measured 60.9-61.1
// us against 61.8 (8), 61.5 (16) and 61.2 (64), and 66.5 -> 68.7 us with
// 512; the other shapes keep 8.
constexpr int kTileChunk = 8;
constexpr int kSpmvTileChunk = 512;
constexpr int kSpmvTileChunk16 = 32;
template <int CHUNK = kTileChunk>
__device__ __forceinline__ int tile_of(int b, int ntiles) {
  constexpr int S = kXcds * CHUNK;
  const int q = b / S;
  if ((q + 1) * S > ntiles) return b;
  const int r = b - q * S;
  return q * S + (r % kXcds) * CHUNK + r / kXcds;
}

// Row-block launch shapes: plan L = kRowBlockL selects the scheme and plan U
// the rows per wave.  Workgroups are kRbWaves waves (128 threads).  Entries
// per lane per pass fill 8 KB of LDS per wave: 8 complex128 or 16 complex64
// products per lane, so each wave keeps the same bytes in flight in both
// precisions, and a 16-row block of 27-entry rows (Q1 hexahedra) takes one
// pass.  On the 1.8M-row system, 32 rows
// per wave in two-wave workgroups measured 106 us per complex128 product,
// against 109-110 us for four or eight waves and 110.6 us for 64 rows per
// wave with 4 waves; 16 complex128 entries per lane (16 KB of LDS per wave)
// measured 113 against 108 us at 64 rows per wave.
constexpr int kRowBlockL = 64;
constexpr int kRbWaves = 2;
constexpr int kRbThreads = kRbWaves * kWave;
template <int R, class V> struct RbCh {
  static constexpr int v = 8192 / (kWave * (int)sizeof(V));
};

// Tiles are dealt to workgroups in launch order with a grid stride: the
// calling workgroup takes tiles blockIdx.x, blockIdx.x + gridDim.x, ...
// Workgroups are placed on the 8 XCDs round-robin, so the resident
// workgroups always cover a narrow run of consecutive tiles and the whole
// chip advances through the matrix as one front.  Two alternatives measured
// slower on the 1.8M-row system: each XCD taking its own contiguous range
// (eight fronts, x windows private to each L2: 118-120 us against 108-113
// us per product) and each workgroup taking a contiguous range of tiles
// (a wide front: 132 against 116 us for the fused product).

// Shape of one SpMV variant.
struct SpmvShape {
  int L;        // lanes per row
  int U;        // rows per lane group
  int rows_per_tile() const { return (kBlock / L) * U; }
};

}  // namespace hk
