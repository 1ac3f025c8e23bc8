// hk_batched.hip -- batched Jacobi-BiCGStab in one persistent launch (gfx950).
//
// Two batch shapes, both solved by a single cooperative kernel that runs
// every iteration of every system, with grid barriers between phases:
//
// (a) Frequency sweep: nsys <= 64 systems A_j = K - kappa_j M sharing one
//     sparsity pattern, with K and M real.  Vectors are interleaved
//     system-fastest (x[node][64]); lane j of every wave works on system j,
//     so a gather of x[col] is one contiguous 1 KB access, the matrix row
//     (col, K, M) is read once per wave for all systems, and each system's
//     reduction terms stay in their own lane.  A_j is formed on the fly.
// (b) Uneven systems: a block-diagonal CSR (systems concatenated, global
//     indices) with per-system row ranges.  Rows are grouped in tiles that
//     never straddle systems; phases walk the list of tiles of the systems
//     still iterating, which is compacted whenever a system finishes.
//
// Jacobi is applied on the right through hatted vectors: phat = D^-1 p and
// shat = D^-1 s are stored, s = D shat and D^-1 v are formed on the fly, and
// x += alpha phat + omega shat.  Per-system scalars, statuses and iteration
// counts live in device memory; at each grid barrier workgroup 0 finishes
// the reductions (fixed order) and updates them.
#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

#include "hk_grid.hpp"
#include "hk_internal.hpp"
#include "hk_spmv.hpp"

namespace hk {

constexpr int kSys = 64;          // systems per launch (lanes of a wave)
constexpr int kPB = 1024;         // threads per workgroup of the persistent kernels
constexpr int kPW = kPB / kWave;  // waves per workgroup

enum : int { B_RUN = 100, B_HALF = 101, B_TAUBD = 102 };

struct BatchState {
  double2 rho[kSys], rho_old[kSys], alpha[kSys], omega[kSys], beta[kSys];
  double rr[kSys], ss[kSys], bb[kSys], theta2[kSys], rr_true[kSys];
  int status[kSys], bd[kSys];
  long long iters[kSys];
  long long iter, maxit;
  int running;
  int changed;       // a system stopped in the last iteration (tile list to rebuild)
  int ntiles_active;
  // sweep: the rows per wave step of the launch that continues the solve
  // (k_sweep_tail<MAP, handoff>: 2 from 32 running systems, 4 from 16), 0
  // while none; the next launch starts at barrier epoch epoch0
  int handoff;
  unsigned epoch0;
};

// ------------------------------------------------------------ shared helpers

// v (this lane's NV partial sums, lane = system) summed over the waves of
// the workgroup and stored at partials[(k*G + block)*64 + lane].
template <int NV>
__device__ __forceinline__ void store_partials64(const double (&v)[NV], double* partials, double* lds) {
  const int w = threadIdx.x >> 6, j = threadIdx.x & 63, G = gridDim.x;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) lds[(k * kPW + w) * kSys + j] = v[k];
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0;
      for (int u = 0; u < kPW; ++u) s += lds[(k * kPW + u) * kSys + j];
      partials[((size_t)k * G + blockIdx.x) * kSys + j] = s;
    }
  }
}

// Group leader b's part of barrier_reduce: the NV sums of its members
// m_i = b + kXcds i (i < nm), thread row q adding members q, q + 16, ... in
// order, then the 16 rows in row order, into gpart[(k*kXcds + b)*64 + j].
// Out of line, so that its loops do not raise the register allocation of
// the persistent kernels that call the barrier at every phase.  All threads
// of the workgroup call it.
template <int NV>
__device__ __noinline__ void group_partials(const double* partials, int G, int b, double* lds, double* gpart) {
  const int j = threadIdx.x & 63, q = threadIdx.x >> 6;  // q < 16
  const int nm = (G - b + kXcds - 1) / kXcds;
  double t[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) t[k] = 0;
  for (int i0 = q; i0 < nm; i0 += 2 * kPW) {
    double v[NV][2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = i0 + u * kPW < nm ? i0 + u * kPW : i0;
#pragma unroll
      for (int k = 0; k < NV; ++k) v[k][u] = partials[((size_t)k * G + b + kXcds * i) * kSys + j];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
      if (i0 + u * kPW < nm) {
#pragma unroll
        for (int k = 0; k < NV; ++k) t[k] += v[k][u];
      }
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) lds[(k * kPW + q) * kSys + j] = t[k];
  __syncthreads();
  if (threadIdx.x < NV * kSys) {
    const int k = threadIdx.x / kSys, jj = threadIdx.x % kSys;
    double g = 0;
    for (int r = 0; r < kPW; ++r) g += lds[(k * kPW + r) * kSys + jj];
    gpart[(k * kXcds + b) * kSys + jj] = g;
  }
  __syncthreads();
}

// Grid barrier that also finishes an NV-sum reduction over the workgroups'
// partials (partials[(k*G + b)*64 + j], k < NV <= 3).  Reading all G x 64 x
// NV partials into workgroup 0 took 4.5-9.5 us per barrier (up to 393 KB
// through one CU, while the other workgroups waited); here the kXcds groups
// of workgroups b = g, g + kXcds, ... are first summed by workgroup g (group
// leader), each into bar->gpart[(k*kXcds + g)*64 + j] (in member order,
// split over 16 thread rows and then added in row order; group_partials),
// and workgroup 0 adds the kXcds group sums in group order and calls
// on_last(tot) in all its threads (tot[k] valid in thread j < 64 for system
// j).  The order is fixed, so the sums are bitwise reproducible.  Waits,
// fences and the abort path as in barrier_last; lds needs 3 x 16 x 64
// doubles.  Returns true if the kernel must stop.  All threads of every
// workgroup call it.
template <int NV, class F>
__device__ __forceinline__ bool barrier_reduce(GridBar* bar, unsigned& epoch, const double* partials, double* lds,
                                               F&& on_last) {
  static_assert(NV >= 1 && NV <= 3, "one to three sums");
  __shared__ int s_stop;
  const unsigned e = ++epoch;
  const int G = gridDim.x, b = blockIdx.x;
  const int j = threadIdx.x & 63;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this workgroup's writes before its flag
    st_relaxed_u32(&bar->arrive[b], e);
  }
  if (b < kXcds) {
    // leader of group b: its members m_i = b + kXcds i, i < nm
    const int nm = (G - b + kXcds - 1) / kXcds;
    bool ok = true;
    for (int i = threadIdx.x; i < nm; i += blockDim.x) ok = wait_epoch(&bar->arrive[b + kXcds * i], e, bar) && ok;
    if (!ok) atomicExch(&bar->abort, 1);
    __syncthreads();
    if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the members' partials
    __syncthreads();
    group_partials<NV>(partials, G, b, lds, bar->gpart);
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the group's sums before its flag
      st_relaxed_u32(&bar->garrive[b], e);
    }
  }
  if (b == 0) {
    bool ok = true;
    if (threadIdx.x < kXcds) ok = wait_epoch(&bar->garrive[threadIdx.x], e, bar);
    if (!ok) atomicExch(&bar->abort, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
      s_stop = ld_relaxed_i32(&bar->abort);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every group's sums
      if (bar->stamps && e < bar->nstamps) bar->stamps[e] = (double)wall_clock64();
    }
    __syncthreads();
    // the kXcds group sums: thread (k, j) adds them in group order, then
    // threads j < 64 take all NV through LDS
    if (threadIdx.x < NV * kSys) {
      const int k = threadIdx.x / kSys;
      double v[kXcds];
#pragma unroll
      for (int g = 0; g < kXcds; ++g) v[g] = bar->gpart[(k * kXcds + g) * kSys + j];
      double tk = 0;
#pragma unroll
      for (int g = 0; g < kXcds; ++g) tk += v[g];
      lds[threadIdx.x] = tk;
    }
    __syncthreads();
    double tot[NV];
    if (threadIdx.x < kSys) {
#pragma unroll
      for (int k = 0; k < NV; ++k) tot[k] = lds[k * kSys + j];
    }
    if (!s_stop) on_last(tot);
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

__device__ __forceinline__ double2 crecip(double2 d) { return cdiv(make_double2(1.0, 0.0), d); }

// Copies of a workgroup's LDS copy of the state to memory, by wave 0 (the
// wave whose thread 0 fences before a barrier's release): the fields the
// phases read, or all of it.  Called by every thread of the workgroup.
__device__ __forceinline__ void publish_phase_state(BatchState* g, const BatchState& l) {
  __syncthreads();
  const int j = threadIdx.x;
  if (j < kSys) {
    g->status[j] = l.status[j];
    g->alpha[j] = l.alpha[j];
    g->omega[j] = l.omega[j];
    g->beta[j] = l.beta[j];
    if (j == 0) {
      g->running = l.running;
      g->iter = l.iter;
      g->handoff = l.handoff;
    }
  }
}
__device__ __forceinline__ void publish_state(BatchState* g, const BatchState& l) {
  __syncthreads();
  if (threadIdx.x < kWave) {
    const unsigned* src = reinterpret_cast<const unsigned*>(&l);
    unsigned* dst = reinterpret_cast<unsigned*>(g);
    for (int i = threadIdx.x; i < (int)(sizeof(BatchState) / 4); i += kWave) dst[i] = src[i];
  }
}

// Scalar updates shared by both batch shapes (thread j = system j).
__device__ __forceinline__ void upd_sigma(BatchState* st, int j, double2 sigma) {
  if (st->status[j] != B_RUN) return;
  if (!cfinite(sigma)) {
    st->status[j] = HK_NONFINITE; st->iters[j] = st->iter - 1; st->changed = 1;
  } else if (sigma.x == 0 && sigma.y == 0) {
    st->status[j] = HK_BREAKDOWN; st->bd[j] = HK_BD_SIGMA; st->iters[j] = st->iter - 1; st->changed = 1;
  } else {
    st->alpha[j] = cdiv(st->rho[j], sigma);
  }
}
__device__ __forceinline__ void upd_s(BatchState* st, int j, double ss) {
  if (st->status[j] != B_RUN) return;
  st->ss[j] = ss;
  if (!isfinite(ss)) { st->status[j] = HK_NONFINITE; st->iters[j] = st->iter - 1; st->changed = 1; }
  else if (ss <= st->theta2[j]) st->status[j] = B_HALF;
}
__device__ __forceinline__ void upd_omega(BatchState* st, int j, double tau, double2 ts) {
  if (st->status[j] != B_RUN) return;
  if (!isfinite(tau) || !cfinite(ts)) { st->status[j] = HK_NONFINITE; st->iters[j] = st->iter - 1; st->changed = 1; }
  else if (tau == 0) st->status[j] = B_TAUBD;
  else st->omega[j] = make_double2(ts.x / tau, ts.y / tau);
}
// end of an iteration; returns 1 if system j is still running afterwards
__device__ __forceinline__ int upd_xr(BatchState* st, int j, double rr, double2 rho) {
  const int s = st->status[j];
  const long long it = st->iter;
  if (s == B_HALF) {
    st->status[j] = HK_OK; st->rr[j] = st->ss[j]; st->iters[j] = it; st->changed = 1; return 0;
  }
  if (s == B_TAUBD) {
    st->status[j] = HK_BREAKDOWN; st->bd[j] = HK_BD_TAU; st->rr[j] = st->ss[j]; st->iters[j] = it;
    st->changed = 1; return 0;
  }
  if (s != B_RUN) return 0;
  st->rr[j] = rr;
  st->rho_old[j] = st->rho[j];
  st->rho[j] = rho;
  st->iters[j] = it;
  const double2 om = st->omega[j];
  int next = B_RUN;
  if (!isfinite(rr) || !cfinite(rho)) next = HK_NONFINITE;
  else if (rr <= st->theta2[j]) next = HK_OK;
  else if (om.x == 0 && om.y == 0) { next = HK_BREAKDOWN; st->bd[j] = HK_BD_OMEGA; }
  else if (rho.x == 0 && rho.y == 0) { next = HK_BREAKDOWN; st->bd[j] = HK_BD_RHO; }
  else if (it >= st->maxit) next = HK_NOT_CONVERGED;
  if (next != B_RUN) { st->status[j] = next; st->changed = 1; return 0; }
  st->beta[j] = cmul(cdiv(rho, st->rho_old[j]), cdiv(st->alpha[j], om));
  return 1;
}
__device__ __forceinline__ void init_sys(BatchState* st, int j, double bb, double tol, long long maxit) {
  st->bb[j] = bb; st->rr[j] = bb; st->theta2[j] = tol * tol * bb;
  st->rho[j] = make_double2(bb, 0); st->rho_old[j] = make_double2(1, 0);
  st->alpha[j] = make_double2(1, 0); st->omega[j] = make_double2(1, 0);
  st->beta[j] = make_double2(0, 0); st->iters[j] = 0; st->bd[j] = HK_BD_NONE; st->rr_true[j] = 0;
  if (!isfinite(bb)) st->status[j] = HK_NONFINITE;
  else if (bb == 0 || bb <= st->theta2[j]) st->status[j] = HK_OK;
  else if (maxit <= 0) st->status[j] = HK_NOT_CONVERGED;
  else st->status[j] = B_RUN;
}

// =============================================================== (a) sweep

struct SweepArgs {
  int n, nsys;
  const int* rowptr;
  const int* col;
  const double* K;
  const double* M;
  const double* kd;   // diag(K)
  const double* md;   // diag(M)
  const double2* kap; // kappa_j (nsys entries)
  const double2* B;   // n x 64, interleaved
  double2* X;
  double2 *R, *RH, *PH, *V, *SH, *T;
  double* partials;
  BatchState* st;
  GridBar* bar;
  double tol;
  long long maxit;
  int tail;  // product form 3: hand the last <= 32 systems to k_sweep_tail
};

// The shared matrix (rowptr, col, K, M and the diagonals) is read-only
// during the kernel and every lane of a wave reads the same entry (lanes are
// systems), so it is read through the scalar unit: constant-address-space
// pointers indexed by wave-uniform values (readfirstlane) compile to scalar
// loads, which keep the matrix stream out of the vector registers and the
// vector memory pipeline.
template <class T> using cptr = const __attribute__((address_space(4))) T*;
template <class T> __device__ __forceinline__ cptr<T> as_const(const T* p) { return (cptr<T>)p; }
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ double2 sweep_diag(const SweepArgs& a, int i, double2 kap) {
  const int iu = uni(i);
  const double k = as_const(a.kd)[iu], m = as_const(a.md)[iu];
  return make_double2(k - kap.x * m, -kap.y * m);
}

// y[row][j] = sum_q (K_q - kap_j M_q) src[col_q][j] for this wave's rows;
// EPI 1: part += conj(RH) y ; EPI 2: part += |y|^2, conj(y) (d .* SH) ;
// EPI 3: y = B - A src, part += |y|^2 (true residual).
template <int EPI, int NV>
__device__ __forceinline__ void sweep_spmv(const SweepArgs& a, int r0, int r1, int rs, const double2* src,
                                           double2* dst, bool act, double2 kap, double (&part)[NV]) {
  const int j = threadIdx.x & 63;
  // lanes of finished systems issue no loads at all
  if (!act) return;
  const cptr<int> rowptr = as_const(a.rowptr), col = as_const(a.col);
  const cptr<double> Kc = as_const(a.K), Mc = as_const(a.M);
  // the next row's extent is loaded while this row's gathers are in flight
  int row = uni(r0);
  int s = row < r1 ? rowptr[row] : 0, e = row < r1 ? rowptr[row + 1] : 0;
  for (; row < r1; row += rs) {
    const int nrow = row + rs;
    const int ns = nrow < r1 ? rowptr[nrow] : 0, ne = nrow < r1 ? rowptr[nrow + 1] : 0;
    // the epilogue's operand is loaded before the gathers as well
    const size_t o = (size_t)row * kSys + j;
    const double2 pre = EPI == 1 ? a.RH[o] : EPI == 2 ? a.SH[o] : a.B[o];
    const double2 dg = EPI == 2 ? sweep_diag(a, row, kap) : make_double2(0, 0);
    double2 acc = make_double2(0, 0);
    // 8 entries at a time, all gathers in flight together; past the row's
    // end an entry re-reads the last column with a zero coefficient
    for (int q0 = s; q0 < e; q0 += 8) {
      int c[8];
      double kv[8], mv[8];
      double2 xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool in = q0 + u < e;
        const int q = in ? q0 + u : e - 1;
        c[u] = col[q];
        kv[u] = in ? Kc[q] : 0.0;
        mv[u] = in ? Mc[q] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) xv[u] = src[(size_t)c[u] * kSys + j];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = cfma(make_double2(kv[u] - kap.x * mv[u], -kap.y * mv[u]), xv[u], acc);
    }
    s = ns;
    e = ne;
    if (EPI == 3) {
      const double2 rt = csub(pre, acc);
      part[0] += cabs2(rt);
      continue;
    }
    stnt(dst + o, acc);
    if (EPI == 1) {
      const double2 h = pre;
      part[0] = fma(h.x, acc.x, fma(h.y, acc.y, part[0]));
      part[1] = fma(h.x, acc.y, fma(-h.y, acc.x, part[1]));
    } else if (EPI == 2) {
      const double2 sv = cmul(dg, pre);
      part[0] = fma(acc.x, acc.x, fma(acc.y, acc.y, part[0]));
      part[1] = fma(acc.x, sv.x, fma(acc.y, sv.y, part[1]));
      part[2] = fma(acc.x, sv.y, fma(-acc.y, sv.x, part[2]));
    }
  }
}

// Rows of the calling wave: r0, r0 + rs, ... < r1.  Three mappings, chosen
// per matrix by timing (hk_sweep_solve):
//  MAP 1: XCD x (the workgroups b with b % 8 == x) owns a contiguous eighth
//         of the rows and its waves take them round-robin, so each XCD
//         advances through its eighth as one front and the x[col] gathers of
//         neighbouring rows meet in its L2 (902 us per iteration on the 48^3
//         sweep with the per-row product);
//  MAP 2: every wave of the grid round-robin over all rows (906 us);
//  MAP 3: each XCD's eighth split into one contiguous range per wave (the
//         entry-stream product needs contiguous rows; 948 us per-row).
template <int MAP>
__device__ __forceinline__ void sweep_rows(int n, int G, int& r0, int& r1, int& rs) {
  const int w = threadIdx.x >> 6;
  if (MAP == 2) {
    r0 = blockIdx.x * kPW + w;
    r1 = n;
    rs = G * kPW;
    return;
  }
  const int x = blockIdx.x % kXcds, i = blockIdx.x / kXcds;
  const int nbx = (G - x + kXcds - 1) / kXcds;  // workgroups on XCD x (G >= kXcds)
  const int X0 = (int)(((long long)x * n) / kXcds), X1 = (int)(((long long)(x + 1) * n) / kXcds);
  if (MAP == 1) {
    r0 = X0 + i * kPW + w;
    r1 = X1;
    rs = nbx * kPW;
    return;
  }
  const int nw = nbx * kPW, wi = i * kPW + w;
  r0 = X0 + (int)(((long long)(X1 - X0) * wi) / nw);
  r1 = X0 + (int)(((long long)(X1 - X0) * (wi + 1)) / nw);
  rs = 1;
}

// ------------------------------------------------ claimed rows (vector phases)
//
// The element-wise phases (p, s and x/r updates) stream their rows with no
// reuse, and the memory system serves the 16 waves of a workgroup unevenly:
// with a fixed share of rows per wave, the first waves of a workgroup were
// done after ~40% of the phase and the last ones set the workgroup's time
// (e.g. 46 to 161 us for the x/r update).  So the waves claim the
// workgroup's rows in units of kUnitRows through an LDS counter, in the
// order row(q) = base + q % kPW + (q / kPW) step, q < nrows (sweep_wg_rows).
//
// A reduction over claimed rows stays bitwise reproducible: each unit's sum
// is formed in row order and parked in an LDS ring (kUnitRing units), and
// the units are added in unit order, a batch of kUnitBatch at a time, by the
// wave that completes the batch, once every earlier batch is added.  A unit
// waits for its ring slot only if the batch kUnitRing / kUnitBatch before it
// is not added yet.  Every wait ends: the batches before any waiting unit
// hold only units that are claimed already (claims go in order) and need
// no slot; the waits also carry the grid barrier's time limit.
constexpr int kUnitRows = 4;
constexpr int kUnitBatch = 16;
constexpr int kUnitRing = 64;
constexpr int kUnitNV = 3;  // at most this many sums per lane

struct WgRows {
  int base, step, nrows;
};

// The element-wise phases have no reuse to keep local; what pays is one
// front: workgroup b takes the groups of kPW rows b kPW + k G kPW (k >= 0), so
// the whole grid streams each vector as a single window of G kPW rows (on the
// 48^3 sweep 642 us per iteration, against 656 with the product phases' XCD
// eighths and 669 with one contiguous range per workgroup).
__device__ __forceinline__ WgRows sweep_wg_rows(int n, int G) {
  const int base = blockIdx.x * kPW, step = G * kPW;
  // full groups of kPW rows, then a partial one
  const int L = n - base;
  const int full = L >= kPW ? (L - kPW) / step + 1 : 0;
  const int rest = min(max(L - full * step, 0), kPW);
  return WgRows{base, step, full * kPW + rest};
}

struct UnitSync {
  int claim;             // 64 x the next unit to hand out
  int added;             // batches added to acc so far
  int count[kUnitRing / kUnitBatch];  // 64 x the units finished per batch in the ring
};

__device__ __forceinline__ int lds_load_acq(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Waits until *p >= v (p in LDS) within the grid barrier's time limit; past
// it the wave raises the abort flag and goes on, and the kernel stops at its
// next grid barrier.
__device__ __forceinline__ void lds_wait_ge(const int* p, int v, GridBar* bar) {
  if (lds_load_acq(p) >= v) return;
  const unsigned long long t0 = wall_clock64();
  while (lds_load_acq(p) < v) {
    __builtin_amdgcn_s_sleep(1);
    if (wall_clock64() - t0 > bar->spin_limit) {
      atomicExch(&bar->abort, 1);
      return;
    }
  }
}

// Resets the claim state (all threads; ends with a workgroup barrier).
__device__ __forceinline__ void units_reset(UnitSync& us, double* acc) {
  if (threadIdx.x == 0) {
    us.claim = 0;
    us.added = 0;
    for (int b = 0; b < kUnitRing / kUnitBatch; ++b) us.count[b] = 0;
  }
  if (threadIdx.x < kUnitNV * kSys) acc[threadIdx.x] = 0;
  __syncthreads();
}

// Runs body(row0, cnt, part) for every unit of UR rows of the workgroup's
// rows, claimed by the calling waves; part[NV] (zeroed per unit) takes the
// unit's sums per lane, and conv(part[k]) turns them into the sums of system
// `lane`.  With NV > 0, acc[k * 64 + lane] ends as the workgroup's sums in
// unit order (after the closing workgroup barrier).  Wave-uniform; all
// threads call it.
template <int NV, int UR, class F, class C>
__device__ __forceinline__ void claim_units(const WgRows& wr, UnitSync& us, double* ring, double* acc, GridBar* bar,
                                            F&& body, C&& conv) {
  static_assert(NV <= kUnitNV, "too many sums");
  static_assert(kPW % UR == 0, "a unit stays within a group of rows");
  const int j = threadIdx.x & 63;
  const int nunits = (wr.nrows + UR - 1) / UR;
  // Counters are advanced by every lane of the wave (one LDS instruction, so
  // the wave's results are consecutive and / 64 names the unit), not by lane 0
  // alone: the compiler may restructure a loop around a lane-0 branch so that
  // lane 0 leaves it apart from the other lanes, and a broadcast of a value
  // only lane 0 holds then reads another lane's.
  for (;;) {
    const int u = __builtin_amdgcn_readfirstlane(atomicAdd(&us.claim, 1)) / kWave;
    if (u >= nunits) break;
    const int q = u * UR;
    const int row0 = wr.base + q % kPW + (q / kPW) * wr.step;
    const int cnt = min(UR, wr.nrows - q);
    double part[NV > 0 ? NV : 1];
#pragma unroll
    for (int k = 0; k < (NV > 0 ? NV : 1); ++k) part[k] = 0;
    body(row0, cnt, part);
    if constexpr (NV > 0) {
#pragma unroll
      for (int k = 0; k < NV; ++k) part[k] = conv(part[k]);
      const int b = u / kUnitBatch, slot = u % kUnitRing;
      // the ring slot is free once the batch kUnitRing / kUnitBatch earlier is added
      lds_wait_ge(&us.added, b - (kUnitRing / kUnitBatch - 1), bar);
#pragma unroll
      for (int k = 0; k < NV; ++k) ring[(slot * kUnitNV + k) * kSys + j] = part[k];
      const int done = __builtin_amdgcn_readfirstlane(__hip_atomic_fetch_add(
                           &us.count[b % (kUnitRing / kUnitBatch)], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP)) /
                           kWave + 1;
      if (done == min(kUnitBatch, nunits - b * kUnitBatch)) {
        // this wave completed batch b: add it once batches 0 .. b-1 are in
        lds_wait_ge(&us.added, b, bar);
        const int s0 = (b * kUnitBatch) % kUnitRing;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
          double t = ring[(s0 * kUnitNV + k) * kSys + j];
          for (int m = 1; m < done; ++m) t += ring[((s0 + m) * kUnitNV + k) * kSys + j];
          acc[k * kSys + j] += t;
        }
        // every lane stores the same values
        us.count[b % (kUnitRing / kUnitBatch)] = 0;
        __hip_atomic_store(&us.added, b + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
  __syncthreads();
}

// The workgroup's sums from claim_units to partials[(k*G + block)*64 + lane].
template <int NV>
__device__ __forceinline__ void store_unit_partials(const double* acc, double* partials) {
  const int j = threadIdx.x & 63, G = gridDim.x;
  if (threadIdx.x < kSys) {
#pragma unroll
    for (int k = 0; k < NV; ++k) partials[((size_t)k * G + blockIdx.x) * kSys + j] = acc[k * kSys + j];
  }
}

// Value of `v` in lane l (wave-uniform), in every lane.
__device__ __forceinline__ int bcast(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ double bcast(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Entry-stream form of sweep_spmv for the wave's contiguous rows [ra, rb)
// (MAP 3): the entries [rowptr[ra], rowptr[rb]) are one contiguous run,
// loaded 64 at a time with one vector load each of col, K and M (lane u
// holds entry c0 + u), the next 64 loaded while the current ones are used.
// Entry p's column and coefficients reach every lane (= system) by
// readlane.  The x gathers go out NG entries at a time regardless of row
// boundaries, each round's gathers issued before the previous round's
// multiply-adds, so 2 NG gathers of 1 KB are in flight; a row's sum is
// finished when the walk passes its last entry.  The product is formed as
// K x - kappa_j (M x), two real-coefficient sums per lane.  Every row must
// have an entry (the sweep's nonzero-diagonal check guarantees it).  Lanes
// of finished systems load from the addresses of a running system's lane
// (same lines, no extra traffic) so every load runs with all lanes on --
// the broadcasts read lanes that must all have loaded -- and they neither
// store nor add to the sums.
template <int EPI, int NV, int NG>
__device__ __forceinline__ void sweep_spmv_stream(const SweepArgs& a, int ra, int rb, const double2* src,
                                                  double2* dst, bool act, double2 kap, double (&part)[NV]) {
  static_assert(64 % NG == 0, "rounds tile a chunk");
  const int j = threadIdx.x & 63;
  const unsigned long long live = __ballot(act);
  if (live == 0 || ra >= rb) return;  // uniform
  const int jl = act ? j : __ffsll((long long)live) - 1;
  const cptr<int> rowptr = as_const(a.rowptr);
  ra = uni(ra);
  rb = uni(rb);
  const int pa = rowptr[ra], pb = rowptr[rb];
  // lane i holds the end of row rbase + i
  int rbase = ra;
  int rpv = a.rowptr[min(rbase + 1 + j, rb)];
  int row = ra;
  int rend = bcast(rpv, 0);
  auto operand = [&](int r) -> double2 {
    const size_t o = (size_t)r * kSys + jl;
    return EPI == 1 ? a.RH[o] : EPI == 2 ? a.SH[o] : a.B[o];
  };
  double2 pre = operand(row);
  double2 dg = EPI == 2 ? sweep_diag(a, row, kap) : make_double2(0, 0);
  auto chunk = [&](int c0, int& cv, double& kv, double& mv) {
    const int q = min(c0 + j, pb - 1);
    cv = ldnt(a.col + q);
    kv = __builtin_nontemporal_load(a.K + q);
    mv = __builtin_nontemporal_load(a.M + q);
  };
  int cv0, cv1;
  double kv0, kv1, mv0, mv1;
  chunk(pa, cv0, kv0, mv0);
  chunk(pa + 64, cv1, kv1, mv1);
  double2 acK = make_double2(0, 0), acM = make_double2(0, 0);
  double2 xv[NG], xn[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) xv[g] = src[(size_t)bcast(cv0, g) * kSys + jl];
  const int nr = (pb - pa + NG - 1) / NG;
  for (int r = 0; r < nr; ++r) {
    const int u = (r * NG) & 63, un = ((r + 1) * NG) & 63;
    const bool next_chunk = un == 0;
    if (r + 1 < nr) {
      const int cvs = next_chunk ? cv1 : cv0;
#pragma unroll
      for (int g = 0; g < NG; ++g) xn[g] = src[(size_t)bcast(cvs, un + g) * kSys + jl];
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int p = pa + r * NG + g;
      if (p < pb) {
        const double k = bcast(kv0, u + g), m = bcast(mv0, u + g);
        acK.x = fma(k, xv[g].x, acK.x);
        acK.y = fma(k, xv[g].y, acK.y);
        acM.x = fma(m, xv[g].x, acM.x);
        acM.y = fma(m, xv[g].y, acM.y);
        while (p + 1 == rend) {
          const double2 y = csub(acK, cmul(kap, acM));
          acK = make_double2(0, 0);
          acM = make_double2(0, 0);
          const size_t o = (size_t)row * kSys + j;
          if (act) {
            if constexpr (EPI == 3) {
              part[0] += cabs2(csub(pre, y));
            } else if constexpr (EPI == 1) {
              stnt(dst + o, y);
              part[0] = fma(pre.x, y.x, fma(pre.y, y.y, part[0]));
              part[1] = fma(pre.x, y.y, fma(-pre.y, y.x, part[1]));
            } else {
              stnt(dst + o, y);
              const double2 sv = cmul(dg, pre);
              part[0] = fma(y.x, y.x, fma(y.y, y.y, part[0]));
              part[1] = fma(y.x, sv.x, fma(y.y, sv.y, part[1]));
              part[2] = fma(y.x, sv.y, fma(-y.y, sv.x, part[2]));
            }
          }
          if (++row >= rb) break;
          pre = operand(row);
          if constexpr (EPI == 2) dg = sweep_diag(a, row, kap);
          if (row - rbase == 64) {
            rbase = row;
            rpv = a.rowptr[min(rbase + 1 + j, rb)];
          }
          rend = bcast(rpv, row - rbase);
        }
      }
    }
    if (next_chunk) {
      cv0 = cv1; kv0 = kv1; mv0 = mv1;
      chunk(pa + (r + 1) * NG + 64, cv1, kv1, mv1);
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) xv[g] = xn[g];
  }
}

// Per-row form with the next row prefetched: lanes 0..15 of the wave hold
// the column, K and M of the current row's first 16 entries (one vector load
// each, issued while the previous row was in flight), so a row's gathers
// need not wait for its matrix entries.  The next row's extent, entries and
// epilogue operand are loaded behind the first gathers; then the
// multiply-adds, with each
// entry's column and coefficients broadcast by readlane.  The gathers go
// in rounds of 4, each issued before the previous round's sums (16 gathers
// at once spill registers; rounds of 8 spilled 25 VGPRs and ran 667 against
// 663 us per 64-system iteration).  Entries past the
// 16th (longer rows) go in rounds of 8 through scalar loads as in
// sweep_spmv.  The matrix loads run in every lane whatever its system's
// state (the broadcasts read lanes 0..15); gathers, sums and stores only in
// the lanes of running systems.  Every row has an entry (nonzero diagonal).
template <int EPI, int NV>
__device__ __forceinline__ void sweep_spmv_pf(const SweepArgs& a, int r0, int r1, int rs, const double2* src,
                                              double2* dst, bool act, double2 kap, double (&part)[NV]) {
  constexpr int W = 16, G = 4;  // entries prefetched per row; gathers per round
  const int j = threadIdx.x & 63;
  if (__ballot(act) == 0) return;  // uniform: no running system
  const cptr<int> rowptr = as_const(a.rowptr), col = as_const(a.col);
  const cptr<double> Kc = as_const(a.K), Mc = as_const(a.M);
  int row = uni(r0);
  if (row >= r1) return;
  int s = rowptr[row], e = rowptr[row + 1];
  auto fetch = [&](int s_, int e_, int& cv, double& kv, double& mv) {
    const int q = min(s_ + (j & (W - 1)), e_ - 1);
    cv = ldnt(a.col + q);
    kv = __builtin_nontemporal_load(a.K + q);
    mv = __builtin_nontemporal_load(a.M + q);
  };
  int cv, cvn = 0;
  double kv, mv, kvn = 0, mvn = 0;
  fetch(s, e, cv, kv, mv);
  for (; row < r1; row += rs) {
    const int len = e - s;
    const size_t o = (size_t)row * kSys + j;
    double2 acK = make_double2(0, 0), acM = make_double2(0, 0);
    double2 xv[G];
    // the first G gathers, then the next row and this row's epilogue
    // operand behind them, then the next G gathers and the sums
#pragma unroll
    for (int u = 0; u < G; ++u)
      if (u < len && act) xv[u] = src[(size_t)bcast(cv, u) * kSys + j];
    const int nrow = row + rs;
    int ns = 0, ne = 0;
    if (nrow < r1) {
      ns = rowptr[nrow];
      ne = rowptr[nrow + 1];
      fetch(ns, ne, cvn, kvn, mvn);
    }
    double2 pre = make_double2(0, 0), dg = make_double2(0, 0);
    if (act) pre = EPI == 1 ? a.RH[o] : EPI == 2 ? a.SH[o] : a.B[o];
    if (EPI == 2) dg = sweep_diag(a, row, kap);
#pragma unroll
    for (int h = 0; h < W / G; ++h) {
      double2 xn[G];
      if (h + 1 < W / G) {
#pragma unroll
        for (int u = 0; u < G; ++u)
          if ((h + 1) * G + u < len && act) xn[u] = src[(size_t)bcast(cv, (h + 1) * G + u) * kSys + j];
      }
#pragma unroll
      for (int u = 0; u < G; ++u) {
        if (h * G + u < len) {
          const double k = bcast(kv, h * G + u), m = bcast(mv, h * G + u);
          if (act) {
            acK.x = fma(k, xv[u].x, acK.x);
            acK.y = fma(k, xv[u].y, acK.y);
            acM.x = fma(m, xv[u].x, acM.x);
            acM.y = fma(m, xv[u].y, acM.y);
          }
        }
      }
      if (h + 1 < W / G) {
#pragma unroll
        for (int u = 0; u < G; ++u) xv[u] = xn[u];
      }
    }
    // entries past the 16th, 8 at a time
    for (int q0 = s + W; q0 < e; q0 += 8) {
      int c[8];
      double k8[8], m8[8];
      double2 x8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool in = q0 + u < e;
        const int q = in ? q0 + u : e - 1;
        c[u] = col[q];
        k8[u] = in ? Kc[q] : 0.0;
        m8[u] = in ? Mc[q] : 0.0;
      }
      if (act) {
#pragma unroll
        for (int u = 0; u < 8; ++u) x8[u] = src[(size_t)c[u] * kSys + j];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          acK.x = fma(k8[u], x8[u].x, acK.x);
          acK.y = fma(k8[u], x8[u].y, acK.y);
          acM.x = fma(m8[u], x8[u].x, acM.x);
          acM.y = fma(m8[u], x8[u].y, acM.y);
        }
      }
    }
    if (act) {
      const double2 y = csub(acK, cmul(kap, acM));
      if constexpr (EPI == 3) {
        part[0] += cabs2(csub(pre, y));
      } else if constexpr (EPI == 1) {
        stnt(dst + o, y);
        part[0] = fma(pre.x, y.x, fma(pre.y, y.y, part[0]));
        part[1] = fma(pre.x, y.y, fma(-pre.y, y.x, part[1]));
      } else {
        stnt(dst + o, y);
        const double2 sv = cmul(dg, pre);
        part[0] = fma(y.x, y.x, fma(y.y, y.y, part[0]));
        part[1] = fma(y.x, sv.x, fma(y.y, sv.y, part[1]));
        part[2] = fma(y.x, sv.y, fma(-y.y, sv.x, part[2]));
      }
    }
    s = ns;
    e = ne;
    cv = cvn;
    kv = kvn;
    mv = mvn;
  }
}

// sweep_diag at a row that differs between lanes (vector loads).
__device__ __forceinline__ double2 sweep_diag_v(const SweepArgs& a, int i, double2 kap) {
  const double k = a.kd[i], m = a.md[i];
  return make_double2(k - kap.x * m, -kap.y * m);
}

// The per-row product with the next row prefetched (sweep_spmv_pf) for RPW
// (2 or 4) rows per wave step: lane group q of 64 / RPW lanes takes rows r0 +
// (RPW k + q) rs, its lanes q*64/RPW + 0..15 hold its current row's first 16
// entries, and entry values reach the group's lanes by __shfl from there.
// Lane l works for system `sys`; part holds its sums (one row in RPW of its
// system's rows).
template <int EPI, int NV, int RPW>
__device__ __forceinline__ void sweep_spmv_hr(const SweepArgs& a, int r0, int r1, int rs, const double2* src,
                                              double2* dst, bool act, int sys, double2 kap, double (&part)[NV]) {
  constexpr int W = 16, G = 4, LPR = kWave / RPW;
  static_assert(LPR >= W, "a lane group holds a row's first 16 entries");
  const int l = threadIdx.x & 63, hl = l & ~(LPR - 1);
  if (__ballot(act) == 0) return;  // uniform: no running system
  const int rb = uni(r0);
  if (rb >= r1) return;
  int row = rb + (l / LPR) * rs;
  int s = 0, e = 0;
  if (row < r1) {
    s = a.rowptr[row];
    e = a.rowptr[row + 1];
  }
  auto fetch = [&](int s_, int e_, int& cv, double& kv, double& mv) {
    const int q = max(min(s_ + (l & (W - 1)), e_ - 1), 0);
    cv = ldnt(a.col + q);
    kv = __builtin_nontemporal_load(a.K + q);
    mv = __builtin_nontemporal_load(a.M + q);
  };
  int cv, cvn = 0;
  double kv, mv, kvn = 0, mvn = 0;
  fetch(s, e, cv, kv, mv);
  for (int base = rb; base < r1; base += RPW * rs) {
    const bool has = row < r1;
    const int len = has ? e - s : 0;
    int lenw = __shfl(len, 0);
#pragma unroll
    for (int q = 1; q < RPW; ++q) lenw = max(lenw, __shfl(len, q * LPR));
    const size_t o = (size_t)(has ? row : 0) * kSys + sys;
    double2 acK = make_double2(0, 0), acM = make_double2(0, 0);
    double2 xv[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int c = __shfl(cv, hl + u);
      if (u < len && act) xv[u] = src[(size_t)c * kSys + sys];
    }
    const int nrow = row + RPW * rs;
    int ns = 0, ne = 0;
    if (nrow < r1) {
      ns = a.rowptr[nrow];
      ne = a.rowptr[nrow + 1];
    }
    fetch(ns, ne, cvn, kvn, mvn);
    double2 pre = make_double2(0, 0), dg = make_double2(0, 0);
    if (act && has) pre = EPI == 1 ? a.RH[o] : EPI == 2 ? a.SH[o] : a.B[o];
    if (EPI == 2 && has) dg = sweep_diag_v(a, row, kap);
#pragma unroll
    for (int h = 0; h < W / G; ++h) {
      double2 xn[G];
      if (h + 1 < W / G) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const int c = __shfl(cv, hl + (h + 1) * G + u);
          if ((h + 1) * G + u < len && act) xn[u] = src[(size_t)c * kSys + sys];
        }
      }
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const double k = __shfl(kv, hl + h * G + u), m = __shfl(mv, hl + h * G + u);
        if (h * G + u < len && act) {
          acK.x = fma(k, xv[u].x, acK.x);
          acK.y = fma(k, xv[u].y, acK.y);
          acM.x = fma(m, xv[u].x, acM.x);
          acM.y = fma(m, xv[u].y, acM.y);
        }
      }
      if (h + 1 < W / G) {
#pragma unroll
        for (int u = 0; u < G; ++u) xv[u] = xn[u];
      }
    }
    // entries past the 16th, 4 at a time (lane-varying indices take vector
    // registers), up to the longer of the two rows
    for (int q0 = W; q0 < lenw; q0 += 4) {
      int c[4];
      double k8[4], m8[4];
      double2 x8[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool in = q0 + u < len;
        const int q = len > 0 ? s + min(q0 + u, len - 1) : 0;
        c[u] = a.col[q];
        k8[u] = in ? a.K[q] : 0.0;
        m8[u] = in ? a.M[q] : 0.0;
      }
      if (act) {
#pragma unroll
        for (int u = 0; u < 4; ++u) x8[u] = src[(size_t)c[u] * kSys + sys];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          acK.x = fma(k8[u], x8[u].x, acK.x);
          acK.y = fma(k8[u], x8[u].y, acK.y);
          acM.x = fma(m8[u], x8[u].x, acM.x);
          acM.y = fma(m8[u], x8[u].y, acM.y);
        }
      }
    }
    if (act && has) {
      const double2 y = csub(acK, cmul(kap, acM));
      if constexpr (EPI == 3) {
        part[0] += cabs2(csub(pre, y));
      } else if constexpr (EPI == 1) {
        stnt(dst + o, y);
        part[0] = fma(pre.x, y.x, fma(pre.y, y.y, part[0]));
        part[1] = fma(pre.x, y.y, fma(-pre.y, y.x, part[1]));
      } else {
        stnt(dst + o, y);
        const double2 sv = cmul(dg, pre);
        part[0] = fma(y.x, y.x, fma(y.y, y.y, part[0]));
        part[1] = fma(y.x, sv.x, fma(y.y, sv.y, part[1]));
        part[2] = fma(y.x, sv.y, fma(-y.y, sv.x, part[2]));
      }
    }
    row = nrow;
    s = ns;
    e = ne;
    cv = cvn;
    kv = kvn;
    mv = mvn;
  }
}

// The product of a phase in the shape PF of the kernel: 1 the per-row form
// (rows r0, r0 + rs, ...), 2 the entry stream over [r0, r1) (rs == 1), 3 the
// per-row form with the next row prefetched.
template <int PF, int EPI, int NV>
__device__ __forceinline__ void sweep_product(const SweepArgs& a, int r0, int r1, int rs, const double2* src,
                                              double2* dst, bool act, double2 kap, double (&part)[NV]) {
  if constexpr (PF == 1) sweep_spmv<EPI, NV>(a, r0, r1, rs, src, dst, act, kap, part);
  else if constexpr (PF == 3) sweep_spmv_pf<EPI, NV>(a, r0, r1, rs, src, dst, act, kap, part);
  else sweep_spmv_stream<EPI, NV, 4>(a, r0, r1, src, dst, act, kap, part);
}

// PF: product form (1 per row, 2 entry stream, 3 per row with the next row
// prefetched); MAP: row mapping (sweep_rows).
template <int PF, int MAP>
__global__ __launch_bounds__(kPB) void k_sweep(SweepArgs a) {
  static_assert(PF != 2 || MAP == 3, "the entry stream walks contiguous rows");
  static_assert(kUnitRing * kUnitNV >= 4 * kPW, "lds holds the unit ring and the per-wave sums");
  __shared__ double lds[kUnitRing * kUnitNV * kSys];
  __shared__ double uacc[kUnitNV * kSys];
  __shared__ UnitSync us;
  // Workgroup 0 keeps every system's scalars in LDS, so that its updates at
  // the barriers do not wait on memory (a chain of dependent loads after the
  // barrier's cache invalidate cost several us per barrier); after each
  // update it copies the fields the phases read to a.st, and all of the state
  // at the end.  The phases read a.st.
  __shared__ BatchState ls;
  unsigned epoch = 0;
  BatchState* st = a.st;
  const int j = threadIdx.x & 63;
  const int G = gridDim.x;
  int r0, r1, rs;
  sweep_rows<MAP>(a.n, G, r0, r1, rs);
  const WgRows wr = sweep_wg_rows(a.n, G);
  const bool lane_ok = j < a.nsys;
  const double2 kap = lane_ok ? a.kap[j] : make_double2(0, 0);

  // ---- start: r = rhat = b, phat = D^-1 b, x = 0
  {
    double part[1] = {0};
    for (int row = r0; row < r1; row += rs) {
      const size_t o = (size_t)row * kSys + j;
      if (!lane_ok) continue;
      const double2 b = a.B[o];
      a.R[o] = b; a.RH[o] = b;
      a.PH[o] = cmul(crecip(sweep_diag(a, row, kap)), b);
      a.X[o] = make_double2(0, 0);
      part[0] += cabs2(b);
    }
    store_partials64<1>(part, a.partials, lds);
    if (barrier_reduce<1>(a.bar, epoch, a.partials, lds, [&](const double(&tot)[1]) {
          for (int i = threadIdx.x; i < (int)(sizeof(BatchState) / 4); i += blockDim.x)
            reinterpret_cast<unsigned*>(&ls)[i] = 0;
          __syncthreads();
          if (threadIdx.x < kSys) {
            if (threadIdx.x < a.nsys) init_sys(&ls, threadIdx.x, tot[0], a.tol, a.maxit);
            else ls.status[threadIdx.x] = HK_OK;
          }
          if (threadIdx.x == 0) { ls.iter = 1; ls.maxit = a.maxit; ls.changed = 0; }
          __syncthreads();
          if (threadIdx.x == 0) {
            int run = 0;
            for (int u = 0; u < a.nsys; ++u) run += ls.status[u] == B_RUN;
            ls.running = run;
          }
          if (PF == 3 && threadIdx.x == 0 && a.tail && ls.running > 0 && ls.running <= 32)
            ls.handoff = ls.running <= 16 ? 4 : 2;
          publish_state(st, ls);
        }))
      return;
  }

  while (st->running > 0 && !(PF == 3 && st->handoff)) {
    const long long it = st->iter;
    bool act = lane_ok && st->status[j] == B_RUN;
    // ---- phat = D^-1 (r - beta omega v) + beta phat
    // (the element-wise phases stream their [node][64] vectors, 120 MB each
    // on the 48^3 sweep, with non-temporal loads and stores: 630 -> 595 us
    // per iteration against plain loads)
    if (it > 1) {
      const double2 beta = st->beta[j], bo = cmul(st->beta[j], st->omega[j]);
      units_reset(us, uacc);
      claim_units<0, kUnitRows>(wr, us, lds, uacc, a.bar, [&](int row0, int cnt, auto&) {
        double2 rv[kUnitRows] = {}, vv[kUnitRows] = {}, pv[kUnitRows] = {}, dv[kUnitRows];
#pragma unroll
        for (int u = 0; u < kUnitRows; ++u) {
          const int r = row0 + min(u, cnt - 1);
          const size_t o = (size_t)r * kSys + j;
          if (act) {
            rv[u] = ldnt(a.R + o); vv[u] = ldnt(a.V + o); pv[u] = ldnt(a.PH + o);
          }
          dv[u] = sweep_diag(a, r, kap);
        }
#pragma unroll
        for (int u = 0; u < kUnitRows; ++u)
          if (act && u < cnt)
            stnt(a.PH + (size_t)(row0 + u) * kSys + j, cfma(beta, pv[u], cmul(crecip(dv[u]), csub(rv[u], cmul(bo, vv[u])))));
      }, [](double v) { return v; });
      if (barrier_last(a.bar, epoch, [] {})) return;
    }
    // ---- v = A phat ; sigma = rhat^H v
    {
      double part[2] = {0, 0};
      sweep_product<PF, 1, 2>(a, r0, r1, rs, a.PH, a.V, act, kap, part);
      store_partials64<2>(part, a.partials, lds);
      if (barrier_reduce<2>(a.bar, epoch, a.partials, lds, [&](const double(&tot)[2]) {
            if (threadIdx.x < a.nsys) upd_sigma(&ls, threadIdx.x, make_double2(tot[0], tot[1]));
            publish_phase_state(st, ls);
          }))
        return;
    }
    act = lane_ok && st->status[j] == B_RUN;
    // ---- s = r - alpha v ; shat = D^-1 s ; ||s||^2
    {
      const double2 alpha = st->alpha[j];
      units_reset(us, uacc);
      claim_units<1, kUnitRows>(wr, us, lds, uacc, a.bar, [&](int row0, int cnt, auto& part) {
        double2 rv[kUnitRows] = {}, vv[kUnitRows] = {}, dv[kUnitRows];
#pragma unroll
        for (int u = 0; u < kUnitRows; ++u) {
          const int r = row0 + min(u, cnt - 1);
          const size_t o = (size_t)r * kSys + j;
          if (act) {
            rv[u] = ldnt(a.R + o); vv[u] = ldnt(a.V + o);
          }
          dv[u] = sweep_diag(a, r, kap);
        }
#pragma unroll
        for (int u = 0; u < kUnitRows; ++u) {
          if (act && u < cnt) {
            const double2 s = csub(rv[u], cmul(alpha, vv[u]));
            stnt(a.SH + (size_t)(row0 + u) * kSys + j, cmul(crecip(dv[u]), s));
            part[0] += cabs2(s);
          }
        }
      }, [](double v) { return v; });
      store_unit_partials<1>(uacc, a.partials);
      if (barrier_reduce<1>(a.bar, epoch, a.partials, lds, [&](const double(&tot)[1]) {
            if (threadIdx.x < a.nsys) upd_s(&ls, threadIdx.x, tot[0]);
            publish_phase_state(st, ls);
          }))
        return;
    }
    act = lane_ok && st->status[j] == B_RUN;
    // ---- t = A shat ; tau = t^H t ; t^H s
    {
      double part[3] = {0, 0, 0};
      sweep_product<PF, 2, 3>(a, r0, r1, rs, a.SH, a.T, act, kap, part);
      store_partials64<3>(part, a.partials, lds);
      if (barrier_reduce<3>(a.bar, epoch, a.partials, lds, [&](const double(&tot)[3]) {
            if (threadIdx.x < a.nsys) upd_omega(&ls, threadIdx.x, tot[0], make_double2(tot[1], tot[2]));
            publish_phase_state(st, ls);
          }))
        return;
    }
    // ---- x += alpha phat + omega shat ; r = s - omega t ; ||r||^2 ; rhat^H r
    {
      const int sj = lane_ok ? st->status[j] : HK_OK;
      const bool run = sj == B_RUN, half = sj == B_HALF || sj == B_TAUBD;
      const double2 alpha = st->alpha[j], omega = st->omega[j];
      units_reset(us, uacc);
      claim_units<3, kUnitRows>(wr, us, lds, uacc, a.bar, [&](int row0, int cnt, auto& part) {
        // two rows at a time (five loads each)
#pragma unroll
        for (int h = 0; h < kUnitRows; h += 2) {
          double2 sh[2] = {}, ph[2] = {}, xv[2] = {}, tv[2] = {}, hv[2] = {}, dv[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int r = row0 + min(h + u, cnt - 1);
            const size_t o = (size_t)r * kSys + j;
            if (run) {
              sh[u] = ldnt(a.SH + o); ph[u] = ldnt(a.PH + o); xv[u] = ldnt(a.X + o); tv[u] = ldnt(a.T + o); hv[u] = ldnt(a.RH + o);
            } else if (half) {
              ph[u] = ldnt(a.PH + o); xv[u] = ldnt(a.X + o);
            }
            dv[u] = sweep_diag(a, r, kap);
          }
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            if (h + u >= cnt) continue;
            const size_t o = (size_t)(row0 + h + u) * kSys + j;
            if (run) {
              stnt(a.X + o, cfma(omega, sh[u], cfma(alpha, ph[u], xv[u])));
              const double2 r = csub(cmul(dv[u], sh[u]), cmul(omega, tv[u]));
              stnt(a.R + o, r);
              part[0] += cabs2(r);
              part[1] = fma(hv[u].x, r.x, fma(hv[u].y, r.y, part[1]));
              part[2] = fma(hv[u].x, r.y, fma(-hv[u].y, r.x, part[2]));
            } else if (half) {
              a.X[o] = cfma(alpha, ph[u], xv[u]);
            }
          }
        }
      }, [](double v) { return v; });
      store_unit_partials<3>(uacc, a.partials);
      if (barrier_reduce<3>(a.bar, epoch, a.partials, lds, [&](const double(&tot)[3]) {
            // wave 0 (thread j = system j) updates and counts the running
            // systems with one ballot
            if (threadIdx.x < kWave) {
              const int r = threadIdx.x < a.nsys ? upd_xr(&ls, threadIdx.x, tot[0], make_double2(tot[1], tot[2])) : 0;
              const int run = __popcll(__ballot(r != 0));
              if (threadIdx.x == 0) {
                ls.running = run;
                ls.iter = ls.iter + 1;
                // at most 32 systems left: hand the rest to the multi-row launches
                if (PF == 3 && a.tail && run > 0 && run <= 32) ls.handoff = run <= 16 ? 4 : 2;
              }
            }
            publish_phase_state(st, ls);
            if constexpr (PF == 3) {
              // a hand-off needs every field in memory
              __syncthreads();
              if (ls.handoff) publish_state(st, ls);
            }
          }))
        return;
    }
  }
  if constexpr (PF == 3) {
    if (st->handoff) {
      // k_sweep_tail continues from here, with the barrier epochs (and
      // stamps) running on from this launch's
      if (blockIdx.x == 0 && threadIdx.x == 0) st->epoch0 = epoch;
      return;
    }
  }
  // ---- true residual ||b - A x||^2 per system
  {
    double part[1] = {0};
    sweep_product<PF, 3, 1>(a, r0, r1, rs, a.X, nullptr, lane_ok, kap, part);
    store_partials64<1>(part, a.partials, lds);
    barrier_reduce<1>(a.bar, epoch, a.partials, lds, [&](const double(&tot)[1]) {
      if (threadIdx.x < a.nsys) ls.rr_true[threadIdx.x] = tot[0];
      publish_state(st, ls);
    });
  }
}

// The rest of a sweep once at most 64 / RPW systems run (product form 3;
// RPW = 2 from 32 systems, 4 from 16): in the last stretch few systems
// remain, and an iteration cost ~350-410 us however few they were (the row
// walks' latency and the barriers stay).  Here a wave step is RPW rows: lane
// group q (64 / RPW lanes) takes row RPW k + q of the wave's rows, its lane p
// working for the p-th running system (s_map; s_inv[j] = the position of
// system j, or -1), and a claimed unit is 4 RPW rows.  Every workgroup builds
// the same map from the statuses the previous launch left in memory;
// workgroup 0 takes the whole state into LDS.  Separate kernels, so that the
// multi-row code does not raise k_sweep's register count.
template <int MAP, int RPW>
__global__ __launch_bounds__(kPB) void k_sweep_tail(SweepArgs a) {
  constexpr int PF = 3, LPR = kWave / RPW;
  __shared__ double lds[kUnitRing * kUnitNV * kSys];
  __shared__ double uacc[kUnitNV * kSys];
  __shared__ UnitSync us;
  __shared__ BatchState ls;
  __shared__ int s_map[LPR], s_inv[kSys];
  BatchState* st = a.st;
  unsigned epoch = st->epoch0;
  const int j = threadIdx.x & 63;
  const int G = gridDim.x;
  int r0, r1, rs;
  sweep_rows<MAP>(a.n, G, r0, r1, rs);
  const WgRows wr = sweep_wg_rows(a.n, G);
  const bool lane_ok = j < a.nsys;
  const double2 kap = lane_ok ? a.kap[j] : make_double2(0, 0);
  if (threadIdx.x < kWave) {
    const bool r = lane_ok && st->status[j] == B_RUN;
    const unsigned long long m = __ballot(r);
    const int pos = __popcll(m & ((1ull << j) - 1ull));
    if (j < LPR) s_map[j] = -1;
    if (r && pos < LPR) s_map[pos] = j;
    s_inv[j] = r && pos < LPR ? pos : -1;
  }
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < (int)(sizeof(BatchState) / 4); i += blockDim.x)
      reinterpret_cast<unsigned*>(&ls)[i] = reinterpret_cast<const unsigned*>(st)[i];
  __syncthreads();
  while (st->running > 0 && !(RPW == 2 && st->handoff == 4)) {
    const int pm = s_map[j & (LPR - 1)], sub = j / LPR;
    const bool mapped = pm >= 0;
    const int sys = mapped ? pm : 0;
    const bool sys_ok = mapped && sys < a.nsys;
    const double2 kap_s = sys_ok ? a.kap[sys] : make_double2(0, 0);
    // a lane's sums as sums of system j = lane: the RPW lanes of a system
    // (p, p + LPR, ...) are added in that order
    const int invj = s_inv[j];
    auto to_sys = [&](double v) -> double {
      const int pp = invj >= 0 ? invj : 0;
      double t = __shfl(v, pp);
#pragma unroll
      for (int q = 1; q < RPW; ++q) t += __shfl(v, pp + q * LPR);
      return invj >= 0 ? t : 0.0;
    };
    auto diag = [&](int r) { return sweep_diag_v(a, r, kap_s); };
    constexpr int UR = kUnitRows * RPW;  // rows per claimed unit; a lane takes row0 + u RPW + sub
    const long long it = st->iter;
    bool act = sys_ok && st->status[sys] == B_RUN;
    // ---- phat = D^-1 (r - beta omega v) + beta phat
    if (it > 1) {
      const double2 beta = st->beta[sys], bo = cmul(st->beta[sys], st->omega[sys]);
      units_reset(us, uacc);
      claim_units<0, UR>(wr, us, lds, uacc, a.bar, [&](int row0, int cnt, auto&) {
        double2 rv[kUnitRows] = {}, vv[kUnitRows] = {}, pv[kUnitRows] = {}, dv[kUnitRows];
#pragma unroll
        for (int u = 0; u < kUnitRows; ++u) {
          const int r = row0 + min(u * RPW + sub, cnt - 1);
          const size_t o = (size_t)r * kSys + sys;
          if (act) {
            rv[u] = ldnt(a.R + o); vv[u] = ldnt(a.V + o); pv[u] = ldnt(a.PH + o);
          }
          dv[u] = diag(r);
        }
#pragma unroll
        for (int u = 0; u < kUnitRows; ++u)
          if (act && u * RPW + sub < cnt)
            stnt(a.PH + (size_t)(row0 + u * RPW + sub) * kSys + sys,
                 cfma(beta, pv[u], cmul(crecip(dv[u]), csub(rv[u], cmul(bo, vv[u])))));
      }, to_sys);
      if (barrier_last(a.bar, epoch, [] {})) return;
    }
    // ---- v = A phat ; sigma = rhat^H v
    {
      double part[2] = {0, 0};
      sweep_spmv_hr<1, 2, RPW>(a, r0, r1, rs, a.PH, a.V, act, sys, kap_s, part);
      part[0] = to_sys(part[0]);
      part[1] = to_sys(part[1]);
      store_partials64<2>(part, a.partials, lds);
      if (barrier_reduce<2>(a.bar, epoch, a.partials, lds, [&](const double(&tot)[2]) {
            if (threadIdx.x < a.nsys) upd_sigma(&ls, threadIdx.x, make_double2(tot[0], tot[1]));
            publish_phase_state(st, ls);
          }))
        return;
    }
    act = sys_ok && st->status[sys] == B_RUN;
    // ---- s = r - alpha v ; shat = D^-1 s ; ||s||^2
    {
      const double2 alpha = st->alpha[sys];
      units_reset(us, uacc);
      claim_units<1, UR>(wr, us, lds, uacc, a.bar, [&](int row0, int cnt, auto& part) {
        double2 rv[kUnitRows] = {}, vv[kUnitRows] = {}, dv[kUnitRows];
#pragma unroll
        for (int u = 0; u < kUnitRows; ++u) {
          const int r = row0 + min(u * RPW + sub, cnt - 1);
          const size_t o = (size_t)r * kSys + sys;
          if (act) {
            rv[u] = ldnt(a.R + o); vv[u] = ldnt(a.V + o);
          }
          dv[u] = diag(r);
        }
#pragma unroll
        for (int u = 0; u < kUnitRows; ++u) {
          if (act && u * RPW + sub < cnt) {
            const double2 s = csub(rv[u], cmul(alpha, vv[u]));
            stnt(a.SH + (size_t)(row0 + u * RPW + sub) * kSys + sys, cmul(crecip(dv[u]), s));
            part[0] += cabs2(s);
          }
        }
      }, to_sys);
      store_unit_partials<1>(uacc, a.partials);
      if (barrier_reduce<1>(a.bar, epoch, a.partials, lds, [&](const double(&tot)[1]) {
            if (threadIdx.x < a.nsys) upd_s(&ls, threadIdx.x, tot[0]);
            publish_phase_state(st, ls);
          }))
        return;
    }
    act = sys_ok && st->status[sys] == B_RUN;
    // ---- t = A shat ; tau = t^H t ; t^H s
    {
      double part[3] = {0, 0, 0};
      sweep_spmv_hr<2, 3, RPW>(a, r0, r1, rs, a.SH, a.T, act, sys, kap_s, part);
#pragma unroll
      for (int k = 0; k < 3; ++k) part[k] = to_sys(part[k]);
      store_partials64<3>(part, a.partials, lds);
      if (barrier_reduce<3>(a.bar, epoch, a.partials, lds, [&](const double(&tot)[3]) {
            if (threadIdx.x < a.nsys) upd_omega(&ls, threadIdx.x, tot[0], make_double2(tot[1], tot[2]));
            publish_phase_state(st, ls);
          }))
        return;
    }
    // ---- x += alpha phat + omega shat ; r = s - omega t ; ||r||^2 ; rhat^H r
    {
      const int sj = sys_ok ? st->status[sys] : HK_OK;
      const bool run = sj == B_RUN, half = sj == B_HALF || sj == B_TAUBD;
      const double2 alpha = st->alpha[sys], omega = st->omega[sys];
      units_reset(us, uacc);
      claim_units<3, UR>(wr, us, lds, uacc, a.bar, [&](int row0, int cnt, auto& part) {
        // two rows at a time (five loads each)
#pragma unroll
        for (int h = 0; h < kUnitRows; h += 2) {
          double2 sh[2] = {}, ph[2] = {}, xv[2] = {}, tv[2] = {}, hv[2] = {}, dv[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int r = row0 + min((h + u) * RPW + sub, cnt - 1);
            const size_t o = (size_t)r * kSys + sys;
            if (run) {
              sh[u] = ldnt(a.SH + o); ph[u] = ldnt(a.PH + o); xv[u] = ldnt(a.X + o); tv[u] = ldnt(a.T + o); hv[u] = ldnt(a.RH + o);
            } else if (half) {
              ph[u] = ldnt(a.PH + o); xv[u] = ldnt(a.X + o);
            }
            dv[u] = diag(r);
          }
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            if ((h + u) * RPW + sub >= cnt) continue;
            const size_t o = (size_t)(row0 + (h + u) * RPW + sub) * kSys + sys;
            if (run) {
              stnt(a.X + o, cfma(omega, sh[u], cfma(alpha, ph[u], xv[u])));
              const double2 r = csub(cmul(dv[u], sh[u]), cmul(omega, tv[u]));
              stnt(a.R + o, r);
              part[0] += cabs2(r);
              part[1] = fma(hv[u].x, r.x, fma(hv[u].y, r.y, part[1]));
              part[2] = fma(hv[u].x, r.y, fma(-hv[u].y, r.x, part[2]));
            } else if (half) {
              a.X[o] = cfma(alpha, ph[u], xv[u]);
            }
          }
        }
      }, to_sys);
      store_unit_partials<3>(uacc, a.partials);
      if (barrier_reduce<3>(a.bar, epoch, a.partials, lds, [&](const double(&tot)[3]) {
            // wave 0 (thread j = system j) updates and counts the running
            // systems with one ballot
            if (threadIdx.x < kWave) {
              const int r = threadIdx.x < a.nsys ? upd_xr(&ls, threadIdx.x, tot[0], make_double2(tot[1], tot[2])) : 0;
              const int run = __popcll(__ballot(r != 0));
              if (threadIdx.x == 0) {
                ls.running = run;
                ls.iter = ls.iter + 1;
                // at most 16 left: hand them to the four-row launch
                if (RPW == 2 && run > 0 && run <= 16) ls.handoff = 4;
              }
            }
            publish_phase_state(st, ls);
            if constexpr (RPW == 2) {
              __syncthreads();
              if (ls.handoff == 4) publish_state(st, ls);
            }
          }))
        return;
    }
  }
  if constexpr (RPW == 2) {
    if (st->handoff == 4) {
      if (blockIdx.x == 0 && threadIdx.x == 0) st->epoch0 = epoch;
      return;
    }
  }
  // ---- true residual ||b - A x||^2 per system (one row per wave step)
  {
    double part[1] = {0};
    sweep_product<PF, 3, 1>(a, r0, r1, rs, a.X, nullptr, lane_ok, kap, part);
    store_partials64<1>(part, a.partials, lds);
    barrier_reduce<1>(a.bar, epoch, a.partials, lds, [&](const double(&tot)[1]) {
      if (threadIdx.x < a.nsys) ls.rr_true[threadIdx.x] = tot[0];
      publish_state(st, ls);
    });
  }
}

// ======================================================= (b) block-diagonal

struct BdArgs {
  int n, nsys, L;
  const int* rowptr;
  const int* col;
  const double2* val;
  const double2* d;      // diag(A)
  const double2* dinv;   // 1 / diag(A)
  const double2* B;
  double2* X;
  double2 *R, *RH, *PH, *V, *SH, *T;
  const int* sys_begin;  // system -> first row
  const int* sys_end;    // system -> one past its last row
  const int* sys_tile0;  // system -> first static tile (nsys+1 entries)
  // active tile list: tile t (of ntiles_active) covers rows act_row0[t] ..
  // act_end[t] - 1 (at most tile_rows rows) of system act_sys[t]
  int* act_sys;
  int* act_row0;
  int* act_end;
  double* partials;
  BatchState* st;
  GridBar* bar;
  double tol;
  long long maxit;
  int tile_rows;
};

// A tile of the active list as the phases see it, and the per-system
// scalars the phases read, staged in LDS at the start of a phase.
struct BdTile {
  int row0, end, sys;
};
struct BdShared {
  double2 alpha[kSys], omega[kSys], beta[kSys];
  int status[kSys];
};

// The phases cut the active tiles into units of UR rows: tile t holds units
// t P .. t P + P - 1, P = tile_rows / UR, unit p covering rows row0 + p UR ..
// (a unit past its tile's end is empty).  Workgroup lb (xcd_block order)
// takes the units [S lb / G, S (lb + 1) / G) of the S = na P, so every
// workgroup gets the same number of units: with whole tiles per workgroup
// (8 or 9 of the 2,112 tiles of the 32-system batch) a workgroup's product
// time followed its row count (correlation 0.84) and spread over 45%.  Its
// waves claim the units in order through an LDS counter, as the sweep's
// element-wise phases do, since the memory system serves a workgroup's
// waves unevenly.  f(tile, r0, acc) runs one unit in one wave; the unit's
// sums (acc, reduced over the wave) are added in unit order into the
// workgroup's per-system sums through an LDS ring, so they stay bitwise
// reproducible whichever wave ran which unit; they end in
// partials[(k*G + block)*64 + sys].  All threads call it.
struct BdRing {
  double v[kUnitRing][4];
  int sys[kUnitRing];
};
template <int NV, int UR, class F>
__device__ __forceinline__ void bd_units(const BdArgs& a, double* lds, BdShared& sh, UnitSync& us, BdRing& ring,
                                         F&& f) {
  static_assert(NV <= 3, "at most three sums");
  double* sysacc = lds;  // NV * 64
  const int G = gridDim.x;
  const int lb = xcd_block(blockIdx.x, G);
  const BatchState* st = a.st;
  const int na = st->ntiles_active;
  const int P = a.tile_rows / UR;
  const long long S = (long long)na * P;
  const int u0 = (int)((S * lb) / G), nunits = (int)((S * (lb + 1)) / G) - u0;
  for (int k = threadIdx.x; k < NV * kSys; k += kPB) sysacc[k] = 0;
  if (threadIdx.x < a.nsys) {
    const int j = threadIdx.x;
    sh.alpha[j] = st->alpha[j];
    sh.omega[j] = st->omega[j];
    sh.beta[j] = st->beta[j];
    sh.status[j] = st->status[j];
  }
  if (threadIdx.x == 0) {
    us.claim = 0;
    us.added = 0;
    for (int b = 0; b < kUnitRing / kUnitBatch; ++b) us.count[b] = 0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  // counters advanced by every lane of the wave, as in claim_units
  for (;;) {
    const int u = __builtin_amdgcn_readfirstlane(atomicAdd(&us.claim, 1)) / kWave;
    if (u >= nunits) break;
    const int t = (u0 + u) / P, p = (u0 + u) % P;
    const BdTile tile{__builtin_amdgcn_readfirstlane(a.act_row0[t]), __builtin_amdgcn_readfirstlane(a.act_end[t]),
                      __builtin_amdgcn_readfirstlane(a.act_sys[t])};
    const int r0 = tile.row0 + p * UR;
    double acc[NV > 0 ? NV : 1];
#pragma unroll
    for (int k = 0; k < (NV > 0 ? NV : 1); ++k) acc[k] = 0;
    if (r0 < tile.end) f(tile, r0, acc);
    if constexpr (NV > 0) {
#pragma unroll
      for (int k = 0; k < NV; ++k) acc[k] = wave_sum(acc[k]);
      const int b = u / kUnitBatch, slot = u % kUnitRing;
      lds_wait_ge(&us.added, b - (kUnitRing / kUnitBatch - 1), a.bar);
      // every lane stores the same values
#pragma unroll
      for (int k = 0; k < NV; ++k) ring.v[slot][k] = acc[k];
      ring.sys[slot] = tile.sys;
      const int done = __builtin_amdgcn_readfirstlane(__hip_atomic_fetch_add(
                           &us.count[b % (kUnitRing / kUnitBatch)], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP)) /
                           kWave + 1;
      if (done == min(kUnitBatch, nunits - b * kUnitBatch)) {
        lds_wait_ge(&us.added, b, a.bar);
        const int s0 = (b * kUnitBatch) % kUnitRing;
        if (lane < NV) {
          for (int m = 0; m < done; ++m) sysacc[lane * kSys + ring.sys[s0 + m]] += ring.v[s0 + m][lane];
        }
        us.count[b % (kUnitRing / kUnitBatch)] = 0;
        __hip_atomic_store(&us.added, b + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
  __syncthreads();
  if constexpr (NV > 0) {
    for (int k = threadIdx.x; k < NV * kSys; k += kPB) {
      const int kk = k / kSys, sy = k % kSys;
      a.partials[((size_t)kk * G + blockIdx.x) * kSys + sy] = sysacc[k];
    }
  }
}

// The rows [r0, min(r0 + UR, tile end)) of one unit in one wave: an R-row
// block (csr_block_rows, UR = R), or UR / (64 / L) passes of 64 / L rows with L
// lanes each; g(row, sum) is called in the lane that holds the row's sum.
template <int L, int R, int CH, class G2>
__device__ __forceinline__ void bd_unit_spmv(const BdArgs& a, const BdTile& tile, int r0, const double2* src,
                                             double2* stage, G2&& g) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if constexpr (L == kRowBlockL) {
    const double2 acc = csr_block_rows<R, CH, double2, int>(r0, tile.end, a.rowptr, a.col, a.val, src,
                                                            stage + w * CH * kWave);
    if (l < R && r0 + l < tile.end) g(r0 + l, acc);
  } else {
    constexpr int UR = 16, RP = kWave / L;
    for (int q = 0; q < UR; q += RP) {
      const int row = r0 + q + l / L;
      if (r0 + q >= tile.end) break;  // uniform across the wave
      double2 acc[1];
      csr_rows<L, 1, double2>(row, tile.end, a.rowptr, a.col, a.val, src, acc);
      if ((l & (L - 1)) == 0 && row < tile.end) g(row, acc[0]);
    }
  }
}

// Tile products: L-lane groups per row (R, CH unused), or L == kRowBlockL
// row blocks of R rows, CH entries per lane per pass (CH = 8 needs more than
// the 128 VGPRs a 1024-thread workgroup allows).  Tiles are a.tile_rows <=
// kPB rows (chosen at run time with the tile shape); the phases run them in
// units (bd_units).
template <int L, int R, int CH>
__global__ __launch_bounds__(kPB) void k_blockdiag(BdArgs a) {
  // [4 kSys] per-system sums | scratch shared by the barrier callbacks
  // (4 kPW kSys doubles) and the row-block staging area, which are never
  // live at the same time
  constexpr int kFin = 4 * kPW * kSys;
  constexpr int kStage = L == kRowBlockL ? kPW * CH * kWave * 2 : 0;
  __shared__ __align__(16) double lds[4 * kSys + (kFin > kStage ? kFin : kStage)];
  unsigned epoch = 0;
  double* fin = lds + 4 * kSys;
  double2* stage = reinterpret_cast<double2*>(fin);
  __shared__ BdShared sh;
  __shared__ UnitSync us;
  __shared__ BdRing ring;
  BatchState* st = a.st;
  // units: kWave rows (one per lane) in the element-wise phases, an R-row
  // block (or 16 rows of L-lane groups) in the products
  constexpr int kUR = L == kRowBlockL ? R : 16;
  auto unit_spmv = [&](const BdTile& tile, int r0, const double2* src, auto&& g) {
    bd_unit_spmv<L, R, CH>(a, tile, r0, src, stage, g);
  };
  // the row of the calling lane in an element-wise unit, or -1
  auto my_row = [](const BdTile& tile, int r0) {
    const int row = r0 + (int)(threadIdx.x & 63);
    return row < tile.end ? row : -1;
  };

  // (workgroup 0, all threads) rebuild the active tile list: the tiles of
  // the systems still running, or of every system when `all`
  auto fill_active = [&](bool all) {
    __shared__ int s_off[kSys + 1];
    if (threadIdx.x == 0) {
      int off = 0;
      for (int q = 0; q < a.nsys; ++q) {
        s_off[q] = off;
        if (all || st->status[q] == B_RUN) off += a.sys_tile0[q + 1] - a.sys_tile0[q];
      }
      s_off[a.nsys] = off;
      st->ntiles_active = off;
      st->changed = 0;
    }
    __syncthreads();
    for (int q = 0; q < a.nsys; ++q) {
      if (!all && st->status[q] != B_RUN) continue;
      const int base = s_off[q], cnt = a.sys_tile0[q + 1] - a.sys_tile0[q];
      const int r0 = a.sys_begin[q], end = a.sys_end[q], tr = a.tile_rows;
      for (int k = threadIdx.x; k < cnt; k += kPB) {
        a.act_sys[base + k] = q;
        a.act_row0[base + k] = r0 + k * tr;
        a.act_end[base + k] = min(r0 + (k + 1) * tr, end);
      }
    }
  };

  // ---- start: r = rhat = b, phat = D^-1 b, x = 0 (all tiles are active)
  bd_units<1, kWave>(a, lds, sh, us, ring, [&](const BdTile& tile, int r0, double(&acc)[1]) {
    const int row = my_row(tile, r0);
    if (row >= 0) {
      const double2 b = a.B[row];
      a.R[row] = b; a.RH[row] = b; a.PH[row] = cmul(a.dinv[row], b); a.X[row] = make_double2(0, 0);
      acc[0] += cabs2(b);
    }
  });
  if (barrier_reduce<1>(a.bar, epoch, a.partials, fin, [&](const double(&tot)[1]) {
        if (threadIdx.x < a.nsys) init_sys(st, threadIdx.x, tot[0], a.tol, a.maxit);
        if (threadIdx.x == 0) { st->iter = 1; st->maxit = a.maxit; }
        __syncthreads();
        if (threadIdx.x == 0) {
          int run = 0;
          for (int u = 0; u < a.nsys; ++u) run += st->status[u] == B_RUN;
          st->running = run;
        }
        __syncthreads();
        fill_active(false);
      }))
    return;

  while (st->running > 0) {
    const long long it = st->iter;
    if (it > 1) {
      bd_units<0, kWave>(a, lds, sh, us, ring, [&](const BdTile& tile, int r0, double(&)[1]) {
        const int row = my_row(tile, r0);
        if (row >= 0) {
          const double2 beta = sh.beta[tile.sys], bo = cmul(beta, sh.omega[tile.sys]);
          const double2 w = csub(a.R[row], cmul(bo, a.V[row]));
          a.PH[row] = cfma(beta, a.PH[row], cmul(a.dinv[row], w));
        }
      });
      if (barrier_last(a.bar, epoch, [] {})) return;
    }
    // v = A phat ; sigma
    bd_units<2, kUR>(a, lds, sh, us, ring, [&](const BdTile& tile, int r0, double(&acc)[2]) {
      unit_spmv(tile, r0, a.PH, [&](int row, double2 v) {
        a.V[row] = v;
        const double2 h = a.RH[row];
        acc[0] = fma(h.x, v.x, fma(h.y, v.y, acc[0]));
        acc[1] = fma(h.x, v.y, fma(-h.y, v.x, acc[1]));
      });
    });
    if (barrier_reduce<2>(a.bar, epoch, a.partials, fin, [&](const double(&tot)[2]) {
          if (threadIdx.x < a.nsys) upd_sigma(st, threadIdx.x, make_double2(tot[0], tot[1]));
        }))
      return;
    // s = r - alpha v ; shat ; ||s||^2
    bd_units<1, kWave>(a, lds, sh, us, ring, [&](const BdTile& tile, int r0, double(&acc)[1]) {
      const int row = my_row(tile, r0);
      if (row >= 0 && sh.status[tile.sys] == B_RUN) {
        const double2 s = csub(a.R[row], cmul(sh.alpha[tile.sys], a.V[row]));
        a.SH[row] = cmul(a.dinv[row], s);
        acc[0] += cabs2(s);
      }
    });
    if (barrier_reduce<1>(a.bar, epoch, a.partials, fin, [&](const double(&tot)[1]) {
          if (threadIdx.x < a.nsys) upd_s(st, threadIdx.x, tot[0]);
        }))
      return;
    // t = A shat ; tau ; t^H s
    bd_units<3, kUR>(a, lds, sh, us, ring, [&](const BdTile& tile, int r0, double(&acc)[3]) {
      if (sh.status[tile.sys] != B_RUN) return;
      unit_spmv(tile, r0, a.SH, [&](int row, double2 t) {
        a.T[row] = t;
        const double2 s = cmul(a.d[row], a.SH[row]);
        acc[0] = fma(t.x, t.x, fma(t.y, t.y, acc[0]));
        acc[1] = fma(t.x, s.x, fma(t.y, s.y, acc[1]));
        acc[2] = fma(t.x, s.y, fma(-t.y, s.x, acc[2]));
      });
    });
    if (barrier_reduce<3>(a.bar, epoch, a.partials, fin, [&](const double(&tot)[3]) {
          if (threadIdx.x < a.nsys) upd_omega(st, threadIdx.x, tot[0], make_double2(tot[1], tot[2]));
        }))
      return;
    // x, r updates ; ||r||^2 ; rhat^H r
    bd_units<3, kWave>(a, lds, sh, us, ring, [&](const BdTile& tile, int r0, double(&acc)[3]) {
      const int row = my_row(tile, r0);
      if (row < 0) return;
      const int ss = sh.status[tile.sys];
      const double2 alpha = sh.alpha[tile.sys], omega = sh.omega[tile.sys];
      if (ss == B_RUN) {
        const double2 shat = a.SH[row];
        a.X[row] = cfma(omega, shat, cfma(alpha, a.PH[row], a.X[row]));
        const double2 r = csub(cmul(a.d[row], shat), cmul(omega, a.T[row]));
        a.R[row] = r;
        acc[0] += cabs2(r);
        const double2 h = a.RH[row];
        acc[1] = fma(h.x, r.x, fma(h.y, r.y, acc[1]));
        acc[2] = fma(h.x, r.y, fma(-h.y, r.x, acc[2]));
      } else if (ss == B_HALF || ss == B_TAUBD) {
        a.X[row] = cfma(alpha, a.PH[row], a.X[row]);
      }
    });
    if (barrier_reduce<3>(a.bar, epoch, a.partials, fin, [&](const double(&tot)[3]) {
          __shared__ int s_run[kSys];
          if (threadIdx.x < kSys)
            s_run[threadIdx.x] = threadIdx.x < a.nsys
                                     ? upd_xr(st, threadIdx.x, tot[0], make_double2(tot[1], tot[2]))
                                     : 0;
          __syncthreads();
          if (threadIdx.x == 0) {
            int run = 0;
            for (int u = 0; u < kSys; ++u) run += s_run[u];
            st->running = run;
            st->iter = st->iter + 1;
          }
          __syncthreads();
          if (st->changed) fill_active(false);
        }))
      return;
  }
  // true residual: all tiles
  if (barrier_last(a.bar, epoch, [&] { fill_active(true); })) return;
  bd_units<1, kUR>(a, lds, sh, us, ring, [&](const BdTile& tile, int r0, double(&acc)[1]) {
    unit_spmv(tile, r0, a.X, [&](int row, double2 ax) {
      acc[0] += cabs2(csub(a.B[row], ax));
    });
  });
  barrier_reduce<1>(a.bar, epoch, a.partials, fin, [&](const double(&tot)[1]) {
    if (threadIdx.x < a.nsys) st->rr_true[threadIdx.x] = tot[0];
  });
}

// ------------------------------------------------------------- set-up kernels

__global__ void k_real_diag(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                            const double* __restrict__ K, const double* __restrict__ M,
                            double* kd, double* md) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double k = 0, m = 0;
  for (int p = rowptr[i]; p < rowptr[i + 1]; ++p)
    if (col[p] == i) { k += K[p]; m += M[p]; }
  kd[i] = k;
  md[i] = m;
}

// zero diagonal for some lane -> flag
__global__ void k_sweep_diag_check(int n, int nsys, const double* kd, const double* md,
                                   const double2* kap, int* flag) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  for (int j = 0; j < nsys; ++j) {
    const double re = kd[i] - kap[j].x * md[i], im = -kap[j].y * md[i];
    if (re == 0 && im == 0) { atomicOr(flag, 1); return; }
  }
}

// d, dinv of a complex CSR; flag[0] |= 1 on a zero diagonal; flag[0] |= 2 if
// a row has a column outside its system's row range.
__global__ void k_bd_diag(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                          const double2* __restrict__ val, const int* __restrict__ sys_of_row,
                          const int* __restrict__ sys_begin, const int* __restrict__ sys_end,
                          double2* d, double2* dinv, int* flag) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int s = sys_of_row[i];
  const int lo = sys_begin[s], hi = sys_end[s];
  double2 dd = make_double2(0, 0);
  for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
    const int c = col[p];
    if (c < lo || c >= hi) atomicOr(flag, 2);
    if (c == i) dd = cadd(dd, val[p]);
  }
  if (dd.x == 0 && dd.y == 0) { atomicOr(flag, 1); dinv[i] = make_double2(0, 0); }
  else dinv[i] = cdiv(make_double2(1, 0), dd);
  d[i] = dd;
}

// ----------------------------------------------------------------- host side

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Arena {
  char* base = nullptr;
  size_t off = 0;
  template <class T> T* take(size_t count) {
    T* p = (T*)(base + off);
    off += a256(sizeof(T) * (count > 0 ? count : 1));
    return p;
  }
};

// Workgroups per CU of the persistent kernels (one and two measured the same).
constexpr int kCoopPerCu = 2;
static int coop_grid(const void* kernel, int* grid) {
  int dev = 0, cus = 0, per = 0, coop = 0;
  HK_HIP(hipGetDevice(&dev));
  HK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HK_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  if (!coop) HK_FAIL(HK_EHIP, "device does not support cooperative launches");
  HK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kPB, 0));
  if (per < 1) HK_FAIL(HK_EHIP, "persistent kernel does not fit on a CU");
  *grid = std::min(cus * std::min(per, kCoopPerCu), kBarMaxBlocks);
  // the sweep's row mappings deal rows per XCD: every XCD needs a workgroup
  if (*grid < kXcds) HK_FAIL(HK_EHIP, "persistent grid of %d workgroups is below %d", *grid, kXcds);
  return HK_OK;
}

static void fill_infos(const BatchState& hs, int nsys, hk_solve_info* infos) {
  for (int j = 0; j < nsys; ++j) {
    hk_solve_info& in = infos[j];
    const int s = hs.status[j];
    in.status = s >= B_RUN ? HK_NOT_CONVERGED : s;
    in.breakdown = hs.bd[j];
    in.iters = hs.iters[j];
    const double bb = hs.bb[j];
    in.relres_rec = bb > 0 ? std::sqrt(hs.rr[j] / bb) : std::sqrt(hs.rr[j]);
    in.relres_true = bb > 0 ? std::sqrt(hs.rr_true[j] / bb) : std::sqrt(hs.rr_true[j]);
    in.inner_iters = 0;
  }
}

static int worst_status(const hk_solve_info* infos, int nsys) {
  int w = HK_OK;
  for (int j = 0; j < nsys; ++j) w = std::max(w, infos[j].status);
  return w;
}

// ---------------------------------------------------- batch-plan autotuner
//
// The counterpart of the paper's per-matrix tuning of the GPU grid
// (Section 3, Table 8) for the persistent solvers: on the first solve of a
// batch shape, each candidate launch shape runs the whole persistent kernel
// for kTuneIters iterations (tolerance 0, so every system keeps iterating)
// on the call's own data, timed with HIP events; the fastest is cached by
// (device, n, nnz, longest row, number of systems) and used for the solve
// and for later calls with the same key.  A shape given in opts->shape is
// used as is.  The trial launches write only the call's workspace and x,
// which the solve then starts over.
constexpr int kTuneIters = 4;

using PlanKey = std::tuple<int, int64_t, int64_t, int, int>;
struct PlanCache {
  std::mutex mu;
  std::map<PlanKey, std::array<int, 4>> shapes;
  bool get(const PlanKey& k, std::array<int, 4>* out) {
    std::lock_guard<std::mutex> lock(mu);
    auto it = shapes.find(k);
    if (it == shapes.end()) return false;
    *out = it->second;
    return true;
  }
  void put(const PlanKey& k, const std::array<int, 4>& v) {
    std::lock_guard<std::mutex> lock(mu);
    shapes[k] = v;
  }
};
static PlanCache g_sweep_plans, g_bd_plans;

static void set_shape(hk_solve_info* infos, int nsys, const std::array<int, 4>& sh, int tuned) {
  for (int j = 0; j < nsys; ++j) {
    for (int k = 0; k < 4; ++k) infos[j].shape[k] = sh[k];
    infos[j].shape_tuned = tuned;
    infos[j].pad = 0;
  }
}

// A pair of HIP events around one persistent launch (the trial timings).
struct EventPair {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~EventPair() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
  hipError_t create() {
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    return e;
  }
};

// Sweep shapes: {product form, row mapping, 0, 0} (k_sweep<PF, MAP>).
static const std::array<int, 4> kSweepShapes[] = {{1, 1, 0, 0}, {1, 2, 0, 0}, {1, 3, 0, 0}, {2, 3, 0, 0},
                                                   {3, 1, 0, 0}, {3, 2, 0, 0}};

static const void* sweep_kernel(const std::array<int, 4>& sh) {
  if (sh[2] != 0 || sh[3] != 0) return nullptr;
  if (sh[0] == 1 && sh[1] == 1) return (const void*)k_sweep<1, 1>;
  if (sh[0] == 1 && sh[1] == 2) return (const void*)k_sweep<1, 2>;
  if (sh[0] == 1 && sh[1] == 3) return (const void*)k_sweep<1, 3>;
  if (sh[0] == 2 && sh[1] == 3) return (const void*)k_sweep<2, 3>;
  if (sh[0] == 3 && sh[1] == 1) return (const void*)k_sweep<3, 1>;
  if (sh[0] == 3 && sh[1] == 2) return (const void*)k_sweep<3, 2>;
  return nullptr;
}

// The launch that continues a shape's solve with rpw rows per wave step
// (product form 3), or null.
static const void* sweep_tail_kernel(const std::array<int, 4>& sh, int rpw) {
  if (sh[0] != 3 || sh[2] != 0 || sh[3] != 0) return nullptr;
  if (sh[1] == 1) return rpw == 2 ? (const void*)k_sweep_tail<1, 2> : rpw == 4 ? (const void*)k_sweep_tail<1, 4> : nullptr;
  if (sh[1] == 2) return rpw == 2 ? (const void*)k_sweep_tail<2, 2> : rpw == 4 ? (const void*)k_sweep_tail<2, 4> : nullptr;
  return nullptr;
}

// Block-diagonal shapes: {lanes per row (64: row blocks), rows per block,
// entries per lane per pass, tile rows} (k_blockdiag<L, R, CH>).
static std::vector<std::array<int, 4>> bd_shapes() {
  std::vector<std::array<int, 4>> v;
  for (int tr : {1024, 512}) {
    for (int r : {64, 32, 16})
      for (int ch : {4, 2}) v.push_back({kRowBlockL, r, ch, tr});
    v.push_back({32, 0, 0, tr});
  }
  return v;
}

static const void* bd_kernel(const std::array<int, 4>& sh) {
  if (sh[3] != 512 && sh[3] != 1024) return nullptr;
  if (sh[0] == 32) return sh[1] == 0 && sh[2] == 0 ? (const void*)k_blockdiag<32, 0, 0> : nullptr;
  if (sh[0] != kRowBlockL) return nullptr;
  if (sh[2] == 4) {
    if (sh[1] == 64) return (const void*)k_blockdiag<kRowBlockL, 64, 4>;
    if (sh[1] == 32) return (const void*)k_blockdiag<kRowBlockL, 32, 4>;
    if (sh[1] == 16) return (const void*)k_blockdiag<kRowBlockL, 16, 4>;
  } else if (sh[2] == 2) {
    if (sh[1] == 64) return (const void*)k_blockdiag<kRowBlockL, 64, 2>;
    if (sh[1] == 32) return (const void*)k_blockdiag<kRowBlockL, 32, 2>;
    if (sh[1] == 16) return (const void*)k_blockdiag<kRowBlockL, 16, 2>;
  }
  return nullptr;
}

static bool shape_given(const hk_solve_opts* o) {
  return o->shape[0] || o->shape[1] || o->shape[2] || o->shape[3];
}

}  // namespace hk

using namespace hk;

extern "C" int hk_sweep_solve(int64_t n, int64_t nnz, const int32_t* d_rowptr, const int32_t* d_col,
                              const double* d_K, const double* d_M, int32_t nsys,
                              const double* kappa, const void* d_B, void* d_X,
                              const hk_solve_opts* opts, hk_solve_info* infos, void* stream) {
  if (!d_rowptr || !d_col || !d_K || !d_M || !kappa || !d_B || !d_X || !opts || !infos)
    HK_FAIL(HK_EINVAL, "hk_sweep_solve: null argument");
  if (nsys < 1 || nsys > kSys) HK_FAIL(HK_EINVAL, "hk_sweep_solve: nsys must be in [1, 64]");
  if (n < 1 || nnz < 1) HK_FAIL(HK_EINVAL, "hk_sweep_solve: empty matrix (n=%lld nnz=%lld)", (long long)n, (long long)nnz);
  if (!(opts->tol >= 0) || opts->max_iter < 0) HK_FAIL(HK_EINVAL, "hk_sweep_solve: bad options");
  if (opts->flags) HK_FAIL(HK_EINVAL, "hk_sweep_solve: no flags apply");
  std::array<int, 4> forced{opts->shape[0], opts->shape[1], opts->shape[2], opts->shape[3]};
  if (shape_given(opts) && !sweep_kernel(forced))
    HK_FAIL(HK_EINVAL, "hk_sweep_solve: unknown shape {%d, %d, %d, %d}", forced[0], forced[1], forced[2], forced[3]);
  hipStream_t s = as_stream(stream);
  // structure check through a temporary handle (real values are not read),
  // which also finds the longest row (part of the plan key)
  hk_csr A = nullptr;
  int rc = hk_csr_create(&A, n, nnz, d_rowptr, d_col, d_K, HK_C128, HK_INT32_COLS, stream);
  if (rc != HK_OK) return rc;
  const int max_row = A->max_row;
  (void)hk_csr_destroy(A);
  int dev = 0;
  HK_HIP(hipGetDevice(&dev));
  // the largest grid of any candidate sizes the partials
  int gmax = 0;
  for (const auto& sh : kSweepShapes) {
    for (const void* k : {sweep_kernel(sh), sweep_tail_kernel(sh, 2), sweep_tail_kernel(sh, 4)}) {
      if (!k) continue;
      int g = 0;
      rc = coop_grid(k, &g);
      if (rc != HK_OK) return rc;
      gmax = std::max(gmax, g);
    }
  }
  const size_t vec = (size_t)n * kSys;
  Arena ar;
  const size_t bytes = 6 * a256(16 * vec) + 2 * a256(8 * n) + a256(16 * kSys) +
                       a256(8 * 4 * (size_t)gmax * kSys) + a256(sizeof(BatchState)) + a256(sizeof(GridBar)) +
                       a256(8 * 4 * (size_t)kXcds * kSys) + a256(64);
  if (hipMalloc((void**)&ar.base, bytes) != hipSuccess) HK_FAIL(HK_ENOMEM, "hk_sweep_solve: hipMalloc(%zu)", bytes);
  SweepArgs a{};
  a.n = (int)n; a.nsys = nsys; a.rowptr = d_rowptr; a.col = d_col; a.K = d_K; a.M = d_M;
  a.R = ar.take<double2>(vec); a.RH = ar.take<double2>(vec); a.PH = ar.take<double2>(vec);
  a.V = ar.take<double2>(vec); a.SH = ar.take<double2>(vec); a.T = ar.take<double2>(vec);
  double* kd = ar.take<double>(n);
  double* md = ar.take<double>(n);
  double2* kap = ar.take<double2>(kSys);
  a.partials = ar.take<double>(4 * (size_t)gmax * kSys);
  a.st = ar.take<BatchState>(1);
  a.bar = ar.take<GridBar>(1);
  // per-XCD-group sums of the reducing barriers
  double* gpart = ar.take<double>(4 * (size_t)kXcds * kSys);
  int* flag = ar.take<int>(16);
  if (ar.off > bytes) {
    (void)hipFree(ar.base);
    HK_FAIL(HK_EINVAL, "hk_sweep_solve: workspace layout exceeds its allocation");
  }
  a.kd = kd; a.md = md; a.kap = kap;
  a.B = (const double2*)d_B; a.X = (double2*)d_X;
  std::vector<double2> hk(kSys, make_double2(0, 0));
  for (int j = 0; j < nsys; ++j) hk[j] = make_double2(kappa[2 * j], kappa[2 * j + 1]);
  int hflag = 0;
  hipError_t e = hipMemcpyAsync(kap, hk.data(), 16 * kSys, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(flag, 0, 64, s);
  const dim3 ew((unsigned)((n + kBlock - 1) / kBlock));
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_real_diag, ew, dim3(kBlock), 0, s, (int)n, d_rowptr, d_col, d_K, d_M, kd, md);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_sweep_diag_check, ew, dim3(kBlock), 0, s, (int)n, nsys, kd, md, kap, flag);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(ar.base);
    HK_FAIL(HK_EHIP, "hk_sweep_solve: %s", hipGetErrorString(e));
  }
  if (hflag) {
    (void)hipFree(ar.base);
    HK_FAIL(HK_EINVAL, "hk_sweep_solve: zero diagonal entry for some system (Jacobi undefined)");
  }
  const unsigned long long spin = barrier_spin_limit();
  // one persistent launch of shape sh: fresh state and barrier, then the kernel
  // (with events: recorded around the kernel alone)
  auto launch = [&](const std::array<int, 4>& sh, double tol, long long maxit, EventPair* ev) -> hipError_t {
    const void* kern = sweep_kernel(sh);
    int grid = 0;
    if (coop_grid(kern, &grid) != HK_OK) return hipErrorInvalidConfiguration;
    a.tol = tol;
    a.maxit = maxit;
    // the tuner's trials (every system running) stay in one launch
    a.tail = !ev && sweep_tail_kernel(sh, 2) ? 1 : 0;
    GridBar bar0{};
    bar0.spin_limit = spin;
    bar0.gpart = gpart;
    // barrier stamps for the solve itself, not for the tuner's trials
    bar0.stamps = ev ? nullptr : opts->d_history;
    bar0.nstamps = bar0.stamps ? 8ull * ((unsigned long long)maxit + 1) : 0;
    hipError_t e2 = hipMemcpyAsync(a.bar, &bar0, sizeof(GridBar), hipMemcpyHostToDevice, s);
    if (e2 == hipSuccess) e2 = hipMemsetAsync(a.st, 0, sizeof(BatchState), s);
    if (e2 == hipSuccess && ev) e2 = hipEventRecord(ev->e0, s);
    void* args[] = {&a};
    if (e2 == hipSuccess) e2 = hipLaunchCooperativeKernel(kern, dim3(grid), dim3(kPB), args, 0, s);
    if (e2 == hipSuccess && ev) e2 = hipEventRecord(ev->e1, s);
    // bar0 lives on this frame: the copy must be done before it goes
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
    // at most 32 (then 16) systems left: the multi-row launches continue
    for (int stage = 1; e2 == hipSuccess && a.tail; ) {
      BatchState hs{};
      GridBar hb{};
      e2 = hipMemcpyAsync(&hs, a.st, sizeof(hs), hipMemcpyDeviceToHost, s);
      if (e2 == hipSuccess) e2 = hipMemcpyAsync(&hb, a.bar, sizeof(hb), hipMemcpyDeviceToHost, s);
      if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
      if (e2 != hipSuccess || hb.abort || hs.handoff <= stage || hs.running <= 0) break;
      const void* tail = sweep_tail_kernel(sh, hs.handoff);
      int grid2 = 0;
      if (!tail || coop_grid(tail, &grid2) != HK_OK) return hipErrorInvalidConfiguration;
      GridBar bar1{};
      bar1.spin_limit = spin;
      bar1.gpart = gpart;
      bar1.stamps = bar0.stamps;
      bar1.nstamps = bar0.nstamps;
      e2 = hipMemcpyAsync(a.bar, &bar1, sizeof(GridBar), hipMemcpyHostToDevice, s);
      if (e2 == hipSuccess) e2 = hipLaunchCooperativeKernel(tail, dim3(grid2), dim3(kPB), args, 0, s);
      if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
      stage = hs.handoff;
    }
    return e2;
  };
  auto aborted = [&](bool* ab) -> hipError_t {
    GridBar hb{};
    hipError_t e2 = hipMemcpyAsync(&hb, a.bar, sizeof(hb), hipMemcpyDeviceToHost, s);
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
    *ab = hb.abort != 0;
    return e2;
  };
  std::array<int, 4> shape = forced;
  int tuned = 0;
  const PlanKey key{dev, n, nnz, max_row, nsys};
  if (!shape_given(opts)) {
    tuned = 1;
    if (!g_sweep_plans.get(key, &shape)) {
      float best = -1;
      EventPair ev;
      e = ev.create();
      for (const auto& sh : kSweepShapes) {
        float ms = -1;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
          float t = 0;
          e = launch(sh, 0.0, kTuneIters, &ev);
          if (e == hipSuccess) e = hipEventElapsedTime(&t, ev.e0, ev.e1);
          ms = rep == 0 ? t : std::min(ms, t);
        }
        bool ab = false;
        if (e == hipSuccess) e = aborted(&ab);
        if (e != hipSuccess || ab) {
          (void)hipFree(ar.base);
          if (ab) HK_FAIL(HK_EHIP, "hk_sweep_solve: grid barrier timed out");
          HK_FAIL(HK_EHIP, "hk_sweep_solve: trial launch: %s", hipGetErrorString(e));
        }
        if (best < 0 || ms < best) {
          best = ms;
          shape = sh;
        }
      }
      g_sweep_plans.put(key, shape);
    }
  }
  e = launch(shape, opts->tol, opts->max_iter, nullptr);
  BatchState hs{};
  GridBar hb{};
  if (e == hipSuccess) e = hipMemcpyAsync(&hs, a.st, sizeof(hs), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&hb, a.bar, sizeof(hb), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(ar.base);
  if (e != hipSuccess) HK_FAIL(HK_EHIP, "hk_sweep_solve: %s", hipGetErrorString(e));
  if (hb.abort) HK_FAIL(HK_EHIP, "hk_sweep_solve: grid barrier timed out");
  fill_infos(hs, nsys, infos);
  set_shape(infos, nsys, shape, tuned);
  return worst_status(infos, nsys);
}

extern "C" int hk_blockdiag_solve(hk_csr A, int32_t nsys, const int64_t* row_off, const void* d_b,
                                  void* d_x, const hk_solve_opts* opts, hk_solve_info* infos,
                                  void* stream) {
  if (!A || !row_off || !d_b || !d_x || !opts || !infos) HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: null argument");
  if (A->dtype != HK_C128) HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: matrix must be complex128");
  if (nsys < 1 || nsys > kSys) HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: nsys must be in [1, 64]");
  if (!(opts->tol >= 0) || opts->max_iter < 0) HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: bad options");
  if (opts->flags) HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: no flags apply");
  if (row_off[0] != 0 || row_off[nsys] != A->n) HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: row offsets must span [0, n]");
  for (int k = 0; k < nsys; ++k)
    if (row_off[k + 1] <= row_off[k]) HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: empty or decreasing system %d", k);
  std::array<int, 4> forced{opts->shape[0], opts->shape[1], opts->shape[2], opts->shape[3]};
  if (shape_given(opts) && !bd_kernel(forced))
    HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: unknown shape {%d, %d, %d, %d}", forced[0], forced[1], forced[2], forced[3]);
  hipStream_t s = as_stream(stream);
  const std::vector<std::array<int, 4>> cands = bd_shapes();
  int dev = 0;
  HK_HIP(hipGetDevice(&dev));
  int gmax = 0;
  for (const auto& sh : cands) {
    int g = 0;
    int rc = coop_grid(bd_kernel(sh), &g);
    if (rc != HK_OK) return rc;
    gmax = std::max(gmax, g);
  }
  std::vector<int> sys_end(kSys, 0), sys_begin(kSys, 0);
  std::vector<int> sys_of_row((size_t)A->n);
  for (int k = 0; k < nsys; ++k) {
    sys_begin[k] = (int)row_off[k];
    sys_end[k] = (int)row_off[k + 1];
    for (int64_t r = row_off[k]; r < row_off[k + 1]; ++r) sys_of_row[r] = k;
  }
  // static tiles of tile_rows rows that never straddle systems; the arrays
  // are sized for the smallest tiles
  int nt_max = 0;
  for (int k = 0; k < nsys; ++k) nt_max += (int)((row_off[k + 1] - row_off[k] + 511) / 512);
  const int64_t n = A->n;
  Arena ar;
  const size_t bytes = 8 * a256(16 * (size_t)n) + 3 * a256(4 * (size_t)nt_max) +
                       a256(4 * (size_t)n) + 4 * a256(4 * (kSys + 1)) + a256(8 * 4 * (size_t)gmax * kSys) +
                       a256(sizeof(BatchState)) + a256(sizeof(GridBar)) + a256(8 * 4 * (size_t)kXcds * kSys) +
                       a256(64);
  if (hipMalloc((void**)&ar.base, bytes) != hipSuccess) HK_FAIL(HK_ENOMEM, "hk_blockdiag_solve: hipMalloc(%zu)", bytes);
  BdArgs a{};
  a.n = (int)n; a.nsys = nsys; a.rowptr = A->rowptr; a.col = A->col;
  a.val = (const double2*)A->val;
  a.R = ar.take<double2>(n); a.RH = ar.take<double2>(n); a.PH = ar.take<double2>(n);
  a.V = ar.take<double2>(n); a.SH = ar.take<double2>(n); a.T = ar.take<double2>(n);
  double2* d = ar.take<double2>(n);
  double2* dinv = ar.take<double2>(n);
  a.act_sys = ar.take<int>(nt_max);
  a.act_row0 = ar.take<int>(nt_max);
  a.act_end = ar.take<int>(nt_max);
  int* d_sor = ar.take<int>(n);
  int* d_send = ar.take<int>(kSys + 1);
  int* d_sbeg = ar.take<int>(kSys + 1);
  int* d_t0 = ar.take<int>(kSys + 1);
  (void)ar.take<int>(kSys + 1);
  a.partials = ar.take<double>(4 * (size_t)gmax * kSys);
  a.st = ar.take<BatchState>(1);
  a.bar = ar.take<GridBar>(1);
  double* gpart = ar.take<double>(4 * (size_t)kXcds * kSys);
  int* flag = ar.take<int>(16);
  if (ar.off > bytes) {
    (void)hipFree(ar.base);
    HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: workspace layout exceeds its allocation");
  }
  a.d = d; a.dinv = dinv; a.sys_begin = d_sbeg; a.sys_end = d_send; a.sys_tile0 = d_t0;
  a.B = (const double2*)d_b; a.X = (double2*)d_x;
  int hflag = 0;
  hipError_t e = hipMemcpyAsync(d_sor, sys_of_row.data(), 4 * (size_t)n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_send, sys_end.data(), 4 * kSys, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_sbeg, sys_begin.data(), 4 * kSys, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(flag, 0, 64, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_bd_diag, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, (int)n,
                       A->rowptr, A->col, (const double2*)A->val, d_sor, d_sbeg, d_send, d, dinv, flag);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host vectors above go out of scope
  if (e != hipSuccess) {
    (void)hipFree(ar.base);
    HK_FAIL(HK_EHIP, "hk_blockdiag_solve: %s", hipGetErrorString(e));
  }
  if (hflag) {
    (void)hipFree(ar.base);
    if (hflag & 2) HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: matrix is not block-diagonal for the given offsets");
    HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: zero diagonal entry (Jacobi undefined)");
  }
  const unsigned long long spin = barrier_spin_limit();
  // one persistent launch of shape sh: its static tile table (the start
  // phase walks every tile), fresh state and barrier, then the kernel
  auto launch = [&](const std::array<int, 4>& sh, double tol, long long maxit, EventPair* ev) -> hipError_t {
    const void* kern = bd_kernel(sh);
    int grid = 0;
    if (coop_grid(kern, &grid) != HK_OK) return hipErrorInvalidConfiguration;
    const int tr = sh[3];
    std::vector<int> tsys, trow, tend, tile0(kSys + 1, 0);
    for (int k = 0; k < nsys; ++k) {
      tile0[k] = (int)tsys.size();
      for (int64_t r = row_off[k]; r < row_off[k + 1]; r += tr) {
        tsys.push_back(k);
        trow.push_back((int)r);
        tend.push_back((int)std::min<int64_t>(r + tr, row_off[k + 1]));
      }
    }
    const int nt = (int)tsys.size();
    for (int k = nsys; k <= kSys; ++k) tile0[k] = nt;
    a.L = sh[0];
    a.tile_rows = tr;
    a.tol = tol;
    a.maxit = maxit;
    BatchState init{};
    init.ntiles_active = nt;
    GridBar bar0{};
    bar0.spin_limit = spin;
    bar0.gpart = gpart;
    // barrier stamps for the solve itself, not for the tuner's trials
    bar0.stamps = ev ? nullptr : opts->d_history;
    bar0.nstamps = bar0.stamps ? 8ull * ((unsigned long long)maxit + 1) : 0;
    hipError_t e2 = hipMemcpyAsync(a.act_sys, tsys.data(), 4 * (size_t)nt, hipMemcpyHostToDevice, s);
    if (e2 == hipSuccess) e2 = hipMemcpyAsync(a.act_row0, trow.data(), 4 * (size_t)nt, hipMemcpyHostToDevice, s);
    if (e2 == hipSuccess) e2 = hipMemcpyAsync(a.act_end, tend.data(), 4 * (size_t)nt, hipMemcpyHostToDevice, s);
    if (e2 == hipSuccess) e2 = hipMemcpyAsync(d_t0, tile0.data(), 4 * (kSys + 1), hipMemcpyHostToDevice, s);
    if (e2 == hipSuccess) e2 = hipMemcpyAsync(a.bar, &bar0, sizeof(GridBar), hipMemcpyHostToDevice, s);
    if (e2 == hipSuccess) e2 = hipMemcpyAsync(a.st, &init, sizeof(init), hipMemcpyHostToDevice, s);
    if (e2 == hipSuccess && ev) e2 = hipEventRecord(ev->e0, s);
    void* args[] = {&a};
    if (e2 == hipSuccess) e2 = hipLaunchCooperativeKernel(kern, dim3(grid), dim3(kPB), args, 0, s);
    if (e2 == hipSuccess && ev) e2 = hipEventRecord(ev->e1, s);
    // the host tables live on this frame: the copies must be done before they go
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
    return e2;
  };
  auto aborted = [&](bool* ab) -> hipError_t {
    GridBar hb{};
    hipError_t e2 = hipMemcpyAsync(&hb, a.bar, sizeof(hb), hipMemcpyDeviceToHost, s);
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
    *ab = hb.abort != 0;
    return e2;
  };
  std::array<int, 4> shape = forced;
  int tuned = 0;
  const PlanKey key{dev, n, A->nnz, A->max_row, nsys};
  if (!shape_given(opts)) {
    tuned = 1;
    if (!g_bd_plans.get(key, &shape)) {
      float best = -1;
      EventPair ev;
      e = ev.create();
      for (const auto& sh : cands) {
        float ms = -1;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
          float t = 0;
          e = launch(sh, 0.0, kTuneIters, &ev);
          if (e == hipSuccess) e = hipEventElapsedTime(&t, ev.e0, ev.e1);
          ms = rep == 0 ? t : std::min(ms, t);
        }
        bool ab = false;
        if (e == hipSuccess) e = aborted(&ab);
        if (e != hipSuccess || ab) {
          (void)hipFree(ar.base);
          if (ab) HK_FAIL(HK_EHIP, "hk_blockdiag_solve: grid barrier timed out");
          HK_FAIL(HK_EHIP, "hk_blockdiag_solve: trial launch: %s", hipGetErrorString(e));
        }
        if (best < 0 || ms < best) {
          best = ms;
          shape = sh;
        }
      }
      g_bd_plans.put(key, shape);
    }
  }
  e = launch(shape, opts->tol, opts->max_iter, nullptr);
  BatchState hs{};
  GridBar hb{};
  if (e == hipSuccess) e = hipMemcpyAsync(&hs, a.st, sizeof(hs), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&hb, a.bar, sizeof(hb), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(ar.base);
  if (e != hipSuccess) HK_FAIL(HK_EHIP, "hk_blockdiag_solve: %s", hipGetErrorString(e));
  if (hb.abort) HK_FAIL(HK_EHIP, "hk_blockdiag_solve: grid barrier timed out");
  fill_infos(hs, nsys, infos);
  set_shape(infos, nsys, shape, tuned);
  return worst_status(infos, nsys);
}
