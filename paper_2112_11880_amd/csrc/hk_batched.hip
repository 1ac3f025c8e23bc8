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
  int pad;
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

// Second stage: out[k] (valid in threads 0..63, thread j = system j) = sum
// over workgroups in a fixed order.  Thread (g, j) sums workgroups g, g +
// kPW, g + 2 kPW, ... in that order; the loads of kFinBatch of them (for all
// NV sums) are issued before any is added, since the partials come from
// memory after the barrier's acquire and a load-add chain would wait out
// every load in turn.
constexpr int kFinBatch = 8;
template <int NV>
__device__ __forceinline__ void final_partials64(const double* partials, double (&out)[NV], double* lds) {
  const int j = threadIdx.x & 63, g = threadIdx.x >> 6, G = gridDim.x;
  double s[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) s[k] = 0;
  for (int b0 = g; b0 < G; b0 += kFinBatch * kPW) {
    double v[NV][kFinBatch];
#pragma unroll
    for (int u = 0; u < kFinBatch; ++u) {
      const int b = b0 + u * kPW < G ? b0 + u * kPW : b0;
#pragma unroll
      for (int k = 0; k < NV; ++k) v[k][u] = partials[((size_t)k * G + b) * kSys + j];
    }
#pragma unroll
    for (int u = 0; u < kFinBatch; ++u)
      if (b0 + u * kPW < G) {
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k] += v[k][u];
      }
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) lds[(k * kPW + g) * kSys + j] = s[k];
  __syncthreads();
  if (threadIdx.x < kSys) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0;
      for (int u = 0; u < kPW; ++u) s += lds[(k * kPW + u) * kSys + j];
      out[k] = s;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ double2 crecip(double2 d) { return cdiv(make_double2(1.0, 0.0), d); }

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
    dst[o] = acc;
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

// Rows r0, r0 + rs, ... < r1 of the calling wave.  XCD x (the workgroups b
// with b % 8 == x) owns a contiguous eighth of the rows and its waves take
// them round-robin, so each XCD advances through its eighth as one front and
// the x[col] gathers of neighbouring rows meet in its L2.  On the 48^3 sweep
// this measured 902 us per iteration against 948 us for one contiguous row
// range per wave and 906 us for waves round-robin over all rows.
__device__ __forceinline__ void sweep_rows(int n, int G, int& r0, int& r1, int& rs) {
  const int w = threadIdx.x >> 6;
  const int x = blockIdx.x % kXcds, i = blockIdx.x / kXcds;
  const int nbx = (G - x + kXcds - 1) / kXcds;  // workgroups on XCD x
  const int X0 = (int)(((long long)x * n) / kXcds), X1 = (int)(((long long)(x + 1) * n) / kXcds);
  r0 = X0 + i * kPW + w;
  r1 = X1;
  rs = nbx * kPW;
}

__global__ __launch_bounds__(kPB) void k_sweep(SweepArgs a) {
  __shared__ double lds[4 * kPW * kSys];
  unsigned epoch = 0;
  BatchState* st = a.st;
  const int j = threadIdx.x & 63;
  const int G = gridDim.x;
  int r0, r1, rs;
  sweep_rows(a.n, G, r0, r1, rs);
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
    if (barrier_last(a.bar, epoch, [&] {
          double tot[1];
          final_partials64<1>(a.partials, tot, lds);
          if (threadIdx.x < kSys) {
            if (threadIdx.x < a.nsys) init_sys(st, threadIdx.x, tot[0], a.tol, a.maxit);
            else st->status[threadIdx.x] = HK_OK;
          }
          if (threadIdx.x == 0) { st->iter = 1; st->maxit = a.maxit; st->changed = 0; }
          __syncthreads();
          if (threadIdx.x == 0) {
            int run = 0;
            for (int u = 0; u < a.nsys; ++u) run += st->status[u] == B_RUN;
            st->running = run;
          }
        }))
      return;
  }

  while (st->running > 0) {
    const long long it = st->iter;
    bool act = lane_ok && st->status[j] == B_RUN;
    // ---- phat = D^-1 (r - beta omega v) + beta phat
    if (it > 1) {
      const double2 beta = st->beta[j], bo = cmul(st->beta[j], st->omega[j]);
      if (act) {
        int row = r0;
        for (; row + 3 * rs < r1; row += 4 * rs) {
          double2 rv[4], vv[4], pv[4], dv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const size_t o = (size_t)(row + u * rs) * kSys + j;
            rv[u] = a.R[o]; vv[u] = a.V[o]; pv[u] = a.PH[o]; dv[u] = sweep_diag(a, row + u * rs, kap);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            a.PH[(size_t)(row + u * rs) * kSys + j] = cfma(beta, pv[u], cmul(crecip(dv[u]), csub(rv[u], cmul(bo, vv[u]))));
        }
        for (; row < r1; row += rs) {
          const size_t o = (size_t)row * kSys + j;
          const double2 w = csub(a.R[o], cmul(bo, a.V[o]));
          a.PH[o] = cfma(beta, a.PH[o], cmul(crecip(sweep_diag(a, row, kap)), w));
        }
      }
      if (barrier_last(a.bar, epoch, [] {})) return;
    }
    // ---- v = A phat ; sigma = rhat^H v
    {
      double part[2] = {0, 0};
      sweep_spmv<1, 2>(a, r0, r1, rs, a.PH, a.V, act, kap, part);
      store_partials64<2>(part, a.partials, lds);
      if (barrier_last(a.bar, epoch, [&] {
            double tot[2];
            final_partials64<2>(a.partials, tot, lds);
            if (threadIdx.x < a.nsys) upd_sigma(st, threadIdx.x, make_double2(tot[0], tot[1]));
          }))
        return;
    }
    act = lane_ok && st->status[j] == B_RUN;
    // ---- s = r - alpha v ; shat = D^-1 s ; ||s||^2
    {
      double part[1] = {0};
      const double2 alpha = st->alpha[j];
      if (act) {
        int row = r0;
        for (; row + 3 * rs < r1; row += 4 * rs) {
          double2 rv[4], vv[4], dv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const size_t o = (size_t)(row + u * rs) * kSys + j;
            rv[u] = a.R[o]; vv[u] = a.V[o]; dv[u] = sweep_diag(a, row + u * rs, kap);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const double2 s = csub(rv[u], cmul(alpha, vv[u]));
            a.SH[(size_t)(row + u * rs) * kSys + j] = cmul(crecip(dv[u]), s);
            part[0] += cabs2(s);
          }
        }
        for (; row < r1; row += rs) {
          const size_t o = (size_t)row * kSys + j;
          const double2 s = csub(a.R[o], cmul(alpha, a.V[o]));
          a.SH[o] = cmul(crecip(sweep_diag(a, row, kap)), s);
          part[0] += cabs2(s);
        }
      }
      store_partials64<1>(part, a.partials, lds);
      if (barrier_last(a.bar, epoch, [&] {
            double tot[1];
            final_partials64<1>(a.partials, tot, lds);
            if (threadIdx.x < a.nsys) upd_s(st, threadIdx.x, tot[0]);
          }))
        return;
    }
    act = lane_ok && st->status[j] == B_RUN;
    // ---- t = A shat ; tau = t^H t ; t^H s
    {
      double part[3] = {0, 0, 0};
      sweep_spmv<2, 3>(a, r0, r1, rs, a.SH, a.T, act, kap, part);
      store_partials64<3>(part, a.partials, lds);
      if (barrier_last(a.bar, epoch, [&] {
            double tot[3];
            final_partials64<3>(a.partials, tot, lds);
            if (threadIdx.x < a.nsys) upd_omega(st, threadIdx.x, tot[0], make_double2(tot[1], tot[2]));
          }))
        return;
    }
    // ---- x += alpha phat + omega shat ; r = s - omega t ; ||r||^2 ; rhat^H r
    {
      const int sj = lane_ok ? st->status[j] : HK_OK;
      double part[3] = {0, 0, 0};
      const double2 alpha = st->alpha[j], omega = st->omega[j];
      if (sj == B_RUN) {
        auto upd = [&](int row, double2 sh, double2 ph, double2 xv, double2 tv, double2 h, double2 d) {
          const size_t o = (size_t)row * kSys + j;
          a.X[o] = cfma(omega, sh, cfma(alpha, ph, xv));
          const double2 r = csub(cmul(d, sh), cmul(omega, tv));
          a.R[o] = r;
          part[0] += cabs2(r);
          part[1] = fma(h.x, r.x, fma(h.y, r.y, part[1]));
          part[2] = fma(h.x, r.y, fma(-h.y, r.x, part[2]));
        };
        int row = r0;
        for (; row + rs < r1; row += 2 * rs) {
          double2 sh[2], ph[2], xv[2], tv[2], hv[2], dv[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const size_t o = (size_t)(row + u * rs) * kSys + j;
            sh[u] = a.SH[o]; ph[u] = a.PH[o]; xv[u] = a.X[o]; tv[u] = a.T[o]; hv[u] = a.RH[o];
            dv[u] = sweep_diag(a, row + u * rs, kap);
          }
#pragma unroll
          for (int u = 0; u < 2; ++u) upd(row + u * rs, sh[u], ph[u], xv[u], tv[u], hv[u], dv[u]);
        }
        for (; row < r1; row += rs) {
          const size_t o = (size_t)row * kSys + j;
          upd(row, a.SH[o], a.PH[o], a.X[o], a.T[o], a.RH[o], sweep_diag(a, row, kap));
        }
      } else if (sj == B_HALF || sj == B_TAUBD) {
        for (int row = r0; row < r1; row += rs) {
          const size_t o = (size_t)row * kSys + j;
          a.X[o] = cfma(alpha, a.PH[o], a.X[o]);
        }
      }
      store_partials64<3>(part, a.partials, lds);
      if (barrier_last(a.bar, epoch, [&] {
            double tot[3];
            final_partials64<3>(a.partials, tot, lds);
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
          }))
        return;
    }
  }
  // ---- true residual ||b - A x||^2 per system
  {
    double part[1] = {0};
    sweep_spmv<3, 1>(a, r0, r1, rs, a.X, nullptr, lane_ok, kap, part);
    store_partials64<1>(part, a.partials, lds);
    barrier_last(a.bar, epoch, [&] {
      double tot[1];
      final_partials64<1>(a.partials, tot, lds);
      if (threadIdx.x < a.nsys) st->rr_true[threadIdx.x] = tot[0];
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
  // min(act_row0[t] + kPB, act_end[t]) - 1 of system act_sys[t]
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

// Flush the workgroup's running sums of the current system into the LDS
// per-system accumulators (thread 0 adds; uniform call).
template <int NV>
__device__ __forceinline__ void bd_flush(double (&acc)[NV], int sys, double* red, double* sysacc) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = wave_sum(acc[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k * kPW + w] = acc[k];
  }
  __syncthreads();
  if (threadIdx.x == 0 && sys >= 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0;
      for (int u = 0; u < kPW; ++u) s += red[k * kPW + u];
      sysacc[k * kSys + sys] += s;
    }
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0;
}

// A tile of the active list as the phases see it, and the per-system
// scalars the phases read, both staged in LDS at the start of a phase.
struct BdTile {
  int row0, end, sys;
};
constexpr int kBdTileBatch = 64;  // active tiles staged in LDS at a time
struct BdShared {
  int tsys[kBdTileBatch], trow0[kBdTileBatch], tend[kBdTileBatch];
  double2 alpha[kSys], omega[kSys], beta[kSys];
  int status[kSys];
};

// Walk this workgroup's share of the active tiles: f(tile, acc) for each,
// with the metadata of up to kBdTileBatch tiles and every system's scalars
// loaded into LDS together (one round of loads instead of a dependent chain
// per tile); per-system sums end in partials[(k*G + block)*64 + sys].
template <int NV, class F>
__device__ __forceinline__ void bd_phase(const BdArgs& a, double* lds, BdShared& sh, F&& f) {
  double* red = lds;                    // NV * kPW
  double* sysacc = lds + 4 * kPW;       // NV * 64
  const int G = gridDim.x;
  const int lb = xcd_block(blockIdx.x, G);
  const BatchState* st = a.st;
  const int na = st->ntiles_active;
  const int t0 = (int)(((long long)lb * na) / G), t1 = (int)(((long long)(lb + 1) * na) / G);
  for (int k = threadIdx.x; k < NV * kSys; k += kPB) sysacc[k] = 0;
  if (threadIdx.x < a.nsys) {
    const int j = threadIdx.x;
    sh.alpha[j] = st->alpha[j];
    sh.omega[j] = st->omega[j];
    sh.beta[j] = st->beta[j];
    sh.status[j] = st->status[j];
  }
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0;
  int cur = -1;
  for (int c = t0; c < t1; c += kBdTileBatch) {
    const int cnt = t1 - c < kBdTileBatch ? t1 - c : kBdTileBatch;
    __syncthreads();  // the previous batch is done with the staged tiles
    if (threadIdx.x >= kSys && threadIdx.x < kSys + cnt) {
      const int t = c + threadIdx.x - kSys;
      sh.tsys[t - c] = a.act_sys[t];
      sh.trow0[t - c] = a.act_row0[t];
      sh.tend[t - c] = a.act_end[t];
    }
    __syncthreads();
    for (int k = 0; k < cnt; ++k) {
      const BdTile tile{sh.trow0[k], sh.tend[k], sh.tsys[k]};
      if (tile.sys != cur) {
        if (cur >= 0) bd_flush<NV>(acc, cur, red, sysacc);
        cur = tile.sys;
      }
      f(tile, acc);
    }
  }
  bd_flush<NV>(acc, cur, red, sysacc);
  __syncthreads();
  for (int k = threadIdx.x; k < NV * kSys; k += kPB) {
    const int kk = k / kSys, s = k % kSys;
    a.partials[((size_t)kk * G + blockIdx.x) * kSys + s] = sysacc[k];
  }
}

// Row sums of the kPB rows of a tile, kPB / L rows at a time (one L-lane
// group per row); each sum goes to callback g(row, acc) on the group's
// first lane.
template <int L, class G2>
__device__ __forceinline__ void bd_tile_spmv(const BdArgs& a, const BdTile& tile, const double2* src, G2&& g) {
  const int grp = threadIdx.x / L, lane = threadIdx.x & (L - 1);
  const int end = tile.end;
  const int base = tile.row0;
  for (int sub = 0; sub < L; ++sub) {
    const int row = base + sub * (kPB / L) + grp;
    if (base + sub * (kPB / L) >= end) break;
    double2 acc[1];
    csr_rows<L, 1, double2>(row, end, a.rowptr, a.col, a.val, src, acc);
    if (lane == 0 && row < end) g(row, acc[0]);
  }
}

// Row-block variant: wave w of the workgroup owns rows trow + 64 w ..
// trow + 64 w + 63 of the tile (kPW waves x 64 rows = one tile) and streams
// their entries with all its lanes (csr_block_rows); each row's sum goes to
// callback g(row, acc) in the lane that owns the row.  `stage` is the
// workgroup's staging area (kPW slices of kBdCh * 64 products).
constexpr int kBdCh = 4;  // entries per lane per pass: 8 needs more than the 128 VGPRs of a 1024-thread workgroup
template <class G2>
__device__ __forceinline__ void bd_tile_spmv_rb(const BdArgs& a, const BdTile& tile, const double2* src,
                                                double2* stage, G2&& g) {
  const int end = tile.end;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int r0 = tile.row0 + w * 64;
  if (r0 >= end) return;  // uniform across the wave
  const double2 acc = csr_block_rows<64, kBdCh, double2, int>(r0, end, a.rowptr, a.col, a.val, src,
                                                              stage + w * kBdCh * kWave);
  if (r0 + l < end) g(r0 + l, acc);
}

// L in {4, 8, 16, 32}: lane-group tile products; L == kRowBlockL: row blocks.
template <int L>
__global__ __launch_bounds__(kPB) void k_blockdiag(BdArgs a) {
  // [4 kPW] wave sums | [4 kSys] per-system sums | scratch shared by the
  // barrier callbacks (4 kPW kSys doubles) and the row-block staging area,
  // which are never live at the same time
  constexpr int kFin = 4 * kPW * kSys;
  constexpr int kStage = L == kRowBlockL ? kPW * kBdCh * kWave * 2 : 0;
  __shared__ __align__(16) double lds[4 * kPW + 4 * kSys + (kFin > kStage ? kFin : kStage)];
  unsigned epoch = 0;
  double* fin = lds + 4 * kPW + 4 * kSys;
  double2* stage = reinterpret_cast<double2*>(fin);
  __shared__ BdShared sh;
  BatchState* st = a.st;
  auto tile_spmv = [&](const BdTile& tile, const double2* src, auto&& g) {
    if constexpr (L == kRowBlockL) bd_tile_spmv_rb(a, tile, src, stage, g);
    else bd_tile_spmv<L>(a, tile, src, g);
  };
  // the row of the calling thread in an element-wise phase (one per thread), or -1
  auto my_row = [](const BdTile& tile) {
    const int row = tile.row0 + (int)threadIdx.x;
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
      const int r0 = a.sys_begin[q], end = a.sys_end[q];
      for (int k = threadIdx.x; k < cnt; k += kPB) {
        a.act_sys[base + k] = q;
        a.act_row0[base + k] = r0 + k * kPB;
        a.act_end[base + k] = end;
      }
    }
  };

  // ---- start: r = rhat = b, phat = D^-1 b, x = 0 (all tiles are active)
  bd_phase<1>(a, lds, sh, [&](const BdTile& tile, double(&acc)[1]) {
    const int row = my_row(tile);
    if (row >= 0) {
      const double2 b = a.B[row];
      a.R[row] = b; a.RH[row] = b; a.PH[row] = cmul(a.dinv[row], b); a.X[row] = make_double2(0, 0);
      acc[0] += cabs2(b);
    }
  });
  if (barrier_last(a.bar, epoch, [&] {
        double tot[1];
        final_partials64<1>(a.partials, tot, fin);
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
      bd_phase<1>(a, lds, sh, [&](const BdTile& tile, double(&)[1]) {
        const int row = my_row(tile);
        if (row >= 0) {
          const double2 beta = sh.beta[tile.sys], bo = cmul(beta, sh.omega[tile.sys]);
          const double2 w = csub(a.R[row], cmul(bo, a.V[row]));
          a.PH[row] = cfma(beta, a.PH[row], cmul(a.dinv[row], w));
        }
      });
      if (barrier_last(a.bar, epoch, [] {})) return;
    }
    // v = A phat ; sigma
    bd_phase<2>(a, lds, sh, [&](const BdTile& tile, double(&acc)[2]) {
      tile_spmv(tile, a.PH, [&](int row, double2 v) {
        a.V[row] = v;
        const double2 h = a.RH[row];
        acc[0] = fma(h.x, v.x, fma(h.y, v.y, acc[0]));
        acc[1] = fma(h.x, v.y, fma(-h.y, v.x, acc[1]));
      });
    });
    if (barrier_last(a.bar, epoch, [&] {
          double tot[2];
          final_partials64<2>(a.partials, tot, fin);
          if (threadIdx.x < a.nsys) upd_sigma(st, threadIdx.x, make_double2(tot[0], tot[1]));
        }))
      return;
    // s = r - alpha v ; shat ; ||s||^2
    bd_phase<1>(a, lds, sh, [&](const BdTile& tile, double(&acc)[1]) {
      const int row = my_row(tile);
      if (row >= 0 && sh.status[tile.sys] == B_RUN) {
        const double2 s = csub(a.R[row], cmul(sh.alpha[tile.sys], a.V[row]));
        a.SH[row] = cmul(a.dinv[row], s);
        acc[0] += cabs2(s);
      }
    });
    if (barrier_last(a.bar, epoch, [&] {
          double tot[1];
          final_partials64<1>(a.partials, tot, fin);
          if (threadIdx.x < a.nsys) upd_s(st, threadIdx.x, tot[0]);
        }))
      return;
    // t = A shat ; tau ; t^H s
    bd_phase<3>(a, lds, sh, [&](const BdTile& tile, double(&acc)[3]) {
      if (sh.status[tile.sys] != B_RUN) return;
      tile_spmv(tile, a.SH, [&](int row, double2 t) {
        a.T[row] = t;
        const double2 s = cmul(a.d[row], a.SH[row]);
        acc[0] = fma(t.x, t.x, fma(t.y, t.y, acc[0]));
        acc[1] = fma(t.x, s.x, fma(t.y, s.y, acc[1]));
        acc[2] = fma(t.x, s.y, fma(-t.y, s.x, acc[2]));
      });
    });
    if (barrier_last(a.bar, epoch, [&] {
          double tot[3];
          final_partials64<3>(a.partials, tot, fin);
          if (threadIdx.x < a.nsys) upd_omega(st, threadIdx.x, tot[0], make_double2(tot[1], tot[2]));
        }))
      return;
    // x, r updates ; ||r||^2 ; rhat^H r
    bd_phase<3>(a, lds, sh, [&](const BdTile& tile, double(&acc)[3]) {
      const int row = my_row(tile);
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
    if (barrier_last(a.bar, epoch, [&] {
          double tot[3];
          final_partials64<3>(a.partials, tot, fin);
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
  bd_phase<1>(a, lds, sh, [&](const BdTile& tile, double(&acc)[1]) {
    tile_spmv(tile, a.X, [&](int row, double2 ax) {
      acc[0] += cabs2(csub(a.B[row], ax));
    });
  });
  barrier_last(a.bar, epoch, [&] {
    double tot[1];
    final_partials64<1>(a.partials, tot, fin);
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
  hipStream_t s = as_stream(stream);
  // structure check through a temporary handle (real values are not read)
  hk_csr A = nullptr;
  int rc = hk_csr_create(&A, n, nnz, d_rowptr, d_col, d_K, HK_C128, HK_INT32_COLS, stream);
  if (rc != HK_OK) return rc;
  (void)hk_csr_destroy(A);
  int grid = 0;
  rc = coop_grid((const void*)k_sweep, &grid);
  if (rc != HK_OK) return rc;
  const size_t vec = (size_t)n * kSys;
  Arena ar;
  const size_t bytes = 6 * a256(16 * vec) + 2 * a256(8 * n) + a256(16 * kSys) +
                       a256(8 * 4 * (size_t)grid * kSys) + a256(sizeof(BatchState)) + a256(sizeof(GridBar)) +
                       a256(64);
  if (hipMalloc((void**)&ar.base, bytes) != hipSuccess) HK_FAIL(HK_ENOMEM, "hk_sweep_solve: hipMalloc(%zu)", bytes);
  SweepArgs a{};
  a.n = (int)n; a.nsys = nsys; a.rowptr = d_rowptr; a.col = d_col; a.K = d_K; a.M = d_M;
  a.R = ar.take<double2>(vec); a.RH = ar.take<double2>(vec); a.PH = ar.take<double2>(vec);
  a.V = ar.take<double2>(vec); a.SH = ar.take<double2>(vec); a.T = ar.take<double2>(vec);
  double* kd = ar.take<double>(n);
  double* md = ar.take<double>(n);
  double2* kap = ar.take<double2>(kSys);
  a.partials = ar.take<double>(4 * (size_t)grid * kSys);
  a.st = ar.take<BatchState>(1);
  a.bar = ar.take<GridBar>(1);
  int* flag = ar.take<int>(16);
  if (ar.off > bytes) {
    (void)hipFree(ar.base);
    HK_FAIL(HK_EINVAL, "hk_sweep_solve: workspace layout exceeds its allocation");
  }
  a.kd = kd; a.md = md; a.kap = kap;
  a.B = (const double2*)d_B; a.X = (double2*)d_X;
  a.tol = opts->tol; a.maxit = opts->max_iter;
  std::vector<double2> hk(kSys, make_double2(0, 0));
  for (int j = 0; j < nsys; ++j) hk[j] = make_double2(kappa[2 * j], kappa[2 * j + 1]);
  int hflag = 0;
  hipError_t e = hipMemcpyAsync(kap, hk.data(), 16 * kSys, hipMemcpyHostToDevice, s);
  GridBar bar0{};
  bar0.spin_limit = barrier_spin_limit();
  if (e == hipSuccess) e = hipMemcpyAsync(a.bar, &bar0, sizeof(GridBar), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(flag, 0, 64, s);
  if (e == hipSuccess) e = hipMemsetAsync(a.st, 0, sizeof(BatchState), s);
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
  if (e == hipSuccess && hflag) {
    (void)hipFree(ar.base);
    HK_FAIL(HK_EINVAL, "hk_sweep_solve: zero diagonal entry for some system (Jacobi undefined)");
  }
  if (e == hipSuccess) {
    void* args[] = {&a};
    e = hipLaunchCooperativeKernel((const void*)k_sweep, dim3(grid), dim3(kPB), args, 0, s);
  }
  BatchState hs{};
  GridBar hb{};
  if (e == hipSuccess) e = hipMemcpyAsync(&hs, a.st, sizeof(hs), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&hb, a.bar, sizeof(hb), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(ar.base);
  if (e != hipSuccess) HK_FAIL(HK_EHIP, "hk_sweep_solve: %s", hipGetErrorString(e));
  if (hb.abort) HK_FAIL(HK_EHIP, "hk_sweep_solve: grid barrier timed out");
  fill_infos(hs, nsys, infos);
  return worst_status(infos, nsys);
}

extern "C" int hk_blockdiag_solve(hk_csr A, int32_t nsys, const int64_t* row_off, const void* d_b,
                                  void* d_x, const hk_solve_opts* opts, hk_solve_info* infos,
                                  void* stream) {
  if (!A || !row_off || !d_b || !d_x || !opts || !infos) HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: null argument");
  if (A->dtype != HK_C128) HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: matrix must be complex128");
  if (nsys < 1 || nsys > kSys) HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: nsys must be in [1, 64]");
  if (!(opts->tol >= 0) || opts->max_iter < 0) HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: bad options");
  if (row_off[0] != 0 || row_off[nsys] != A->n) HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: row offsets must span [0, n]");
  for (int k = 0; k < nsys; ++k)
    if (row_off[k + 1] <= row_off[k]) HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: empty or decreasing system %d", k);
  hipStream_t s = as_stream(stream);
  // tile products: row blocks (one wave per 64 rows) unless the rows are
  // long (mean above 32 entries), then 32-lane groups per row
  const double mean_row = (double)A->nnz / (double)A->n;
  const int L = mean_row > 32 ? 32 : kRowBlockL;
  const int TR = kPB;
  // static tiles
  std::vector<int> tsys, trow, sys_end(kSys, 0), sys_begin(kSys, 0), tile0(kSys + 1, 0);
  std::vector<int> sys_of_row((size_t)A->n);
  for (int k = 0; k < nsys; ++k) {
    tile0[k] = (int)tsys.size();
    sys_begin[k] = (int)row_off[k];
    sys_end[k] = (int)row_off[k + 1];
    for (int64_t r = row_off[k]; r < row_off[k + 1]; r += TR) {
      tsys.push_back(k);
      trow.push_back((int)r);
    }
    for (int64_t r = row_off[k]; r < row_off[k + 1]; ++r) sys_of_row[r] = k;
  }
  tile0[nsys] = (int)tsys.size();
  for (int k = nsys + 1; k <= kSys; ++k) tile0[k] = tile0[nsys];
  const int nt = (int)tsys.size();
  const void* kern = nullptr;
  if (L == kRowBlockL) kern = (const void*)k_blockdiag<kRowBlockL>;
  else kern = (const void*)k_blockdiag<32>;
  int grid = 0;
  int rc = coop_grid(kern, &grid);
  if (rc != HK_OK) return rc;
  const int64_t n = A->n;
  Arena ar;
  const size_t bytes = 8 * a256(16 * (size_t)n) + 3 * a256(4 * (size_t)nt) +
                       a256(4 * (size_t)n) + 4 * a256(4 * (kSys + 1)) + a256(8 * 4 * (size_t)grid * kSys) +
                       a256(sizeof(BatchState)) + a256(sizeof(GridBar)) + a256(64);
  if (hipMalloc((void**)&ar.base, bytes) != hipSuccess) HK_FAIL(HK_ENOMEM, "hk_blockdiag_solve: hipMalloc(%zu)", bytes);
  BdArgs a{};
  a.n = (int)n; a.nsys = nsys; a.L = L; a.rowptr = A->rowptr; a.col = A->col;
  a.val = (const double2*)A->val;
  a.R = ar.take<double2>(n); a.RH = ar.take<double2>(n); a.PH = ar.take<double2>(n);
  a.V = ar.take<double2>(n); a.SH = ar.take<double2>(n); a.T = ar.take<double2>(n);
  double2* d = ar.take<double2>(n);
  double2* dinv = ar.take<double2>(n);
  a.act_sys = ar.take<int>(nt);
  a.act_row0 = ar.take<int>(nt);
  a.act_end = ar.take<int>(nt);
  int* d_sor = ar.take<int>(n);
  int* d_send = ar.take<int>(kSys + 1);
  int* d_sbeg = ar.take<int>(kSys + 1);
  int* d_t0 = ar.take<int>(kSys + 1);
  (void)ar.take<int>(kSys + 1);
  a.partials = ar.take<double>(4 * (size_t)grid * kSys);
  a.st = ar.take<BatchState>(1);
  a.bar = ar.take<GridBar>(1);
  int* flag = ar.take<int>(16);
  if (ar.off > bytes) {
    (void)hipFree(ar.base);
    HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: workspace layout exceeds its allocation");
  }
  a.d = d; a.dinv = dinv; a.sys_begin = d_sbeg; a.sys_end = d_send; a.sys_tile0 = d_t0;
  a.B = (const double2*)d_b; a.X = (double2*)d_x; a.tol = opts->tol; a.maxit = opts->max_iter;
  a.tile_rows = TR;
  int hflag = 0;
  // the start phase walks every tile
  std::vector<int> tend(nt);
  for (int k = 0; k < nt; ++k) tend[k] = sys_end[tsys[k]];
  hipError_t e = hipMemcpyAsync(a.act_sys, tsys.data(), 4 * (size_t)nt, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(a.act_row0, trow.data(), 4 * (size_t)nt, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(a.act_end, tend.data(), 4 * (size_t)nt, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_sor, sys_of_row.data(), 4 * (size_t)n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_send, sys_end.data(), 4 * kSys, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_sbeg, sys_begin.data(), 4 * kSys, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_t0, tile0.data(), 4 * (kSys + 1), hipMemcpyHostToDevice, s);
  GridBar bar0{};
  bar0.spin_limit = barrier_spin_limit();
  if (e == hipSuccess) e = hipMemcpyAsync(a.bar, &bar0, sizeof(GridBar), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(flag, 0, 64, s);
  if (e == hipSuccess) e = hipMemsetAsync(a.st, 0, sizeof(BatchState), s);
  BatchState init{};
  init.ntiles_active = nt;
  if (e == hipSuccess) e = hipMemcpyAsync(a.st, &init, sizeof(init), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // host vectors above go out of scope
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_bd_diag, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, (int)n,
                       A->rowptr, A->col, (const double2*)A->val, d_sor, d_sbeg, d_send, d, dinv, flag);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && hflag) {
    (void)hipFree(ar.base);
    if (hflag & 2) HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: matrix is not block-diagonal for the given offsets");
    HK_FAIL(HK_EINVAL, "hk_blockdiag_solve: zero diagonal entry (Jacobi undefined)");
  }
  if (e == hipSuccess) {
    void* args[] = {&a};
    e = hipLaunchCooperativeKernel(kern, dim3(grid), dim3(kPB), args, 0, s);
  }
  BatchState hs{};
  GridBar hb{};
  if (e == hipSuccess) e = hipMemcpyAsync(&hs, a.st, sizeof(hs), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&hb, a.bar, sizeof(hb), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(ar.base);
  if (e != hipSuccess) HK_FAIL(HK_EHIP, "hk_blockdiag_solve: %s", hipGetErrorString(e));
  if (hb.abort) HK_FAIL(HK_EHIP, "hk_blockdiag_solve: grid barrier timed out");
  fill_infos(hs, nsys, infos);
  return worst_status(infos, nsys);
}
