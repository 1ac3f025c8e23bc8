// hk_solver.hip -- Jacobi right-preconditioned BiCGStab on gfx950, with
// device-resident scalars, and the complex64/complex128 refinement loop.
//
// The paper's P-BiCGSTAB (Section 4) copies every dot product and norm back
// to the host.  Here every reduction stays on the device: the kernel that
// produces the terms stores one partial sum per workgroup, and a one-
// workgroup finalize kernel sums them in a fixed order, updates the scalars
// (rho, alpha, omega, beta), tests convergence / breakdown and writes a
// status word.  The host enqueues iterations in chunks and reads the status
// word once per chunk; kernels enqueued after the solve has ended return at
// once.
//
// The inner products, norms and scalars are double for both vector
// precisions.  In the complex64 solve the vectors, the matrix and its
// products stay complex64 (the bytes moved are those of complex64), but each
// product of two floats is formed exactly in double and summed in double,
// and each vector update uses its scalar rounded to complex64.  With float
// sums the rounding error of a dot over n terms, about sqrt(n) 2^-24
// ||rhat|| ||r||, exceeds |rhat^H r| itself once the iteration has lost
// bi-orthogonality (|rhat^H r| ~ 1e-7 ||rhat|| ||r|| on the FE Helmholtz
// systems), and the iteration then breaks down or stalls depending on the
// summation order.
//
// Jacobi is applied on the right by scaling the columns once per solve:
// Ahat = A D^-1 (a workspace copy of the values), and the iteration runs the
// unpreconditioned recurrences on Ahat y = b with x = D^-1 y at the end.
// Mathematically this is the preconditioned method with phat = D^-1 p and
// shat = D^-1 s; it saves one vector pass per preconditioner application.
//
// One iteration (each reduction followed by its finalize kernel):
//   K_p   : p = r + beta (p - omega v)                      (iteration > 1)
//   K_v   : v = Ahat p,  sigma = rhat^H v  -> alpha = rho / sigma
//   K_s   : s = r - alpha v
//   K_t   : t = Ahat s,  tau = t^H t, t^H s, ||s||^2
//           -> half-step convergence test, then omega
//   K_xr  : y += alpha p + omega s, r = s - omega t, ||r||^2, rhat^H r
//           -> rho, beta, convergence / breakdown / cap tests
// ||s||^2 comes from the epilogue of K_t, which reads s at its own rows for
// t^H s anyway; in the iteration that converges at the half step, t is
// computed and not used.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "hk_internal.hpp"
#include "hk_spmv.hpp"

namespace hk {

int spmv_dispatch(const hk_csr_s* A, const void* x, void* y, const void* b, const void* alpha,
                  const void* beta, int mode, hipStream_t s);

// Transient statuses (>= S_RUN): the solve goes on, or an exit is pending
// until the kernels of the current iteration have applied their last update.
enum : int { S_RUN = 100, S_HALF = 101, S_TAUBD = 102, S_HALF2 = 103, S_RHOBD = 104 };

struct SolveState {
  double2 rho, rho_old, alpha, omega, beta;
  double rr, ss, bb, theta2, rr_true;
  int status, bd;
  long long iter, maxit, iters_done;
  double* history;
  // TFQMR: theta, tau, the two half-steps' eta (their x updates are applied
  // by the next kernel that reads d) and the d-update coefficients
  double tq_theta, tq_tau;
  double2 tq_eta1, tq_eta2, tq_coef1, tq_coef2;
  // BiCGStab(l): the minimal-residual coefficients gamma_1..gamma_l
  double2 bl_gamma[8];
};

// Most workgroups of a fused SpMV+dot launch (one partial-sum slot each).
// A launch shape with grid 0 gets one tile per workgroup up to this cap: on
// the 1.8M-row system, walking 7,094 tiles with 2,048 workgroups cost ~20 us
// per product (132 vs 116 us).  Row-block shapes widen their workgroups (2,
// 4 or 8 waves) until the tiles fit under the cap, because a finalize kernel
// over 28,374 partials (32-row blocks in 2-wave workgroups) took 8.8-15.5 us
// instead of 4.6-6.6.
constexpr int kMaxGrid = 8192;
constexpr int kEw = 4;           // elements per thread in the element-wise solver kernels

// workgroups of an element-wise solver kernel over n elements
static inline int ew_blocks(int64_t n) {
  const int64_t b = (n + kBlock * kEw - 1) / (kBlock * kEw);
  return (int)(b < 1 ? 1 : b);
}
// partial-sum slots needed by any solver reduction
static inline int64_t partial_slots(int64_t n) {
  const int64_t e = ew_blocks(n);
  return e > kMaxGrid ? e : kMaxGrid;
}

// a solver scalar (double) rounded to the vector type
template <class V> __device__ __forceinline__ V vscal(double2 a) {
  return cmake<V>((decltype(V::x))a.x, (decltype(V::x))a.y);
}
// |a|^2 in double
template <class V> __device__ __forceinline__ double nrm2d(V a) {
  const double x = a.x, y = a.y;
  return x * x + y * y;
}
// acc += conj(a) * b in double (two partial sums: re, im)
template <class V> __device__ __forceinline__ void dotc_acc(V a, V b, double& re, double& im) {
  const double ax = a.x, ay = a.y, bx = b.x, by = b.y;
  re = fma(ax, bx, fma(ay, by, re));
  im = fma(ax, by, fma(-ay, bx, im));
}

// ------------------------------------------------------------ set-up kernels

// dinv_i = 1 / a_ii (flag[0] = 1 if a row has no nonzero diagonal); with
// precond == 0, dinv = 1.
template <class V>
__global__ void k_diag_inv(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                           const V* __restrict__ val, V* __restrict__ dinv, int precond, int* flag) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  if (!precond) { dinv[i] = cmake<V>(1, 0); return; }
  V d = czero<V>();
  for (int p = rowptr[i]; p < rowptr[i + 1]; ++p)
    if (col[p] == i) d = cadd(d, val[p]);
  if (d.x == 0 && d.y == 0) { atomicOr(flag, 1); dinv[i] = cmake<V>(0, 0); return; }
  dinv[i] = cdiv(cmake<V>(1, 0), d);
}

// ahat_p = a_p * dinv_col(p): one thread per entry, so the streams are
// coalesced (a thread per row, walking its row, took ~10x the memory time)
template <class V>
__global__ __launch_bounds__(kBlock) void k_scale_cols(int64_t nnz, const int* __restrict__ col,
                                                       const V* __restrict__ val, const V* __restrict__ dinv,
                                                       V* __restrict__ ahat) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p < nnz) ahat[p] = cmul(val[p], dinv[col[p]]);
}
template <class V>
static void launch_scale_cols(int64_t nnz, const int* col, const V* val, const V* dinv, V* ahat, hipStream_t s) {
  if (nnz > 0)
    hipLaunchKernelGGL(k_scale_cols<V>, dim3((unsigned)((nnz + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, nnz,
                       col, val, dinv, ahat);
}

// Start of the iteration: r = b - A x0 (already in r when use_x0) or r = b,
// rhat = p = r, y = x0 / dinv or 0, zero = 0 (when given); partials of
// ||b||^2 and ||r||^2.
template <class R>
__global__ __launch_bounds__(kBlock) void k_init(int n, int use_x0, const cplx<R>* __restrict__ b,
                                                 const cplx<R>* __restrict__ x0,
                                                 const cplx<R>* __restrict__ dinv,
                                                 cplx<R>* __restrict__ r, cplx<R>* __restrict__ rh,
                                                 cplx<R>* __restrict__ p, cplx<R>* __restrict__ y,
                                                 cplx<R>* __restrict__ zero, double* partials) {
  using V = cplx<R>;
  __shared__ double lds[2 * (kBlock / kWave)];
  double acc[2] = {0, 0};
  const int base = blockIdx.x * (kBlock * kEw) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kEw; ++k) {
    const int i = base + k * kBlock;
    if (i >= n) break;
    const V bi = b[i];
    V ri = bi;
    V yi = czero<V>();
    if (use_x0) {
      ri = r[i];
      yi = cdiv(x0[i], dinv[i]);
    } else {
      r[i] = bi;
    }
    rh[i] = ri;
    p[i] = ri;
    y[i] = yi;
    if (zero) zero[i] = czero<V>();
    acc[0] += nrm2d(bi);
    acc[1] += nrm2d(ri);
  }
  block_sum<2>(acc, lds);
  store_block_partials<2>(acc, partials);
}

// ----------------------------------------------------------- iteration kernels

template <class R>
__global__ __launch_bounds__(kBlock) void k_p(int n, const SolveState* __restrict__ st,
                                              const cplx<R>* __restrict__ r, cplx<R>* __restrict__ p,
                                              const cplx<R>* __restrict__ v) {
  using V = cplx<R>;
  if (st->status != S_RUN || st->iter == 1) return;
  const V beta = vscal<V>(st->beta), omega = vscal<V>(st->omega);
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  // p = r + beta (p - omega v)
  V q = csub(p[i], cmul(omega, v[i]));
  p[i] = cfma(beta, q, r[i]);
}

// v = Ahat p and partials of sigma = rhat^H v  (DOT == 1), or
// t = Ahat s and partials of tau = t^H t, t^H s, ||s||^2 (DOT == 2).
template <int L, int U, class R, int DOT>
__global__ __launch_bounds__(kBlock) void k_spmv_dot(int n, int ntiles, const int* __restrict__ rowptr,
                                                     const int* __restrict__ col,
                                                     const cplx<R>* __restrict__ val,
                                                     const cplx<R>* __restrict__ x,
                                                     cplx<R>* __restrict__ y,
                                                     const cplx<R>* __restrict__ w,
                                                     const SolveState* __restrict__ st, double* partials) {
  using V = cplx<R>;
  constexpr int NV = DOT == 1 ? 2 : 4;
  __shared__ double lds[NV * (kBlock / kWave)];
  if (st->status != S_RUN) return;
  constexpr int RT = (kBlock / L) * U;
  const int g = threadIdx.x / L, lane = threadIdx.x & (L - 1);
  double part[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) part[k] = 0;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int r0 = t * RT + g * U;
    // the epilogue operand of the row this lane will write, loaded early
    const int rw = r0 + (lane < U ? lane : 0);
    const V wr = w[rw < n ? rw : n - 1];
    V acc[U];
    csr_rows<L, U, V>(r0, n, rowptr, col, val, x, acc);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = r0 + u;
      if (lane == u && r < n) {
        y[r] = acc[u];
        if (DOT == 1) {
          dotc_acc(wr, acc[u], part[0], part[1]);  // conj(rhat_r) * v_r
        } else {
          part[0] += nrm2d(acc[u]);
          dotc_acc(acc[u], wr, part[1], part[2]);  // conj(t_r) * s_r
          part[3] += nrm2d(wr);
        }
      }
    }
  }
  block_sum<NV>(part, lds);
  store_block_partials<NV>(part, partials);
}

// Row-block variant of k_spmv_dot (one wave per RW rows); the row's sum
// lands in the lane that owns the row.
template <int RW, int NW, class R, int DOT, class CI, bool PAIRS>
__global__ __launch_bounds__(NW * kWave) void k_spmv_dot_rb(int n, int ntiles, const int* __restrict__ rowptr,
                                                            const CI* __restrict__ col,
                                                            const cplx<R>* __restrict__ val,
                                                            const cplx<R>* __restrict__ x,
                                                            cplx<R>* __restrict__ y,
                                                            const cplx<R>* __restrict__ w,
                                                            const SolveState* __restrict__ st, double* partials) {
  using V = cplx<R>;
  constexpr int NV = DOT == 1 ? 2 : 4;
  constexpr int CH = RbCh<RW, V>::v;
  __shared__ V lds[NW * CH * kWave];
  if (st->status != S_RUN) return;
  V* buf = lds + (threadIdx.x / kWave) * CH * kWave;
  const int l = threadIdx.x & (kWave - 1);
  double part[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) part[k] = 0;
  for (int tb = blockIdx.x; tb < ntiles; tb += gridDim.x) {
    const int t = tile_of(tb, ntiles);
    const int r0 = t * (NW * RW) + (threadIdx.x / kWave) * RW;
    const int r = r0 + l;
    const V wr = w[r < n ? r : n - 1];
    V acc;
    if constexpr (PAIRS) acc = csr_block_rows_pairs<RW, CH, V>(r0, n, rowptr, col, val, x, buf);
    else acc = csr_block_rows<RW, CH, V, CI>(r0, n, rowptr, col, val, x, buf);
    if (l < RW && r < n) {
      y[r] = acc;
      if (DOT == 1) {
        dotc_acc(wr, acc, part[0], part[1]);
      } else {
        part[0] += nrm2d(acc);
        dotc_acc(acc, wr, part[1], part[2]);
        part[3] += nrm2d(wr);
      }
    }
  }
  __syncthreads();
  block_sum<NV, double, NW>(part, reinterpret_cast<double*>(lds));
  store_block_partials<NV>(part, partials);
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_s(int n, const SolveState* __restrict__ st,
                                              const cplx<R>* __restrict__ r,
                                              const cplx<R>* __restrict__ v, cplx<R>* __restrict__ s) {
  using V = cplx<R>;
  if (st->status != S_RUN) return;
  const V alpha = vscal<V>(st->alpha);
  const int base = blockIdx.x * (kBlock * kEw) + threadIdx.x;
  if (base + (kEw - 1) * kBlock < n) {
    V rv[kEw], vv[kEw];
#pragma unroll
    for (int k = 0; k < kEw; ++k) { rv[k] = r[base + k * kBlock]; vv[k] = v[base + k * kBlock]; }
#pragma unroll
    for (int k = 0; k < kEw; ++k) s[base + k * kBlock] = csub(rv[k], cmul(alpha, vv[k]));  // s = r - alpha v
  } else {
#pragma unroll
    for (int k = 0; k < kEw; ++k) {
      const int i = base + k * kBlock;
      if (i >= n) break;
      s[i] = csub(r[i], cmul(alpha, v[i]));
    }
  }
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_xr(int n, const SolveState* __restrict__ st,
                                               const cplx<R>* __restrict__ rh,
                                               cplx<R>* __restrict__ r, const cplx<R>* __restrict__ p,
                                               const cplx<R>* __restrict__ s,
                                               const cplx<R>* __restrict__ t, cplx<R>* __restrict__ y,
                                               double* partials) {
  using V = cplx<R>;
  __shared__ double lds[3 * (kBlock / kWave)];
  const int status = st->status;
  if (status != S_RUN && status != S_HALF && status != S_TAUBD) return;
  const V alpha = vscal<V>(st->alpha), omega = vscal<V>(st->omega);
  const int base = blockIdx.x * (kBlock * kEw) + threadIdx.x;
  if (status != S_RUN) {
    // half-step exit (converged on s) or tau breakdown: y += alpha p
#pragma unroll
    for (int k = 0; k < kEw; ++k) {
      const int i = base + k * kBlock;
      if (i < n) y[i] = cfma(alpha, p[i], y[i]);
    }
    return;
  }
  double acc[3] = {0, 0, 0};
  // y += alpha p + omega s ; r = s - omega t ; ||r||^2 ; rhat^H r
  auto upd = [&](int i, V si, V pi, V ti, V yi, V hi) {
    y[i] = cfma(omega, si, cfma(alpha, pi, yi));
    const V ri = csub(si, cmul(omega, ti));
    r[i] = ri;
    acc[0] += nrm2d(ri);
    dotc_acc(hi, ri, acc[1], acc[2]);
  };
  if (base + (kEw - 1) * kBlock < n) {
    V sv[kEw], pv[kEw], tv[kEw], yv[kEw], hv[kEw];
#pragma unroll
    for (int k = 0; k < kEw; ++k) {
      const int i = base + k * kBlock;
      sv[k] = s[i]; pv[k] = p[i]; tv[k] = t[i]; yv[k] = y[i]; hv[k] = rh[i];
    }
#pragma unroll
    for (int k = 0; k < kEw; ++k) upd(base + k * kBlock, sv[k], pv[k], tv[k], yv[k], hv[k]);
  } else {
#pragma unroll
    for (int k = 0; k < kEw; ++k) {
      const int i = base + k * kBlock;
      if (i >= n) break;
      upd(i, s[i], p[i], t[i], y[i], rh[i]);
    }
  }
  block_sum<3>(acc, lds);
  store_block_partials<3>(acc, partials);
}

// x = dinv .* y
template <class V>
__global__ void k_unscale(int n, const V* __restrict__ dinv, const V* __restrict__ y, V* __restrict__ x) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = cmul(dinv[i], y[i]);
}

// partials of ||w||^2
template <class R>
__global__ __launch_bounds__(kBlock) void k_norm2_partials(int n, const cplx<R>* __restrict__ w, double* partials) {
  __shared__ double lds[kBlock / kWave];
  double acc[1] = {0};
  const int base = blockIdx.x * (kBlock * kEw) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kEw; ++k) {
    const int i = base + k * kBlock;
    if (i < n) acc[0] += nrm2d(w[i]);
  }
  block_sum<1>(acc, lds);
  store_block_partials<1>(acc, partials);
}

// ------------------------------------------------------------ finalize kernels

enum : int { F_INIT = 0, F_SIGMA = 1, F_OMEGA = 3, F_XR = 4, F_TRUE = 5, F_TUNE = 6 };

template <int F> struct FinNV { static constexpr int v = 1; };
template <> struct FinNV<F_INIT> { static constexpr int v = 2; };
template <> struct FinNV<F_SIGMA> { static constexpr int v = 2; };
template <> struct FinNV<F_TUNE> { static constexpr int v = 2; };
template <> struct FinNV<F_OMEGA> { static constexpr int v = 4; };
template <> struct FinNV<F_XR> { static constexpr int v = 3; };

// One workgroup: sums the nb partials of the preceding kernel and applies
// the scalar update of step F.
template <class R, int F, int BS>
__global__ __launch_bounds__(BS) void k_fin(SolveState* st, const double* partials, int nb, double tol,
                                            long long maxit) {
  using V = double2;
  constexpr int NV = FinNV<F>::v;
  __shared__ double lds[NV * (BS / kWave)];
  // The status and the fields the scalar update reads are loaded before the
  // partials are summed, so their latency overlaps that of the sum's loads
  // instead of following it.  The sum runs whatever the status: the partials
  // are in bounds even when the producing kernel returned early, and are then
  // ignored.
  const int status = st->status;
  const V rho0 = st->rho, alpha0 = st->alpha, omega0 = st->omega;
  const double theta2 = st->theta2, bb = st->bb;
  const long long it0 = st->iter, maxit0 = st->maxit;
  double* const history = st->history;
  double tot[NV];
  final_sum<NV, double, BS>(partials, nb, tot, lds);
  if (F == F_XR) {
    if (status == S_HALF || status == S_TAUBD) {
      if (threadIdx.x == 0) {
        const long long it = st->iter;
        st->rr = st->ss;
        st->iters_done = it;
        if (status == S_HALF) {
          st->status = HK_OK;
          if (st->history) st->history[it] = st->bb > 0 ? sqrt((double)st->ss / (double)st->bb) : 0.0;
        } else {
          st->status = HK_BREAKDOWN;
          st->bd = HK_BD_TAU;
        }
      }
      return;
    }
  }
  if (F != F_INIT && F != F_TRUE && F != F_TUNE && status != S_RUN) return;
  if (threadIdx.x != 0) return;
  if (F == F_INIT) {
    st->bb = tot[0];
    st->rr = tot[1];
    st->theta2 = tol * tol * tot[0];
    st->rho = cmake<V>(tot[1], 0);
    st->rho_old = cmake<V>(1, 0);
    st->alpha = cmake<V>(1, 0);
    st->omega = cmake<V>(1, 0);
    st->beta = czero<V>();
    st->iter = 1;
    st->maxit = maxit;
    st->iters_done = 0;
    st->bd = HK_BD_NONE;
    if (!isfinite(tot[0]) || !isfinite(tot[1])) st->status = HK_NONFINITE;
    else if (tot[1] <= st->theta2) st->status = HK_OK;
    else if (maxit <= 0) st->status = HK_NOT_CONVERGED;
    else st->status = S_RUN;
    if (st->history) st->history[0] = tot[0] > 0 ? sqrt((double)tot[1] / (double)tot[0]) : 0.0;
  } else if (F == F_SIGMA) {
    const V sigma = cmake<V>(tot[0], tot[1]);
    if (!cfinite(sigma)) {
      st->status = HK_NONFINITE;
      st->iters_done = it0 - 1;
    } else if (sigma.x == 0 && sigma.y == 0) {
      st->status = HK_BREAKDOWN;
      st->bd = HK_BD_SIGMA;
      st->iters_done = it0 - 1;
    } else {
      st->alpha = cdiv(rho0, sigma);
    }
  } else if (F == F_OMEGA) {
    const double tau = tot[0];
    const V ts = cmake<V>(tot[1], tot[2]);
    st->ss = tot[3];
    if (!isfinite(tot[3])) {
      st->status = HK_NONFINITE;
      st->iters_done = it0 - 1;
    } else if (tot[3] <= theta2) {
      st->status = S_HALF;
    } else if (!isfinite(tau) || !cfinite(ts)) {
      st->status = HK_NONFINITE;
      st->iters_done = it0 - 1;
    } else if (tau == 0) {
      st->status = S_TAUBD;
    } else {
      st->omega = cmake<V>(ts.x / tau, ts.y / tau);
    }
  } else if (F == F_XR) {
    const long long it = it0;
    const double rr = tot[0];
    const V rho = cmake<V>(tot[1], tot[2]);
    st->rr = rr;
    st->rho_old = rho0;
    st->rho = rho;
    st->iters_done = it;
    if (history) history[it] = bb > 0 ? sqrt((double)rr / (double)bb) : 0.0;
    if (!isfinite(rr) || !cfinite(rho)) {
      st->status = HK_NONFINITE;
    } else if (rr <= theta2) {
      st->status = HK_OK;
    } else if (omega0.x == 0 && omega0.y == 0) {
      st->status = HK_BREAKDOWN;
      st->bd = HK_BD_OMEGA;
    } else if (rho.x == 0 && rho.y == 0) {
      st->status = HK_BREAKDOWN;
      st->bd = HK_BD_RHO;
    } else if (it >= maxit0) {
      st->status = HK_NOT_CONVERGED;
    } else {
      // beta = (rho / rho_old) (alpha / omega)
      st->beta = cmul(cdiv(rho, rho0), cdiv(alpha0, omega0));
      st->iter = it + 1;
    }
  } else if (F == F_TRUE) {
    st->rr_true = tot[0];
  } else {  // F_TUNE: the summation of F_SIGMA without its scalar updates
    st->rr_true = tot[0] + tot[1];
  }
}

// --------------------------------------------------------- mixed-precision helpers

// b = round_to_c64(scale * a); scale is a power of two, so the scaling is exact
__global__ void k_round_c64(int64_t m, const double2* __restrict__ a, float2* __restrict__ b, double scale) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < m) {
    const double2 v = a[i];
    b[i] = make_float2((float)(scale * v.x), (float)(scale * v.y));
  }
}
// u += scale * d (complex128 accumulation; scale a power of two)
__global__ void k_add_c64(int n, const float2* __restrict__ d, double2* __restrict__ u, double scale) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    const double2 a = u[i];
    const float2 e = d[i];
    u[i] = make_double2(a.x + scale * (double)e.x, a.y + scale * (double)e.y);
  }
}

// ------------------------------------------------------------------- driver

template <class R> struct Work {
  using V = cplx<R>;
  V *y, *r, *rh, *p, *v, *s, *t, *dinv, *ahat;
  V *u, *d;  // TFQMR only
  double* partials;
  SolveState* st;
  int* flag;
};

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// The workspace layout is written once, as a sequence of take(bytes) calls;
// work_bytes runs it with a counting take, carve with one that hands out
// addresses, so the size and the layout cannot disagree.
template <class R, class Take> static Work<R> layout(Take take, int64_t n, int64_t nnz) {
  using V = cplx<R>;
  Work<R> w;
  w.y = (V*)take(sizeof(V) * n);
  w.r = (V*)take(sizeof(V) * n);
  w.rh = (V*)take(sizeof(V) * n);
  w.p = (V*)take(sizeof(V) * n);
  w.v = (V*)take(sizeof(V) * n);
  w.s = (V*)take(sizeof(V) * n);
  w.t = (V*)take(sizeof(V) * n);
  w.dinv = (V*)take(sizeof(V) * n);
  w.u = (V*)take(sizeof(V) * n);
  w.d = (V*)take(sizeof(V) * n);
  w.ahat = (V*)take(sizeof(V) * (nnz + 1));  // one padding entry (paired-entry products)
  w.partials = (double*)take(sizeof(double) * 4 * partial_slots(n));
  w.st = (SolveState*)take(sizeof(SolveState));
  w.flag = (int*)take(64);
  return w;
}

template <class R> static size_t work_bytes(int64_t n, int64_t nnz) {
  size_t q = 0;
  (void)layout<R>([&](size_t bytes) { q += align_up(bytes); return (char*)nullptr; }, n, nnz);
  return q;
}

template <class R> static Work<R> carve(void* base, int64_t n, int64_t nnz) {
  char* q = static_cast<char*>(base);
  return layout<R>([&](size_t bytes) { char* r = q; q += align_up(bytes); return r; }, n, nnz);
}

static int ensure_ws(void** ws, size_t* have, size_t need, hipStream_t s) {
  if (*have >= need) return HK_OK;
  if (*ws) {
    HK_HIP(hipStreamSynchronize(s));
    HK_HIP(hipFree(*ws));
    *ws = nullptr;
    *have = 0;
  }
  if (hipMalloc(ws, need) != hipSuccess) HK_FAIL(HK_ENOMEM, "solver workspace: hipMalloc(%zu) failed", need);
  *have = need;
  return HK_OK;
}

// Tiles of the fused SpMV+dot launches for launch shape p, and for
// row-block shapes the waves per workgroup: p.nw when set, else the fewest
// of 2, 4, 8 that keep the tiles within kMaxGrid.
static int dot_tiles(const hk_csr_s* A, const SpmvPlan& p, int* nw_out) {
  int nw = 0;
  int64_t tiles = spmv_tiles(A, p.L, p.U);
  if (p.L == kRowBlockL) {
    if (p.nw == 2 || p.nw == 4 || p.nw == 8) {
      nw = p.nw;
    } else {
      for (nw = 2; nw < 8; nw *= 2)
        if ((A->n + (int64_t)nw * p.U - 1) / ((int64_t)nw * p.U) <= kMaxGrid) break;
    }
    tiles = (A->n + (int64_t)nw * p.U - 1) / ((int64_t)nw * p.U);
  }
  if (nw_out) *nw_out = nw;
  return (int)tiles;
}

// workgroups of a fused launch for shape p
static int dot_grid(const hk_csr_s* A, const SpmvPlan& p) {
  const int ntiles = dot_tiles(A, p, nullptr);
  const int g = p.grid > 0 ? p.grid : kMaxGrid;
  return std::max(1, std::min(g, std::min(ntiles, kMaxGrid)));
}

template <class R>
static hipError_t launch_spmv_dot(const hk_csr_s* A, const SpmvPlan& p, int dot, const cplx<R>* val,
                                  const cplx<R>* x, cplx<R>* y, const cplx<R>* w, const Work<R>& wk,
                                  hipStream_t s) {
  int nw = 0;
  const int ntiles = dot_tiles(A, p, &nw);
  const int grid = dot_grid(A, p);
  const int L = p.L, U = p.U;
  const int n = (int)A->n;
#define HK_SD_CASE(LL, UU)                                                                          \
  if (L == LL && U == UU) {                                                                         \
    if (dot == 1)                                                                                   \
      hipLaunchKernelGGL((k_spmv_dot<LL, UU, R, 1>), dim3(grid), dim3(kBlock), 0, s, n, ntiles,     \
                         A->rowptr, A->col, val, x, y, w, wk.st, wk.partials);                      \
    else                                                                                            \
      hipLaunchKernelGGL((k_spmv_dot<LL, UU, R, 2>), dim3(grid), dim3(kBlock), 0, s, n, ntiles,     \
                         A->rowptr, A->col, val, x, y, w, wk.st, wk.partials);                      \
    return hipGetLastError();                                                                       \
  }
  HK_SD_CASE(4, 1) HK_SD_CASE(4, 2) HK_SD_CASE(4, 4)
  HK_SD_CASE(8, 1) HK_SD_CASE(8, 2) HK_SD_CASE(8, 4) HK_SD_CASE(8, 8)
  HK_SD_CASE(16, 1) HK_SD_CASE(16, 2) HK_SD_CASE(16, 4) HK_SD_CASE(16, 8)
  HK_SD_CASE(32, 1) HK_SD_CASE(32, 2) HK_SD_CASE(32, 4) HK_SD_CASE(32, 8)
#undef HK_SD_CASE
#define HK_SDRB_LAUNCH(RR, NWW, DD, CI, PP, COL)                                                        \
  hipLaunchKernelGGL((k_spmv_dot_rb<RR, NWW, R, DD, CI, PP>), dim3(grid), dim3(NWW * kWave), 0, s, n,    \
                     ntiles, A->rowptr, COL, val, x, y, w, wk.st, wk.partials)
#define HK_SDRB_DOT(RR, NWW, DD)                                                                       \
  if (c16 && p.pairs) HK_SDRB_LAUNCH(RR, NWW, DD, short, true, c16);                                   \
  else if (c16) HK_SDRB_LAUNCH(RR, NWW, DD, short, false, c16);                                        \
  else HK_SDRB_LAUNCH(RR, NWW, DD, int, false, A->col);
#define HK_SDRB_CASE(RR, NWW)                                                                          \
  if (L == kRowBlockL && U == RR && nw == NWW) {                                                       \
    const short* c16 = (const short*)A->col16;                                                         \
    if (dot == 1) {                                                                                    \
      HK_SDRB_DOT(RR, NWW, 1)                                                                          \
    } else {                                                                                           \
      HK_SDRB_DOT(RR, NWW, 2)                                                                          \
    }                                                                                                  \
    return hipGetLastError();                                                                          \
  }
  HK_SDRB_CASE(16, 2) HK_SDRB_CASE(32, 2) HK_SDRB_CASE(64, 2)
  HK_SDRB_CASE(16, 4) HK_SDRB_CASE(32, 4) HK_SDRB_CASE(64, 4)
  HK_SDRB_CASE(16, 8) HK_SDRB_CASE(32, 8) HK_SDRB_CASE(64, 8)
#undef HK_SDRB_CASE
#undef HK_SDRB_DOT
#undef HK_SDRB_LAUNCH
  return hipErrorInvalidValue;
}

template <class R, int F>
static hipError_t launch_fin(const Work<R>& wk, int nb, double tol, long long maxit, hipStream_t s) {
  if (nb <= kFinSmallNb)
    hipLaunchKernelGGL((k_fin<R, F, kFinBlockSmall>), dim3(1), dim3(kFinBlockSmall), 0, s, wk.st, wk.partials, nb,
                       tol, maxit);
  else
    hipLaunchKernelGGL((k_fin<R, F, kFinBlock>), dim3(1), dim3(kFinBlock), 0, s, wk.st, wk.partials, nb, tol, maxit);
  return hipGetLastError();
}

// Times the fused SpMV+dot kernel (with its finalize) in every launch shape
// on A's pattern and keeps the fastest in *out (HIP events on stream s).
// Row-block shapes are tried with 2, 4 and 8 waves per workgroup where the
// tiles fit under kMaxGrid, and on the 16-bit column stream in both entry
// layouts (the products read the solver's padded copy of the values); every
// shape with one workgroup per tile and with 2,048 workgroups walking the
// tiles (fewer partials for the finalize).  The workspace vectors serve as operands (their
// values do not matter for timing); the scalar state is set to running here,
// left so by the F_TUNE finalize, and re-initialised by the solve afterwards.
template <class R>
static int tune_dot(const hk_csr_s* A, const Work<R>& wk, SpmvPlan* out, hipStream_t s) {
  std::vector<SpmvPlan> cands;
  for (int grid : {0, 2048}) {
    for (int L : {4, 8, 16, 32})
      for (int U : {1, 2, 4, 8})
        if (U <= L) { SpmvPlan p; p.L = L; p.U = U; p.grid = grid; cands.push_back(p); }
    for (int U : {16, 32, 64})
      for (int nw : {2, 4, 8})
        for (int pairs : {0, 1}) {
          if (pairs && !A->col16) continue;
          SpmvPlan p; p.L = kRowBlockL; p.U = U; p.nw = nw; p.grid = grid; p.pairs = pairs;
          if ((A->n + (int64_t)nw * U - 1) / ((int64_t)nw * U) <= kMaxGrid || nw == 8) cands.push_back(p);
        }
  }
  SolveState run{};
  run.status = S_RUN;
  HK_HIP(hipMemcpyAsync(wk.st, &run, sizeof(run), hipMemcpyHostToDevice, s));
  hipEvent_t e0, e1;
  HK_HIP(hipEventCreate(&e0));
  HK_HIP(hipEventCreate(&e1));
  SpmvPlan best = cands[0];
  float best_ms = 1e30f;
  int rc = HK_OK;
  for (const SpmvPlan& p : cands) {
    const int g = dot_grid(A, p);
    hipError_t err = hipSuccess;
    const int reps = 5;
    for (int it = 0; it < reps + 1 && err == hipSuccess; ++it) {
      if (it == 1) err = hipEventRecord(e0, s);
      if (err == hipSuccess) err = launch_spmv_dot<R>(A, p, 1, wk.ahat, wk.p, wk.v, wk.rh, wk, s);
      if (err == hipSuccess) err = launch_fin<R, F_TUNE>(wk, g, 0, 0, s);
    }
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err != hipSuccess) {
      set_error_text("solver tuning: %s", hipGetErrorString(err));
      rc = HK_EHIP;
      break;
    }
    if (ms < best_ms) { best_ms = ms; best = p; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != HK_OK) return rc;
  if (best.L == kRowBlockL) {
    int nw = 0;
    (void)dot_tiles(A, best, &nw);
    best.nw = nw;
  }
  best.tuned = 1;
  *out = best;
  return HK_OK;
}

// End of a solve: x = D^-1 y, the true residual ||b - A x|| with the
// original values, and *info from the device state (synchronises).
template <class R>
static int finish_solve(const hk_csr_s* A, const cplx<R>* val, const cplx<R>* b, cplx<R>* x, const Work<R>& wk,
                        hk_solve_info* info, hipStream_t s) {
  using V = cplx<R>;
  const int n = (int)A->n;
  const dim3 ew((unsigned)((n + kBlock - 1) / kBlock));
  const int gv = ew_blocks(n);
  hipLaunchKernelGGL(k_unscale<V>, ew, dim3(kBlock), 0, s, n, wk.dinv, wk.y, x);
  HK_CHECK_LAUNCH();
  {
    hk_csr_s tmp = *A;
    tmp.val = val;
    int rc2 = spmv_dispatch(&tmp, x, wk.t, b, nullptr, nullptr, 1, s);
    if (rc2 != HK_OK) return rc2;
  }
  hipLaunchKernelGGL(k_norm2_partials<R>, dim3(gv), dim3(kBlock), 0, s, n, wk.t, wk.partials);
  HK_CHECK_LAUNCH();
  HK_HIP((launch_fin<R, F_TRUE>(wk, gv, 0, 0, s)));
  SolveState hs;
  HK_HIP(hipMemcpyAsync(&hs, wk.st, sizeof(hs), hipMemcpyDeviceToHost, s));
  HK_HIP(hipStreamSynchronize(s));
  info->status = hs.status >= S_RUN ? HK_NOT_CONVERGED : hs.status;
  info->breakdown = hs.bd;
  info->iters = hs.status >= S_RUN ? hs.iter : hs.iters_done;
  const double bb = (double)hs.bb;
  info->relres_rec = bb > 0 ? std::sqrt((double)hs.rr / bb) : std::sqrt((double)hs.rr);
  info->relres_true = bb > 0 ? std::sqrt((double)hs.rr_true / bb) : std::sqrt((double)hs.rr_true);
  info->inner_iters = 0;
  return HK_OK;
}

// Runs the whole solve for precision R on values `val` (A's pattern), right
// side b, solution x (input when use_x0).  Fills info (host), synchronises.
// Chunked iteration driver shared by the three methods.  enqueue(q)
// enqueues one chunk (m iterations) on stream q and returns the first launch
// error.  After each chunk the status word is copied to pinned memory and
// read one chunk behind, so the GPU always has the next chunk queued; the
// loop ends once a solve has stopped or max_iter iterations are enqueued.
// The chunk is recorded once into a HIP graph on a private stream and
// replayed, one launch per chunk instead of one per kernel: on small systems
// the kernels take a few microseconds each and the host's launch rate would
// otherwise bound the solve.  The chunk holds kernels only (no memset or
// copy), on buffers fixed for the solve.  If the graph cannot be built, the
// chunk is longer than 256 iterations, or HK_SOLVE_GRAPHS=0 is set, the
// chunks are launched on s directly.  s is
// idle on return or holds only work ordered after the chunks.
template <class Enq>
static int run_chunks(int* pin, SolveState* st, int m, long long max_iter, hipStream_t s, Enq&& enqueue) {
  const char* env = getenv("HK_SOLVE_GRAPHS");
  // a chunk of at most 256 iterations is recorded (a few thousand graph nodes)
  const bool want_graph = !(env && env[0] == '0') && m <= 256;
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr}, fork = nullptr;
  HK_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  HK_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  if (want_graph) {
    bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventRecord(fork, s) == hipSuccess && hipStreamWaitEvent(cs, fork, 0) == hipSuccess;
    if (ok && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      const hipError_t le = enqueue(cs);
      hipGraph_t g = nullptr;
      const hipError_t ce = hipStreamEndCapture(cs, &g);
      if (le == hipSuccess && ce == hipSuccess && g) {
        graph = g;
        ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
      } else {
        if (g) (void)hipGraphDestroy(g);
        ok = false;
      }
    } else {
      ok = false;
    }
    if (!ok) {  // direct launches on s instead
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      exec = nullptr;
      graph = nullptr;
      if (cs) {
        (void)hipStreamSynchronize(cs);
        (void)hipStreamDestroy(cs);
      }
      cs = nullptr;
      (void)hipGetLastError();
    }
  }
  hipStream_t q = exec ? cs : s;
  int rc = HK_OK;
  long long enq = 0;
  const size_t status_off = offsetof(SolveState, status);
  for (int k = 0;; ++k) {
    hipError_t e = exec ? hipGraphLaunch(exec, q) : enqueue(q);
    if (e != hipSuccess) {
      set_error_text("krylov solve: launch failed: %s", hipGetErrorString(e));
      rc = HK_EHIP;
      break;
    }
    enq += m;
    e = hipMemcpyAsync(&pin[k & 1], (char*)st + status_off, sizeof(int), hipMemcpyDeviceToHost, q);
    if (e == hipSuccess) e = hipEventRecord(ev[k & 1], q);
    if (e == hipSuccess && k > 0) e = hipEventSynchronize(ev[(k - 1) & 1]);
    if (e != hipSuccess) {
      set_error_text("krylov solve: %s", hipGetErrorString(e));
      rc = HK_EHIP;
      break;
    }
    if (k > 0 && pin[(k - 1) & 1] < S_RUN) break;
    if (enq >= max_iter) break;
  }
  if (cs) {
    // the graph and its stream are released once the last chunk has run
    if (hipStreamSynchronize(cs) != hipSuccess && rc == HK_OK) {
      set_error_text("krylov solve: stream synchronisation failed");
      rc = HK_EHIP;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);
  }
  if (fork) (void)hipEventDestroy(fork);
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  return rc;
}

template <class R>
static int bicgstab(hk_csr_s* A, const cplx<R>* val, const cplx<R>* b, cplx<R>* x,
                    const hk_solve_opts& o, void* wsbase, hk_solve_info* info, hipStream_t s) {
  using V = cplx<R>;
  const int n = (int)A->n;
  const Work<R> wk = carve<R>(wsbase, A->n, A->nnz);
  const dim3 ew((unsigned)((n + kBlock - 1) / kBlock));
  const int gv = ew_blocks(n);

  // set-up: D^-1, Ahat = A D^-1, initial residual
  HK_HIP(hipMemsetAsync(wk.flag, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_diag_inv<V>, ew, dim3(kBlock), 0, s, n, A->rowptr, A->col, val, wk.dinv,
                     o.precond ? 1 : 0, wk.flag);
  HK_CHECK_LAUNCH();
  launch_scale_cols<V>(A->nnz, A->col, val, wk.dinv, wk.ahat, s);
  HK_CHECK_LAUNCH();
  if (o.use_x0) {
    hk_csr_s tmp = *A;
    tmp.val = val;
    int rc = spmv_dispatch(&tmp, x, wk.r, b, nullptr, nullptr, 1, s);
    if (rc != HK_OK) return rc;
  }
  // fused-product shape: one fixed by hk_csr_set_solver_plan or tuned (on
  // the first solve of a tuned handle), else the handle's CSR shape
  SpmvPlan dp = A->plan;
  dp.nw = 0;
  SpmvPlan& cached = A->dot_plan[sizeof(R) == 4 ? 1 : 0];
  if (!cached.tuned && A->plan.tuned) {
    int rc = tune_dot<R>(A, wk, &cached, s);
    if (rc != HK_OK) return rc;
  }
  if (cached.tuned) dp = cached;
  const int gs = dot_grid(A, dp);
  SolveState init{};
  init.history = o.d_history;
  init.status = S_RUN;
  HK_HIP(hipMemcpyAsync(wk.st, &init, sizeof(init), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_init<R>, dim3(gv), dim3(kBlock), 0, s, n, o.use_x0 ? 1 : 0, b, x, wk.dinv,
                     wk.r, wk.rh, wk.p, wk.y, (cplx<R>*)nullptr, wk.partials);
  HK_CHECK_LAUNCH();
  HK_HIP((launch_fin<R, F_INIT>(wk, gv, o.tol, (long long)o.max_iter, s)));
  int hflag = 0;
  HK_HIP(hipMemcpyAsync(&hflag, wk.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HK_HIP(hipStreamSynchronize(s));
  if (hflag) HK_FAIL(HK_EINVAL, "krylov solve: zero diagonal entry (Jacobi undefined)");

  // iterations, in chunks; the status word is read one chunk behind
  int m = o.check_every > 0 ? o.check_every : (n < 200000 ? 64 : 16);
  const int rc = run_chunks(A->pinned, wk.st, m, o.max_iter, s, [&](hipStream_t q) {
    hipError_t e = hipSuccess;
    for (int j = 0; j < m && e == hipSuccess; ++j) {
      hipLaunchKernelGGL(k_p<R>, ew, dim3(kBlock), 0, q, n, wk.st, wk.r, wk.p, wk.v);
      e = hipGetLastError();
      if (e == hipSuccess) e = launch_spmv_dot<R>(A, dp, 1, wk.ahat, wk.p, wk.v, wk.rh, wk, q);
      if (e == hipSuccess) e = launch_fin<R, F_SIGMA>(wk, gs, 0, 0, q);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_s<R>, dim3(gv), dim3(kBlock), 0, q, n, wk.st, wk.r, wk.v, wk.s);
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = launch_spmv_dot<R>(A, dp, 2, wk.ahat, wk.s, wk.t, wk.s, wk, q);
      if (e == hipSuccess) e = launch_fin<R, F_OMEGA>(wk, gs, 0, 0, q);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_xr<R>, dim3(gv), dim3(kBlock), 0, q, n, wk.st, wk.rh, wk.r, wk.p, wk.s,
                           wk.t, wk.y, wk.partials);
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = launch_fin<R, F_XR>(wk, gv, 0, 0, q);
    }
    return e;
  });
  if (rc != HK_OK) return rc;

  return finish_solve<R>(A, val, b, x, wk, info, s);
}

// =================================================================== TFQMR
//
// Right-preconditioned TFQMR (Section 4: P-TFQMR, after Saad's book) on
// Ahat = A D^-1 for y, x = D^-1 y at the end.  Iteration k, in the notation
// of Freund's method (two products with Ahat):
//   alpha = rho / (rhat^H v);  y2 = y1 - alpha v;  u2 = Ahat y2
//   half-step j = 1, 2:  w -= alpha u_j;  d = y_j + (theta^2 eta / alpha) d;
//     theta = ||w|| / tau;  c = (1 + theta^2)^-1/2;  tau *= theta c;
//     eta = c^2 alpha;  y += eta d;  stop when sqrt(m+1) tau <= tol ||b||
//   rho' = rhat^H w;  beta = rho' / rho;  y1 = w + beta y2;  u1 = Ahat y1;
//   v = u1 + beta (u2 + beta v)
// Kernels of one iteration (each reduction followed by its finalize):
//   K_a  : y2 = y1 - alpha v, w -= alpha u1, d = y1 + coef1 d, ||w||^2
//          -> half-step 1 scalars (theta, tau, eta1), stop test
//   K_b  : u2 = Ahat y2 fused with half-step 2: y += eta1 d (the deferred
//          update of half-step 1), w -= alpha u2, d = y2 + coef2 d,
//          ||w||^2, rhat^H w  -> half-step 2 scalars, stop test, rho, beta
//   K_c  : y += eta2 d (or eta1 d after a half-step-1 exit), y1 = w + beta y2
//   K_d  : u1 = Ahat y1 fused with v = u1 + beta (u2 + beta v), rhat^H v
//          -> end of the iteration, alpha and coef1 for the next one
// Workspace roles: w = r, y1 = p, y2 = s, u2 = t, u1 = u, plus d.

// Products of Ahat and x handed row by row to an epilogue E (in the lane
// that owns the row).  E provides: V, NV (partial sums), Pre load(int r)
// (operands of row r, loaded before the product), static Sc scalars(st),
// static bool active(st), and apply(r, pre, acc, sc, part).
template <class E, int L, int U>
__global__ __launch_bounds__(kBlock) void k_fused_lg(int n, int ntiles, const int* __restrict__ rowptr,
                                                     const int* __restrict__ col,
                                                     const typename E::V* __restrict__ val,
                                                     const typename E::V* __restrict__ x, E e,
                                                     const SolveState* __restrict__ st, double* partials) {
  using V = typename E::V;
  constexpr int NV = E::NV;
  __shared__ double lds[NV * (kBlock / kWave)];
  if (!E::active(st)) return;
  const typename E::Sc sc = E::scalars(st);
  constexpr int RT = (kBlock / L) * U;
  const int g = threadIdx.x / L, lane = threadIdx.x & (L - 1);
  double part[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) part[k] = 0;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int r0 = t * RT + g * U;
    const int rw = r0 + (lane < U ? lane : 0);
    const typename E::Pre pre = e.load(rw < n ? rw : n - 1);
    V acc[U];
    csr_rows<L, U, V>(r0, n, rowptr, col, val, x, acc);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (lane == u && r0 + u < n) e.apply(r0 + u, pre, acc[u], sc, part);
  }
  block_sum<NV>(part, lds);
  store_block_partials<NV>(part, partials);
}

template <class E, int RW, int NW, class CI, bool PAIRS>
__global__ __launch_bounds__(NW * kWave) void k_fused_rb(int n, int ntiles, const int* __restrict__ rowptr,
                                                         const CI* __restrict__ col,
                                                         const typename E::V* __restrict__ val,
                                                         const typename E::V* __restrict__ x, E e,
                                                         const SolveState* __restrict__ st, double* partials) {
  using V = typename E::V;
  constexpr int NV = E::NV;
  constexpr int CH = RbCh<RW, V>::v;
  __shared__ V lds[NW * CH * kWave];
  if (!E::active(st)) return;
  const typename E::Sc sc = E::scalars(st);
  V* buf = lds + (threadIdx.x / kWave) * CH * kWave;
  const int l = threadIdx.x & (kWave - 1);
  double part[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) part[k] = 0;
  for (int tb = blockIdx.x; tb < ntiles; tb += gridDim.x) {
    const int t = tile_of(tb, ntiles);
    const int r0 = t * (NW * RW) + (threadIdx.x / kWave) * RW;
    const int r = r0 + l;
    const typename E::Pre pre = e.load(r < n ? r : n - 1);
    V acc;
    if constexpr (PAIRS) acc = csr_block_rows_pairs<RW, CH, V>(r0, n, rowptr, col, val, x, buf);
    else acc = csr_block_rows<RW, CH, V, CI>(r0, n, rowptr, col, val, x, buf);
    if (l < RW && r < n) e.apply(r, pre, acc, sc, part);
  }
  __syncthreads();
  block_sum<NV, double, NW>(part, reinterpret_cast<double*>(lds));
  store_block_partials<NV>(part, partials);
}

template <class E>
static hipError_t launch_fused(const hk_csr_s* A, const SpmvPlan& p, const typename E::V* val,
                               const typename E::V* x, const E& e, const SolveState* st, double* partials,
                               hipStream_t s) {
  int nw = 0;
  const int ntiles = dot_tiles(A, p, &nw);
  const int grid = dot_grid(A, p);
  const int n = (int)A->n;
#define HK_FLG(LL, UU)                                                                               \
  if (p.L == LL && p.U == UU) {                                                                      \
    hipLaunchKernelGGL((k_fused_lg<E, LL, UU>), dim3(grid), dim3(kBlock), 0, s, n, ntiles, A->rowptr, \
                       A->col, val, x, e, st, partials);                                             \
    return hipGetLastError();                                                                        \
  }
  HK_FLG(4, 1) HK_FLG(4, 2) HK_FLG(4, 4)
  HK_FLG(8, 1) HK_FLG(8, 2) HK_FLG(8, 4) HK_FLG(8, 8)
  HK_FLG(16, 1) HK_FLG(16, 2) HK_FLG(16, 4) HK_FLG(16, 8)
  HK_FLG(32, 1) HK_FLG(32, 2) HK_FLG(32, 4) HK_FLG(32, 8)
#undef HK_FLG
#define HK_FRB(RR, NWW)                                                                              \
  if (p.L == kRowBlockL && p.U == RR && nw == NWW) {                                                 \
    if (A->col16 && p.pairs)                                                                         \
      hipLaunchKernelGGL((k_fused_rb<E, RR, NWW, short, true>), dim3(grid), dim3(NWW * kWave), 0, s, \
                         n, ntiles, A->rowptr, (const short*)A->col16, val, x, e, st, partials);     \
    else if (A->col16)                                                                               \
      hipLaunchKernelGGL((k_fused_rb<E, RR, NWW, short, false>), dim3(grid), dim3(NWW * kWave), 0,   \
                         s, n, ntiles, A->rowptr, (const short*)A->col16, val, x, e, st, partials);  \
    else                                                                                             \
      hipLaunchKernelGGL((k_fused_rb<E, RR, NWW, int, false>), dim3(grid), dim3(NWW * kWave), 0, s,  \
                         n, ntiles, A->rowptr, A->col, val, x, e, st, partials);                     \
    return hipGetLastError();                                                                        \
  }
  HK_FRB(16, 2) HK_FRB(32, 2) HK_FRB(64, 2)
  HK_FRB(16, 4) HK_FRB(32, 4) HK_FRB(64, 4)
  HK_FRB(16, 8) HK_FRB(32, 8) HK_FRB(64, 8)
#undef HK_FRB
  return hipErrorInvalidValue;
}

// K_b epilogue: u2 = acc; y += eta1 d; w -= alpha u2; d = y2 + coef2 d;
// partials ||w||^2, rhat^H w.
template <class R> struct EpiTqB {
  using V = cplx<R>;
  static constexpr int NV = 3;
  struct Pre { V w, d, y, rh, y2; };
  struct Sc { V alpha, eta1, coef2; };
  V *w, *d, *y, *u2;
  const V *rh, *y2;
  __device__ static bool active(const SolveState* st) { return st->status == S_RUN; }
  __device__ static Sc scalars(const SolveState* st) {
    return Sc{vscal<V>(st->alpha), vscal<V>(st->tq_eta1), vscal<V>(st->tq_coef2)};
  }
  __device__ Pre load(int r) const { return Pre{w[r], d[r], y[r], rh[r], y2[r]}; }
  __device__ void apply(int r, const Pre& q, V acc, const Sc& c, double (&part)[NV]) const {
    u2[r] = acc;
    y[r] = cfma(c.eta1, q.d, q.y);
    const V wn = csub(q.w, cmul(c.alpha, acc));
    w[r] = wn;
    d[r] = cfma(c.coef2, q.d, q.y2);
    part[0] += nrm2d(wn);
    dotc_acc(q.rh, wn, part[1], part[2]);
  }
};

// K_d epilogue: u1 = acc; v = u1 + beta (u2 + beta v) (v = u1 on the first
// product, INIT); partials rhat^H v.
template <class R, int INIT> struct EpiTqD {
  using V = cplx<R>;
  static constexpr int NV = 2;
  struct Pre { V u2, v, rh; };
  struct Sc { V beta; };
  V *u1, *v;
  const V *u2, *rh;
  __device__ static bool active(const SolveState* st) { return st->status == S_RUN; }
  __device__ static Sc scalars(const SolveState* st) { return Sc{vscal<V>(st->beta)}; }
  __device__ Pre load(int r) const {
    if (INIT) return Pre{czero<V>(), czero<V>(), rh[r]};
    return Pre{u2[r], v[r], rh[r]};
  }
  __device__ void apply(int r, const Pre& q, V acc, const Sc& c, double (&part)[NV]) const {
    u1[r] = acc;
    const V vn = INIT ? acc : cfma(c.beta, cfma(c.beta, q.v, q.u2), acc);
    v[r] = vn;
    dotc_acc(q.rh, vn, part[0], part[1]);
  }
};

// K_a: y2 = y1 - alpha v; w -= alpha u1; d = y1 + coef1 d; partials ||w||^2.
template <class R>
__global__ __launch_bounds__(kBlock) void k_tq_a(int n, const SolveState* __restrict__ st,
                                                 const cplx<R>* __restrict__ y1, const cplx<R>* __restrict__ v,
                                                 const cplx<R>* __restrict__ u1, cplx<R>* __restrict__ y2,
                                                 cplx<R>* __restrict__ w, cplx<R>* __restrict__ d,
                                                 double* partials) {
  using V = cplx<R>;
  __shared__ double lds[kBlock / kWave];
  if (st->status != S_RUN) return;
  const V alpha = vscal<V>(st->alpha), coef = vscal<V>(st->tq_coef1);
  double acc[1] = {0};
  const int base = blockIdx.x * (kBlock * kEw) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kEw; ++k) {
    const int i = base + k * kBlock;
    if (i >= n) break;
    const V y1i = y1[i], vi = v[i], ui = u1[i], wi = w[i], di = d[i];
    y2[i] = csub(y1i, cmul(alpha, vi));
    const V wn = csub(wi, cmul(alpha, ui));
    w[i] = wn;
    d[i] = cfma(coef, di, y1i);
    acc[0] += nrm2d(wn);
  }
  block_sum<1>(acc, lds);
  store_block_partials<1>(acc, partials);
}

// K_c: the deferred x update of the iteration's last half-step (y += eta d)
// and, while running, y1 = w + beta y2.
template <class R>
__global__ __launch_bounds__(kBlock) void k_tq_c(int n, const SolveState* __restrict__ st,
                                                 const cplx<R>* __restrict__ w, const cplx<R>* __restrict__ y2,
                                                 const cplx<R>* __restrict__ d, cplx<R>* __restrict__ y,
                                                 cplx<R>* __restrict__ y1) {
  using V = cplx<R>;
  const int status = st->status;
  if (status != S_RUN && status != S_HALF && status != S_HALF2 && status != S_RHOBD) return;
  const V eta = vscal<V>(status == S_HALF ? st->tq_eta1 : st->tq_eta2), beta = vscal<V>(st->beta);
  const int base = blockIdx.x * (kBlock * kEw) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kEw; ++k) {
    const int i = base + k * kBlock;
    if (i >= n) break;
    y[i] = cfma(eta, d[i], y[i]);
    if (status == S_RUN) y1[i] = cfma(beta, y2[i], w[i]);
  }
}

enum : int { TQ_INIT = 0, TQ_SIGMA0 = 1, TQ_H1 = 2, TQ_H2 = 3, TQ_SIGMA = 4 };
template <int F> struct TqNV { static constexpr int v = 2; };
template <> struct TqNV<TQ_H1> { static constexpr int v = 1; };
template <> struct TqNV<TQ_H2> { static constexpr int v = 3; };

// One workgroup: sums the partials of the preceding kernel and applies the
// TFQMR scalar step F.
template <int F, int BS>
__global__ __launch_bounds__(BS) void k_tq_fin(SolveState* st, const double* partials, int nb, double tol,
                                                      long long maxit) {
  using V = double2;
  constexpr int NV = TqNV<F>::v;
  __shared__ double lds[NV * (BS / kWave)];
  // As in k_fin: the status and the fields the update reads are loaded before
  // the sum, which runs whatever the status.
  const int status = st->status;
  const long long k = st->iter, maxit0 = st->maxit;
  const V rho0 = st->rho, alpha0 = st->alpha, eta20 = st->tq_eta2;
  const double theta0 = st->tq_theta, tau0 = st->tq_tau, theta2 = st->theta2, bb = st->bb;
  double* const history = st->history;
  double tot[NV];
  final_sum<NV, double, BS>(partials, nb, tot, lds);
  if (F == TQ_H1 && status != S_RUN) return;
  if (F == TQ_H2 && status != S_RUN) return;
  if (F == TQ_SIGMA0 && status != S_RUN) return;
  if (F == TQ_SIGMA) {
    if (status == S_HALF || status == S_HALF2 || status == S_RHOBD) {
      if (threadIdx.x == 0) {
        st->status = status == S_RHOBD ? HK_BREAKDOWN : HK_OK;
        if (status == S_RHOBD) st->bd = HK_BD_RHO;
      }
      return;
    }
    if (status != S_RUN) return;
  }
  if (threadIdx.x != 0) return;
  if (F == TQ_INIT) {
    st->bb = tot[0];
    st->rr = tot[1];
    st->theta2 = tol * tol * tot[0];
    st->rho = cmake<V>(tot[1], 0);
    st->tq_tau = sqrt(tot[1]);
    st->tq_theta = 0;
    st->tq_eta1 = st->tq_eta2 = st->tq_coef1 = st->tq_coef2 = czero<V>();
    st->alpha = st->beta = czero<V>();
    st->iter = 1;
    st->maxit = maxit;
    st->iters_done = 0;
    st->bd = HK_BD_NONE;
    if (!isfinite(tot[0]) || !isfinite(tot[1])) st->status = HK_NONFINITE;
    else if (tot[1] <= st->theta2) st->status = HK_OK;
    else if (maxit <= 0) st->status = HK_NOT_CONVERGED;
    else st->status = S_RUN;
    if (st->history) st->history[0] = tot[0] > 0 ? sqrt(tot[1] / tot[0]) : 0.0;
  } else if (F == TQ_SIGMA0 || F == TQ_SIGMA) {
    long long it = k;
    if (F == TQ_SIGMA) {
      // the iteration ended without an exit
      if (k >= maxit0) { st->status = HK_NOT_CONVERGED; st->iters_done = k; return; }
      it = k + 1;
      st->iter = it;
    }
    const V sigma = cmake<V>(tot[0], tot[1]);
    if (!cfinite(sigma)) {
      st->status = HK_NONFINITE;
      st->iters_done = it - 1;
    } else if (sigma.x == 0 && sigma.y == 0) {
      st->status = HK_BREAKDOWN;
      st->bd = HK_BD_SIGMA;
      st->iters_done = it - 1;
    } else {
      const V alpha = cdiv(rho0, sigma);
      st->alpha = alpha;
      st->tq_coef1 = cdiv(cmul(cmake<V>(theta0 * theta0, 0), eta20), alpha);
    }
  } else {  // TQ_H1, TQ_H2: a half-step's theta, tau, eta and stop test
    const double theta = sqrt(tot[0]) / tau0;
    const double c = 1.0 / sqrt(1.0 + theta * theta);
    const double tau = tau0 * theta * c;
    const V alpha = alpha0;
    const V eta = cmake<V>(c * c * alpha.x, c * c * alpha.y);
    st->tq_theta = theta;
    st->tq_tau = tau;
    const long long m = F == TQ_H1 ? 2 * k - 1 : 2 * k;  // half-step index, from 1
    const double bound = tau * sqrt((double)(m + 1));
    st->rr = bound * bound;
    if (history) history[k] = bb > 0 ? bound / sqrt(bb) : 0.0;
    if (F == TQ_H1) {
      st->tq_eta1 = eta;
      st->tq_coef2 = cdiv(cmul(cmake<V>(theta * theta, 0), eta), alpha);
    } else {
      st->tq_eta2 = eta;
    }
    if (!isfinite(tau) || !cfinite(eta)) {
      st->status = HK_NONFINITE;
      st->iters_done = k;
    } else if (bound * bound <= theta2) {
      st->status = F == TQ_H1 ? S_HALF : S_HALF2;
      st->iters_done = k;
    } else if (F == TQ_H2) {
      const V rho = cmake<V>(tot[1], tot[2]);
      st->iters_done = k;
      if (!cfinite(rho)) {
        st->status = HK_NONFINITE;
      } else if (rho.x == 0 && rho.y == 0) {
        st->status = S_RHOBD;
      } else {
        st->beta = cdiv(rho, rho0);
        st->rho = rho;
      }
    }
  }
}

template <int F>
static hipError_t launch_tq_fin(SolveState* st, const double* partials, int nb, double tol, long long maxit,
                                hipStream_t s) {
  if (nb <= kFinSmallNb)
    hipLaunchKernelGGL((k_tq_fin<F, kFinBlockSmall>), dim3(1), dim3(kFinBlockSmall), 0, s, st, partials, nb, tol,
                       maxit);
  else
    hipLaunchKernelGGL((k_tq_fin<F, kFinBlock>), dim3(1), dim3(kFinBlock), 0, s, st, partials, nb, tol, maxit);
  return hipGetLastError();
}

// Whole TFQMR solve (complex128), the same contract as bicgstab<R>.
static int tfqmr(hk_csr_s* A, const double2* val, const double2* b, double2* x, const hk_solve_opts& o,
                 void* wsbase, hk_solve_info* info, hipStream_t s) {
  using R = double;
  using V = double2;
  const int n = (int)A->n;
  const Work<R> wk = carve<R>(wsbase, A->n, A->nnz);
  const dim3 ew((unsigned)((n + kBlock - 1) / kBlock));
  const int gv = ew_blocks(n);
  V *w = wk.r, *y1 = wk.p, *y2 = wk.s, *u2 = wk.t, *u1 = wk.u, *d = wk.d, *v = wk.v;

  HK_HIP(hipMemsetAsync(wk.flag, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_diag_inv<V>, ew, dim3(kBlock), 0, s, n, A->rowptr, A->col, val, wk.dinv,
                     o.precond ? 1 : 0, wk.flag);
  HK_CHECK_LAUNCH();
  launch_scale_cols<V>(A->nnz, A->col, val, wk.dinv, wk.ahat, s);
  HK_CHECK_LAUNCH();
  if (o.use_x0) {
    hk_csr_s tmp = *A;
    tmp.val = val;
    int rc = spmv_dispatch(&tmp, x, wk.r, b, nullptr, nullptr, 1, s);
    if (rc != HK_OK) return rc;
  }
  SpmvPlan dp = A->plan;
  dp.nw = 0;
  SpmvPlan& cached = A->dot_plan[0];
  if (!cached.tuned && A->plan.tuned) {
    int rc = tune_dot<R>(A, wk, &cached, s);
    if (rc != HK_OK) return rc;
  }
  if (cached.tuned) dp = cached;
  const int gs = dot_grid(A, dp);
  SolveState init{};
  init.history = o.d_history;
  init.status = S_RUN;
  HK_HIP(hipMemcpyAsync(wk.st, &init, sizeof(init), hipMemcpyHostToDevice, s));
  // w = r0, rhat = y1 = r0, y = x0 / dinv or 0, d = 0
  hipLaunchKernelGGL(k_init<R>, dim3(gv), dim3(kBlock), 0, s, n, o.use_x0 ? 1 : 0, b, x, wk.dinv, w, wk.rh,
                     y1, wk.y, d, wk.partials);
  HK_CHECK_LAUNCH();
  HK_HIP(launch_tq_fin<TQ_INIT>(wk.st, wk.partials, gv, o.tol, (long long)o.max_iter, s));
  {
    EpiTqD<R, 1> e0{u1, v, u2, wk.rh};
    HK_HIP(launch_fused(A, dp, wk.ahat, y1, e0, wk.st, wk.partials, s));
    HK_HIP(launch_tq_fin<TQ_SIGMA0>(wk.st, wk.partials, gs, 0, 0, s));
  }
  int hflag = 0;
  HK_HIP(hipMemcpyAsync(&hflag, wk.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HK_HIP(hipStreamSynchronize(s));
  if (hflag) HK_FAIL(HK_EINVAL, "krylov solve: zero diagonal entry (Jacobi undefined)");

  const EpiTqB<R> eb{w, d, wk.y, u2, wk.rh, y2};
  const EpiTqD<R, 0> ed{u1, v, u2, wk.rh};
  int m = o.check_every > 0 ? o.check_every : (n < 200000 ? 64 : 16);
  const int rc = run_chunks(A->pinned, wk.st, m, o.max_iter, s, [&](hipStream_t q) {
    hipError_t e = hipSuccess;
    for (int j = 0; j < m && e == hipSuccess; ++j) {
      hipLaunchKernelGGL(k_tq_a<R>, dim3(gv), dim3(kBlock), 0, q, n, wk.st, y1, v, u1, y2, w, d, wk.partials);
      e = hipGetLastError();
      if (e == hipSuccess) e = launch_tq_fin<TQ_H1>(wk.st, wk.partials, gv, 0, 0, q);
      if (e == hipSuccess) e = launch_fused(A, dp, wk.ahat, y2, eb, wk.st, wk.partials, q);
      if (e == hipSuccess) e = launch_tq_fin<TQ_H2>(wk.st, wk.partials, gs, 0, 0, q);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_tq_c<R>, dim3(gv), dim3(kBlock), 0, q, n, wk.st, w, y2, d, wk.y, y1);
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = launch_fused(A, dp, wk.ahat, y1, ed, wk.st, wk.partials, q);
      if (e == hipSuccess) e = launch_tq_fin<TQ_SIGMA>(wk.st, wk.partials, gs, 0, 0, q);
    }
    return e;
  });
  if (rc != HK_OK) return rc;
  return finish_solve<R>(A, val, b, x, wk, info, s);
}

// ============================================================ BiCGStab(l)
//
// Right-preconditioned BiCGStab(l) (Section 4: P-BiCGSTAB(l), l = 8 in the
// paper; Sleijpen and Fokkema's method) on Ahat = A D^-1 for y, x = D^-1 y.
// A cycle (one iteration) is l BiCG steps and a minimal-residual step:
//   step j: beta (from rho) -> u_i = r_i - beta u_i (i <= j)      [k_bl_u]
//           u_{j+1} = Ahat u_j, rt^H u_{j+1} -> alpha             [fused]
//           r_i -= alpha u_{i+1} (i <= j), y += alpha u_0, ||r_0||^2
//             -> stop test                                         [k_bl_r]
//           r_{j+1} = Ahat r_j, rt^H r_{j+1} -> rho, beta          [fused]
//   MR:     Z_ij = r_i^H r_j, z_i = r_i^H r_0 (i, j = 1..l) in one pass
//             -> gamma = Z^-1 z by Cholesky (one thread)           [k_bl_gram]
//           y += sum gamma_j r_{j-1}, r_0 -= sum gamma_j r_j,
//           u_0 -= sum gamma_j u_j; ||r_0||^2, rt^H r_0
//             -> stop test, omega = gamma_l, next cycle's rho, beta [k_bl_mr]
// The minimal-residual coefficients come from the normal equations of the
// Gram matrix (one multi-vector reduction on the GPU) rather than modified
// Gram-Schmidt (l(l+1)/2 dependent reductions); the oracle uses the same
// form and its pins tie it to the Gram-Schmidt form.

constexpr int kMaxEll = 8;
template <class R> struct BlVecs {
  cplx<R>* r[kMaxEll + 1];
  cplx<R>* u[kMaxEll + 1];
};

template <int ELL> struct BlNV { static constexpr int v = 2 * (ELL + ELL * (ELL + 1) / 2); };

template <class R> struct BlWork {
  using V = cplx<R>;
  V *y, *rt, *dinv, *ahat;
  BlVecs<R> vec;
  double* partials;
  SolveState* st;
  int* flag;
};

template <class R> static size_t bl_partial_doubles(int64_t n) {
  const int64_t gv = ew_blocks(n);
  const int64_t a = 4 * partial_slots(n), b = (int64_t)BlNV<kMaxEll>::v * gv;
  return (size_t)(a > b ? a : b);
}

// One layout for sizing and carving, as for the BiCGStab/TFQMR workspace.
template <class R, class Take> static BlWork<R> bl_layout(Take take, int64_t n, int64_t nnz, int ell) {
  using V = cplx<R>;
  BlWork<R> w{};
  w.y = (V*)take(sizeof(V) * n);
  w.rt = (V*)take(sizeof(V) * n);
  w.dinv = (V*)take(sizeof(V) * n);
  for (int j = 0; j <= ell; ++j) {
    w.vec.r[j] = (V*)take(sizeof(V) * n);
    w.vec.u[j] = (V*)take(sizeof(V) * n);
  }
  w.ahat = (V*)take(sizeof(V) * (nnz + 1));  // one padding entry (paired-entry products)
  w.partials = (double*)take(sizeof(double) * bl_partial_doubles<R>(n));
  w.st = (SolveState*)take(sizeof(SolveState));
  w.flag = (int*)take(64);
  return w;
}

template <class R> static size_t bl_work_bytes(int64_t n, int64_t nnz, int ell) {
  size_t q = 0;
  (void)bl_layout<R>([&](size_t bytes) { q += align_up(bytes); return (char*)nullptr; }, n, nnz, ell);
  return q;
}

template <class R> static BlWork<R> bl_carve(void* base, int64_t n, int64_t nnz, int ell) {
  char* q = static_cast<char*>(base);
  return bl_layout<R>([&](size_t bytes) { char* r = q; q += align_up(bytes); return r; }, n, nnz, ell);
}

// u_i = r_i - beta u_i, i = 0..j
template <class R>
__global__ __launch_bounds__(kBlock) void k_bl_u(int n, const SolveState* __restrict__ st, int j, BlVecs<R> v) {
  using V = cplx<R>;
  if (st->status != S_RUN) return;
  const V beta = vscal<V>(st->beta);
  const int base = blockIdx.x * (kBlock * kEw) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kEw; ++k) {
    const int q = base + k * kBlock;
    if (q >= n) break;
    for (int i = 0; i <= j; ++i) v.u[i][q] = csub(v.r[i][q], cmul(beta, v.u[i][q]));
  }
}

// r_i -= alpha u_{i+1} (i = 0..j); y += alpha u_0; partials ||r_0||^2
template <class R>
__global__ __launch_bounds__(kBlock) void k_bl_r(int n, const SolveState* __restrict__ st, int j, BlVecs<R> v,
                                                 cplx<R>* __restrict__ y, double* partials) {
  using V = cplx<R>;
  __shared__ double lds[kBlock / kWave];
  if (st->status != S_RUN) return;
  const V alpha = vscal<V>(st->alpha);
  double acc[1] = {0};
  const int base = blockIdx.x * (kBlock * kEw) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kEw; ++k) {
    const int q = base + k * kBlock;
    if (q >= n) break;
    for (int i = 0; i <= j; ++i) v.r[i][q] = csub(v.r[i][q], cmul(alpha, v.u[i + 1][q]));
    y[q] = cfma(alpha, v.u[0][q], y[q]);
    acc[0] += nrm2d(v.r[0][q]);
  }
  block_sum<1>(acc, lds);
  store_block_partials<1>(acc, partials);
}

// Products of the minimal-residual step, in partial-component order: first
// z_i = r_i^H r_0 (i = 1..l), then Z_ij = r_i^H r_j (1 <= i <= j <= l).
template <int ELL> struct BlProducts {
  static constexpr int np = ELL + ELL * (ELL + 1) / 2;
  int a[np], b[np];
  constexpr BlProducts() : a(), b() {
    int m = 0;
    for (int i = 1; i <= ELL; ++i, ++m) { a[m] = i; b[m] = 0; }
    for (int i = 1; i <= ELL; ++i)
      for (int j = i; j <= ELL; ++j, ++m) { a[m] = i; b[m] = j; }
  }
};

// Gram partials.  Wave w of a workgroup accumulates products m = w, w + NW,
// ... over the workgroup's kBlock*kEw elements, so a lane holds a quarter of
// the products instead of all of them (88 doubles at l = 8, which left one
// wave per SIMD).  The waves of a workgroup load the same elements at about
// the same time, so HBM sees each once and the repeats hit the caches.  Each
// wave owns its products: its lane 0 stores their block partials directly.
template <class R, int ELL>
__global__ __launch_bounds__(kBlock) void k_bl_gram(int n, const SolveState* __restrict__ st, BlVecs<R> v,
                                                    double* partials) {
  using V = cplx<R>;
  constexpr BlProducts<ELL> P{};
  constexpr int NW = kBlock / kWave;
  constexpr int PW = (P.np + NW - 1) / NW;  // products per wave (at most)
  if (st->status != S_RUN) return;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  double acc[2 * PW];
#pragma unroll
  for (int k = 0; k < 2 * PW; ++k) acc[k] = 0;
  const int base = blockIdx.x * (kBlock * kEw);
  for (int e = lane; e < kBlock * kEw; e += kWave) {
    const int q = base + e;
    if (q >= n) break;
    V x[ELL + 1];
#pragma unroll
    for (int i = 0; i <= ELL; ++i) x[i] = v.r[i][q];
    // wave w's products; the branch is uniform over the wave
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) {
      if (ww != w) continue;
#pragma unroll
      for (int p = 0; p < PW; ++p) {
        const int m = ww + p * NW;
        if (m < P.np) dotc_acc(x[P.a[m]], x[P.b[m]], acc[2 * p], acc[2 * p + 1]);
      }
    }
  }
#pragma unroll
  for (int p = 0; p < PW; ++p) {
    const int m = w + p * NW;
    const double re = wave_sum(acc[2 * p]), im = wave_sum(acc[2 * p + 1]);
    if (lane == 0 && m < P.np) {
      partials[(size_t)(2 * m) * gridDim.x + blockIdx.x] = re;
      partials[(size_t)(2 * m + 1) * gridDim.x + blockIdx.x] = im;
    }
  }
}

// y += sum gamma_j r_{j-1}; r_0 -= sum gamma_j r_j; u_0 -= sum gamma_j u_j;
// partials ||r_0||^2, rt^H r_0
template <class R, int ELL>
__global__ __launch_bounds__(kBlock) void k_bl_mr(int n, const SolveState* __restrict__ st, BlVecs<R> v,
                                                  cplx<R>* __restrict__ y, const cplx<R>* __restrict__ rt,
                                                  double* partials) {
  using V = cplx<R>;
  __shared__ double lds[3 * (kBlock / kWave)];
  if (st->status != S_RUN) return;
  V g[ELL];
#pragma unroll
  for (int j = 0; j < ELL; ++j) g[j] = vscal<V>(st->bl_gamma[j]);
  double acc[3] = {0, 0, 0};
  const int base = blockIdx.x * (kBlock * kEw) + threadIdx.x;
  for (int k = 0; k < kEw; ++k) {
    const int q = base + k * kBlock;
    if (q >= n) break;
    V yq = y[q], r0 = v.r[0][q], u0 = v.u[0][q];
    V rprev = r0;
#pragma unroll
    for (int j = 1; j <= ELL; ++j) {
      const V rj = v.r[j][q];
      yq = cfma(g[j - 1], rprev, yq);
      r0 = csub(r0, cmul(g[j - 1], rj));
      u0 = csub(u0, cmul(g[j - 1], v.u[j][q]));
      rprev = rj;
    }
    y[q] = yq;
    v.r[0][q] = r0;
    v.u[0][q] = u0;
    acc[0] += nrm2d(r0);
    dotc_acc(rt[q], r0, acc[1], acc[2]);
  }
  block_sum<3>(acc, lds);
  store_block_partials<3>(acc, partials);
}

// out = Ahat x (fused product); partials rt^H out
template <class R> struct EpiStoreDot {
  using V = cplx<R>;
  static constexpr int NV = 2;
  struct Pre { V rt; };
  struct Sc {};
  V* out;
  const V* rt;
  __device__ static bool active(const SolveState* st) { return st->status == S_RUN; }
  __device__ static Sc scalars(const SolveState*) { return Sc{}; }
  __device__ Pre load(int r) const { return Pre{rt[r]}; }
  __device__ void apply(int r, const Pre& q, V acc, const Sc&, double (&part)[NV]) const {
    out[r] = acc;
    dotc_acc(q.rt, acc, part[0], part[1]);
  }
};

enum : int { BL_INIT = 0, BL_ALPHA = 1, BL_R = 2, BL_RHO = 3, BL_MR = 5 };
template <int F, int ELL> struct BlFinNV { static constexpr int v = 2; };
template <int ELL> struct BlFinNV<BL_R, ELL> { static constexpr int v = 1; };
template <int ELL> struct BlFinNV<BL_MR, ELL> { static constexpr int v = 3; };

// Start of a BiCG sequence with rho1 = rt^H r_0: rho0 = -omega rho0 at the
// cycle start, then beta = alpha rho1 / rho0, rho0 = rho1.  (rho0 is kept in
// rho, rho1 arrives in tot.)
__device__ __forceinline__ void bl_cycle_start(SolveState* st, double2 rho1) {
  const double2 rho0 = cmul(cmake<double2>(-1, 0), cmul(st->omega, st->rho));
  if (!cfinite(rho1)) {
    st->status = HK_NONFINITE;
    st->iters_done = st->iter - 1;
  } else if (rho1.x == 0 && rho1.y == 0) {
    st->status = HK_BREAKDOWN;
    st->bd = HK_BD_RHO;
    st->iters_done = st->iter - 1;
  } else {
    st->beta = cdiv(cmul(st->alpha, rho1), rho0);
    st->rho = rho1;
  }
}

template <int F, int ELL, int BS>
__global__ __launch_bounds__(BS) void k_bl_fin(SolveState* st, const double* partials, int nb, double tol,
                                                      long long maxit) {
  using V = double2;
  constexpr int NV = BlFinNV<F, ELL>::v;
  __shared__ double lds[NV * (BS / kWave)];
  // As in k_fin: the status and the fields the update reads are loaded before
  // the sum, which runs whatever the status.
  const int status = st->status;
  const long long k = st->iter, maxit0 = st->maxit;
  const V rho0 = st->rho, alpha0 = st->alpha, omega0 = st->omega;
  const double theta2 = st->theta2, bb = st->bb;
  double* const history = st->history;
  double tot[NV];
  final_sum<NV, double, BS>(partials, nb, tot, lds);
  if (F != BL_INIT && status != S_RUN) return;
  if (threadIdx.x != 0) return;
  if (F == BL_INIT) {
    st->bb = tot[0];
    st->rr = tot[1];
    st->theta2 = tol * tol * tot[0];
    st->alpha = czero<V>();
    st->omega = cmake<V>(1, 0);
    st->rho = cmake<V>(1, 0);
    st->iter = 1;
    st->maxit = maxit;
    st->iters_done = 0;
    st->bd = HK_BD_NONE;
    if (st->history) st->history[0] = tot[0] > 0 ? sqrt(tot[1] / tot[0]) : 0.0;
    if (!isfinite(tot[0]) || !isfinite(tot[1])) st->status = HK_NONFINITE;
    else if (tot[1] <= st->theta2) st->status = HK_OK;
    else if (maxit <= 0) st->status = HK_NOT_CONVERGED;
    else { st->status = S_RUN; bl_cycle_start(st, cmake<V>(tot[1], 0)); }
  } else if (F == BL_ALPHA) {
    const V gam = cmake<V>(tot[0], tot[1]);
    if (!cfinite(gam)) { st->status = HK_NONFINITE; st->iters_done = k - 1; }
    else if (gam.x == 0 && gam.y == 0) { st->status = HK_BREAKDOWN; st->bd = HK_BD_SIGMA; st->iters_done = k - 1; }
    else st->alpha = cdiv(rho0, gam);
  } else if (F == BL_R) {
    st->rr = tot[0];
    if (!isfinite(tot[0])) { st->status = HK_NONFINITE; st->iters_done = k; }
    else if (tot[0] <= theta2) {
      st->status = HK_OK;
      st->iters_done = k;
      if (history) history[k] = bb > 0 ? sqrt(tot[0] / bb) : 0.0;
    }
  } else if (F == BL_RHO) {
    const V rho1 = cmake<V>(tot[0], tot[1]);
    if (!cfinite(rho1)) { st->status = HK_NONFINITE; st->iters_done = k - 1; }
    else if (rho1.x == 0 && rho1.y == 0) { st->status = HK_BREAKDOWN; st->bd = HK_BD_RHO; st->iters_done = k - 1; }
    else { st->beta = cdiv(cmul(alpha0, rho1), rho0); st->rho = rho1; }
  } else {  // BL_MR: end of a cycle
    st->rr = tot[0];
    st->iters_done = k;
    if (history) history[k] = bb > 0 ? sqrt(tot[0] / bb) : 0.0;
    const V om = omega0;
    if (!isfinite(tot[0])) st->status = HK_NONFINITE;
    else if (tot[0] <= theta2) st->status = HK_OK;
    else if (om.x == 0 && om.y == 0) { st->status = HK_BREAKDOWN; st->bd = HK_BD_OMEGA; }
    else if (k >= maxit0) st->status = HK_NOT_CONVERGED;
    else { st->iter = k + 1; bl_cycle_start(st, cmake<V>(tot[1], tot[2])); }
  }
}

// Finalize of the Gram partials (NV = l(l+3) sums): wave w sums components
// w, w+16, ... over the nb partials (lane j takes partials j, j+64, ... in
// order, then a fixed butterfly), into LDS; thread 0 then solves Z gamma = z
// by Cholesky.  A lane issues the loads of U partials of each of its
// components before adding them, so the latency is paid once per 64*U
// partials rather than once per 64.
template <int ELL>
__global__ __launch_bounds__(kFinBlock) void k_bl_fin_gram(SolveState* st, const double* partials, int nb) {
  using V = double2;
  constexpr int NV = BlNV<ELL>::v;
  constexpr int W = kFinBlock / kWave;
  constexpr int CW = (NV + W - 1) / W;  // components per wave (at most)
  constexpr int U = 4;                  // CW*U loads in flight per lane, within 128 VGPRs
  __shared__ double tot[NV];
  // the status is checked after the sum, so the two loads overlap
  const int status = st->status;
  const long long k = st->iter;
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  double sacc[CW];
#pragma unroll
  for (int q = 0; q < CW; ++q) sacc[q] = 0;
  for (int j0 = lane; j0 < nb; j0 += kWave * U) {
    double x[CW][U];
#pragma unroll
    for (int q = 0; q < CW; ++q)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = wv + q * W, j = j0 + u * kWave;
        x[q][u] = c < NV && j < nb ? partials[(size_t)c * nb + j] : 0.0;
      }
#pragma unroll
    for (int q = 0; q < CW; ++q)
#pragma unroll
      for (int u = 0; u < U; ++u) sacc[q] += x[q][u];
  }
#pragma unroll
  for (int q = 0; q < CW; ++q) {
    const int c = wv + q * W;
    const double t = wave_sum(sacc[q]);
    if (lane == 0 && c < NV) tot[c] = t;
  }
  __syncthreads();
  if (status != S_RUN || threadIdx.x != 0) return;
  {
    // Z gamma = z by Cholesky, Z = L L^H (Hermitian positive definite).  The
    // arrays are in LDS: as thread-private arrays they were placed in scratch
    // memory, and the dependent scratch accesses made this kernel take ~90 us.
    __shared__ V z[ELL], Z[ELL][ELL], L[ELL][ELL], w[ELL], g[ELL];
    __shared__ double rl[ELL];  // 1 / L_jj: one division per column
    int m = 0;
    for (int i = 0; i < ELL; ++i, m += 2) z[i] = cmake<V>(tot[m], tot[m + 1]);
    for (int i = 0; i < ELL; ++i)
      for (int j = i; j < ELL; ++j, m += 2) {
        Z[i][j] = cmake<V>(tot[m], tot[m + 1]);
        Z[j][i] = cconj(Z[i][j]);
      }
#pragma unroll 1
    for (int j = 0; j < ELL; ++j) {
      double d = Z[j][j].x;
      for (int q = 0; q < j; ++q) d -= cabs2(L[j][q]);
      if (!(d > 0.0)) { st->status = HK_BREAKDOWN; st->bd = HK_BD_TAU; st->iters_done = k; return; }
      const double ljj = sqrt(d), rj = 1.0 / ljj;
      L[j][j] = cmake<V>(ljj, 0);
      rl[j] = rj;
#pragma unroll 1
      for (int i = j + 1; i < ELL; ++i) {
        V sij = Z[i][j];
        for (int q = 0; q < j; ++q) sij = csub(sij, cmul(L[i][q], cconj(L[j][q])));
        L[i][j] = cmake<V>(sij.x * rj, sij.y * rj);
      }
    }
#pragma unroll 1
    for (int i = 0; i < ELL; ++i) {
      V sum = z[i];
      for (int q = 0; q < i; ++q) sum = csub(sum, cmul(L[i][q], w[q]));
      w[i] = cmake<V>(sum.x * rl[i], sum.y * rl[i]);
    }
#pragma unroll 1
    for (int i = ELL - 1; i >= 0; --i) {
      V sum = w[i];
      for (int q = i + 1; q < ELL; ++q) sum = csub(sum, cmul(cconj(L[q][i]), g[q]));
      g[i] = cmake<V>(sum.x * rl[i], sum.y * rl[i]);
    }
    for (int i = 0; i < ELL; ++i) st->bl_gamma[i] = g[i];
    st->omega = g[ELL - 1];
    if (!cfinite(st->omega)) { st->status = HK_NONFINITE; st->iters_done = k; }
  }
}

template <int F, int ELL>
static hipError_t launch_bl_fin(SolveState* st, const double* partials, int nb, double tol, long long maxit,
                                hipStream_t s) {
  if (nb <= kFinSmallNb)
    hipLaunchKernelGGL((k_bl_fin<F, ELL, kFinBlockSmall>), dim3(1), dim3(kFinBlockSmall), 0, s, st, partials, nb,
                       tol, maxit);
  else
    hipLaunchKernelGGL((k_bl_fin<F, ELL, kFinBlock>), dim3(1), dim3(kFinBlock), 0, s, st, partials, nb, tol, maxit);
  return hipGetLastError();
}

// Whole BiCGStab(ELL) solve (complex128), the same contract as bicgstab<R>.
template <int ELL>
static int bicgstab_l(hk_csr_s* A, const double2* val, const double2* b, double2* x, const hk_solve_opts& o,
                      void* wsbase, hk_solve_info* info, hipStream_t s) {
  using R = double;
  using V = double2;
  const int n = (int)A->n;
  const BlWork<R> wk = bl_carve<R>(wsbase, A->n, A->nnz, ELL);
  const dim3 ew((unsigned)((n + kBlock - 1) / kBlock));
  const int gv = ew_blocks(n);

  HK_HIP(hipMemsetAsync(wk.flag, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_diag_inv<V>, ew, dim3(kBlock), 0, s, n, A->rowptr, A->col, val, wk.dinv,
                     o.precond ? 1 : 0, wk.flag);
  HK_CHECK_LAUNCH();
  launch_scale_cols<V>(A->nnz, A->col, val, wk.dinv, wk.ahat, s);
  HK_CHECK_LAUNCH();
  if (o.use_x0) {
    hk_csr_s tmp = *A;
    tmp.val = val;
    int rc = spmv_dispatch(&tmp, x, wk.vec.r[0], b, nullptr, nullptr, 1, s);
    if (rc != HK_OK) return rc;
  }
  SpmvPlan dp = A->plan;
  dp.nw = 0;
  SpmvPlan& cached = A->dot_plan[0];
  if (!cached.tuned && A->plan.tuned) {
    // the workspace vectors serve as tuning operands before the solve starts
    Work<R> tv{};
    tv.ahat = wk.ahat;
    tv.p = wk.vec.r[1];
    tv.v = wk.vec.u[1];
    tv.rh = wk.rt;
    tv.partials = wk.partials;
    tv.st = wk.st;
    int rc = tune_dot<R>(A, tv, &cached, s);
    if (rc != HK_OK) return rc;
  }
  if (cached.tuned) dp = cached;
  const int gs = dot_grid(A, dp);
  SolveState init{};
  init.history = o.d_history;
  init.status = S_RUN;
  HK_HIP(hipMemcpyAsync(wk.st, &init, sizeof(init), hipMemcpyHostToDevice, s));
  // r_0 = b - A x0, rt = r_0, y = x0 / dinv or 0, u_0 = 0
  hipLaunchKernelGGL(k_init<R>, dim3(gv), dim3(kBlock), 0, s, n, o.use_x0 ? 1 : 0, b, x, wk.dinv, wk.vec.r[0],
                     wk.rt, wk.vec.u[1], wk.y, wk.vec.u[0], wk.partials);
  HK_CHECK_LAUNCH();
  HK_HIP((launch_bl_fin<BL_INIT, ELL>(wk.st, wk.partials, gv, o.tol, (long long)o.max_iter, s)));
  int hflag = 0;
  HK_HIP(hipMemcpyAsync(&hflag, wk.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HK_HIP(hipStreamSynchronize(s));
  if (hflag) HK_FAIL(HK_EINVAL, "krylov solve: zero diagonal entry (Jacobi undefined)");

  const int m = o.check_every > 0 ? o.check_every : std::max(1, (n < 200000 ? 64 : 16) / ELL);
  const int rc = run_chunks(A->pinned, wk.st, m, o.max_iter, s, [&](hipStream_t q) {
    hipError_t e = hipSuccess;
    for (int c = 0; c < m && e == hipSuccess; ++c) {
      for (int j = 0; j < ELL && e == hipSuccess; ++j) {
        hipLaunchKernelGGL(k_bl_u<R>, dim3(gv), dim3(kBlock), 0, q, n, wk.st, j, wk.vec);
        e = hipGetLastError();
        if (e == hipSuccess) {
          EpiStoreDot<R> eu{wk.vec.u[j + 1], wk.rt};
          e = launch_fused(A, dp, wk.ahat, wk.vec.u[j], eu, wk.st, wk.partials, q);
        }
        if (e == hipSuccess) e = launch_bl_fin<BL_ALPHA, ELL>(wk.st, wk.partials, gs, 0, 0, q);
        if (e == hipSuccess) {
          hipLaunchKernelGGL(k_bl_r<R>, dim3(gv), dim3(kBlock), 0, q, n, wk.st, j, wk.vec, wk.y, wk.partials);
          e = hipGetLastError();
        }
        if (e == hipSuccess) e = launch_bl_fin<BL_R, ELL>(wk.st, wk.partials, gv, 0, 0, q);
        if (e == hipSuccess) {
          EpiStoreDot<R> er{wk.vec.r[j + 1], wk.rt};
          e = launch_fused(A, dp, wk.ahat, wk.vec.r[j], er, wk.st, wk.partials, q);
        }
        if (e == hipSuccess && j + 1 < ELL) e = launch_bl_fin<BL_RHO, ELL>(wk.st, wk.partials, gs, 0, 0, q);
      }
      if (e == hipSuccess) {
        hipLaunchKernelGGL((k_bl_gram<R, ELL>), dim3(gv), dim3(kBlock), 0, q, n, wk.st, wk.vec, wk.partials);
        e = hipGetLastError();
      }
      if (e == hipSuccess) {
        hipLaunchKernelGGL((k_bl_fin_gram<ELL>), dim3(1), dim3(kFinBlock), 0, q, wk.st, wk.partials, gv);
        e = hipGetLastError();
      }
      if (e == hipSuccess) {
        hipLaunchKernelGGL((k_bl_mr<R, ELL>), dim3(gv), dim3(kBlock), 0, q, n, wk.st, wk.vec, wk.y, wk.rt,
                           wk.partials);
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = launch_bl_fin<BL_MR, ELL>(wk.st, wk.partials, gv, 0, 0, q);
    }
    return e;
  });
  if (rc != HK_OK) return rc;
  // the common ending (x = D^-1 y, true residual, info) through a Work view
  Work<R> view{};
  view.y = wk.y;
  view.dinv = wk.dinv;
  view.t = wk.vec.u[1];
  view.partials = wk.partials;
  view.st = wk.st;
  return finish_solve<R>(A, val, b, x, view, info, s);
}

static int bicgstab_l_dispatch(hk_csr_s* A, int ell, const double2* val, const double2* b, double2* x,
                               const hk_solve_opts& o, void* ws, hk_solve_info* info, hipStream_t s) {
  switch (ell) {
    case 1: return bicgstab_l<1>(A, val, b, x, o, ws, info, s);
    case 2: return bicgstab_l<2>(A, val, b, x, o, ws, info, s);
    case 4: return bicgstab_l<4>(A, val, b, x, o, ws, info, s);
    case 8: return bicgstab_l<8>(A, val, b, x, o, ws, info, s);
    default: HK_FAIL(HK_EINVAL, "hk_krylov_solve: BiCGStab(l) needs l in {1, 2, 4, 8} (got %d)", ell);
  }
}

static int ensure_pinned(hk_csr_s* A) {
  if (A->pinned) return HK_OK;
  HK_HIP(hipHostMalloc((void**)&A->pinned, 64, hipHostMallocDefault));
  return HK_OK;
}

// info->shape of the plain and mixed solves: the fused products' shape
// {lanes per row (64: row blocks), rows per group or wave, waves per
// workgroup, paired layout} of precision slot prec (0 complex128, 1
// complex64), or the handle's CSR shape when none was fixed or tuned.
static void report_shape(const hk_csr_s* A, int prec, hk_solve_info* info) {
  const SpmvPlan& d = A->dot_plan[prec].tuned ? A->dot_plan[prec] : A->plan;
  info->shape[0] = d.L;
  info->shape[1] = d.U;
  info->shape[2] = d.nw;
  info->shape[3] = d.pairs;
  info->shape_tuned = d.tuned == 1 ? 1 : 0;
  info->pad = 0;
}

static int check_opts(const hk_solve_opts* o, const char* who) {
  if (!o) HK_FAIL(HK_EINVAL, "%s: opts is NULL", who);
  if (o->shape[0] || o->shape[1] || o->shape[2] || o->shape[3])
    HK_FAIL(HK_EINVAL, "%s: opts->shape applies to the batched solves only", who);
  if (o->flags & ~HK_MIXED_LITERAL_INNER) HK_FAIL(HK_EINVAL, "%s: unknown flags 0x%x", who, (unsigned)o->flags);
  if (!(o->tol >= 0) || o->max_iter < 0 || o->check_every < 0)
    HK_FAIL(HK_EINVAL, "%s: bad options (tol=%g max_iter=%lld)", who, o->tol, (long long)o->max_iter);
  if (o->method != HK_BICGSTAB && o->method != HK_TFQMR && o->method != HK_BICGSTAB_L)
    HK_FAIL(HK_EINVAL, "%s: unknown method %d", who, (int)o->method);
  if (o->method == HK_BICGSTAB_L && o->ell != 1 && o->ell != 2 && o->ell != 4 && o->ell != 8)
    HK_FAIL(HK_EINVAL, "%s: BiCGStab(l) needs l in {1, 2, 4, 8} (got %d)", who, (int)o->ell);
  return HK_OK;
}

}  // namespace hk

using namespace hk;

extern "C" int hk_krylov_solve(hk_csr A, const void* d_b, void* d_x, const hk_solve_opts* opts,
                               hk_solve_info* info, void* stream) {
  if (!A || !d_b || !d_x || !info) HK_FAIL(HK_EINVAL, "hk_krylov_solve: null argument");
  int rc = check_opts(opts, "hk_krylov_solve");
  if (rc != HK_OK) return rc;
  hipStream_t s = as_stream(stream);
  rc = ensure_pinned(A);
  if (rc != HK_OK) return rc;
  if (A->dtype == HK_C64) {
    if (opts->method != HK_BICGSTAB) HK_FAIL(HK_EINVAL, "hk_krylov_solve: complex64 solves use BiCGStab only");
    rc = ensure_ws(&A->ws32, &A->ws32_bytes, work_bytes<float>(A->n, A->nnz), s);
    if (rc != HK_OK) return rc;
    rc = bicgstab<float>(A, (const float2*)A->val, (const float2*)d_b, (float2*)d_x, *opts, A->ws32,
                         info, s);
  } else {
    const size_t need = opts->method == HK_BICGSTAB_L ? bl_work_bytes<double>(A->n, A->nnz, opts->ell)
                                                      : work_bytes<double>(A->n, A->nnz);
    rc = ensure_ws(&A->ws, &A->ws_bytes, need, s);
    if (rc != HK_OK) return rc;
    if (opts->method == HK_BICGSTAB_L)
      rc = bicgstab_l_dispatch(A, opts->ell, (const double2*)A->val, (const double2*)d_b, (double2*)d_x, *opts,
                               A->ws, info, s);
    else if (opts->method == HK_TFQMR)
      rc = tfqmr(A, (const double2*)A->val, (const double2*)d_b, (double2*)d_x, *opts, A->ws, info, s);
    else
      rc = bicgstab<double>(A, (const double2*)A->val, (const double2*)d_b, (double2*)d_x, *opts, A->ws,
                            info, s);
  }
  if (rc != HK_OK) return rc;
  report_shape(A, A->dtype == HK_C64 ? 1 : 0, info);
  return info->status;
}

extern "C" int hk_krylov_solve_mixed(hk_csr A, const void* d_b, void* d_x, double inner_tol,
                                     double outer_tol, int32_t max_outer, const hk_solve_opts* opts,
                                     hk_solve_info* info, void* stream) {
  if (!A || !d_b || !d_x || !info) HK_FAIL(HK_EINVAL, "hk_krylov_solve_mixed: null argument");
  if (A->dtype != HK_C128) HK_FAIL(HK_EINVAL, "hk_krylov_solve_mixed: matrix must be complex128");
  int rc = check_opts(opts, "hk_krylov_solve_mixed");
  if (rc != HK_OK) return rc;
  if (!(inner_tol > 0) || !(outer_tol >= 0) || max_outer < 0)
    HK_FAIL(HK_EINVAL, "hk_krylov_solve_mixed: bad tolerances");
  if (opts->method != HK_BICGSTAB) HK_FAIL(HK_EINVAL, "hk_krylov_solve_mixed: the inner solve is BiCGStab");
  hipStream_t s = as_stream(stream);
  const int64_t n = A->n;
  // complex64 workspace + r (c128) + r32, d32 (c64) + norm scratch
  const size_t extra = align_up(16 * n) + 2 * align_up(8 * n) + align_up(64);
  rc = ensure_pinned(A);
  if (rc != HK_OK) return rc;
  rc = ensure_ws(&A->ws32, &A->ws32_bytes, work_bytes<float>(A->n, A->nnz) + extra, s);
  if (rc != HK_OK) return rc;
  if (!A->val32) {
    if (hipMalloc(&A->val32, 8 * (size_t)(A->nnz > 0 ? A->nnz : 1)) != hipSuccess)
      HK_FAIL(HK_ENOMEM, "hk_krylov_solve_mixed: hipMalloc failed");
  }
  char* tail = (char*)A->ws32 + work_bytes<float>(A->n, A->nnz);
  double2* r = (double2*)tail;
  float2* r32 = (float2*)(tail + align_up(16 * n));
  float2* d32 = (float2*)(tail + align_up(16 * n) + align_up(8 * n));
  double* dnorm = (double*)(tail + align_up(16 * n) + 2 * align_up(8 * n));
  const dim3 ew((unsigned)((n + kBlock - 1) / kBlock));
  // A32 = round-to-nearest of each component of A
  if (A->nnz > 0) {
    hipLaunchKernelGGL(k_round_c64, dim3((unsigned)((A->nnz + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, (int64_t)A->nnz, (const double2*)A->val, (float2*)A->val32, 1.0);
    HK_CHECK_LAUNCH();
  }
  if (!opts->use_x0) HK_HIP(hipMemsetAsync(d_x, 0, 16 * n, s));
  rc = hk_dznrm2(n, d_b, dnorm, stream);
  if (rc != HK_OK) return rc;
  double bn = 0;
  HK_HIP(hipMemcpyAsync(&bn, dnorm, sizeof(double), hipMemcpyDeviceToHost, s));
  HK_HIP(hipStreamSynchronize(s));
  hk_solve_opts io = *opts;
  io.tol = inner_tol;
  io.use_x0 = 0;
  io.d_history = nullptr;
  int64_t inner_total = 0;
  double prev = INFINITY, rel = 0;
  int status = HK_NOT_CONVERGED, k = 0;
  hk_csr_s A32 = *A;
  A32.val = A->val32;
  A32.dtype = HK_C64;
  if (A->plan.tuned) {
    // a tuned handle gets its own launch shape for the complex64 copy
    if (!A->plan32.tuned) {
      rc = spmv_autotune(&A32, s);
      if (rc != HK_OK) return rc;
      A->plan32 = A32.plan;
    }
    A32.plan = A->plan32;
  }
  const bool trace = getenv("HK_TRACE") != nullptr;
  const bool literal = (opts->flags & HK_MIXED_LITERAL_INNER) != 0;
  io.flags = 0;
  for (k = 0; k <= max_outer; ++k) {
    rc = spmv_dispatch(A, d_x, r, d_b, nullptr, nullptr, 1, s);   // r = b - A u (complex128)
    if (rc != HK_OK) return rc;
    rc = hk_dznrm2(n, r, dnorm, stream);
    if (rc != HK_OK) return rc;
    double rn = 0;
    HK_HIP(hipMemcpyAsync(&rn, dnorm, sizeof(double), hipMemcpyDeviceToHost, s));
    HK_HIP(hipStreamSynchronize(s));
    rel = bn > 0 ? rn / bn : rn;
    if (!std::isfinite(rn)) { status = HK_NONFINITE; break; }
    if (rel <= outer_tol) { status = HK_OK; break; }
    if (rn >= prev || k == max_outer) { status = HK_NOT_CONVERGED; break; }
    prev = rn;
    // the inner right-hand side is r scaled by a power of two to unit size, so
    // the complex64 iteration runs far from its under/overflow range
    const double scale = std::ldexp(1.0, -std::ilogb(rn));
    hipLaunchKernelGGL(k_round_c64, ew, dim3(kBlock), 0, s, n, (const double2*)r, r32, scale);
    HK_CHECK_LAUNCH();
    // inner tolerance: inner_tol, or, where a smaller reduction reaches
    // outer_tol, half of that reduction (the last cycle stops early);
    // HK_MIXED_LITERAL_INNER keeps inner_tol in every cycle
    io.tol = literal ? inner_tol : std::max(inner_tol, 0.5 * outer_tol / rel);
    hk_solve_info ii{};
    rc = bicgstab<float>(&A32, (const float2*)A->val32, r32, d32, io, A->ws32, &ii, s);
    A->dot_plan[1] = A32.dot_plan[1];  // the inner solve's tuned fused shape
    if (rc != HK_OK) return rc;
    if (trace)
      fprintf(stderr, "[hk mixed] cycle %d: ||r||/||b|| = %.3e, inner status %d (breakdown %d) after %lld iterations, inner relres %.3e\n",
              k, rel, ii.status, ii.breakdown, (long long)ii.iters, ii.relres_rec);
    inner_total += ii.iters;
    if (ii.status == HK_NONFINITE) { status = HK_NONFINITE; break; }
    hipLaunchKernelGGL(k_add_c64, ew, dim3(kBlock), 0, s, (int)n, (const float2*)d32, (double2*)d_x,
                       1.0 / scale);
    HK_CHECK_LAUNCH();
  }
  info->status = status;
  info->breakdown = HK_BD_NONE;
  info->iters = k;
  info->relres_rec = rel;
  info->relres_true = rel;
  info->inner_iters = inner_total;
  report_shape(A, 1, info);
  return status;
}
