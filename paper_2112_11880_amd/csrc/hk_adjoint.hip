// hk_adjoint.hip -- the speed-dependent Helmholtz operator and its adjoint
// sensitivities (gfx950).
//
// The paper's operator is -lap(u) - k^2 u with k = 2 pi F / c and a speed c
// that varies in space (Introduction).  For a piecewise-constant speed c_b
// per block of elements, the FE matrix is
//     A(c) = K - omega^2 (1 + i damp) sum_b c_b^-2 M_b,
// M_b the mass matrix of the elements of block b (Dirichlet rows and columns
// removed).  Given u = A^-1 g and the adjoint state lambda with
// A lambda = conj(dL/du) (A is complex symmetric), a real loss L has
//     dL/dc_b = -Re( lambda^T (dA/dc_b) u ),
//     dA/dc_b = 2 omega^2 (1 + i damp) c_b^-3 M_b,
// and lambda^T M_e u = vol_e/20 * (sum_a lambda_a sum_a u_a + sum_a lambda_a u_a)
// for the P1 element mass matrix M_e = vol_e/20 (1 + delta_ab).
#include "hk_common.hpp"
#include "hk_internal.hpp"

namespace hk {

// val[p] = K[p] - kappa * sum_{q in list(p)} m_q / c_{blk(q)}^2
__global__ void k_assemble(int nnz, const double* __restrict__ K, const int* __restrict__ bm_ptr,
                           const int* __restrict__ bm_blk, const double* __restrict__ bm_val,
                           int nlist, const double* __restrict__ c, int nblocks, double2 kappa,
                           double2* __restrict__ val, int* flag) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= nnz) return;
  int q0 = bm_ptr[p], q1 = bm_ptr[p + 1];
  if (q0 < 0 || q1 > nlist || q1 < q0) { atomicOr(flag, 1); q1 = q0; }
  double m = 0;
  for (int q = q0; q < q1; ++q) {
    const int b = bm_blk[q];
    if (b < 0 || b >= nblocks) { atomicOr(flag, 1); continue; }
    const double cb = c[b];
    m += bm_val[q] / (cb * cb);
  }
  val[p] = make_double2(K[p] - kappa.x * m, -kappa.y * m);
}

// One workgroup per speed block: s_b = sum over its elements of
// lambda_e^T M_e u_e (Dirichlet nodes masked), then
// grad_c[b] = -Re(2 kappa c_b^-3 s_b).
__global__ __launch_bounds__(kBlock) void k_elem_sens(int n, int nblocks, const int* __restrict__ tet_nodes,
                                                      const int* __restrict__ tet_ptr,
                                                      const double* __restrict__ tet_vol,
                                                      const unsigned char* __restrict__ dir,
                                                      const double2* __restrict__ lam,
                                                      const double2* __restrict__ u,
                                                      const double* __restrict__ c, double2 kappa,
                                                      double* __restrict__ grad_c, int* flag) {
  __shared__ double lds[2 * (kBlock / kWave)];
  const int b = blockIdx.x;
  const int e0 = tet_ptr[b], e1 = tet_ptr[b + 1];
  double acc[2] = {0, 0};
  for (int e = e0 + threadIdx.x; e < e1; e += kBlock) {
    double2 sl = make_double2(0, 0), su = make_double2(0, 0), sd = make_double2(0, 0);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int v = tet_nodes[4 * e + a];
      if (v < 0 || v >= n) { atomicOr(flag, 1); continue; }
      if (dir[v]) continue;
      const double2 l = lam[v], x = u[v];
      sl = cadd(sl, l);
      su = cadd(su, x);
      sd = cfma(l, x, sd);
    }
    const double w = tet_vol[e] / 20.0;
    const double2 se = cfma(sl, su, sd);
    acc[0] = fma(w, se.x, acc[0]);
    acc[1] = fma(w, se.y, acc[1]);
  }
  block_sum<2>(acc, lds);
  if (threadIdx.x == 0) {
    const double cb = c[b];
    const double f = 2.0 / (cb * cb * cb);
    // -Re(f kappa s)
    grad_c[b] = -f * (kappa.x * acc[0] - kappa.y * acc[1]);
  }
}

__global__ void k_check_ptr(int nblocks, int ntet, const int* ptr, int* flag) {
  const int b = blockIdx.x * kBlock + threadIdx.x;
  if (b > nblocks) return;
  const int v = ptr[b];
  if (v < 0 || v > ntet || (b == 0 && v != 0) || (b == nblocks && v != ntet)) atomicOr(flag, 2);
  if (b < nblocks && ptr[b + 1] < v) atomicOr(flag, 2);
}

}  // namespace hk

using namespace hk;

extern "C" int hk_assemble_helmholtz(int64_t nnz, const double* d_K, const int32_t* d_bm_ptr,
                                     const int32_t* d_bm_blk, const double* d_bm_val, int64_t nlist,
                                     int32_t nblocks, const double* d_c, double omega, double damp,
                                     void* d_val, void* stream) {
  if (nnz <= 0 || nnz >= (1ll << 31) - 1 || nlist < 0 || nlist >= (1ll << 31) - 1 || nblocks <= 0 ||
      !d_K || !d_bm_ptr || !d_bm_blk ||
      !d_bm_val || !d_c || !d_val)
    HK_FAIL(HK_EINVAL, "hk_assemble_helmholtz: bad argument");
  hipStream_t s = as_stream(stream);
  // the error word lives in the stream's reduction scratch (allocated once)
  ReduceScratch* scr = nullptr;
  const int rc = reduce_scratch(s, sizeof(int), &scr);
  if (rc != HK_OK) return rc;
  int* flag = static_cast<int*>(scr->partials);
  int h = 0;
  hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), s);
  if (e == hipSuccess) {
    const double w2 = omega * omega;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)((nnz + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       (int)nnz, d_K, d_bm_ptr, d_bm_blk, d_bm_val, (int)nlist, d_c, nblocks,
                       make_double2(w2, damp * w2), (double2*)d_val, flag);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) HK_FAIL(HK_EHIP, "hk_assemble_helmholtz: %s", hipGetErrorString(e));
  if (h) HK_FAIL(HK_EINVAL, "hk_assemble_helmholtz: malformed block-mass lists");
  return HK_OK;
}

extern "C" int hk_elem_sens(int64_t n, int64_t ntet, int32_t nblocks, const int32_t* d_tet_nodes,
                            const int32_t* d_tet_ptr, const double* d_tet_vol,
                            const uint8_t* d_dirichlet, const void* d_lambda, const void* d_u,
                            const double* d_c, double omega, double damp, double* d_grad_c,
                            void* stream) {
  if (n <= 0 || ntet <= 0 || nblocks <= 0 || n >= (1ll << 31) - 1 || ntet >= (1ll << 29) ||
      !d_tet_nodes || !d_tet_ptr || !d_tet_vol || !d_dirichlet || !d_lambda || !d_u || !d_c ||
      !d_grad_c)
    HK_FAIL(HK_EINVAL, "hk_elem_sens: bad argument");
  hipStream_t s = as_stream(stream);
  // the error word lives in the stream's reduction scratch (allocated once)
  ReduceScratch* scr = nullptr;
  const int rc = reduce_scratch(s, sizeof(int), &scr);
  if (rc != HK_OK) return rc;
  int* flag = static_cast<int*>(scr->partials);
  int h = 0;
  hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_check_ptr, dim3((unsigned)((nblocks + 1 + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, (int)nblocks, (int)ntet, d_tet_ptr, flag);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && h) HK_FAIL(HK_EINVAL, "hk_elem_sens: element block offsets are not a partition of [0, ntet]");
  if (e == hipSuccess) {
    const double w2 = omega * omega;
    hipLaunchKernelGGL(k_elem_sens, dim3((unsigned)nblocks), dim3(kBlock), 0, s, (int)n, (int)nblocks,
                       d_tet_nodes, d_tet_ptr, d_tet_vol, d_dirichlet, (const double2*)d_lambda,
                       (const double2*)d_u, d_c, make_double2(w2, damp * w2), d_grad_c, flag);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) HK_FAIL(HK_EHIP, "hk_elem_sens: %s", hipGetErrorString(e));
  if (h) HK_FAIL(HK_EINVAL, "hk_elem_sens: element node index out of range");
  return HK_OK;
}
