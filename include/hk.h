/*
 * hk.h -- C ABI of libhk: complex Krylov solvers for finite-element Helmholtz
 * systems on AMD Instinct MI355X (gfx950).
 *
 * Problem (the paper, arXiv 2112.11880, Introduction and Section 2): the
 * finite-element discretisation of -lap(u) - k^2 u = g with Dirichlet
 * conditions on part of the boundary gives a large sparse complex system
 * A u = g, stored in compressed sparse row (CSR) form.  Section 3 defines the
 * complex double BLAS-1 operations (scale, axpy, element-wise product, dot,
 * L2 norm) and the CSR product; Section 4 composes them into a
 * preconditioned BiCGStab started from zero with a residual tolerance and an
 * iteration cap.
 *
 * Conventions for every entry point:
 *   - Complex vectors are interleaved (re, im) pairs: complex128 = two
 *     doubles (16 bytes), complex64 = two floats (8 bytes).
 *   - Pointers named d_* are device pointers (HIP device memory of the
 *     current device); all other pointers are host pointers.
 *   - The caller owns every buffer passed in.  The library never frees
 *     caller memory; a matrix handle owns only its launch plan and workspace.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue work
 *     on it and return without waiting, except where stated.
 *   - Return value: HK_OK (0); a negative code for a usage or runtime error,
 *     raised before any work is enqueued where possible (the text is
 *     available from hk_last_error()); a positive code for a numerical
 *     outcome of a solve.
 *   - Indices are int32 (rowptr has n+1 entries, col has nnz entries, column
 *     indices ascending within a row, 0 <= col < n).
 *   - A matrix handle carries its solvers' workspace and tuned shapes: calls
 *     on one handle must not overlap (from several threads, or on several
 *     streams at once); use one handle per concurrent stream.  Distinct
 *     handles, and the BLAS-1 calls on distinct streams, are independent.
 */
#ifndef HK_H_
#define HK_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum hk_status {
  HK_OK = 0,
  HK_EINVAL = -1,          /* invalid argument (null pointer, bad size, bad matrix) */
  HK_EHIP = -2,            /* a HIP runtime call failed */
  HK_ENOMEM = -3,          /* device allocation failed */
  HK_NOT_CONVERGED = 1,    /* iteration cap reached; x holds the last iterate */
  HK_BREAKDOWN = 2,        /* a BiCGStab scalar vanished; x holds the last iterate */
  HK_NONFINITE = 3         /* Inf/NaN in the input or in an iteration scalar */
};

enum hk_dtype { HK_C128 = 0, HK_C64 = 1 };

enum hk_csr_flags {
  HK_VALIDATE = 1,   /* structure check at creation (always done) */
  HK_AUTOTUNE = 2,   /* time the SpMV launch shapes on this matrix and keep the fastest */
  HK_INT32_COLS = 4  /* do not build the 16-bit column stream (products read d_col itself) */
};

enum hk_breakdown { HK_BD_NONE = 0, HK_BD_RHO = 1, HK_BD_SIGMA = 2, HK_BD_TAU = 3, HK_BD_OMEGA = 4 };

typedef struct hk_csr_s* hk_csr;

/* Text of the last error raised on the calling thread ("" if none). */
const char* hk_last_error(void);

/* ------------------------------------------------------------ matrices */

/*
 * Wrap a CSR matrix that lives in caller-owned device memory (Section 2:
 * FE matrices in CSR).  d_val holds nnz complex values of type dtype.  The
 * buffers must stay valid while the handle lives, and rowptr and col must
 * not change; values may be updated between calls.  The structure is always
 * checked on the device (rowptr non-decreasing from 0 to nnz, every col in
 * [0, n) and strictly ascending within its row; HK_EINVAL otherwise), which
 * also finds the longest row; this synchronises `stream`.  HK_VALIDATE is
 * accepted and implied.  When every entry lies within 32767 columns of its
 * row's 64-aligned base (row & ~63), as in a banded FE matrix, the handle
 * also keeps the column indices as 16-bit offsets from that base (2 bytes
 * per entry, device memory it owns), which the row-block products stream
 * instead of col; HK_INT32_COLS turns this off.  Results are the same bits
 * either way.  HK_AUTOTUNE times the candidate launch shapes on this matrix
 * (values are not modified) and keeps the fastest.
 */
int hk_csr_create(hk_csr* out, int64_t n, int64_t nnz, const int32_t* d_rowptr,
                  const int32_t* d_col, const void* d_val, int dtype, int flags, void* stream);

/* Release the handle and its workspace (not the caller's buffers). NULL is a no-op. */
int hk_csr_destroy(hk_csr A);

/* Launch shape chosen for the matrix: lanes per row, rows per lane group,
 * workgroups per launch, and whether it was chosen by timing. */
int hk_csr_plan(hk_csr A, int32_t* lanes_per_row, int32_t* rows_per_group, int32_t* grid,
                int32_t* tuned);

/* Size and storage of the matrix: n, nnz, longest row, and the bytes per
 * entry of the column stream the row-block products read (2: 16-bit
 * offsets, 4: the int32 indices).  Null outputs are skipped. */
int hk_csr_info(hk_csr A, int64_t* n, int64_t* nnz, int32_t* max_row, int32_t* col_bytes);

/* Override the launch shape: lanes_per_row in {4,8,16,32} with
 * rows_per_group in {1,2,4,8} not above lanes_per_row (a group of lanes per
 * row), or lanes_per_row = 64 with rows_per_group in {16,32,64} (the
 * row-block scheme: one wave per rows_per_group consecutive rows, all 64
 * lanes streaming their entries); grid > 0 (tiles dealt to workgroups with a
 * grid stride), or 0 for one workgroup per tile.  Anything else gives
 * HK_EINVAL. */
int hk_csr_set_plan(hk_csr A, int32_t lanes_per_row, int32_t rows_per_group, int32_t grid);

/* Fix the launch shape of the solvers' fused products (the CSR products
 * with a dot or vector-update epilogue inside hk_krylov_solve and the
 * mixed solve's inner iteration), for both precisions: the row-block scheme
 * with rows_per_wave in {16,32,64} consecutive rows per wave, waves in
 * {2,4,8} per workgroup, grid workgroups (0: one per tile, at most 8192),
 * and paired = 1 for the paired-entry layout (each lane loads two
 * consecutive entries; needs the 16-bit column stream, see hk_csr_info).
 * Without it, a tuned handle times the candidates on its first solve and an
 * untuned one uses its CSR shape.  hk_csr_set_plan clears it.  Anything
 * else gives HK_EINVAL. */
int hk_csr_set_solver_plan(hk_csr A, int32_t rows_per_wave, int32_t waves, int32_t grid, int32_t paired);

/*
 * y = alpha * A x + beta * y (Section 3, Table 8: CSR SpMV).  alpha and
 * beta are host complex scalars {re, im} of A's precision (double[2] for
 * complex128, float[2] for complex64); beta == 0 does not read y.  x and y
 * have n entries and must not overlap.
 */
int hk_spmv(hk_csr A, const void* alpha, const void* d_x, const void* beta, void* d_y,
            void* stream);

/* r = b - A x (the residual of the refinement loop; complex128 or complex64). */
int hk_residual(hk_csr A, const void* d_b, const void* d_x, void* d_r, void* stream);

/* ------------------------------------------------ BLAS-1, complex128 */

/* *d_res = x^H y = sum conj(x_i) y_i (Section 3, ZDOT: element-wise product,
 * then a two-stage sum: per-workgroup partials, then their sum).  d_res is
 * one complex128 in device memory.  Deterministic: the same bits on every
 * call for the same n and data.  n = 0 gives 0 (x and y may then be NULL);
 * n < 0 gives HK_EINVAL. */
int hk_zdotc(int64_t n, const void* d_x, const void* d_y, void* d_res, void* stream);

/* The same *d_res = x^H y as hk_zdotc, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): no hipMalloc, hipFree or allocating
 * library call is made.  The per-workgroup partials go to a static 64 KiB
 * device array of the library (one per GPU, held until the process ends,
 * its address looked up on the first call on each device), enough for the
 * reduction's at most 4096 workgroups; nothing in it needs clearing.  Same
 * kernels, so the same bits as hk_zdotc.  n up to 2^40 (HK_EINVAL above);
 * n = 0 gives 0.  Calls that overlap on one GPU (several streams or host
 * threads at once) race on the shared array and must be serialised by the
 * caller. */
int hk_zdotc_noalloc(int64_t n, const void* d_x, const void* d_y, void* d_res, void* stream);

/* *d_res = x^T y = sum x_i y_i (unconjugated form of the same reduction). */
int hk_zdotu(int64_t n, const void* d_x, const void* d_y, void* d_res, void* stream);

/* *d_res = ||x||_2 = sqrt(sum re^2 + im^2) (Section 3, ZNORM); one double in
 * device memory; n = 0 gives 0. */
int hk_dznrm2(int64_t n, const void* d_x, double* d_res, void* stream);

/* y = alpha x + y (Section 3, ZAXPY listing); alpha is a host double[2]. */
int hk_zaxpy(int64_t n, const double* alpha, const void* d_x, void* d_y, void* stream);

/* x = alpha x (Section 3, ZSCAL listing); alpha is a host double[2]. */
int hk_zscal(int64_t n, const double* alpha, void* d_x, void* stream);

/* y = x .* y (Section 3, element-wise product listing, ZAXMY). */
int hk_zaxmy(int64_t n, const void* d_x, void* d_y, void* stream);

/* y = x (Section 3, ZASSIGN). */
int hk_zcopy(int64_t n, const void* d_x, void* d_y, void* stream);

/* y = conj(x) (x == y allowed); used to form adjoint right-hand sides. */
int hk_zconj(int64_t n, const void* d_x, void* d_y, void* stream);

/* ------------------------------------------------------------- solvers */

typedef struct {
  double tol;            /* stop when ||b - A x||_2 <= tol * ||b||_2 (recursive residual) */
  int64_t max_iter;      /* iteration cap (the paper uses 1000; larger FE systems need more) */
  int32_t precond;       /* 0: none, 1: Jacobi (diagonal), applied on the right */
  int32_t check_every;   /* iterations enqueued between host status reads (0: automatic) */
  int32_t use_x0;        /* 0: start from x = 0 (the paper's choice), 1: from d_x */
  int32_t method;        /* hk_method; HK_TFQMR and HK_BICGSTAB_L are complex128 only */
  double* d_history;     /* optional device buffer of max_iter+1 doubles: ||r_k||/||b||
                            (TFQMR: the quasi-residual bound sqrt(m+1) tau / ||b||) */
  int32_t ell;           /* HK_BICGSTAB_L: BiCG steps per cycle, 1, 2, 4 or 8 (the paper: 8) */
  int32_t flags;         /* hk_solve_flags bits (0: none) */
  int32_t shape[4];      /* batched solves: a launch shape to use instead of the tuned one
                            (all 0: autotune; see hk_sweep_solve / hk_blockdiag_solve);
                            other solves: must be all 0 */
} hk_solve_opts;

/* Bits of hk_solve_opts.flags. */
enum hk_solve_flags {
  /* hk_krylov_solve_mixed: solve every cycle to inner_tol, without the
   * last cycle's clamp to half the reduction still needed */
  HK_MIXED_LITERAL_INNER = 1
};

/* Krylov method of hk_krylov_solve (Section 4 implements all three). */
typedef enum { HK_BICGSTAB = 0, HK_TFQMR = 1, HK_BICGSTAB_L = 2 } hk_method;

typedef struct {
  int64_t iters;         /* completed iterations (a half-step exit counts as one) */
  double relres_rec;     /* recursive ||r|| / ||b|| at exit (TFQMR: the quasi-residual bound) */
  double relres_true;    /* ||b - A x|| / ||b|| recomputed at exit */
  int32_t status;        /* HK_OK / HK_NOT_CONVERGED / HK_BREAKDOWN / HK_NONFINITE */
  int32_t breakdown;     /* hk_breakdown: which scalar vanished */
  int64_t inner_iters;   /* mixed precision: total inner iterations; else 0 */
  int32_t shape[4];      /* launch shape of the solve's products (see each solve) */
  int32_t shape_tuned;   /* 1 if that shape was chosen by timing on the device */
  int32_t pad;
} hk_solve_info;

/*
 * Preconditioned Krylov solve of A x = b (Section 4: zero initial guess,
 * residual tolerance, iteration cap; Jacobi preconditioner on the right).
 * opts->method selects P-BiCGSTAB (van der Vorst's recurrences; stops on
 * ||r|| <= tol ||b|| after a half or full step), P-TFQMR (Freund's method
 * as in Saad's book; two products per iteration; stops when the
 * quasi-residual bound sqrt(m+1) tau <= tol ||b||, m the half-step) or
 * P-BiCGSTAB(l) (Sleijpen and Fokkema's method, l = opts->ell BiCG steps and
 * one minimal-residual step per iteration, the MR step through the normal
 * equations of the Gram matrix of r_1..r_l; stops on ||r|| <= tol ||b||
 * after any BiCG step or MR step; info->iters counts cycles).  A
 * complex128 matrix gives a complex128 solve; a complex64 matrix (BiCGStab
 * only) a complex64 solve whose vectors and products are complex64 and whose
 * dots and scalars are double (b and x then complex64).  Scalars stay in
 * device memory; the host reads a status word every check_every iterations
 * and synchronises the stream once at the end to fill *info.  A chunk of
 * check_every iterations (up to 256) is recorded once into a HIP graph on a
 * private stream that waits for `stream`, and replayed; the environment
 * variable HK_SOLVE_GRAPHS=0 launches every kernel on `stream` instead (same
 * results, bit for bit).  A zero
 * diagonal entry with precond = 1, or an unknown method, gives HK_EINVAL.
 * info->shape reports the fused products' launch shape {lanes per row (64:
 * row blocks), rows per lane group or per wave, waves per workgroup, paired
 * layout}, and info->shape_tuned whether the solver timed it.
 * Returns info->status (>= 0) or an error.  x always holds the last iterate.
 */
int hk_krylov_solve(hk_csr A, const void* d_b, void* d_x, const hk_solve_opts* opts,
                    hk_solve_info* info, void* stream);

/*
 * Mixed-precision iterative refinement (not in the paper): r = b - A u, its
 * norm, the stopping test ||r|| <= outer_tol ||b|| and the update u += d run
 * in complex128; d solves A d = r with Jacobi BiCGStab in complex64 (values
 * of A rounded to nearest per component; complex64 vectors and products,
 * dots and scalars in double) to a tolerance relative to ||r|| of
 * max(inner_tol, outer_tol ||b|| / (2 ||r||)): inner_tol, except in a cycle
 * that needs less than that to reach outer_tol, which stops at half the
 * reduction it needs (with HK_MIXED_LITERAL_INNER in opts->flags: inner_tol
 * in every cycle).  At most
 * max_outer cycles; a cycle that does not lower ||r|| ends the loop
 * (HK_NOT_CONVERGED).  opts->max_iter caps each inner solve; opts->method
 * must be HK_BICGSTAB.  The complex64 copy of A is kept in the handle.
 * With the environment variable HK_TRACE set, each cycle's relative
 * residual and inner iteration count are printed to stderr.  info->iters
 * counts cycles, info->inner_iters the inner iterations; info->shape is
 * the complex64 fused products' shape, as for hk_krylov_solve.
 */
int hk_krylov_solve_mixed(hk_csr A, const void* d_b, void* d_x, double inner_tol,
                          double outer_tol, int32_t max_outer, const hk_solve_opts* opts,
                          hk_solve_info* info, void* stream);

/* ------------------------------------------------------ batched solves */

/*
 * Both batched solves run one cooperative launch whose workgroups meet at
 * grid barriers.  Every barrier wait is bounded: a workgroup that waits
 * longer than the limit (default 4 s; the environment variable
 * HK_BARRIER_SPIN_TICKS, read at each call, sets it in 100 MHz ticks) raises
 * an abort flag, every workgroup leaves at its next barrier, and the call
 * frees its workspace and returns HK_EHIP with "grid barrier timed out".
 * With opts->d_history non-null (device, 8 (max_iter + 1) doubles, caller
 * owned) the solve records barrier times in it: entry e (e >= 1, the e-th
 * barrier of the launch) = the device's 100 MHz wall clock when the last
 * workgroup arrived (at a barrier that also sums per-system dot products:
 * once the last group of workgroups has summed its part); entries of
 * barriers that did not happen are left
 * untouched.  The barriers of both solves are: 1 after the start phase;
 * then per iteration (4 in the first, which has no p update) after the p
 * update, the v product, the s update, the t product and the x/r update;
 * then the sweep has one after its true-residual product, the uneven batch
 * one before (the full tile list rebuilt) and one after it.  The time between
 * two entries is the phase between those barriers, the barrier included.
 */

/*
 * Frequency sweep in one persistent launch (not in the paper; it batches the
 * paper's P-BiCGSTAB over systems that share a sparsity pattern): for
 * j < nsys (nsys <= 64), solve (K - kappa_j M) x_j = b_j with Jacobi
 * BiCGStab, K and M real (double) CSR values on one pattern (d_rowptr,
 * d_col, nnz entries), kappa a host array of nsys complex values
 * {re, im}.  d_B and d_X are n x 64 complex128, interleaved system-fastest
 * (entry (i, j) at index i*64 + j; columns j >= nsys are ignored).  x starts
 * at 0.  opts->tol, max_iter apply to every system; infos receives nsys
 * records.  Synchronises `stream`.  Returns the largest per-system status.
 * Launch shape {product form, row mapping, 0, 0}: product form 1 walks a
 * wave's rows one at a time, 2 streams the entries of a wave's contiguous
 * rows across row boundaries, 3 walks rows one at a time with the next
 * row's first 16 entries loaded while the current row's gathers are in
 * flight; row mapping 1 deals each XCD's eighth of the rows round-robin to
 * its waves, 2 deals all rows round-robin to all waves, 3 gives each wave a
 * contiguous range of its XCD's eighth (form 2 needs mapping 3).  The
 * candidates are {1,1}, {1,2}, {1,3}, {2,3}, {3,1} and {3,2}.  With form 3
 * the solve continues in a second cooperative launch once at most 32
 * systems run (two rows per wave step, one per half-wave, for the running
 * systems only) and in a third once at most 16 run (four rows per step);
 * the barrier stamps run on across the launches.  With
 * opts->shape all 0, the first call for a given (device, n, nnz, longest
 * row, nsys) runs every candidate for 4 iterations, timed with HIP events,
 * and keeps the fastest for this and later calls (the batch-plan analogue
 * of the paper's per-matrix tuning of the GPU grid, Section 3); the trial
 * launches write only the call's workspace and X.  A nonzero opts->shape
 * must be a candidate (HK_EINVAL otherwise) and is used as is.  Every
 * infos[j].shape holds the shape used, shape_tuned whether it was timed.
 */
int hk_sweep_solve(int64_t n, int64_t nnz, const int32_t* d_rowptr, const int32_t* d_col,
                   const double* d_K, const double* d_M, int32_t nsys, const double* kappa,
                   const void* d_B, void* d_X, const hk_solve_opts* opts, hk_solve_info* infos,
                   void* stream);

/*
 * Uneven batch in one persistent launch: A (complex128) is block-diagonal
 * with nsys <= 64 diagonal blocks; system k owns rows and columns
 * [row_off[k], row_off[k+1]) (host array, row_off[0] = 0, row_off[nsys] =
 * n).  Each system is solved with Jacobi BiCGStab from x = 0 to its own
 * relative tolerance; systems that finish drop out of the work list.
 * d_b, d_x: n complex128 (systems concatenated).  A column outside its
 * row's system gives HK_EINVAL.  Synchronises `stream`.  Rows are dealt in
 * tiles that never straddle systems.  Launch shape {lanes per row, rows
 * per block, entries per lane per pass, tile rows}: {64, R, CH, TR} cuts a
 * tile of TR rows (512 or 1024) into blocks of R rows (16, 32 or 64), each
 * streamed by one wave with CH entries (2 or 4) per lane per pass;
 * {32, 0, 0, TR} gives each row 32 lanes.  With opts->shape all 0 the
 * shape is tuned and cached as for hk_sweep_solve (key: device, n, nnz,
 * longest row, nsys) over all 14 candidates; a nonzero opts->shape must be
 * one of them.  infos[k].shape holds the shape used.
 */
int hk_blockdiag_solve(hk_csr A, int32_t nsys, const int64_t* row_off, const void* d_b, void* d_x,
                       const hk_solve_opts* opts, hk_solve_info* infos, void* stream);

/* --------------------------------------------- operator and adjoint */

/*
 * Helmholtz matrix values for a piecewise-constant sound speed (the paper's
 * operator -lap(u) - k^2 u with a speed that varies in space, Introduction):
 *   val[p] = K[p] - omega^2 (1 + i damp) * sum_q bm_val[q] / c[bm_blk[q]]^2,
 * q over [bm_ptr[p], bm_ptr[p+1]): the mass of entry p split by speed block
 * (element masses of the elements of each block, Dirichlet entries
 * removed).  d_K, d_bm_val, d_c: double; d_bm_ptr: nnz+1 int32 offsets into
 * the nlist-long lists d_bm_blk (int32 block ids < nblocks) and d_bm_val;
 * d_val: nnz complex128 (output).  Malformed lists give HK_EINVAL.
 * Synchronises `stream` (error check).
 */
int hk_assemble_helmholtz(int64_t nnz, const double* d_K, const int32_t* d_bm_ptr,
                          const int32_t* d_bm_blk, const double* d_bm_val, int64_t nlist,
                          int32_t nblocks, const double* d_c, double omega, double damp,
                          void* d_val, void* stream);

/*
 * Adjoint sensitivities of a real loss to the block speeds (not in the
 * paper; differentiation of the operator above): with u = A(c)^-1 g and
 * lambda solving A lambda = conj(dL/du) (A is complex symmetric, so this is
 * the forward solver on the same matrix),
 *   grad_c[b] = -Re( 2 omega^2 (1 + i damp) c_b^-3 sum_{e in b} lambda_e^T M_e u_e ),
 * M_e the P1 element mass matrix vol_e/20 (1 + delta_ab) with Dirichlet
 * nodes masked.  Elements of block b are d_tet_nodes[4*e .. 4*e+3] for e in
 * [d_tet_ptr[b], d_tet_ptr[b+1]); d_tet_vol their volumes; d_dirichlet one
 * byte per node (nonzero: Dirichlet).  d_lambda, d_u: n complex128;
 * d_grad_c: nblocks doubles (output).  One workgroup per block, fixed
 * summation order.  Synchronises `stream` (error checks).
 */
int hk_elem_sens(int64_t n, int64_t ntet, int32_t nblocks, const int32_t* d_tet_nodes,
                 const int32_t* d_tet_ptr, const double* d_tet_vol, const uint8_t* d_dirichlet,
                 const void* d_lambda, const void* d_u, const double* d_c, double omega,
                 double damp, double* d_grad_c, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HK_H_ */
