/*
 * hk_oracle.c -- plain CPU oracle for the complex Helmholtz Krylov path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header or constant with the HIP library and never calls it.
 *
 * Everything is written the slow, obvious way in double precision (complex
 * double, as the paper fixes), except the inner solve of the mixed-precision
 * refinement, whose vectors and matrix are complex float (its dots are
 * accumulated in double, see orc_bicgstab_c64).  Sums run left to right
 * in index order; the only parallelism is over independent rows or elements
 * (OpenMP), which leaves every result bitwise identical to a serial run.
 *
 * Sources (the paper, arXiv 2112.11880):
 *   - CSR storage of the FE matrices: Section 2.
 *   - complex scal / axpy / element-wise product: Section 3 listings.
 *   - dot product as element-wise product followed by a sum: Section 3 (ZDOT).
 *   - L2 norm: Section 3 (ZNORM, Table 7).
 *   - preconditioned BiCGStab with zero initial guess, residual tolerance and
 *     an iteration cap: Section 4.  The preconditioner is Jacobi (diagonal),
 *     applied on the right (readings in the design notes).
 * The mixed-precision refinement, the adjoint and the element sensitivities
 * are not in the paper; they follow the mathematics stated at each function.
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* loops shorter than this run on one thread (team start-up would dominate) */
#define OR_PAR_MIN 65536

typedef double _Complex zd;
typedef float _Complex zf;

/* status codes (same meaning as the library's, defined independently) */
enum { OR_OK = 0, OR_NOT_CONVERGED = 1, OR_BREAKDOWN = 2, OR_NONFINITE = 3, OR_EINVAL = -1 };
/* which scalar broke down */
enum { OR_BD_NONE = 0, OR_BD_RHO = 1, OR_BD_SIGMA = 2, OR_BD_TAU = 3, OR_BD_OMEGA = 4 };

typedef struct {
    int64_t iters;
    double relres_rec;   /* recursive residual norm / ||b|| */
    double relres_true;  /* ||b - A x|| / ||b|| recomputed at exit */
    int32_t status;
    int32_t breakdown;   /* OR_BD_* */
} or_info;

/* Thread count of the OpenMP loops, for the host-baseline timings.  Every
 * parallel loop writes independent rows or elements and every sum runs on
 * one thread in index order, so results do not depend on it. */
void orc_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }

/* ---------------------------------------------------------------- kernels */

/* y_i = sum_{p=rowptr[i]}^{rowptr[i+1]-1} val[p] * x[col[p]], ascending p. */
void orc_spmv(int64_t n, const int32_t *rowptr, const int32_t *col, const zd *val,
              const zd *x, zd *y)
{
#pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
    for (int64_t i = 0; i < n; ++i) {
        zd acc = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            acc += val[p] * x[col[p]];
        y[i] = acc;
    }
}

/* r = b - A x */
void orc_residual(int64_t n, const int32_t *rowptr, const int32_t *col, const zd *val,
                  const zd *b, const zd *x, zd *r)
{
#pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
    for (int64_t i = 0; i < n; ++i) {
        zd acc = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            acc += val[p] * x[col[p]];
        r[i] = b[i] - acc;
    }
}

/* x^H y = sum conj(x_i) y_i */
zd orc_zdotc_v(int64_t n, const zd *x, const zd *y)
{
    zd s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += conj(x[i]) * y[i];
    return s;
}

/* x^T y = sum x_i y_i */
zd orc_zdotu_v(int64_t n, const zd *x, const zd *y)
{
    zd s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

/* ||x||_2 = sqrt(sum re^2 + im^2) */
double orc_dznrm2(int64_t n, const zd *x)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
    return sqrt(s);
}

void orc_zdotc(int64_t n, const zd *x, const zd *y, zd *out) { *out = orc_zdotc_v(n, x, y); }
void orc_zdotu(int64_t n, const zd *x, const zd *y, zd *out) { *out = orc_zdotu_v(n, x, y); }

/* y = alpha x + y */
void orc_zaxpy(int64_t n, const zd *alpha, const zd *x, zd *y)
{
    zd a = *alpha;
#pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
    for (int64_t i = 0; i < n; ++i) y[i] = a * x[i] + y[i];
}

/* x = alpha x */
void orc_zscal(int64_t n, const zd *alpha, zd *x)
{
    zd a = *alpha;
#pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
    for (int64_t i = 0; i < n; ++i) x[i] = a * x[i];
}

/* y = x .* y (element-wise product) */
void orc_zaxmy(int64_t n, const zd *x, zd *y)
{
#pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
    for (int64_t i = 0; i < n; ++i) y[i] = x[i] * y[i];
}

/* y = x */
void orc_zcopy(int64_t n, const zd *x, zd *y)
{
    for (int64_t i = 0; i < n; ++i) y[i] = x[i];
}

/* ---------------------------------------------------- BiCGStab (FP64) */

static int isfinite_z(zd z) { return isfinite(creal(z)) && isfinite(cimag(z)); }

/* diagonal of a CSR matrix; returns 0 if a row has no (nonzero) diagonal */
static int diag_inverse(int64_t n, const int32_t *rowptr, const int32_t *col, const zd *val,
                        zd *dinv)
{
    for (int64_t i = 0; i < n; ++i) {
        zd d = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            if (col[p] == i) d += val[p];
        if (d == 0.0) return 0;
        dinv[i] = 1.0 / d;
    }
    return 1;
}

/*
 * Right-preconditioned BiCGStab (van der Vorst's recurrences, as given in
 * Saad's book which the paper cites for P-BiCGSTAB), preconditioner
 * M = diag(A) when precond != 0, identity otherwise.
 *
 * x holds the initial guess on entry (the paper starts from zero) and the
 * last iterate on exit.  Stops when ||r||_2 <= tol * ||b||_2, checked after
 * the half step (s) and after the full step (r).  A breakdown is declared
 * when rho = rhat^H r, sigma = rhat^H v, tau = t^H t or omega is exactly
 * zero; a non-finite scalar ends the solve with OR_NONFINITE.  A half-step
 * exit counts as an iteration; a breakdown at rho or sigma does not.
 * history (optional, maxit+1 entries) receives ||r_k|| / ||b||.
 */
int orc_bicgstab(int64_t n, const int32_t *rowptr, const int32_t *col, const zd *val,
                 const zd *b, zd *x, double tol, int64_t maxit, int precond,
                 or_info *info, double *history)
{
    memset(info, 0, sizeof(*info));
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite_z(b[i]) || !isfinite_z(x[i])) { info->status = OR_NONFINITE; return OR_NONFINITE; }

    zd *dinv = malloc(sizeof(zd) * n), *r = malloc(sizeof(zd) * n), *rh = malloc(sizeof(zd) * n);
    zd *p = malloc(sizeof(zd) * n), *v = malloc(sizeof(zd) * n), *s = malloc(sizeof(zd) * n);
    zd *t = malloc(sizeof(zd) * n), *ph = malloc(sizeof(zd) * n), *sh = malloc(sizeof(zd) * n);
    int status = OR_NOT_CONVERGED, bd = OR_BD_NONE;
    int64_t it = 0;
    double bnorm = 0.0, rnorm = 0.0;

    if (precond) {
        if (!diag_inverse(n, rowptr, col, val, dinv)) { status = OR_EINVAL; goto done; }
    } else {
        for (int64_t i = 0; i < n; ++i) dinv[i] = 1.0;
    }

    bnorm = orc_dznrm2(n, b);
    orc_residual(n, rowptr, col, val, b, x, r);
    for (int64_t i = 0; i < n; ++i) rh[i] = r[i];
    rnorm = orc_dznrm2(n, r);
    double theta = tol * bnorm;
    if (history) history[0] = bnorm > 0 ? rnorm / bnorm : 0.0;
    if (rnorm <= theta) { status = OR_OK; goto done; }

    zd rho_old = 1.0, alpha = 1.0, omega = 1.0;
    for (int64_t i = 0; i < n; ++i) { p[i] = 0.0; v[i] = 0.0; }

    for (it = 1; it <= maxit; ++it) {
        zd rho = orc_zdotc_v(n, rh, r);
        if (!isfinite_z(rho)) { status = OR_NONFINITE; break; }
        if (rho == 0.0) { status = OR_BREAKDOWN; bd = OR_BD_RHO; it -= 1; break; }
        if (it == 1) {
            for (int64_t i = 0; i < n; ++i) p[i] = r[i];
        } else {
            zd beta = (rho / rho_old) * (alpha / omega);
            for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        }
        for (int64_t i = 0; i < n; ++i) ph[i] = dinv[i] * p[i];
        orc_spmv(n, rowptr, col, val, ph, v);
        zd sigma = orc_zdotc_v(n, rh, v);
        if (!isfinite_z(sigma)) { status = OR_NONFINITE; break; }
        if (sigma == 0.0) { status = OR_BREAKDOWN; bd = OR_BD_SIGMA; it -= 1; break; }
        alpha = rho / sigma;
        for (int64_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        double snorm = orc_dznrm2(n, s);
        if (snorm <= theta) {
            for (int64_t i = 0; i < n; ++i) x[i] += alpha * ph[i];
            rnorm = snorm;
            status = OR_OK;
            break;
        }
        for (int64_t i = 0; i < n; ++i) sh[i] = dinv[i] * s[i];
        orc_spmv(n, rowptr, col, val, sh, t);
        double tau = creal(orc_zdotc_v(n, t, t));
        if (tau == 0.0) {
            for (int64_t i = 0; i < n; ++i) x[i] += alpha * ph[i];
            rnorm = snorm;
            status = OR_BREAKDOWN; bd = OR_BD_TAU;
            break;
        }
        omega = orc_zdotc_v(n, t, s) / tau;
        for (int64_t i = 0; i < n; ++i) x[i] += alpha * ph[i] + omega * sh[i];
        for (int64_t i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
        rho_old = rho;
        rnorm = orc_dznrm2(n, r);
        if (history) history[it] = rnorm / bnorm;
        if (!isfinite(rnorm) || !isfinite_z(omega)) { status = OR_NONFINITE; break; }
        if (rnorm <= theta) { status = OR_OK; break; }
        if (omega == 0.0) { status = OR_BREAKDOWN; bd = OR_BD_OMEGA; break; }
    }
    if (it > maxit) it = maxit;

done:
    info->relres_rec = bnorm > 0 ? rnorm / bnorm : rnorm;
    info->iters = it;
    info->status = status;
    info->breakdown = bd;
    if (status != OR_EINVAL) {
        orc_residual(n, rowptr, col, val, b, x, r);
        double bn = orc_dznrm2(n, b);
        info->relres_true = bn > 0 ? orc_dznrm2(n, r) / bn : orc_dznrm2(n, r);
    }
    free(dinv); free(r); free(rh); free(p); free(v); free(s); free(t); free(ph); free(sh);
    return status;
}

/*
 * Right-preconditioned transpose-free QMR (Freund's method, as given in
 * Saad's book which the paper cites for P-TFQMR), preconditioner M = diag(A)
 * when precond != 0, identity otherwise.  The recurrences run on
 * Ahat = A M^-1; the iterate is kept in x directly (x += eta M^-1 d).
 *
 * Start: w = y_1 = r_0 = b - A x_0, rhat = r_0, u_1 = Ahat y_1, v = u_1,
 * d = 0, theta = eta = 0, tau = ||r_0||, rho = rhat^H r_0.  Iteration k:
 *   alpha = rho / (rhat^H v),  y_2 = y_1 - alpha v,  u_2 = Ahat y_2
 *   half-steps j = 1, 2 (overall half-step m = 2k - 2 + j):
 *     w = w - alpha u_j
 *     d = y_j + (theta^2 eta / alpha) d
 *     theta = ||w|| / tau,  c = (1 + theta^2)^(-1/2)
 *     tau = tau theta c,  eta = c^2 alpha
 *     x += eta M^-1 d
 *   rho' = rhat^H w,  beta = rho' / rho,  rho = rho'
 *   y_1 = w + beta y_2,  u_1 = Ahat y_1,  v = u_1 + beta (u_2 + beta v)
 * Two products with Ahat per iteration.  The solve stops as soon as the
 * quasi-residual bound sqrt(m+1) tau <= tol ||b|| (an exit after the first
 * half-step counts the iteration).  A breakdown is declared when rhat^H v
 * (OR_BD_SIGMA, before the iteration counts) or rhat^H w (OR_BD_RHO, after
 * it) is exactly zero; a non-finite scalar ends the solve with OR_NONFINITE.
 * relres_rec is the last bound divided by ||b||; history (optional, maxit+1
 * entries) receives it at the end of every iteration.
 */
int orc_tfqmr(int64_t n, const int32_t *rowptr, const int32_t *col, const zd *val,
              const zd *b, zd *x, double tol, int64_t maxit, int precond,
              or_info *info, double *history)
{
    memset(info, 0, sizeof(*info));
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite_z(b[i]) || !isfinite_z(x[i])) { info->status = OR_NONFINITE; return OR_NONFINITE; }

    zd *dinv = malloc(sizeof(zd) * n), *w = malloc(sizeof(zd) * n), *rh = malloc(sizeof(zd) * n);
    zd *y1 = malloc(sizeof(zd) * n), *y2 = malloc(sizeof(zd) * n), *u1 = malloc(sizeof(zd) * n);
    zd *u2 = malloc(sizeof(zd) * n), *v = malloc(sizeof(zd) * n), *d = malloc(sizeof(zd) * n);
    zd *tmp = malloc(sizeof(zd) * n);
    int status = OR_NOT_CONVERGED, bd = OR_BD_NONE;
    int64_t it = 0;
    double bnorm = 0.0, bound = 0.0;

    if (precond) {
        if (!diag_inverse(n, rowptr, col, val, dinv)) { status = OR_EINVAL; goto done; }
    } else {
        for (int64_t i = 0; i < n; ++i) dinv[i] = 1.0;
    }

    bnorm = orc_dznrm2(n, b);
    orc_residual(n, rowptr, col, val, b, x, w);
    for (int64_t i = 0; i < n; ++i) { rh[i] = w[i]; y1[i] = w[i]; d[i] = 0.0; }
    double tau = orc_dznrm2(n, w), theta = 0.0;
    const double thr = tol * bnorm;
    zd eta = 0.0, rho = orc_zdotc_v(n, rh, w);
    bound = tau;
    if (history) history[0] = bnorm > 0 ? tau / bnorm : 0.0;
    if (tau <= thr) { status = OR_OK; goto done; }

    for (int64_t i = 0; i < n; ++i) tmp[i] = dinv[i] * y1[i];
    orc_spmv(n, rowptr, col, val, tmp, u1);
    for (int64_t i = 0; i < n; ++i) v[i] = u1[i];

    for (it = 1; it <= maxit; ++it) {
        zd sigma = orc_zdotc_v(n, rh, v);
        if (!isfinite_z(sigma)) { status = OR_NONFINITE; it -= 1; break; }
        if (sigma == 0.0) { status = OR_BREAKDOWN; bd = OR_BD_SIGMA; it -= 1; break; }
        const zd alpha = rho / sigma;
        for (int64_t i = 0; i < n; ++i) y2[i] = y1[i] - alpha * v[i];
        for (int64_t i = 0; i < n; ++i) tmp[i] = dinv[i] * y2[i];
        orc_spmv(n, rowptr, col, val, tmp, u2);
        int stop = 0;
        for (int j = 1; j <= 2 && !stop; ++j) {
            const zd *yj = j == 1 ? y1 : y2, *uj = j == 1 ? u1 : u2;
            const int64_t m = 2 * it - 2 + j;
            for (int64_t i = 0; i < n; ++i) w[i] -= alpha * uj[i];
            const zd coef = theta * theta * eta / alpha;
            for (int64_t i = 0; i < n; ++i) d[i] = yj[i] + coef * d[i];
            theta = orc_dznrm2(n, w) / tau;
            const double c = 1.0 / sqrt(1.0 + theta * theta);
            tau = tau * theta * c;
            eta = c * c * alpha;
            for (int64_t i = 0; i < n; ++i) x[i] += eta * (dinv[i] * d[i]);
            bound = tau * sqrt((double)(m + 1));
            if (!isfinite(tau) || !isfinite_z(eta)) { status = OR_NONFINITE; stop = 1; }
            else if (bound <= thr) { status = OR_OK; stop = 1; }
        }
        if (history) history[it] = bnorm > 0 ? bound / bnorm : bound;
        if (stop) break;
        zd rho_new = orc_zdotc_v(n, rh, w);
        if (!isfinite_z(rho_new)) { status = OR_NONFINITE; break; }
        if (rho_new == 0.0) { status = OR_BREAKDOWN; bd = OR_BD_RHO; break; }
        const zd beta = rho_new / rho;
        rho = rho_new;
        for (int64_t i = 0; i < n; ++i) y1[i] = w[i] + beta * y2[i];
        for (int64_t i = 0; i < n; ++i) tmp[i] = dinv[i] * y1[i];
        orc_spmv(n, rowptr, col, val, tmp, u1);
        for (int64_t i = 0; i < n; ++i) v[i] = u1[i] + beta * (u2[i] + beta * v[i]);
    }
    if (it > maxit) it = maxit;

done:
    info->relres_rec = bnorm > 0 ? bound / bnorm : bound;
    info->iters = it;
    info->status = status;
    info->breakdown = bd;
    if (status != OR_EINVAL) {
        orc_residual(n, rowptr, col, val, b, x, w);
        info->relres_true = bnorm > 0 ? orc_dznrm2(n, w) / bnorm : orc_dznrm2(n, w);
    }
    free(dinv); free(w); free(rh); free(y1); free(y2); free(u1); free(u2); free(v); free(d); free(tmp);
    return status;
}

/*
 * Right-preconditioned BiCGStab(l) (Sleijpen and Fokkema's method; the
 * paper's P-BiCGSTAB(l) with l = 8 in Section 4), preconditioner M = diag(A)
 * when precond != 0, identity otherwise, on Ahat = A M^-1 with the iterate
 * kept in x (x += M^-1 ...).  One iteration is a cycle of l BiCG steps and
 * one minimal-residual step (2 l products with Ahat):
 *
 *   rho0 = -omega rho0
 *   for j = 0 .. l-1:
 *     rho1 = rt^H r_j,  beta = alpha rho1 / rho0,  rho0 = rho1
 *     u_i = r_i - beta u_i (i <= j);   u_{j+1} = Ahat u_j
 *     alpha = rho0 / (rt^H u_{j+1})
 *     r_i = r_i - alpha u_{i+1} (i <= j);   r_{j+1} = Ahat r_j
 *     x += alpha M^-1 u_0
 *   MR: gamma minimises ||r_0 - sum_{j>=1} gamma_j r_j||, taken from the
 *   normal equations Z gamma = z with Z_ij = r_i^H r_j, z_i = r_i^H r_0
 *   (i, j = 1..l; Cholesky), then
 *     x += sum_j gamma_j M^-1 r_{j-1},  r_0 -= sum_j gamma_j r_j,
 *     u_0 -= sum_j gamma_j u_j,  omega = gamma_l
 *
 * starting from r_0 = b - A x_0, rt = r_0, u_0 = 0, rho0 = omega = 1,
 * alpha = 0.  (For l = 1 this is BiCGStab.)  Stops when ||r_0|| <= tol ||b||,
 * tested after every BiCG step and after the minimal-residual step (an exit
 * inside a cycle counts the cycle).  Breakdown when rt^H r_j (OR_BD_RHO) or rt^H u_{j+1}
 * (OR_BD_SIGMA) is exactly zero (the cycle does not count), when a Cholesky
 * pivot of Z is not positive (OR_BD_TAU), or when omega = 0 (OR_BD_OMEGA).
 * history (optional, maxit+1 entries) receives ||r_0|| / ||b|| per cycle.
 */
#define OR_MAXL 16
int orc_bicgstab_l(int64_t n, const int32_t *rowptr, const int32_t *col, const zd *val,
                   const zd *b, zd *x, double tol, int64_t maxit, int ell, int precond,
                   or_info *info, double *history)
{
    memset(info, 0, sizeof(*info));
    if (ell < 1 || ell > OR_MAXL) { info->status = OR_EINVAL; return OR_EINVAL; }
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite_z(b[i]) || !isfinite_z(x[i])) { info->status = OR_NONFINITE; return OR_NONFINITE; }

    zd *r[OR_MAXL + 1], *u[OR_MAXL + 1];
    for (int j = 0; j <= ell; ++j) { r[j] = malloc(sizeof(zd) * n); u[j] = malloc(sizeof(zd) * n); }
    zd *dinv = malloc(sizeof(zd) * n), *rt = malloc(sizeof(zd) * n), *tmp = malloc(sizeof(zd) * n);
    int status = OR_NOT_CONVERGED, bd = OR_BD_NONE;
    int64_t it = 0;
    double bnorm = 0.0, rnorm = 0.0;

    if (precond) {
        if (!diag_inverse(n, rowptr, col, val, dinv)) { status = OR_EINVAL; goto done; }
    } else {
        for (int64_t i = 0; i < n; ++i) dinv[i] = 1.0;
    }
    bnorm = orc_dznrm2(n, b);
    orc_residual(n, rowptr, col, val, b, x, r[0]);
    for (int64_t i = 0; i < n; ++i) { rt[i] = r[0][i]; u[0][i] = 0.0; }
    rnorm = orc_dznrm2(n, r[0]);
    const double thr = tol * bnorm;
    if (history) history[0] = bnorm > 0 ? rnorm / bnorm : 0.0;
    if (rnorm <= thr) { status = OR_OK; goto done; }

    zd rho0 = 1.0, alpha = 0.0, omega = 1.0;
    for (it = 1; it <= maxit; ++it) {
        rho0 = -omega * rho0;
        int fail = 0;
        for (int j = 0; j < ell && !fail; ++j) {
            zd rho1 = orc_zdotc_v(n, rt, r[j]);
            if (!isfinite_z(rho1)) { status = OR_NONFINITE; fail = 1; break; }
            if (rho1 == 0.0) { status = OR_BREAKDOWN; bd = OR_BD_RHO; fail = 1; break; }
            const zd beta = alpha * rho1 / rho0;
            rho0 = rho1;
            for (int i = 0; i <= j; ++i)
                for (int64_t q = 0; q < n; ++q) u[i][q] = r[i][q] - beta * u[i][q];
            for (int64_t q = 0; q < n; ++q) tmp[q] = dinv[q] * u[j][q];
            orc_spmv(n, rowptr, col, val, tmp, u[j + 1]);
            zd gam = orc_zdotc_v(n, rt, u[j + 1]);
            if (!isfinite_z(gam)) { status = OR_NONFINITE; fail = 1; break; }
            if (gam == 0.0) { status = OR_BREAKDOWN; bd = OR_BD_SIGMA; fail = 1; break; }
            alpha = rho0 / gam;
            for (int i = 0; i <= j; ++i)
                for (int64_t q = 0; q < n; ++q) r[i][q] -= alpha * u[i + 1][q];
            for (int64_t q = 0; q < n; ++q) tmp[q] = dinv[q] * r[j][q];
            orc_spmv(n, rowptr, col, val, tmp, r[j + 1]);
            for (int64_t q = 0; q < n; ++q) x[q] += alpha * (dinv[q] * u[0][q]);
            rnorm = orc_dznrm2(n, r[0]);
            if (rnorm <= thr) { status = OR_OK; fail = 2; }
        }
        if (fail == 2) { if (history) history[it] = rnorm / bnorm; break; }
        if (fail) { it -= 1; break; }
        /* minimal-residual step through the normal equations */
        zd Z[OR_MAXL][OR_MAXL], z[OR_MAXL], L[OR_MAXL][OR_MAXL], g[OR_MAXL], w[OR_MAXL];
        for (int i = 1; i <= ell; ++i) {
            z[i - 1] = orc_zdotc_v(n, r[i], r[0]);
            for (int j = 1; j <= ell; ++j) Z[i - 1][j - 1] = orc_zdotc_v(n, r[i], r[j]);
        }
        /* Z = L L^H */
        for (int j = 0; j < ell && !fail; ++j) {
            double d = creal(Z[j][j]);
            for (int k = 0; k < j; ++k) d -= creal(L[j][k] * conj(L[j][k]));
            if (!(d > 0.0)) { status = OR_BREAKDOWN; bd = OR_BD_TAU; fail = 1; break; }
            L[j][j] = sqrt(d);
            for (int i = j + 1; i < ell; ++i) {
                zd sij = Z[i][j];
                for (int k = 0; k < j; ++k) sij -= L[i][k] * conj(L[j][k]);
                L[i][j] = sij / L[j][j];
            }
        }
        if (fail) break;
        for (int i = 0; i < ell; ++i) {          /* L w = z */
            zd sum = z[i];
            for (int k = 0; k < i; ++k) sum -= L[i][k] * w[k];
            w[i] = sum / L[i][i];
        }
        for (int i = ell - 1; i >= 0; --i) {     /* L^H g = w */
            zd sum = w[i];
            for (int k = i + 1; k < ell; ++k) sum -= conj(L[k][i]) * g[k];
            g[i] = sum / L[i][i];
        }
        for (int j = 1; j <= ell; ++j) {
            const zd gj = g[j - 1];
            for (int64_t q = 0; q < n; ++q) {
                x[q] += gj * (dinv[q] * r[j - 1][q]);
                r[0][q] -= gj * r[j][q];
                u[0][q] -= gj * u[j][q];
            }
        }
        omega = g[ell - 1];
        rnorm = orc_dznrm2(n, r[0]);
        if (history) history[it] = bnorm > 0 ? rnorm / bnorm : 0.0;
        if (!isfinite(rnorm) || !isfinite_z(omega)) { status = OR_NONFINITE; break; }
        if (rnorm <= thr) { status = OR_OK; break; }
        if (omega == 0.0) { status = OR_BREAKDOWN; bd = OR_BD_OMEGA; break; }
    }
    if (it > maxit) it = maxit;

done:
    info->relres_rec = bnorm > 0 ? rnorm / bnorm : rnorm;
    info->iters = it;
    info->status = status;
    info->breakdown = bd;
    if (status != OR_EINVAL) {
        orc_residual(n, rowptr, col, val, b, x, tmp);
        info->relres_true = bnorm > 0 ? orc_dznrm2(n, tmp) / bnorm : orc_dznrm2(n, tmp);
    }
    for (int j = 0; j <= ell; ++j) { free(r[j]); free(u[j]); }
    free(dinv); free(rt); free(tmp);
    return status;
}

/* ------------------------------------------ complex-float inner BiCGStab */

static void spmv_f(int64_t n, const int32_t *rowptr, const int32_t *col, const zf *val,
                   const zf *x, zf *y)
{
#pragma omp parallel for schedule(static) if (n >= OR_PAR_MIN)
    for (int64_t i = 0; i < n; ++i) {
        zf acc = 0.0f;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            acc += val[p] * x[col[p]];
        y[i] = acc;
    }
}

/* conj(x)^T y of complex-float vectors, accumulated in double (each product
 * of two floats is exact in double) */
static zd dotc_fd(int64_t n, const zf *x, const zf *y)
{
    zd s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += conj((zd)x[i]) * (zd)y[i];
    return s;
}

static double nrm2_fd(int64_t n, const zf *x)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double re = crealf(x[i]), im = cimagf(x[i]);
        s += re * re + im * im;
    }
    return sqrt(s);
}

/*
 * The same right-preconditioned BiCGStab with complex-float vectors, matrix
 * and matrix-vector products, x0 = 0, relative tolerance on ||r|| / ||b||.
 * The inner products and norms are accumulated in double and the scalars
 * (rho, sigma, alpha, omega, beta, tau) are formed in double; each vector
 * update uses the scalar rounded to complex float.  (With float
 * accumulation the dot of n terms carries a rounding error of order
 * sqrt(n) 2^-24 ||rhat|| ||r||, which on these systems exceeds |rhat^H r|
 * itself once bi-orthogonality is lost, and the iteration then breaks down
 * or stalls depending on the summation order.)  On a breakdown (the same
 * exact-zero tests) the current iterate is kept and returned.
 */
int orc_bicgstab_c64(int64_t n, const int32_t *rowptr, const int32_t *col, const zf *val,
                     const zf *b, zf *x, float tol, int64_t maxit, or_info *info)
{
    memset(info, 0, sizeof(*info));
    zf *dinv = malloc(sizeof(zf) * n), *r = malloc(sizeof(zf) * n), *rh = malloc(sizeof(zf) * n);
    zf *p = malloc(sizeof(zf) * n), *v = malloc(sizeof(zf) * n), *s = malloc(sizeof(zf) * n);
    zf *t = malloc(sizeof(zf) * n), *ph = malloc(sizeof(zf) * n), *sh = malloc(sizeof(zf) * n);
    int status = OR_NOT_CONVERGED, bd = OR_BD_NONE;
    int64_t it = 0;
    for (int64_t i = 0; i < n; ++i) {
        zf d = 0.0f;
        for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q)
            if (col[q] == i) d += val[q];
        if (d == 0.0f) { status = OR_EINVAL; goto done; }
        dinv[i] = 1.0f / d;
    }
    for (int64_t i = 0; i < n; ++i) { x[i] = 0.0f; r[i] = b[i]; rh[i] = b[i]; p[i] = 0.0f; v[i] = 0.0f; }
    double bnorm = nrm2_fd(n, b), rnorm = bnorm, theta = (double)tol * bnorm;
    if (rnorm <= theta) { status = OR_OK; goto done; }
    zd rho_old = 1.0, alpha = 1.0, omega = 1.0;
    for (it = 1; it <= maxit; ++it) {
        zd rho = dotc_fd(n, rh, r);
        if (!isfinite(creal(rho)) || !isfinite(cimag(rho))) { status = OR_NONFINITE; break; }
        if (rho == 0.0) { status = OR_BREAKDOWN; bd = OR_BD_RHO; it -= 1; break; }
        if (it == 1) {
            for (int64_t i = 0; i < n; ++i) p[i] = r[i];
        } else {
            zf beta = (zf)((rho / rho_old) * (alpha / omega)), om = (zf)omega;
            for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - om * v[i]);
        }
        for (int64_t i = 0; i < n; ++i) ph[i] = dinv[i] * p[i];
        spmv_f(n, rowptr, col, val, ph, v);
        zd sigma = dotc_fd(n, rh, v);
        if (!isfinite(creal(sigma)) || !isfinite(cimag(sigma))) { status = OR_NONFINITE; break; }
        if (sigma == 0.0) { status = OR_BREAKDOWN; bd = OR_BD_SIGMA; it -= 1; break; }
        alpha = rho / sigma;
        const zf al = (zf)alpha;
        for (int64_t i = 0; i < n; ++i) s[i] = r[i] - al * v[i];
        double snorm = nrm2_fd(n, s);
        if (snorm <= theta) {
            for (int64_t i = 0; i < n; ++i) x[i] += al * ph[i];
            rnorm = snorm; status = OR_OK; break;
        }
        for (int64_t i = 0; i < n; ++i) sh[i] = dinv[i] * s[i];
        spmv_f(n, rowptr, col, val, sh, t);
        double tau = creal(dotc_fd(n, t, t));
        if (tau == 0.0) {
            for (int64_t i = 0; i < n; ++i) x[i] += al * ph[i];
            rnorm = snorm; status = OR_BREAKDOWN; bd = OR_BD_TAU; break;
        }
        omega = dotc_fd(n, t, s) / tau;
        const zf om = (zf)omega;
        for (int64_t i = 0; i < n; ++i) x[i] += al * ph[i] + om * sh[i];
        for (int64_t i = 0; i < n; ++i) r[i] = s[i] - om * t[i];
        rho_old = rho;
        rnorm = nrm2_fd(n, r);
        if (!isfinite(rnorm)) { status = OR_NONFINITE; break; }
        if (rnorm <= theta) { status = OR_OK; break; }
        if (omega == 0.0) { status = OR_BREAKDOWN; bd = OR_BD_OMEGA; break; }
    }
    if (it > maxit) it = maxit;
    info->relres_rec = bnorm > 0 ? rnorm / bnorm : 0.0;
done:
    info->iters = it;
    info->status = status;
    info->breakdown = bd;
    free(dinv); free(r); free(rh); free(p); free(v); free(s); free(t); free(ph); free(sh);
    return status;
}

/*
 * Mixed-precision iterative refinement: the residual r = b - A u, its norm,
 * the test ||r|| <= outer_tol ||b|| and the update u += d are double; the
 * correction d solves A d = r approximately with the complex-float BiCGStab
 * above on the complex-float rounding of A (each component rounded to
 * nearest) to a tolerance relative to ||r|| of
 * max(inner_tol, outer_tol ||b|| / (2 ||r||)): inner_tol, except in a cycle
 * that needs a smaller reduction to reach outer_tol, which stops at half of
 * that reduction.  u holds the initial guess on entry.  info->iters counts outer cycles, *inner_total the inner
 * iterations.  A cycle that does not lower ||r|| counts as stagnation and
 * ends the loop with OR_NOT_CONVERGED.
 */
int orc_mixed_refine(int64_t n, const int32_t *rowptr, const int32_t *col, const zd *val,
                     const zd *b, zd *u, double inner_tol, double outer_tol, int max_outer,
                     int64_t max_inner, or_info *info, int64_t *inner_total)
{
    int64_t nnz = rowptr[n];
    zf *val32 = malloc(sizeof(zf) * nnz), *r32 = malloc(sizeof(zf) * n), *d32 = malloc(sizeof(zf) * n);
    zd *r = malloc(sizeof(zd) * n);
    for (int64_t q = 0; q < nnz; ++q) val32[q] = (float)creal(val[q]) + I * (float)cimag(val[q]);
    double bnorm = orc_dznrm2(n, b);
    int status = OR_NOT_CONVERGED;
    int k;
    double prev = INFINITY, rel = 0.0;
    *inner_total = 0;
    memset(info, 0, sizeof(*info));
    for (k = 0; k <= max_outer; ++k) {
        orc_residual(n, rowptr, col, val, b, u, r);
        double rn = orc_dznrm2(n, r);
        rel = bnorm > 0 ? rn / bnorm : rn;
        if (!isfinite(rn)) { status = OR_NONFINITE; break; }
        if (rel <= outer_tol) { status = OR_OK; break; }
        if (rn >= prev || k == max_outer) { status = OR_NOT_CONVERGED; break; }
        prev = rn;
        for (int64_t i = 0; i < n; ++i) r32[i] = (float)creal(r[i]) + I * (float)cimag(r[i]);
        double itol = 0.5 * outer_tol / rel;
        if (itol < inner_tol) itol = inner_tol;
        or_info in;
        int st = orc_bicgstab_c64(n, rowptr, col, val32, r32, d32, (float)itol, max_inner, &in);
        *inner_total += in.iters;
        if (st == OR_EINVAL || st == OR_NONFINITE) { status = st; break; }
        for (int64_t i = 0; i < n; ++i) u[i] += (double)crealf(d32[i]) + I * (double)cimagf(d32[i]);
    }
    info->iters = k;
    info->status = status;
    info->relres_rec = rel;
    info->relres_true = rel;
    free(val32); free(r32); free(d32); free(r);
    return status;
}

/* ------------------------------------------------ FE operator and adjoint */

/* Position of column j in CSR row i (linear search), or -1. */
static int64_t csr_find(const int32_t *rowptr, const int32_t *col, int64_t i, int64_t j)
{
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
        if (col[p] == j) return p;
    return -1;
}

static double tet_volume(const double *X, const int32_t *nd)
{
    const double *a = X + 3 * (int64_t)nd[0], *b = X + 3 * (int64_t)nd[1];
    const double *c = X + 3 * (int64_t)nd[2], *d = X + 3 * (int64_t)nd[3];
    double e1[3], e2[3], e3[3];
    for (int k = 0; k < 3; ++k) { e1[k] = b[k] - a[k]; e2[k] = c[k] - a[k]; e3[k] = d[k] - a[k]; }
    double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1])
               - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0])
               + e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
    return fabs(det) / 6.0;
}

/*
 * Complex Helmholtz operator for a piecewise-constant sound speed:
 *   A(c) = K - omega^2 (1 + i damp) sum_e c_{blk(e)}^-2 M_e,
 * where M_e[a][b] = vol_e / 20 * (1 + delta_ab) is the P1 element mass
 * matrix, entries touching a Dirichlet node are left out (symmetric
 * elimination; K already carries the unit diagonal of those rows), and the
 * result goes into the CSR pattern of K.  Returns -1 if an element entry has
 * no slot in the pattern.
 */
int orc_assemble_helmholtz(int64_t n, const int32_t *rowptr, const int32_t *col, const double *K,
                           const uint8_t *dirichlet, int64_t ntet, const int32_t *tet_nodes,
                           const int32_t *tet_block, const double *coords, const double *c,
                           double omega, double damp, zd *val)
{
    int64_t nnz = rowptr[n];
    double *Mc = calloc(nnz, sizeof(double));
    for (int64_t e = 0; e < ntet; ++e) {
        const int32_t *nd = tet_nodes + 4 * e;
        double vol = tet_volume(coords, nd);
        double w = 1.0 / (c[tet_block[e]] * c[tet_block[e]]);
        for (int a = 0; a < 4; ++a) {
            if (dirichlet[nd[a]]) continue;
            for (int b = 0; b < 4; ++b) {
                if (dirichlet[nd[b]]) continue;
                int64_t p = csr_find(rowptr, col, nd[a], nd[b]);
                if (p < 0) { free(Mc); return -1; }
                Mc[p] += w * vol / 20.0 * (a == b ? 2.0 : 1.0);
            }
        }
    }
    zd kappa2 = omega * omega * (1.0 + I * damp);
    for (int64_t p = 0; p < nnz; ++p) val[p] = K[p] - kappa2 * Mc[p];
    free(Mc);
    return 0;
}

/*
 * Gradient of a real loss with respect to the block speeds through
 * u = A(c)^-1 g, given u and the adjoint state lambda solving
 * A lambda = conj(dL/du-bar * 2) (A is complex symmetric):
 *   dL/dc_b = -Re( lambda^T (dA/dc_b) u ),
 *   dA/dc_b = 2 omega^2 (1 + i damp) c_b^-3 sum_{e in b} M_e  (Dirichlet entries removed).
 * The element term lambda_e^T M_e u_e is the plain double sum over a, b.
 */
void orc_elem_sens(int64_t ntet, const int32_t *tet_nodes, const int32_t *tet_block,
                   const double *coords, const uint8_t *dirichlet, const zd *lambda, const zd *u,
                   const double *c, int64_t nblocks, double omega, double damp, double *grad_c)
{
    zd *acc = calloc(nblocks, sizeof(zd));
    for (int64_t e = 0; e < ntet; ++e) {
        const int32_t *nd = tet_nodes + 4 * e;
        double vol = tet_volume(coords, nd);
        zd s = 0.0;
        for (int a = 0; a < 4; ++a) {
            if (dirichlet[nd[a]]) continue;
            for (int b = 0; b < 4; ++b) {
                if (dirichlet[nd[b]]) continue;
                s += lambda[nd[a]] * (vol / 20.0 * (a == b ? 2.0 : 1.0)) * u[nd[b]];
            }
        }
        acc[tet_block[e]] += s;
    }
    for (int64_t b = 0; b < nblocks; ++b) {
        zd dA = 2.0 * omega * omega * (1.0 + I * damp) / (c[b] * c[b] * c[b]);
        grad_c[b] = -creal(dA * acc[b]);
    }
    free(acc);
}
