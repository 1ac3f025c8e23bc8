"""Pins of the CPU oracle (CPU only).

Each oracle function is checked against something other than itself: dense
matrix-vector products and LU solves (LAPACK), exact rational sums
(fractions.Fraction), exact small-integer arithmetic, a closed-form plane-wave
response of the unjittered Kuhn stencil, SciPy's independent BiCGStab, torch's
dense complex autograd, and central finite differences.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from synth import helmholtz as H
from synth import configs


def tiny_problem(nc=3, jitter=0.2, seed=3, kappa2=complex(40.0, 0.4)):
    m = H.make_mesh(nc, nc, nc, 1.0 / nc, jitter=jitter, rng=np.random.default_rng(seed))
    p = H.build_problem(m)
    return p, H.helmholtz_values(p, kappa2)


def dense(p, val):
    A = np.zeros((p.n, p.n), dtype=np.complex128)
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    A[rows, p.col] = val
    return A


def crandn(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


# ------------------------------------------------------------------ SpMV

@pytest.mark.parametrize("nc", [2, 3, 4])
def test_spmv_matches_dense(oracle, nc):
    p, val = tiny_problem(nc)
    x = crandn(np.random.default_rng(nc), p.n)
    A = dense(p, val)
    y = oracle.spmv(p.rowptr, p.col, val, x)
    ref = A @ x
    bound = 1e-15 * 16 * (np.abs(A) @ np.abs(x))
    assert np.all(np.abs(y - ref) <= bound)


def test_spmv_plane_wave_closed_form(oracle):
    """Interior rows of A = K - kappa2 M on the unjittered mesh applied to
    x_j = exp(i theta . j) give x_i [h(6 - 2 sum cos) - kappa2 h^3 (0.4 +
    0.1 sum cos th_d + 1/15 sum_{d<e} cos(th_d + th_e) + 0.1 cos(th1+th2+th3))]."""
    nc = 8
    h = 1.0 / nc
    m = H.make_mesh(nc, nc, nc, h)
    p = H.build_problem(m)
    kappa2 = complex(250.0, 2.5)
    val = H.helmholtz_values(p, kappa2)
    th = np.array([0.3, -0.7, 1.1])
    i, j, k = m.ijk()
    x = np.exp(1j * (th[0] * i + th[1] * j + th[2] * k))
    y = oracle.spmv(p.rowptr, p.col, val, x)
    cs = np.cos(th)
    sym = (0.4 + 0.1 * cs.sum() + (np.cos(th[0] + th[1]) + np.cos(th[0] + th[2]) + np.cos(th[1] + th[2])) / 15.0
           + 0.1 * np.cos(th.sum()))
    lam = h * (6 - 2 * cs.sum()) - kappa2 * h ** 3 * sym
    inner = (i > 0) & (i < nc) & (j > 0) & (j < nc) & (k > 1) & (k < nc)
    assert np.max(np.abs(y[inner] - lam * x[inner])) < 1e-14


# -------------------------------------------------------------- BLAS-1

def _frac(z):
    return Fraction(z.real), Fraction(z.imag)


def _exact_dot(x, y, conj):
    sr, si = Fraction(0), Fraction(0)
    for a, b in zip(x, y):
        ar, ai = _frac(a)
        br, bi = _frac(b)
        if conj:
            ai = -ai
        sr += ar * br - ai * bi
        si += ar * bi + ai * br
    return sr, si


@pytest.mark.parametrize("conj", [True, False])
def test_dots_exact_on_dyadic_inputs(oracle, conj):
    rng = np.random.default_rng(11)
    n = 64
    x = (rng.integers(-1000, 1000, n) + 1j * rng.integers(-1000, 1000, n)) / 1024.0
    y = (rng.integers(-1000, 1000, n) + 1j * rng.integers(-1000, 1000, n)) / 512.0
    d = oracle.zdotc(x, y) if conj else oracle.zdotu(x, y)
    sr, si = _exact_dot(x, y, conj)
    assert Fraction(d.real) == sr and Fraction(d.imag) == si


@pytest.mark.parametrize("conj", [True, False])
def test_dots_within_rounding_of_exact(oracle, conj):
    rng = np.random.default_rng(12)
    n = 61
    x, y = crandn(rng, n), crandn(rng, n)
    d = oracle.zdotc(x, y) if conj else oracle.zdotu(x, y)
    sr, si = _exact_dot(x, y, conj)
    bound = 2 * n * 2.0 ** -53 * float(np.sum(np.abs(x) * np.abs(y)))
    assert abs(d.real - float(sr)) <= bound and abs(d.imag - float(si)) <= bound


def test_norm_and_dot_identities(oracle):
    rng = np.random.default_rng(13)
    x = crandn(rng, 50)
    nrm = oracle.dznrm2(x)
    exact = math.sqrt(float(sum(Fraction(v.real) ** 2 + Fraction(v.imag) ** 2 for v in x)))
    assert abs(nrm - exact) <= 1e-15 * exact * 4
    dxx = oracle.zdotc(x, x)
    assert dxx.imag == 0.0 and abs(dxx.real - nrm ** 2) <= 1e-13 * nrm ** 2
    dxi = oracle.zdotc(x, 1j * x)
    assert dxi.real == 0.0 and dxi.imag == dxx.real
    assert oracle.zdotu(np.ones(37), np.ones(37)) == 37


def test_axpy_scal_axmy_exact_on_integers(oracle):
    rng = np.random.default_rng(14)
    n = 40
    x = rng.integers(-50, 50, n) + 1j * rng.integers(-50, 50, n)
    y = rng.integers(-50, 50, n) + 1j * rng.integers(-50, 50, n)
    a = complex(3, -2)
    ex_axpy = [complex(a * complex(int(u.real), int(u.imag)) + complex(int(v.real), int(v.imag)))
               for u, v in zip(x, y)]
    assert np.array_equal(oracle.zaxpy(a, x, y), np.array(ex_axpy))
    assert np.array_equal(oracle.zscal(a, x), np.array([a * complex(u) for u in x]))
    assert np.array_equal(oracle.zaxmy(x, y), np.array([complex(u) * complex(v) for u, v in zip(x, y)]))


# ------------------------------------------------------------- BiCGStab

@pytest.mark.parametrize("nc,seed", [(3, 3), (4, 5)])
def test_bicgstab_matches_dense_lu(oracle, nc, seed):
    p, val = tiny_problem(nc, seed=seed)
    b = crandn(np.random.default_rng(seed), p.n)
    b[p.dirichlet] = 0
    x, info = oracle.bicgstab(p.rowptr, p.col, val, b, tol=1e-13)
    assert info["status"] == 0 and info["relres_true"] <= 2e-13
    xs = np.linalg.solve(dense(p, val), b)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_bicgstab_diagonal_converges_in_one_iteration(oracle):
    n = 20
    rng = np.random.default_rng(2)
    d = crandn(rng, n) + 3.0
    rowptr = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    b = crandn(rng, n)
    x, info = oracle.bicgstab(rowptr, col, d, b, tol=1e-12)
    assert info["status"] == 0 and info["iters"] == 1
    assert np.allclose(x, b / d, rtol=1e-14, atol=0)


def test_bicgstab_cube16_true_residual_and_scipy(oracle):
    c1 = configs.cube16()
    x8, i8 = oracle.bicgstab(c1["rowptr"], c1["col"], c1["val"], c1["g"], tol=1e-8)
    assert i8["status"] == 0 and i8["relres_true"] <= 1.05e-8
    x10, i10 = oracle.bicgstab(c1["rowptr"], c1["col"], c1["val"], c1["g"], tol=1e-10)
    assert i10["status"] == 0 and i10["relres_true"] <= 1.05e-10
    n = int(c1["n"])
    A = sp.csr_matrix((c1["val"], c1["col"], c1["rowptr"]), shape=(n, n))
    dinv = 1.0 / A.diagonal()
    M = spla.LinearOperator((n, n), matvec=lambda v: dinv * v, dtype=np.complex128)
    xs, flag = spla.bicgstab(A, c1["g"], rtol=1e-11, atol=0.0, maxiter=20000, M=M)
    assert flag == 0
    assert np.linalg.norm(x10 - xs) <= 1e-7 * np.linalg.norm(xs)


def test_bicgstab_sigma_breakdown(oracle):
    # D = I and g^H A g = 1*(-1.5) + 2*0.75 = 0 exactly at the first step
    rowptr = np.array([0, 2, 4], dtype=np.int32)
    col = np.array([0, 1, 0, 1], dtype=np.int32)
    val = np.array([1.0, -1.25, -1.25, 1.0], dtype=np.complex128)
    x, info = oracle.bicgstab(rowptr, col, val, np.array([1.0, 2.0]), tol=1e-12)
    assert info["status"] == oracle.BREAKDOWN and info["breakdown"] == oracle.BD_SIGMA
    assert info["iters"] == 0 and np.all(x == 0)


def test_bicgstab_omega_breakdown(oracle):
    """b = e1 and a11 = 1 give alpha = 1 and s = -(0, a21, a31) = -(0, 1, 1);
    with a22 + a23 + a32 + a33 = 0 the first omega = t^H s / t^H t is exactly 0."""
    A = np.array([[1, 1, 0], [1, 1, -1], [1, -1, 1]], dtype=np.complex128)
    rowptr = np.array([0, 3, 6, 9], dtype=np.int32)
    col = np.tile(np.arange(3, dtype=np.int32), 3)
    for pre in (False, True):  # diag(A) = I, so Jacobi changes nothing
        x, info = oracle.bicgstab(rowptr, col, A.ravel(), np.array([1.0, 0, 0]), tol=1e-14,
                                  precond=pre)
        assert info["status"] == oracle.BREAKDOWN and info["breakdown"] == oracle.BD_OMEGA
        assert info["iters"] == 1 and np.array_equal(x, np.array([1.0, 0, 0]))


def test_bicgstab_error_paths(oracle):
    c1 = configs.cube16()
    g = c1["g"].copy()
    g[5] = np.nan
    _, info = oracle.bicgstab(c1["rowptr"], c1["col"], c1["val"], g)
    assert info["status"] == oracle.NONFINITE
    rowptr = np.array([0, 1, 2], dtype=np.int32)
    col = np.array([1, 0], dtype=np.int32)
    _, info = oracle.bicgstab(rowptr, col, np.array([1.0, 1.0], dtype=complex), np.array([1.0, 1.0]))
    assert info["status"] == oracle.EINVAL
    x, info = oracle.bicgstab(c1["rowptr"], c1["col"], c1["val"], c1["g"], maxit=1)
    assert info["status"] == oracle.NOT_CONVERGED and info["iters"] == 1
    assert 0 < info["relres_true"] < 1 and np.any(x != 0)


# ------------------------------------------------------------- TFQMR

@pytest.mark.parametrize("nc,seed", [(3, 3), (4, 5)])
def test_tfqmr_matches_scipy_steps_and_dense_lu(oracle, nc, seed):
    """Right-preconditioned TFQMR: after k iterations (2k half-steps) the
    iterate equals SciPy's unpreconditioned TFQMR on the explicitly scaled
    operator A D^-1, mapped back by D^-1; to tolerance it reaches the LAPACK
    solution."""
    p, val = tiny_problem(nc, seed=seed)
    b = crandn(np.random.default_rng(seed), p.n)
    b[p.dirichlet] = 0
    A = sp.csr_matrix((val, p.col, p.rowptr), shape=(p.n, p.n))
    dinv = 1.0 / A.diagonal()
    Ah = (A @ sp.diags(dinv)).tocsr()
    for k in (1, 2, 3, 5):
        xo, info = oracle.tfqmr(p.rowptr, p.col, val, b, tol=1e-15, maxit=k)
        assert info["iters"] == k and info["status"] == oracle.NOT_CONVERGED
        ys, _ = spla.tfqmr(Ah, b, rtol=1e-15, atol=0.0, maxiter=2 * k)
        assert np.linalg.norm(dinv * ys - xo) <= 1e-11 * np.linalg.norm(xo), k
    # the quasi-residual bound bounds the true residual (in exact arithmetic:
    # checked at 1e-6, far above the rounding level of the recurrences)
    x, info = oracle.tfqmr(p.rowptr, p.col, val, b, tol=1e-6)
    assert info["status"] == 0 and info["relres_true"] <= info["relres_rec"] <= 1e-6
    x, info = oracle.tfqmr(p.rowptr, p.col, val, b, tol=1e-12)
    assert info["status"] == 0 and info["relres_true"] <= 2e-12
    xs = np.linalg.solve(dense(p, val), b)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_tfqmr_cube16_diagonal_breakdown_and_errors(oracle):
    c1 = configs.cube16()
    x, info = oracle.tfqmr(c1["rowptr"], c1["col"], c1["val"], c1["g"], tol=1e-8)
    assert info["status"] == 0 and info["relres_true"] <= 1e-8 <= 1e-8 + info["relres_rec"]
    xb, _ = oracle.bicgstab(c1["rowptr"], c1["col"], c1["val"], c1["g"], tol=1e-12)
    x10, i10 = oracle.tfqmr(c1["rowptr"], c1["col"], c1["val"], c1["g"], tol=1e-12)
    assert i10["status"] == 0 and np.linalg.norm(x10 - xb) <= 1e-8 * np.linalg.norm(xb)
    # D = A: the first half-step gives x = b / d exactly, tau = 0
    n = 20
    rng = np.random.default_rng(2)
    d = crandn(rng, n) + 3.0
    b = crandn(rng, n)
    x, info = oracle.tfqmr(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d, b, tol=1e-12)
    assert info["status"] == 0 and info["iters"] == 1
    assert np.allclose(x, b / d, rtol=1e-14, atol=0)
    # g^H A g = 0 at the first step (D = I): sigma breakdown before any iteration
    x, info = oracle.tfqmr(np.array([0, 2, 4], dtype=np.int32), np.array([0, 1, 0, 1], dtype=np.int32),
                           np.array([1.0, -1.25, -1.25, 1.0], dtype=np.complex128), np.array([1.0, 2.0]))
    assert info["status"] == oracle.BREAKDOWN and info["breakdown"] == oracle.BD_SIGMA
    assert info["iters"] == 0 and np.all(x == 0)
    g = c1["g"].copy()
    g[3] = np.nan
    assert oracle.tfqmr(c1["rowptr"], c1["col"], c1["val"], g)[1]["status"] == oracle.NONFINITE
    x, info = oracle.tfqmr(c1["rowptr"], c1["col"], c1["val"], c1["g"], maxit=1)
    assert info["status"] == oracle.NOT_CONVERGED and info["iters"] == 1 and np.any(x != 0)


# ----------------------------------------------------------- BiCGStab(l)

def _bicgstab_l_mgs(A, dinv, b, ell, cycles):
    """Sleijpen-Fokkema BiCGStab(l) with the minimal-residual step by modified
    Gram-Schmidt (their original form), right-preconditioned, dense numpy:
    an independent route to the same iterates as the oracle's
    normal-equations form."""
    Ah = A * dinv[None, :]
    r = [b.copy()] + [None] * ell
    u = [np.zeros_like(b)] + [None] * ell
    rt = b.copy()
    y = np.zeros_like(b)
    rho0, alpha, omega = 1.0 + 0j, 0j, 1.0 + 0j
    for _ in range(cycles):
        rho0 = -omega * rho0
        for j in range(ell):
            rho1 = np.vdot(rt, r[j])
            beta = alpha * rho1 / rho0
            rho0 = rho1
            for i in range(j + 1):
                u[i] = r[i] - beta * u[i]
            u[j + 1] = Ah @ u[j]
            alpha = rho0 / np.vdot(rt, u[j + 1])
            for i in range(j + 1):
                r[i] = r[i] - alpha * u[i + 1]
            r[j + 1] = Ah @ r[j]
            y = y + alpha * u[0]
        tau = np.zeros((ell + 1, ell + 1), dtype=complex)
        sigma = np.zeros(ell + 1)
        gp = np.zeros(ell + 1, dtype=complex)
        for j in range(1, ell + 1):
            for i in range(1, j):
                tau[i, j] = np.vdot(r[i], r[j]) / sigma[i]
                r[j] = r[j] - tau[i, j] * r[i]
            sigma[j] = np.vdot(r[j], r[j]).real
            gp[j] = np.vdot(r[j], r[0]) / sigma[j]
        g = np.zeros(ell + 1, dtype=complex)
        g[ell] = gp[ell]
        for j in range(ell - 1, 0, -1):
            g[j] = gp[j] - sum(tau[j, i] * g[i] for i in range(j + 1, ell + 1))
        g2 = np.zeros(ell + 1, dtype=complex)
        for j in range(1, ell):
            g2[j] = g[j + 1] + sum(tau[j, i] * g[i + 1] for i in range(j + 1, ell))
        omega = g[ell]
        y = y + g[1] * r[0]
        r[0] = r[0] - gp[ell] * r[ell]
        u[0] = u[0] - g[ell] * u[ell]
        for j in range(1, ell):
            u[0] = u[0] - g[j] * u[j]
            y = y + g2[j] * r[j]
            r[0] = r[0] - gp[j] * r[j]
    return dinv * y


@pytest.mark.parametrize("nc,seed", [(3, 3), (4, 5)])
def test_bicgstab_l_pins(oracle, nc, seed):
    """l = 1 reproduces BiCGStab's iterates; l = 2, 4 the iterates of the
    Gram-Schmidt form of the method; every l reaches the LAPACK solution."""
    p, val = tiny_problem(nc, seed=seed)
    b = crandn(np.random.default_rng(seed), p.n)
    b[p.dirichlet] = 0
    # (rounding differences grow with the steps on these indefinite systems:
    # 2e-14 after 4 iterations, 2e-10 after 6)
    for k in (1, 2, 3, 4):
        x1, i1 = oracle.bicgstab_l(p.rowptr, p.col, val, b, ell=1, tol=1e-15, maxit=k)
        xb, ib = oracle.bicgstab(p.rowptr, p.col, val, b, tol=1e-15, maxit=k)
        assert i1["iters"] == ib["iters"] == k
        assert np.linalg.norm(x1 - xb) <= 1e-12 * np.linalg.norm(xb), k
    Ad = dense(p, val)
    dinv = 1.0 / np.diag(Ad)
    for ell in (2, 4):
        for k in (1, 2):
            xo, io = oracle.bicgstab_l(p.rowptr, p.col, val, b, ell=ell, tol=1e-15, maxit=k)
            assert io["iters"] == k and io["status"] == oracle.NOT_CONVERGED
            xm = _bicgstab_l_mgs(Ad, dinv, b, ell, k)
            assert np.linalg.norm(xo - xm) <= 1e-9 * np.linalg.norm(xm), (ell, k)
    xs = np.linalg.solve(Ad, b)
    for ell in (2, 4, 8):
        # at 1e-12 the recursive residual runs ahead of the true one by the
        # rounding of the power basis r_j = (A D^-1)^j r_0 (1.2e-11 true
        # against 9.4e-13 recursive for l = 8 on the 4^3 system)
        x, info = oracle.bicgstab_l(p.rowptr, p.col, val, b, ell=ell, tol=1e-12)
        assert info["status"] == 0 and info["relres_true"] <= 5e-11, (ell, info)
        assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def _cyclic_shift_system(n, seed):
    """Dense complex n x n: diagonal 2 e^{i phi}, cyclic super-diagonal
    e^{i psi}, one small random entry per row (phases and values from
    default_rng(seed)).  After Jacobi scaling the operator is I plus a shift
    of modulus 1/2 (eigenvalues near a circle of radius 1/2 about 1), so the
    power basis of an 8-step cycle stays well conditioned and BiCGStab(8)
    converges in a few cycles."""
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n), dtype=complex)
    for i in range(n):
        A[i, i] = 2.0 * np.exp(1j * rng.uniform(0, 2 * np.pi))
        A[i, (i + 1) % n] = np.exp(1j * rng.uniform(0, 2 * np.pi))
        j = int(rng.integers(n))
        if j not in (i, (i + 1) % n):
            A[i, j] = 0.005 * complex(rng.standard_normal(), rng.standard_normal())
    rowptr = np.zeros(n + 1, dtype=np.int32)
    cols, vals = [], []
    for i in range(n):
        nz = np.flatnonzero(A[i])
        cols.extend(nz)
        vals.extend(A[i, nz])
        rowptr[i + 1] = len(cols)
    return A, rowptr, np.array(cols, dtype=np.int32), np.array(vals)


@pytest.mark.parametrize("n,seed", [(40, 1), (57, 2), (64, 3), (71, 4)])
def test_bicgstab_l8_pin(oracle, n, seed):
    """l = 8, the paper's P-BiCGSTAB(8): the oracle's iterates after one and
    two cycles (16 and 32 products) are those of the Gram-Schmidt form of the
    method to 1e-9.  The two forms of the minimal-residual step differ in
    rounding by about the square of the condition number of the cycle's
    Krylov basis times the unit roundoff; on these systems they agree to
    4e-11, while a wrong term would move the iterate by the size of the
    residual (3e-5 after one cycle, 5e-10 after two)."""
    A, rowptr, col, val = _cyclic_shift_system(n, seed)
    b = crandn(np.random.default_rng(seed + 10), n)
    dinv = 1.0 / np.diag(A)
    for k in (1, 2):
        xo, io = oracle.bicgstab_l(rowptr, col, val, b, ell=8, tol=1e-15, maxit=k)
        assert io["iters"] == k and io["status"] == oracle.NOT_CONVERGED, io
        xm = _bicgstab_l_mgs(A, dinv, b, 8, k)
        assert np.linalg.norm(xo - xm) <= 1e-9 * np.linalg.norm(xm), k
    x, info = oracle.bicgstab_l(rowptr, col, val, b, ell=8, tol=1e-12)
    assert info["status"] == 0 and info["iters"] <= 4, info
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-10 * np.linalg.norm(x)


def test_bicgstab_l_cube16_edges_and_errors(oracle):
    c1 = configs.cube16()
    x, info = oracle.bicgstab_l(c1["rowptr"], c1["col"], c1["val"], c1["g"], ell=8, tol=1e-8)
    assert info["status"] == 0 and info["relres_true"] <= 1e-8
    xb, _ = oracle.bicgstab(c1["rowptr"], c1["col"], c1["val"], c1["g"], tol=1e-12)
    x12, i12 = oracle.bicgstab_l(c1["rowptr"], c1["col"], c1["val"], c1["g"], ell=8, tol=1e-12)
    assert i12["status"] == 0 and np.linalg.norm(x12 - xb) <= 1e-8 * np.linalg.norm(xb)
    n = 20
    rng = np.random.default_rng(2)
    d = crandn(rng, n) + 3.0
    b = crandn(rng, n)
    rp, cl = np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32)
    for ell in (1, 8):
        # D = A: the first BiCG step solves the system exactly (exit inside the cycle)
        x, info = oracle.bicgstab_l(rp, cl, d, b, ell=ell, tol=1e-12)
        assert info["status"] == 0 and info["iters"] == 1
        assert np.allclose(x, b / d, rtol=1e-14, atol=0)
    x, info = oracle.bicgstab_l(np.array([0, 2, 4], dtype=np.int32), np.array([0, 1, 0, 1], dtype=np.int32),
                                np.array([1.0, -1.25, -1.25, 1.0], dtype=np.complex128), np.array([1.0, 2.0]),
                                ell=4)
    assert info["status"] == oracle.BREAKDOWN and info["breakdown"] == oracle.BD_SIGMA
    assert info["iters"] == 0 and np.all(x == 0)
    for bad in (0, 17):
        assert oracle.bicgstab_l(rp, cl, d, b, ell=bad)[1]["status"] == oracle.EINVAL
    g = c1["g"].copy()
    g[0] = np.nan
    assert oracle.bicgstab_l(c1["rowptr"], c1["col"], c1["val"], g)[1]["status"] == oracle.NONFINITE


@pytest.mark.parametrize("nc,seed", [(3, 3), (4, 5)])
def test_bicgstab_c64_matches_dense_lu_and_complex128_steps(oracle, nc, seed):
    """The complex-float solver (FP64-accumulated dots) reaches the LAPACK
    solution of the same rounded system, and its first two iterates equal
    the complex128 solver's on that matrix to float rounding."""
    p, val = tiny_problem(nc, seed=seed)
    v32 = val.astype(np.complex64)
    b = crandn(np.random.default_rng(seed), p.n)
    b[p.dirichlet] = 0
    b32 = b.astype(np.complex64)
    x, info = oracle.bicgstab_c64(p.rowptr, p.col, v32, b32, tol=1e-5)
    assert info["status"] == 0 and info["relres_rec"] <= 1e-5
    xs = np.linalg.solve(dense(p, v32.astype(np.complex128)), b32.astype(np.complex128))
    # cond(A) is 99 and 961 here; the measured errors are 9e-6 and 3e-5
    assert np.linalg.norm(x - xs) <= 1e-4 * np.linalg.norm(xs)
    for k in (1, 2):
        x1, i1 = oracle.bicgstab_c64(p.rowptr, p.col, v32, b32, tol=1e-12, maxit=k)
        x2, _ = oracle.bicgstab(p.rowptr, p.col, v32.astype(np.complex128), b32.astype(np.complex128),
                                tol=1e-12, maxit=k)
        assert i1["iters"] == k and i1["status"] == oracle.NOT_CONVERGED
        assert np.linalg.norm(x1 - x2) <= 1e-6 * np.linalg.norm(x2), k


def test_bicgstab_c64_diagonal_and_sigma_breakdown(oracle):
    n = 20
    rng = np.random.default_rng(2)
    d = (crandn(rng, n) + 3.0).astype(np.complex64)
    b = crandn(rng, n).astype(np.complex64)
    rowptr = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    x, info = oracle.bicgstab_c64(rowptr, col, d, b, tol=1e-6)
    assert info["status"] == 0 and info["iters"] == 1
    ref = b.astype(np.complex128) / d.astype(np.complex128)
    assert np.all(np.abs(x - ref) <= 1e-6 * np.abs(ref))
    # the same exactly representable sigma = 0 case as the complex128 test
    x, info = oracle.bicgstab_c64(np.array([0, 2, 4], dtype=np.int32), np.array([0, 1, 0, 1], dtype=np.int32),
                                  np.array([1.0, -1.25, -1.25, 1.0], dtype=np.complex64),
                                  np.array([1.0, 2.0], dtype=np.complex64), tol=1e-6)
    assert info["status"] == oracle.BREAKDOWN and info["breakdown"] == oracle.BD_SIGMA
    assert info["iters"] == 0 and np.all(x == 0)


def test_mixed_refinement_cube16(oracle):
    c1 = configs.cube16()
    u, info = oracle.mixed_refine(c1["rowptr"], c1["col"], c1["val"], c1["g"])
    assert info["status"] == 0 and info["relres_true"] <= 1e-10
    x, _ = oracle.bicgstab(c1["rowptr"], c1["col"], c1["val"], c1["g"], tol=1e-12)
    assert np.linalg.norm(u - x) <= 1e-8 * np.linalg.norm(x)


def test_mixed_refinement_diagonal_closed_form(oracle):
    """Iterative refinement with an inner solver exact to float rounding: on a
    diagonal system Jacobi BiCGStab converges in one iteration (d = r / diag
    rounded to complex64), so each cycle shrinks the FP64 residual by about
    2^-24: two cycles of one inner iteration each reach 1e-10, and the result
    is b / diag to double rounding.  A residual formed in complex64, an update
    that replaces u instead of adding to it, or an unscaled rounding of tiny
    residuals would stall near 1e-7 or lose the second cycle's gain."""
    n = 64
    rng = np.random.default_rng(12)
    d = crandn(rng, n) + 3.0
    b = crandn(rng, n)
    rowptr = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    u, info = oracle.mixed_refine(rowptr, col, d, b, inner_tol=1e-4, outer_tol=1e-10)
    assert info["status"] == 0 and info["iters"] == 2 and info["inner_iters"] == 2, info
    assert info["relres_true"] <= 1e-13, info
    assert np.linalg.norm(u - b / d) <= 1e-14 * np.linalg.norm(b / d)
    # one cycle alone stops at complex64 rounding of the solution
    u1, i1 = oracle.mixed_refine(rowptr, col, d, b, inner_tol=1e-4, outer_tol=1e-10, max_outer=1)
    assert i1["iters"] == 1 and i1["status"] == oracle.NOT_CONVERGED, i1
    assert 1e-9 < i1["relres_true"] < 2 ** -22, i1


def test_mixed_refinement_last_cycle_stops_near_the_tolerance(oracle):
    """A cycle's inner tolerance is max(inner_tol, outer_tol ||b|| / (2 ||r||)):
    the last cycle stops once it has halved the remaining distance to the
    outer tolerance, so the final residual lands within a small factor below
    it instead of orders of magnitude below (a cycle run to inner_tol = 1e-4
    from just above 1e-8 would end near 1e-12)."""
    c1 = configs.cube16()
    for outer in (1e-8, 1e-10):
        u, info = oracle.mixed_refine(c1["rowptr"], c1["col"], c1["val"], c1["g"], inner_tol=1e-4,
                                      outer_tol=outer)
        assert info["status"] == 0, info
        assert 0.02 * outer < info["relres_true"] <= outer, (outer, info)
        r = oracle.residual(c1["rowptr"], c1["col"], c1["val"], c1["g"], u)
        assert np.linalg.norm(r) / np.linalg.norm(c1["g"]) == pytest.approx(info["relres_true"], rel=1e-6)


# ------------------------------------------------------------- adjoint

def _block_problem(nc=4, bs=2, seed=1):
    m = H.make_mesh(nc, nc, nc, 1.0 / nc, jitter=0.2, rng=np.random.default_rng(seed))
    nb = (nc // bs) ** 3
    c = np.random.default_rng(seed + 10).uniform(300, 400, nb)
    (_, nby, nbz), blk = H.cell_blocks(m, bs)
    p = H.build_problem(m)
    tn, tb, tv, tp = H.tets_by_block(m, bs)
    omega = 2 * math.pi * c.min() / (10 * m.h)
    return m, p, c, tn, tb, omega, blk


def test_oracle_assembly_matches_generator(oracle):
    m, p, c, tn, tb, omega, blk = _block_problem(6, 3, 2)
    pw = H.build_problem(m, cell_weight=lambda I, J, K: 1.0 / c[blk(I, J, K)] ** 2)
    ref = H.helmholtz_values(pw, complex(omega ** 2, 0.01 * omega ** 2))
    val = oracle.assemble_helmholtz(p.rowptr, p.col, p.K, p.dirichlet, tn, tb, m.coords, c, omega)
    assert np.max(np.abs(val - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_adjoint_matches_torch_dense_autograd(oracle):
    torch = pytest.importorskip("torch")
    m, p, c, tn, tb, omega, blk = _block_problem(4, 2, 1)
    val = oracle.assemble_helmholtz(p.rowptr, p.col, p.K, p.dirichlet, tn, tb, m.coords, c, omega)
    g = crandn(np.random.default_rng(3), p.n)
    g[p.dirichlet] = 0
    S = np.flatnonzero(~p.dirichlet)[::5]
    L, gg, gc, u, _ = oracle.adjoint_gradients(p.rowptr, p.col, val, g, S, tn, tb, m.coords,
                                               p.dirichlet, c, omega, tol=1e-14)
    # torch: dense A(c) = K - omega^2 (1+0.01i) sum_b c_b^-2 M_b with M_b from one-hot speeds
    nb = c.shape[0]
    Mb = []
    for b in range(nb):
        cb = np.full(nb, np.inf)
        cb[b] = 1.0
        vb = oracle.assemble_helmholtz(p.rowptr, p.col, np.zeros_like(p.K), p.dirichlet, tn, tb,
                                       m.coords, cb, 1.0, damp=0.0)
        Mb.append(-dense(p, vb).real)
    Kd = torch.tensor(dense(p, p.K.astype(complex)).real)
    Mb = torch.tensor(np.stack(Mb))
    ct = torch.tensor(c, requires_grad=True)
    gt = torch.tensor(g, requires_grad=True)
    kap = omega ** 2 * (1 + 0.01j)
    A = Kd.to(torch.complex128) - kap * torch.einsum("b,bij->ij", ct ** -2, Mb).to(torch.complex128)
    ut = torch.linalg.solve(A, gt)
    Lt = (ut[torch.tensor(S)].abs() ** 2).sum()
    Lt.backward()
    assert abs(L - Lt.item()) <= 1e-10 * L
    assert np.linalg.norm(gg - gt.grad.numpy()) <= 1e-8 * np.linalg.norm(gg)
    assert np.linalg.norm(gc - ct.grad.numpy()) <= 1e-8 * np.linalg.norm(gc)


def test_adjoint_matches_central_differences(oracle):
    m, p, c, tn, tb, omega, blk = _block_problem(6, 3, 4)
    asm = lambda cc: oracle.assemble_helmholtz(p.rowptr, p.col, p.K, p.dirichlet, tn, tb, m.coords,
                                               cc, omega)
    val = asm(c)
    g = crandn(np.random.default_rng(8), p.n)
    g[p.dirichlet] = 0
    S = np.flatnonzero(~p.dirichlet)[::7]

    def loss(v, gg):
        u, info = oracle.bicgstab(p.rowptr, p.col, v, gg, tol=1e-14)
        return float(np.sum(np.abs(u[S]) ** 2))

    L, grad_g, grad_c, u, _ = oracle.adjoint_gradients(p.rowptr, p.col, val, g, S, tn, tb, m.coords,
                                                       p.dirichlet, c, omega, tol=1e-14)
    rng = np.random.default_rng(9)
    for b in rng.choice(c.shape[0], 3, replace=False):
        hstep = 1e-6 * c[b]
        cp, cm = c.copy(), c.copy()
        cp[b] += hstep
        cm[b] -= hstep
        fd = (loss(asm(cp), g) - loss(asm(cm), g)) / (2 * hstep)
        assert abs(fd - grad_c[b]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(grad_c).max())
    for _ in range(2):
        d = crandn(rng, p.n)
        d[p.dirichlet] = 0
        d /= np.linalg.norm(d)
        hstep = 1e-6 * np.linalg.norm(g)
        fd = (loss(val, g + hstep * d) - loss(val, g - hstep * d)) / (2 * hstep)
        # dL = Re(conj(grad_g) . dg) for the dL/dRe + i dL/dIm convention
        assert abs(fd - np.real(np.vdot(grad_g, d))) <= 1e-6 * np.linalg.norm(grad_g)
