"""Python wrapper of the plain CPU oracle (hk_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library.  It shares no code with
the HIP path.  Functions take and return numpy arrays; complex vectors are
complex128 (complex64 for the inner solve of the refinement).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hk_oracle.c")
LIB = os.path.join(HERE, "libhk_oracle.so")

OK, NOT_CONVERGED, BREAKDOWN, NONFINITE, EINVAL = 0, 1, 2, 3, -1
BD_NONE, BD_RHO, BD_SIGMA, BD_TAU, BD_OMEGA = 0, 1, 2, 3, 4


class Info(C.Structure):
    _fields_ = [("iters", C.c_int64), ("relres_rec", C.c_double), ("relres_true", C.c_double),
                ("status", C.c_int32), ("breakdown", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def build(force=True):
    """Compile the oracle with gcc (plain C99, OpenMP over independent rows)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-fopenmp", "-fcx-fortran-rules",
           "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_sanitized(path):
    """Compile the same source with AddressSanitizer and UndefinedBehaviorSanitizer
    (host code; any report aborts) into path, for a run of the oracle's checks
    with HK_ORACLE_LIB=path and the sanitizer runtimes preloaded."""
    cmd = ["gcc", "-O1", "-g", "-std=gnu99", "-fPIC", "-shared", "-fopenmp", "-fcx-fortran-rules",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           "-o", path, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return path


_lib = None


def lib():
    global _lib
    if _lib is None:
        # HK_ORACLE_LIB names another build of the same source (the sanitized
        # build of the oracle's own checks); by default the library is built here
        path = os.environ.get("HK_ORACLE_LIB")
        if not path:
            build(force=False)
            path = LIB
        L = C.CDLL(path)
        P = C.c_void_p
        i64, dbl, i32 = C.c_int64, C.c_double, C.c_int
        L.orc_spmv.argtypes = [i64, P, P, P, P, P]
        L.orc_residual.argtypes = [i64, P, P, P, P, P, P]
        for f in ("orc_zdotc", "orc_zdotu"):
            getattr(L, f).argtypes = [i64, P, P, P]
        L.orc_dznrm2.argtypes = [i64, P]
        L.orc_dznrm2.restype = dbl
        L.orc_zaxpy.argtypes = [i64, P, P, P]
        L.orc_zscal.argtypes = [i64, P, P]
        L.orc_zaxmy.argtypes = [i64, P, P]
        L.orc_zcopy.argtypes = [i64, P, P]
        L.orc_bicgstab.argtypes = [i64, P, P, P, P, P, dbl, i64, i32, C.POINTER(Info), P]
        L.orc_tfqmr.argtypes = [i64, P, P, P, P, P, dbl, i64, i32, C.POINTER(Info), P]
        L.orc_bicgstab_l.argtypes = [i64, P, P, P, P, P, dbl, i64, i32, i32, C.POINTER(Info), P]
        L.orc_bicgstab_c64.argtypes = [i64, P, P, P, P, P, C.c_float, i64, C.POINTER(Info)]
        L.orc_mixed_refine.argtypes = [i64, P, P, P, P, P, dbl, dbl, i32, i64, C.POINTER(Info),
                                       C.POINTER(C.c_int64)]
        L.orc_assemble_helmholtz.argtypes = [i64, P, P, P, P, i64, P, P, P, P, dbl, dbl, P]
        L.orc_assemble_helmholtz.restype = i32
        L.orc_elem_sens.argtypes = [i64, P, P, P, P, P, P, P, i64, dbl, dbl, P]
        L.orc_set_threads.argtypes = [i32]
        L.orc_max_threads.restype = i32
        _lib = L
    return _lib


def set_threads(t):
    """Thread count of the oracle's OpenMP loops (results do not depend on it)."""
    lib().orc_set_threads(int(t))


def max_threads():
    return int(lib().orc_max_threads())


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _csr(rowptr, col, val, dtype=np.complex128):
    return (np.ascontiguousarray(rowptr, dtype=np.int32), np.ascontiguousarray(col, dtype=np.int32),
            np.ascontiguousarray(val, dtype=dtype))


def spmv(rowptr, col, val, x):
    rowptr, col, val = _csr(rowptr, col, val)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    n = rowptr.shape[0] - 1
    y = np.empty(n, dtype=np.complex128)
    lib().orc_spmv(n, _p(rowptr), _p(col), _p(val), _p(x), _p(y))
    return y


def residual(rowptr, col, val, b, x):
    rowptr, col, val = _csr(rowptr, col, val)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    r = np.empty_like(b)
    lib().orc_residual(b.shape[0], _p(rowptr), _p(col), _p(val), _p(b), _p(x), _p(r))
    return r


def zdotc(x, y):
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.ascontiguousarray(y, dtype=np.complex128)
    out = np.zeros(1, dtype=np.complex128)
    lib().orc_zdotc(x.shape[0], _p(x), _p(y), _p(out))
    return complex(out[0])


def zdotu(x, y):
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.ascontiguousarray(y, dtype=np.complex128)
    out = np.zeros(1, dtype=np.complex128)
    lib().orc_zdotu(x.shape[0], _p(x), _p(y), _p(out))
    return complex(out[0])


def dznrm2(x):
    x = np.ascontiguousarray(x, dtype=np.complex128)
    return float(lib().orc_dznrm2(x.shape[0], _p(x)))


def zaxpy(alpha, x, y):
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.array(y, dtype=np.complex128, copy=True)
    a = np.array([alpha], dtype=np.complex128)
    lib().orc_zaxpy(x.shape[0], _p(a), _p(x), _p(y))
    return y


def zscal(alpha, x):
    x = np.array(x, dtype=np.complex128, copy=True)
    a = np.array([alpha], dtype=np.complex128)
    lib().orc_zscal(x.shape[0], _p(a), _p(x))
    return x


def zaxmy(x, y):
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.array(y, dtype=np.complex128, copy=True)
    lib().orc_zaxmy(x.shape[0], _p(x), _p(y))
    return y


def bicgstab(rowptr, col, val, b, x0=None, tol=1e-8, maxit=400000, precond=True, history=False):
    """Jacobi right-preconditioned BiCGStab; returns (x, info dict[, history])."""
    rowptr, col, val = _csr(rowptr, col, val)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    n = b.shape[0]
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    info = Info()
    hist = np.zeros(maxit + 1) if history else None
    lib().orc_bicgstab(n, _p(rowptr), _p(col), _p(val), _p(b), _p(x), float(tol), int(maxit),
                       1 if precond else 0, C.byref(info), _p(hist) if history else None)
    d = info.as_dict()
    if history:
        return x, d, hist[: d["iters"] + 1]
    return x, d


def tfqmr(rowptr, col, val, b, x0=None, tol=1e-8, maxit=400000, precond=True, history=False):
    """Jacobi right-preconditioned TFQMR; returns (x, info dict[, history]).
    iters counts pairs of half-steps; relres_rec is the quasi-residual bound."""
    rowptr, col, val = _csr(rowptr, col, val)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    n = b.shape[0]
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    info = Info()
    hist = np.zeros(maxit + 1) if history else None
    lib().orc_tfqmr(n, _p(rowptr), _p(col), _p(val), _p(b), _p(x), float(tol), int(maxit),
                    1 if precond else 0, C.byref(info), _p(hist) if history else None)
    d = info.as_dict()
    if history:
        return x, d, hist[: d["iters"] + 1]
    return x, d


def bicgstab_l(rowptr, col, val, b, ell=8, x0=None, tol=1e-8, maxit=400000, precond=True, history=False):
    """Jacobi right-preconditioned BiCGStab(l); iters counts cycles of l BiCG steps."""
    rowptr, col, val = _csr(rowptr, col, val)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    n = b.shape[0]
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    info = Info()
    hist = np.zeros(maxit + 1) if history else None
    lib().orc_bicgstab_l(n, _p(rowptr), _p(col), _p(val), _p(b), _p(x), float(tol), int(maxit), int(ell),
                         1 if precond else 0, C.byref(info), _p(hist) if history else None)
    d = info.as_dict()
    if history:
        return x, d, hist[: d["iters"] + 1]
    return x, d


def bicgstab_c64(rowptr, col, val32, b32, tol=1e-4, maxit=400000):
    rowptr, col, val32 = _csr(rowptr, col, val32, np.complex64)
    b32 = np.ascontiguousarray(b32, dtype=np.complex64)
    x = np.zeros_like(b32)
    info = Info()
    lib().orc_bicgstab_c64(b32.shape[0], _p(rowptr), _p(col), _p(val32), _p(b32), _p(x),
                           float(tol), int(maxit), C.byref(info))
    return x, info.as_dict()


def mixed_refine(rowptr, col, val, b, inner_tol=1e-4, outer_tol=1e-10, max_outer=50,
                 max_inner=400000, u0=None):
    rowptr, col, val = _csr(rowptr, col, val)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    u = np.zeros_like(b) if u0 is None else np.array(u0, dtype=np.complex128)
    info = Info()
    tot = C.c_int64(0)
    lib().orc_mixed_refine(b.shape[0], _p(rowptr), _p(col), _p(val), _p(b), _p(u),
                           float(inner_tol), float(outer_tol), int(max_outer), int(max_inner),
                           C.byref(info), C.byref(tot))
    d = info.as_dict()
    d["inner_iters"] = tot.value
    return u, d


def assemble_helmholtz(rowptr, col, K, dirichlet, tet_nodes, tet_block, coords, c, omega,
                       damp=0.01):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    K = np.ascontiguousarray(K, dtype=np.float64)
    dirm = np.ascontiguousarray(dirichlet, dtype=np.uint8)
    tn = np.ascontiguousarray(tet_nodes, dtype=np.int32)
    tb = np.ascontiguousarray(tet_block, dtype=np.int32)
    X = np.ascontiguousarray(coords, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    val = np.empty(col.shape[0], dtype=np.complex128)
    rc = lib().orc_assemble_helmholtz(rowptr.shape[0] - 1, _p(rowptr), _p(col), _p(K), _p(dirm),
                                      tn.shape[0], _p(tn), _p(tb), _p(X), _p(c), float(omega),
                                      float(damp), _p(val))
    if rc != 0:
        raise ValueError("element entry outside the CSR pattern")
    return val


def elem_sens(tet_nodes, tet_block, coords, dirichlet, lam, u, c, omega, damp=0.01):
    tn = np.ascontiguousarray(tet_nodes, dtype=np.int32)
    tb = np.ascontiguousarray(tet_block, dtype=np.int32)
    X = np.ascontiguousarray(coords, dtype=np.float64)
    dirm = np.ascontiguousarray(dirichlet, dtype=np.uint8)
    lam = np.ascontiguousarray(lam, dtype=np.complex128)
    u = np.ascontiguousarray(u, dtype=np.complex128)
    c = np.ascontiguousarray(c, dtype=np.float64)
    out = np.zeros(c.shape[0])
    lib().orc_elem_sens(tn.shape[0], _p(tn), _p(tb), _p(X), _p(dirm), _p(lam), _p(u), _p(c),
                        c.shape[0], float(omega), float(damp), _p(out))
    return out


def adjoint_gradients(rowptr, col, val, g, samples, tet_nodes, tet_block, coords, dirichlet, c,
                      omega, damp=0.01, tol=1e-12, maxit=400000):
    """Loss L = sum_{i in S} |u_i|^2 with u = A^-1 g.  Returns (L, grad_g, grad_c, u, infos).

    grad_g follows the complex-gradient convention dL/dRe + i dL/dIm:
    with gu = 2 u on S (0 elsewhere), A lambda = conj(gu), grad_g = conj(lambda).
    """
    u, i1 = bicgstab(rowptr, col, val, g, tol=tol, maxit=maxit)
    gu = np.zeros_like(u)
    gu[samples] = 2.0 * u[samples]
    lam, i2 = bicgstab(rowptr, col, val, np.conj(gu), tol=tol, maxit=maxit)
    grad_g = np.conj(lam)
    grad_c = elem_sens(tet_nodes, tet_block, coords, dirichlet, lam, u, c, omega, damp)
    L = float(np.sum(np.abs(u[samples]) ** 2))
    return L, grad_g, grad_c, u, (i1, i2)
