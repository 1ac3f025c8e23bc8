"""ctypes binding of libhk (argument marshalling only).

Every computation runs in the HIP library; this module passes device
pointers of torch tensors, the current HIP stream and host scalars, and turns
status codes into exceptions.  torch supplies device memory and streams.
The library must be built (``__graft_entry__.build()``); there is no
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhk.so")

HK_OK, HK_EINVAL, HK_EHIP, HK_ENOMEM = 0, -1, -2, -3
HK_NOT_CONVERGED, HK_BREAKDOWN, HK_NONFINITE = 1, 2, 3
HK_C128, HK_C64 = 0, 1
HK_VALIDATE, HK_AUTOTUNE, HK_INT32_COLS = 1, 2, 4
BD_NAMES = {0: "none", 1: "rho", 2: "sigma", 3: "tau", 4: "omega"}


class HKError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libhk error {code}: {msg}")
        self.code = code


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int64), ("precond", C.c_int32),
                ("check_every", C.c_int32), ("use_x0", C.c_int32), ("method", C.c_int32),
                ("d_history", C.c_void_p), ("ell", C.c_int32), ("flags", C.c_int32),
                ("shape", C.c_int32 * 4)]


HK_MIXED_LITERAL_INNER = 1


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int64), ("relres_rec", C.c_double), ("relres_true", C.c_double),
                ("status", C.c_int32), ("breakdown", C.c_int32), ("inner_iters", C.c_int64),
                ("shape", C.c_int32 * 4), ("shape_tuned", C.c_int32), ("pad", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}
        d["shape"] = list(self.shape)
        d["shape_tuned"] = bool(self.shape_tuned)
        return d


# Exported entry points and their ctypes signatures (restype int unless noted).
P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int32, C.c_double
SIGNATURES = {
    "hk_last_error": ([], C.c_char_p),
    "hk_csr_create": ([C.POINTER(P), I64, I64, P, P, P, C.c_int, C.c_int, P], C.c_int),
    "hk_csr_destroy": ([P], C.c_int),
    "hk_csr_plan": ([P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32), C.POINTER(I32)], C.c_int),
    "hk_csr_set_plan": ([P, I32, I32, I32], C.c_int),
    "hk_csr_info": ([P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I32), C.POINTER(I32)], C.c_int),
    "hk_csr_set_solver_plan": ([P, I32, I32, I32, I32], C.c_int),
    "hk_spmv": ([P, P, P, P, P, P], C.c_int),
    "hk_residual": ([P, P, P, P, P], C.c_int),
    "hk_zdotc": ([I64, P, P, P, P], C.c_int),
    "hk_zdotc_noalloc": ([I64, P, P, P, P], C.c_int),
    "hk_zdotu": ([I64, P, P, P, P], C.c_int),
    "hk_dznrm2": ([I64, P, P, P], C.c_int),
    "hk_zaxpy": ([I64, P, P, P, P], C.c_int),
    "hk_zscal": ([I64, P, P, P], C.c_int),
    "hk_zaxmy": ([I64, P, P, P], C.c_int),
    "hk_zcopy": ([I64, P, P, P], C.c_int),
    "hk_zconj": ([I64, P, P, P], C.c_int),
    "hk_krylov_solve": ([P, P, P, C.POINTER(SolveOpts), C.POINTER(SolveInfo), P], C.c_int),
    "hk_krylov_solve_mixed": ([P, P, P, D, D, I32, C.POINTER(SolveOpts), C.POINTER(SolveInfo), P],
                              C.c_int),
    "hk_sweep_solve": ([I64, I64, P, P, P, P, I32, P, P, P, C.POINTER(SolveOpts), P, P], C.c_int),
    "hk_blockdiag_solve": ([P, I32, P, P, P, C.POINTER(SolveOpts), P, P], C.c_int),
    "hk_assemble_helmholtz": ([I64, P, P, P, P, I64, I32, P, D, D, P, P], C.c_int),
    "hk_elem_sens": ([I64, I64, I32, P, P, P, P, P, P, P, D, D, P, P], C.c_int),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libhk.so and declare its signatures; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise HKError(HK_EINVAL, f"{path} is not built; run __graft_entry__.build()")
    lib = C.CDLL(path)
    for name, (args, res) in SIGNATURES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc, allow_positive=False):
    if rc == HK_OK or (allow_positive and rc > 0):
        return rc
    raise HKError(rc, load().hk_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _cvec(t, dtype=torch.complex128, name="vector", n=None):
    """Checks that t is a contiguous device tensor of dtype (and, given n, of
    n elements): the library takes raw pointers and cannot check lengths."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise HKError(HK_EINVAL, f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise HKError(HK_EINVAL, f"{name} must be a contiguous {dtype} tensor")
    if n is not None and t.numel() != n:
        raise HKError(HK_EINVAL, f"{name} has {t.numel()} elements, expected {n}")
    return t


def _scalar(z, dtype=torch.complex128):
    z = complex(z)
    if dtype == torch.complex64:
        return (C.c_float * 2)(z.real, z.imag)
    return (C.c_double * 2)(z.real, z.imag)


class CSR:
    """Handle on a CSR matrix in device memory (rowptr/col int32, val complex)."""

    def __init__(self, rowptr, col, val, autotune=False, compact_cols=True):
        lib = load()
        self.rowptr = rowptr.contiguous()
        self.col = col.contiguous()
        self.val = val.contiguous()
        if self.rowptr.dtype != torch.int32 or self.col.dtype != torch.int32:
            raise HKError(HK_EINVAL, "rowptr and col must be int32")
        if self.val.dtype not in (torch.complex128, torch.complex64):
            raise HKError(HK_EINVAL, "val must be complex128 or complex64")
        for t in (self.rowptr, self.col, self.val):
            if not t.is_cuda:
                raise HKError(HK_EINVAL, "CSR arrays must be device tensors")
        if self.rowptr.numel() < 1 or self.val.numel() != self.col.numel():
            raise HKError(HK_EINVAL, "rowptr needs n + 1 entries and val as many as col")
        self.n = self.rowptr.numel() - 1
        self.nnz = self.col.numel()
        self.dtype = self.val.dtype
        h = C.c_void_p()
        flags = HK_VALIDATE | (HK_AUTOTUNE if autotune else 0) | (0 if compact_cols else HK_INT32_COLS)
        dt = HK_C128 if self.dtype == torch.complex128 else HK_C64
        _check(lib.hk_csr_create(C.byref(h), self.n, self.nnz, _ptr(self.rowptr), _ptr(self.col),
                                 _ptr(self.val), dt, flags, _stream()))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().hk_csr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        n, nnz, mr, cb = C.c_int64(), C.c_int64(), I32(), I32()
        _check(load().hk_csr_info(self.h, C.byref(n), C.byref(nnz), C.byref(mr), C.byref(cb)))
        return {"n": n.value, "nnz": nnz.value, "max_row": mr.value, "col_bytes": cb.value}

    def plan(self):
        L, U, g, t = I32(), I32(), I32(), I32()
        _check(load().hk_csr_plan(self.h, C.byref(L), C.byref(U), C.byref(g), C.byref(t)))
        return {"lanes_per_row": L.value, "rows_per_group": U.value, "grid": g.value,
                "tuned": bool(t.value)}

    def set_plan(self, lanes_per_row, rows_per_group, grid=0):
        _check(load().hk_csr_set_plan(self.h, lanes_per_row, rows_per_group, grid))

    def set_solver_plan(self, rows_per_wave, waves, grid=0, paired=False):
        _check(load().hk_csr_set_solver_plan(self.h, int(rows_per_wave), int(waves), int(grid), int(bool(paired))))

    def spmv(self, x, y=None, alpha=1.0, beta=0.0):
        """y = alpha A x + beta y (y allocated when None)."""
        _cvec(x, self.dtype, "x", self.n)
        if y is None:
            y = torch.empty_like(x)
            beta = 0.0
        _cvec(y, self.dtype, "y", self.n)
        _check(load().hk_spmv(self.h, _scalar(alpha, self.dtype), _ptr(x), _scalar(beta, self.dtype),
                              _ptr(y), _stream()))
        return y

    def residual(self, b, x, r=None):
        """r = b - A x."""
        _cvec(b, self.dtype, "b", self.n)
        _cvec(x, self.dtype, "x", self.n)
        r = torch.empty_like(b) if r is None else _cvec(r, self.dtype, "r", self.n)
        _check(load().hk_residual(self.h, _ptr(b), _ptr(x), _ptr(r), _stream()))
        return r


def zdotc(x, y, out=None):
    _cvec(x, name="x"), _cvec(y, name="y", n=x.numel())
    out = torch.empty(1, dtype=torch.complex128, device=x.device) if out is None else _cvec(out, name="out", n=1)
    _check(load().hk_zdotc(x.numel(), _ptr(x), _ptr(y), _ptr(out), _stream()))
    return out


def zdotc_noalloc(x, y, out):
    """x^H y into out (one complex128 on the device) without any allocation:
    partials in the library's static per-GPU scratch (calls on one GPU must
    not overlap)."""
    _cvec(x, name="x"), _cvec(y, name="y", n=x.numel()), _cvec(out, name="out", n=1)
    _check(load().hk_zdotc_noalloc(x.numel(), _ptr(x), _ptr(y), _ptr(out), _stream()))
    return out


def zdotu(x, y, out=None):
    _cvec(x, name="x"), _cvec(y, name="y", n=x.numel())
    out = torch.empty(1, dtype=torch.complex128, device=x.device) if out is None else _cvec(out, name="out", n=1)
    _check(load().hk_zdotu(x.numel(), _ptr(x), _ptr(y), _ptr(out), _stream()))
    return out


def dznrm2(x, out=None):
    _cvec(x, name="x")
    out = (torch.empty(1, dtype=torch.float64, device=x.device) if out is None
           else _cvec(out, torch.float64, name="out", n=1))
    _check(load().hk_dznrm2(x.numel(), _ptr(x), _ptr(out), _stream()))
    return out


def zaxpy(alpha, x, y):
    """y = alpha x + y (in place)."""
    _cvec(x, name="x"), _cvec(y, name="y", n=x.numel())
    _check(load().hk_zaxpy(x.numel(), _scalar(alpha), _ptr(x), _ptr(y), _stream()))
    return y


def zscal(alpha, x):
    """x = alpha x (in place)."""
    _cvec(x, name="x")
    _check(load().hk_zscal(x.numel(), _scalar(alpha), _ptr(x), _stream()))
    return x


def zaxmy(x, y):
    """y = x .* y (in place)."""
    _cvec(x, name="x"), _cvec(y, name="y", n=x.numel())
    _check(load().hk_zaxmy(x.numel(), _ptr(x), _ptr(y), _stream()))
    return y


def zcopy(x, y):
    _cvec(x, name="x"), _cvec(y, name="y", n=x.numel())
    _check(load().hk_zcopy(x.numel(), _ptr(x), _ptr(y), _stream()))
    return y


def zconj(x, y=None):
    _cvec(x, name="x")
    y = torch.empty_like(x) if y is None else _cvec(y, name="y", n=x.numel())
    _check(load().hk_zconj(x.numel(), _ptr(x), _ptr(y), _stream()))
    return y


METHODS = {"bicgstab": 0, "tfqmr": 1, "bicgstab_l": 2}


def _opts(tol, max_iter, precond, check_every, use_x0, history, method="bicgstab", ell=8, flags=0,
          shape=None):
    if method not in METHODS:
        raise HKError(HK_EINVAL, f"unknown method {method!r}; one of {sorted(METHODS)}")
    o = SolveOpts()
    o.flags = int(flags)
    if shape is not None:
        if len(shape) != 4:
            raise HKError(HK_EINVAL, "shape has 4 entries")
        for k, v in enumerate(shape):
            o.shape[k] = int(v)
    o.method = METHODS[method]
    o.ell = int(ell)
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.precond = 1 if precond else 0
    o.check_every = int(check_every)
    o.use_x0 = 1 if use_x0 else 0
    o.d_history = history.data_ptr() if history is not None else None
    return o


def krylov_solve(A: CSR, b, x=None, tol=1e-8, max_iter=400000, precond=True, check_every=0,
                 history=False, method="bicgstab", ell=8):
    """Jacobi right-preconditioned BiCGStab, TFQMR or BiCGStab(ell) (the last two
    complex128) in A's precision; returns (x, info dict[, history]).  For
    BiCGStab(ell), iters counts cycles of ell BiCG steps."""
    _cvec(b, A.dtype, name="b", n=A.n)
    use_x0 = x is not None
    x = torch.zeros_like(b) if x is None else _cvec(x, A.dtype, name="x", n=A.n)
    hist = torch.zeros(int(max_iter) + 1, dtype=torch.float64, device=b.device) if history else None
    info = SolveInfo()
    o = _opts(tol, max_iter, precond, check_every, use_x0, hist, method, ell)
    _check(load().hk_krylov_solve(A.h, _ptr(b), _ptr(x), C.byref(o), C.byref(info), _stream()),
           allow_positive=True)
    d = info.as_dict()
    if history:
        return x, d, hist[: d["iters"] + 1]
    return x, d


def krylov_solve_mixed(A: CSR, b, x=None, inner_tol=1e-4, outer_tol=1e-10, max_outer=50,
                       max_inner=400000, check_every=0, literal_inner=False):
    """complex64-inner / complex128-outer refinement; returns (x, info dict).
    literal_inner: every cycle to inner_tol (no clamp of the last cycle)."""
    _cvec(b, name="b", n=A.n)
    use_x0 = x is not None
    x = torch.zeros_like(b) if x is None else _cvec(x, name="x", n=A.n)
    info = SolveInfo()
    o = _opts(0.0, max_inner, True, check_every, use_x0, None,
              flags=HK_MIXED_LITERAL_INNER if literal_inner else 0)
    _check(load().hk_krylov_solve_mixed(A.h, _ptr(b), _ptr(x), float(inner_tol), float(outer_tol),
                                        int(max_outer), C.byref(o), C.byref(info), _stream()),
           allow_positive=True)
    return x, info.as_dict()


SWEEP_LANES = 64
# launch shapes the batched solvers time (and accept as `shape`)
SWEEP_SHAPES = [(1, 1, 0, 0), (1, 2, 0, 0), (1, 3, 0, 0), (2, 3, 0, 0), (3, 1, 0, 0), (3, 2, 0, 0)]
BLOCKDIAG_SHAPES = ([(64, r, ch, tr) for tr in (1024, 512) for r in (64, 32, 16) for ch in (4, 2)]
                    + [(32, 0, 0, tr) for tr in (1024, 512)])


def sweep_solve(rowptr, col, K, M, kappa, B, tol=1e-8, max_iter=400000, shape=None, stamps=None):
    """Frequency sweep: solve (K - kappa_j M) X[:, j] = B[:, j] for j < len(kappa).

    rowptr/col int32, K/M float64 device tensors on one pattern; kappa a
    sequence of complex numbers (<= 64); B an (n, 64) complex128 device tensor
    (columns >= len(kappa) ignored).  shape: a launch shape (product form, row
    mapping, 0, 0) to use instead of the tuned one.  stamps: a float64 device tensor
    of 8 (max_iter + 1) entries that receives the barrier times (100 MHz
    clock ticks, see hk.h).  Returns (X, list of info dicts).
    """
    nsys = len(kappa)
    _cvec(rowptr, torch.int32, name="rowptr")
    _cvec(col, torch.int32, name="col")
    n = rowptr.numel() - 1
    if B.shape != (n, SWEEP_LANES):
        raise HKError(HK_EINVAL, "B must have shape (n, 64)")
    _cvec(B, name="B")
    for t, nm in ((K, "K"), (M, "M")):
        _cvec(t, torch.float64, name=nm, n=col.numel())
    X = torch.zeros_like(B)
    kap = (C.c_double * (2 * nsys))(*[v for z in kappa for v in (complex(z).real, complex(z).imag)])
    infos = (SolveInfo * nsys)()
    o = _opts(tol, max_iter, True, 0, False, None, shape=shape)
    if stamps is not None:
        o.d_history = _ptr(_cvec(stamps, torch.float64, name="stamps", n=8 * (int(max_iter) + 1)))
    _check(load().hk_sweep_solve(n, col.numel(), _ptr(rowptr), _ptr(col), _ptr(K), _ptr(M), nsys, kap,
                                 _ptr(B), _ptr(X), C.byref(o), infos, _stream()), allow_positive=True)
    return X, [i.as_dict() for i in infos]


def blockdiag_solve(A: CSR, row_off, b, tol=1e-8, max_iter=400000, shape=None, stamps=None):
    """Uneven batch: A block-diagonal with systems [row_off[k], row_off[k+1]).
    shape: a tile shape (lanes per row, rows per block, entries per lane,
    tile rows) to use instead of the tuned one.  stamps: a float64 device
    tensor of 8 (max_iter + 1) entries that receives the grid barriers' times
    (as for sweep_solve)."""
    _cvec(b, name="b", n=A.n)
    nsys = len(row_off) - 1
    offs = (C.c_int64 * (nsys + 1))(*[int(v) for v in row_off])
    x = torch.zeros_like(b)
    infos = (SolveInfo * max(nsys, 1))()
    o = _opts(tol, max_iter, True, 0, False, None, shape=shape)
    if stamps is not None:
        o.d_history = _ptr(_cvec(stamps, torch.float64, name="stamps", n=8 * (int(max_iter) + 1)))
    _check(load().hk_blockdiag_solve(A.h, nsys, offs, _ptr(b), _ptr(x), C.byref(o), infos, _stream()),
           allow_positive=True)
    return x, [infos[k].as_dict() for k in range(nsys)]
