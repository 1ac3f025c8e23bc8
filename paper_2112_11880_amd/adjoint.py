"""torch.autograd.Function for u = A(c)^-1 g with the hand-written adjoint.

A(c) = K - omega^2 (1 + i damp) sum_b c_b^-2 M_b is assembled by the library
(hk_assemble_helmholtz), the forward solve is the library's Jacobi
BiCGStab, and the backward pass solves A lambda = conj(grad_u) with the same
solver on the same matrix (A is complex symmetric), returns
grad_g = conj(lambda) and grad_c from hk_elem_sens.  grad_u and the returned
gradients follow torch's convention for complex tensors
(dL/dRe + i dL/dIm).  This module only marshals arguments.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import torch

from . import hk as _hk


def _declare():
    return _hk.load()


@dataclass
class HelmholtzProblem:
    """Device-resident description of the speed-dependent FE operator."""
    rowptr: torch.Tensor      # int32 (n+1)
    col: torch.Tensor         # int32 (nnz)
    K: torch.Tensor           # float64 (nnz), Dirichlet rows carry 1 on the diagonal
    bm_ptr: torch.Tensor      # int32 (nnz+1): per-entry lists of (block, mass)
    bm_blk: torch.Tensor      # int32
    bm_val: torch.Tensor      # float64
    tet_nodes: torch.Tensor   # int32 (T, 4), grouped by block
    tet_ptr: torch.Tensor     # int32 (nblocks+1)
    tet_vol: torch.Tensor     # float64 (T)
    dirichlet: torch.Tensor   # uint8 (n)
    omega: float
    damp: float = 0.01
    # the assembled operator: one value buffer and one CSR handle on it, made
    # on the first solve and reused (the pattern never changes), and the
    # forward solve whose speeds the buffer holds
    _val: torch.Tensor = field(default=None, repr=False, compare=False)
    _A: object = field(default=None, repr=False, compare=False)
    _owner: int = field(default=-1, repr=False, compare=False)
    # records of the last forward and adjoint solves (iterations, residuals)
    last_forward_info: dict = field(default=None, repr=False, compare=False)
    last_adjoint_info: dict = field(default=None, repr=False, compare=False)

    @property
    def n(self):
        return self.rowptr.numel() - 1

    @property
    def nblocks(self):
        return self.tet_ptr.numel() - 1


def _check_problem(prob: HelmholtzProblem, c: torch.Tensor):
    """Dtypes and lengths of the problem arrays and the speeds: the library
    takes raw pointers and cannot check them."""
    nnz, cv = prob.col.numel(), _hk._cvec
    cv(prob.rowptr, torch.int32, "rowptr"), cv(prob.col, torch.int32, "col")
    cv(prob.K, torch.float64, "K", nnz), cv(prob.bm_ptr, torch.int32, "bm_ptr", nnz + 1)
    cv(prob.bm_blk, torch.int32, "bm_blk"), cv(prob.bm_val, torch.float64, "bm_val", prob.bm_blk.numel())
    cv(prob.tet_ptr, torch.int32, "tet_ptr"), cv(prob.tet_vol, torch.float64, "tet_vol", prob.tet_nodes.shape[0])
    cv(prob.tet_nodes, torch.int32, "tet_nodes", 4 * prob.tet_nodes.shape[0])
    cv(prob.dirichlet, torch.uint8, "dirichlet", prob.n)
    cv(c, torch.float64, "c", prob.nblocks)


def assemble(prob: HelmholtzProblem, c: torch.Tensor, out=None):
    """Complex128 CSR values of A(c) (library kernel)."""
    lib = _declare()
    c = c.detach().contiguous()
    _check_problem(prob, c)
    val = (torch.empty(prob.col.numel(), dtype=torch.complex128, device=prob.col.device) if out is None
           else _hk._cvec(out, name="out", n=prob.col.numel()))
    _hk._check(lib.hk_assemble_helmholtz(prob.col.numel(), _hk._ptr(prob.K), _hk._ptr(prob.bm_ptr),
                                         _hk._ptr(prob.bm_blk), _hk._ptr(prob.bm_val),
                                         prob.bm_blk.numel(), prob.nblocks, _hk._ptr(c),
                                         float(prob.omega), float(prob.damp), _hk._ptr(val),
                                         _hk._stream()))
    return val


def elem_sens(prob: HelmholtzProblem, lam, u, c):
    """dL/dc_b from the adjoint state (library kernel)."""
    lib = _declare()
    c = c.detach().contiguous()
    _check_problem(prob, c)
    _hk._cvec(lam, name="lambda", n=prob.n), _hk._cvec(u, name="u", n=prob.n)
    out = torch.empty(prob.nblocks, dtype=torch.float64, device=c.device)
    _hk._check(lib.hk_elem_sens(prob.n, prob.tet_nodes.shape[0], prob.nblocks, _hk._ptr(prob.tet_nodes),
                                _hk._ptr(prob.tet_ptr), _hk._ptr(prob.tet_vol), _hk._ptr(prob.dirichlet),
                                _hk._ptr(lam), _hk._ptr(u), _hk._ptr(c), float(prob.omega),
                                float(prob.damp), _hk._ptr(out), _hk._stream()))
    return out


_tokens = itertools.count()


def _operator(prob: HelmholtzProblem, c: torch.Tensor, owner: int):
    """A(c) assembled into the problem's value buffer, and the CSR handle on
    it (created once per problem), marked as holding the speeds of `owner`."""
    if prob._val is None:
        prob._val = torch.empty(prob.col.numel(), dtype=torch.complex128, device=prob.col.device)
    assemble(prob, c, out=prob._val)
    if prob._A is None:
        prob._A = _hk.CSR(prob.rowptr, prob.col, prob._val)
    prob._owner = owner
    return prob._A


class HelmholtzSolve(torch.autograd.Function):
    """u = A(c)^-1 g (Jacobi BiCGStab) with the adjoint backward pass."""

    @staticmethod
    def forward(ctx, g, c, prob: HelmholtzProblem, tol: float, max_iter: int):
        ctx.token = next(_tokens)
        A = _operator(prob, c, ctx.token)
        u, info = _hk.krylov_solve(A, g.detach().contiguous(), tol=tol, max_iter=max_iter)
        prob.last_forward_info = info
        if info["status"] != _hk.HK_OK:
            raise _hk.HKError(info["status"], f"forward solve did not converge: {info}")
        ctx.prob, ctx.tol, ctx.max_iter = prob, tol, max_iter
        ctx.info_forward = info
        ctx.save_for_backward(c, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        c, u = ctx.saved_tensors
        prob = ctx.prob
        # another forward on the same problem may have reassembled the buffer
        A = prob._A if prob._owner == ctx.token else _operator(prob, c, ctx.token)
        rhs = _hk.zconj(grad_u.contiguous())
        lam, info = _hk.krylov_solve(A, rhs, tol=ctx.tol, max_iter=ctx.max_iter)
        prob.last_adjoint_info = info
        if info["status"] != _hk.HK_OK:
            raise _hk.HKError(info["status"], f"adjoint solve did not converge: {info}")
        grad_g = _hk.zconj(lam) if ctx.needs_input_grad[0] else None
        grad_c = elem_sens(ctx.prob, lam, u, c) if ctx.needs_input_grad[1] else None
        return grad_g, grad_c, None, None, None


def helmholtz_solve(g, c, prob: HelmholtzProblem, tol=1e-8, max_iter=400000):
    return HelmholtzSolve.apply(g, c, prob, tol, max_iter)
