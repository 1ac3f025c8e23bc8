"""Q1 (trilinear hexahedral) finite-element Helmholtz systems (input generation).

The paper's car-cavity matrices have up to 27-39 entries per row, mean 9.5-24
(Table 1), the row length of trilinear hexahedra: each node couples to the
27 nodes of the 3x3x3 block around it.  This module builds such stand-ins on
the same structured box meshes as the tetrahedral generator (``make_mesh``,
node id ``(i*(ny+1)+j)*(nz+1)+k``, optional jitter):

* one trilinear element per cube, local node l = 4a + 2b + c at offset
  (a, b, c) in {0, 1}^3, shape functions on the reference cube [-1, 1]^3;
* ``K_e = sum_q det(J) grad N grad N^T`` and ``M_e = sum_q det(J) N N^T`` by
  2x2x2 Gauss quadrature (exact for the mass of a parallelepiped; the
  jittered elements are general trilinear maps);
* 27 neighbour slots per node in ascending linear offset, so a CSR row built
  slot by slot is column-sorted;
* Dirichlet u = 0 on the z = 0 face by the same symmetric elimination as the
  tetrahedral generator.

Assembly adds the (a,b) and (b,a) contributions of an element in the same
statement, so K and M are exactly symmetric.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .helmholtz import FEProblem, Mesh

OFFSETS27 = np.array(list(itertools.product((-1, 0, 1), repeat=3)), dtype=np.int64)
SELF27 = 13
_SLOT27 = {tuple(int(v) for v in o): s for s, o in enumerate(OFFSETS27)}
# local node l = 4a + 2b + c at offset (a, b, c)
_LOCAL = np.array(list(itertools.product((0, 1), repeat=3)), dtype=np.int64)
_GAUSS = (-1.0 / math.sqrt(3.0), 1.0 / math.sqrt(3.0))


def _reference_shapes():
    """Shape values (8 points, 8 nodes) and reference gradients (8, 8, 3) at
    the 2x2x2 Gauss points (unit weights)."""
    s = 2 * _LOCAL - 1  # node sign per axis
    pts = np.array(list(itertools.product(_GAUSS, repeat=3)))
    N = np.empty((8, 8))
    dN = np.empty((8, 8, 3))
    for q, (x, y, z) in enumerate(pts):
        fx, fy, fz = (1 + s[:, 0] * x) / 2, (1 + s[:, 1] * y) / 2, (1 + s[:, 2] * z) / 2
        N[q] = fx * fy * fz
        dN[q, :, 0] = s[:, 0] / 2 * fy * fz
        dN[q, :, 1] = fx * s[:, 1] / 2 * fz
        dN[q, :, 2] = fx * fy * s[:, 2] / 2
    return N, dN


def element_matrices(X):
    """Stiffness and mass (E, 8, 8) of trilinear hexahedra with nodes X (E, 8, 3)."""
    N, dN = _reference_shapes()
    Ke = np.zeros((X.shape[0], 8, 8))
    Me = np.zeros((X.shape[0], 8, 8))
    for q in range(8):
        J = np.einsum("eli,lj->eij", X, dN[q])          # dx_i / dxi_j
        det = np.linalg.det(J)
        G = np.einsum("lj,eji->eli", dN[q], np.linalg.inv(J))  # physical gradients (E, 8, 3)
        Ke += det[:, None, None] * np.einsum("eai,ebi->eab", G, G)
        Me += det[:, None, None] * np.outer(N[q], N[q])[None]
    return Ke, Me


def assemble_hex(m: Mesh, slab=8):
    """Assemble K and M into per-node slot arrays of shape (n, 27)."""
    n = m.n
    VK = np.zeros(n * 27)
    VM = np.zeros(n * 27)
    vlin = (_LOCAL[:, 0] * (m.ny + 1) + _LOCAL[:, 1]) * (m.nz + 1) + _LOCAL[:, 2]
    for x0 in range(0, m.nx, slab):
        x1 = min(m.nx, x0 + slab)
        I, J, K = np.meshgrid(np.arange(x0, x1), np.arange(m.ny), np.arange(m.nz), indexing="ij")
        corner = m.node_id(I.ravel(), J.ravel(), K.ravel())
        nodes = corner[:, None] + vlin[None, :]
        Ke, Me = element_matrices(m.coords[nodes])
        for a in range(8):
            for b in range(a, 8):
                sab = _SLOT27[tuple(int(v) for v in (_LOCAL[b] - _LOCAL[a]))]
                ia = nodes[:, a] * 27 + sab
                VK[ia] += Ke[:, a, b]
                VM[ia] += Me[:, a, b]
                if a != b:
                    sba = _SLOT27[tuple(int(v) for v in (_LOCAL[a] - _LOCAL[b]))]
                    ib = nodes[:, b] * 27 + sba
                    VK[ib] += Ke[:, a, b]
                    VM[ib] += Me[:, a, b]
    return VK.reshape(n, 27), VM.reshape(n, 27)


def build_hex_problem(m: Mesh) -> FEProblem:
    """CSR K and M of the Q1 discretisation after Dirichlet elimination on z = 0."""
    VK, VM = assemble_hex(m)
    dirm = m.dirichlet()
    i, j, k = m.ijk()
    ok = np.ones((m.n, 27), dtype=bool)
    for s, (di, dj, dk) in enumerate(OFFSETS27):
        ok[:, s] = ((i + di >= 0) & (i + di <= m.nx) & (j + dj >= 0) & (j + dj <= m.ny)
                    & (k + dk >= 0) & (k + dk <= m.nz))
    lin = (OFFSETS27[:, 0] * (m.ny + 1) + OFFSETS27[:, 1]) * (m.nz + 1) + OFFSETS27[:, 2]
    nbr = np.arange(m.n, dtype=np.int64)[:, None] + lin[None, :]
    nbr_dir = np.zeros_like(ok)
    nbr_dir[ok] = dirm[nbr[ok]]
    keep = ok & ~dirm[:, None] & ~nbr_dir
    keep[dirm, :] = False
    keep[:, SELF27] = True
    VK[dirm, :] = 0.0
    VM[dirm, :] = 0.0
    VK[dirm, SELF27] = 1.0
    rowptr = np.zeros(m.n + 1, dtype=np.int64)
    np.cumsum(keep.sum(axis=1), out=rowptr[1:])
    slots = np.broadcast_to(np.arange(27, dtype=np.int8)[None, :], keep.shape)[keep]
    return FEProblem(m, rowptr.astype(np.int32), nbr[keep].astype(np.int32), VK[keep].copy(),
                     VM[keep].copy(), dirm, slots.copy())
