"""P1 finite-element Helmholtz systems on a Kuhn-split box (input generation).

The paper's test matrices come from a finite-element discretisation of the
Helmholtz equation -lap(u) - k^2 u = g in a bounded domain, with a sound
speed that varies in space and Dirichlet conditions on part of the boundary
(Introduction), stored in CSR (Section 2).  Its car-cavity meshes are not
available, so this module builds stand-ins of the same kind:

* a box [0,Lx]x[0,Ly]x[0,Lz] cut into nx*ny*nz cubes of edge h, node id
  ``(i*(ny+1)+j)*(nz+1)+k`` (k fastest);
* each cube split into 6 tetrahedra along its (0,0,0)->(1,1,1) diagonal
  (Kuhn/Freudenthal split, conforming across cubes), so each node couples to
  itself and at most 14 neighbours (the 15 ``OFFSETS``);
* optional node jitter of +-20% h with the normal component zeroed on
  boundary nodes, so faces stay planar;
* element stiffness ``K_e = vol * G G^T`` (G = barycentric gradients) and
  mass ``M_e = vol/20 * (1 + delta_ab)``, optionally weighted by c_e^-2;
* Dirichlet u = 0 on the z = 0 face by symmetric elimination: the row and the
  column of a Dirichlet node are removed, its diagonal is 1 in K and 0 in M,
  and its right-hand side entry is 0.

Assembly adds the (a,b) and (b,a) contributions of an element in the same
statement, element by element, so the assembled K and M are exactly
symmetric, not just up to rounding.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Kuhn-split neighbour offsets (di, dj, dk), in ascending order of the linear
# node-id offset; a CSR row built slot by slot is therefore column-sorted.
OFFSETS = np.array([
    (-1, -1, -1), (-1, -1, 0), (-1, 0, -1), (-1, 0, 0), (0, -1, -1),
    (0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0),
    (0, 1, 1), (1, 0, 0), (1, 0, 1), (1, 1, 0), (1, 1, 1)], dtype=np.int64)
SELF_SLOT = 7
_SLOT = {tuple(int(v) for v in o): s for s, o in enumerate(OFFSETS)}

# The six axis orders; tet = (corner, +e_s0, +e_s0+e_s1, far corner).
PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def _tet_vertex_offsets(perm):
    e = np.eye(3, dtype=np.int64)
    v0 = np.zeros(3, dtype=np.int64)
    v1 = v0 + e[perm[0]]
    v2 = v1 + e[perm[1]]
    v3 = np.ones(3, dtype=np.int64)
    return np.stack([v0, v1, v2, v3])


@dataclasses.dataclass
class Mesh:
    nx: int
    ny: int
    nz: int
    h: float
    coords: np.ndarray          # (n, 3) float64

    @property
    def dims(self):
        return (self.nx + 1, self.ny + 1, self.nz + 1)

    @property
    def n(self) -> int:
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    def node_id(self, i, j, k):
        return (np.asarray(i) * (self.ny + 1) + np.asarray(j)) * (self.nz + 1) + np.asarray(k)

    def ijk(self):
        idx = np.arange(self.n, dtype=np.int64)
        k = idx % (self.nz + 1)
        j = (idx // (self.nz + 1)) % (self.ny + 1)
        i = idx // ((self.nz + 1) * (self.ny + 1))
        return i, j, k

    def dirichlet(self) -> np.ndarray:
        """Boolean mask of the Dirichlet nodes (the z = 0 face)."""
        return self.ijk()[2] == 0

    def linear_offsets(self) -> np.ndarray:
        o = OFFSETS
        return (o[:, 0] * (self.ny + 1) + o[:, 1]) * (self.nz + 1) + o[:, 2]


def make_mesh(nx, ny, nz, h, jitter=0.0, rng=None) -> Mesh:
    """Structured box mesh with optional uniform node jitter of +-jitter*h.

    The jitter draw is one ``rng.uniform(-jitter*h, jitter*h, (n, 3))`` in node
    order; the component normal to each boundary face a node lies on is then
    set to zero.
    """
    m = Mesh(nx, ny, nz, float(h), None)
    i, j, k = m.ijk()
    coords = np.stack([i, j, k], axis=1).astype(np.float64) * h
    if jitter:
        d = rng.uniform(-jitter * h, jitter * h, size=(m.n, 3))
        for ax, (ii, nn) in enumerate(((i, nx), (j, ny), (k, nz))):
            d[(ii == 0) | (ii == nn), ax] = 0.0
        coords = coords + d
    m.coords = coords
    return m


def _cell_corner_ids(m: Mesh, x0, x1):
    """Corner node ids of the cells with i in [x0, x1), all j, k (cell order)."""
    ci = np.arange(x0, x1, dtype=np.int64)
    cj = np.arange(m.ny, dtype=np.int64)
    ck = np.arange(m.nz, dtype=np.int64)
    I, J, K = np.meshgrid(ci, cj, ck, indexing="ij")
    return m.node_id(I.ravel(), J.ravel(), K.ravel()), I.ravel(), J.ravel(), K.ravel()


def _element_geometry(X):
    """Barycentric gradients (T,4,3) and volumes (T,) of tets with vertices X (T,4,3)."""
    e1 = X[:, 1] - X[:, 0]
    e2 = X[:, 2] - X[:, 0]
    e3 = X[:, 3] - X[:, 0]
    c23 = np.cross(e2, e3)
    c31 = np.cross(e3, e1)
    c12 = np.cross(e1, e2)
    det = np.einsum("ij,ij->i", e1, c23)
    g1 = c23 / det[:, None]
    g2 = c31 / det[:, None]
    g3 = c12 / det[:, None]
    g0 = -(g1 + g2 + g3)
    G = np.stack([g0, g1, g2, g3], axis=1)
    vol = np.abs(det) / 6.0
    return G, vol


def assemble(m: Mesh, cell_weight=None, slab=16):
    """Assemble K and (weighted) M into per-node slot arrays of shape (n, 15).

    ``cell_weight``: optional callable (I, J, K) -> weight per cell, applied to
    M_e (c_e^-2 for a piecewise-constant speed).  Cells are processed in
    x-slabs of ``slab`` cells; within a slab, element by element in order
    (perm, local pair), adding each symmetric pair in the same step.
    """
    n = m.n
    VK = np.zeros(n * 15)
    VM = np.zeros(n * 15)
    for x0 in range(0, m.nx, slab):
        x1 = min(m.nx, x0 + slab)
        corner, I, J, K = _cell_corner_ids(m, x0, x1)
        w = None if cell_weight is None else cell_weight(I, J, K)
        for perm in PERMS:
            vo = _tet_vertex_offsets(perm)
            vlin = (vo[:, 0] * (m.ny + 1) + vo[:, 1]) * (m.nz + 1) + vo[:, 2]
            nodes = corner[:, None] + vlin[None, :]
            G, vol = _element_geometry(m.coords[nodes])
            mvol = vol / 20.0 if w is None else vol / 20.0 * w
            for a in range(4):
                for b in range(a, 4):
                    kab = vol * np.einsum("ij,ij->i", G[:, a], G[:, b])
                    mab = mvol * (2.0 if a == b else 1.0)
                    sab = _SLOT[tuple(int(v) for v in (vo[b] - vo[a]))]
                    ia = nodes[:, a] * 15 + sab
                    VK[ia] += kab
                    VM[ia] += mab
                    if a != b:
                        sba = _SLOT[tuple(int(v) for v in (vo[a] - vo[b]))]
                        ib = nodes[:, b] * 15 + sba
                        VK[ib] += kab
                        VM[ib] += mab
    return VK.reshape(n, 15), VM.reshape(n, 15)


def _inbounds(m: Mesh):
    i, j, k = m.ijk()
    ok = np.ones((m.n, 15), dtype=bool)
    for s, (di, dj, dk) in enumerate(OFFSETS):
        ok[:, s] = ((i + di >= 0) & (i + di <= m.nx) & (j + dj >= 0) & (j + dj <= m.ny)
                    & (k + dk >= 0) & (k + dk <= m.nz))
    return ok


@dataclasses.dataclass
class FEProblem:
    """CSR pattern plus real stiffness/mass values after Dirichlet elimination."""
    mesh: Mesh
    rowptr: np.ndarray      # int32 (n+1,)
    col: np.ndarray         # int32 (nnz,)
    K: np.ndarray           # float64 (nnz,) ; Dirichlet rows: 1 on the diagonal
    M: np.ndarray           # float64 (nnz,) ; Dirichlet rows: 0
    dirichlet: np.ndarray   # bool (n,)
    slot_of_nnz: np.ndarray  # int8 (nnz,)  neighbour slot of each entry

    @property
    def n(self):
        return self.mesh.n

    @property
    def nnz(self):
        return int(self.col.shape[0])


def build_problem(m: Mesh, cell_weight=None) -> FEProblem:
    VK, VM = assemble(m, cell_weight)
    dirm = m.dirichlet()
    ok = _inbounds(m)
    lin = m.linear_offsets()
    nbr = np.arange(m.n, dtype=np.int64)[:, None] + lin[None, :]
    nbr_dir = np.zeros_like(ok)
    nbr_dir[ok] = dirm[nbr[ok]]
    keep = ok & ~dirm[:, None] & ~nbr_dir
    keep[dirm, :] = False
    keep[:, SELF_SLOT] = True
    VK[dirm, :] = 0.0
    VM[dirm, :] = 0.0
    VK[dirm, SELF_SLOT] = 1.0
    counts = keep.sum(axis=1)
    rowptr = np.zeros(m.n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = nbr[keep].astype(np.int32)
    slots = np.broadcast_to(np.arange(15, dtype=np.int8)[None, :], keep.shape)[keep]
    return FEProblem(m, rowptr.astype(np.int32), col, VK[keep].copy(), VM[keep].copy(),
                     dirm, slots.copy())


def helmholtz_values(p: FEProblem, kappa2: complex) -> np.ndarray:
    """Complex CSR values of A = K - kappa2 * M (kappa2 = k^2 (1 + 0.01 i))."""
    v = np.empty(p.nnz, dtype=np.complex128)
    v.real = p.K - kappa2.real * p.M
    v.imag = -kappa2.imag * p.M
    return v


def complex_rhs(rng, n, dirichlet=None) -> np.ndarray:
    """g = (N(0,1) + i N(0,1)) / sqrt(2), real parts drawn first; g_D = 0."""
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    g = (re + 1j * im) / math.sqrt(2.0)
    if dirichlet is not None:
        g[dirichlet] = 0.0
    return g


def cell_blocks(m: Mesh, bs=8):
    """Block id of every cell for bs^3-cell speed blocks (block k fastest)."""
    nbx, nby, nbz = m.nx // bs, m.ny // bs, m.nz // bs

    def blk(I, J, K):
        return ((I // bs) * nby + (J // bs)) * nbz + (K // bs)
    return (nbx, nby, nbz), blk


def tets_by_block(m: Mesh, bs=8):
    """All tetrahedra, grouped by speed block (stable within a block).

    Returns (nodes int32 (T,4), block int32 (T,), vol float64 (T,),
    block_ptr int32 (nb+1,)); tets of block b are rows block_ptr[b]:block_ptr[b+1].
    """
    (nbx, nby, nbz), blk = cell_blocks(m, bs)
    corner, I, J, K = _cell_corner_ids(m, 0, m.nx)
    b = blk(I, J, K)
    allnodes, allblk, allvol = [], [], []
    for perm in PERMS:
        vo = _tet_vertex_offsets(perm)
        vlin = (vo[:, 0] * (m.ny + 1) + vo[:, 1]) * (m.nz + 1) + vo[:, 2]
        nodes = corner[:, None] + vlin[None, :]
        _, vol = _element_geometry(m.coords[nodes])
        allnodes.append(nodes)
        allblk.append(b)
        allvol.append(vol)
    # element order: cell-major, perm-minor
    nodes = np.stack(allnodes, axis=1).reshape(-1, 4)
    bb = np.stack(allblk, axis=1).reshape(-1)
    vol = np.stack(allvol, axis=1).reshape(-1)
    order = np.argsort(bb, kind="stable")
    nb = nbx * nby * nbz
    ptr = np.zeros(nb + 1, dtype=np.int64)
    np.cumsum(np.bincount(bb, minlength=nb), out=ptr[1:])
    return (nodes[order].astype(np.int32), bb[order].astype(np.int32), vol[order].copy(),
            ptr.astype(np.int32))


def block_mass_lists(p: FEProblem, bs=8):
    """Per-entry decomposition of the unweighted mass matrix by speed block.

    For CSR entry q, entries bm_ptr[q]:bm_ptr[q+1] list (block, mass) pairs with
    sum_b mass = M[q] (up to rounding), restricted to the Dirichlet-eliminated
    pattern.  Then Mc[q] = sum over the list of mass * c_block^-2.
    """
    m = p.mesh
    nodes, blk, vol, _ = tets_by_block(m, bs)
    # contributions are taken in element order (block-sorted, stable) so the
    # (i, j) and (j, i) sums see the same sequence of values
    rows, cols, vals, bl = [], [], [], []
    for a in range(4):
        for b in range(4):
            rows.append(nodes[:, a].astype(np.int64))
            cols.append(nodes[:, b].astype(np.int64))
            vals.append(vol / 20.0 * (2.0 if a == b else 1.0))
            bl.append(blk)
    rows = np.stack(rows, 1).reshape(-1)
    cols = np.stack(cols, 1).reshape(-1)
    vals = np.stack(vals, 1).reshape(-1)
    bl = np.stack(bl, 1).reshape(-1)
    # CSR position of (row, col)
    rp = p.rowptr.astype(np.int64)
    dirm = p.dirichlet
    live = ~dirm[rows] & ~dirm[cols]
    rows, cols, vals, bl = rows[live], cols[live], vals[live], bl[live]
    key_rc = rows * p.n + cols
    csr_rows = np.repeat(np.arange(p.n, dtype=np.int64), np.diff(rp))
    csr_key = csr_rows * p.n + p.col.astype(np.int64)
    pos = np.searchsorted(csr_key, key_rc)
    assert np.all(csr_key[pos] == key_rc)
    order = np.lexsort((bl, pos))          # by position, then block; stable
    pos, bl, vals = pos[order], bl[order], vals[order]
    grp = np.ones(pos.shape[0], dtype=bool)
    grp[1:] = (pos[1:] != pos[:-1]) | (bl[1:] != bl[:-1])
    starts = np.flatnonzero(grp)
    gsum = np.add.reduceat(vals, starts)
    gpos = pos[starts]
    gblk = bl[starts]
    bm_ptr = np.zeros(p.nnz + 1, dtype=np.int64)
    np.cumsum(np.bincount(gpos, minlength=p.nnz), out=bm_ptr[1:])
    return bm_ptr.astype(np.int32), gblk.astype(np.int32), gsum
