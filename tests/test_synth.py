"""Pins of the seeded FE input generator (CPU only).

These check the generator against facts fixed by the mathematics, not against
itself: stiffness rows of a P1 discretisation sum to zero (constants are in
the kernel of the Laplacian), the consistent mass matrix integrates to the
domain volume, element-by-element assembly is exactly symmetric, Dirichlet
elimination leaves identity rows, and on an unjittered Kuhn mesh interior rows
reduce to closed-form stencils.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from synth import helmholtz as H
from synth import configs


def _csr(p, vals):
    return sp.csr_matrix((vals, p.col, p.rowptr), shape=(p.n, p.n))


@pytest.mark.parametrize("dims,extent", [((4, 3, 5), (1.0, 0.75, 1.25)), ((6, 3, 3), (2.0, 1.0, 1.0))])
def test_stiffness_rows_sum_to_zero_and_mass_is_volume(dims, extent):
    h = extent[0] / dims[0]
    m = H.make_mesh(*dims, h, jitter=0.2, rng=np.random.default_rng(7))
    VK, VM = H.assemble(m)
    assert np.max(np.abs(VK.sum(axis=1))) <= 1e-13 * np.max(np.abs(VK))
    vol = dims[0] * dims[1] * dims[2] * h ** 3
    assert abs(VM.sum() - vol) <= 1e-14 * vol


def test_jitter_keeps_faces_planar_and_tets_valid():
    m = H.make_mesh(10, 10, 10, 0.1, jitter=0.2, rng=np.random.default_rng(1))
    i, j, k = m.ijk()
    assert np.all(m.coords[i == 0, 0] == 0.0) and np.allclose(m.coords[i == 10, 0], 1.0, rtol=0, atol=1e-15)
    assert np.all(m.coords[k == 0, 2] == 0.0)
    nodes, blk, vol, ptr = H.tets_by_block(m, bs=5)
    assert vol.min() > 0.0
    assert abs(vol.sum() - 1.0) < 1e-13
    assert ptr[-1] == nodes.shape[0] == 6000 and np.all(np.diff(ptr) == 750)
    assert np.all(blk[ptr[3]:ptr[4]] == 3)


def test_assembly_exactly_symmetric_and_sorted():
    m = H.make_mesh(5, 4, 3, 0.25, jitter=0.2, rng=np.random.default_rng(3))
    c = np.random.default_rng(4).uniform(300, 400, 60)
    p = H.build_problem(m, cell_weight=lambda I, J, K: 1.0 / c[(I * 4 + J) * 3 + K] ** 2)
    for vals in (p.K, p.M):
        A = _csr(p, vals)
        assert (A - A.T).count_nonzero() == 0
    v = H.helmholtz_values(p, complex(1e5, 1e3))
    A = _csr(p, v)
    assert (A - A.T).count_nonzero() == 0
    for i in range(p.n):
        cols = p.col[p.rowptr[i]:p.rowptr[i + 1]]
        assert np.all(np.diff(cols) > 0)


def test_dirichlet_rows_are_identity_and_columns_eliminated():
    m = H.make_mesh(4, 4, 4, 0.25, jitter=0.2, rng=np.random.default_rng(1))
    p = H.build_problem(m)
    d = p.dirichlet
    assert d.sum() == 25
    for i in np.flatnonzero(d):
        a, b = p.rowptr[i], p.rowptr[i + 1]
        assert b - a == 1 and p.col[a] == i and p.K[a] == 1.0 and p.M[a] == 0.0
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    off = rows != p.col
    assert not np.any(d[p.col[off]])


def test_interior_rows_closed_form_stencils():
    """Unjittered Kuhn mesh: K row = h * 7-point Laplacian; M row / h^3 has
    0.4 on the diagonal, 0.05 on axis and body-diagonal neighbours and 1/30
    on face-diagonal neighbours (derived from M_e = vol/20 (1 + delta) and
    the 24 tets around an interior node)."""
    h = 1.0 / 6
    m = H.make_mesh(6, 6, 6, h)
    p = H.build_problem(m)
    i, j, k = m.ijk()
    interior = np.flatnonzero((i > 0) & (i < 6) & (j > 0) & (j < 6) & (k > 1) & (k < 6))
    for r in interior[::7]:
        a, b = p.rowptr[r], p.rowptr[r + 1]
        assert b - a == 15
        for q in range(a, b):
            o = tuple(int(v) for v in H.OFFSETS[p.slot_of_nnz[q]])
            nz = sum(abs(v) for v in o)
            if nz == 0:
                ek, em = 6.0, 0.4
            elif nz == 1:
                ek, em = -1.0, 0.05
            elif nz == 3:
                ek, em = 0.0, 0.05
            else:
                ek, em = 0.0, 1.0 / 30.0
            assert abs(p.K[q] - h * ek) <= 1e-15 * 8
            assert abs(p.M[q] / h ** 3 - em) <= 1e-14


def test_cube16_shape():
    c1 = configs.cube16()
    assert int(c1["n"]) == 4913 and c1["col"].shape[0] == 63183
    assert abs(c1["k"] - 2 * math.pi * 16 / 10) < 1e-12
    assert np.all(c1["g"][c1["dirichlet"]] == 0)


def test_block_mass_lists_reassemble_mass():
    m = H.make_mesh(4, 4, 4, 0.25, jitter=0.2, rng=np.random.default_rng(1))
    c = np.random.default_rng(9).uniform(300, 400, 8)
    (_, nby, nbz), blk = H.cell_blocks(m, 2)
    pw = H.build_problem(m, cell_weight=lambda I, J, K: 1.0 / c[blk(I, J, K)] ** 2)
    pu = H.build_problem(m)
    ptr, bb, bv = H.block_mass_lists(pu, 2)
    assert ptr[-1] == bb.shape[0]
    seg = np.repeat(np.arange(pu.nnz), np.diff(ptr))
    Mu = np.bincount(seg, weights=bv, minlength=pu.nnz)
    Mw = np.bincount(seg, weights=bv / c[bb] ** 2, minlength=pu.nnz)
    assert np.max(np.abs(Mu - pu.M)) <= 1e-15 * np.max(pu.M) * 4
    assert np.max(np.abs(Mw - pw.M)) <= 1e-15 * np.max(pw.M) * 4


# ------------------------------------------------------------ Q1 hexahedra

def test_hex_interior_closed_form_stencils_and_invariants():
    """Unjittered interior rows equal the Q1 tensor-product stencils (stiffness
    8h/3, 0, -h/6, -h/12 and mass 8h^3/27, 2h^3/27, h^3/54, h^3/216 for the
    centre, face, edge and corner neighbours); K rows sum to zero and the
    mass sums to the volume, also on a jittered mesh."""
    from synth import hexahedra as Q
    h = 0.2
    m = H.make_mesh(5, 5, 5, h)
    VK, VM = Q.assemble_hex(m)
    i, j, k = m.ijk()
    interior = np.where((i > 0) & (i < 5) & (j > 0) & (j < 5) & (k > 0) & (k < 5))[0]
    kd = {0: 8 * h / 3, 1: 0.0, 2: -h / 6, 3: -h / 12}
    md = {0: 8 * h ** 3 / 27, 1: 2 * h ** 3 / 27, 2: h ** 3 / 54, 3: h ** 3 / 216}
    nnzo = np.count_nonzero(Q.OFFSETS27, axis=1)
    for r in interior:
        assert np.allclose(VK[r], [kd[c] for c in nnzo], rtol=0, atol=1e-14)
        assert np.allclose(VM[r], [md[c] for c in nnzo], rtol=0, atol=1e-16)
    mj = H.make_mesh(6, 5, 4, 0.25, jitter=0.2, rng=np.random.default_rng(3))
    VK, VM = Q.assemble_hex(mj)
    assert np.abs(VK.sum(axis=1)).max() <= 1e-13
    assert abs(VM.sum() - 6 * 5 * 4 * 0.25 ** 3) <= 1e-13


def test_hex_problem_symmetric_sorted_dirichlet():
    from synth import hexahedra as Q
    m = H.make_mesh(5, 4, 6, 0.2, jitter=0.2, rng=np.random.default_rng(4))
    p = Q.build_hex_problem(m)
    A = sp.csr_matrix((p.K + 1j * p.M, p.col, p.rowptr), shape=(p.n, p.n))
    assert (A != A.T).nnz == 0
    lens = np.diff(p.rowptr)
    assert lens.max() == 27
    for r in range(p.n):
        c = p.col[p.rowptr[r]:p.rowptr[r + 1]]
        assert np.all(np.diff(c) > 0)
    for r in np.where(p.dirichlet)[0]:
        assert lens[r] == 1 and p.col[p.rowptr[r]] == r and p.K[p.rowptr[r]] == 1.0 and p.M[p.rowptr[r]] == 0.0
    dcols = np.isin(p.col, np.where(p.dirichlet)[0])
    rows = np.repeat(np.arange(p.n), lens)
    assert np.all(rows[dcols] == p.col[dcols])
