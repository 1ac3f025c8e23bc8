"""GPU parity of the CSR product, BLAS-1 and BiCGStab against the CPU oracle.

Every case prints its name before launching anything.  Bounds:
  * SpMV: |dy_i| <= 1e-12 * sum_p |a_ip| |x_col(p)| per row (rows can cancel).
  * dots / norms: |d - d_ref| <= 1e-12 * sum |x_i| |y_i|.
  * element-wise ops: |d| <= 4 eps |result terms| per element.
  * solves at tol 1e-8: the oracle recomputes ||b - A x|| / ||b|| <= 1.05e-8;
    at tol 1e-10 the solution is within 1e-7 of the oracle's solution.
"""
import os
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from synth import helmholtz as H
from synth import configs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hk():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2112_11880_amd as hk
    hk.load()
    return hk


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def crandn(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def spmv_bound(rowptr, col, val, x):
    n = rowptr.shape[0] - 1
    A = sp.csr_matrix((np.abs(val), col, rowptr), shape=(n, n))
    return A @ np.abs(x)


def make_csr(hk, rowptr, col, val, autotune=False):
    return hk.CSR(dev(rowptr), dev(col), dev(val), autotune=autotune)


def small_mesh_problem(nc=(7, 5, 6), seed=3):
    m = H.make_mesh(*nc, 1.0 / nc[0], jitter=0.2, rng=np.random.default_rng(seed))
    p = H.build_problem(m)
    val = H.helmholtz_values(p, complex(300.0, 3.0))
    return p.rowptr, p.col, val


# ------------------------------------------------------------------ SpMV

SHAPES = ([(L, U, g) for L in (4, 8, 16, 32) for U in (1, 2, 4, 8) for g in (0, 3, 64) if U <= L]
          + [(64, rw, g) for rw in (16, 32, 64) for g in (0, 3, 64)])


def test_spmv_all_shapes_ragged(hk, oracle):
    """Every launch shape, with the 16-bit column stream (the default for
    this banded matrix) and with the int32 indices: oracle parity, and the
    row-block shapes give the same bits from either stream."""
    rowptr, col, val = small_mesh_problem()
    n = rowptr.shape[0] - 1
    x = crandn(np.random.default_rng(1), n)
    ref = oracle.spmv(rowptr, col, val, x)
    bound = 1e-12 * spmv_bound(rowptr, col, val, x)
    xd = dev(x)
    outs = {}
    for compact in (True, False):
        A = hk.CSR(dev(rowptr), dev(col), dev(val), compact_cols=compact)
        assert A.info() == {"n": n, "nnz": col.shape[0], "max_row": int(np.diff(rowptr).max()),
                            "col_bytes": 2 if compact else 4}
        for L, U, g in SHAPES:
            say("spmv shape", L, U, g, "n", n, "compact", compact)
            A.set_plan(L, U, g)
            # NaN-filled output: a row the kernel fails to write cannot pass
            y = host(A.spmv(xd, torch.full_like(xd, complex("nan+nanj")), beta=0.0))
            assert np.all(np.abs(y - ref) <= bound), (L, U, g, compact)
            outs[(L, U, g, compact)] = y
        for bad in ((4, 8, 0), (64, 8, 0), (64, 128, 0), (2, 1, 0)):
            with pytest.raises(hk.HKError):
                A.set_plan(*bad)
    for L, U, g in SHAPES:
        if L == 64:
            assert np.array_equal(outs[(L, U, g, True)], outs[(L, U, g, False)]), (U, g)


def random_structure(rng, n, max_row):
    """CSR with row lengths drawn from [0, max_row] (a quarter of the rows
    empty), sorted distinct columns anywhere in [0, n), random values."""
    lens = rng.integers(0, max_row + 1, n)
    lens[rng.random(n) < 0.25] = 0
    lens = np.minimum(lens, n)
    rowptr = np.zeros(n + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum(lens)
    col = np.concatenate([np.sort(rng.choice(n, size=k, replace=False)) for k in lens]
                         + [np.zeros(0, dtype=np.int64)]).astype(np.int32)
    val = crandn(rng, int(rowptr[-1]))
    return rowptr, col, val


def test_spmv_random_structures(hk, oracle):
    """Unstructured matrices: rows of 0 to 700 entries (longer than one pass
    of a row-block wave, 512 entries), columns anywhere, n not a multiple of
    64; every launch shape on both column streams against the oracle."""
    for seed, n, max_row in ((31, 1001, 40), (32, 2500, 700), (33, 77, 77)):
        rng = np.random.default_rng(seed)
        rowptr, col, val = random_structure(rng, n, max_row)
        x = crandn(rng, n)
        ref = oracle.spmv(rowptr, col, val, x)
        bound = 1e-12 * spmv_bound(rowptr, col, val, x)
        xd = dev(x)
        for compact in (True, False):
            A = hk.CSR(dev(rowptr), dev(col), dev(val), compact_cols=compact)
            for L, U, g in SHAPES:
                say("spmv random", seed, n, max_row, "shape", L, U, g, "compact", compact)
                A.set_plan(L, U, g)
                y = host(A.spmv(xd, torch.full_like(xd, complex("nan+nanj")), beta=0.0))
                assert np.all(np.abs(y - ref) <= bound), (seed, L, U, g, compact)


def test_spmv_column_stream_limits(hk, oracle):
    """The 16-bit column stream is built exactly when every |col - (row &
    ~63)| <= 32767; at the limit, one past it and with offsets of both signs
    the row-block products match the oracle."""
    rng = np.random.default_rng(8)
    n = 40000
    for name, extra, want in (("limit +32767", (100, 64 + 32767), 2),
                              ("past +32768", (100, 64 + 32768), 4),
                              ("limit -32767", (39999, 39936 - 32767), 2),
                              ("past -32768", (39999, 39936 - 32768), 4)):
        rows = [np.array([i - 1, i, i + 1]) for i in range(n)]
        rows[0], rows[-1] = np.array([0, 1]), np.array([n - 2, n - 1])
        r, c = extra
        rows[r] = np.unique(np.append(rows[r], c))
        rows = [q[(q >= 0) & (q < n)] for q in rows]
        rowptr = np.zeros(n + 1, dtype=np.int32)
        rowptr[1:] = np.cumsum([len(q) for q in rows])
        col = np.concatenate(rows).astype(np.int32)
        val = crandn(rng, col.shape[0])
        x = crandn(rng, n)
        ref = oracle.spmv(rowptr, col, val, x)
        bound = 1e-12 * spmv_bound(rowptr, col, val, x)
        A = make_csr(hk, rowptr, col, val)
        assert A.info()["col_bytes"] == want, name
        for U in (16, 32, 64):
            say("column stream", name, "rows per wave", U)
            A.set_plan(64, U, 0)
            y = host(A.spmv(dev(x)))
            assert np.all(np.abs(y - ref) <= bound), (name, U)


def test_spmv_alpha_beta_and_residual(hk, oracle):
    say("spmv alpha/beta/residual")
    rowptr, col, val = small_mesh_problem((5, 6, 4), 5)
    n = rowptr.shape[0] - 1
    rng = np.random.default_rng(2)
    x, y0, b = crandn(rng, n), crandn(rng, n), crandn(rng, n)
    A = make_csr(hk, rowptr, col, val)
    al, be = complex(0.5, -2.0), complex(-1.25, 0.75)
    y = host(A.spmv(dev(x), dev(y0), al, be))
    ax = oracle.spmv(rowptr, col, val, x)
    ref = al * ax + be * y0
    bnd = 1e-12 * (abs(al) * spmv_bound(rowptr, col, val, x) + abs(be) * np.abs(y0))
    assert np.all(np.abs(y - ref) <= bnd)
    r = host(A.residual(dev(b), dev(x)))
    ref = oracle.residual(rowptr, col, val, b, x)
    bnd = 1e-12 * (spmv_bound(rowptr, col, val, x) + np.abs(b))
    assert np.all(np.abs(r - ref) <= bnd)


def test_spmv_edge_structures(hk, oracle):
    """Empty rows, a single row, rows longer than every lane group."""
    rng = np.random.default_rng(4)
    cases = []
    # empty rows interleaved, a 150-entry row, a 1-entry matrix
    n = 300
    lens = rng.integers(0, 6, n)
    lens[::7] = 0
    lens[123] = 150
    rowptr = np.zeros(n + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum(lens)
    col = np.concatenate([np.sort(rng.choice(n, l, replace=False)) for l in lens]).astype(np.int32)
    cases.append(("ragged", rowptr, col))
    cases.append(("one", np.array([0, 1], dtype=np.int32), np.array([0], dtype=np.int32)))
    # no entries at all: y = 0, and the residual is b
    cases.append(("empty", np.zeros(40, dtype=np.int32), np.zeros(0, dtype=np.int32)))
    # 30 entries per row: a 64-row block spans several passes of the row-block scheme
    n2 = 200
    rowptr2 = np.arange(n2 + 1, dtype=np.int32) * 30
    col2 = np.concatenate([np.sort(rng.choice(n2, 30, replace=False)) for _ in range(n2)]).astype(np.int32)
    cases.append(("wide", rowptr2, col2))
    for name, rowptr, col in cases:
        n = rowptr.shape[0] - 1
        val = crandn(rng, col.shape[0])
        x = crandn(rng, n)
        ref = oracle.spmv(rowptr, col, val, x)
        bound = 1e-12 * spmv_bound(rowptr, col, val, x)
        A = make_csr(hk, rowptr, col, val)
        for L, U, g in SHAPES[::5] + SHAPES[-9:]:
            say("spmv edge", name, L, U, g)
            A.set_plan(L, U, g)
            xd = dev(x)
            y = host(A.spmv(xd, torch.full_like(xd, complex("nan+nanj")), beta=0.0))
            assert np.all(np.abs(y - ref) <= bound), (name, L, U, g)
        if name == "empty":
            assert np.all(y == 0)
            bb = crandn(rng, n)
            assert np.array_equal(host(A.residual(dev(bb), xd)), bb)


def test_reductions_of_length_zero_and_one(hk):
    """An empty dot or norm is 0; a length-1 one is the single term."""
    say("reductions n = 0, 1")
    e = torch.zeros(0, dtype=torch.complex128, device=DEV)
    out = torch.full((1,), complex(7, 7), dtype=torch.complex128, device=DEV)
    assert host(hk.zdotc(e, e, out))[0] == 0 and host(hk.zdotu(e, e, out))[0] == 0
    nrm = torch.full((1,), 7.0, dtype=torch.float64, device=DEV)
    assert host(hk.dznrm2(e, nrm))[0] == 0
    x, y = complex(3, -4), complex(0.5, 2)
    xd = torch.tensor([x], dtype=torch.complex128, device=DEV)
    yd = torch.tensor([y], dtype=torch.complex128, device=DEV)
    assert host(hk.zdotc(xd, yd))[0] == x.conjugate() * y
    assert host(hk.zdotu(xd, yd))[0] == x * y
    assert host(hk.dznrm2(xd))[0] == 5.0


def test_graph_replays_match_direct_launches(hk, monkeypatch):
    """The solvers replay one recorded chunk of iterations as a HIP graph; with
    HK_SOLVE_GRAPHS=0 they launch every kernel directly.  Both give the same
    bits, in every method, with a chunk of 3 iterations (many replays, each
    followed by the host's status read) and with the default chunk."""
    rowptr, col, val = small_mesh_problem()
    n = rowptr.shape[0] - 1
    b = crandn(np.random.default_rng(21), n)
    A = make_csr(hk, rowptr, col, val, autotune=True)
    for method, kw in (("bicgstab", {}), ("tfqmr", {}), ("bicgstab_l", {"ell": 4})):
        for every in (3, 0):
            got = {}
            for graphs in ("1", "0"):
                monkeypatch.setenv("HK_SOLVE_GRAPHS", graphs)
                say("graph replay", method, "check_every", every, "graphs", graphs)
                x, info = hk.krylov_solve(A, dev(b), tol=1e-10, check_every=every, method=method, **kw)
                got[graphs] = (host(x), info)
            assert got["1"][1] == got["0"][1], (method, every)
            assert np.array_equal(got["1"][0], got["0"][0]), (method, every)
            assert got["1"][1]["status"] == hk.HK_OK, got["1"][1]
    monkeypatch.delenv("HK_SOLVE_GRAPHS")


def test_binding_rejects_wrong_lengths(hk):
    """The library takes raw pointers, so the binding checks every vector's
    length against the matrix (or its partner) before any launch."""
    say("binding length checks")
    rowptr = np.array([0, 1, 2, 3], dtype=np.int32)
    col = np.array([0, 1, 2], dtype=np.int32)
    A = make_csr(hk, rowptr, col, np.ones(3, dtype=np.complex128))
    x3, x2 = dev(np.ones(3, dtype=np.complex128)), dev(np.ones(2, dtype=np.complex128))
    with pytest.raises(hk.HKError, match="elements"):
        A.spmv(x2)
    with pytest.raises(hk.HKError, match="elements"):
        A.spmv(x3, x2)
    with pytest.raises(hk.HKError, match="elements"):
        A.residual(x3, x2)
    with pytest.raises(hk.HKError, match="elements"):
        hk.krylov_solve(A, x2)
    with pytest.raises(hk.HKError, match="elements"):
        hk.krylov_solve(A, x3, x=x2)
    for f in (hk.zdotc, hk.zdotu, hk.zcopy, hk.zaxmy):
        with pytest.raises(hk.HKError, match="elements"):
            f(x3, x2)
    with pytest.raises(hk.HKError, match="elements"):
        hk.zaxpy(1.0, x3, x2)
    with pytest.raises(hk.HKError):
        hk.CSR(dev(rowptr), dev(col), dev(np.ones(2, dtype=np.complex128)))
    # the checks pass matching lengths through
    assert np.allclose(host(A.spmv(x3)), np.ones(3))


def test_csr_create_rejects_bad_structure(hk):
    say("csr validation")
    rowptr = np.array([0, 2, 3], dtype=np.int32)
    for col in (np.array([1, 0, 0], dtype=np.int32), np.array([0, 5, 1], dtype=np.int32)):
        with pytest.raises(hk.HKError):
            make_csr(hk, rowptr, col, np.ones(3, dtype=np.complex128))
    with pytest.raises(hk.HKError):
        make_csr(hk, np.array([0, 3, 2], dtype=np.int32), np.array([0, 1, 0], dtype=np.int32),
                 np.ones(3, dtype=np.complex128))


def test_spmv_complex64(hk, oracle):
    say("spmv complex64")
    rowptr, col, val = small_mesh_problem((6, 6, 6), 7)
    n = rowptr.shape[0] - 1
    x = crandn(np.random.default_rng(9), n).astype(np.complex64)
    v32 = val.astype(np.complex64)
    ref = oracle.spmv(rowptr, col, v32.astype(np.complex128), x.astype(np.complex128))
    bound = 1e-5 * spmv_bound(rowptr, col, v32, x)
    A = make_csr(hk, rowptr, col, v32)
    y = host(A.spmv(dev(x)))
    assert np.all(np.abs(y - ref) <= bound)


def c64_row_bound(rowptr, col, v32, x32, b32=None):
    """Rounding bound of a complex64 CSR row (float32 products summed in
    float32, any order): (len + 4) * 2u * (sum |a||x| (+ |b|)), u = 2^-24."""
    lens = np.diff(rowptr).astype(np.float64)
    s = spmv_bound(rowptr, col, v32.astype(np.complex128), x32.astype(np.complex128))
    if b32 is not None:
        s = s + np.abs(b32.astype(np.complex128))
    return (lens + 5) * 2.0 ** -23 * s


def test_spmv_complex64_all_shapes(hk, oracle):
    """complex64 CSR product and residual in every launch shape, on both
    column streams, for a mesh matrix and a random structure with rows of 0 to
    700 entries: within the float32 rounding bound of each row of the oracle's
    exact (FP64) product of the same float32 values; the row-block shapes
    give the same bits from either stream."""
    rng = np.random.default_rng(41)
    cases = [("mesh", *small_mesh_problem((6, 7, 5), 11)),
             ("random", *random_structure(np.random.default_rng(42), 2500, 700))]
    for name, rowptr, col, val in cases:
        n = rowptr.shape[0] - 1
        v32 = val.astype(np.complex64)
        x32 = crandn(rng, n).astype(np.complex64)
        b32 = crandn(rng, n).astype(np.complex64)
        ref = oracle.spmv(rowptr, col, v32.astype(np.complex128), x32.astype(np.complex128))
        bound = c64_row_bound(rowptr, col, v32, x32)
        rbound = c64_row_bound(rowptr, col, v32, x32, b32)
        xd, bd = dev(x32), dev(b32)
        outs = {}
        for compact in (True, False):
            A = hk.CSR(dev(rowptr), dev(col), dev(v32), compact_cols=compact)
            for L, U, g in SHAPES:
                say("spmv complex64", name, "n", n, "shape", L, U, g, "compact", compact)
                A.set_plan(L, U, g)
                y = host(A.spmv(xd, torch.full_like(xd, complex("nan+nanj")), beta=0.0))
                assert np.all(np.abs(y - ref) <= bound), (name, L, U, g, compact)
                outs[(L, U, g, compact)] = y
                r = host(A.residual(bd, xd))
                assert np.all(np.abs(r - (b32.astype(np.complex128) - ref)) <= rbound), (name, L, U, g)
        for L, U, g in SHAPES:
            if L == 64:
                assert np.array_equal(outs[(L, U, g, True)], outs[(L, U, g, False)]), (name, U, g)


def test_spmv_cube16_and_autotune(hk, oracle):
    c = configs.cube16()
    x = crandn(np.random.default_rng(5), int(c["n"]))
    ref = oracle.spmv(c["rowptr"], c["col"], c["val"], x)
    bound = 1e-12 * spmv_bound(c["rowptr"], c["col"], c["val"], x)
    say("spmv cube16 autotune")
    A = make_csr(hk, c["rowptr"], c["col"], c["val"], autotune=True)
    assert A.plan()["tuned"]
    y = host(A.spmv(dev(x)))
    assert np.all(np.abs(y - ref) <= bound)


def test_spmv_box192_full(hk, oracle):
    """The 1.8M-row / 26.6M-nnz matrix, every row, in the benchmark's launch
    shapes: the autotuned handle on the arrays as given (int32 columns, the
    benchmark's headline product) and on the 16-bit column stream (the
    solvers' handle), each launched as the benchmark does (back to back, then
    checked)."""
    c = configs.box192()
    n = int(c["n"])
    x = crandn(np.random.default_rng(6), n)
    ref = oracle.spmv(c["rowptr"], c["col"], c["val"], x)
    bound = 1e-12 * spmv_bound(c["rowptr"], c["col"], c["val"], x)
    xd = dev(x)
    for compact in (False, True):
        say("spmv box192 autotune, 16-bit columns" if compact else "spmv box192 autotune, int32 columns", n)
        A = hk.CSR(dev(c["rowptr"]), dev(c["col"]), dev(c["val"]), autotune=True, compact_cols=compact)
        say("plan", A.plan(), A.info())
        assert A.info()["col_bytes"] == (2 if compact else 4)
        y = torch.full_like(xd, complex("nan+nanj"))
        for _ in range(4):
            A.spmv(xd, y)
        assert np.all(np.abs(host(y) - ref) <= bound), compact


# -------------------------------------------------------------- BLAS-1

SIZES = [1, 63, 255, 1000, 4913, 100003, 648849]


def test_dots_and_norm_parity(hk, oracle):
    rng = np.random.default_rng(7)
    for n in SIZES:
        say("dots n", n)
        x, y = crandn(rng, n), crandn(rng, n)
        xd, yd = dev(x), dev(y)
        scale = np.sum(np.abs(x) * np.abs(y))
        for f, g in ((hk.zdotc, oracle.zdotc), (hk.zdotu, oracle.zdotu)):
            d = host(f(xd, yd))[0]
            assert abs(d - g(x, y)) <= 1e-12 * scale, (n, f.__name__)
        nr = host(hk.dznrm2(xd))[0]
        assert abs(nr - oracle.dznrm2(x)) <= 1e-12 * oracle.dznrm2(x)


def test_dots_and_norm_parity_large(hk, oracle):
    """Sizes that take the reductions' other paths: 2,097,153 elements (1,025
    partials, the first size whose finalize runs 1,024 threads) and the
    paper's 9M and 14M (the 4,096-workgroup cap, each workgroup walking a
    longer chunk, with a ragged last chunk)."""
    rng = np.random.default_rng(17)
    for n in (2097153, 9000000, 14000000):
        say("dots large n", n)
        x, y = crandn(rng, n), crandn(rng, n)
        xd, yd = dev(x), dev(y)
        scale = np.sum(np.abs(x) * np.abs(y))
        for f, g in ((hk.zdotc, oracle.zdotc), (hk.zdotu, oracle.zdotu)):
            d = host(f(xd, yd))[0]
            assert abs(d - g(x, y)) <= 1e-12 * scale, (n, f.__name__)
        nr = host(hk.dznrm2(xd))[0]
        assert abs(nr - oracle.dznrm2(x)) <= 1e-12 * oracle.dznrm2(x), n
        del xd, yd
        torch.cuda.empty_cache()


def test_dot_deterministic_14m(hk):
    """Bitwise the same result on every call at the paper's largest size
    (4,096 workgroups, the 1,024-thread finalize)."""
    say("dot determinism 14M")
    rng = np.random.default_rng(18)
    n = 14000000
    x, y = dev(crandn(rng, n)), dev(crandn(rng, n))
    ref_c, ref_u, ref_n = host(hk.zdotc(x, y)), host(hk.zdotu(x, y)), host(hk.dznrm2(x))
    for _ in range(5):
        assert np.array_equal(host(hk.zdotc(x, y)), ref_c)
        assert np.array_equal(host(hk.zdotu(x, y)), ref_u)
        assert np.array_equal(host(hk.dznrm2(x)), ref_n)


def test_dot_deterministic(hk):
    say("dot determinism")
    rng = np.random.default_rng(8)
    x, y = dev(crandn(rng, 1 << 20)), dev(crandn(rng, 1 << 20))
    ref = host(hk.zdotc(x, y))
    for _ in range(10):
        assert np.array_equal(host(hk.zdotc(x, y)), ref)


def test_elementwise_parity(hk, oracle):
    rng = np.random.default_rng(9)
    a = complex(0.75, -1.5)
    eps = 2.0 ** -52
    for n in (1, 257, 100003):
        say("elementwise n", n)
        x, y = crandn(rng, n), crandn(rng, n)
        got = host(hk.zaxpy(a, dev(x), dev(y)))
        ref = oracle.zaxpy(a, x, y)
        assert np.all(np.abs(got - ref) <= 4 * eps * (abs(a) * np.abs(x) + np.abs(y)))
        got = host(hk.zscal(a, dev(x)))
        assert np.all(np.abs(got - oracle.zscal(a, x)) <= 4 * eps * abs(a) * np.abs(x))
        got = host(hk.zaxmy(dev(x), dev(y)))
        assert np.all(np.abs(got - oracle.zaxmy(x, y)) <= 4 * eps * np.abs(x) * np.abs(y))
        got = host(hk.zcopy(dev(x), dev(np.zeros_like(x))))
        assert np.array_equal(got, x)
        assert np.array_equal(host(hk.zconj(dev(x))), np.conj(x))


# ------------------------------------------------------------- BiCGStab

def test_solve_cube16(hk, oracle):
    c = configs.cube16()
    A = make_csr(hk, c["rowptr"], c["col"], c["val"], autotune=True)
    b = dev(c["g"])
    say("solve cube16 tol 1e-8")
    x8, info8 = hk.krylov_solve(A, b, tol=1e-8)
    assert info8["status"] == hk.HK_OK, info8
    xh = host(x8)
    r = oracle.residual(c["rowptr"], c["col"], c["val"], c["g"], xh)
    assert np.linalg.norm(r) / np.linalg.norm(c["g"]) <= 1.05e-8
    assert abs(info8["relres_true"] - np.linalg.norm(r) / np.linalg.norm(c["g"])) <= 1e-10
    _, oi8 = oracle.bicgstab(c["rowptr"], c["col"], c["val"], c["g"], tol=1e-8)
    say("iterations gpu", info8["iters"], "oracle", oi8["iters"])
    # BiCGStab on this indefinite system is sensitive to rounding order: the
    # oracle (2,410), a NumPy run of the same recurrences (1,960) and this
    # path all reach 1e-8, at counts up to ~20% apart.
    assert abs(info8["iters"] - oi8["iters"]) <= 0.25 * oi8["iters"]
    say("solve cube16 tol 1e-10")
    x10, info10 = hk.krylov_solve(A, b, tol=1e-10)
    assert info10["status"] == hk.HK_OK
    xo, _ = oracle.bicgstab(c["rowptr"], c["col"], c["val"], c["g"], tol=1e-10)
    assert np.linalg.norm(host(x10) - xo) <= 1e-7 * np.linalg.norm(xo)
    say("solve determinism")
    x10b, info10b = hk.krylov_solve(A, b, tol=1e-10)
    assert np.array_equal(host(x10b), host(x10)) and info10b["iters"] == info10["iters"]


def test_solve_small_matches_oracle_iterates(hk, oracle):
    """Few iterations on a small system: same iterate as the oracle to rounding."""
    rowptr, col, val = small_mesh_problem((5, 5, 5), 11)
    n = rowptr.shape[0] - 1
    b = crandn(np.random.default_rng(3), n)
    A = make_csr(hk, rowptr, col, val)
    # rounding differences (Jacobi folded into the matrix, reduction order)
    # grow with each step of the recurrence
    for k, bound in ((1, 1e-12), (2, 1e-11), (5, 1e-10)):
        say("solve maxit", k)
        x, info = hk.krylov_solve(A, dev(b), tol=1e-14, max_iter=k)
        xo, oi = oracle.bicgstab(rowptr, col, val, b, tol=1e-14, maxit=k)
        assert info["status"] == hk.HK_NOT_CONVERGED and info["iters"] == k
        assert np.linalg.norm(host(x) - xo) <= bound * np.linalg.norm(xo)
        assert abs(info["relres_rec"] - oi["relres_rec"]) <= bound * 10


def test_solve_every_launch_shape(hk, oracle):
    """The fused SpMV+dot kernels of the solver in every launch shape: two
    iterations give the oracle's iterate to rounding."""
    rowptr, col, val = small_mesh_problem((7, 6, 5), 13)
    n = rowptr.shape[0] - 1
    b = crandn(np.random.default_rng(4), n)
    xo, oi = oracle.bicgstab(rowptr, col, val, b, tol=1e-14, maxit=2)
    A = make_csr(hk, rowptr, col, val)
    for L, U, g in SHAPES:
        say("solve shape", L, U, g)
        A.set_plan(L, U, g)
        x, info = hk.krylov_solve(A, dev(b), tol=1e-14, max_iter=2)
        assert info["iters"] == 2
        assert np.linalg.norm(host(x) - xo) <= 1e-11 * np.linalg.norm(xo), (L, U, g)


def test_solve_complex64_matches_oracle_iterates(hk, oracle):
    """complex64 BiCGStab (float accumulation) vs the oracle's complex-float
    solver: a few iterations in every launch shape, then two full solves in a
    row on one handle (workspace reuse) with different right-hand sides."""
    rowptr, col, val = small_mesh_problem((5, 5, 5), 11)
    n = rowptr.shape[0] - 1
    v32 = val.astype(np.complex64)
    rng = np.random.default_rng(21)
    b1 = crandn(rng, n).astype(np.complex64)
    b2 = (1e-3 * crandn(rng, n)).astype(np.complex64)
    A = make_csr(hk, rowptr, col, v32)
    # On this indefinite system the oracle's own complex-float iterate
    # differs from its complex128 iterate (same rounded matrix) by 1.0e-7
    # after one step and 4.8e-7 after two (5.9e-6 after three, 5e-4 after
    # five): rounding differences grow quickly, so only two steps are compared.
    xo1, _ = oracle.bicgstab_c64(rowptr, col, v32, b1, tol=1e-9, maxit=1)
    xo2, oi2 = oracle.bicgstab_c64(rowptr, col, v32, b1, tol=1e-9, maxit=2)
    assert oi2["iters"] == 2
    for L, U, g in SHAPES[::3]:
        say("c64 solve shape", L, U, g)
        A.set_plan(L, U, g)
        for k, xo, bound in ((1, xo1, 1e-6), (2, xo2, 1e-5)):
            x, info = hk.krylov_solve(A, dev(b1), tol=1e-9, max_iter=k)
            assert info["iters"] == k and info["status"] == hk.HK_NOT_CONVERGED
            assert np.linalg.norm(host(x) - xo) <= bound * np.linalg.norm(xo), (L, U, g, k)
    A.set_plan(16, 1, 0)
    for b in (b1, b2, b1):
        say("c64 full solve", float(np.linalg.norm(b)))
        x, info = hk.krylov_solve(A, dev(b), tol=1e-4)
        xo, oi = oracle.bicgstab_c64(rowptr, col, v32, b, tol=1e-4)
        say("gpu", info, "oracle", oi)
        assert info["status"] == 0 and oi["status"] == 0
        r = oracle.residual(rowptr, col, val, b.astype(np.complex128), host(x).astype(np.complex128))
        assert np.linalg.norm(r) <= 2e-4 * np.linalg.norm(b)


def test_solve_breakdowns_and_errors(hk, oracle):
    say("sigma breakdown")
    A = make_csr(hk, np.array([0, 2, 4], dtype=np.int32), np.array([0, 1, 0, 1], dtype=np.int32),
                 np.array([1.0, -1.25, -1.25, 1.0], dtype=np.complex128))
    x, info = hk.krylov_solve(A, dev(np.array([1.0, 2.0], dtype=np.complex128)), tol=1e-12)
    assert info["status"] == hk.HK_BREAKDOWN and hk.BD_NAMES[info["breakdown"]] == "sigma"
    assert info["iters"] == 0 and np.all(host(x) == 0)
    say("omega breakdown")
    M = np.array([[1, 1, 0], [1, 1, -1], [1, -1, 1]], dtype=np.complex128)
    A = make_csr(hk, np.array([0, 3, 6, 9], dtype=np.int32), np.tile(np.arange(3, dtype=np.int32), 3),
                 M.ravel())
    x, info = hk.krylov_solve(A, dev(np.array([1.0, 0, 0], dtype=np.complex128)), tol=1e-14)
    assert info["status"] == hk.HK_BREAKDOWN and hk.BD_NAMES[info["breakdown"]] == "omega"
    assert info["iters"] == 1 and np.array_equal(host(x), np.array([1.0, 0, 0]))
    say("zero diagonal")
    A = make_csr(hk, np.array([0, 1, 2], dtype=np.int32), np.array([1, 0], dtype=np.int32),
                 np.ones(2, dtype=np.complex128))
    with pytest.raises(hk.HKError):
        hk.krylov_solve(A, dev(np.ones(2, dtype=np.complex128)))
    say("nonfinite rhs")
    c = configs.cube16()
    A = make_csr(hk, c["rowptr"], c["col"], c["val"])
    g = c["g"].copy()
    g[7] = np.nan
    _, info = hk.krylov_solve(A, dev(g))
    assert info["status"] == hk.HK_NONFINITE
    say("zero rhs and exact start")
    x, info = hk.krylov_solve(A, dev(np.zeros_like(c["g"])))
    assert info["status"] == hk.HK_OK and info["iters"] == 0
    xo, _ = oracle.bicgstab(c["rowptr"], c["col"], c["val"], c["g"], tol=1e-12)
    x, info = hk.krylov_solve(A, dev(c["g"]), x=dev(xo), tol=1e-8)
    assert info["status"] == hk.HK_OK and info["iters"] == 0
    say("diagonal one step")
    rng = np.random.default_rng(2)
    d = crandn(rng, 50) + 3.0
    bb = crandn(rng, 50)
    A = make_csr(hk, np.arange(51, dtype=np.int32), np.arange(50, dtype=np.int32), d)
    x, info = hk.krylov_solve(A, dev(bb), tol=1e-12)
    assert info["status"] == hk.HK_OK and info["iters"] == 1
    assert np.allclose(host(x), bb / d, rtol=1e-14, atol=0)


def test_solve_history(hk):
    say("history")
    c = configs.cube16()
    A = make_csr(hk, c["rowptr"], c["col"], c["val"])
    x, info, hist = hk.krylov_solve(A, dev(c["g"]), tol=1e-6, history=True)
    h = host(hist)
    assert h[0] == pytest.approx(1.0) and h[-1] <= 1e-6 and h[-1] == pytest.approx(info["relres_rec"])


def test_mixed_cube16(hk, oracle):
    c = configs.cube16()
    A = make_csr(hk, c["rowptr"], c["col"], c["val"], autotune=True)
    say("mixed cube16", A.plan())
    x, info = hk.krylov_solve_mixed(A, dev(c["g"]), inner_tol=1e-4, outer_tol=1e-10)
    assert info["status"] == hk.HK_OK, info
    xh = host(x)
    r = oracle.residual(c["rowptr"], c["col"], c["val"], c["g"], xh)
    assert np.linalg.norm(r) / np.linalg.norm(c["g"]) <= 1.05e-10
    xo, _ = oracle.bicgstab(c["rowptr"], c["col"], c["val"], c["g"], tol=1e-12)
    err = np.linalg.norm(xh - xo) / np.linalg.norm(xo)
    say("mixed outer", info["iters"], "inner", info["inner_iters"], "err vs fp64", err)
    assert err <= 1e-7


def test_solve_box192(hk, oracle):
    c = configs.box192()
    say("solve box192 tol 1e-8")
    A = make_csr(hk, c["rowptr"], c["col"], c["val"], autotune=True)
    x, info = hk.krylov_solve(A, dev(c["g"]), tol=1e-8)
    say("box192", info)
    assert info["status"] == hk.HK_OK, info
    r = oracle.residual(c["rowptr"], c["col"], c["val"], c["g"], host(x))
    assert np.linalg.norm(r) / np.linalg.norm(c["g"]) <= 1.05e-8


GOLDEN_BOX192 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "box192_oracle_solution.txt")


def box192_golden():
    """Sampled rows of the oracle's FP64 solution of the 192x96x96 system
    (tests/golden/make_box192_solution.py: oracle BiCGStab to 1e-12)."""
    idx, ref = [], []
    with open(GOLDEN_BOX192) as fh:
        for line in fh:
            t = line.split()
            if t and t[0] == "x":
                idx.append(int(t[1]))
                ref.append(complex(float(t[2]), float(t[3])))
    return np.array(idx), np.array(ref)


@pytest.mark.parametrize("literal", [False, True], ids=["clamped", "literal"])
def test_mixed_box192(hk, oracle, literal):
    """The mixed-precision workload at its own size: 192x96x96 system, complex64
    inner BiCGStab to 1e-4 (with and without the last cycle's clamp), complex128
    outer loop to 1e-10.  The oracle recomputes the true residual (<= 1.05e-10),
    and the solution is within 1e-7 of the oracle's FP64 solution on its 4,098
    sampled rows."""
    c = configs.box192()
    idx, ref = box192_golden()
    A = make_csr(hk, c["rowptr"], c["col"], c["val"], autotune=True)
    say("mixed box192 inner 1e-4 outer 1e-10", "literal" if literal else "clamped")
    x, info = hk.krylov_solve_mixed(A, dev(c["g"]), inner_tol=1e-4, outer_tol=1e-10, literal_inner=literal)
    say("mixed box192", info)
    assert info["status"] == hk.HK_OK, info
    xh = host(x)
    r = oracle.residual(c["rowptr"], c["col"], c["val"], c["g"], xh)
    rel = np.linalg.norm(r) / np.linalg.norm(c["g"])
    err = np.linalg.norm(xh[idx] - ref) / np.linalg.norm(ref)
    say("mixed box192 true relres", rel, "err vs fp64 oracle", err)
    assert rel <= 1.05e-10
    assert err <= 1e-7


def test_solve_box192_wide_workgroup_shapes(hk, oracle):
    """The fused products of the 1.8M-row solve in row-block shapes whose
    workgroups widen to stay under the workgroup cap (64-row blocks: 4 waves;
    16-row blocks: 8 waves and a grid-stride walk); 6 iterations each give
    the same iterate as the oracle to rounding.  (On this indefinite system
    iterates from different summation orders separate quickly: numpy vs the
    oracle differ by 6e-14 after 6 iterations, 8e-13 after 8, 2e-9 after 10
    and 0.44 after 20.)"""
    c = configs.box192()
    A = make_csr(hk, c["rowptr"], c["col"], c["val"])
    g = dev(c["g"])
    xo, _ = oracle.bicgstab(c["rowptr"], c["col"], c["val"], c["g"], tol=1e-14, maxit=6)
    for plan in ((64, 32, 0), (64, 64, 0), (64, 16, 0), (16, 1, 0)):
        say("box192 6 iterations, plan", plan)
        A.set_plan(*plan)
        x, info = hk.krylov_solve(A, g, tol=1e-14, max_iter=6)
        assert info["iters"] == 6 and info["status"] == hk.HK_NOT_CONVERGED, info
        assert np.linalg.norm(host(x) - xo) <= 1e-10 * np.linalg.norm(xo), plan


def test_solvers_same_bits_from_either_column_stream(hk):
    """The three methods give the same iterate bits whether the row-block
    products stream 16-bit column offsets or int32 indices (same shape on
    both handles)."""
    rowptr, col, val = small_mesh_problem((9, 8, 7), 6)
    n = rowptr.shape[0] - 1
    b = dev(crandn(np.random.default_rng(9), n))
    for method in ("bicgstab", "tfqmr", "bicgstab_l"):
        xs = []
        for compact in (True, False):
            say("solver column streams", method, "compact", compact)
            A = hk.CSR(dev(rowptr), dev(col), dev(val), compact_cols=compact)
            A.set_plan(64, 32, 0)
            x, info = hk.krylov_solve(A, b, tol=1e-12, max_iter=25, method=method, ell=4)
            xs.append((host(x), info["iters"], info["relres_rec"]))
        assert xs[0][1:] == xs[1][1:] and np.array_equal(xs[0][0], xs[1][0]), method


def test_solver_plans_random_structure(hk, oracle):
    """The solvers' fused products on an unstructured, diagonally dominant
    matrix whose rows hold 1 to 301 entries (a 64-row block spans many passes,
    rows and blocks start at odd entries), in a spread of fixed shapes and
    both entry layouts: two BiCGStab and two TFQMR steps and one BiCGStab(2)
    cycle in complex128, one BiCGStab step in complex64, give the oracle's
    iterate."""
    rng = np.random.default_rng(42)
    n = 1500
    cols, vals = [], []
    rowptr = np.zeros(n + 1, dtype=np.int32)
    for i in range(n):
        k = int(rng.integers(0, 301))
        off = rng.choice(np.delete(np.arange(n), i), size=k, replace=False)
        c = np.sort(np.append(off, i))
        v = crandn(rng, k + 1) * 0.1
        v[c == i] = (np.abs(v).sum() + 1.0) * (1 + 0.1j)
        cols.append(c)
        vals.append(v)
        rowptr[i + 1] = rowptr[i] + k + 1
    col = np.concatenate(cols).astype(np.int32)
    val = np.concatenate(vals)
    assert col.shape[0] % 2 == 1  # the paired layout's last pass reads the padding entry
    b = crandn(rng, n)
    ref = {"bicgstab": oracle.bicgstab(rowptr, col, val, b, tol=1e-14, maxit=2)[0],
           "tfqmr": oracle.tfqmr(rowptr, col, val, b, tol=1e-14, maxit=2)[0],
           "bicgstab_l": oracle.bicgstab_l(rowptr, col, val, b, ell=2, tol=1e-14, maxit=1)[0]}
    b32, v32 = b.astype(np.complex64), val.astype(np.complex64)
    ref64 = oracle.bicgstab_c64(rowptr, col, v32, b32, tol=1e-9, maxit=1)[0]
    A = make_csr(hk, rowptr, col, val)
    A32 = make_csr(hk, rowptr, col, v32)
    assert A.info()["col_bytes"] == 2
    for rw, nw in ((16, 8), (32, 2), (64, 2), (64, 8)):
        for paired in (False, True):
            for grid in (0, 3):
                say("solver plan random", rw, nw, "paired" if paired else "lanes", grid)
                A.set_solver_plan(rw, nw, grid, paired)
                for method, its in (("bicgstab", 2), ("tfqmr", 2), ("bicgstab_l", 1)):
                    x, info = hk.krylov_solve(A, dev(b), tol=1e-14, max_iter=its, method=method, ell=2)
                    assert info["iters"] == its, (method, info)
                    xo = ref[method]
                    assert np.linalg.norm(host(x) - xo) <= 1e-10 * np.linalg.norm(xo), (method, rw, nw, paired, grid)
                A32.set_solver_plan(rw, nw, grid, paired)
                x, info = hk.krylov_solve(A32, dev(b32), tol=1e-9, max_iter=1)
                assert info["iters"] == 1
                assert np.linalg.norm(host(x) - ref64) <= 1e-6 * np.linalg.norm(ref64), (rw, nw, paired, grid)


def test_solver_plans_every_shape(hk, oracle):
    """Every fixed shape of the solvers' fused products (16/32/64 rows per
    wave, 2/4/8 waves, lane-per-entry and paired layouts, one workgroup per
    tile and a 3-workgroup grid stride) gives the oracle's iterate: two
    BiCGStab and two TFQMR steps and one BiCGStab(2) cycle in complex128,
    one BiCGStab step in complex64.  The matrix has an odd entry count, so
    the paired layout's last pass reads the padding entry, and its blocks
    start at odd entries."""
    rowptr, col, val = small_mesh_problem((8, 6, 4), 3)
    n = rowptr.shape[0] - 1
    assert col.shape[0] % 2 == 1 and np.any(rowptr[::16] % 2 == 1)
    rng = np.random.default_rng(31)
    b = crandn(rng, n)
    b32 = b.astype(np.complex64)
    v32 = val.astype(np.complex64)
    ref = {"bicgstab": oracle.bicgstab(rowptr, col, val, b, tol=1e-14, maxit=2)[0],
           "tfqmr": oracle.tfqmr(rowptr, col, val, b, tol=1e-14, maxit=2)[0],
           "bicgstab_l": oracle.bicgstab_l(rowptr, col, val, b, ell=2, tol=1e-14, maxit=1)[0]}
    ref64 = oracle.bicgstab_c64(rowptr, col, v32, b32, tol=1e-9, maxit=1)[0]
    A = make_csr(hk, rowptr, col, val)
    A32 = make_csr(hk, rowptr, col, v32)
    for rw in (16, 32, 64):
        for nw in (2, 4, 8):
            for paired in (False, True):
                for grid in (0, 3):
                    say("solver plan", rw, nw, "paired" if paired else "lanes", grid)
                    A.set_solver_plan(rw, nw, grid, paired)
                    for method, its in (("bicgstab", 2), ("tfqmr", 2), ("bicgstab_l", 1)):
                        x, info = hk.krylov_solve(A, dev(b), tol=1e-14, max_iter=its, method=method, ell=2)
                        assert info["iters"] == its, (method, info)
                        xo = ref[method]
                        assert np.linalg.norm(host(x) - xo) <= 1e-10 * np.linalg.norm(xo), (method, rw, nw, paired, grid)
                    A32.set_solver_plan(rw, nw, grid, paired)
                    x, info = hk.krylov_solve(A32, dev(b32), tol=1e-9, max_iter=1)
                    assert info["iters"] == 1
                    assert np.linalg.norm(host(x) - ref64) <= 1e-6 * np.linalg.norm(ref64), (rw, nw, paired, grid)
    for bad in ((8, 4, 0, False), (32, 3, 0, False), (32, 4, -1, False)):
        with pytest.raises(hk.HKError):
            A.set_solver_plan(*bad)
    Ai = hk.CSR(dev(rowptr), dev(col), dev(val), compact_cols=False)
    with pytest.raises(hk.HKError):
        Ai.set_solver_plan(32, 4, 0, True)
    Ai.set_solver_plan(32, 4, 0, False)
    x, info = hk.krylov_solve(Ai, dev(b), tol=1e-14, max_iter=2)
    assert np.linalg.norm(host(x) - ref["bicgstab"]) <= 1e-10 * np.linalg.norm(ref["bicgstab"])
