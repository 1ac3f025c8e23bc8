"""GPU parity on Q1 hexahedral systems (27-point rows, the row length of the
paper's car-cavity matrices).  Bounds as in tests/test_gpu_core.py."""
import math
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from synth import helmholtz as H
from synth import hexahedra as Q
from synth import configs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SHAPES = ([(L, U, g) for L in (4, 8, 16, 32) for U in (1, 2, 4, 8) for g in (0, 3) if U <= L]
          + [(64, rw, g) for rw in (16, 32, 64) for g in (0, 3)])


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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def crandn(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def spmv_bound(rowptr, col, val, x):
    n = rowptr.shape[0] - 1
    return sp.csr_matrix((np.abs(val), col, rowptr), shape=(n, n)) @ np.abs(x)


def hex_problem(ns, seed=1):
    m = H.make_mesh(ns, ns, ns, 1.0 / ns, jitter=0.2, rng=np.random.default_rng(seed))
    p = Q.build_hex_problem(m)
    k = 2 * math.pi / (10 * m.h)
    val = H.helmholtz_values(p, complex(k * k, 0.01 * k * k))
    g = H.complex_rhs(np.random.default_rng(0), p.n, p.dirichlet)
    return p.rowptr, p.col, val, g


def test_hex_spmv_every_shape(hk, oracle):
    rowptr, col, val, _ = hex_problem(7, 3)
    n = rowptr.shape[0] - 1
    x = crandn(np.random.default_rng(1), n)
    ref = oracle.spmv(rowptr, col, val, x)
    bound = 1e-12 * spmv_bound(rowptr, col, val, x)
    A = hk.CSR(dev(rowptr), dev(col), dev(val))
    xd = dev(x)
    for L, U, g in SHAPES:
        say("hex spmv shape", L, U, g, "n", n)
        A.set_plan(L, U, g)
        y = host(A.spmv(xd, torch.full_like(xd, complex("nan+nanj")), beta=0.0))
        assert np.all(np.abs(y - ref) <= bound), (L, U, g)


def test_hex86_spmv_full(hk, oracle):
    """The 658,503-row / 17.2M-nnz matrix, every row, in the tuned shape."""
    c = configs.hex_box()
    n = int(c["n"])
    x = crandn(np.random.default_rng(6), n)
    ref = oracle.spmv(c["rowptr"], c["col"], c["val"], x)
    bound = 1e-12 * spmv_bound(c["rowptr"], c["col"], c["val"], x)
    A = hk.CSR(dev(c["rowptr"]), dev(c["col"]), dev(c["val"]), autotune=True)
    say("hex86 spmv", n, A.plan())
    y = host(A.spmv(dev(x)))
    assert np.all(np.abs(y - ref) <= bound)


@pytest.mark.parametrize("method", ["bicgstab", "tfqmr"])
def test_hex_solve_matches_oracle(hk, oracle, method):
    rowptr, col, val, g = hex_problem(16)
    A = hk.CSR(dev(rowptr), dev(col), dev(val), autotune=True)
    say("hex 16^3", method, "tol 1e-8")
    x, info = hk.krylov_solve(A, dev(g), tol=1e-8, method=method)
    solve = oracle.tfqmr if method == "tfqmr" else oracle.bicgstab
    xo, oi = solve(rowptr, col, val, g, tol=1e-8)
    say("gpu", info, "oracle", oi)
    assert info["status"] == hk.HK_OK and oi["status"] == 0
    r = oracle.residual(rowptr, col, val, g, host(x))
    assert np.linalg.norm(r) / np.linalg.norm(g) <= 1.05e-8
    assert abs(info["iters"] - oi["iters"]) <= max(10, 0.25 * oi["iters"])
    say("hex 16^3", method, "tol 1e-11 vs the oracle solution")
    x, info = hk.krylov_solve(A, dev(g), tol=1e-11, method=method)
    xs, _ = oracle.bicgstab(rowptr, col, val, g, tol=1e-12)
    assert info["status"] == hk.HK_OK
    assert np.linalg.norm(host(x) - xs) <= 1e-7 * np.linalg.norm(xs)
