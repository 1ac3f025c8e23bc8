"""GPU parity of the P-TFQMR solve against the CPU oracle.

Bounds as for BiCGStab (tests/test_gpu_core.py): iterates after a few steps
equal the oracle's to rounding; full solves meet the tolerance in the true
residual recomputed by the oracle (the quasi-residual bound that stops the
iteration bounds it).
"""
import sys

import numpy as np
import pytest

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def crandn(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def make_csr(hk, rowptr, col, val, autotune=False):
    return hk.CSR(dev(rowptr), dev(col), dev(val), autotune=autotune)


def small_mesh_problem(nc, seed):
    m = H.make_mesh(*nc, 1.0 / nc[0], jitter=0.2, rng=np.random.default_rng(seed))
    p = H.build_problem(m)
    return p.rowptr, p.col, H.helmholtz_values(p, complex(300.0, 3.0))


SHAPES = ([(L, U, 0) for L in (4, 8, 16, 32) for U in (1, 2, 4, 8) if U <= L]
          + [(16, 2, 3), (64, 32, 3)] + [(64, rw, 0) for rw in (16, 32, 64)])


def test_tfqmr_iterates_every_launch_shape(hk, oracle):
    """1, 2 and 3 iterations in every fused-product shape give the oracle's
    iterate to rounding (the recurrences amplify rounding differences with
    every step on this indefinite system)."""
    rowptr, col, val = small_mesh_problem((5, 5, 5), 11)
    n = rowptr.shape[0] - 1
    b = crandn(np.random.default_rng(3), n)
    A = make_csr(hk, rowptr, col, val)
    ref = {k: oracle.tfqmr(rowptr, col, val, b, tol=1e-15, maxit=k) for k in (1, 2, 3)}
    for L, U, g in SHAPES:
        A.set_plan(L, U, g)
        for k, bound in ((1, 1e-12), (2, 1e-11), (3, 1e-10)):
            say("tfqmr shape", L, U, g, "iterations", k)
            x, info = hk.krylov_solve(A, dev(b), tol=1e-15, max_iter=k, method="tfqmr")
            xo, oi = ref[k]
            assert info["status"] == hk.HK_NOT_CONVERGED and info["iters"] == k, info
            assert np.linalg.norm(host(x) - xo) <= bound * np.linalg.norm(xo), (L, U, g, k)
            assert abs(info["relres_rec"] - oi["relres_rec"]) <= 10 * bound * oi["relres_rec"]


def test_tfqmr_cube16_full_solve(hk, oracle):
    c = configs.cube16()
    A = make_csr(hk, c["rowptr"], c["col"], c["val"], autotune=True)
    say("tfqmr cube16 tol 1e-8")
    x, info, hist = hk.krylov_solve(A, dev(c["g"]), tol=1e-8, method="tfqmr", history=True)
    xo, oi = oracle.tfqmr(c["rowptr"], c["col"], c["val"], c["g"], tol=1e-8)
    say("gpu", info, "oracle", oi)
    assert info["status"] == hk.HK_OK and oi["status"] == 0
    r = oracle.residual(c["rowptr"], c["col"], c["val"], c["g"], host(x))
    assert np.linalg.norm(r) / np.linalg.norm(c["g"]) <= 1.05e-8
    assert abs(info["relres_true"] - np.linalg.norm(r) / np.linalg.norm(c["g"])) <= 1e-12
    # iteration counts depend on the summation order of the dots (see the BiCGStab tests)
    assert abs(info["iters"] - oi["iters"]) <= max(10, 0.25 * oi["iters"])
    h = host(hist)
    assert h.shape[0] == info["iters"] + 1 and abs(h[0] - 1.0) < 1e-12 and h[-1] <= 1e-8
    say("tfqmr cube16 tol 1e-11 vs the oracle solution")
    x, info = hk.krylov_solve(A, dev(c["g"]), tol=1e-11, method="tfqmr")
    xo, _ = oracle.bicgstab(c["rowptr"], c["col"], c["val"], c["g"], tol=1e-12)
    assert info["status"] == hk.HK_OK
    assert np.linalg.norm(host(x) - xo) <= 1e-8 * np.linalg.norm(xo)


def test_tfqmr_breakdown_edges_and_errors(hk, oracle):
    say("tfqmr sigma breakdown")
    A = make_csr(hk, np.array([0, 2, 4], dtype=np.int32), np.array([0, 1, 0, 1], dtype=np.int32),
                 np.array([1.0, -1.25, -1.25, 1.0], dtype=np.complex128))
    x, info = hk.krylov_solve(A, dev(np.array([1.0, 2.0], dtype=np.complex128)), method="tfqmr")
    assert info["status"] == hk.HK_BREAKDOWN and hk.BD_NAMES[info["breakdown"]] == "sigma"
    assert info["iters"] == 0 and np.all(host(x) == 0)
    say("tfqmr diagonal system: one half-step")
    n = 40
    rng = np.random.default_rng(2)
    d = crandn(rng, n) + 3.0
    b = crandn(rng, n)
    A = make_csr(hk, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    x, info = hk.krylov_solve(A, dev(b), tol=1e-12, method="tfqmr")
    assert info["status"] == hk.HK_OK and info["iters"] == 1
    assert np.allclose(host(x), b / d, rtol=1e-14, atol=0)
    c = configs.cube16()
    A = make_csr(hk, c["rowptr"], c["col"], c["val"])
    say("tfqmr zero rhs, nonfinite rhs, cap, warm start")
    x, info = hk.krylov_solve(A, dev(np.zeros_like(c["g"])), method="tfqmr")
    assert info["status"] == hk.HK_OK and info["iters"] == 0
    g = c["g"].copy()
    g[11] = np.inf
    assert hk.krylov_solve(A, dev(g), method="tfqmr")[1]["status"] == hk.HK_NONFINITE
    x, info = hk.krylov_solve(A, dev(c["g"]), max_iter=7, method="tfqmr")
    xo, oi = oracle.tfqmr(c["rowptr"], c["col"], c["val"], c["g"], maxit=7)
    assert info["status"] == hk.HK_NOT_CONVERGED and info["iters"] == 7 == oi["iters"]
    assert np.linalg.norm(host(x) - xo) <= 1e-9 * np.linalg.norm(xo)
    xs, _ = oracle.tfqmr(c["rowptr"], c["col"], c["val"], c["g"], tol=1e-12)
    x, info = hk.krylov_solve(A, dev(c["g"]), x=dev(xs), tol=1e-8, method="tfqmr")
    assert info["status"] == hk.HK_OK and info["iters"] == 0
    with pytest.raises(hk.HKError):
        hk.krylov_solve(A, dev(c["g"]), method="gmres")
    A32 = make_csr(hk, c["rowptr"], c["col"], c["val"].astype(np.complex64))
    with pytest.raises(hk.HKError):
        hk.krylov_solve(A32, dev(c["g"].astype(np.complex64)), method="tfqmr")


def test_tfqmr_box192(hk, oracle):
    """The 1.8M-row system with the tuned fused-product shape, to 1e-8."""
    c = configs.box192()
    A = make_csr(hk, c["rowptr"], c["col"], c["val"], autotune=True)
    say("tfqmr box192 tol 1e-8")
    x, info = hk.krylov_solve(A, dev(c["g"]), tol=1e-8, method="tfqmr")
    say("box192", info)
    assert info["status"] == hk.HK_OK, info
    r = oracle.residual(c["rowptr"], c["col"], c["val"], c["g"], host(x))
    assert np.linalg.norm(r) / np.linalg.norm(c["g"]) <= 1.05e-8
