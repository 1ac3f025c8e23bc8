"""GPU parity of P-BiCGSTAB(l) against the CPU oracle (bounds as for
BiCGStab in tests/test_gpu_core.py)."""
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


def test_bicgstab_l_iterates(hk, oracle):
    """One and two cycles for l = 1, 2, 4, 8 in a lane-group and a row-block
    shape give the oracle's iterate to rounding (which grows with the 2l
    products of a cycle on this indefinite system)."""
    m = H.make_mesh(5, 5, 5, 0.2, jitter=0.2, rng=np.random.default_rng(11))
    p = H.build_problem(m)
    val = H.helmholtz_values(p, complex(300.0, 3.0))
    b = crandn(np.random.default_rng(3), p.n)
    A = make_csr(hk, p.rowptr, p.col, val)
    # measured: <= 6e-15 for l <= 4, 1.2e-13 for l = 8
    for ell, cycles, bound in ((1, 2, 1e-12), (2, 2, 1e-12), (4, 1, 1e-12), (8, 1, 1e-11)):
        ref = {k: oracle.bicgstab_l(p.rowptr, p.col, val, b, ell=ell, tol=1e-15, maxit=k)
               for k in range(1, cycles + 1)}
        for plan in ((16, 2, 0), (64, 32, 0)):
            A.set_plan(*plan)
            for k in range(1, cycles + 1):
                x, info = hk.krylov_solve(A, dev(b), tol=1e-15, max_iter=k, method="bicgstab_l", ell=ell)
                xo, oi = ref[k]
                err = np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)
                say("bicgstab_l", ell, "plan", plan, "cycles", k, "rel err", err)
                assert info["status"] == hk.HK_NOT_CONVERGED and info["iters"] == k, info
                assert err <= bound, (ell, plan, k, err)


@pytest.mark.parametrize("ell", [2, 8])
def test_bicgstab_l_cube16(hk, oracle, ell):
    c = configs.cube16()
    A = make_csr(hk, c["rowptr"], c["col"], c["val"], autotune=True)
    say("bicgstab_l cube16 l", ell)
    x, info, hist = hk.krylov_solve(A, dev(c["g"]), tol=1e-8, method="bicgstab_l", ell=ell, history=True)
    xo, oi = oracle.bicgstab_l(c["rowptr"], c["col"], c["val"], c["g"], ell=ell, tol=1e-8)
    say("gpu", info, "oracle", oi)
    assert info["status"] == hk.HK_OK and oi["status"] == 0
    r = oracle.residual(c["rowptr"], c["col"], c["val"], c["g"], host(x))
    assert np.linalg.norm(r) / np.linalg.norm(c["g"]) <= 1.05e-8
    assert abs(info["iters"] - oi["iters"]) <= max(5, 0.25 * oi["iters"])
    h = host(hist)
    assert h.shape[0] == info["iters"] + 1 and h[-1] <= 1.0001e-8


def test_bicgstab_l_edges_and_errors(hk, oracle):
    n = 40
    rng = np.random.default_rng(2)
    d = crandn(rng, n) + 3.0
    b = crandn(rng, n)
    A = make_csr(hk, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    for ell in (1, 8):
        say("bicgstab_l diagonal l", ell)
        x, info = hk.krylov_solve(A, dev(b), tol=1e-12, method="bicgstab_l", ell=ell)
        assert info["status"] == hk.HK_OK and info["iters"] == 1
        assert np.allclose(host(x), b / d, rtol=1e-14, atol=0)
    say("bicgstab_l sigma breakdown")
    A2 = make_csr(hk, np.array([0, 2, 4], dtype=np.int32), np.array([0, 1, 0, 1], dtype=np.int32),
                  np.array([1.0, -1.25, -1.25, 1.0], dtype=np.complex128))
    x, info = hk.krylov_solve(A2, dev(np.array([1.0, 2.0], dtype=np.complex128)), method="bicgstab_l", ell=4)
    assert info["status"] == hk.HK_BREAKDOWN and hk.BD_NAMES[info["breakdown"]] == "sigma"
    assert info["iters"] == 0 and np.all(host(x) == 0)
    c = configs.cube16()
    A = make_csr(hk, c["rowptr"], c["col"], c["val"])
    for bad in (0, 3, 16):
        with pytest.raises(hk.HKError):
            hk.krylov_solve(A, dev(c["g"]), method="bicgstab_l", ell=bad)
    say("bicgstab_l cap and zero rhs")
    x, info = hk.krylov_solve(A, dev(c["g"]), max_iter=3, method="bicgstab_l", ell=4)
    assert info["status"] == hk.HK_NOT_CONVERGED and info["iters"] == 3
    x, info = hk.krylov_solve(A, dev(np.zeros_like(c["g"])), method="bicgstab_l")
    assert info["status"] == hk.HK_OK and info["iters"] == 0
    A32 = make_csr(hk, c["rowptr"], c["col"], c["val"].astype(np.complex64))
    with pytest.raises(hk.HKError):
        hk.krylov_solve(A32, dev(c["g"].astype(np.complex64)), method="bicgstab_l")


def test_bicgstab_l_box192(hk, oracle):
    c = configs.box192()
    A = make_csr(hk, c["rowptr"], c["col"], c["val"], autotune=True)
    say("bicgstab_l(8) box192 tol 1e-8")
    x, info = hk.krylov_solve(A, dev(c["g"]), tol=1e-8, method="bicgstab_l", ell=8)
    say("box192", info)
    assert info["status"] == hk.HK_OK, info
    r = oracle.residual(c["rowptr"], c["col"], c["val"], c["g"], host(x))
    assert np.linalg.norm(r) / np.linalg.norm(c["g"]) <= 1.05e-8
