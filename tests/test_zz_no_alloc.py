"""The allocation-free dot (hk_zdotc_noalloc) against hk_zdotc and the oracle.

Both entry points are called through the C ABI (ctypes) on the same device
vectors.  hk_zdotc_noalloc runs the same two kernels with its partials in the
library's static scratch array, so its result must be the same bits as
hk_zdotc's; both must lie within 1e-12 * sum |x_i| |y_i| of the oracle's dot.
Two calls in a row, the second on a smaller input, check that the second call
is not disturbed by what the first left in the shared scratch.
"""
import ctypes as C
import sys

import numpy as np
import pytest

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


def _dot_both(hk, lib, x, y):
    """(noalloc result, hk_zdotc result) as numpy complex, via the C ABI."""
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    r0 = torch.full((1,), complex(np.nan, np.nan), dtype=torch.complex128, device=DEV)
    r1 = torch.full((1,), complex(np.nan, np.nan), dtype=torch.complex128, device=DEV)
    n = x.numel()
    assert lib.hk_zdotc_noalloc(n, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                C.c_void_p(r0.data_ptr()), stream) == hk.HK_OK, lib.hk_last_error()
    assert lib.hk_zdotc(n, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                        C.c_void_p(r1.data_ptr()), stream) == hk.HK_OK, lib.hk_last_error()
    torch.cuda.synchronize()
    return r0.cpu().numpy()[0], r1.cpu().numpy()[0]


def test_noalloc_dot_matches_zdotc_two_calls(hk, oracle):
    lib = hk.load()
    rng = np.random.default_rng(21)
    # first call at the largest partial count (9,000,000 elements: the grid is
    # capped at 4,096 workgroups), then a smaller ragged one (49 workgroups)
    for n in (9_000_000, 100_003):
        say("zdotc_noalloc", "n", n)
        xh = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        yh = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        x, y = torch.from_numpy(xh).to(DEV), torch.from_numpy(yh).to(DEV)
        d0, d1 = _dot_both(hk, lib, x, y)
        assert d0.tobytes() == d1.tobytes(), (n, d0, d1)
        ref = oracle.zdotc(xh, yh)
        bound = 1e-12 * float(np.sum(np.abs(xh) * np.abs(yh)))
        assert abs(d0 - ref) <= bound, (n, d0, ref, bound)


def test_noalloc_dot_edge_cases(hk):
    lib = hk.load()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    say("zdotc_noalloc", "n", 0)
    r = torch.full((1,), complex(5.0, 5.0), dtype=torch.complex128, device=DEV)
    assert lib.hk_zdotc_noalloc(0, None, None, C.c_void_p(r.data_ptr()), stream) == hk.HK_OK
    torch.cuda.synchronize()
    assert r.cpu().numpy()[0] == 0
    say("zdotc_noalloc", "argument errors")
    assert lib.hk_zdotc_noalloc(-1, None, None, C.c_void_p(r.data_ptr()), stream) == hk.HK_EINVAL
    assert lib.hk_zdotc_noalloc((1 << 40) + 1, C.c_void_p(r.data_ptr()), C.c_void_p(r.data_ptr()),
                                C.c_void_p(r.data_ptr()), stream) == hk.HK_EINVAL
    assert b"limit" in lib.hk_last_error()
    # single element and a ragged tail below one workgroup
    rng = np.random.default_rng(22)
    for n in (1, 2049):
        say("zdotc_noalloc", "n", n)
        xh = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        yh = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        d0, d1 = _dot_both(hk, lib, torch.from_numpy(xh).to(DEV), torch.from_numpy(yh).to(DEV))
        assert d0.tobytes() == d1.tobytes(), (n, d0, d1)
