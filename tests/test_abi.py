"""The C-ABI library loads and exports what include/hk.h declares (CPU only).

No compute is launched: only calls that fail argument validation before any
HIP call are made.
"""
import ctypes as C
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hk.h")
LIB = os.path.join(ROOT, "paper_2112_11880_amd", "libhk.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hk_[a-z0-9_]+)\s*\(", txt)))


def exported():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    return {l.split()[-1] for l in out.splitlines() if " T " in l}


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libhk.so is not built; run __graft_entry__.build()")
    from paper_2112_11880_amd import hk
    return hk.load(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 17
    missing = [n for n in names if n not in exported()]
    assert not missing, missing


def test_binding_declares_every_symbol(lib):
    from paper_2112_11880_amd import hk
    assert sorted(hk.SIGNATURES) == declared()


def test_argument_errors_without_device(lib):
    from paper_2112_11880_amd import hk
    assert lib.hk_csr_destroy(None) == hk.HK_OK
    assert lib.hk_spmv(None, None, None, None, None, None) == hk.HK_EINVAL
    assert b"hk_spmv" in lib.hk_last_error()
    assert lib.hk_zdotc(0, None, None, None, None) == hk.HK_EINVAL
    assert lib.hk_zaxpy(-1, None, None, None, None) == hk.HK_EINVAL
    assert lib.hk_zaxpy(0, (C.c_double * 2)(1, 0), None, None, None) == hk.HK_OK
    h = C.c_void_p()
    assert lib.hk_csr_create(C.byref(h), 0, 0, None, None, None, 0, 0, None) == hk.HK_EINVAL
    assert lib.hk_csr_create(C.byref(h), 10, 5, None, None, None, 0, 0, None) == hk.HK_EINVAL
    info = hk.SolveInfo()
    assert lib.hk_krylov_solve(None, None, None, None, C.byref(info), None) == hk.HK_EINVAL


def test_library_has_no_oracle_dependency():
    """The product library must not link or name the CPU oracle."""
    out = subprocess.run(["nm", "-D", LIB], capture_output=True, text=True, check=True).stdout
    assert "orc_" not in out
    src = os.path.join(ROOT, "paper_2112_11880_amd")
    for dirpath, _, files in os.walk(src):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


def test_binding_rejects_host_tensors(lib):
    """The binding refuses host memory instead of silently computing on the CPU."""
    import torch
    from paper_2112_11880_amd import hk
    x = torch.zeros(8, dtype=torch.complex128)
    for f in (lambda: hk.zdotc(x, x), lambda: hk.dznrm2(x), lambda: hk.zaxpy(1.0, x, x),
              lambda: hk.CSR(torch.zeros(9, dtype=torch.int32), torch.zeros(0, dtype=torch.int32),
                             torch.zeros(0, dtype=torch.complex128))):
        with pytest.raises(hk.HKError):
            f()


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
