"""GPU parity of the speed-dependent operator and the adjoint gradients.

* A(c) assembled by the library equals the oracle's element assembly
  (1e-13 relative, max norm).
* Small problem: the autograd gradient (forward + adjoint BiCGStab to 1e-12
  on the GPU) matches the oracle's adjoint gradient to 1e-8 relative and
  central finite differences (GPU solves, step 1e-6 relative) to 1e-5.
* Full 48^3 / 216-block problem: grad_c and sampled grad_g match the stored
  oracle gradient (tests/golden/adjoint48_oracle_gradient.txt) to 1e-8.
"""
import math
import os
import sys

import numpy as np
import pytest

from synth import helmholtz as H
from synth import configs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint48_oracle_gradient.txt")


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


def make_problem(hk, d):
    return hk.HelmholtzProblem(
        rowptr=dev(d["rowptr"]), col=dev(d["col"]), K=dev(d["K"]), bm_ptr=dev(d["bm_ptr"]),
        bm_blk=dev(d["bm_blk"]), bm_val=dev(d["bm_val"]), tet_nodes=dev(d["tet_nodes"]),
        tet_ptr=dev(d["tet_ptr"]), tet_vol=dev(d["tet_vol"]),
        dirichlet=dev(d["dirichlet"].astype(np.uint8)), omega=float(d["omega"]))


def small(nc=6, bs=3, seed=4):
    m = H.make_mesh(nc, nc, nc, 1.0 / nc, jitter=0.2, rng=np.random.default_rng(seed))
    p = H.build_problem(m)
    nb = (nc // bs) ** 3
    c = np.random.default_rng(seed + 1).uniform(300, 400, nb)
    bm_ptr, bm_blk, bm_val = H.block_mass_lists(p, bs)
    tn, tb, tv, tp = H.tets_by_block(m, bs)
    g = (np.random.default_rng(seed + 2).standard_normal(p.n)
         + 1j * np.random.default_rng(seed + 3).standard_normal(p.n))
    g[p.dirichlet] = 0
    S = np.flatnonzero(~p.dirichlet)[::7]
    return {"rowptr": p.rowptr, "col": p.col, "K": p.K, "dirichlet": p.dirichlet, "bm_ptr": bm_ptr,
            "bm_blk": bm_blk, "bm_val": bm_val, "tet_nodes": tn, "tet_block": tb, "tet_vol": tv,
            "tet_ptr": tp, "coords": m.coords, "c": c, "omega": 2 * math.pi * c.min() / (10 * m.h),
            "g": g, "samples": S, "n": p.n}


def gpu_grad(hk, prob, d, tol):
    g = dev(d["g"]).requires_grad_(True)
    c = dev(d["c"]).requires_grad_(True)
    u = hk.helmholtz_solve(g, c, prob, tol=tol)
    S = dev(d["samples"].astype(np.int64))
    L = (u[S].abs() ** 2).sum()
    L.backward()
    torch.cuda.synchronize()
    return L.item(), g.grad.cpu().numpy(), c.grad.cpu().numpy()


def test_assembly_matches_oracle(hk, oracle):
    d = small()
    prob = make_problem(hk, d)
    say("assemble small")
    val = hk.assemble(prob, dev(d["c"])).cpu().numpy()
    ref = oracle.assemble_helmholtz(d["rowptr"], d["col"], d["K"], d["dirichlet"], d["tet_nodes"],
                                    d["tet_block"], d["coords"], d["c"], d["omega"])
    assert np.max(np.abs(val - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_adjoint_small_vs_oracle_and_fd(hk, oracle):
    d = small()
    prob = make_problem(hk, d)
    say("adjoint small")
    L, gg, gc = gpu_grad(hk, prob, d, 1e-12)
    val = oracle.assemble_helmholtz(d["rowptr"], d["col"], d["K"], d["dirichlet"], d["tet_nodes"],
                                    d["tet_block"], d["coords"], d["c"], d["omega"])
    Lo, ggo, gco, _, _ = oracle.adjoint_gradients(d["rowptr"], d["col"], val, d["g"], d["samples"],
                                                  d["tet_nodes"], d["tet_block"], d["coords"],
                                                  d["dirichlet"], d["c"], d["omega"], tol=1e-12)
    assert abs(L - Lo) <= 1e-9 * Lo
    assert np.linalg.norm(gg - ggo) <= 1e-8 * np.linalg.norm(ggo)
    assert np.linalg.norm(gc - gco) <= 1e-8 * np.linalg.norm(gco)

    def loss(cc, gvec):
        with torch.no_grad():
            u = hk.helmholtz_solve(dev(gvec), dev(cc), prob, tol=1e-13)
            return float((u[dev(d["samples"].astype(np.int64))].abs() ** 2).sum().item())

    rng = np.random.default_rng(3)
    for b in rng.choice(d["c"].shape[0], 3, replace=False):
        say("fd block", b)
        h = 1e-6 * d["c"][b]
        cp, cm = d["c"].copy(), d["c"].copy()
        cp[b] += h
        cm[b] -= h
        fd = (loss(cp, d["g"]) - loss(cm, d["g"])) / (2 * h)
        assert abs(fd - gc[b]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(gc).max())
    for _ in range(2):
        say("fd direction")
        v = rng.standard_normal(d["n"]) + 1j * rng.standard_normal(d["n"])
        v[d["dirichlet"]] = 0
        v /= np.linalg.norm(v)
        h = 1e-6 * np.linalg.norm(d["g"])
        fd = (loss(d["c"], d["g"] + h * v) - loss(d["c"], d["g"] - h * v)) / (2 * h)
        assert abs(fd - np.real(np.vdot(gg, v))) <= 1e-6 * np.linalg.norm(gg)


def read_golden():
    L, gc, gg = None, {}, {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#"):
                continue
            t = line.split()
            if t[0] == "L":
                L = float(t[1])
            elif t[0] == "grad_c":
                gc[int(t[1])] = float(t[2])
            elif t[0] == "grad_g":
                gg[int(t[1])] = complex(float(t[2]), float(t[3]))
    return L, gc, gg


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="golden oracle gradient not generated")
def test_adjoint_adjoint48_full(hk):
    d = configs.adjoint48()
    prob = make_problem(hk, d)
    say("adjoint adjoint48")
    L, gg, gc = gpu_grad(hk, prob, d, 1e-12)
    Lo, gco, ggo = read_golden()
    assert abs(L - Lo) <= 1e-8 * Lo
    gco = np.array([gco[b] for b in range(len(gco))])
    assert np.linalg.norm(gc - gco) <= 1e-8 * np.linalg.norm(gco)
    idx = np.array(sorted(ggo))
    ref = np.array([ggo[i] for i in idx])
    assert np.linalg.norm(gg[idx] - ref) <= 1e-8 * np.linalg.norm(ref)
