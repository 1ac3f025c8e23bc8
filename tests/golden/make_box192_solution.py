"""Write a sample of the CPU oracle's FP64 solution of the 192x96x96 system.

Calls only the input generator (synth/) and the CPU oracle (oracle/).  The
system is the jittered 192x96x96-cell P1 Helmholtz problem with 3,456
speed blocks (1,815,937 rows, 26,606,015 entries); the oracle's Jacobi
BiCGStab solves it in double precision to a relative residual of 1e-12.  The
stored values are the reference of the mixed-precision refinement's accuracy
check: the solution's 2-norm and its entries at 4,096 seeded rows (plus the
first and last row), with the solve's record.
Run:  python tests/golden/make_box192_solution.py   (about an hour on 8 cores)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from synth import configs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "box192_oracle_solution.txt")
TOL = 1e-12
NSAMPLE = 4096


def main():
    c = configs.box192()
    n = int(c["n"])
    t0 = time.time()
    x, info = oracle.bicgstab(c["rowptr"], c["col"], c["val"], c["g"], tol=TOL, maxit=400000)
    took = time.time() - t0
    if info["status"] != oracle.OK:
        raise SystemExit(f"oracle solve did not converge: {info}")
    idx = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(77).choice(n, NSAMPLE, replace=False)]))
    with open(OUT, "w") as f:
        f.write("# CPU-oracle FP64 solution, jittered 192x96x96 P1 Helmholtz box, 3,456 speed blocks\n")
        f.write("# written by tests/golden/make_box192_solution.py (oracle/ + synth/ only)\n")
        f.write(f"# Jacobi BiCGStab to {TOL:g}: {info}, {took:.0f} s\n")
        f.write(f"n {n}\n")
        f.write(f"relres_true {float(info['relres_true'])!r}\n")
        f.write(f"norm {float(np.linalg.norm(x))!r}\n")
        for i in idx:
            f.write(f"x {int(i)} {float(x[i].real)!r} {float(x[i].imag)!r}\n")
    print("wrote", OUT, info, f"{took:.0f} s")


if __name__ == "__main__":
    main()
