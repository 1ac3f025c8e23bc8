"""Write the CPU oracle's adjoint gradient for the 48^3, 216-block problem.

Calls only the input generator (synth/) and the CPU oracle (oracle/).  The
stored values are the expected results of the GPU adjoint test at full size:
loss L = sum over the 256 sample nodes of |u_i|^2, u = A(c)^-1 g, solved to a
relative residual of 1e-12; grad_c (dL/dc_b, 216 blocks) and grad_g
(dL/dRe g + i dL/dIm g) at the sample nodes and 64 further seeded nodes.
Run:  python tests/golden/make_adjoint48_gradient.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from synth import configs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint48_oracle_gradient.txt")


def main():
    c = configs.adjoint48()
    t0 = time.time()
    val = oracle.assemble_helmholtz(c["rowptr"], c["col"], c["K"], c["dirichlet"], c["tet_nodes"],
                                    c["tet_block"], c["coords"], c["c"], float(c["omega"]))
    L, gg, gc, u, infos = oracle.adjoint_gradients(c["rowptr"], c["col"], val, c["g"], c["samples"],
                                                   c["tet_nodes"], c["tet_block"], c["coords"],
                                                   c["dirichlet"], c["c"], float(c["omega"]), tol=1e-12)
    extra = np.sort(np.random.default_rng(55).choice(int(c["n"]), 64, replace=False))
    idx = np.unique(np.concatenate([c["samples"], extra]))
    with open(OUT, "w") as f:
        f.write("# CPU-oracle adjoint gradient, 48^3 jittered P1 Helmholtz mesh, 216 speed blocks\n")
        f.write("# written by tests/golden/make_adjoint48_gradient.py (oracle/ + synth/ only)\n")
        f.write(f"# forward solve {infos[0]}, adjoint solve {infos[1]}, {time.time() - t0:.0f} s\n")
        f.write(f"L {float(L)!r}\n")
        for b, v in enumerate(gc):
            f.write(f"grad_c {b} {float(v)!r}\n")
        for i in idx:
            f.write(f"grad_g {int(i)} {float(gg[i].real)!r} {float(gg[i].imag)!r}\n")
    print("wrote", OUT, infos)


if __name__ == "__main__":
    main()
