"""The five workloads of the Helmholtz Krylov path, built from fixed seeds.

Readings of the workload descriptions (each is listed with its reason in the
design notes):

* "~10 nodes per wavelength" -> k = 2*pi / (10 h); with a variable speed,
  omega = 2*pi*c_min / (10 h) with c_min the realised minimum block speed, so
  the shortest local wavelength is exactly 10 h.
* 1% damping -> k^2 (1 + 0.01 i) (or omega^2 (1 + 0.01 i) with M weighted by c^-2).
* Jitter: +-20% h uniform from ``default_rng(1)``, normal component zeroed on
  boundary nodes; block speeds are drawn from the same generator afterwards.
* Right-hand side g = (N + iN)/sqrt(2) from ``default_rng(0)``, g_D = 0.
* Uneven batch: cube sizes ``default_rng(2).integers(8, 49, 32)``, unjittered,
  k = 2*pi*n_s/10, right-hand sides from the same generator afterwards.
* Frequency sweep: k_j = linspace(0.5 k0, 1.5 k0, 64) on the 48^3 mesh, c = 340.
* Sample nodes of the differentiable loss: ``default_rng(5).choice`` of 256
  distinct non-Dirichlet nodes.
"""
from __future__ import annotations

import math
import os

import numpy as np

from .helmholtz import (make_mesh, build_problem, helmholtz_values, complex_rhs,
                        cell_blocks, block_mass_lists, tets_by_block)

DAMP = 0.01
C_CONST = 340.0


def _cache_dir():
    d = os.environ.get("HK_SYNTH_CACHE", "/tmp/hk_synth_cache")
    os.makedirs(d, exist_ok=True)
    return d


def _cached(name, fn):
    path = os.path.join(_cache_dir(), name + ".npz")
    if os.path.exists(path):
        try:
            with np.load(path, allow_pickle=False) as z:
                return {k: z[k] for k in z.files}
        except Exception:
            pass
    out = fn()
    tmp = path + f".tmp{os.getpid()}.npz"
    np.savez(tmp, **out)
    os.replace(tmp, path)
    return out


def cube(ns, jitter=0.0, seed_jitter=1, extent=(1.0, 1.0, 1.0), cells=None):
    """Mesh + FE problem on a box of ``cells`` (default ns^3) cubes of edge 1/ns."""
    nx, ny, nz = cells if cells is not None else (ns, ns, ns)
    h = extent[0] / nx
    rng = np.random.default_rng(seed_jitter) if jitter else None
    m = make_mesh(nx, ny, nz, h, jitter=jitter, rng=rng)
    return m, rng


def _pack(p, kappa2, g, extra=None):
    out = {
        "n": np.int64(p.n), "rowptr": p.rowptr, "col": p.col,
        "K": p.K, "M": p.M, "dirichlet": p.dirichlet,
        "kappa2": np.array([kappa2.real, kappa2.imag]),
        "val": helmholtz_values(p, kappa2), "g": g,
        "dims": np.array([p.mesh.nx, p.mesh.ny, p.mesh.nz]), "h": np.float64(p.mesh.h),
    }
    if extra:
        out.update(extra)
    return out


def cube16():
    """16^3 unit cube, constant c = 340, unjittered (4,913 nodes)."""
    def make():
        m, _ = cube(16)
        p = build_problem(m)
        k = 2 * math.pi / (10 * m.h)
        g = complex_rhs(np.random.default_rng(0), p.n, p.dirichlet)
        return _pack(p, complex(k * k, DAMP * k * k), g, {"k": np.float64(k)})
    return _cached("cube16", make)


def _variable_speed(m, rng, bs):
    (nbx, nby, nbz), blk = cell_blocks(m, bs)
    c = rng.uniform(300.0, 400.0, size=nbx * nby * nbz)
    omega = 2 * math.pi * c.min() / (10 * m.h)
    return c, blk, omega


def box192():
    """2:1:1 box, 192x96x96 cells, jittered, 8^3-cell speed blocks (1,815,937 nodes)."""
    def make():
        m, rng = cube(96, jitter=0.2, extent=(2.0, 1.0, 1.0), cells=(192, 96, 96))
        c, blk, omega = _variable_speed(m, rng, 8)
        p = build_problem(m, cell_weight=lambda I, J, K: 1.0 / c[blk(I, J, K)] ** 2)
        g = complex_rhs(np.random.default_rng(0), p.n, p.dirichlet)
        return _pack(p, complex(omega ** 2, DAMP * omega ** 2), g,
                     {"c": c, "omega": np.float64(omega)})
    return _cached("box192", make)


def hex_box(cells=86):
    """Q1 hexahedra (27-point rows) on a jittered unit cube of ``cells``^3,
    c = 340, k = 2*pi/(10 h), 1% damping: the row structure of the paper's
    car-cavity matrices (86^3: 658,503 nodes, 17.2M nonzeros, up to 27 per
    row, against Audi3D-4's 648,849 and 15.4M)."""
    from .hexahedra import build_hex_problem

    def make():
        m, _ = cube(cells, jitter=0.2)
        p = build_hex_problem(m)
        k = 2 * math.pi / (10 * m.h)
        g = complex_rhs(np.random.default_rng(0), p.n, p.dirichlet)
        return _pack(p, complex(k * k, DAMP * k * k), g)
    return _cached(f"hex_box{cells}", make)


def mesh48():
    m, rng = cube(48, jitter=0.2)
    return m, rng


def sweep48(nfreq=64):
    """Frequency sweep: 48^3 jittered mesh, c = 340, k_j over [0.5 k0, 1.5 k0]."""
    def make():
        m, _ = mesh48()
        p = build_problem(m)
        k0 = 2 * math.pi / (10 * m.h)
        ks = np.linspace(0.5 * k0, 1.5 * k0, nfreq)
        g = complex_rhs(np.random.default_rng(0), p.n, p.dirichlet)
        return {"n": np.int64(p.n), "rowptr": p.rowptr, "col": p.col, "K": p.K, "M": p.M,
                "dirichlet": p.dirichlet, "ks": ks,
                "kappa2": np.stack([ks ** 2, DAMP * ks ** 2], 1), "g": g,
                "dims": np.array([48, 48, 48]), "h": np.float64(m.h)}
    return _cached(f"sweep48_{nfreq}", make)


def uneven_sizes(nsys=32):
    rng = np.random.default_rng(2)
    return rng.integers(8, 49, nsys), rng


def uneven(nsys=32):
    """Uneven batch: nsys unjittered cubes with n_s from default_rng(2)."""
    def make():
        sizes, rng = uneven_sizes(nsys)
        out = {"sizes": sizes}
        for s, ns in enumerate(sizes):
            m, _ = cube(int(ns))
            p = build_problem(m)
            k = 2 * math.pi * int(ns) / 10
            g = complex_rhs(rng, p.n, p.dirichlet)
            for key, v in _pack(p, complex(k * k, DAMP * k * k), g).items():
                out[f"s{s}_{key}"] = v
        return out
    return _cached(f"uneven_{nsys}", make)


def uneven_systems(nsys=32):
    z = uneven(nsys)
    return [{k[len(f"s{s}_"):]: v for k, v in z.items() if k.startswith(f"s{s}_")}
            for s in range(len(z["sizes"]))]


def adjoint48():
    """Differentiable case: 48^3 jittered mesh, 216 speed blocks, 256 sample nodes."""
    def make():
        m, rng = mesh48()
        c, blk, omega = _variable_speed(m, rng, 8)
        p = build_problem(m, cell_weight=lambda I, J, K: 1.0 / c[blk(I, J, K)] ** 2)
        q = build_problem(m)  # unweighted M and the same K / pattern
        bm_ptr, bm_blk, bm_val = block_mass_lists(q, 8)
        tnodes, tblk, tvol, tptr = tets_by_block(m, 8)
        g = complex_rhs(np.random.default_rng(0), p.n, p.dirichlet)
        free = np.flatnonzero(~p.dirichlet)
        S = np.sort(np.random.default_rng(5).choice(free, 256, replace=False))
        out = _pack(p, complex(omega ** 2, DAMP * omega ** 2), g,
                    {"c": c, "omega": np.float64(omega), "coords": m.coords,
                     "bm_ptr": bm_ptr, "bm_blk": bm_blk, "bm_val": bm_val,
                     "tet_nodes": tnodes, "tet_block": tblk, "tet_vol": tvol,
                     "tet_ptr": tptr, "samples": S})
        return out
    return _cached("adjoint48", make)
