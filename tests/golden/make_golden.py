"""Writes the stored oracle results that the GPU parity tests compare with.

Runs only the CPU oracle (oracle/) on the seeded workloads of lattice_inputs;
nothing here touches the GPU library.  Usage:
    python tests/golden/make_golden.py [lattice32] [lattice256] [lattice2048]
                                       [lattice2048corner] [continuum70] [delta100]

Each JSON file holds the workload name, the number of steps, the Newton
tolerance (and whether it is relative to ||u_0||_inf), the oracle's stage solver, the site indices compared (all sites,
or a fixed sample for the large lattices), Re/Im of psi there after the run,
the energies logged along the run and the oracle's Newton iteration counts.
Floats are stored with repr, which round-trips exactly.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import lattice_inputs as L  # noqa: E402
import oracle as O  # noqa: E402

# The Newton tolerance is the paper's, an absolute bound on ||r^l||_inf
# (Algorithm 1; epsilon = 1e-13 in Sec. 3).
CASES = {
    # name: (steps, eps, solver, energy_every, sampled)
    "lattice32": (1000, 1e-13, "direct", 100, False),
    "lattice256": (1000, 1e-13, "gmres", 100, True),
    "lattice2048": (20, 1e-13, "gmres", 5, True),
    # The same with the packet on the lattice corner (wrapping every edge).
    "lattice2048corner": (20, 1e-13, "gmres", 5, True),
    # The continuum runs of Sec. 3: the whole t in [0, 0.5] of the 70 x 70
    # comparison run, and the whole t in [0, 20] of the delta run.
    "continuum70": (50, 1e-13, "direct", 5, True),
    "delta100": (2000, 1e-13, "direct", 125, True),
}
# Runs whose stopping test is relative to ||u_0||_inf (|u| reaches 5 there,
# and the residual's rounding floor lies above the absolute 1e-13).
RELATIVE = {"continuum70"}


def sample_sites(cfg, n_packet=512, n_uniform=512, seed=2024):
    """Half of the sample inside three packet widths of the packet's centre
    (periodic distance), half uniform over the lattice; fixed by the seed."""
    rng = np.random.default_rng(seed)
    cx, cy = (cfg.nx // 2, cfg.ny // 2) if cfg.centre is None else cfg.centre
    x = np.arange(cfg.nx)
    y = np.arange(cfg.ny)
    dx = np.abs(x - cx)
    dx = np.minimum(dx, cfg.nx - dx)
    dy = np.abs(y - cy)
    dy = np.minimum(dy, cfg.ny - dy)
    d2 = (dy[:, None] ** 2 + dx[None, :] ** 2).reshape(-1)
    near = np.flatnonzero(d2 <= (3 * cfg.sigma) ** 2)
    a = rng.choice(near, size=min(n_packet, near.size), replace=False)
    b = rng.choice(cfg.sites, size=n_uniform, replace=False)
    return np.unique(np.concatenate([a, b]))


def make(name: str) -> str:
    steps, eps, solver, every, sampled = CASES[name]
    cfg = L.CONFIGS[name]
    v, p, q = L.make_inputs(cfg)
    relative = name in RELATIVE
    orc = O.oracle_for(cfg, v, eps=eps, solver=solver, relative=relative)
    t0 = time.time()
    u, energies = orc.run(p + 1j * q, steps, energy_every=every)
    dt = time.time() - t0
    sites = sample_sites(cfg) if sampled else np.arange(cfg.sites)
    out = {
        "workload": name, "steps": steps, "eps": eps, "eps_relative": relative, "solver": solver,
        "generated_by": "tests/golden/make_golden.py (CPU oracle only)",
        "oracle_seconds": round(dt, 1),
        "sites": [int(s) for s in sites],
        "p": [repr(float(x)) for x in u.real[sites]],
        "q": [repr(float(x)) for x in u.imag[sites]],
        "energies": [[int(n), repr(float(e))] for n, e in energies],
        "newton_iterations": orc.iteration_log,
    }
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh, separators=(",", ":"))
    return path


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(CASES)):
        print(nm, make(nm), flush=True)
