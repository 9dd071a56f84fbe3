"""Seeded random cases of the whole step against the oracle.

Each case draws, from its own seed: the lattice (3 to 200 sites per side,
so ragged tiles, both wrap paths and the smallest lattice all occur), the
launch shape (region and 1 to 6 block-Jacobi sweeps, i.e. the fused and the
plain path, FP32 inner solves where they are built), the problem (g, h of
either sign, t_hop, diag_shift, disorder and defects) and a delocalised
initial state with signal on every site.  Two steps of Algorithm 1 (time
loop) must match the oracle's site by site.  Cases the draws might miss are
listed explicitly: the 3 x 3 lattice, g = 0, a negative step, no potential.
"""
import numpy as np
import pytest

import lattice_inputs as L
import oracle as O
from gpu_common import torch_cuda
from paper_2003_04345_amd import mb4 as M

pytestmark = pytest.mark.gpu

STEPS = 2
EPS = 1e-14


def _draw(case):
    rng = np.random.default_rng(9000 + case)
    nx, ny = (int(x) for x in rng.integers(3, 201, size=2))
    region = int(rng.integers(0, M.MB4_REGION_COUNT))
    sweeps = int(rng.integers(1, 7))
    fp32 = bool(rng.random() < 0.3) and region == M.MB4_REGION_32x32 and sweeps <= 4
    return dict(nx=nx, ny=ny, region=region, sweeps=sweeps, fp32=fp32,
                g=float(rng.uniform(-2.0, 3.0)), h=float(rng.choice([0.01, -0.01, 0.02])),
                t_hop=float(rng.uniform(0.5, 1.5)), diag_shift=float(rng.uniform(-1.0, 4.0)),
                disorder_w=float(rng.uniform(0.0, 2.0)),
                defects=int(rng.integers(0, max(1, nx * ny // 100) + 1)), seed=case)


EXPLICIT = [
    dict(nx=3, ny=3, region=0, sweeps=3, fp32=False, g=1.0, h=0.01, t_hop=1.0, diag_shift=0.0,
         disorder_w=1.0, defects=1, seed=1),
    dict(nx=3, ny=150, region=1, sweeps=4, fp32=False, g=2.0, h=0.01, t_hop=1.0, diag_shift=0.0,
         disorder_w=1.0, defects=2, seed=2),
    dict(nx=90, ny=70, region=2, sweeps=2, fp32=False, g=0.0, h=0.01, t_hop=1.0, diag_shift=0.0,
         disorder_w=1.0, defects=5, seed=3),
    dict(nx=64, ny=33, region=0, sweeps=3, fp32=True, g=1.5, h=-0.01, t_hop=1.0, diag_shift=0.0,
         disorder_w=1.0, defects=3, seed=4),
    dict(nx=47, ny=47, region=0, sweeps=5, fp32=False, g=-1.0, h=0.01, t_hop=1.2, diag_shift=4.8,
         disorder_w=0.0, defects=0, seed=5),
]
CASES = EXPLICIT + [_draw(c) for c in range(24)]


@pytest.mark.parametrize("c", CASES, ids=lambda c: (
    f"{c['nx']}x{c['ny']}-r{c['region']}-s{c['sweeps']}{'-f32' if c['fp32'] else ''}"
    f"-g{c['g']:.2f}-h{c['h']}"))
def test_random_case_matches_oracle(c):
    torch_cuda()
    cfg = L.config("lattice256", nx=c["nx"], ny=c["ny"], t_hop=c["t_hop"],
                   diag_shift=c["diag_shift"], disorder_w=c["disorder_w"],
                   defect_count=c["defects"], g=c["g"], h=c["h"], initial="random",
                   seed=c["seed"], steps=STEPS, energy_every=0)
    v, p, q = L.make_inputs(cfg)
    solver = "direct" if cfg.sites <= 64 * 64 else "gmres"
    ref, _ = O.oracle_for(cfg, v, eps=EPS, solver=solver).run(p + 1j * q, STEPS)
    with M.MB4State(cfg.nx, cfg.ny, v, cfg.g, cfg.h, t_hop=cfg.t_hop,
                    diag_shift=cfg.diag_shift, eps=EPS, inner_sweeps=c["sweeps"],
                    fp32_solve=c["fp32"]) as st:
        st.set_region(c["region"])
        st.set_state(p, q)
        assert st.step(STEPS) == M.MB4_OK, M.error_detail()
        err = float(np.max(np.abs(st.psi() - ref)))
    assert err <= 1e-13, err
