"""GPU parity with a site-dependent nonlinearity g_j (the Appendix's
U_I = -1/2 sum_i gamma_i n_i^2, gamma_i = -g_i), set through
mb4_set_nonlinearity_sites, against the oracle with the same g_j."""
import numpy as np
import pytest

import lattice_inputs as L
import oracle as O
from gpu_common import torch_cuda
from paper_2003_04345_amd import mb4 as M

pytestmark = pytest.mark.gpu

EPS = 1e-14
STEPS = 4
_REF = {}


def _problem(nx, ny):
    return L.config("lattice256", nx=nx, ny=ny, initial="random", seed=41 + nx + ny,
                    defect_count=max(1, int(round(0.005 * nx * ny))), steps=STEPS,
                    energy_every=0, g_range=(-1.5, 2.5))


def _reference(nx, ny):
    if (nx, ny) not in _REF:
        cfg = _problem(nx, ny)
        v, p, q = L.make_inputs(cfg)
        gs = L.make_nonlinearity(cfg)
        ref, _ = O.oracle_for(cfg, v, eps=EPS, solver="gmres", g=gs).run(p + 1j * q, STEPS)
        _REF[(nx, ny)] = (cfg, v, p, q, gs, ref)
    return _REF[(nx, ny)]


@pytest.mark.parametrize("nx,ny", [(100, 65), (37, 20)])
@pytest.mark.parametrize("region,fp32", [(M.MB4_REGION_32x32, False), (M.MB4_REGION_64x16, False),
                                         (M.MB4_REGION_32x16, False), (M.MB4_REGION_32x32, True)])
def test_per_site_g_steps_match_oracle(nx, ny, region, fp32):
    torch_cuda()
    cfg, v, p, q, gs, ref = _reference(nx, ny)
    with M.MB4State(cfg.nx, cfg.ny, v, cfg.g, cfg.h, eps=EPS, fp32_solve=fp32) as st:
        st.set_region(region)
        st.set_nonlinearity_sites(gs)
        st.set_state(p, q)
        assert st.step(STEPS) == M.MB4_OK, M.error_detail()
        err = float(np.max(np.abs(st.psi() - ref)))
    print(f"{nx}x{ny} {M.REGION_NAMES[region]}{' fp32' if fp32 else ''}: per-site g, "
          f"max-abs vs oracle {err:.3e}")
    assert err <= 1e-13


def test_per_site_g_on_the_plain_path_matches_oracle():
    # Six sweeps: the fused solve plus plain sweeps, and the plain update pass.
    torch_cuda()
    cfg, v, p, q, gs, ref = _reference(100, 65)
    with M.MB4State(cfg.nx, cfg.ny, v, cfg.g, cfg.h, eps=EPS, inner_sweeps=6) as st:
        st.set_nonlinearity_sites(gs)
        st.set_state(p, q)
        assert st.step(STEPS) == M.MB4_OK, M.error_detail()
        assert np.max(np.abs(st.psi() - ref)) <= 1e-13


def test_per_site_g_with_spectral_solves_matches_oracle():
    torch_cuda()
    n = 32
    cfg = L.config("continuum70", nx=n, ny=n, t_hop=L.continuum_hopping(n),
                   diag_shift=4.0 * L.continuum_hopping(n), g_range=(-0.15, -0.05), seed=5)
    v, p, q = L.make_inputs(cfg)
    gs = L.make_nonlinearity(cfg)
    with M.MB4State(cfg.nx, cfg.ny, v, cfg.g, cfg.h, t_hop=cfg.t_hop, diag_shift=cfg.diag_shift,
                    eps=1e-13, relative_eps=True, inner_sweeps=6, spectral_solve=True) as st:
        st.set_nonlinearity_sites(gs)
        st.set_state(p, q)
        assert st.step(5) == M.MB4_OK, M.error_detail()
        gpu = st.psi()
    ref, _ = O.oracle_for(cfg, v, eps=1e-13, relative=True, g=gs).run(p + 1j * q, 5)
    err = float(np.max(np.abs(gpu - ref)))
    print(f"continuum 32x32, per-site g, spectral solves: max-abs vs oracle {err:.3e}")
    assert err <= 1e-12


def test_equal_site_values_give_the_uniform_bits_and_null_restores_them():
    torch_cuda()
    cfg = L.CONFIGS["lattice32"]
    v, p, q = L.make_inputs(cfg)
    runs = []
    for mode in ("uniform", "equal", "reset"):
        with M.MB4State(cfg.nx, cfg.ny, v, cfg.g, cfg.h) as st:
            if mode != "uniform":
                st.set_nonlinearity_sites(np.full(cfg.sites, cfg.g))
            if mode == "reset":
                st.set_nonlinearity_sites(np.linspace(0.0, 3.0, cfg.sites))
                st.set_nonlinearity_sites(None)
            st.set_state(p, q)
            assert st.step(40) == M.MB4_OK, M.error_detail()
            runs.append((st.psi(), st.energy()))
    for psi, h in runs[1:]:
        assert np.array_equal(psi, runs[0][0]) and h == runs[0][1]


def test_per_site_g_energy_components_match_oracle():
    torch_cuda()
    cfg, v, p, q, gs, _ = _reference(100, 65)
    lat = O.LatticeNLS(cfg.nx, cfg.ny, v, gs)
    want = lat.energy_components(p + 1j * q)
    with M.MB4State(cfg.nx, cfg.ny, v, cfg.g, cfg.h) as st:
        st.set_nonlinearity_sites(gs)
        st.set_state(p, q)
        got = st.energy_components()
    for key in ("H", "U_K", "U_I", "U_E", "prob", "participation"):
        assert abs(got[key] - want[key]) <= 1e-15 * max(abs(want[key]), 1e-300), key


def test_per_site_g_full_run_conserves_energy():
    # A 256^2 wavepacket run with g_j ~ U[0, 2]: H (with U_I = sum g_j n_j^2 / 4)
    # is kept to the workloads' 1e-14 over 2000 steps.
    torch_cuda()
    cfg = L.config("lattice256", g_range=(0.0, 2.0))
    v, p, q = L.make_inputs(cfg)
    with M.MB4State(cfg.nx, cfg.ny, v, cfg.g, cfg.h) as st:
        st.set_nonlinearity_sites(L.make_nonlinearity(cfg))
        st.set_state(p, q)
        h0 = st.energy()
        worst = 0.0
        for _ in range(10):
            assert st.step(200) == M.MB4_OK, M.error_detail()
            worst = max(worst, abs(st.energy() - h0) / abs(h0))
    print(f"256x256, per-site g, 2000 steps: energy drift {worst:.3e}")
    assert worst <= 1e-14


def test_per_site_g_validation_and_budget():
    torch_cuda()
    cfg = L.CONFIGS["lattice32"]
    v, p, q = L.make_inputs(cfg)
    with M.MB4State(cfg.nx, cfg.ny, v, cfg.g, cfg.h) as st:
        bad = np.full(cfg.sites, 1.0)
        bad[7] = np.nan
        with pytest.raises(M.Mb4Error) as e:
            st.set_nonlinearity_sites(bad)
        assert e.value.code == M.MB4_EINVAL
    # The smallest budget (in steps of one byte per site) that holds the
    # state leaves less than 8 more bytes per site.
    need = None
    for budget in range(200 * cfg.sites, 100 * cfg.sites, -cfg.sites):
        try:
            with M.MB4State(cfg.nx, cfg.ny, v, cfg.g, cfg.h, mem_budget=budget):
                need = budget
        except M.Mb4Error:
            break
    assert need is not None
    with M.MB4State(cfg.nx, cfg.ny, v, cfg.g, cfg.h, mem_budget=need) as st:
        with pytest.raises(M.Mb4Error) as e:
            st.set_nonlinearity_sites(np.ones(cfg.sites))
        assert e.value.code == M.MB4_ENOMEM
