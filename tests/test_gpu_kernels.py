"""GPU parity of single kernels, through the C ABI, against the oracle and
plain references (Sec. 2.2-2.3 of the paper)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import lattice_inputs as L
import oracle as O
from gpu_common import (block_jacobi_reference, from_device_planes, oracle_update_residual,
                        to_device_planes, torch_cuda)
from paper_2003_04345_amd import mb4 as M

pytestmark = pytest.mark.gpu

SHAPES = [(32, 32), (33, 17), (3, 3), (130, 7), (64, 8), (5, 67)]


def _problem(nx, ny, seed, g=1.3, h=0.01, t=1.0, shift=0.0, defects=2):
    rng = np.random.default_rng(seed)
    v = rng.uniform(-0.5, 0.5, nx * ny)
    v[rng.choice(nx * ny, size=min(defects, nx * ny), replace=False)] = 50.0
    u0 = (rng.standard_normal(nx * ny) + 1j * rng.standard_normal(nx * ny)) * 0.3
    return v, u0, g, h, t, shift


@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("with_rbar", [True, False])
def test_newton_update_matches_oracle(nx, ny, with_rbar):
    torch_cuda()
    v, u0, g, h, t, shift = _problem(nx, ny, seed=nx * 1000 + ny)
    s = nx * ny
    rng = np.random.default_rng(s)
    U = u0[None, :] + 0.05 * (rng.standard_normal((3, s)) + 1j * rng.standard_normal((3, s)))
    rbar = 0.01 * (rng.standard_normal((3, s)) + 1j * rng.standard_normal((3, s)))
    lat = O.LatticeNLS(nx, ny, v, g, t_hop=t, diag_shift=shift)
    orc = O.MB4Oracle(lat, h)
    Un_ref, phib_ref = oracle_update_residual(orc, u0, U, rbar if with_rbar else None)
    with M.MB4State(nx, ny, v, g, h, t_hop=t, diag_shift=shift) as st:
        st.set_state(u0.real, u0.imag)
        dU = to_device_planes(U)
        dr = to_device_planes(rbar) if with_rbar else None
        dphib = to_device_planes(np.zeros((3, s), dtype=complex))
        rnorm = M.mb4_newton_update(st.handle, dU, dr, dphib)
        Un = from_device_planes(dU, s)
        phib = from_device_planes(dphib, s)
    # FP64 rounding of sums whose terms reach |h| (4|t| + max|V|) max|W|.
    scale = np.max(np.abs(Un_ref)) * (1 + abs(h) * (4 * abs(t) + np.max(np.abs(v))) * 16)
    assert np.max(np.abs(Un - Un_ref)) <= 4e-16 * np.max(np.abs(Un_ref)) * 4
    assert np.max(np.abs(phib - phib_ref)) <= 1e-14 * scale
    if with_rbar:
        r = np.tensordot(orc.k.T, rbar, axes=(1, 0))
        rref = max(np.max(np.abs(r.real)), np.max(np.abs(r.imag)))
        assert abs(rnorm - rref) <= 1e-15 * rref
    else:
        assert rnorm == 0.0


@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("sweeps", [1, 2, 3, 4, 5, 7])
def test_stage_sweeps_match_block_jacobi_reference(nx, ny, sweeps):
    torch_cuda()
    v, u0, g, h, t, shift = _problem(nx, ny, seed=7 + nx + ny, shift=0.3)
    s = nx * ny
    rng = np.random.default_rng(s + sweeps)
    phib = 0.01 * (rng.standard_normal((3, s)) + 1j * rng.standard_normal((3, s)))
    lam = O.method_constants().lam
    ref = block_jacobi_reference(nx, ny, v, shift, t, g, h, lam, u0, phib, sweeps)
    with M.MB4State(nx, ny, v, g, h, t_hop=t, diag_shift=shift) as st:
        st.set_state(u0.real, u0.imag)
        dphib = to_device_planes(phib)
        dr = to_device_planes(np.zeros((3, s), dtype=complex))
        M.mb4_stage_solve(st.handle, dphib, dr, sweeps)
        got = from_device_planes(dr, s)
    assert np.max(np.abs(got - ref)) <= 1e-15 * np.max(np.abs(ref)) * 8


@pytest.mark.parametrize("nx,ny", [(32, 32), (33, 17)])
def test_stage_sweeps_converge_to_the_exact_stage_solution(nx, ny):
    # Many sweeps reach (I - h lambda_i J)^-1 (-Phibar_i) (Eq. MB4_5) with J
    # from the oracle (Eqs. JL, JR), solved by SuperLU.
    torch_cuda()
    v, u0, g, h, t, shift = _problem(nx, ny, seed=99)
    s = nx * ny
    rng = np.random.default_rng(5)
    phib = 0.01 * (rng.standard_normal((3, s)) + 1j * rng.standard_normal((3, s)))
    lat = O.LatticeNLS(nx, ny, v, g, t_hop=t, diag_shift=shift)
    jac = lat.jacobian(u0)
    lam = O.method_constants().lam
    with M.MB4State(nx, ny, v, g, h, t_hop=t, diag_shift=shift) as st:
        st.set_state(u0.real, u0.imag)
        dphib = to_device_planes(phib)
        dr = to_device_planes(np.zeros((3, s), dtype=complex))
        M.mb4_stage_solve(st.handle, dphib, dr, 40)
        got = from_device_planes(dr, s)
    for i in range(3):
        m = (sp.identity(2 * s) - h * lam[i] * jac).tocsc()
        x = spla.spsolve(m, -np.concatenate([phib[i].real, phib[i].imag]))
        exact = x[:s] + 1j * x[s:]
        assert np.max(np.abs(got[i] - exact)) <= 1e-14 * np.max(np.abs(exact))


def test_device_state_roundtrip():
    torch = torch_cuda()
    cfg = L.CONFIGS["lattice32"]
    v, p, q = L.make_inputs(cfg)
    with M.MB4State(cfg.nx, cfg.ny, v, cfg.g, cfg.h) as st:
        dp = torch.from_numpy(p).to("cuda")
        dq = torch.from_numpy(q).to("cuda")
        torch.cuda.synchronize()
        M.mb4_set_state_device(st.handle, dp, dq)
        hp, hq = st.get_state()
        assert np.array_equal(hp, p) and np.array_equal(hq, q)
        op = torch.empty_like(dp)
        oq = torch.empty_like(dq)
        M.mb4_get_state_device(st.handle, op, oq)
        assert np.array_equal(op.cpu().numpy(), p) and np.array_equal(oq.cpu().numpy(), q)


def test_energy_components_match_oracle():
    torch_cuda()
    for name in ("lattice32", "lattice256"):
        cfg = L.CONFIGS[name]
        v, p, q = L.make_inputs(cfg)
        lat = O.LatticeNLS(cfg.nx, cfg.ny, v, cfg.g, t_hop=cfg.t_hop, diag_shift=cfg.diag_shift)
        ref = lat.energy_components(p + 1j * q)
        with M.MB4State(cfg.nx, cfg.ny, v, cfg.g, cfg.h) as st:
            st.set_state(p, q)
            got = st.energy_components()
        for key in ("H", "U_K", "U_I", "U_E", "prob", "participation"):
            assert abs(got[key] - ref[key]) <= 4e-16 * max(abs(ref[key]), 1e-300) + 1e-300, key
