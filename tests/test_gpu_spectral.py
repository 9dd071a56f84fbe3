"""GPU parity of the spectrally preconditioned stage solves against the oracle,
through the C ABI: the paper's continuum runs of Sec. 3 (K = -Delta_h on
[0, 2 pi)^2, u_0 = 1 + 2 cos x + 2 cos y), where block-Jacobi sweeps diverge."""
import numpy as np
import pytest

import lattice_inputs as L
import oracle as O
from gpu_common import torch_cuda
from paper_2003_04345_amd import mb4 as M

pytestmark = pytest.mark.gpu

EPS_PARITY = 1e-14


def _continuum(name, n, **kw):
    return L.config(name, nx=n, ny=n, t_hop=L.continuum_hopping(n),
                    diag_shift=4.0 * L.continuum_hopping(n), **kw)


def _state(cfg, v, sweeps, eps=EPS_PARITY, spectral=True, **kw):
    return M.MB4State(cfg.nx, cfg.ny, v, cfg.g, cfg.h, t_hop=cfg.t_hop,
                      diag_shift=cfg.diag_shift, eps=eps, inner_sweeps=sweeps,
                      spectral_solve=spectral, **kw)


@pytest.mark.parametrize("n,steps,sweeps", [(32, 10, 6), (70, 5, 6), (33, 4, 6), (70, 5, 2)])
def test_continuum_steps_match_oracle(n, steps, sweeps):
    # u_0 reaches 5 here, so both sides stop at 1e-13 * ||u_0||_inf: with U
    # stored, the oracle's own residual has a rounding floor of about 2e-13
    # on the 70 x 70 continuum (h lambda ||K|| ~ 15).
    torch_cuda()
    cfg = _continuum("continuum70", n)
    v, p, q = L.make_inputs(cfg)
    with _state(cfg, v, sweeps, eps=1e-13, relative_eps=True) as st:
        st.set_state(p, q)
        assert st.step(steps) == M.MB4_OK, M.error_detail()
        gpu = st.psi()
        iters = st.last_stats()["newton_iters"]
    ref, _ = O.oracle_for(cfg, v, eps=1e-13, relative=True).run(p + 1j * q, steps)
    err = np.max(np.abs(gpu - ref))
    print(f"continuum {n}x{n}, {steps} steps, {sweeps} Richardson iterations: max-abs vs oracle "
          f"{err:.3e}, {iters} Newton iterations")
    assert err <= 1e-12


def test_continuum70_conserves_energy_and_probability():
    # Sec. 3, Fig. 1 setup over t in [0, 0.5]: the energy is kept to 1e-14;
    # the total probability is not an invariant of MB4 and drifts by about
    # 6e-8 here (the oracle gives 6.3e-8 at t = 0.5).  Read literally
    # (u_0 = 1 + 2 cos x + 2 cos y, gamma = 0.1, focusing) the solution
    # concentrates, max |u| 5 -> 32 by t = 0.86, and the simplified Newton
    # iteration at h = 0.01 stops converging at t = 0.87 in the oracle too.
    # The tolerance is 1e-13 relative to ||u_0||_inf: evaluating the residual
    # with h ||K|| ~ 10 and |u| >= 5 leaves a rounding floor of about 3e-13.
    # The energy itself is evaluated with error-free per-site terms: with the
    # diagonal shift 4t each site's terms cancel to the much smaller kinetic
    # density, and a plain FP64 evaluation alone put about 2e-14 of rounding
    # into the logged drift.
    torch_cuda()
    cfg = L.CONFIGS["continuum70"]
    v, p, q = L.make_inputs(cfg)
    with _state(cfg, v, 6, eps=1e-13, relative_eps=True) as st:
        st.set_state(p, q)
        c0 = st.energy_components()
        worst_h = worst_p = 0.0
        for _ in range(5):
            assert st.step(10) == M.MB4_OK, M.error_detail()
            c = st.energy_components()
            worst_h = max(worst_h, abs(c["H"] - c0["H"]) / abs(c0["H"]))
            worst_p = max(worst_p, abs(c["prob"] - c0["prob"]) / c0["prob"])
    print(f"continuum70, 50 steps: energy drift {worst_h:.3e}, probability drift {worst_p:.3e}")
    assert worst_h <= 1e-14
    assert worst_p <= 1e-7


@pytest.mark.parametrize("n,sweeps", [(40, 12), (100, 4)])
def test_delta_potential_matches_oracle(n, sweeps):
    # The delta-function-like potential of Sec. 3 (V = -50 at the origin):
    # the site the preconditioner leaves out needs more Richardson
    # iterations, or more Newton iterations, not a different root.  100 x 100
    # with 4 Richardson iterations is the full-size run as bench.py times it.
    torch_cuda()
    cfg = _continuum("delta100", n, origin_v=-50.0)
    v, p, q = L.make_inputs(cfg)
    with _state(cfg, v, sweeps) as st:
        st.set_state(p, q)
        h0 = st.energy()
        assert st.step(6) == M.MB4_OK, M.error_detail()
        gpu = st.psi()
        h1 = st.energy()
    ref, _ = O.oracle_for(cfg, v, eps=EPS_PARITY).run(p + 1j * q, 6)
    err = np.max(np.abs(gpu - ref))
    print(f"delta potential {n}x{n}, {sweeps} Richardson iterations, 6 steps: max-abs vs oracle {err:.3e}")
    assert err <= 1e-13
    assert abs(h1 - h0) <= 1e-14 * abs(h0)


def test_block_jacobi_fails_where_spectral_solves_converge():
    # On the continuum, h lambda t is ~1.6 per link at 32 x 32: block-Jacobi
    # sweeps diverge and the step is reported as not converged.
    torch_cuda()
    cfg = _continuum("continuum70", 32)
    v, p, q = L.make_inputs(cfg)
    with _state(cfg, v, 3, spectral=False, max_newton=20) as st:
        st.set_state(p, q)
        assert st.step(1) == M.MB4_ENOCONV
        assert st.steps_done() == 0
    with _state(cfg, v, 6) as st:
        st.set_state(p, q)
        assert st.step(1) == M.MB4_OK


@pytest.mark.parametrize("graphs", [True, False])
def test_spectral_and_block_jacobi_reach_the_same_root(graphs):
    # On the hopping lattice both inner solvers work; the converged steps
    # agree to the Newton tolerance.
    torch_cuda()
    cfg = L.CONFIGS["lattice32"]
    v, p, q = L.make_inputs(cfg)
    out = []
    for spectral in (False, True):
        with _state(cfg, v, 4, spectral=spectral, graphs=graphs) as st:
            st.set_state(p, q)
            assert st.step(20) == M.MB4_OK, M.error_detail()
            out.append(st.psi())
    assert np.max(np.abs(out[0] - out[1])) <= 1e-13
