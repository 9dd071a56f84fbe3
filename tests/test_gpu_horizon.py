"""Checks of the full 2048^2 run beyond the oracle's horizon (the stored
oracle run covers its first 20 of 2000 steps).

* Order under step halving (Sec. 3.1: MB4 is of order 4): the full run at h,
  h/2 and h/4 to the same final time.  The differences e(h) = |u_h - u_{h/2}|
  and e(h/2) = |u_{h/2} - u_{h/4}| must fall by 2^4 = 16.  The +100 defect
  sites hold bound states at h * omega ~ 0.5, outside the asymptotic regime
  of R(z) - e^z = O(z^5) (their phase error per step at h is ~6e-3 rad), so
  the ratio is read on the sites more than six links from every defect:
  a bound state falls off by about t / V = 1e-2 per link, so its error of
  ~1e-2 is ~1e-14 there, far below e(h/2) ~ 5e-9.
* Tight stage solves: the same run with 16 block-Jacobi sweeps per stage
  solve (exact to rounding: the sweep contraction is ~0.03 here) and a
  Newton tolerance of 1e-16, against the default run (3 sweeps, 1e-13).
  Both reach the collocation root of every step (Eqs. Phidefinition,
  MB4_4 - MB4_6), so the two trajectories may differ only by the Newton
  error left at the default tolerance (~rho * 1e-13 per step) and rounding.
"""
import numpy as np
import pytest

import lattice_inputs as L
from gpu_common import torch_cuda
from paper_2003_04345_amd import mb4 as M

pytestmark = pytest.mark.gpu

_RUNS = {}


def _run(h_div=1, sweeps=0, eps=0.0):
    key = (h_div, sweeps, eps)
    if key not in _RUNS:
        cfg = L.CONFIGS["lattice2048"]
        v, p, q = L.make_inputs(cfg)
        with M.MB4State(cfg.nx, cfg.ny, v, cfg.g, cfg.h / h_div, eps=eps,
                        inner_sweeps=sweeps) as st:
            st.set_state(p, q)
            h0 = st.energy()
            rc = st.step(cfg.steps * h_div)
            assert rc == M.MB4_OK, M.error_detail()
            _RUNS[key] = (st.psi(), h0, st.energy())
    return _RUNS[key]


def _away_from_defects(cfg, v, links=6):
    """Mask of sites more than `links` lattice links from every defect."""
    d = (v == cfg.defect_v).reshape(cfg.ny, cfg.nx)
    near = d.copy()
    for _ in range(links):
        near = (near | np.roll(near, 1, 0) | np.roll(near, -1, 0)
                | np.roll(near, 1, 1) | np.roll(near, -1, 1))
    return ~near.reshape(-1)


def test_full_run_converges_with_order_four():
    torch_cuda()
    cfg = L.CONFIGS["lattice2048"]
    v, _, _ = L.make_inputs(cfg)
    u1, _, _ = _run(1)
    u2, _, _ = _run(2)
    u4, _, _ = _run(4)
    e1 = np.abs(u1 - u2)
    e2 = np.abs(u2 - u4)
    for links in (2, 3, 4, 6, 8):
        m = _away_from_defects(cfg, v, links)
        print(f"  more than {links} links from defects: l2 ratio "
              f"{np.sqrt(np.sum(e1[m] ** 2) / np.sum(e2[m] ** 2)):.3f}")
    mask = _away_from_defects(cfg, v)
    l2 = float(np.sqrt(np.sum(e1[mask] ** 2) / np.sum(e2[mask] ** 2)))
    mx = float(e1[mask].max() / e2[mask].max())
    print(f"lattice2048, T = {cfg.steps * cfg.h}: e(h) {np.sqrt(np.sum(e1[mask]**2)):.3e}, "
          f"e(h/2) {np.sqrt(np.sum(e2[mask]**2)):.3e} (l2, away from defects); "
          f"ratio l2 {l2:.2f}, max {mx:.2f}; at defects max e(h) {e1[~mask].max():.3e}, "
          f"e(h/2) {e2[~mask].max():.3e}")
    assert 16 * 0.9 <= l2 <= 16 * 1.1
    assert 16 * 0.9 <= mx <= 16 * 1.1
    # The errors are far above the rounding and Newton floors of the runs.
    assert np.sqrt(np.sum(e2[mask] ** 2)) > 1e3 * 1e-13


def test_tight_stage_solves_give_the_same_trajectory():
    torch_cuda()
    base, h0, h1 = _run(1)
    tight, t0, t1 = _run(1, sweeps=16, eps=1e-16)
    err = float(np.max(np.abs(base - tight)))
    print(f"lattice2048, 2000 steps: default (3 sweeps, 1e-13) vs tight (16 sweeps, 1e-16) "
          f"max-abs {err:.3e}; drift {abs(h1 - h0) / abs(h0):.2e} / {abs(t1 - t0) / abs(t0):.2e}")
    assert err <= 1e-12
    assert abs(t1 - t0) <= 1e-14 * abs(t0)
