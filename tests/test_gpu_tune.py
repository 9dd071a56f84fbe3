"""Launch shape of single states through the C ABI (mb4_set_region,
mb4_set_sweeps, mb4_tune): every shape reaches the oracle's root, the region
shapes give identical bits, and the autotuner leaves the run where it was."""
import numpy as np
import pytest

import lattice_inputs as L
import oracle as O
from gpu_common import torch_cuda
from paper_2003_04345_amd import mb4 as M

pytestmark = pytest.mark.gpu

EPS_PARITY = 1e-14


def _state(cfg, v, **kw):
    return M.MB4State(cfg.nx, cfg.ny, v, cfg.g, cfg.h, t_hop=cfg.t_hop,
                      diag_shift=cfg.diag_shift, eps=EPS_PARITY, **kw)


@pytest.mark.parametrize("nx,ny", [(32, 32), (100, 65)])
def test_every_shape_matches_the_oracle_and_regions_agree_bitwise(nx, ny):
    # Regions only change which block computes a site; sweeps change the
    # inexact stage solves of the simplified Newton iteration, not its root.
    torch_cuda()
    cfg = L.config("lattice32", nx=nx, ny=ny, sigma=1.5)
    v, p, q = L.make_inputs(cfg)
    ref, _ = O.oracle_for(cfg, v, eps=EPS_PARITY).run(p + 1j * q, 10)
    for sweeps in (2, 3, 4):
        out = []
        for region in range(M.MB4_REGION_COUNT):
            with _state(cfg, v) as st:
                st.set_region(region)
                st.set_sweeps(sweeps)
                assert (st.region(), st.sweeps()) == (region, sweeps)
                st.set_state(p, q)
                assert st.step(10) == M.MB4_OK, M.error_detail()
                out.append(st.psi())
        err = np.max(np.abs(out[0] - ref))
        print(f"{nx}x{ny}, {sweeps} sweeps: max-abs vs oracle {err:.3e}")
        assert err <= 1e-13
        for o in out[1:]:
            assert np.array_equal(o, out[0])


@pytest.mark.parametrize("fp32", [False, True])
def test_tune_restores_the_run_and_keeps_the_fastest_pair(fp32):
    torch_cuda()
    cfg = L.config("lattice256", nx=128, ny=128)
    v, p, q = L.make_inputs(cfg)
    with _state(cfg, v, fp32_solve=fp32) as st, _state(cfg, v, fp32_solve=fp32) as plain:
        for s in (st, plain):
            s.set_state(p, q)
            assert s.step(7) == M.MB4_OK, M.error_detail()
        before = st.psi()
        stats0 = st.last_stats()
        st.profile_enable(True)
        prof0 = st.profile_read()
        region, sweeps, ms = st.tune(4)
        # Trials stay out of the kernel profile.
        assert st.profile_read() == prof0
        st.profile_enable(False)
        print(f"fp32={fp32}: kept {M.REGION_NAMES[region]}/{sweeps}; "
              + ", ".join(f"{M.REGION_NAMES[r]}/{sw} {t:.4f}" for (r, sw), t in sorted(ms.items())))
        # Every pair was timed (FP32 solves: 32 x 32 only), the fastest kept.
        expected = {(r, sw) for sw in (2, 3, 4)
                    for r in ([M.MB4_REGION_32x32] if fp32 else range(M.MB4_REGION_COUNT))}
        assert set(ms) == expected
        assert ms[(region, sweeps)] == min(ms.values())
        assert (st.region(), st.sweeps()) == (region, sweeps)
        # The state, the step count and the statistics are those of before.
        assert np.array_equal(st.psi(), before)
        assert st.steps_done() == 7
        assert st.last_stats() == stats0
        # The run continues to the same root as an untuned one.
        assert st.step(10) == M.MB4_OK, M.error_detail()
        assert plain.step(10) == M.MB4_OK, M.error_detail()
        assert st.steps_done() == 17
        assert np.max(np.abs(st.psi() - plain.psi())) <= 1e-13


def test_shape_setters_reject_what_is_not_built():
    torch_cuda()
    cfg = L.CONFIGS["lattice32"]
    v, p, q = L.make_inputs(cfg)
    with _state(cfg, v, fp32_solve=True) as st:
        with pytest.raises(M.Mb4Error):
            st.set_region(M.MB4_REGION_64x16)
        with pytest.raises(M.Mb4Error):
            st.set_sweeps(5)
        assert (st.region(), st.sweeps()) == (M.MB4_REGION_32x32, 3)
    with _state(cfg, v) as st:
        with pytest.raises(M.Mb4Error):
            st.set_region(M.MB4_REGION_COUNT)
        with pytest.raises(M.Mb4Error):
            st.set_sweeps(0)
    with _state(cfg, v, spectral_solve=True) as st:
        with pytest.raises(M.Mb4Error):
            st.tune(2)
