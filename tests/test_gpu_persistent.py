"""GPU tests of the persistent form of ensemble batches
(mb4_ensemble_set_persistent): one launch per batch in which each block owns
whole members and runs their time loop and Newton loop (Algorithm 1) on the
device.  Every member must follow, bit for bit, the trajectory of the
per-phase form (itself checked against single states and the oracle in
test_gpu_ensemble.py), with the same Newton iteration counts, whatever the
region shape, sweeps and precision, with more members than blocks, across
batches and when the form is switched mid-run."""
import numpy as np
import pytest

import lattice_inputs as L
import oracle as O
from gpu_common import torch_cuda
from paper_2003_04345_amd import mb4 as M

pytestmark = pytest.mark.gpu

# Uneven members: ragged and tiny lattices, different g, signs of h, and a
# member (h = 0.03) that needs more Newton iterations than the others.
MEMBERS = [
    L.config("lattice32", seed=11),
    L.config("lattice32", nx=33, ny=17, sigma=2.0, defect_count=3, seed=12, g=2.0),
    L.config("lattice32", nx=5, ny=67, sigma=1.5, defect_count=2, seed=13, h=0.03),
    L.config("lattice32", nx=64, ny=8, sigma=2.0, defect_count=2, seed=14, g=0.0),
    L.config("lattice32", nx=3, ny=3, sigma=1.0, defect_count=1, seed=15, h=-0.01),
    L.config("lattice32", nx=70, ny=45, initial="random", defect_count=6, seed=16),
]


def _ensemble(members, inputs, persistent, **kw):
    ens = M.MB4Ensemble(members, [v for v, _, _ in inputs], **kw)
    for i, (_, p, q) in enumerate(inputs):
        ens.set_state(i, p, q)
    if persistent:
        ens.set_persistent(True)
        assert ens.persistent()
    return ens


def _run(members, inputs, persistent, steps, setup=None, **kw):
    with _ensemble(members, inputs, persistent, **kw) as ens:
        if setup is not None:
            setup(ens)
        rc = ens.step(steps)
        detail = M.error_detail() if rc != M.MB4_OK else ""
        states = [ens.get_state(i) for i in range(len(members))]
        stats = [ens.member_stats(i) for i in range(len(members))]
    return rc, detail, states, stats


def _assert_same(a, b):
    rc_a, det_a, st_a, stats_a = a
    rc_b, det_b, st_b, stats_b = b
    assert rc_a == rc_b, (det_a, det_b)
    assert det_a == det_b
    for i, ((pa, qa), (pb, qb)) in enumerate(zip(st_a, st_b)):
        assert np.array_equal(pa, pb) and np.array_equal(qa, qb), i
    assert stats_a == stats_b


@pytest.mark.parametrize("region", [M.MB4_REGION_32x32, M.MB4_REGION_64x16, M.MB4_REGION_32x16])
@pytest.mark.parametrize("sweeps", [1, 2, 3, 4])
def test_persistent_matches_per_phase_bitwise(region, sweeps):
    torch_cuda()
    inputs = [L.make_inputs(m) for m in MEMBERS]

    def setup(ens):
        ens.set_region(region)

    steps = 45   # more than one batch of 32
    ref = _run(MEMBERS, inputs, False, steps, setup, inner_sweeps=sweeps)
    got = _run(MEMBERS, inputs, True, steps, setup, inner_sweeps=sweeps)
    assert ref[0] == M.MB4_OK, ref[1]
    _assert_same(ref, got)
    iters = [s["newton_iters"] for s in got[3]]
    print(f"{M.REGION_NAMES[region]} sweeps {sweeps}: newton iterations {iters}")


@pytest.mark.parametrize("opts", [dict(fp32_solve=True), dict(relative_eps=True, eps=1e-13),
                                  dict(graphs=False)],
                         ids=["fp32", "relative-eps", "no-graphs"])
def test_persistent_options_match_per_phase_bitwise(opts):
    torch_cuda()
    inputs = [L.make_inputs(m) for m in MEMBERS]
    ref = _run(MEMBERS, inputs, False, 40, **opts)
    got = _run(MEMBERS, inputs, True, 40, **opts)
    assert ref[0] == M.MB4_OK, ref[1]
    _assert_same(ref, got)


def test_more_members_than_blocks_match_bitwise():
    # 1,100 small members: more than the persistent launch's blocks, so that
    # blocks run several members one after the other.
    torch_cuda()
    rng = np.random.default_rng(7)
    members = [L.config("lattice32", nx=int(rng.integers(3, 13)), ny=int(rng.integers(3, 13)),
                        sigma=1.0, defect_count=1, seed=100 + r,
                        g=float(rng.uniform(0.0, 2.0)))
               for r in range(1100)]
    inputs = [L.make_inputs(m) for m in members]
    ref = _run(members, inputs, False, 12)
    got = _run(members, inputs, True, 12)
    assert ref[0] == M.MB4_OK, ref[1]
    _assert_same(ref, got)


def test_switching_forms_mid_run_matches_one_form():
    torch_cuda()
    inputs = [L.make_inputs(m) for m in MEMBERS]
    with _ensemble(MEMBERS, inputs, False) as a, _ensemble(MEMBERS, inputs, False) as b:
        assert a.step(30) == M.MB4_OK
        for on in (True, False, True):
            b.set_persistent(on)
            assert b.step(10) == M.MB4_OK
        for i in range(len(MEMBERS)):
            assert all(np.array_equal(x, y) for x, y in zip(a.get_state(i), b.get_state(i))), i
            assert a.member_stats(i) == b.member_stats(i)


def test_failing_members_match_per_phase():
    # max_newton = 5 is too few for some members at 3 sweeps (the h = 5
    # member never converges): both forms report MB4_ENOCONV for the same
    # member, keep each failed member's last accepted state and let the
    # others advance.
    torch_cuda()
    members = MEMBERS + [L.config("lattice32", h=5.0, seed=21)]
    inputs = [L.make_inputs(m) for m in members]
    ref = _run(members, inputs, False, 20, max_newton=5)
    got = _run(members, inputs, True, 20, max_newton=5)
    assert ref[0] == M.MB4_ENOCONV
    _assert_same(ref, got)
    p, q = got[2][-1]
    assert np.array_equal(p, inputs[-1][1]) and np.array_equal(q, inputs[-1][2])
    assert got[3][-1]["steps_done"] == 0
    assert max(s["steps_done"] for s in got[3]) > 0
    print("steps done:", [s["steps_done"] for s in got[3]])


def test_persistent_member_matches_oracle():
    torch_cuda()
    members = [L.CONFIGS["lattice32"], MEMBERS[1], MEMBERS[5]]
    inputs = [L.make_inputs(m) for m in members]
    with _ensemble(members, inputs, True, eps=1e-14) as ens:
        assert ens.step(6) == M.MB4_OK, M.error_detail()
        for i, (m, (v, p, q)) in enumerate(zip(members, inputs)):
            solver = "direct" if m.nx * m.ny <= 64 * 64 else "gmres"
            ref, _ = O.oracle_for(m, v, eps=1e-14, solver=solver).run(p + 1j * q, 6)
            err = float(np.max(np.abs(ens.psi(i) - ref)))
            assert err <= 1e-13, (i, err)


def test_persistent_workload_slice_conserves_energy():
    # A slice of the 128^2 disorder ensemble (seeds 1000 + r) over 300 steps.
    torch_cuda()
    members = [L.ensemble_member(r) for r in range(8)]
    inputs = [L.make_inputs(m) for m in members]
    with _ensemble(members, inputs, True) as ens:
        h0 = ens.energies()
        assert ens.step(300) == M.MB4_OK, M.error_detail()
        h1 = ens.energies()
    drift = float(np.max(np.abs(h1 - h0) / np.abs(h0)))
    print(f"ensemble128 x8, persistent, 300 steps: max energy drift {drift:.3e}")
    assert drift <= 1e-14


def test_tune_launch_keeps_the_trajectory():
    torch_cuda()
    inputs = [L.make_inputs(m) for m in MEMBERS]
    with _ensemble(MEMBERS, inputs, False) as a, _ensemble(MEMBERS, inputs, False) as b:
        assert a.step(5) == M.MB4_OK and b.step(5) == M.MB4_OK
        pe, ms = b.tune_launch(4)
        assert b.persistent() == pe and len(ms) == 2 and min(ms) > 0
        assert ms[1 if pe else 0] == min(ms)
        assert a.step(7) == M.MB4_OK and b.step(7) == M.MB4_OK
        for i in range(len(MEMBERS)):
            assert all(np.array_equal(x, y) for x, y in zip(a.get_state(i), b.get_state(i))), i
            assert a.member_stats(i) == b.member_stats(i)


def test_member_failing_at_an_odd_step_keeps_that_steps_state():
    # A focusing member (g = -40) whose Newton iteration count grows from 12
    # to 13 at step 11 (0-based) of its run: with max_newton = 12 it fails
    # there, in the middle of a batch and on a step that reads the batch's
    # second u_0 buffer.  Both forms keep the state after its 11 accepted
    # steps, which is the single state's after 11 steps, bit for bit.
    torch_cuda()
    focus = L.config("lattice32", nx=8, ny=8, sigma=1.0, defect_count=1, seed=31, g=-40.0,
                     h=0.01)
    members = [MEMBERS[0], focus]
    inputs = [L.make_inputs(m) for m in members]
    ref = _run(members, inputs, False, 20, max_newton=12)
    got = _run(members, inputs, True, 20, max_newton=12)
    assert ref[0] == M.MB4_ENOCONV and "member 1" in got[1]
    _assert_same(ref, got)
    assert got[3][0]["steps_done"] == 20 and got[3][1]["steps_done"] == 11
    v, p, q = inputs[1]
    with M.MB4State(focus.nx, focus.ny, v, focus.g, focus.h) as st:
        st.set_state(p, q)
        assert st.step(11) == M.MB4_OK, M.error_detail()
        assert st.last_stats()["newton_iters"] == 12
        sp, sq = st.get_state()
    assert np.array_equal(got[2][1][0], sp) and np.array_equal(got[2][1][1], sq)
