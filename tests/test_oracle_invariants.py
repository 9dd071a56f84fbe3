"""Pins for the oracle's MB4 step: brute force, exact linear solutions and the
invariants the paper states (Sec. 2.2 and Sec. 3)."""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle as O
import lattice_inputs as L
from brute_mb4 import collocation_step, lattice_f


def _oracle(nx, ny, v, g, h, t_hop=1.0, diag_shift=0.0, eps=1e-15, c=None, solver="direct"):
    lat = O.LatticeNLS(nx, ny, v, g, t_hop=t_hop, diag_shift=diag_shift)
    k = O.method_constants(c=c) if c is not None else None
    return O.MB4Oracle(lat, h, eps=eps, max_newton=60, constants=k, solver=solver)


def test_step_matches_bruteforce_collocation_3x3():
    # Full nonlinear step on a 3x3 lattice (18 real unknowns per stage):
    # the oracle's simplified Newton with E, T, Lambda and the cubic table
    # against a direct 32-digit solve of the collocation equations.
    rng = np.random.default_rng(123)
    nx = ny = 3
    v = rng.uniform(-2, 2, 9)
    g = 1.3
    h = 0.05
    u0 = (rng.standard_normal(9) + 1j * rng.standard_normal(9)) * 0.8
    orc = _oracle(nx, ny, v, g, h, t_hop=0.9)
    u1 = orc.step(u0)
    ref = collocation_step(lattice_f(nx, ny, 0.9, v.tolist(), g), u0.tolist(), h,
                           dps=32, tol_digits=26)
    ref = np.array([complex(z) for z in ref])
    assert np.max(np.abs(u1 - ref)) < 5e-15
    # and the step really moved the state
    assert np.max(np.abs(u1 - u0)) > 1e-2


def test_scalar_linear_step_is_brute_force_stability_function():
    # g = 0 on a lattice: the step is u_1 = Q R(-i h D) Q^T u_0 with A = Q D Q^T,
    # where R(z) is MB4's one-step map for y' = z y, computed here by a
    # brute-force collocation solve of the scalar problem at each eigenvalue.
    rng = np.random.default_rng(9)
    nx, ny = 4, 3
    v = rng.uniform(-1, 1, nx * ny)
    h = 0.1
    orc = _oracle(nx, ny, v, 0.0, h)
    a = orc.prob.A.toarray()
    d, q = np.linalg.eigh(a)
    r = []
    for lam in d:
        f = (lambda lam_: (lambda y: [-1j * mpmath.mpf(float(lam_)) * y[0]]))(lam)
        r.append(complex(collocation_step(f, [1.0], h, dps=30, tol_digits=25)[0]))
    u0 = rng.standard_normal(nx * ny) + 1j * rng.standard_normal(nx * ny)
    expect = q @ (np.array(r) * (q.T @ u0))
    got = orc.step(u0)
    assert np.max(np.abs(got - expect)) < 1e-14 * np.max(np.abs(u0))


def test_linear_case_converges_to_exact_exponential_at_fourth_order():
    # g = 0: exact solution exp(-i A t) u_0 by dense eigendecomposition.
    # Sec. 3.1: MB4 is of order 4.
    rng = np.random.default_rng(4)
    nx, ny = 5, 4
    v = rng.uniform(-1, 1, nx * ny)
    u0 = rng.standard_normal(nx * ny) + 1j * rng.standard_normal(nx * ny)
    u0 /= np.linalg.norm(u0)
    t_end = 0.8
    errs = []
    for nsteps in (16, 32, 64):
        orc = _oracle(nx, ny, v, 0.0, t_end / nsteps)
        d, q = np.linalg.eigh(orc.prob.A.toarray())
        exact = q @ (np.exp(-1j * d * t_end) * (q.T @ u0))
        u, _ = orc.run(u0, nsteps)
        errs.append(np.max(np.abs(u - exact)))
    assert errs[-1] < 1e-6
    for e1, e2 in zip(errs, errs[1:]):
        assert 16 * 0.9 < e1 / e2 < 16 * 1.1


def test_linear_case_preserves_probability():
    # With g = 0 the one-step map is R(-i h A) with |R(i y)| = 1 on the real
    # spectrum, so sum |u|^2 is conserved (Sec. 3.1 discusses the probability).
    cfg = L.config("lattice32", g=0.0)
    v, p, q = L.make_inputs(cfg)
    orc = O.oracle_for(cfg, v, eps=1e-15)
    u, _ = orc.run(p + 1j * q, 20)
    assert abs(np.sum(np.abs(u) ** 2) - 1.0) < 1e-14


def test_nonlinear_order_four_by_step_halving():
    rng = np.random.default_rng(21)
    nx, ny = 6, 5
    v = rng.uniform(-1, 1, nx * ny)
    u0 = (rng.standard_normal(nx * ny) + 1j * rng.standard_normal(nx * ny)) * 0.7
    g = 1.5
    t_end = 0.4
    ref, _ = _oracle(nx, ny, v, g, t_end / 256).run(u0, 256)
    errs = []
    for n in (16, 32, 64):
        u, _ = _oracle(nx, ny, v, g, t_end / n).run(u0, n)
        errs.append(np.max(np.abs(u - ref)))
    for e1, e2 in zip(errs, errs[1:]):
        assert 16 * 0.9 < e1 / e2 < 16 * 1.1


def test_energy_conserved_on_lattice_workload():
    # Sec. 3 reports the energy kept to 1e-14 (70x70) and 1e-16 (100x100).
    cfg = L.CONFIGS["lattice32"]
    v, p, q = L.make_inputs(cfg)
    orc = O.oracle_for(cfg, v, eps=1e-14)
    _, energies = orc.run(p + 1j * q, 60, energy_every=10)
    assert O.energy_drift(energies) < 1e-14


def test_energy_conserved_on_paper_continuum_problem():
    # The paper's default conditions (Sec. 3): [0, 2 pi]^2 periodic, 5-point
    # -Laplacian, u_0 = 1 + 2 cos x + 2 cos y, gamma = 0.1 (g = -0.1),
    # h = 0.01, V = 0; on a 12x12 grid for a fifth of the time span.
    n = 12
    hx = 2 * math.pi / n
    x = np.arange(n) * hx
    u0 = (1 + 2 * np.cos(x)[None, :] + 2 * np.cos(x)[:, None]).reshape(-1).astype(complex)
    orc = _oracle(n, n, np.zeros(n * n), -0.1, 0.01, t_hop=1 / hx ** 2,
                  diag_shift=4 / hx ** 2, eps=1e-13)
    _, energies = orc.run(u0, 20, energy_every=1)
    assert O.energy_drift(energies) < 1e-14
    comp0 = orc.prob.energy_components(u0)
    assert comp0["U_I"] < 0          # attractive nonlinearity lowers the energy


def test_time_reversal():
    # A_{tau,zeta} + A_{1-tau,1-zeta} = B_zeta makes MB4 symmetric: n steps
    # with +h then n steps with -h return to u_0.
    cfg = L.CONFIGS["lattice32"]
    v, p, q = L.make_inputs(cfg)
    u0 = p + 1j * q
    fwd = O.oracle_for(cfg, v, eps=1e-15)
    u, _ = fwd.run(u0, 15)
    bwd = O.oracle_for(L.config("lattice32", h=-cfg.h), v, eps=1e-15)
    back, _ = bwd.run(u, 15)
    assert np.max(np.abs(back - u0)) < 1e-14
    assert np.max(np.abs(u - u0)) > 1e-3


def test_phase_equivariance():
    cfg = L.CONFIGS["lattice32"]
    v, p, q = L.make_inputs(cfg)
    u0 = p + 1j * q
    theta = 0.7
    a, _ = O.oracle_for(cfg, v, eps=1e-15).run(u0, 3)
    b, _ = O.oracle_for(cfg, v, eps=1e-15).run(np.exp(1j * theta) * u0, 3)
    assert np.max(np.abs(b - np.exp(1j * theta) * a)) < 1e-15


def test_translation_and_transpose_symmetry_without_potential():
    n = 9
    rng = np.random.default_rng(3)
    u0 = (rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)) * 0.5
    orc = _oracle(n, n, np.zeros(n * n), 1.0, 0.02)
    a = orc.step(u0).reshape(n, n)
    shifted = np.roll(np.roll(u0.reshape(n, n), 2, axis=1), -3, axis=0).reshape(-1)
    b = orc.step(shifted).reshape(n, n)
    assert np.max(np.abs(b - np.roll(np.roll(a, 2, axis=1), -3, axis=0))) < 1e-15
    c = orc.step(u0.reshape(n, n).T.reshape(-1)).reshape(n, n)
    assert np.max(np.abs(c - a.T)) < 1e-15


def test_plane_wave_follows_scalar_mb4():
    # With V = 0 a plane wave a e^{i k.r} stays one; its amplitude obeys
    # c' = -i (eps_k + g |c|^2) c, eps_k = -2 t (cos kx + cos ky).  One MB4
    # step of that scalar problem is solved by brute force in mpmath.
    nx, ny = 8, 4
    kx, ky = 2 * math.pi * 1 / nx, 2 * math.pi * 1 / ny
    a = 0.9 + 0.4j
    g, h = 2.0, 0.05
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    wave = np.exp(1j * (kx * x + ky * y)).reshape(-1)
    orc = _oracle(nx, ny, np.zeros(nx * ny), g, h)
    u = a * wave
    eps_k = -2.0 * (math.cos(kx) + math.cos(ky))
    c = mpmath.mpc(a)
    for _ in range(3):
        u = orc.step(u)
        f = lambda y_: [-1j * (mpmath.mpf(eps_k) + g * abs(y_[0]) ** 2) * y_[0]]
        c = collocation_step(f, [c], h, dps=30, tol_digits=25)[0]
    assert np.max(np.abs(u - complex(c) * wave)) < 2e-15
    # energy preservation keeps |c| here, since H depends on |c| only
    assert abs(abs(complex(c)) - abs(a)) < 1e-14


def test_result_does_not_depend_on_interior_nodes():
    # With c_3 = 1 the step map does not depend on c_1, c_2 (the stage
    # polynomial is the same cubic; only its sample points change).
    cfg = L.CONFIGS["lattice32"]
    v, p, q = L.make_inputs(cfg)
    u0 = p + 1j * q
    lat = O.LatticeNLS(cfg.nx, cfg.ny, v, cfg.g)
    a = O.MB4Oracle(lat, cfg.h, eps=1e-15).step(u0)
    k2 = O.method_constants(c=(Fraction(1, 4), Fraction(1, 2), Fraction(1)))
    b = O.MB4Oracle(lat, cfg.h, eps=1e-15, constants=k2).step(u0)
    assert np.max(np.abs(a - b)) < 1e-15


def test_direct_and_iterative_stage_solvers_reach_the_same_root():
    cfg = L.CONFIGS["lattice32"]
    v, p, q = L.make_inputs(cfg)
    u0 = p + 1j * q
    a, _ = O.oracle_for(cfg, v, eps=1e-15, solver="direct").run(u0, 2)
    b, _ = O.oracle_for(cfg, v, eps=1e-15, solver="gmres").run(u0, 2)
    assert np.max(np.abs(a - b)) < 1e-16 * 50


def test_newton_failure_is_reported():
    # Sec. 2.2: non-convergence is detected from ||r|| after a maximum number
    # of iterations.
    cfg = L.CONFIGS["lattice32"]
    v, p, q = L.make_inputs(cfg)
    orc = O.oracle_for(cfg, v, eps=1e-14, max_newton=1)
    with pytest.raises(O.NewtonDivergence):
        orc.step(p + 1j * q)


def test_zero_state_is_a_fixed_point():
    cfg = L.CONFIGS["lattice32"]
    v, _, _ = L.make_inputs(cfg)
    orc = O.oracle_for(cfg, v)
    u = orc.step(np.zeros(cfg.sites, dtype=complex))
    assert np.all(u == 0)


_BRUTE_CACHE = {}


def _brute_case():
    """A fixed 3x3 nonlinear case and its brute-force step (computed once)."""
    if "case" not in _BRUTE_CACHE:
        rng = np.random.default_rng(77)
        v = rng.uniform(-2, 2, 9)
        u0 = (rng.standard_normal(9) + 1j * rng.standard_normal(9)) * 0.6
        g, h, t = 1.1, 0.04, 1.2
        ref = collocation_step(lattice_f(3, 3, t, v.tolist(), g), u0.tolist(), h,
                               dps=32, tol_digits=26)
        _BRUTE_CACHE["case"] = (v, u0, g, h, t, np.array([complex(z) for z in ref]))
    return _BRUTE_CACHE["case"]


def _mutate_drop_e0(orc):
    orc.k.E_full[:, 0] = 0.0


def _mutate_transpose_e(orc):
    orc.k.E[:] = orc.k.E.T.copy()


def _mutate_nonlinear_sign(orc):
    orc.k.cubic[:] = -orc.k.cubic


def _mutate_cubic_drop_u0(orc):
    orc.k.cubic[:, 0, :, :] = 0.0


def _mutate_hopping_sign(orc):
    orc.prob.A = (orc.prob.A - 2 * (orc.prob.K - sp_diag(orc.prob.K))).tocsr()


def sp_diag(m):
    import scipy.sparse as sp
    return sp.diags(m.diagonal())


def _mutate_alpha(orc):
    k2 = O.method_constants(alpha1=Fraction(-1424, 2))
    orc.k.E_full[:] = k2.E_full
    orc.k.E[:] = k2.E
    orc.k.cubic[:] = k2.cubic


@pytest.mark.parametrize("mutation", [None, _mutate_drop_e0, _mutate_transpose_e,
                                      _mutate_nonlinear_sign, _mutate_cubic_drop_u0,
                                      _mutate_hopping_sign, _mutate_alpha])
def test_planted_oracle_mistakes_fail_the_bruteforce_pin(mutation):
    # Plants a plausible mistake in the oracle (on the CPU) and checks that the
    # brute-force pin tells it apart from the unmodified oracle.
    v, u0, g, h, t, ref = _brute_case()
    orc = _oracle(3, 3, v, g, h, t_hop=t)
    if mutation is not None:
        mutation(orc)
    try:
        err = np.max(np.abs(orc.step(u0) - ref))
    except O.NewtonDivergence:
        err = math.inf
    if mutation is None:
        assert err < 5e-15
    else:
        assert err > 1e-12


def test_stopping_rule_absolute_and_relative():
    # Algorithm 1 stops once ||r^l||_inf <= eps (absolute).  For g = 0 the
    # step is linear in u_0, so scaling u_0 by 2^-50 scales every Newton
    # update exactly: the relative rule then takes the same iterations and
    # returns exactly the scaled result, while the absolute rule stops
    # earlier on the small state.
    rng = np.random.default_rng(77)
    nx = ny = 8
    v = rng.uniform(-1, 1, nx * ny)
    u0 = (rng.standard_normal(nx * ny) + 1j * rng.standard_normal(nx * ny)) * 0.5
    scale = 2.0 ** -50
    lat = O.LatticeNLS(nx, ny, v, 0.0)
    rel = O.MB4Oracle(lat, 0.05, eps=1e-13, relative=True)
    a = rel.step(u0)
    ia = rel.last_iterations
    b = rel.step(scale * u0)
    assert rel.last_iterations == ia
    assert np.array_equal(b, scale * a)
    ab = O.MB4Oracle(lat, 0.05, eps=1e-13)
    c = ab.step(u0)
    ic = ab.last_iterations
    ab.step(scale * u0)
    assert ab.last_iterations < ic
    # The absolute rule at eps equals the relative rule at eps / ||u_0||_inf
    # up to the rounding of that quotient.
    m = max(np.max(np.abs(u0.real)), np.max(np.abs(u0.imag)))
    rel2 = O.MB4Oracle(lat, 0.05, eps=1e-13 / m, relative=True)
    assert np.array_equal(rel2.step(u0), c) and rel2.last_iterations == ic
