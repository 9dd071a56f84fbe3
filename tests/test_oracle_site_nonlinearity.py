"""Pins of the oracle with a site-dependent nonlinearity (the Appendix:
U_I = -1/2 sum_i gamma_i n_i^2, gamma_i = -g_i, with G = U_K + U_I conserved).

Each checks the per-site path against something other than itself: the
brute-force collocation solve with per-site g written out site by site, the
uniform path when every g_i is equal, finite differences of f, and the
energy invariant of the method."""
import numpy as np

import lattice_inputs as L
import oracle as O
from brute_mb4 import collocation_step, lattice_f


def test_step_matches_bruteforce_with_per_site_g_3x3():
    rng = np.random.default_rng(77)
    nx = ny = 3
    v = rng.uniform(-2, 2, 9)
    g = rng.uniform(-1.0, 2.0, 9)
    h = 0.05
    u0 = (rng.standard_normal(9) + 1j * rng.standard_normal(9)) * 0.8
    lat = O.LatticeNLS(nx, ny, v, g, t_hop=0.9)
    u1 = O.MB4Oracle(lat, h, eps=1e-15, max_newton=60).step(u0)
    ref = collocation_step(lattice_f(nx, ny, 0.9, v.tolist(), g.tolist()), u0.tolist(), h,
                           dps=32, tol_digits=26)
    ref = np.array([complex(z) for z in ref])
    assert np.max(np.abs(u1 - ref)) < 5e-15
    # A per-site g that differs from its mean matters at this size.
    lat_mean = O.LatticeNLS(nx, ny, v, float(np.mean(g)), t_hop=0.9)
    u_mean = O.MB4Oracle(lat_mean, h, eps=1e-15, max_newton=60).step(u0)
    assert np.max(np.abs(u_mean - ref)) > 1e-4


def test_equal_site_values_reproduce_the_uniform_nonlinearity():
    cfg = L.config("lattice32", nx=6, ny=5, defect_count=1, steps=5)
    v, p, q = L.make_inputs(cfg)
    u0 = p + 1j * q
    uni = O.oracle_for(cfg, v, eps=1e-14)
    site = O.oracle_for(cfg, v, eps=1e-14, g=np.full(cfg.sites, cfg.g))
    a, ea = uni.run(u0, 5)
    b, eb = site.run(u0, 5)
    assert np.array_equal(a, b)
    assert [e for _, e in ea] == [e for _, e in eb]


def test_jacobian_matches_finite_differences_with_per_site_g():
    rng = np.random.default_rng(8)
    nx, ny = 4, 3
    lat = O.LatticeNLS(nx, ny, rng.uniform(-1, 1, nx * ny), rng.uniform(-2, 2, nx * ny))
    u = rng.standard_normal(lat.s) + 1j * rng.standard_normal(lat.s)
    jac = lat.jacobian(u).toarray()
    s, step = lat.s, 1e-6
    fd = np.zeros((2 * s, 2 * s))
    for col in range(2 * s):
        e = np.zeros(s, dtype=complex)
        if col < s:
            e[col] = step
        else:
            e[col - s] = 1j * step
        df = (lat.f(u + e) - lat.f(u - e)) / (2 * step)
        fd[:s, col] = df.real
        fd[s:, col] = df.imag
    np.testing.assert_allclose(jac, fd, rtol=0, atol=1e-7)


def test_energy_with_per_site_g_is_conserved():
    # G = U_K + U_E + U_I with U_I = sum_i g_i n_i^2 / 4 (library convention)
    # is the invariant of the flow, so MB4 keeps it at its root.
    cfg = L.config("lattice32", nx=10, ny=8, defect_count=2, initial="random", seed=31,
                   g_range=(-1.5, 2.5), steps=40)
    v, p, q = L.make_inputs(cfg)
    gs = L.make_nonlinearity(cfg)
    orc = O.oracle_for(cfg, v, eps=1e-15, g=gs)
    _, energies = orc.run(p + 1j * q, 40, energy_every=5)
    assert O.energy_drift(energies) < 1e-14
    # and U_I is the per-site sum, not the mean g times sum n^2
    comps = orc.prob.energy_components(p + 1j * q)
    n = p * p + q * q
    assert abs(comps["U_I"] - 0.25 * float(np.sum(gs * n * n))) < 1e-14 * abs(comps["U_I"])
    assert abs(comps["U_I"] - 0.25 * float(np.mean(gs)) * float(np.sum(n * n))) > 1e-6


def test_per_site_g_draws_are_seeded_and_in_range():
    cfg = L.config("lattice32", nx=9, ny=7, g_range=(0.5, 1.5))
    a = L.make_nonlinearity(cfg)
    b = L.make_nonlinearity(cfg)
    assert a.shape == (63,) and np.array_equal(a, b)
    assert a.min() >= 0.5 and a.max() < 1.5
    assert L.make_nonlinearity(L.config("lattice32")) is None
