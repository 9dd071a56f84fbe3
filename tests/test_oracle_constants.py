"""Pins for the oracle's method constants (Sec. 2.2 of the paper).

Each check is a property the paper or the mathematics fixes, not a re-typing
of the oracle's formulas.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from oracle.mb4_oracle import a_of_tau, lagrange_basis, _pint01, _pmul


def test_a_vanishes_at_tau0_and_b_is_a_at_tau1():
    # Sec. 2.2: A_{0,zeta} = 0 and B_zeta = A_{1,zeta}.  Consistency of the
    # quadrature u_1 = u_0 + h int B f needs int B = 1; for MB4, A_{1,zeta} is
    # identically 1 (the method's weight function is the AVF one).
    assert a_of_tau(0, O.ALPHA1_PAPER) == [0, 0, 0]
    assert a_of_tau(1, O.ALPHA1_PAPER) == [1, 0, 0]


def test_dA_dtau_is_symmetric():
    # Energy preservation of a CSRK method needs d/dtau A_{tau,zeta} to be
    # symmetric in (tau, zeta) when B = 1 (Miyatake-Butcher's condition);
    # check on a grid of rational points by exact differencing of the cubic.
    def dA(tau, zeta):
        # derivative in tau of the cubic A(tau, zeta), exact by polynomial algebra
        eps = Fraction(1, 10 ** 6)
        a1 = a_of_tau(tau + eps, O.ALPHA1_PAPER)
        a0 = a_of_tau(tau - eps, O.ALPHA1_PAPER)
        v1 = sum(c * zeta ** k for k, c in enumerate(a1))
        v0 = sum(c * zeta ** k for k, c in enumerate(a0))
        return (v1 - v0) / (2 * eps)   # exact up to O(eps^2) * tau-cubic term
    pts = [Fraction(k, 7) for k in range(8)]
    for s in pts:
        for z in pts:
            assert abs(float(dA(s, z) - dA(z, s))) < 1e-6


def test_last_stage_row_is_simpson_three_eighths():
    # With c_3 = 1, A_{c_3,zeta} = 1, so E_3j = int l_j: the Newton-Cotes
    # weights of the nodes (0, 1/3, 2/3, 1), i.e. Simpson's 3/8 rule.
    k = O.method_constants()
    assert k.E_exact[2] == [Fraction(1, 8), Fraction(3, 8), Fraction(3, 8), Fraction(1, 8)]


def test_row_sums_are_the_nodes():
    # sum_j l_j = 1, and int_0^1 A_{tau,zeta} dzeta = tau (first-order
    # consistency of the stages), so E_i0 + sum_j E_ij = c_i.
    for c in (O.C_PAPER, (Fraction(1, 4), Fraction(1, 2), Fraction(1)),
              (Fraction(1, 10), Fraction(7, 10), Fraction(1))):
        k = O.method_constants(c=c)
        for i in range(3):
            assert sum(k.E_exact[i]) == c[i]


def test_eigenvalues_do_not_depend_on_c():
    # Sec. 2.2: E is diagonalisable with real eigenvalues independent of the
    # choice of c_1, c_2, c_3.
    ref = O.method_constants().lam
    for c in ((Fraction(1, 4), Fraction(1, 2), Fraction(1)),
              (Fraction(1, 10), Fraction(7, 10), Fraction(1)),
              (Fraction(1, 5), Fraction(3, 5), Fraction(4, 5))):
        lam = O.method_constants(c=c).lam
        np.testing.assert_allclose(lam, ref, rtol=0, atol=1e-13)


def test_eigendecomposition_reconstructs_E():
    k = O.method_constants()
    np.testing.assert_allclose(k.T @ np.diag(k.lam) @ k.Tinv, k.E, rtol=0, atol=1e-14)
    np.testing.assert_allclose(k.T @ k.Tinv, np.eye(3), rtol=0, atol=1e-15)


def test_eigenvalues_for_general_alpha_are_real_only_below_threshold():
    # Eq. Adefinition: alpha_1 must lie below -300 * 0.7770503941 for the
    # method's properties; just above 0 the eigenvalues of E turn complex.
    # The paper's value is far inside the admissible range.
    k = O.method_constants(alpha1=Fraction(-1425, 2))
    assert np.all(np.isfinite(k.lam))
    with pytest.raises(ValueError):
        O.method_constants(alpha1=Fraction(1))


def test_lagrange_basis_is_cardinal():
    nodes = [Fraction(0)] + list(O.C_PAPER)
    ell = lagrange_basis(nodes)
    for j in range(4):
        for kk, ck in enumerate(nodes):
            val = sum(c * ck ** p for p, c in enumerate(ell[j]))
            assert val == (1 if j == kk else 0)


def test_cubic_table_matches_gauss_legendre_quadrature():
    # Eq. fIu2 by the precomputed cubic polynomial against direct numerical
    # integration of A_{c_i,z} |U_z|^2 U_z with a 20-node Gauss-Legendre
    # rule (numpy's leggauss), on random complex stage values.
    k = O.method_constants()
    rng = np.random.default_rng(7)
    ys = rng.standard_normal((4, 5)) + 1j * rng.standard_normal((4, 5))
    cub = k.cubic
    poly = np.zeros((3, 5), dtype=complex)
    for a in range(4):
        for b in range(4):
            for d in range(4):
                poly += cub[:, a, b, d][:, None] * (np.conj(ys[a]) * ys[b] * ys[d])[None, :]
    x, w = np.polynomial.legendre.leggauss(20)
    z = (x + 1) / 2
    w = w / 2
    nodes = [Fraction(0)] + list(O.C_PAPER)
    ell = lagrange_basis(nodes)
    lz = np.array([[float(sum(float(c) * zz ** p for p, c in enumerate(ell[j]))) for j in range(4)]
                   for zz in z])
    quad = np.zeros((3, 5), dtype=complex)
    for i in range(3):
        a_poly = [float(c) for c in a_of_tau(nodes[i + 1], O.ALPHA1_PAPER)]
        for qi, zz in enumerate(z):
            uz = lz[qi] @ ys
            aval = a_poly[0] + a_poly[1] * zz + a_poly[2] * zz ** 2
            quad[i] += w[qi] * aval * np.abs(uz) ** 2 * uz
    np.testing.assert_allclose(poly, quad, rtol=0, atol=1e-9 * np.max(np.abs(quad)))


def test_E_is_exact_integral_of_polynomials():
    # E_ij against a 20-node Gauss-Legendre integral in float64.
    k = O.method_constants()
    x, w = np.polynomial.legendre.leggauss(20)
    z = (x + 1) / 2
    w = w / 2
    nodes = [Fraction(0)] + list(O.C_PAPER)
    ell = lagrange_basis(nodes)
    for i in range(3):
        a_poly = [float(c) for c in a_of_tau(nodes[i + 1], O.ALPHA1_PAPER)]
        for j in range(4):
            lj = [float(c) for c in ell[j]]
            vals = [(a_poly[0] + a_poly[1] * zz + a_poly[2] * zz ** 2)
                    * sum(c * zz ** p for p, c in enumerate(lj)) for zz in z]
            assert abs(float(np.dot(w, vals)) - k.E_full[i, j]) < 1e-9


def test_exact_integral_helper():
    assert _pint01([Fraction(0), Fraction(0), Fraction(3)]) == 1
    assert _pmul([Fraction(1), Fraction(1)], [Fraction(-1), Fraction(1)]) == [-1, 0, 1]
