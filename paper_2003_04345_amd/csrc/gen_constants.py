"""Writes mb4_constants.h: the MB4 constants the HIP kernels compile in.

Run as ``python gen_constants.py [--check]`` from any directory.  Every value
is derived in exact arithmetic (sympy) from the method's definition in
Sakai et al., arXiv 2003.04345, Sec. 2.2, and rounded once to the nearest
double:

* A_{tau,zeta} = [tau, tau^2/2, tau^3/3] M(alpha_1) [1, zeta, zeta^2]^T
  (Eq. Adefinition) with alpha_1 = -300 * 19/8 and c = (1/3, 2/3, 1)
  (Sec. 3, computational conditions);
* E_ij = int_0^1 A_{c_i,zeta} l_j(zeta) dzeta for j = 0..3 (Eqs. defE, Ei0);
* the eigenvalues Lambda of E (closed form, with sqrt(6)) and its
  eigenvectors T (unit columns, first row positive, eigenvalues ascending),
  and T^-1 (Eq. Newton3);
* the 6-node Gauss-Legendre rule on [0, 1] and the tables
  Q_iq = w_q A_{c_i,zeta_q}, L_qj = l_j(zeta_q).  The stage integrand of the
  cubic term has degree 2 + 9 = 11 in zeta, so six nodes integrate it
  exactly; this replaces the paper's table of cubic-polynomial coefficients
  (Eq. fIu2) by a quadrature with the same value.
* TC_i = sum_m (T^-1)_im c_m: at U = e_3 (x) u_0 the residual of stage m is
  -h c_m f(u_0), so the transformed residual is -h TC_i f(u_0).
* E_i0 + sum_j E_ij = int_0^1 A_{c_i,zeta} dzeta = c_i (checked here): with
  the stage values held as U_j = u_0 + X_j, the linear part of stage i is
  c_i u_0 + sum_j E_ij X_j.
"""
from __future__ import annotations

import argparse
import os
import sys

import mpmath
import sympy as sp

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "mb4_constants.h")
DIGITS = 60


def derive():
    z, tau = sp.symbols("zeta tau")
    a = sp.Rational(-300) * sp.Rational(19, 8)
    m = sp.Matrix([[a + 4, -6 * a - 6, 6 * a],
                   [-6 * a - 6, 36 * a + 12, -36 * a],
                   [6 * a, -36 * a, 36 * a]])
    a_tz = (sp.Matrix([[tau, tau ** 2 / 2, tau ** 3 / 3]]) * m * sp.Matrix([1, z, z ** 2]))[0]
    c = [sp.Integer(0), sp.Rational(1, 3), sp.Rational(2, 3), sp.Integer(1)]
    ell = []
    for j in range(4):
        lj = sp.Integer(1)
        for k in range(4):
            if k != j:
                lj *= (z - c[k]) / (c[j] - c[k])
        ell.append(sp.expand(lj))
    a_c = [sp.expand(a_tz.subs(tau, c[i + 1])) for i in range(3)]
    e_full = sp.Matrix(3, 4, lambda i, j: sp.integrate(a_c[i] * ell[j], (z, 0, 1)))
    e = e_full[:, 1:]
    # Exact eigenpairs; sort ascending by numeric value.
    pairs = []
    for lam, mult, vecs in e.eigenvects():
        assert mult == 1
        v = vecs[0]
        v = v / sp.sqrt(sum(x ** 2 for x in v))
        v = sp.simplify(v)
        if sp.N(v[0], DIGITS) < 0:
            v = -v
        pairs.append((sp.N(lam, DIGITS), sp.nsimplify(lam), v))
    pairs.sort(key=lambda p: p[0])
    lam = [p[1] for p in pairs]
    t = sp.Matrix.hstack(*[p[2] for p in pairs])
    tinv = t.inv()
    # Sanity: E T = T Lambda exactly.
    resid = (e * t - t * sp.diag(*lam)).applyfunc(lambda x: sp.N(x, DIGITS))
    assert max(abs(x) for x in resid) < sp.Float(10) ** (-40)

    # 6-node Gauss-Legendre on [0, 1], nodes and weights to DIGITS digits.
    mpmath.mp.dps = DIGITS + 10
    x = sp.symbols("x")
    p6 = sp.legendre_poly(6, x)
    dp6 = sp.diff(p6, x)
    roots = sorted(sp.Poly(p6, x).nroots(n=DIGITS + 10))
    nodes, weights = [], []
    for r in roots:
        w = 2 / ((1 - r ** 2) * dp6.subs(x, r) ** 2)
        nodes.append((r + 1) / 2)
        weights.append(w / 2)
    q_tab = [[weights[q] * a_c[i].subs(z, nodes[q]) for q in range(6)] for i in range(3)]
    l_tab = [[ell[j].subs(z, nodes[q]) for j in range(4)] for q in range(6)]
    # Check: sum_q Q_iq L_qj = E_ij (exactness of the rule on degree 5).
    for i in range(3):
        for j in range(4):
            s = sum(q_tab[i][q] * l_tab[q][j] for q in range(6))
            assert abs(sp.N(s - e_full[i, j], DIGITS)) < sp.Float(10) ** (-40)
    tc = [sum(tinv[i, mm] * c[mm + 1] for mm in range(3)) for i in range(3)]
    # Row sums of the full E (j = 0..3) are int_0^1 A_{c_i,zeta} dzeta (the l_j
    # sum to one), which equal c_i: the kernels take c_i for them.
    for i in range(3):
        assert sp.simplify(sum(e_full[i, j] for j in range(4)) - c[i + 1]) == 0
    return {
        "c": c[1:], "e0": [e_full[i, 0] for i in range(3)],
        "e": [[e[i, j] for j in range(3)] for i in range(3)],
        "lam": lam, "t": [[t[i, j] for j in range(3)] for i in range(3)],
        "tinv": [[tinv[i, j] for j in range(3)] for i in range(3)],
        "gl_q": q_tab, "gl_l": l_tab, "tc": tc,
        "gl_nodes": nodes, "gl_weights": weights,
    }


def _hex(v) -> str:
    f = float(sp.N(v, DIGITS))
    if f == 0.0:
        return "0.0"
    return f.hex()


def _arr1(name, vals, comment):
    body = ", ".join(_hex(v) for v in vals)
    return f"// {comment}\nstatic constexpr double {name}[{len(vals)}] = {{{body}}};\n"


def _arr2(name, rows, comment):
    inner = ",\n    ".join("{" + ", ".join(_hex(v) for v in row) + "}" for row in rows)
    return (f"// {comment}\nstatic constexpr double {name}[{len(rows)}][{len(rows[0])}] = {{\n"
            f"    {inner}}};\n")


def render(k) -> str:
    parts = [
        "// Generated by gen_constants.py; do not edit.\n",
        "// MB4 constants for alpha_1 = -1425/2, c = (1/3, 2/3, 1), each the double\n",
        "// nearest to its exact value (Sakai et al., arXiv 2003.04345, Sec. 2.2).\n",
        "#pragma once\n\n",
        _arr1("MB4_C", k["c"], "stage nodes c_1..c_3"),
        _arr1("MB4_E0", k["e0"], "E_i0 = int A_{c_i,z} l_0(z) dz (Eq. Ei0)"),
        _arr2("MB4_E", k["e"], "E_ij = int A_{c_i,z} l_j(z) dz (Eq. defE)"),
        _arr1("MB4_LAMBDA", k["lam"], "eigenvalues of E, ascending (Eq. Newton3)"),
        _arr2("MB4_T", k["t"], "eigenvectors of E as columns (unit 2-norm, first row > 0)"),
        _arr2("MB4_TINV", k["tinv"], "inverse of MB4_T"),
        _arr1("MB4_TC", k["tc"], "TC_i = sum_m TINV_im c_m"),
        _arr2("MB4_GL_Q", k["gl_q"], "Q_iq = w_q A_{c_i,z_q}, 6-node Gauss-Legendre on [0,1]"),
        _arr2("MB4_GL_L", k["gl_l"], "L_qj = l_j(z_q)"),
        _arr1("MB4_GL_NODES", k["gl_nodes"], "Gauss-Legendre nodes z_q on [0,1]"),
        _arr1("MB4_GL_WEIGHTS", k["gl_weights"], "Gauss-Legendre weights w_q on [0,1]"),
    ]
    return "".join(parts)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--check", action="store_true",
                    help="exit 1 if the header on disk differs from a fresh derivation")
    args = ap.parse_args(argv)
    text = render(derive())
    if args.check:
        try:
            with open(OUT) as fh:
                same = fh.read() == text
        except FileNotFoundError:
            same = False
        if not same:
            print("mb4_constants.h is stale", file=sys.stderr)
            return 1
        return 0
    with open(OUT, "w") as fh:
        fh.write(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
