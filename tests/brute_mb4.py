"""Brute-force MB4 step in mpmath, used to pin the oracle on tiny inputs.

This solves the continuous-stage collocation equations of the method directly
(Sec. 2.2, Eqs. MB4_1 and MB4_3): the unknowns are the stage values U_{c_i},
the integrals over zeta use a 12-node Gauss-Legendre rule in high precision
(exact for the degree-11 integrands that arise), and the nonlinear system is
solved by Newton's method with a finite-difference Jacobian.  It shares
nothing with the oracle's route (no E matrix, no eigendecomposition, no
simplified Newton, no cubic coefficient table), so agreement between the two
checks all of those.
"""
from __future__ import annotations

import mpmath
from mpmath.calculus.quadrature import GaussLegendre

mp = mpmath.mp


def _a_tau_zeta(tau, zeta, alpha1):
    """A_{tau,zeta} of Eq. Adefinition for s = 3."""
    a = alpha1
    m = [[a + 4, -6 * a - 6, 6 * a],
         [-6 * a - 6, 36 * a + 12, -36 * a],
         [6 * a, -36 * a, 36 * a]]
    left = [tau, tau ** 2 / 2, tau ** 3 / 3]
    right = [1, zeta, zeta ** 2]
    return mpmath.fsum(left[r] * m[r][k] * right[k] for r in range(3) for k in range(3))


def _lagrange(nodes, j, z):
    out = mpmath.mpf(1)
    for k, ck in enumerate(nodes):
        if k != j:
            out *= (z - ck) / (nodes[j] - ck)
    return out


def _gl_rule():
    """12 Gauss-Legendre nodes and weights mapped to [0, 1]."""
    gl = GaussLegendre(mp)
    nodes = gl.calc_nodes(3, mp.prec)
    return [((x + 1) / 2, w / 2) for x, w in nodes]


def collocation_step(f, u0, h, alpha1=mpmath.mpf(-1425) / 2,
                     c=(mpmath.mpf(1) / 3, mpmath.mpf(2) / 3, mpmath.mpf(1)),
                     dps=40, tol_digits=30, max_iter=30):
    """One MB4 step for u' = f(u), u a list of mpc, by solving Eq. MB4_3.

    Returns U_{c_3} (= u_1 when c_3 = 1).
    """
    with mpmath.workdps(dps):
        u0 = [mpmath.mpc(x) for x in u0]
        n = len(u0)
        h = mpmath.mpf(h)
        alpha1 = mpmath.mpf(alpha1)
        nodes = [mpmath.mpf(0)] + [mpmath.mpf(x) for x in c]
        rule = _gl_rule()
        # Tabulate l_j(zeta_q) and A_{c_i,zeta_q} w_q.
        lq = [[_lagrange(nodes, j, z) for j in range(4)] for z, _ in rule]
        aq = [[_a_tau_zeta(nodes[i + 1], z, alpha1) * w for z, w in rule] for i in range(3)]

        def unpack(x):
            stages = []
            for i in range(3):
                stages.append([mpmath.mpc(x[2 * (i * n + k)], x[2 * (i * n + k) + 1])
                               for k in range(n)])
            return stages

        def residual(x):
            stages = unpack(x)
            ys = [u0] + stages
            fz = []
            for q in range(len(rule)):
                uz = [mpmath.fsum(lq[q][j] * ys[j][k] for j in range(4)) for k in range(n)]
                fz.append(f(uz))
            out = []
            for i in range(3):
                for k in range(n):
                    integral = mpmath.fsum(aq[i][q] * fz[q][k] for q in range(len(rule)))
                    val = stages[i][k] - u0[k] - h * integral
                    out.extend([mpmath.re(val), mpmath.im(val)])
            return out

        x = []
        for i in range(3):
            for k in range(n):
                x.extend([mpmath.re(u0[k]), mpmath.im(u0[k])])
        m = len(x)
        delta = mpmath.mpf(10) ** (-(dps // 2))

        def jacobian(x0, f0):
            # forward differences of the residual, column by column
            jac = mpmath.matrix(m, m)
            for col in range(m):
                xp = list(x0)
                xp[col] += delta
                fp = residual(xp)
                for row in range(m):
                    jac[row, col] = (fp[row] - f0[row]) / delta
            return jac

        fx = residual(x)
        jac = None
        for it in range(max_iter):
            # Newton's method; the Jacobian is refreshed on the first two
            # iterations and then kept (a chord iteration near the root).
            if it < 2:
                jac = jacobian(x, fx)
            step = mpmath.lu_solve(jac, mpmath.matrix([-v for v in fx]))
            x = [x[k] + step[k] for k in range(m)]
            fx = residual(x)
            if max(abs(v) for v in fx) < mpmath.mpf(10) ** (-tol_digits):
                break
        else:
            raise RuntimeError("brute-force collocation did not converge")
        return unpack(x)[2]


def lattice_f(nx, ny, t_hop, v, g):
    """f(psi) = -i((K + V) psi + g |psi|^2 psi), K = -t on periodic links,
    written out site by site from the lattice definition; g is one number
    or a list with one per site."""
    v = [mpmath.mpf(x) for x in v]
    t_hop = mpmath.mpf(t_hop)
    gs = [mpmath.mpf(x) for x in g] if isinstance(g, (list, tuple)) else [mpmath.mpf(g)] * len(v)

    def f(psi):
        out = []
        for y in range(ny):
            for x in range(nx):
                k = y * nx + x
                nb = (psi[y * nx + (x + 1) % nx] + psi[y * nx + (x - 1) % nx]
                      + psi[((y + 1) % ny) * nx + x] + psi[((y - 1) % ny) * nx + x])
                a_psi = -t_hop * nb + v[k] * psi[k]
                n_k = mpmath.re(psi[k]) ** 2 + mpmath.im(psi[k]) ** 2
                out.append(-1j * (a_psi + gs[k] * n_k * psi[k]))
        return out
    return f
