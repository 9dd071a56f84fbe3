"""Plain FP64 CPU oracle for one MB4 time step on the periodic 2D lattice NLS.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import or run this module; the product path never does.
It shares no code with the GPU library: its method constants are computed
here, numerically, from the paper's definitions, and it takes only the seeded
problem inputs (potential, initial state) from the input generator.

What it computes, following Sakai et al., "A Parallelizable Energy-Preserving
Integrator MB4 and Its Application to Quantum-Mechanical Wavepacket Dynamics"
(arXiv 2003.04345):

* the CSRK coefficient polynomial A_{tau,zeta} of MB4 (Sec. 2.2, Eq. Adefinition);
* the Lagrange form of the stage polynomial on c_0 = 0, c_1, c_2, c_3
  (Eq. Lagrange);
* E_ij and E_i0 (Eqs. defE, Ei0) and the eigendecomposition E = T Lambda T^-1
  (Eq. Newton3; Algorithm 1, first two steps);
* the coefficients of the cubic homogeneous polynomial that gives the stage
  integrals of the nonlinear term (Eq. fIu2; Algorithm 1, third step);
* the residual Phi(U) (Eq. Phidefinition, with Eqs. fKu2 and fIu2);
* the frozen Jacobian J at u_0 (Eqs. Jacobianall, JL, JR);
* the simplified Newton loop with the three decoupled stage solves
  (Eqs. MB4_4 - MB4_6; Algorithm 1, time loop and Newton loop);
* the energy H = U_K + U_I + U_E (Sec. 2.1, Eqs. U_K - U_E).

Conventions.  The state is complex psi (paper's u) with Re/Im = (p, q).  The
flow is i psi' = (A + g |psi|^2) psi with A = K + V, K the periodic
nearest-neighbour hopping (-t per link) plus an optional diagonal shift, V the
on-site potential.  In the paper's notation (Eq. dNLS) this is gamma = -g;
the paper's K = -Laplacian_h is the case t = 1/h_x^2, shift = 4 t.  Energies
are reported in the library's convention H = (U_K + U_I + U_E) / 2, i.e. half
the paper's H, so that the flow reads u' = S grad H with S = [[0, I], [-I, 0]].

Readings of points the paper leaves open (each one listed in the design
notes): the Newton loop stops once ||r^l||_inf <= eps, an absolute bound as in
Algorithm 1 (eps = 1e-13 in Sec. 3), or, with relative=True, once
||r^l||_inf <= eps * ||u_0||_inf; the initial Newton guess is e_3 (x) u_0;
eigenvalues are sorted ascending.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# Sec. 3, computational conditions: alpha_1 = -300 * 19/8, c = (1/3, 2/3, 1).
# Kept as exact rationals: the constants of the method are computed in exact
# arithmetic and rounded once, because alpha_1 is large and the polynomial
# integrals cancel heavily in floating point.
ALPHA1_PAPER = Fraction(-300) * Fraction(19, 8)
C_PAPER = (Fraction(1, 3), Fraction(2, 3), Fraction(1))
EPS_PAPER = 1e-13


class NewtonDivergence(RuntimeError):
    """The simplified Newton loop did not converge (Sec. 2.2, last paragraphs)."""


# ---------------------------------------------------------------------------
# Method constants (Sec. 2.2), in exact rational arithmetic
# ---------------------------------------------------------------------------
# A polynomial is a list of Fractions, coefficient k multiplying zeta^k.

def _pmul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _pint01(a) -> Fraction:
    """Integral over [0, 1]: sum of a_k / (k + 1)."""
    return sum((x / (k + 1) for k, x in enumerate(a)), Fraction(0))


def _peval(a, z):
    return sum((x * z ** k for k, x in enumerate(a)), Fraction(0))


def csrk_middle_matrix(alpha1) -> list:
    """The 3x3 matrix between [tau, tau^2/2, tau^3/3] and [1, zeta, zeta^2]^T
    in the definition of A_{tau,zeta} (Eq. Adefinition)."""
    a = Fraction(alpha1)
    return [[a + 4, -6 * a - 6, 6 * a],
            [-6 * a - 6, 36 * a + 12, -36 * a],
            [6 * a, -36 * a, 36 * a]]


def a_of_tau(tau, alpha1) -> list:
    """A_{tau,zeta} as a polynomial in zeta for a fixed tau (Eq. Adefinition)."""
    tau = Fraction(tau)
    m = csrk_middle_matrix(alpha1)
    left = [tau, tau ** 2 / 2, tau ** 3 / 3]
    return [sum((left[r] * m[r][col] for r in range(3)), Fraction(0)) for col in range(3)]


def lagrange_basis(nodes) -> list:
    """l_j with l_j(c_k) = delta_jk on the nodes c_0 .. c_3 (Eq. Lagrange)."""
    nodes = [Fraction(x) for x in nodes]
    basis = []
    for j, cj in enumerate(nodes):
        lj = [Fraction(1)]
        for k, ck in enumerate(nodes):
            if k != j:
                lj = _pmul(lj, [-ck / (cj - ck), 1 / (cj - ck)])
        basis.append(lj)
    return basis


@dataclass
class MB4Constants:
    alpha1: Fraction
    c: tuple
    E_full: np.ndarray      # (3, 4): columns j = 0..3, E_full[:, 0] = E_i0
    E: np.ndarray           # (3, 3): E_ij, i, j = 1..3
    lam: np.ndarray         # (3,) eigenvalues of E, ascending
    T: np.ndarray           # (3, 3) eigenvectors as columns
    Tinv: np.ndarray
    cubic: np.ndarray       # (3, 4, 4, 4): int A_{c_i,z} l_a l_b l_d dz
    E_exact: list           # the same E_full as Fractions


def method_constants(alpha1=ALPHA1_PAPER, c=C_PAPER) -> MB4Constants:
    """Algorithm 1, first three steps: E, its eigendecomposition and the
    coefficients of the cubic stage polynomial."""
    nodes = [Fraction(0)] + [Fraction(x) for x in c]
    ell = lagrange_basis(nodes)
    a_ci = [a_of_tau(ci, alpha1) for ci in nodes[1:]]
    # Eqs. defE and Ei0: E_ij = int_0^1 A_{c_i,zeta} l_j(zeta) dzeta, j = 0..3.
    e_exact = [[_pint01(_pmul(a_ci[i], ell[j])) for j in range(4)] for i in range(3)]
    e_full = np.array([[float(x) for x in row] for row in e_exact])
    e = e_full[:, 1:].copy()
    # Eq. Newton3: E = T Lambda T^-1; the eigenvalues are real (the paper
    # cites Theorem 5.1 of Miyatake and Butcher for this).
    lam, t = np.linalg.eig(e)
    if np.max(np.abs(np.imag(lam))) > 1e-12:
        raise ValueError("E has complex eigenvalues for these constants")
    order = np.argsort(np.real(lam))
    lam = np.real(lam)[order]
    t = np.real(t)[:, order]
    # The scaling of each eigenvector is free (the Newton root does not depend
    # on it); fix the sign so that the first row is positive, as the GPU side
    # does, which makes the transformed quantities of both sides comparable.
    t = t * np.where(t[0, :] < 0, -1.0, 1.0)[None, :]
    tinv = np.linalg.inv(t)
    # Eq. fIu2: |U_z|^2 U_z = sum_{a,b,d} conj(Y_a) Y_b Y_d l_a l_b l_d with
    # Y_0 = u_0, Y_j = U_{c_j}; the coefficient of each product in stage i
    # is the integral of a degree-11 polynomial.
    cubic = np.zeros((3, 4, 4, 4))
    for a in range(4):
        for b in range(4):
            lab = _pmul(ell[a], ell[b])
            for d in range(4):
                labd = _pmul(lab, ell[d])
                for i in range(3):
                    cubic[i, a, b, d] = float(_pint01(_pmul(a_ci[i], labd)))
    return MB4Constants(alpha1=Fraction(alpha1), c=tuple(nodes[1:]), E_full=e_full,
                        E=e, lam=lam, T=t, Tinv=tinv, cubic=cubic, E_exact=e_exact)


# ---------------------------------------------------------------------------
# The lattice problem (Sec. 2.1 and Sec. 2.3)
# ---------------------------------------------------------------------------

def hopping_matrix(nx: int, ny: int, t_hop: float, diag_shift: float = 0.0) -> sp.csr_matrix:
    """K: -t between the four periodic nearest neighbours, plus shift * I.

    Site (x, y) has index y * nx + x.  With t = 1/h^2 and shift = 4/h^2 this is
    the paper's 5-point periodic K = -Laplacian_h (Eq. Kdefinition, h_x = h_y).
    """
    s = nx * ny
    idx = np.arange(s)
    x = idx % nx
    y = idx // nx
    rows, cols = [], []
    for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        rows.append(idx)
        cols.append(((y + dy) % ny) * nx + (x + dx) % nx)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.full(rows.shape, -float(t_hop))
    k = sp.coo_matrix((vals, (rows, cols)), shape=(s, s)).tocsr()
    k.sum_duplicates()
    if diag_shift != 0.0:
        k = k + float(diag_shift) * sp.identity(s, format="csr")
    return k.tocsr()


class LatticeNLS:
    """i psi' = (K + V) psi + g |psi|^2 psi on an nx x ny periodic lattice.

    g is one number, or one per site: the site-dependent nonlinearity of the
    Appendix, U_I = -1/2 sum_i gamma_i n_i^2 (gamma_i = -g_i), for which the
    energy U_K + U_E + U_I is conserved all the same.
    """

    def __init__(self, nx, ny, potential, g, t_hop=1.0, diag_shift=0.0):
        if nx < 3 or ny < 3:
            raise ValueError("lattice sides must be at least 3")
        self.nx, self.ny = int(nx), int(ny)
        self.s = self.nx * self.ny
        self.v = np.asarray(potential, dtype=np.float64).reshape(self.s)
        if np.ndim(g) == 0:
            self.g = float(g)
        else:
            self.g = np.asarray(g, dtype=np.float64).reshape(self.s).copy()
        self.gamma = -self.g                     # paper's gamma (Eq. dNLS)
        self.t_hop = float(t_hop)
        self.diag_shift = float(diag_shift)
        self.K = hopping_matrix(self.nx, self.ny, self.t_hop, self.diag_shift)
        self.A = (self.K + sp.diags(self.v)).tocsr()   # A = K + V (Eq. JL)

    # Eqs. fdivide - fEu: f = -i K u + i gamma |u|^2 u - i V u.
    def f(self, u: np.ndarray) -> np.ndarray:
        return -1j * (self.A @ u) + 1j * self.gamma * (np.abs(u) ** 2) * u

    def jacobian(self, u0: np.ndarray) -> sp.csr_matrix:
        """J = df/du at u_0 in the real (p, q) variables (Eqs. JL, JR)."""
        p, q = u0.real, u0.imag
        s = self.s
        z = sp.csr_matrix((s, s))
        jl = sp.bmat([[z, self.A], [-self.A, z]])
        gm = self.gamma
        ji = sp.bmat([[sp.diags(gm * (-2.0 * p * q)), sp.diags(gm * (-p * p - 3.0 * q * q))],
                      [sp.diags(gm * (3.0 * p * p + q * q)), sp.diags(gm * (2.0 * p * q))]])
        return (jl + ji).tocsr()

    def energy_components(self, u: np.ndarray) -> dict:
        """Energies of Eqs. U_K - U_E, summed with math.fsum.

        Returned in the library convention (half the paper's values):
        U_K = u^H K u / 2, U_I = (g/4) sum n^2, U_E = u^H V u / 2,
        H = U_K + U_I + U_E; plus the probability sum n and the participation
        ratio sum n^2 (Sec. 3.2) with n = |u|^2.
        """
        n = (u.real ** 2 + u.imag ** 2)
        ku = self.K @ u
        uk_terms = u.real * ku.real + u.imag * ku.imag      # Re(conj(u) K u)
        ue_terms = self.v * n
        ui_terms = n * n
        uk = 0.5 * math.fsum(uk_terms.tolist())
        ue = 0.5 * math.fsum(ue_terms.tolist())
        if np.ndim(self.g) == 0:
            ui = 0.25 * self.g * math.fsum(ui_terms.tolist())
        else:
            ui = 0.25 * math.fsum((self.g * ui_terms).tolist())
        h_total = 0.5 * math.fsum(np.concatenate(
            [uk_terms, ue_terms, 0.5 * self.g * ui_terms]).tolist())
        return {"H": h_total, "U_K": uk, "U_I": ui, "U_E": ue,
                "prob": math.fsum(n.tolist()), "participation": math.fsum(ui_terms.tolist())}

    def energy(self, u: np.ndarray) -> float:
        return self.energy_components(u)["H"]


# ---------------------------------------------------------------------------
# One MB4 step (Algorithm 1)
# ---------------------------------------------------------------------------

class MB4Oracle:
    """Algorithm 1 for one LatticeNLS, literally, one step at a time.

    solver: "direct" factorises I - h lambda_i J once per step with SuperLU
    (the paper uses a sparse direct solver); "gmres" solves each stage system
    with restarted GMRES to a tight tolerance, for lattices too large to
    factorise.  Either way the Newton root is the same; only the iteration
    path differs.
    """

    def __init__(self, problem: LatticeNLS, h: float, eps: float = EPS_PAPER,
                 max_newton: int = 50, constants: MB4Constants | None = None,
                 solver: str = "direct", gmres_rtol: float = 1e-14, relative: bool = False):
        self.prob = problem
        self.h = float(h)
        self.eps = float(eps)
        self.relative = bool(relative)
        self.max_newton = int(max_newton)
        self.k = constants if constants is not None else method_constants()
        self.solver = solver
        self.gmres_rtol = gmres_rtol
        self.last_iterations = 0
        self.iteration_log: list[int] = []

    # Eq. fIu2 with Algorithm 1's precomputed coefficients.
    def nonlinear_stage_integrals(self, u0: np.ndarray, U: np.ndarray) -> np.ndarray:
        ys = (u0, U[0], U[1], U[2])
        out = np.zeros_like(U)
        cub = self.k.cubic
        for a in range(4):
            ya = np.conj(ys[a])
            for b in range(4):
                for d in range(b, 4):
                    prod = ya * ys[b] * ys[d]
                    for i in range(3):
                        coef = cub[i, a, b, d] if b == d else cub[i, a, b, d] + cub[i, a, d, b]
                        out[i] += coef * prod
        return 1j * self.prob.gamma * out

    def residual(self, u0: np.ndarray, U: np.ndarray) -> np.ndarray:
        """Phi(U) of Eq. Phidefinition: U_i - u_0 - h int A_{c_i,z} f(U_z) dz,
        the linear part by Eq. fKu2 and the nonlinear part by Eq. fIu2."""
        e0, e = self.k.E_full[:, 0], self.k.E
        nl = self.nonlinear_stage_integrals(u0, U)
        phi = np.empty_like(U)
        for i in range(3):
            w = e0[i] * u0 + e[i, 0] * U[0] + e[i, 1] * U[1] + e[i, 2] * U[2]
            lin = -1j * (self.prob.A @ w)
            phi[i] = U[i] - u0 - self.h * (lin + nl[i])
        return phi

    def _stage_solvers(self, u0: np.ndarray):
        jac = self.prob.jacobian(u0)
        eye = sp.identity(2 * self.prob.s, format="csc")
        mats = [(eye - self.h * lam_i * jac).tocsc() for lam_i in self.k.lam]
        if self.solver == "direct":
            # COLAMD: with a stiff kinetic operator (h lambda K ~ 7.5 off the
            # diagonal on the 70 x 70 continuum of Sec. 3) partial pivoting
            # under a minimum-degree ordering of A^T + A fills the factors in
            # (about 40 s a factorisation); COLAMD keeps them sparse.
            lus = [spla.splu(m, permc_spec="COLAMD") for m in mats]
            return [lu.solve for lu in lus]
        if self.solver == "gmres":
            def make(m):
                def solve(b):
                    x, info = spla.gmres(m, b, rtol=self.gmres_rtol, atol=0.0,
                                         restart=80, maxiter=2000)
                    if info != 0:
                        raise NewtonDivergence(f"GMRES did not converge (info={info})")
                    return x
                return solve
            return [make(m) for m in mats]
        raise ValueError(f"unknown solver {self.solver}")

    def step(self, u0: np.ndarray) -> np.ndarray:
        """u(t + h) from u(t) (Algorithm 1, body of the time loop)."""
        s = self.prob.s
        solves = self._stage_solvers(u0)             # J frozen at u_0 (Eq. Jacobian2)
        U = np.stack([u0, u0, u0]).astype(np.complex128)   # U^0 = e_3 (x) u_0
        # Stopping test of Algorithm 1: ||r^l||_inf against eps, absolute
        # unless a bound relative to ||u_0||_inf was asked for.
        tol = self.eps
        if self.relative:
            scale = max(float(np.max(np.abs(u0.real), initial=0.0)),
                        float(np.max(np.abs(u0.imag), initial=0.0)))
            tol = self.eps * max(scale, np.finfo(np.float64).tiny)
        r = math.inf
        it = 0
        T, Tinv = self.k.T, self.k.Tinv
        while r > tol:
            if it >= self.max_newton:
                raise NewtonDivergence(
                    f"no convergence in {self.max_newton} iterations (last |r| = {r:.3e})")
            phi = self.residual(u0, U)
            phib = np.tensordot(Tinv, phi, axes=(1, 0))       # Eq. MB4_4
            rbar = np.empty_like(phib)
            for i in range(3):                                  # Eq. MB4_5
                rhs = -np.concatenate([phib[i].real, phib[i].imag])
                x = solves[i](rhs)
                rbar[i] = x[:s] + 1j * x[s:]
            rvec = np.tensordot(T, rbar, axes=(1, 0))          # Eq. MB4_6
            U = U + rvec
            r = max(float(np.max(np.abs(rvec.real))), float(np.max(np.abs(rvec.imag))))
            if not math.isfinite(r):
                raise NewtonDivergence("non-finite Newton update")
            it += 1
        self.last_iterations = it
        self.iteration_log.append(it)
        return U[2].copy()                                     # u_1 = U_{c_3}, c_3 = 1

    def run(self, u0: np.ndarray, steps: int, energy_every: int = 0):
        """steps MB4 steps from u0; returns (u, energies) where energies is a
        list of (step, H) at step 0, every energy_every steps and the end."""
        u = np.asarray(u0, dtype=np.complex128).copy()
        energies = [(0, self.prob.energy(u))]
        for n in range(1, steps + 1):
            u = self.step(u)
            if (energy_every and n % energy_every == 0) or n == steps:
                if energies[-1][0] != n:
                    energies.append((n, self.prob.energy(u)))
        return u, energies


def energy_drift(energies) -> float:
    """max_n |H_n - H_0| / |H_0| over logged energies."""
    h0 = energies[0][1]
    return max(abs(e - h0) for _, e in energies) / abs(h0)


def oracle_for(prob_cfg, potential, eps=EPS_PAPER, max_newton=50, solver="direct",
               constants=None, relative=False, g=None) -> MB4Oracle:
    """Oracle for a lattice_inputs.LatticeProblem-like object; g (one value
    per site) replaces the problem's uniform g when given."""
    lat = LatticeNLS(prob_cfg.nx, prob_cfg.ny, potential, prob_cfg.g if g is None else g,
                     t_hop=prob_cfg.t_hop, diag_shift=prob_cfg.diag_shift)
    return MB4Oracle(lat, prob_cfg.h, eps=eps, max_newton=max_newton,
                     solver=solver, constants=constants, relative=relative)
