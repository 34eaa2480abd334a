"""Galerkin bases for the boundary conditions of the integration method
(oracle; test infrastructure only).

Paper Sect. 3.2.2 and Appendix B.  Instead of tau rows on top of the
operator, the unknowns are expanded on functions that satisfy the boundary
conditions already:

  * Psi (eq. bc_varPsi, bc_d3psi): phi_n = sum_{i=0}^{4} gamma_i^n T_{n+i},
    with gamma_0^n = 1 and gamma_1..4^n the closed forms of Appendix B
    (they make phi_n vanish at x = +-1, its first derivative vanish at
    x = -1 and its third derivative vanish at x = +1);
  * zonal flow and temperature (Dirichlet at both walls, eq.
    galerkin_dirichlet): phi_n = T_{n+2} - T_n.

With Chebyshev coefficients y = S y~ (S the stencil matrix, K x (K - q),
q = 4 or 2 boundary conditions), a system (mass - a dt L) y = r becomes
P_q (mass - a dt L) S y~ = P_q r (eq. psiint_galerkin, uphi_galerkin,
temp_galerkin): P_q drops the first q rows, which are exactly the rows the
tau method overwrites with boundary rows, so the right-hand sides of the
two formulations are the same vectors.  The square (K - q) system is a
pure band: for Psi 8 sub- and 12 super-diagonals (the paper's Fig. 1c),
for the Dirichlet systems 4 and 6.  It is factored as a band LU (LAPACK
?gbtrf with partial pivoting, as the paper does, or the plain band LU
without interchanges of oracle.bordered), and the state is returned as
Chebyshev coefficients S y~.

Readings:
  * The Dirichlet set has K - 2 members, n = 0..K-3 (T_{K-1} the highest
    polynomial, as the Psi set's n = 0..K-5 reaches T_{K-1}); the paper's
    bound n < N_r - 3 is one short of the set that spans every K-mode
    function with the two boundary values zero.
  * The Psi set's boundary conditions are the tau rows of the tau method
    (Dirichlet at both walls, d^3/dx^3 at x = +1, d/dx at x = -1), so both
    formulations solve for the same Chebyshev coefficients: the K-mode
    functions satisfying the q conditions are exactly the span of S, and
    the remaining K - q equations are the same rows.
"""
from fractions import Fraction

import numpy as np
import scipy.sparse as sp

from .bordered import BandLU

# Band widths of the Galerkin systems: (sub-, super-diagonals).
BAND_PSI = (8, 12)
BAND_DIRICHLET = (4, 6)


def gamma_psi(n):
    """(gamma_0^n, .., gamma_4^n) of Appendix B for the Psi basis; n may be
    an int (exact Fractions) or a float array (floating point)."""
    if isinstance(n, (int, np.integer)):
        n = Fraction(int(n))
        one = Fraction(1)
    else:
        n = np.asarray(n, dtype=np.float64)
        one = np.ones_like(n)
    q = 2 * n**4 + 20 * n**3 + 78 * n**2 + 140 * n + 95
    g1 = 8 * (n + 1) * (n**2 + 4 * n + 5) / q
    g2 = -2 * (n + 2) * (2 * n**4 + 16 * n**3 + 58 * n**2 + 104 * n + 75) / (
        (n + 3) * q)
    g3 = -g1
    g4 = (n + 1) * (2 * n**4 + 12 * n**3 + 30 * n**2 + 36 * n + 15) / (
        (n + 3) * q)
    return one, g1, g2, g3, g4


def stencil_psi(K):
    """S_Psi, K x (K - 4): column n holds gamma_i^n in rows n + i."""
    n = np.arange(K - 4)
    g = gamma_psi(n.astype(np.float64))
    rows = np.concatenate([n + i for i in range(5)])
    cols = np.concatenate([n] * 5)
    vals = np.concatenate([np.broadcast_to(gi, n.shape) for gi in g])
    return sp.csr_matrix((vals, (rows, cols)), shape=(K, K - 4))


def stencil_dirichlet(K):
    """S_D, K x (K - 2): column n is T_{n+2} - T_n."""
    n = np.arange(K - 2)
    rows = np.concatenate([n, n + 2])
    cols = np.concatenate([n, n])
    vals = np.concatenate([-np.ones(K - 2), np.ones(K - 2)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(K, K - 2))


class GalerkinSolver:
    """(mass - a dt L) y = r on the Galerkin basis: op is the K x K
    operator (rows q.. meaningful), S the stencil; solve() takes the full
    K-vector right-hand side (its first q rows are dropped) and returns
    Chebyshev coefficients."""

    def __init__(self, op, S, band, pivot=True):
        op = np.asarray(op)
        self.q = S.shape[0] - S.shape[1]
        self.S = S
        G = np.asarray((sp.csr_matrix(op[self.q:]) @ S).todense())
        kl, ku = band
        i, j = np.nonzero(G)
        d = j - i
        if d.min() < -kl or d.max() > ku:
            raise ValueError("Galerkin matrix wider than its stated band")
        self.G = G
        self.lu = BandLU(G, pivot)

    def solve(self, f):
        f = np.asarray(f)
        x = self.lu.solve(f[self.q:])
        return self.S @ x
