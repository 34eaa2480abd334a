"""Linear onset eigen-solver (oracle test tool; test infrastructure only).

Paper Sect. 6.1, eq. (lin): normal modes f_m(s) e^{i m phi + lambda t},
lambda = tau + i omega_d, of the linearised QG equations, here written for
the regularised streamfunction Psi of Sect. 3.2.1 (psi = h^2 Psi), without
Ekman pumping:
    lambda L_I Psi = Lap_m L_I Psi + (2/E) i m Psi + (Ra/Pr)(i m/s_o) theta
    lambda theta   = (1/Pr) Lap_m theta - i m (h^2/s) dTc/ds Psi
with Psi(s_o) = Psi(s_i) = d^3Psi/ds^3(s_o) = dPsi/ds(s_i) = 0 and
theta(s_o) = theta(s_i) = 0.

Discretisation: Chebyshev collocation in physical space on N Gauss-Lobatto
points (the paper solves eq. lin by collocation and the QZ algorithm), with
the two-field splitting G = L_I Psi of the vorticity/streamfunction form
(eq. psiomcoll) so that no operator above second order carries lambda:
    G rows:     lambda G = Lap_m G + (2/E) i m Psi + (Ra/Pr)(i m/s_o) theta,
                boundary rows Psi = 0 at s_o and s_i;
    Psi rows:   0 = G - L_I Psi,
                boundary rows Psi'''(s_o) = 0, Psi'(s_i) = 0;
    theta rows: as above, boundary rows theta = 0.
Readings: the 1/Pr on the diffusion term, missing from eq. (lin) as
printed, follows eq. (temp), as does the sign of the background advection.
"""
import numpy as np
import scipy.linalg as sla

from . import grid
from .operators import evaluate_op, laplacian_m, qg_operators


def cheb_diff_matrix(N):
    """Chebyshev differentiation matrix on x_k = cos(pi k/(N-1))
    (standard construction, diagonal from the negative row sums)."""
    x = grid.gl_nodes(N)
    c = np.ones(N)
    c[0] = c[-1] = 2.0
    c *= (-1.0) ** np.arange(N)
    X = x[:, None] - x[None, :]
    Dm = np.outer(c, 1.0 / c) / (X + np.eye(N))
    Dm -= np.diag(Dm.sum(axis=1))
    return Dm


def linear_operator(E, Ra, Pr, eta, m, N):
    """(A, B), A v = lambda B v, v = (G, Psi, theta) on the grid."""
    s_i, s_o = grid.radii(eta)
    s = grid.s_nodes(eta, N)
    Dx = cheb_diff_matrix(N) / (0.5 * (s_o - s_i))        # d/ds
    Dp = [np.eye(N), Dx, Dx @ Dx, Dx @ Dx @ Dx]
    defs = qg_operators(eta)
    sc = s[:, None]
    LI = evaluate_op(defs["L_I"], m, Dp, sc)
    lap = evaluate_op(laplacian_m(), m, Dp, sc)
    Z = np.zeros((N, N), np.complex128)
    I = np.eye(N)
    A = np.block([[Z, Z, Z], [Z, Z, Z], [Z, Z, Z]])
    B = A.copy()
    g, p, t = slice(0, N), slice(N, 2 * N), slice(2 * N, 3 * N)
    # G rows
    A[g, g] = lap
    A[g, p] = (2.0j * m / E) * I
    A[g, t] = (Ra / Pr) * (1j * m / s_o) * I
    B[g, g] = I
    # Psi rows
    A[p, g] = I
    A[p, p] = -LI
    # theta rows
    A[t, t] = lap / Pr
    h2 = s_o**2 - s**2
    A[t, p] = np.diag(-1j * m * (h2 / s) * grid.dtc_ds(s, eta))
    B[t, t] = I
    # boundary rows (index 0 is s_o, N-1 is s_i); no lambda on them
    for row, blk, vec in ((0, g, np.eye(N)[0]), (N - 1, g, np.eye(N)[-1]),
                          (N, p, Dp[3][0]), (2 * N - 1, p, Dp[1][-1]),
                          (2 * N, t, np.eye(N)[0]),
                          (3 * N - 1, t, np.eye(N)[-1])):
        A[row, :] = 0
        B[row, :] = 0
        if blk is g:      # Psi Dirichlet conditions live in the G block rows
            A[row, N:2 * N] = vec
        else:
            A[row, blk] = vec
    return A, B


def eigenvalues(E, Ra, Pr, eta, m, N):
    A, B = linear_operator(E, Ra, Pr, eta, m, N)
    lam = sla.eig(A, B, right=False)
    return lam[np.isfinite(lam)]


def leading(E, Ra, Pr, eta, m, N):
    """Finite eigenvalue with the largest real part."""
    lam = eigenvalues(E, Ra, Pr, eta, m, N)
    return lam[np.argmax(lam.real)]


def leading_mode(E, Ra, Pr, eta, m, N):
    """Leading eigenvalue with Psi and theta on the N-point grid."""
    A, B = linear_operator(E, Ra, Pr, eta, m, N)
    lam, vec = sla.eig(A, B)
    ok = np.isfinite(lam)
    i = np.flatnonzero(ok)[np.argmax(lam[ok].real)]
    return lam[i], vec[N:2 * N, i], vec[2 * N:, i]


def critical_rayleigh(E, Pr, eta, m, N, lo, hi, rtol=1e-8):
    """Ra at which the leading growth rate of mode m changes sign."""
    def g(ra):
        return leading(E, ra, Pr, eta, m, N).real
    if g(lo) > 0 or g(hi) < 0:
        raise ValueError("bracket does not contain the onset")
    while hi - lo > rtol * hi:
        mid = 0.5 * (lo + hi)
        if g(mid) > 0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def integration_operator(E, Ra, Pr, eta, m, K):
    """(A, B) for the same eigenproblem posed with the integration-method
    matrices of Sect. 3.2 (eq. psi_int, temp_int) and their tau rows:
        lambda [A_m Psi; D theta] = [B_m Psi + C (Ra/Pr)(i m/s_o) theta;
                                     (1/Pr) F_m theta - i m D_bg Psi],
    D_bg = int^2 s^2 (h^2/s) dTc/ds = (alpha/ln eta) int^2 h^2 (exact, the
    background coefficient times s^2 being a polynomial)."""
    from .operators import (PAD, ChebAlgebra, IntegrationOperators,
                            tau_rows_dirichlet, tau_rows_psi)
    s_i, s_o = grid.radii(eta)
    o = IntegrationOperators(eta, K)
    alg = ChebAlgebra(eta, K + PAD)
    c = grid.alpha_tc(eta) / np.log(eta)
    dbg = alg.integrated({0: {(0, 0): c * s_o**2, (2, 0): -c}}, 2)[0]
    dbg = np.asarray(dbg[:K, :K].todense())
    A = np.zeros((2 * K, 2 * K), np.complex128)
    B = np.zeros_like(A)
    A[:K, :K] = o.B(m, E)
    A[:K, K:] = (Ra / Pr) * (1j * m / s_o) * o.C
    B[:K, :K] = o.A(m)
    A[K:, K:] = o.F(m) / Pr
    A[K:, :K] = -1j * m * dbg
    B[K:, K:] = o.D
    A[:4, :] = 0
    B[:4, :] = 0
    A[:4, :K] = tau_rows_psi(K)
    A[K:K + 2, :] = 0
    B[K:K + 2, :] = 0
    A[K:K + 2, K:] = tau_rows_dirichlet(K)
    return A, B


def integration_leading(E, Ra, Pr, eta, m, K):
    """Leading eigenvalue; rows are equilibrated first (the integrated rows
    scale like k^-4), which leaves the eigenvalues unchanged."""
    A, B = integration_operator(E, Ra, Pr, eta, m, K)
    sc = 1.0 / np.maximum(np.abs(A).max(axis=1), np.abs(B).max(axis=1))
    lam = sla.eig(A * sc[:, None], B * sc[:, None], right=False)
    lam = lam[np.isfinite(lam)]
    return lam[np.argmax(lam.real)]
