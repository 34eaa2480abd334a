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

Ekman pumping (optional, `pumping=True`): the G rows gain -F with
F = -Upsilon [omega - (beta/2) u_phi + beta (d/dphi - 5 s_o/(2h)) u_s]
(eq. pumping_full), Upsilon = (s_o/E)^{1/2} (s_o^2 - s^2)^{-3/4}; written
for Psi (omega = -G, u_phi = -h^2 Psi' + 3 s Psi, u_s = (h^2/s) i m Psi,
beta = -s/h^2) it is
    F = Upsilon [G + (s/2) Psi' - (3 s^2/(2 h^2) + m^2 + 5 i m s_o/(2h)) Psi],
evaluated at the interior points only (Upsilon is singular at s_o, where
the boundary rows stand).  The integration-method operators take the
approximated form F_eps of eq. approx_pump (h -> h_eps = ((s_o + eps)^2 -
s^2)^{1/2} in Upsilon and in the bracket's coefficients, L_I unchanged),
projected on the Chebyshev basis through the n_r-point grid as the time
step evaluates it (an explicit term there).
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


def linear_operator(E, Ra, Pr, eta, m, N, pumping=False):
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
    if pumping:
        h2 = s_o**2 - s**2
        ii = np.arange(1, N - 1)                 # interior points
        ups = np.sqrt(s_o / E) / h2[ii]**0.75
        coef = 1.5 * s[ii]**2 / h2[ii] + m * m + 2.5j * m * s_o / np.sqrt(h2[ii])
        A[ii, ii] -= ups
        A[ii, N:2 * N] -= (0.5 * ups * s[ii])[:, None] * Dx[ii]
        A[ii, N + ii] += ups * coef
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


def eigenvalues(E, Ra, Pr, eta, m, N, pumping=False):
    A, B = linear_operator(E, Ra, Pr, eta, m, N, pumping)
    lam = sla.eig(A, B, right=False)
    return lam[np.isfinite(lam)]


def leading(E, Ra, Pr, eta, m, N, pumping=False):
    """Finite eigenvalue with the largest real part."""
    lam = eigenvalues(E, Ra, Pr, eta, m, N, pumping)
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


def pumping_matrix(E, eta, m, K, n_r, eps):
    """Chebyshev coefficients (n < K) of F_eps(Psi) for Psi = T_n, n < K,
    evaluated on the n_r-point radial grid (eq. approx_pump)."""
    from . import transforms as tr
    s_i, s_o = grid.radii(eta)
    s = grid.s_nodes(eta, n_r)
    he2 = (s_o + eps)**2 - s**2
    he = np.sqrt(he2)
    ups = np.sqrt(s_o / E) / he**1.5
    LI = qg_operators(eta)["L_I"]
    F = np.zeros((K, K), np.complex128)
    for n in range(K):
        e = np.zeros(K)
        e[n] = 1.0
        P = [tr.cheb_to_grid(tr.cheb_ds(e, q), n_r) for q in range(4)]
        f = ups * (evaluate_op(LI, m, P, s) + 0.5 * s * P[1]
                   - (1.5 * s**2 / he2 + m * m + 2.5j * m * s_o / he) * P[0])
        F[:, n] = tr.grid_to_cheb(f, K)
    return F


def integration_operator(E, Ra, Pr, eta, m, K, pump=None):
    """(A, B) for the same eigenproblem posed with the integration-method
    matrices of Sect. 3.2 (eq. psi_int, temp_int) and their tau rows:
        lambda [A_m Psi; D theta] = [B_m Psi + C (Ra/Pr)(i m/s_o) theta;
                                     (1/Pr) F_m theta - i m D_bg Psi],
    D_bg = int^2 s^2 (h^2/s) dTc/ds = (alpha/ln eta) int^2 h^2 (exact, the
    background coefficient times s^2 being a polynomial).  pump = (n_r, eps)
    adds -C F_eps to the Psi rows (pumping_matrix)."""
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
    if pump is not None:
        A[:K, :K] -= o.C @ pumping_matrix(E, eta, m, K, *pump)
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
