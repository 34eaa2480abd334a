"""Chebyshev-collocation CNAB2 step (oracle cross-check; test
infrastructure only).

The paper's first radial scheme (Sect. 3.1, eq. psiomcoll, tempcoll,
uphicoll): grid values on the N_r Gauss-Lobatto points, derivatives by the
collocation differentiation matrix, boundary conditions imposed on the
boundary rows.  Written, like the eigen-solver, for the regularised Psi
with the two-field splitting G = L_I Psi (no operator above second order is
differentiated in time), no Ekman pumping:
    G rows (interior):     dG/dt = Lap_m G + (2/E) i m Psi
                                   + (Ra/Pr)(i m/s_o) theta + N_omega
    Psi rows (interior):   0 = G - L_I Psi
    boundary rows:         Psi(s_o) = Psi(s_i) = 0 (G block),
                           Psi'''(s_o) = 0, Psi'(s_i) = 0 (Psi block)
    theta rows (interior): dtheta/dt = (1/Pr) Lap_m theta - N_theta,
                           theta = 0 on both boundaries
    zonal flow (interior): du/dt = Lap_1 u - N_uphi, u = 0 on both
                           boundaries.
The advection terms are evaluated on the (s, phi) grid from the grid
values and the differentiation matrix (omega = -G, d_s omega = -D G; the
zonal vorticity u' + u/s), without radial dealiasing; buoyancy and
advection explicit (CNAB2, E^{-1} := E^0); the algebraic rows are imposed
at the new time level.  It shares the operator definitions and the
azimuthal transforms with the integration oracle, not its radial
discretisation, so the two steps agree to the truncation error of either.
"""
import numpy as np

from . import grid, transforms as tr
from .eigen import cheb_diff_matrix
from .operators import evaluate_op, laplacian_m, qg_operators


class CollocationCNAB2:
    def __init__(self, E, Ra, Pr, eta, n_phi, n_r):
        self.E, self.Ra, self.Pr, self.eta = E, Ra, Pr, eta
        self.n_phi, self.N = n_phi, n_r
        self.M = n_phi // 3 + 1
        self.s_i, self.s_o = grid.radii(eta)
        self.s = grid.s_nodes(eta, n_r)
        self.h2 = self.s_o**2 - self.s**2
        self.dtc = grid.dtc_ds(self.s, eta)
        Dx = cheb_diff_matrix(n_r) / (0.5 * (self.s_o - self.s_i))
        self.Dp = [np.eye(n_r), Dx, Dx @ Dx, Dx @ Dx @ Dx]
        self.defs = qg_operators(eta)
        self._lhs = {}
        self._hist = None

    # -------------------------------------------------------------- state
    def set_state(self, Psi, theta, u):
        """Grid values: Psi, theta (M, N) complex, u (N,) real."""
        self.Psi = np.array(Psi, np.complex128)
        self.theta = np.array(theta, np.complex128)
        self.u = np.array(u, np.float64)
        self.G = np.zeros_like(self.Psi)
        for m in range(1, self.M):
            self.G[m] = self._LI(m) @ self.Psi[m]
        self._hist = None

    def _LI(self, m):
        return evaluate_op(self.defs["L_I"], m, self.Dp, self.s[:, None])

    def _lap(self, m):
        return evaluate_op(laplacian_m(), m, self.Dp, self.s[:, None])

    # ---------------------------------------------------------- explicit
    def explicit(self):
        N, M, n_phi = self.N, self.M, self.n_phi
        D = self.Dp[1]
        s = self.s
        im = 1j * np.arange(M)[:, None]
        Psi, G, th, u = self.Psi, self.G, self.theta, self.u
        dPsi = Psi @ D.T
        us = (self.h2 / s) * im * Psi
        uph = -self.h2 * dPsi + 3.0 * s * Psi
        uph[0] += u
        om = -G
        om[0] = D @ u + u / s
        dom = om @ D.T
        dth = th @ D.T

        def g(c):
            return tr.phi_to_grid(c.T, n_phi)
        us_g, uph_g, om_g = g(us), g(uph), g(om)
        n_om = (us_g * g(dom) + uph_g / s[:, None] * g(im * om)
                + om_g * g(im * Psi))
        n_th = us_g * (g(dth) + self.dtc[:, None]) + uph_g / s[:, None] * g(im * th)
        n_u = np.mean(us_g * om_g, axis=1)
        Nom = tr.grid_to_phi(n_om, M).T
        Nth = tr.grid_to_phi(n_th, M).T
        Nth[0] = Nth[0].real
        EG = (self.Ra / self.Pr) * im / self.s_o * th + Nom
        EG[0] = 0.0
        return EG, -Nth, -n_u

    # ------------------------------------------------------------ implicit
    def _systems(self, a):
        """LHS matrices of (mass - a L) with algebraic and boundary rows."""
        if a in self._lhs:
            return self._lhs[a]
        N = self.N
        I = np.eye(N)
        psi_sys = [None]
        for m in range(1, self.M):
            A = np.zeros((2 * N, 2 * N), np.complex128)
            A[:N, :N] = I - a * self._lap(m)
            A[:N, N:] = -a * (2.0j * m / self.E) * I
            A[N:, :N] = I
            A[N:, N:] = -self._LI(m)
            for row, vec in ((0, I[0]), (N - 1, I[-1])):        # Psi = 0
                A[row] = 0
                A[row, N:] = vec
            for row, vec in ((N, self.Dp[3][0]), (2 * N - 1, self.Dp[1][-1])):
                A[row] = 0
                A[row, N:] = vec
            psi_sys.append(A)
        th_sys = []
        for m in range(self.M):
            A = (I - a * self._lap(m) / self.Pr).astype(np.complex128)
            A[0], A[-1] = I[0], I[-1]
            th_sys.append(A)
        Au = I - a * self._lap(1)
        Au[0], Au[-1] = I[0], I[-1]
        self._lhs = {a: (psi_sys, th_sys, Au)}
        return self._lhs[a]

    def step(self, dt):
        N = self.N
        EG, Et, Eu = self.explicit()
        pG, pt, pu = (EG, Et, Eu) if self._hist is None else self._hist
        a = 0.5 * dt
        psi_sys, th_sys, Au = self._systems(a)
        newG = np.zeros_like(self.G)
        newP = np.zeros_like(self.Psi)
        for m in range(1, self.M):
            lin = self._lap(m) @ self.G[m] + (2.0j * m / self.E) * self.Psi[m]
            r = np.zeros(2 * N, np.complex128)
            r[:N] = self.G[m] + a * lin + dt * (1.5 * EG[m] - 0.5 * pG[m])
            r[0] = r[N - 1] = 0.0           # boundary rows; Psi rows are 0
            x = np.linalg.solve(psi_sys[m], r)
            newG[m], newP[m] = x[:N], x[N:]
        newT = np.zeros_like(self.theta)
        for m in range(self.M):
            r = (self.theta[m] + a * (self._lap(m) @ self.theta[m]) / self.Pr
                 + dt * (1.5 * Et[m] - 0.5 * pt[m]))
            r[0] = r[-1] = 0.0
            newT[m] = np.linalg.solve(th_sys[m], r)
        newT[0] = newT[0].real
        r = self.u + a * (self._lap(1) @ self.u) + dt * (1.5 * Eu - 0.5 * pu)
        r[0] = r[-1] = 0.0
        self.u = np.linalg.solve(Au, r)
        self.G, self.Psi, self.theta = newG, newP, newT
        self._hist = (EG, Et, Eu)
