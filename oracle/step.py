"""One IMEX step of the spherical QG equations, integration method + tau
(oracle; test infrastructure only).

Equations (paper Sect. 2 and 3.2), without Ekman pumping (for the optional
explicit pumping see the last reading below):
  Psi, m >= 1 (eq. psi_int):
    d/dt A_m Psi - B_m Psi = C [ (Ra/Pr)(i m/s_o) theta_m + N_omega,m ]
  theta, m >= 0 (eq. temp_int):
    d/dt D theta - (1/Pr) F_m theta = -D [ i m (h^2/s dTc/ds Psi)_m + N_theta,m ]
  zonal flow (eq. uphi_int):
    d/dt D u - E u = -D [ N_uphi ],   N_uphi = mean over phi of u_s omega
with tau boundary rows on top of every matrix.

Readings (where the paper is silent or inconsistent):
  * Nonlinear terms are evaluated pointwise on the (s, phi) grid.  By QG
    continuity (eq. cont) div(u f) = u.grad f - beta u_s f, and
    -beta u_s = dPsi/dphi exactly (beta h^2/s = -1), so
      N_omega = u_s d_s omega + (u_phi/s) d_phi omega + omega dPsi/dphi,
      N_theta = u_s (d_s theta + dTc/ds) + (u_phi/s) d_phi theta,
    the second one carrying the background advection u_s dTc/ds of eq. temp.
  * Buoyancy and background advection are explicit (allowed by Sect. 4),
    unless buoyancy="implicit": then the buoyancy term (Ra/Pr)(i m/s_o) C
    theta belongs to the implicit operator L (and leaves E_psi), and every
    implicit solve advances theta first and then Psi with the new theta's
    buoyancy on its right-hand side (the order Sect. 4 gives: the
    temperature system does not involve Psi, so the coupled system is
    block triangular).
  * Chebyshev coefficients n >= N_c of every nonlinear term are zeroed
    (radial dealiasing, Sect. 3.2.1); N_c = floor(2(N_r-1)/3) by default.
  * Multistep schemes carry the mass matrix (A_m or D) on both sides of
    eq. (multistep1), as the paper shows for the DIRK case (Sect. 4).
  * CNAB2 starts with E^{n-1} := E^n.
  * BPR353: the tableau of Boscarino, Pareschi & Russo (2013, Sect. 8.3),
    five stages, a_ii = 1/2, first stage explicit, stiffly accurate.
  * ARS222 and ARS443 (Table 1): the stiffly accurate SDIRK tableaux of
    Ascher, Ruuth & Spiteri (1997, Sects. 2.6 and 2.8); a_ii = 1 - 1/sqrt 2
    and 1/2.
  * SBDF2, SBDF3, SBDF4 (Table 1): the semi-implicit backward-difference
    schemes sum_j a_j y^{n+1-j} = dt (L y^{n+1} + sum_j b_j E^{n+1-j}), with
    the mass matrix on every y (as for CNAB2).  They are not self-starting:
    SBDFk takes BPR353 steps until k levels are stored, which keeps the
    global order k for k <= 4.
  * A multistep history belongs to the scheme and dt that made it: a step
    with another scheme or dt starts afresh.
  * Ekman pumping (optional, ekman_eps = eps > 0), explicit like the
    advection (Sect. 3.2: its coefficients are not rational): E_psi gains
    -C[F_eps], F_eps = Upsilon_eps [L_I + (s/2) d/ds - (3 s^2/(2 h_eps^2)
    + m^2 + 5 i m s_o/(2 h_eps))] Psi (eq. approx_pump), and the zonal flow
    -D[Upsilon_eps u + (E/2) Upsilon_eps u omega_0] (the pumping term of
    eq. uphi and the self-interaction of the zonal wind in N_uphi, with
    Upsilon_eps for Upsilon as the integration method needs), all
    evaluated on the radial grid and transformed with the other explicit
    terms.
"""
import numpy as np
import scipy.sparse as sp

from . import grid, transforms as tr
from .bordered import BorderedSolver
from .galerkin import (BAND_DIRICHLET, BAND_PSI, GalerkinSolver,
                       stencil_dirichlet, stencil_psi)
from .operators import (D1, IntegrationOperators, bordered_lhs, evaluate_op,
                        mono, mult, op_compose, qg_operators,
                        tau_rows_dirichlet, tau_rows_psi)

# CNAB2 (Sect. 4, eq. multistep1): a = (1, 0), b^I = (1/2, 1/2),
# b^E = (3/2, -1/2).
CNAB2_BI0 = 0.5

# BPR353 Butcher tables (explicit A^E, implicit A^I), stiffly accurate.
BPR353_AE = np.array([[0, 0, 0, 0, 0],
                      [1, 0, 0, 0, 0],
                      [4 / 9, 2 / 9, 0, 0, 0],
                      [1 / 4, 0, 3 / 4, 0, 0],
                      [1 / 4, 0, 3 / 4, 0, 0]], dtype=np.float64)
BPR353_AI = np.array([[0, 0, 0, 0, 0],
                      [1 / 2, 1 / 2, 0, 0, 0],
                      [5 / 18, -1 / 9, 1 / 2, 0, 0],
                      [1 / 2, 0, 0, 1 / 2, 0],
                      [1 / 4, 0, 3 / 4, -1 / 2, 1 / 2]], dtype=np.float64)


# ARS(2,2,2) (Ascher, Ruuth & Spiteri 1997, Sect. 2.6): gamma = 1 - 1/sqrt 2,
# delta = 1 - 1/(2 gamma); first stage explicit, stiffly accurate.
_GAM = 1.0 - 1.0 / np.sqrt(2.0)
_DEL = 1.0 - 1.0 / (2.0 * _GAM)
ARS222_AE = np.array([[0, 0, 0],
                      [_GAM, 0, 0],
                      [_DEL, 1 - _DEL, 0]], dtype=np.float64)
ARS222_AI = np.array([[0, 0, 0],
                      [0, _GAM, 0],
                      [0, 1 - _GAM, _GAM]], dtype=np.float64)

# ARS(4,4,3) (same paper, Sect. 2.8): a_ii = 1/2, stiffly accurate.
ARS443_AE = np.array([[0, 0, 0, 0, 0],
                      [1 / 2, 0, 0, 0, 0],
                      [11 / 18, 1 / 18, 0, 0, 0],
                      [5 / 6, -5 / 6, 1 / 2, 0, 0],
                      [1 / 4, 7 / 4, 3 / 4, -7 / 4, 0]], dtype=np.float64)
ARS443_AI = np.array([[0, 0, 0, 0, 0],
                      [0, 1 / 2, 0, 0, 0],
                      [0, 1 / 6, 1 / 2, 0, 0],
                      [0, -1 / 2, 1 / 2, 1 / 2, 0],
                      [0, 3 / 2, -3 / 2, 1 / 2, 1 / 2]], dtype=np.float64)

DIRK = {"bpr353": (BPR353_AE, BPR353_AI),
        "ars222": (ARS222_AE, ARS222_AI),
        "ars443": (ARS443_AE, ARS443_AI)}

# SBDFk: a = (a_0 .. a_k) on y^{n+1} .. y^{n+1-k}, b = (b_1 .. b_k) on
# E^n .. E^{n+1-k} (backward-difference formulas of orders 2, 3, 4 with
# explicit terms extrapolated to the same order).
SBDF = {"sbdf2": ((3 / 2, -2, 1 / 2), (2, -1)),
        "sbdf3": ((11 / 6, -3, 3 / 2, -1 / 3), (3, -3, 1)),
        "sbdf4": ((25 / 12, -4, 3, -4 / 3, 1 / 4), (4, -6, 4, -1))}

SCHEMES = ("cnab2", "sbdf2", "sbdf3", "sbdf4", "bpr353", "ars222", "ars443")


# Extended-precision reference mode: the bordered solves iterate a
# correction (an FP64 bordered solve of the residual, the residual in the
# working precision) until it falls below REFINE_TOL of the solution or
# stops shrinking (the floor of the working precision times the
# conditioning); a floor above REFINE_FAIL would make the reference no
# better than FP64, and is an error.
REFINE_TOL = 2.0**-60
REFINE_FAIL = 2.0**-43
REFINE_MAXIT = 12


class QGOracle:
    """The step in the floating type `dtype`: FP64 (default), or numpy's
    long double as an extended-precision reference for measuring FP64
    rounding.  In long double every product, transform and operator is
    evaluated in long double (parameters are the exact values of the
    binary64 numbers given) and each bordered solve is refined: starting
    from the FP64 solve, the residual of the long-double system is solved
    again in FP64 and added, until the correction is below REFINE_TOL of
    the solution (LAPACK has no long-double band LU).

    pivot=False factors the band blocks without row interchanges
    (oracle.bordered): a second binary64 implementation of the same step,
    whose distance from the first measures the rounding spread of the
    solves.

    method="galerkin" imposes the boundary conditions with the Galerkin
    bases of Sect. 3.2.2 (oracle.galerkin) instead of tau rows: pure band
    systems on the Galerkin coefficients, the state still held as
    Chebyshev coefficients (FP64 only)."""

    def __init__(self, E, Ra, Pr, eta, n_phi, n_r, n_c=None, ekman_eps=None,
                 dtype=np.float64, pivot=True, method="tau",
                 buoyancy="explicit"):
        if method not in ("tau", "galerkin"):
            raise ValueError(method)
        if buoyancy not in ("explicit", "implicit"):
            raise ValueError(buoyancy)
        self.implicit_buoyancy = buoyancy == "implicit"
        if method == "galerkin" and dtype is not np.float64:
            raise ValueError("the Galerkin solves are FP64 only")
        self.method = method
        if n_phi % 3:
            raise ValueError("N_phi must be a multiple of 3 (N_m = N_phi/3)")
        self.E, self.Ra, self.Pr, self.eta = E, Ra, Pr, eta
        self.ekman_eps = ekman_eps
        self.pivot = pivot
        self.rdt = dtype
        self.cdt = np.result_type(dtype, 1j).type
        self.n_phi, self.n_r = n_phi, n_r
        self.M = n_phi // 3 + 1
        self.K = (2 * (n_r - 1)) // 3 if n_c is None else n_c
        d = dtype
        self.s_i, self.s_o = grid.radii(d(eta))
        self.s = grid.s_nodes(eta, n_r, d)
        self.h2 = self.s_o**2 - self.s**2
        self.dtc = grid.dtc_ds(self.s, d(eta))
        self.mvec = np.arange(self.M)
        self.ops = IntegrationOperators(eta, self.K, d)
        # the factorisations are FP64 (LAPACK); in long double they serve
        # as the preconditioner of the refined solves
        self.ops64 = (self.ops if d is np.float64
                      else IntegrationOperators(eta, self.K))
        defs = qg_operators(eta, d)
        self.L_I = defs["L_I"]
        self.dL_I = op_compose(D1, self.L_I)
        # zonal vorticity omega_0 = (1/s) d(s u)/ds and its s-derivative
        self.om0 = op_compose(mult(mono(-1)), op_compose(D1, mult(mono(1))))
        self.dom0 = op_compose(D1, self.om0)
        self.bc_psi = tau_rows_psi(self.K, d)
        self.bc_dir = tau_rows_dirichlet(self.K, d)
        self.refine_its = []      # refinement iterations of the last solves
        self._factors = {}
        self.t = 0.0
        self.nstep = 0
        self._hist = None
        self._ms = None
        self._last = None

    # ---------------------------------------------------------------- state
    def set_state(self, psi, theta, uphi0):
        self.psi = np.array(psi, self.cdt, copy=True)
        self.theta = np.array(theta, self.cdt, copy=True)
        self.uphi = np.array(uphi0, self.rdt, copy=True)
        self._hist = None
        self._ms = None
        self._last = None

    # ------------------------------------------------------------ operators
    def mass(self, psi, theta, uphi):
        o = self.ops
        mp = np.zeros_like(psi)
        for m in range(1, self.M):
            mp[m] = o.A(m) @ psi[m]
        return mp, theta @ o.D.T, o.D @ uphi

    def buoyancy(self, theta):
        """C [(Ra/Pr)(i m/s_o) theta] for every m (row 0 zero)."""
        d = self.rdt
        im = 1j * self.mvec[:, None]
        b = ((d(self.Ra) / d(self.Pr)) * im / self.s_o * theta) @ self.ops.C.T
        b[0] = 0
        return b

    def linear(self, psi, theta, uphi):
        """Implicit operator L y: B_m Psi (+ the buoyancy of theta when it
        is implicit), F_m theta / Pr, E u."""
        o = self.ops
        lp = np.zeros_like(psi)
        lt = np.zeros_like(theta)
        for m in range(self.M):
            if m:
                lp[m] = o.B(m, self.E) @ psi[m]
            lt[m] = o.F(m) @ theta[m] / self.Pr
        if self.implicit_buoyancy:
            lp = lp + self.buoyancy(theta)
        return lp, lt, o.E @ uphi

    def factor(self, a_dt):
        """Bordered LU of (mass - a dt L) for every m (Appendix A), FP64."""
        key = float(a_dt)
        if key in self._factors:
            return self._factors[key]
        o = self.ops64
        if self.method == "galerkin":
            return self._factor_galerkin(key, o, a_dt)
        bp, bd = tau_rows_psi(self.K), tau_rows_dirichlet(self.K)
        fp = [None]
        for m in range(1, self.M):
            fp.append(BorderedSolver(
                bordered_lhs(bp, o.A(m) - a_dt * o.B(m, self.E)), 4,
                self.pivot))
        ft = [BorderedSolver(bordered_lhs(
            bd, o.D - a_dt * o.F(m) / self.Pr), 2, self.pivot)
            for m in range(self.M)]
        fu = BorderedSolver(bordered_lhs(bd, o.D - a_dt * o.E), 2, self.pivot)
        self._factors = {key: (fp, ft, fu)}
        return self._factors[key]

    def _factor_galerkin(self, key, o, a_dt):
        """Pure band LUs of P_q (mass - a dt L) S (eq. psiint_galerkin,
        uphi_galerkin, temp_galerkin) for every m."""
        Sp, Sd = stencil_psi(self.K), stencil_dirichlet(self.K)
        fp = [None] + [GalerkinSolver(o.A(m) - a_dt * o.B(m, self.E), Sp,
                                      BAND_PSI, self.pivot)
                       for m in range(1, self.M)]
        ft = [GalerkinSolver(o.D - a_dt * o.F(m) / self.Pr, Sd,
                             BAND_DIRICHLET, self.pivot)
              for m in range(self.M)]
        fu = GalerkinSolver(o.D - a_dt * o.E, Sd, BAND_DIRICHLET, self.pivot)
        self._factors = {key: (fp, ft, fu)}
        return self._factors[key]

    def _bordered_solve(self, a_dt, rp, rt, ru):
        """The bordered systems of every m with right-hand sides whose tau
        rows are taken as given (FP64 solves); with the Galerkin bases the
        band systems, whose right-hand sides have no such rows."""
        fp, ft, fu = self.factor(a_dt)
        c128 = np.complex128
        theta = np.stack([ft[m].solve(rt[m].astype(c128))
                          for m in range(self.M)])
        if self.implicit_buoyancy:
            # (A - a dt B) Psi = r + a dt C[(Ra/Pr)(i m/s_o) theta_new]
            # (rows 4.. only: the tau rows keep their given values)
            rp = rp.astype(c128, copy=True)
            rp[:, 4:] += (a_dt * self.buoyancy(
                theta.astype(self.cdt))).astype(c128)[:, 4:]
        psi = np.zeros(rp.shape, c128)
        for m in range(1, self.M):
            psi[m] = fp[m].solve(rp[m].astype(c128))
        return psi, theta, fu.solve(ru.astype(np.float64))

    def _apply_bordered(self, a_dt, xp, xt, xu):
        """S x for every system in the working precision: tau rows on top,
        rows p.. of (mass - a dt L) below (the matrices the solves invert),
        using the sparse band form of the m-split operators."""
        if not hasattr(self, "_sparse"):
            o = self.ops
            self._sparse = {n: sp.csr_matrix(getattr(o, n)) for n in
                            ("A0", "A2", "B0", "B2", "B4", "C", "D", "F0",
                             "F2", "E")}
        S = self._sparse
        d = self.rdt
        a = d(a_dt)
        m = self.mvec.astype(d)
        m2 = m * m
        X = xp.T
        yp = (S["A0"] @ X + (S["A2"] @ X) * m2
              - a * (S["B0"] @ X + (S["B2"] @ X) * m2 + (S["B4"] @ X) * m2 * m2
                     + (S["C"] @ X) * (1j * (d(2) * m / d(self.E)))))
        if self.implicit_buoyancy:
            yp = yp - a * self.buoyancy(xt).T
        yp[:4] = self.bc_psi @ X
        T = xt.T
        yt = S["D"] @ T - (a / d(self.Pr)) * (S["F0"] @ T + (S["F2"] @ T) * m2)
        yt[:2] = self.bc_dir @ T
        yu = S["D"] @ xu - a * (S["E"] @ xu)
        yu[:2] = self.bc_dir @ xu
        return yp.T, yt.T, yu

    def solve(self, a_dt, rp, rt, ru):
        """New state from a step's right-hand sides: tau rows set to zero
        (homogeneous boundary conditions), the bordered solves, Psi_0 = 0
        and theta_0 real."""
        rp = rp.copy()
        rt = rt.copy()
        ru = ru.copy()
        rp[:, :4] = 0
        rt[:, :2] = 0
        ru[:2] = 0
        x = list(self._bordered_solve(a_dt, rp, rt, ru))
        if self.rdt is not np.float64:
            x = [x[0].astype(self.cdt), x[1].astype(self.cdt),
                 x[2].astype(self.rdt)]
            x[0][0] = 0
            x[1][0] = x[1][0].real
            prev = np.inf
            for it in range(1, REFINE_MAXIT + 1):
                sx = self._apply_bordered(a_dt, *x)
                r = [rp - sx[0], rt - sx[1], ru - sx[2]]
                r[0][0] = 0                  # Psi_0 is not solved for
                r[1][0] = r[1][0].real       # theta_0 is kept real
                dx = self._bordered_solve(a_dt, *r)
                rel = 0.0
                for i in range(3):
                    scale = float(np.abs(x[i]).max())
                    if scale > 0:
                        rel = max(rel, float(np.abs(dx[i]).max()) / scale)
                    x[i] = x[i] + dx[i]
                x[0][0] = 0
                x[1][0] = x[1][0].real
                if rel <= REFINE_TOL or rel > 0.5 * prev:
                    break
                prev = rel
            if rel > REFINE_FAIL:
                raise RuntimeError(
                    f"refined bordered solve stalled at {rel:.2e} relative")
            self.refine_its.append((it, rel))
        psi, theta, u = x
        theta[0] = theta[0].real
        return psi, theta, u

    # ------------------------------------------------------- explicit terms
    def spectral_fields(self, psi, theta, uphi):
        """Fourier coefficients on the radial grid, arrays (M, N_r): u_s,
        u_phi, omega, d_s omega, theta, d_s theta, dPsi/dphi."""
        R = self.n_r
        s = self.s[None, :]
        m = self.mvec[:, None]
        P = [tr.cheb_to_grid(tr.cheb_ds(psi, p), R) for p in range(4)]
        T = [tr.cheb_to_grid(tr.cheb_ds(theta, p), R) for p in range(2)]
        U = [tr.cheb_to_grid(tr.cheb_ds(uphi, p), R) for p in range(3)]
        im = 1j * m
        us = (self.h2 / self.s)[None, :] * im * P[0]
        uph = -self.h2[None, :] * P[1] + 3.0 * s * P[0]
        uph[0] += U[0]
        om = -evaluate_op(self.L_I, m, P, s)
        dom = -evaluate_op(self.dL_I, m, P, s)
        om[0] += evaluate_op(self.om0, 0, U, self.s)
        dom[0] += evaluate_op(self.dom0, 0, U, self.s)
        return dict(us=us, uphi=uph, om=om, dom=dom, th=T[0], dth=T[1],
                    dphi_psi=im * P[0])

    def advection_grid(self, psi, theta, uphi):
        """Advection terms on the (N_r, N_phi) grid, eqs. vort, uphi, temp:
        N_omega = div(u omega), N_theta = u.grad(theta) + u_s dT_c/ds
        (div(u theta) + beta u_s theta = u.grad(theta) by eq. cont) and the
        zonal forcing mean_phi(u_s omega); also u_s, omega and theta on the
        grid."""
        f = self.spectral_fields(psi, theta, uphi)
        n_phi = self.n_phi
        im = 1j * self.mvec[:, None]

        def to_grid(c):          # (M, R) -> (R, N_phi), eq. (fft)
            return tr.phi_to_grid(c.T, n_phi)
        us, uph = to_grid(f["us"]), to_grid(f["uphi"])
        om, dom = to_grid(f["om"]), to_grid(f["dom"])
        dpom = to_grid(im * f["om"])
        th, dth = to_grid(f["th"]), to_grid(f["dth"])
        dpth = to_grid(im * f["th"])
        divu = to_grid(f["dphi_psi"])          # = -beta u_s
        s = self.s[:, None]
        n_om = us * dom + uph / s * dpom + om * divu
        n_th = us * (dth + self.dtc[:, None]) + uph / s * dpth
        n_u = np.mean(us * om, axis=1)
        return dict(n_om=n_om, n_th=n_th, n_u=n_u, us=us, th=th, om=om)

    def pumping_grid(self, psi, uphi):
        """Ekman pumping terms on the radial grid, (M, N_r): F_eps(Psi_m)
        for m >= 1, Upsilon_eps u (1 + (E/2) omega_0) for m = 0."""
        R, eps = self.n_r, self.ekman_eps
        s = self.s
        he2 = (self.s_o + eps)**2 - s**2
        he = np.sqrt(he2)
        ups = np.sqrt(self.s_o / self.E) / he**1.5
        m = self.mvec[:, None]
        P = [tr.cheb_to_grid(tr.cheb_ds(psi, p), R) for p in range(4)]
        li = evaluate_op(self.L_I, m, P, s[None, :])
        F = ups * (li + 0.5 * s * P[1]
                   - (1.5 * s**2 / he2 + m * m + 2.5j * m * self.s_o / he) * P[0])
        U = [tr.cheb_to_grid(tr.cheb_ds(uphi, p), R) for p in range(2)]
        om0 = evaluate_op(self.om0, 0, U, s)
        F[0] = ups * U[0] * (1.0 + 0.5 * self.E * om0)
        return F

    def explicit(self, psi, theta, uphi):
        """Explicit right-hand sides (K-vectors, rows >= q meaningful):
        E_psi = C[(Ra/Pr)(i m/s_o) theta + N_omega], E_theta = -D[N_theta],
        E_u = -D[N_uphi]."""
        a = self.advection_grid(psi, theta, uphi)
        n_om, n_th, n_u = a["n_om"], a["n_th"], a["n_u"]
        M, K = self.M, self.K
        im = 1j * self.mvec[:, None]

        def to_spec(g):          # (R, N_phi) -> (M, K), eq. (ifft), (icheb)
            return tr.grid_to_cheb(tr.grid_to_phi(g, M).T, K)
        Nom = to_spec(n_om)
        Nth = to_spec(n_th)
        Nth[0] = Nth[0].real
        Nu = tr.grid_to_cheb(n_u, K)
        if self.ekman_eps is not None:
            Fk = tr.grid_to_cheb(self.pumping_grid(psi, uphi), K)
            Nom[1:] -= Fk[1:]
            Nu = Nu + Fk[0].real
        o = self.ops
        d = self.rdt
        if self.implicit_buoyancy:      # buoyancy is in L
            Ep = Nom @ o.C.T
        else:
            buoy = (d(self.Ra) / d(self.Pr)) * im / self.s_o * theta
            Ep = (buoy + Nom) @ o.C.T
        Ep[0] = 0
        Et = -(Nth @ o.D.T)
        Eu = -(o.D @ Nu)
        return Ep, Et, Eu

    # ---------------------------------------------------------------- steps
    def step_cnab2(self, dt):
        y = (self.psi, self.theta, self.uphi)
        Ex = self.explicit(*y)
        prev = Ex if self._hist is None else self._hist
        My = self.mass(*y)
        Ly = self.linear(*y)
        rhs = [My[i] + 0.5 * dt * Ly[i] + dt * (1.5 * Ex[i] - 0.5 * prev[i])
               for i in range(3)]
        self.psi, self.theta, self.uphi = self.solve(CNAB2_BI0 * dt, *rhs)
        self._hist = Ex
        self.t += dt
        self.nstep += 1

    def step_dirk(self, dt, AE, AI):
        """One stiffly accurate IMEX DIRK step with a first explicit stage
        (Sect. 4, eq. dirks): (M - a_ii dt L) y_i = M y^n
        + dt sum_{j<i} (aE_ij E(y_j) + aI_ij L y_j); y^{n+1} = y_last."""
        nu = AE.shape[0]
        y = [(self.psi, self.theta, self.uphi)]
        My = self.mass(*y[0])
        Ex, Ly = [], []
        for i in range(1, nu):
            j = i - 1
            if np.any(AE[:, j] != 0):
                Ex.append(self.explicit(*y[j]))
            else:
                Ex.append(None)
            Ly.append(self.linear(*y[j]))
            rhs = []
            for f in range(3):
                r = My[f].copy()
                for jj in range(i):
                    if AE[i, jj]:
                        r = r + dt * AE[i, jj] * Ex[jj][f]
                    if AI[i, jj]:
                        r = r + dt * AI[i, jj] * Ly[jj][f]
                rhs.append(r)
            y.append(self.solve(AI[i, i] * dt, *rhs))
        self.psi, self.theta, self.uphi = y[-1]
        self.t += dt
        self.nstep += 1

    def step_bpr353(self, dt):
        self.step_dirk(dt, BPR353_AE, BPR353_AI)

    def step_sbdf(self, dt, a, b):
        """One SBDFk step, k = len(b):
        (M - (dt/a_0) L) y^{n+1} = sum_{j=1}^{k} (-a_j/a_0) M y^{n+1-j}
                                   + (dt/a_0) sum_{j=1}^{k} b_j E^{n+1-j};
        BPR353 steps while fewer than k levels are stored."""
        k = len(b)
        y = (self.psi, self.theta, self.uphi)
        if self._ms is None:
            self._ms = []
        self._ms.insert(0, (y, self.explicit(*y)))     # most recent first
        del self._ms[k:]
        if len(self._ms) < k:
            self.step_dirk(dt, BPR353_AE, BPR353_AI)
            return
        masses = [self.mass(*lev[0]) for lev in self._ms]
        rhs = []
        for f in range(3):
            r = np.zeros_like(y[f])
            for j in range(k):
                r = r + (-a[j + 1] / a[0]) * masses[j][f]
                r = r + (dt * b[j] / a[0]) * self._ms[j][1][f]
            rhs.append(r)
        self.psi, self.theta, self.uphi = self.solve(dt / a[0], *rhs)
        self.t += dt
        self.nstep += 1

    def step(self, dt, scheme="cnab2", n=1):
        if scheme not in SCHEMES:
            raise ValueError(scheme)
        for _ in range(n):
            if self._last != (scheme, dt):
                self._hist = None
                self._ms = None
                self._last = (scheme, dt)
            if scheme == "cnab2":
                self.step_cnab2(dt)
            elif scheme in DIRK:
                self.step_dirk(dt, *DIRK[scheme])
            else:
                self.step_sbdf(dt, *SBDF[scheme])
