"""Discrete adjoint of the CNAB2 step (oracle; test infrastructure only).

Gradient of the time-integrated kinetic energy
    J = dt sum_{n=0}^{N} w_n E_K(y^n),   w = trapezoid weights (1/2 at ends),
E_K = (1/2) <u_s^2 + u_phi^2> as in the paper's Sect. 6.2, with respect to
the free Chebyshev coefficients of the initial temperature (n >= 2; theta_0
and theta_1 follow from the Dirichlet rows of eq. bcs_coll_dirichlet), by
reverse-mode differentiation of the oracle's own CNAB2 step (eq. multistep1
with E^{-1} := E^0): transposed bordered solves, transposed mass and linear
operators, and the transposed explicit terms (Fourier and Chebyshev
transforms, pointwise products linearised about the stored trajectory).

Conventions: states are complex arrays; for a real function of complex
variables the gradient is stored as d/dRe + i d/dIm.  Complex-linear maps A
then have the adjoint A^H.  The per-m field maps, the Chebyshev transforms
and the Fourier transforms are built as explicit matrices by applying the
oracle's functions to unit vectors, so each transpose is exact by
construction.  Sizes: the test grids (dense per-m matrices).
"""
import numpy as np

from . import grid, transforms as tr
from .operators import bordered_lhs
from .step import CNAB2_BI0

FIELDS = ("us", "uphi", "om", "dom", "th", "dth", "dphi_psi")


class CNAB2Adjoint:
    def __init__(self, o):
        """o: a step.QGOracle (its operators and parameters are used)."""
        self.o = o
        M, K, R, n_phi = o.M, o.K, o.n_r, o.n_phi
        self.M, self.K, self.R, self.n_phi = M, K, R, n_phi
        z = np.zeros((M, K), np.complex128)
        zu = np.zeros(K)
        # per-m field matrices: F[var][f] has shape (M, R, K)
        self.F = {"psi": {f: np.zeros((M, R, K), np.complex128) for f in FIELDS},
                  "th": {f: np.zeros((M, R, K), np.complex128) for f in FIELDS},
                  "u": {f: np.zeros((R, K), np.complex128) for f in FIELDS}}
        for n in range(K):
            e = z.copy()
            e[:, n] = 1.0
            fp = o.spectral_fields(e, z, zu)
            ft = o.spectral_fields(z, e, zu)
            eu = zu.copy()
            eu[n] = 1.0
            fu = o.spectral_fields(z, z, eu)
            for f in FIELDS:
                self.F["psi"][f][:, :, n] = fp[f]
                self.F["th"][f][:, :, n] = ft[f]
                self.F["u"][f][:, n] = fu[f][0]
        # Chebyshev analysis matrix G (K x R): coefficients = G @ values
        self.G = tr.grid_to_cheb(np.eye(R), K).T
        self.w = (grid.clenshaw_curtis(R) * 0.5 * (o.s_o - o.s_i) * o.s)
        self._S = {}

    # ---------------------------------------------------------- transposes
    def to_grid_T(self, g):
        """Adjoint of c -> phi_to_grid(c.T, n_phi): (R, n_phi) -> (M, R)."""
        c = tr.grid_to_phi(g, self.M) * self.n_phi     # sum_j g_j e^{-i m phi_j}
        c[:, 1:] *= 2.0
        c[:, 0] = c[:, 0].real
        return c.T

    def to_spec_T(self, X):
        """Adjoint of g -> grid_to_cheb(grid_to_phi(g, M).T, K): (M, K) ->
        (R, n_phi)."""
        c = X @ self.G                                  # (M, R): G^T per row
        c = c.T.copy()                                  # (R, M)
        c[:, 1:] *= 0.5                                 # adjoint of rfft / n_phi
        return tr.phi_to_grid(c, self.n_phi) / self.n_phi

    def fields_T(self, fbar):
        """Adjoint of spectral_fields: {f: (M, R)} -> (psi, theta, u)."""
        ps = np.zeros((self.M, self.K), np.complex128)
        th = np.zeros_like(ps)
        u = np.zeros(self.K)
        for f, v in fbar.items():
            ps += np.einsum("mrk,mr->mk", self.F["psi"][f].conj(), v)
            th += np.einsum("mrk,mr->mk", self.F["th"][f].conj(), v)
            u += (self.F["u"][f].conj().T @ v[0]).real
        ps[0] = 0.0
        return ps, th, u

    # ------------------------------------------------------------ pieces
    def grad_EK(self, y):
        """d E_K / d y."""
        o = self.o
        f = o.spectral_fields(*y)
        dphi = 2.0 * np.pi / self.n_phi
        W = self.w[:, None] * dphi
        us = tr.phi_to_grid(f["us"].T, self.n_phi)
        uph = tr.phi_to_grid(f["uphi"].T, self.n_phi)
        return self.fields_T({"us": self.to_grid_T(W * us),
                              "uphi": self.to_grid_T(W * uph)})

    def explicit_T(self, y, Ep_b, Et_b, Eu_b):
        """Adjoint of the explicit terms at state y applied to (Ep_b, Et_b,
        Eu_b), following step.QGOracle.explicit."""
        o = self.o
        ops = o.ops
        a = o.advection_grid(*y)
        f = o.spectral_fields(*y)
        im = 1j * o.mvec[:, None]
        n_phi = self.n_phi

        def g(c):
            return tr.phi_to_grid(c.T, n_phi)
        us, uph, om, dom = a["us"], g(f["uphi"]), a["om"], g(f["dom"])
        dpom, dth, dpth, divu = g(im * f["om"]), g(f["dth"]), g(im * f["th"]), g(f["dphi_psi"])
        s = o.s[:, None]
        Ep_b = Ep_b.copy()
        Ep_b[0] = 0.0
        X_b = Ep_b @ ops.C                              # adjoint of X @ C.T
        th_b = np.conj((o.Ra / o.Pr) * im / o.s_o) * X_b
        Nth_b = -(Et_b @ ops.D)
        Nth_b[0] = Nth_b[0].real
        Nu_b = -(ops.D.T @ Eu_b)
        n_om_b = self.to_spec_T(X_b)
        n_th_b = self.to_spec_T(Nth_b)
        n_u_b = self.G.T @ Nu_b                         # (R,)
        # products (real, on the grid)
        us_b = n_om_b * dom + n_th_b * (dth + o.dtc[:, None]) + n_u_b[:, None] * om / n_phi
        uph_b = (n_om_b * dpom + n_th_b * dpth) / s
        om_b = n_om_b * divu + n_u_b[:, None] * us / n_phi
        fb = {"us": self.to_grid_T(us_b), "uphi": self.to_grid_T(uph_b),
              "om": self.to_grid_T(om_b) - im * self.to_grid_T(n_om_b * uph / s),
              "dom": self.to_grid_T(n_om_b * us),
              "th": -im * self.to_grid_T(n_th_b * uph / s),
              "dth": self.to_grid_T(n_th_b * us),
              "dphi_psi": self.to_grid_T(n_om_b * om)}
        ps, th, u = self.fields_T(fb)
        return ps, th + th_b, u

    def _lhs(self, adt):
        if adt not in self._S:
            o, ops = self.o, self.o.ops
            Sp = [None] + [bordered_lhs(o.bc_psi, ops.A(m) - adt * ops.B(m, o.E))
                           for m in range(1, self.M)]
            St = [bordered_lhs(o.bc_dir, ops.D - adt * ops.F(m) / o.Pr)
                  for m in range(self.M)]
            Su = bordered_lhs(o.bc_dir, ops.D - adt * ops.E)
            self._S = {adt: (Sp, St, Su)}
        return self._S[adt]

    def solve_T(self, adt, yb):
        """Adjoint of y = P S^{-1} Z r (P: Psi_0 = 0, theta_0 real; Z: tau
        rows of r zeroed) applied to yb = (psi, theta, u)."""
        Sp, St, Su = self._lhs(adt)
        pb, tb, ub = (yb[0].copy(), yb[1].copy(), yb[2].copy())
        pb[0] = 0.0
        tb[0] = tb[0].real
        rp = np.zeros_like(pb)
        rt = np.zeros_like(tb)
        for m in range(1, self.M):
            rp[m] = np.linalg.solve(Sp[m].conj().T, pb[m])
        for m in range(self.M):
            rt[m] = np.linalg.solve(St[m].T, tb[m])
        ru = np.linalg.solve(Su.T, ub)
        rp[:, :4] = 0.0
        rt[:, :2] = 0.0
        ru[:2] = 0.0
        return rp, rt, ru

    def mass_lin_T(self, cL, rb):
        """Adjoint of y -> M y + cL L y."""
        o, ops = self.o, self.o.ops
        pb = np.zeros_like(rb[0])
        for m in range(1, self.M):
            Op = ops.A(m) + cL * ops.B(m, o.E)
            pb[m] = Op.conj().T @ rb[0][m]
        tb = np.stack([(ops.D + cL * ops.F(m) / o.Pr).T @ rb[1][m] for m in range(self.M)])
        ub = (ops.D + cL * ops.E).T @ rb[2]
        return pb, tb, ub

    # ---------------------------------------------------------- gradient
    def gradient(self, y0, dt, nsteps):
        """J and dJ/dtheta^0 (full coefficient array; the caller projects
        onto its free coefficients) for nsteps CNAB2 steps from y0."""
        o = self.o
        o.set_state(*y0)
        ys = [tuple(np.copy(v) for v in y0)]
        for _ in range(nsteps):
            o.step(dt, "cnab2", 1)
            ys.append((o.psi.copy(), o.theta.copy(), o.uphi.copy()))
        w = np.ones(nsteps + 1)
        w[0] = w[-1] = 0.5
        from .diagnostics import diagnostics
        J = 0.0
        for n, y in enumerate(ys):
            o.set_state(*y)
            J += dt * w[n] * diagnostics(o)["E_kin"]
        adt = CNAB2_BI0 * dt
        rb = [None] * (nsteps + 1)     # rb[n]: adjoint of step n's right-hand side
        yb = None
        for n in range(nsteps, -1, -1):
            g = self.grad_EK(ys[n])
            acc = [dt * w[n] * v for v in g]
            if n < nsteps:
                ml = self.mass_lin_T(0.5 * dt, rb[n])
                c1 = 1.0 if n == 0 else 1.5
                eb = [c1 * dt * v for v in rb[n]]
                if n + 1 < nsteps:
                    eb = [a - 0.5 * dt * b for a, b in zip(eb, rb[n + 1])]
                ex = self.explicit_T(ys[n], *eb)
                acc = [a + b + c for a, b, c in zip(acc, ml, ex)]
            yb = acc
            if n > 0:
                rb[n - 1] = self.solve_T(adt, yb)
        return J, yb[1]


def transpose_map(adj, y0, dt, nsteps, w):
    """J^T w for the map y^0 -> y^N of nsteps CNAB2 steps from y0 (J its
    derivative at y0; real inner product sum Re(conj(a) b) over every
    component): the reverse sweep of CNAB2Adjoint.gradient with the
    terminal adjoint w and no energy terms."""
    o = adj.o
    o.set_state(*y0)
    ys = [tuple(np.copy(v) for v in y0)]
    for _ in range(nsteps):
        o.step(dt, "cnab2", 1)
        ys.append((o.psi.copy(), o.theta.copy(), o.uphi.copy()))
    adt = CNAB2_BI0 * dt
    rb = [None] * (nsteps + 1)
    yb = None
    for n in range(nsteps, -1, -1):
        if n == nsteps:
            acc = [np.array(v, dtype=np.result_type(v, np.float64)) for v in w]
        else:
            ml = adj.mass_lin_T(0.5 * dt, rb[n])
            c1 = 1.0 if n == 0 else 1.5
            eb = [c1 * dt * v for v in rb[n]]
            if n + 1 < nsteps:
                eb = [a - 0.5 * dt * b for a, b in zip(eb, rb[n + 1])]
            ex = adj.explicit_T(ys[n], *eb)
            acc = [a + b for a, b in zip(ml, ex)]
        yb = acc
        if n > 0:
            rb[n - 1] = adj.solve_T(adt, yb)
    return yb


def dirichlet_free_to_full(c):
    """theta coefficients from the free ones (n >= 2) by the Dirichlet rows:
    theta_0 = -sum of even n >= 2, theta_1 = -sum of odd n >= 3."""
    full = np.zeros(c.shape[:-1] + (c.shape[-1] + 2,), c.dtype)
    full[..., 2:] = c
    n = np.arange(2, c.shape[-1] + 2)
    full[..., 0] = -c[..., n % 2 == 0].sum(-1)
    full[..., 1] = -c[..., n % 2 == 1].sum(-1)
    return full


def full_to_free_T(g):
    """Adjoint of dirichlet_free_to_full."""
    K = g.shape[-1]
    n = np.arange(2, K)
    out = g[..., 2:].copy()
    out -= np.where(n % 2 == 0, 1.0, 0.0) * g[..., :1]
    out -= np.where(n % 2 == 1, 1.0, 0.0) * g[..., 1:2]
    return out
