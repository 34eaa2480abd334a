"""Energy budgets of the QG step (oracle; test infrastructure only).

The paper gives no budget formula.  These are the budgets of the
semi-discrete equations the step integrates (eq. psi_int, uphi_int,
temp_int): mass matrix times d/dt of the state = sum of terms, each term
with the tau rows of the homogeneous boundary conditions.  Every term T
alone gives a state derivative y'_T = S^-1 [0; T] (bordered solve with the
mass matrix A_m or D, Appendix A), and since the energies are quadratic in
the state,

    kinetic  E_K = (1/2) <u_s^2 + u_phi^2>,  dE_K/dt = sum_T <u(y) . u(y'_T)>
    thermal  E_T = (1/2) <theta^2>,          dE_T/dt = sum_T <theta(y) theta(y'_T)>

(<f> = int int f s ds dphi, Sect. 4; E_T is a reading, the paper does not
define it).  Terms, kinetic: viscous (B_m without Coriolis; E for the zonal
flow), Coriolis ((2/E) i m C), buoyancy (C (Ra/Pr)(i m/s_o) theta),
advection (C N_omega; -D N_uphi).  Thermal: diffusion (F_m / Pr),
background (-D [u_s dT_c/ds]), advection (-D [u . grad theta]).  These
powers are exact for the semi-discrete system, so a time step's budget,
(E(y^{n+1}) - E(y^n)) / dt against the mean of the summed powers at both
ends, measures the time discretisation alone: O(dt^2) for CNAB2 (its
first step, whose E^{-1} := E^0, only O(dt)).
"""
import numpy as np

from . import grid, transforms as tr


def _weights(o):
    """Clenshaw-Curtis weights of int f s ds on the radial grid."""
    return grid.clenshaw_curtis(o.n_r) * 0.5 * (o.s_o - o.s_i) * o.s


def _mode_weights(o):
    """Parseval in phi: int_0^{2 pi} f g dphi = 2 pi sum_m w_m Re(f_m g_m*),
    w_0 = 1, w_m = 2."""
    return np.where(o.mvec == 0, 1.0, 2.0)[:, None]


def kinetic_product(o, psi_a, u_a, psi_b, u_b):
    """<u(a) . u(b)>."""
    z = np.zeros_like(psi_a)
    fa = o.spectral_fields(psi_a, z, u_a)
    fb = o.spectral_fields(psi_b, z, u_b)
    dot = (fa["us"] * np.conj(fb["us"]) + fa["uphi"] * np.conj(fb["uphi"])).real
    return float(2 * np.pi * np.sum(_weights(o)[None, :] * _mode_weights(o) * dot))


def thermal_product(o, th_a, th_b):
    """<theta(a) theta(b)>."""
    ga = tr.cheb_to_grid(th_a, o.n_r)
    gb = tr.cheb_to_grid(th_b, o.n_r)
    dot = (ga * np.conj(gb)).real
    return float(2 * np.pi * np.sum(_weights(o)[None, :] * _mode_weights(o) * dot))


def kinetic_energy(o, psi, uphi):
    return 0.5 * kinetic_product(o, psi, uphi, psi, uphi)


def thermal_energy(o, theta):
    return 0.5 * thermal_product(o, theta, theta)


def _spec(o, g):
    """(N_r, N_phi) grid field to (M, K) coefficients (eq. ifft, icheb)."""
    return tr.grid_to_cheb(tr.grid_to_phi(g, o.M).T, o.K)


def tendencies(o, psi, theta, uphi):
    """State derivative of each term: {name: (psi', theta', u')}."""
    ops = o.ops
    M, K = o.M, o.K
    im = 1j * o.mvec[:, None]
    f = o.spectral_fields(psi, theta, uphi)
    adv = o.advection_grid(psi, theta, uphi)

    def g(c):
        return tr.phi_to_grid(c.T, o.n_phi)
    s = o.s[:, None]
    us = g(f["us"])
    n_bg = us * o.dtc[:, None]                          # u_s dT_c/ds
    n_th = us * g(f["dth"]) + g(f["uphi"]) / s * g(im * f["th"])   # u . grad theta
    Nom = _spec(o, adv["n_om"])
    Nbg, Nth = _spec(o, n_bg), _spec(o, n_th)
    Nbg[0], Nth[0] = Nbg[0].real, Nth[0].real
    Nu = tr.grid_to_cheb(adv["n_u"], K)
    zp, zt, zu = np.zeros_like(psi), np.zeros_like(theta), np.zeros_like(uphi)
    visc, cor, diff = zp.copy(), zp.copy(), zt.copy()
    for m in range(M):
        m2 = float(m * m)
        if m:
            visc[m] = (ops.B0 + m2 * ops.B2 + m2 * m2 * ops.B4) @ psi[m]
            cor[m] = (2.0j * m / o.E) * (ops.C @ psi[m])
        diff[m] = ops.F(m) @ theta[m] / o.Pr
    buoy = ((o.Ra / o.Pr) * im / o.s_o * theta) @ ops.C.T
    advp = Nom @ ops.C.T
    buoy[0] = advp[0] = 0
    terms = {
        "viscous": (visc, zt, ops.E @ uphi),
        "coriolis": (cor, zt, zu),
        "buoyancy": (buoy, zt, zu),
        "advection": (advp, -(Nth @ ops.D.T), -(ops.D @ Nu)),
        "diffusion": (zp, diff, zu),
        "background": (zp, -(Nbg @ ops.D.T), zu),
    }
    return {k: o.solve(0.0, *v) for k, v in terms.items()}


def powers(o, psi, theta, uphi):
    """{"kinetic": {term: power}, "thermal": {term: power}}."""
    out = {"kinetic": {}, "thermal": {}}
    for k, (p, t, u) in tendencies(o, psi, theta, uphi).items():
        if k in ("viscous", "coriolis", "buoyancy", "advection"):
            out["kinetic"][k] = kinetic_product(o, psi, uphi, p, u)
        if k in ("advection", "diffusion", "background"):
            out["thermal"][k] = thermal_product(o, theta, t)
    return out
