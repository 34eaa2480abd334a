"""Diagnostics of a QG state (oracle; test infrastructure only).

Paper Sect. 6.2: E_K = (1/2) <u_s^2 + u_phi^2>, E_Z = (1/2) <<u_phi>^2>,
with <f> = int_0^{2 pi} int_{s_i}^{s_o} f s ds dphi (Sect. 4, convergence
test); Sect. 6.3: Re = [2 E_K / (pi (s_o^2 - s_i^2))]^{1/2}, Ro = Re E;
enstrophy <omega^2> (Sect. 4, stability study); eq. (cfl) for the
Courant time step with alpha = 1, delta phi = 2 pi / N_phi and delta s the
local Gauss-Lobatto spacing (reading: the smaller of the two neighbour
gaps).  Thermal energy is not defined in the paper; E_T = (1/2) <theta^2>
(reading).  Radial integrals use Clenshaw-Curtis quadrature on the
Gauss-Lobatto nodes, azimuthal ones the uniform grid sum.
"""
import numpy as np

from . import grid, transforms as tr


def diagnostics(o):
    """o: a step.QGOracle holding a state."""
    f = o.spectral_fields(o.psi, o.theta, o.uphi)
    n_phi = o.n_phi
    g = {k: tr.phi_to_grid(v.T, n_phi) for k, v in f.items()
         if k in ("us", "uphi", "om", "th")}
    w = grid.clenshaw_curtis(o.n_r) * 0.5 * (o.s_o - o.s_i) * o.s
    dphi = 2.0 * np.pi / n_phi

    def avg(field):
        return float(np.sum(w[:, None] * field) * dphi)
    ubar = tr.cheb_to_grid(o.uphi, o.n_r)
    e_kin = 0.5 * avg(g["us"] ** 2 + g["uphi"] ** 2)
    e_zon = 0.5 * avg(np.repeat(ubar[:, None] ** 2, n_phi, axis=1))
    e_th = 0.5 * avg(g["th"] ** 2)
    enst = avg(g["om"] ** 2)
    re = np.sqrt(2.0 * e_kin / (np.pi * (o.s_o**2 - o.s_i**2)))
    s = o.s
    gaps = np.abs(np.diff(s))
    ds = np.empty_like(s)
    ds[0], ds[-1] = gaps[0], gaps[-1]
    ds[1:-1] = np.minimum(gaps[:-1], gaps[1:])
    with np.errstate(divide="ignore"):
        rate_s = np.max(np.abs(g["us"]) / ds[:, None])
        rate_p = np.max(np.abs(g["uphi"]) / (s[:, None] * dphi))
    rate = max(rate_s, rate_p)
    dt_cfl = np.inf if rate == 0 else 1.0 / rate
    finite = all(np.all(np.isfinite(a)) for a in (o.psi, o.theta, o.uphi))
    return dict(t=o.t, step=o.nstep, E_kin=e_kin, E_zon=e_zon, E_therm=e_th,
                enstrophy=enst, Re=float(re), Ro=float(re * o.E),
                dt_cfl=float(dt_cfl), nonfinite=int(not finite))
