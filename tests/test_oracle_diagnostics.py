"""Diagnostics of the oracle against closed forms (CPU).

A state with one non-axisymmetric Psi mode, one theta mode plus an
axisymmetric theta and a zonal flow, all low-degree polynomials that meet
the boundary conditions.  Its kinetic, zonal and thermal energies,
enstrophy, Re and Ro (Sect. 6.2, 6.3) are integrals of rational functions
of s over the gap, done exactly with sympy (eta = 7/20, the binary64 0.35
to 2e-17) from the definitions:
    u_s = (h^2/s) dPsi/dphi,  u_phi = <u_phi> - h^2 dPsi/ds + 3 s Psi,
    omega = (1/s) d(s <u_phi>)/ds - L_I Psi,
    L_I Psi = Lap(h^2 Psi) - (1/s) d(s^2 Psi)/ds         (Sect. 3.2.1),
    <f> = int_0^2pi int f s ds dphi,  Re = [2 E_K / (pi (s_o^2 - s_i^2))]^1/2,
    Ro = Re E,
and the CFL rate of eq. (cfl) (alpha = 1) from the velocity at the grid
points, evaluated from the polynomials.  The oracle instead transforms
the coefficients (DCT-I, inverse FFT) and integrates with Clenshaw-Curtis
quadrature.  A dropped factor 2 of the m >= 1 modes, a wrong power of h
or s, or a sign error in u_phi or omega fails here.
"""
import numpy as np
import sympy as sy

from oracle.diagnostics import diagnostics
from oracle.step import QGOracle
from paper_1902_07092_amd import inputs

E_, N_PHI, N_R = 1e-3, 96, 33
K = (2 * (N_R - 1)) // 3
M = N_PHI // 3 + 1
MP, MT = 4, 3            # the Psi mode and the theta mode


def _state():
    psi = np.zeros((M, K), complex)
    theta = np.zeros((M, K), complex)
    cp = np.zeros(K)
    cp[:3] = (1.0, 0.5, -0.25)
    psi[MP] = inputs.psi_from_basis(cp, K) * (0.8 + 0.6j)
    ct = np.zeros(K)
    ct[:3] = (0.3, -0.2, 0.1)
    theta[MT] = inputs.dirichlet_from_basis(ct, K) * (0.5 - 1.2j)
    theta[0] = inputs.dirichlet_from_basis(np.array([0.7, 0.1] + [0] * (K - 2)), K)
    uphi = inputs.dirichlet_from_basis(np.array([0.4, -0.3, 0.2] + [0] * (K - 3)), K).real
    return psi, theta, uphi


def _poly(coef, x):
    """sum_n a_n T_n(x) with the binary64 coefficients as exact rationals."""
    return sum(sy.nsimplify(float(c), rational=True) * sy.chebyshevt(n, x)
               for n, c in enumerate(coef) if c != 0)


def _closed_forms():
    psi, theta, uphi = _state()
    s = sy.symbols("s", positive=True)
    eta = sy.Rational(7, 20)
    s_i, s_o = eta / (1 - eta), 1 / (1 - eta)
    x = 2 * s - (s_o + s_i)
    h2 = s_o**2 - s**2

    def cplx(row):
        return _poly(row.real, x), _poly(row.imag, x)
    pr, pi_ = cplx(psi[MP])
    tr_, ti = cplx(theta[MT])
    t0 = _poly(theta[0].real, x)
    ub = _poly(uphi, x)

    def lap(f, m):
        return sy.diff(f, s, 2) + sy.diff(f, s) / s - m**2 * f / s**2

    def om(f, m):
        return -(lap(h2 * f, m) - sy.diff(s**2 * f, s) / s)

    def integ(expr):
        return sy.integrate(sy.expand(expr * s), (s, s_i, s_o))

    # mode m: u_s = (h^2/s) i m Psi, u_phi = -h^2 Psi' + 3 s Psi
    usr, usi = -(h2 / s) * MP * pi_, (h2 / s) * MP * pr
    upr = -h2 * sy.diff(pr, s) + 3 * s * pr
    upi = -h2 * sy.diff(pi_, s) + 3 * s * pi_
    ek_m = 2 * sy.pi * integ(sy.cancel(usr**2 + usi**2) + upr**2 + upi**2)
    ez = sy.pi * integ(ub**2)
    et = sy.pi * integ(t0**2) + 2 * sy.pi * integ(tr_**2 + ti**2)
    om0 = sy.diff(ub, s) + ub / s
    omr, omi = om(pr, MP), om(pi_, MP)
    ens = 2 * sy.pi * (integ(sy.cancel(om0**2)) + 2 * integ(sy.cancel(omr**2 + omi**2)))
    ek = ek_m + ez
    vals = {k: float(sy.N(v, 30)) for k, v in
            (("E_kin", ek), ("E_zon", ez), ("E_therm", et), ("enstrophy", ens))}
    vals["Re"] = float(sy.N(sy.sqrt(2 * ek / (sy.pi * (s_o**2 - s_i**2))), 30))
    vals["Ro"] = vals["Re"] * E_
    # CFL rate at the grid points from the polynomials (eq. cfl, alpha = 1)
    f_us = sy.lambdify(s, (usr, usi), "mpmath")
    f_up = sy.lambdify(s, (upr, upi, ub), "mpmath")
    k = np.arange(N_R)
    sk = 0.5 * (float(s_o) - float(s_i)) * np.cos(np.pi * k / (N_R - 1)) \
        + 0.5 * (float(s_o) + float(s_i))
    gaps = np.abs(np.diff(sk))
    ds = np.concatenate([[gaps[0]], np.minimum(gaps[:-1], gaps[1:]), [gaps[-1]]])
    phi = 2 * np.pi * np.arange(N_PHI) / N_PHI
    rate = 0.0
    for j, sv in enumerate(sk):
        a = complex(*[float(v) for v in f_us(sv)])
        ur, ui, u0 = [float(v) for v in f_up(sv)]
        us = 2 * np.real(a * np.exp(1j * MP * phi))
        up = u0 + 2 * np.real(complex(ur, ui) * np.exp(1j * MP * phi))
        rate = max(rate, np.abs(us).max() / ds[j],
                   np.abs(up).max() / (sv * 2 * np.pi / N_PHI))
    vals["dt_cfl"] = 1.0 / rate
    return vals


def test_diagnostics_match_closed_forms():
    psi, theta, uphi = _state()
    o = QGOracle(E_, 1e5, 1.0, 0.35, N_PHI, N_R, K)
    o.set_state(psi, theta, uphi)
    d = diagnostics(o)
    exact = _closed_forms()
    for key, v in exact.items():
        print(f"{key:10s} oracle {d[key]:.15e} closed form {v:.15e}")
        assert abs(d[key] - v) <= 1e-12 * abs(v), (key, d[key], v)
