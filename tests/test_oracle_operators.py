"""Pins of the integration-method operators (paper Sect. 3.2).

The oracle builds A_m, B_m, C, D, E, F_m by integrating by parts and
multiplying sparse Chebyshev matrices in floating point.  Here each column
is rebuilt from the paper's definitions with exact rational arithmetic
(sympy): T_n(x(s)) is differentiated, multiplied and integrated q times
symbolically, then expanded back into Chebyshev polynomials.  Rows k >= q
must agree (rows < q hold integration constants and are replaced by tau
rows).  eta = 7/20 makes s_i, s_o rational.
"""
import numpy as np
import pytest
import sympy as sy

from oracle import grid
from oracle.operators import (IntegrationOperators, tau_rows_dirichlet,
                              tau_rows_psi)

ETA = sy.Rational(7, 20)
S_I = ETA / (1 - ETA)
S_O = 1 / (1 - ETA)
s, x, m = sy.symbols("s x m")


def lap(f):
    return sy.diff(f, s, 2) + sy.diff(f, s) / s - m**2 * f / s**2


def L_I(f):                       # Sect. 3.2.1
    h2 = S_O**2 - s**2
    return lap(h2 * f) - sy.diff(s**2 * f, s) / s


def integrate(expr, q):
    for _ in range(q):
        expr = sy.integrate(sy.expand(expr), s)
    return sy.expand(expr)


def cheb_coeffs(poly_s, K):
    """Exact Chebyshev coefficients (in x) of a polynomial in s."""
    px = sy.Poly(sy.expand(poly_s.subs(s, x / 2 + (S_O + S_I) / 2)), x)
    if px.is_zero:
        return [sy.Integer(0)]
    out = [sy.Integer(0)] * (px.degree() + 1)
    rem = px
    while not rem.is_zero:
        d = rem.degree()
        lead = rem.LC()
        c = lead if d == 0 else lead / sy.Integer(2) ** (d - 1)
        out[d] = c
        rem = rem - sy.Poly(c * sy.chebyshevt(d, x), x)
    return out


def exact_operator(op, q, K, mval):
    cols = []
    for n in range(K):
        Tn = sy.chebyshevt(n, 2 * (s - (S_O + S_I) / 2))
        expr = integrate(op(Tn).subs(m, mval), q)
        co = cheb_coeffs(sy.simplify(expr), K)
        cols.append([float(co[k]) if k < len(co) else 0.0 for k in range(K)])
    return np.array(cols).T


K = 12


@pytest.fixture(scope="module")
def ops():
    return IntegrationOperators(0.35, K)


def _close(A, B, q):
    A, B = A[q:], B[q:]
    scale = np.abs(B).max()
    assert np.max(np.abs(A - B)) <= 1e-12 * scale


def test_A_operator_exact(ops):
    for mval in (0, 3):
        ex = exact_operator(lambda f: s**4 * L_I(f), 4, K, mval)
        _close(ops.A(mval), ex, 4)


def test_B_operator_exact(ops):
    E = 1e-3
    for mval in (1, 2):
        ex = exact_operator(lambda f: s**4 * lap(L_I(f)), 4, K, mval)
        exC = exact_operator(lambda f: s**4 * f, 4, K, mval)
        _close(ops.B(mval, E), ex + (2j * mval / E) * exC, 4)


def test_C_D_E_F_exact(ops):
    _close(ops.C, exact_operator(lambda f: s**4 * f, 4, K, 0), 4)
    _close(ops.D, exact_operator(lambda f: s**2 * f, 2, K, 0), 2)
    for mval in (0, 5):
        _close(ops.F(mval), exact_operator(lambda f: s**2 * lap(f), 2, K,
                                           mval), 2)
    # E = int^2 s^2 (Lap - 1/s^2) and also s^2 - 3 int s (Sect. 3.2.1)
    ex_E = exact_operator(lambda f: s**2 * (lap(f).subs(m, 1)), 2, K, 1)
    _close(ops.E, ex_E, 2)
    ex_E2 = exact_operator(
        lambda f: sy.diff(s**2 * f - 3 * sy.integrate(sy.expand(s * f), s),
                          s, 2), 2, K, 0)
    _close(ops.E, ex_E2, 2)


def test_bandwidths_match_paper():
    # Sect. 3.2.1: A, B, C have bandwidths 17, 13 (17 with the Coriolis
    # term), 17; D, E, F have 9, 5, 5.
    o = IntegrationOperators(0.35, 40)

    def bw(Mx, q):
        nz = np.argwhere(np.abs(Mx[q:]) > 1e-14 * np.abs(Mx[q:]).max())
        d = nz[:, 1] - (nz[:, 0] + q)
        return d.max() - d.min() + 1
    assert bw(o.A(3), 4) == 17
    assert bw(o.B0 + 9 * o.B2 + 81 * o.B4, 4) == 13
    assert bw(o.B(3, 1e-3), 4) == 17
    assert bw(o.C, 4) == 17
    assert bw(o.D, 2) == 9
    assert bw(o.E, 2) == 5
    assert bw(o.F(3), 2) == 5


def test_tau_rows_are_boundary_values():
    # rows: f(s_o), f(s_i), f'''(s_o), f'(s_i) (up to the x->s scale)
    Kt = 15
    rng = np.random.Generator(np.random.PCG64(3))
    a = rng.standard_normal(Kt)
    P = np.polynomial.Chebyshev(a)
    rows = tau_rows_psi(Kt)
    assert np.isclose(rows[0] @ a, P(1.0))
    assert np.isclose(rows[1] @ a, P(-1.0))
    assert np.isclose(rows[2] @ a, P.deriv(3)(1.0), rtol=1e-12)
    assert np.isclose(rows[3] @ a, P.deriv(1)(-1.0), rtol=1e-12)
    assert np.allclose(tau_rows_dirichlet(Kt), rows[:2])


def test_galerkin_gamma_satisfy_tau_rows():
    # Appendix B's gamma_i^n satisfy the four Psi tau conditions exactly;
    # this checks the tau rows against an independent printed result.
    for n in range(0, 12):
        d = 2 * n**4 + 20 * n**3 + 78 * n**2 + 140 * n + 95
        g = [1.0,
             8 * (n + 1) * (n**2 + 4 * n + 5) / d,
             -2 * (n + 2) * (2 * n**4 + 16 * n**3 + 58 * n**2 + 104 * n + 75)
             / ((n + 3) * d),
             -8 * (n + 1) * (n**2 + 4 * n + 5) / d,
             (n + 1) * (2 * n**4 + 12 * n**3 + 30 * n**2 + 36 * n + 15)
             / ((n + 3) * d)]
        a = np.zeros(n + 5)
        a[n:n + 5] = g
        rows = tau_rows_psi(n + 5)
        assert np.allclose(rows @ a, 0.0, atol=1e-10 * (n + 5) ** 6)


def test_qg_continuity_and_curl():
    """u_s, u_phi from Psi (Sect. 3.2.1) satisfy eq. (cont), and the
    oracle's omega equals the curl (1/s) d(s u_phi)/ds - (1/s) d u_s/dphi."""
    from oracle.step import QGOracle
    o = QGOracle(1e-3, 1e4, 1.0, 0.35, 24, 41, 20)
    rng = np.random.Generator(np.random.PCG64(7))
    psi = np.zeros((o.M, o.K), complex)
    psi[1:, :10] = rng.standard_normal((o.M - 1, 10))
    theta = np.zeros_like(psi)
    uphi = np.zeros(o.K)
    uphi[:8] = rng.standard_normal(8)
    f = o.spectral_fields(psi, theta, uphi)
    sg = o.s
    # s u_phi is a polynomial of degree < 13 in s: fit and differentiate
    x = grid.gl_nodes(o.n_r)
    mv = np.arange(o.M)[:, None]
    su = sg * f["uphi"]
    coef = np.polynomial.chebyshev.chebfit(x, su.T, 20)
    dsu = 2 * np.polynomial.chebyshev.chebval(
        x, np.polynomial.chebyshev.chebder(coef)).reshape(o.M, -1)
    curl = dsu / sg - 1j * mv * f["us"] / sg
    assert np.allclose(f["om"], curl, atol=1e-9 * np.abs(curl).max())
    # continuity: (1/s) d(s u_s)/ds + (1/s) d u_phi/dphi + beta u_s = 0
    sus = sg * f["us"]
    coef = np.polynomial.chebyshev.chebfit(x, sus.T, 20)
    dsus = 2 * np.polynomial.chebyshev.chebval(
        x, np.polynomial.chebyshev.chebder(coef)).reshape(o.M, -1)
    h2 = o.h2
    inner = slice(1, -1)          # beta is singular at s_o
    beta = -sg / h2
    res = (dsus / sg + 1j * mv * f["uphi"] / sg + beta * f["us"])[:, inner]
    res[0] = 0                    # m = 0: u_phi is zonal, u_s = 0
    assert np.max(np.abs(res)) < 1e-9 * np.abs(f["us"]).max()
    # d_s omega against a spectral derivative of omega on a fine fit
    coef = np.polynomial.chebyshev.chebfit(x, f["om"].T, o.n_r - 1)
    dom = 2 * np.polynomial.chebyshev.chebval(
        x, np.polynomial.chebyshev.chebder(coef)).reshape(o.M, -1)
    assert np.allclose(f["dom"], dom, atol=1e-7 * np.abs(dom).max())
