"""Pins of the oracle's transforms against closed forms and library
routines (Fourier pair eq. fft/ifft; Chebyshev pair eq. cheb/icheb)."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from oracle import grid, transforms as tr


@pytest.mark.parametrize("n_phi", [96, 768])
def test_fourier_single_mode(n_phi):
    # cos(m phi) has f_m = 1/2 under eq. (fft); sin(m phi) has f_m = -i/2.
    M = n_phi // 3 + 1
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    for m in (0, 1, 7, M - 1):
        fm = tr.grid_to_phi(np.cos(m * phi), M)
        exp = np.zeros(M, complex)
        exp[m] = 1.0 if m == 0 else 0.5
        assert np.allclose(fm, exp, atol=1e-14)
        if m:
            fm = tr.grid_to_phi(np.sin(m * phi), M)
            exp = np.zeros(M, complex)
            exp[m] = -0.5j
            assert np.allclose(fm, exp, atol=1e-14)


def test_fourier_round_trip(rng):
    n_phi = 96
    M = n_phi // 3 + 1
    fm = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    fm[0] = fm[0].real
    f = tr.phi_to_grid(fm, n_phi)
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    direct = fm[0].real + 2 * sum(
        (fm[m] * np.exp(1j * m * phi)).real for m in range(1, M))
    assert np.allclose(f, direct, atol=1e-13)
    assert np.allclose(tr.grid_to_phi(f, M), fm, atol=1e-14)


@pytest.mark.parametrize("n_r", [5, 33, 257])
def test_chebyshev_pair_self_inverse(n_r):
    # eq. (cheb) and eq. (icheb) with double-primed sums are mutual inverses
    rng = np.random.Generator(np.random.PCG64(n_r))
    f = rng.standard_normal(n_r)
    back = tr.cheb_paper_synthesis(tr.cheb_paper_analysis(f))
    assert np.allclose(back, f, atol=1e-12 * np.sqrt(n_r))


def test_chebyshev_single_coefficient():
    n_r = 17
    x = grid.gl_nodes(n_r)
    for n in (0, 3, 16):
        a = np.zeros(n_r)
        a[n] = 1.0
        assert np.allclose(tr.cheb_to_grid(a, n_r), np.cos(n * np.arccos(x)),
                           atol=1e-14)


def test_standard_coefficients_match_paper_normalisation(rng):
    n_r = 33
    fhat = rng.standard_normal(n_r)
    f = tr.cheb_paper_synthesis(fhat)
    a = tr.paper_to_standard(fhat)
    assert np.allclose(tr.cheb_to_grid(a, n_r), f, atol=1e-13)
    assert np.allclose(tr.grid_to_cheb(f), a, atol=1e-14)
    # and against numpy's Chebyshev evaluation
    assert np.allclose(npcheb.chebval(grid.gl_nodes(n_r), a), f, atol=1e-13)


def test_derivative_in_s(rng):
    # s = x/2 + c: d/ds = 2 d/dx.  Compare with exact polynomial derivative.
    eta = 0.35
    n_r = 40
    a = rng.standard_normal(20)
    s = grid.s_nodes(eta, n_r)
    x = grid.gl_nodes(n_r)
    d1 = tr.cheb_to_grid(tr.cheb_ds(a, 1), n_r)
    d2 = tr.cheb_to_grid(tr.cheb_ds(a, 2), n_r)
    poly = np.polynomial.Chebyshev(a)
    assert np.allclose(d1, 2 * poly.deriv(1)(x), rtol=1e-12, atol=1e-10)
    assert np.allclose(d2, 4 * poly.deriv(2)(x), rtol=1e-12, atol=1e-8)
    assert s[0] > s[-1]


def test_clenshaw_curtis_exact_on_polynomials():
    for n_r in (9, 33, 34):
        w = grid.clenshaw_curtis(n_r)
        x = grid.gl_nodes(n_r)
        for deg in range(n_r):
            exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
            assert abs(w @ x**deg - exact) < 1e-13


def test_alpha_value():
    # alpha(0.35) from the fixed-temperature formula of Sect. 2
    assert abs(grid.alpha_tc(0.35) - 0.4449580) < 5e-8
    s_i, s_o = grid.radii(0.35)
    assert abs(s_o - s_i - 1) < 1e-15 and abs(s_i / s_o - 0.35) < 1e-15


def test_derivatives_match_closed_forms(rng):
    """cheb_ds against the closed forms of Chebyshev derivatives (not a
    library call): with x = cos(theta), T_n'(x) = n sin(n theta)/sin(theta)
    inside, T_n'(+-1) = (+-1)^(n+1) n^2; T_n'' from the Chebyshev equation
    (1 - x^2) T_n'' = x T_n' - n^2 T_n inside; T_n'''(1) =
    n^2 (n^2 - 1)(n^2 - 4)/15.  d/ds = 2 d/dx on the unit gap.  A missing
    factor 2 (d/dx for d/ds) or an index shift in the recurrence fails."""
    n_r, K = 33, 21
    a = rng.standard_normal(K)
    k = np.arange(n_r)
    th = np.pi * k / (n_r - 1)
    x = np.cos(th)
    n = np.arange(K)
    inner = slice(1, n_r - 1)
    T = np.cos(np.outer(th, n))
    dT = np.empty((n_r, K))
    dT[inner] = n[None, :] * np.sin(np.outer(th[inner], n)) / np.sin(th[inner])[:, None]
    dT[0] = n**2
    dT[-1] = (-1.0) ** (n + 1) * n**2
    d2T = np.zeros((n_r, K))
    d2T[inner] = ((x[inner, None] * dT[inner] - n[None, :] ** 2 * T[inner])
                  / (1 - x[inner] ** 2)[:, None])
    d1 = tr.cheb_to_grid(tr.cheb_ds(a, 1), n_r)
    d2 = tr.cheb_to_grid(tr.cheb_ds(a, 2), n_r)
    scale1 = np.abs(dT @ a).max()
    assert np.allclose(d1, 2 * dT @ a, rtol=0, atol=1e-12 * scale1)
    scale2 = np.abs(d2T @ a).max()
    assert np.allclose(d2[inner], 4 * d2T[inner] @ a, rtol=0, atol=1e-11 * scale2)
    d3_outer = tr.cheb_to_grid(tr.cheb_ds(a, 3), n_r)[0]
    exact3 = 8 * np.sum(a * n**2 * (n**2 - 1) * (n**2 - 4) / 15.0)
    assert abs(d3_outer - exact3) <= 1e-12 * np.sum(np.abs(a) * n**6)
