"""Geometry of the QG annulus (oracle; test infrastructure only).

Paper Sect. 2: lengths are scaled by the gap d = s_o - s_i = 1, eta = s_i/s_o.
Paper Sect. 3 (Chebyshev expansion): Gauss-Lobatto nodes
x_k = cos(pi (k-1)/(N_r-1)), k = 1..N_r, mapped affinely onto [s_i, s_o].
Here k is 0-based, so index 0 is x = +1, i.e. s = s_o.
"""
import numpy as np


def radii(eta):
    """(s_i, s_o) with s_o - s_i = 1 and s_i/s_o = eta."""
    return eta / (1.0 - eta), 1.0 / (1.0 - eta)


def gl_nodes(n_r):
    """Gauss-Lobatto nodes x_k = cos(pi k/(N_r-1)), k = 0..N_r-1."""
    k = np.arange(n_r)
    return np.cos(np.pi * k / (n_r - 1))


def s_nodes(eta, n_r):
    """Radial collocation points s_k = (s_o-s_i)/2 x_k + (s_o+s_i)/2."""
    s_i, s_o = radii(eta)
    return 0.5 * (s_o - s_i) * gl_nodes(n_r) + 0.5 * (s_o + s_i)


def alpha_tc(eta):
    """Rescaling constant alpha of the conducting background for fixed
    temperature boundaries (Sect. 2, formula below the T_c definition)."""
    r = np.sqrt(1.0 - eta**2)
    return eta / (1.0 - eta) * (np.arcsinh(r / eta) / r - 1.0)


def dtc_ds(s, eta):
    """dT_c/ds = alpha / (s ln eta) (Sect. 2)."""
    return alpha_tc(eta) / (s * np.log(eta))


def clenshaw_curtis(n_r):
    """Clenshaw-Curtis weights w_k on the Gauss-Lobatto nodes for
    int_{-1}^{1} f dx; exact for polynomials of degree <= N_r - 1.
    (Standard quadrature; the paper's annulus integral <f> is evaluated
    with it.)"""
    N = n_r - 1
    theta = np.pi * np.arange(n_r) / N
    w = np.zeros(n_r)
    v = np.ones(n_r - 2)
    if N % 2 == 0:
        w[0] = w[N] = 1.0 / (N**2 - 1)
        for j in range(1, N // 2):
            v -= 2.0 * np.cos(2 * j * theta[1:-1]) / (4 * j * j - 1)
        v -= np.cos(N * theta[1:-1]) / (N**2 - 1)
    else:
        w[0] = w[N] = 1.0 / N**2
        for j in range(1, (N - 1) // 2 + 1):
            v -= 2.0 * np.cos(2 * j * theta[1:-1]) / (4 * j * j - 1)
    w[1:-1] = 2.0 * v / N
    return w
