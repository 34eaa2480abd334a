"""Geometry of the QG annulus (oracle; test infrastructure only).

Paper Sect. 2: lengths are scaled by the gap d = s_o - s_i = 1, eta = s_i/s_o.
Paper Sect. 3 (Chebyshev expansion): Gauss-Lobatto nodes
x_k = cos(pi (k-1)/(N_r-1)), k = 1..N_r, mapped affinely onto [s_i, s_o].
Here k is 0-based, so index 0 is x = +1, i.e. s = s_o.

Every function computes in the floating type `dtype` (FP64 by default;
numpy's long double gives the extended-precision reference the parity
tests measure FP64 rounding against).  Parameters are taken as the exact
values of the binary64 numbers passed in.
"""
import numpy as np


def pi_of(dtype):
    """pi in the precision of dtype."""
    return np.arccos(dtype(-1))


def radii(eta):
    """(s_i, s_o) with s_o - s_i = 1 and s_i/s_o = eta (in the type of eta)."""
    return eta / (1 - eta), 1 / (1 - eta)


def gl_nodes(n_r, dtype=np.float64):
    """Gauss-Lobatto nodes x_k = cos(pi k/(N_r-1)), k = 0..N_r-1."""
    k = np.arange(n_r, dtype=dtype)
    return np.cos(pi_of(dtype) * k / (n_r - 1))


def s_nodes(eta, n_r, dtype=np.float64):
    """Radial collocation points s_k = (s_o-s_i)/2 x_k + (s_o+s_i)/2."""
    s_i, s_o = radii(dtype(eta))
    return (s_o - s_i) / 2 * gl_nodes(n_r, dtype) + (s_o + s_i) / 2


def alpha_tc(eta):
    """Rescaling constant alpha of the conducting background for fixed
    temperature boundaries (Sect. 2, formula below the T_c definition)."""
    r = np.sqrt(1.0 - eta**2)
    return eta / (1.0 - eta) * (np.arcsinh(r / eta) / r - 1.0)


def dtc_ds(s, eta):
    """dT_c/ds = alpha / (s ln eta) (Sect. 2)."""
    return alpha_tc(eta) / (s * np.log(eta))


def clenshaw_curtis(n_r, dtype=np.float64):
    """Clenshaw-Curtis weights w_k on the Gauss-Lobatto nodes for
    int_{-1}^{1} f dx; exact for polynomials of degree <= N_r - 1.
    (Standard quadrature; the paper's annulus integral <f> is evaluated
    with it.)"""
    N = n_r - 1
    theta = pi_of(dtype) * np.arange(n_r, dtype=dtype) / N
    w = np.zeros(n_r, dtype)
    v = np.ones(n_r - 2, dtype)
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
