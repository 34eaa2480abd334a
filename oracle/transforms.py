"""Spectral transforms (oracle; test infrastructure only).

Fourier pair, paper Sect. 3, eq. (fft) and eq. (ifft):
    f(s, phi_k) = 2 sum'_{m=0}^{N_m} Re{ f_m e^{i m phi_k} }   (spectral->grid,
                                                  prime: m = 0 weighted 1/2)
    f_m = (1/N_phi) sum_k f(s, phi_k) e^{-i m phi_k}            (grid->spectral)
Modes N_m < m <= N_phi/2 are zero on the way to the grid and dropped on the
way back (the paper's wording of which transform pads and which truncates is
swapped relative to its formulas; the formulas are followed).

Chebyshev pair, paper eq. (cheb) and eq. (icheb), with C = sqrt(2/(N_r-1)) and
double-primed sums.  Internally the step uses standard coefficients a_n,
f(x) = sum_n a_n T_n(x), related to the paper's normalised coefficients by
a_n = C fhat_n w_n with w_n = 1/2 at n = 0 and n = N_r - 1 and 1 otherwise
(reading: the halved end terms are the DCT end points; coefficients
n >= N_c are zero).  With this reading the pair is exactly self-inverse.
"""
import numpy as np
import scipy.fft as sfft
from numpy.polynomial import chebyshev as npcheb

WORKERS = -1   # scipy.fft: use every host core


# ---------------------------------------------------------------- Fourier
def phi_to_grid(fm, n_phi):
    """eq. (fft): spectral coefficients f_m (last axis, m = 0..N_m) to
    N_phi real grid values.  numpy's irfft applies the Hermitian sum."""
    fm = np.asarray(fm)
    M = fm.shape[-1]
    F = np.zeros(fm.shape[:-1] + (n_phi // 2 + 1,), np.result_type(fm, 1j))
    F[..., :M] = fm * n_phi
    return sfft.irfft(F, n=n_phi, axis=-1, workers=WORKERS)


def grid_to_phi(f, M):
    """eq. (ifft): N_phi grid values (last axis) to f_m, m = 0..M-1."""
    n_phi = f.shape[-1]
    return sfft.rfft(f, axis=-1, workers=WORKERS)[..., :M] / n_phi


# ---------------------------------------------------------------- Chebyshev
def cheb_matrix(n_r):
    """T_kn = T_n(x_k) = cos(pi n k/(N_r-1)) on the Gauss-Lobatto grid."""
    k = np.arange(n_r)
    return np.cos(np.pi * np.outer(k, k) / (n_r - 1))


def cheb_paper_synthesis(fhat):
    """eq. (cheb) as printed: f_k = C sum''_n fhat_n T_n(x_k) (last axis)."""
    n_r = fhat.shape[-1]
    C = np.sqrt(2.0 / (n_r - 1))
    w = np.ones(n_r)
    w[0] = w[-1] = 0.5
    return C * (fhat * w) @ cheb_matrix(n_r).T


def cheb_paper_analysis(f):
    """eq. (icheb) as printed: fhat_n = C sum''_k f_k T_n(x_k)."""
    n_r = f.shape[-1]
    C = np.sqrt(2.0 / (n_r - 1))
    w = np.ones(n_r)
    w[0] = w[-1] = 0.5
    return C * (f * w) @ cheb_matrix(n_r)


def paper_to_standard(fhat):
    n_r = fhat.shape[-1]
    C = np.sqrt(2.0 / (n_r - 1))
    a = C * np.array(fhat, copy=True)
    a[..., 0] *= 0.5
    a[..., -1] *= 0.5
    return a


def cheb_to_grid(a, n_r):
    """Standard coefficients a_n (last axis, length <= N_r) to values on
    the N_r Gauss-Lobatto nodes: f_k = sum_n a_n T_n(x_k).  Same map as
    eq. (cheb); evaluated with a type-I DCT."""
    a = np.asarray(a)
    K = a.shape[-1]
    b = np.zeros(a.shape[:-1] + (n_r,), a.dtype)
    b[..., :K] = a
    b[..., 0] *= 2.0
    b[..., n_r - 1] *= 2.0
    return 0.5 * sfft.dct(b, type=1, axis=-1, workers=WORKERS)


def grid_to_cheb(f, K=None):
    """Values on the N_r Gauss-Lobatto nodes to standard coefficients
    a_n, n < K (all N_r if K is None).  Same map as eq. (icheb)."""
    f = np.asarray(f)
    n_r = f.shape[-1]
    a = sfft.dct(f, type=1, axis=-1, workers=WORKERS) / (n_r - 1)
    a[..., 0] *= 0.5
    a[..., n_r - 1] *= 0.5
    return a if K is None else a[..., :K]


def cheb_ds(a, order=1):
    """Coefficients of d^order f/ds^order.  ds = dx/2 on the unit gap, so
    each derivative in s is twice the derivative in x (numpy's chebder is
    the textbook coefficient recurrence)."""
    a = np.asarray(a)
    if order == 0:
        return a
    K = a.shape[-1]
    out = npcheb.chebder(a, m=order, scl=a.real.dtype.type(2), axis=-1)
    pad = np.zeros(a.shape[:-1] + (K,), out.dtype)
    pad[..., :out.shape[-1]] = out
    return pad
