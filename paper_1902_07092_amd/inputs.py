"""Seeded synthetic workloads for the spherical QG step.

This module is the single source of inputs for both the CPU oracle and the
HIP path.  It draws random Chebyshev/Fourier coefficients and makes them
satisfy the boundary conditions; it holds none of the time-stepping,
transform or operator arithmetic of the method.

Coefficient convention: standard Chebyshev coefficients a_n with
f(x) = sum_n a_n T_n(x), x in [-1, 1] mapped affinely onto [s_i, s_o] with
x = +1 at the outer radius s_o.  Complex fields are stored as complex128
arrays of shape (M, K), M = N_phi/3 + 1 azimuthal wavenumbers m >= 0 and
K = N_c Chebyshev modes.

Boundary conditions built into every state (paper, Sect. 3.2.2):
  Psi:   Psi(s_o) = Psi(s_i) = 0, d^3Psi/ds^3(s_o) = 0, dPsi/ds(s_i) = 0
  theta, zonal flow:  f(s_o) = f(s_i) = 0
Random coefficients are drawn on bases that satisfy these conditions by
construction, so that every spectrum stays smooth: for Psi the basis
phi_n = sum_{i=0..4} gamma_i^n T_{n+i} of the paper's Appendix B
(gamma_0^n = 1), for theta and the zonal flow phi_n = T_{n+2} - T_n
(eq. galerkin_dirichlet).  The amplitude envelopes below are laws in
(m, n) with n the index of the basis function.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Critical Rayleigh numbers without Ekman pumping at eta = 0.35, Pr = 1
# (linear onset, minimised over m).  Used only to set Ra = k x Ra_c.
RA_CRIT = {1e-3: 5.48836e4, 1e-5: 9.956584e6, 1e-6: 1.696285e8,
           1e-8: 6.155224e10}


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    E: float
    Ra: float
    Pr: float
    eta: float
    n_phi: int
    n_r: int
    n_c: int
    scheme: str          # "cnab2" | "bpr353"
    dt: float
    steps: int
    ic: str              # "theta_noise" | "theta_smooth" | "decaying" | "kolmogorov"
    seed: int

    @property
    def n_m(self) -> int:
        return self.n_phi // 3

    @property
    def M(self) -> int:
        return self.n_phi // 3 + 1

    @property
    def grid_points(self) -> int:
        return self.n_phi * self.n_r


def default_nc(n_r: int) -> int:
    """Radial dealiasing cut: coefficients n >= N_c are zero."""
    return (2 * (n_r - 1)) // 3


def _wl(name, E, ra_factor, n_phi, n_r, scheme, dt, steps, ic, seed, Pr=1.0,
        eta=0.35, n_c=None):
    return Workload(name=name, E=E, Ra=ra_factor * RA_CRIT[E], Pr=Pr, eta=eta,
                    n_phi=n_phi, n_r=n_r,
                    n_c=default_nc(n_r) if n_c is None else n_c,
                    scheme=scheme, dt=dt, steps=steps, ic=ic, seed=seed)


# The five workloads the step is exercised and measured on.
SMALL = _wl("small_96x33_E1e-3_cnab2", 1e-3, 1.5, 96, 33, "cnab2", 1e-4,
            100, "theta_noise", 1)
MEDIUM = _wl("medium_768x257_E1e-6_bpr353", 1e-6, 5.0, 768, 257, "bpr353",
             1e-7, 500, "decaying", 2)
LARGE = _wl("large_3072x1025_E1e-8_cnab2", 1e-8, 20.0, 3072, 1025, "cnab2",
            2.5e-10, 50, "kolmogorov", 3)
LARGE_MID = _wl("large_6144x2049_E1e-8_cnab2", 1e-8, 20.0, 6144, 2049,
                "cnab2", 1e-10, 50, "kolmogorov", 3)
LARGE_TOP = _wl("large_12288x4097_E1e-8_cnab2", 1e-8, 20.0, 12288, 4097,
                "cnab2", 2e-11, 50, "kolmogorov", 3)
ADJOINT = _wl("adjoint_768x257_E1e-6_cnab2", 1e-6, 5.0, 768, 257, "cnab2",
              1e-7, 200, "decaying", 2)
WORKLOADS = {w.name: w for w in (SMALL, MEDIUM, LARGE, LARGE_MID, LARGE_TOP,
                                   ADJOINT)}

# Ensemble of independent runs (sizes across the paper's range of problem
# sizes): N_r uniform on {65, 129, 257}, N_phi = 3 (N_r - 1), Ra
# log-uniform on [2, 50] x Ra_c, E = 1e-5, Pr = 1, CNAB2, dt = 1e-6, 200
# steps; member i starts from the theta_smooth recipe with seed 400 + i.
ENSEMBLE_SEED = 4
ENSEMBLE_SIZE = 64


def ensemble_workloads(n: int = ENSEMBLE_SIZE,
                       seed: int = ENSEMBLE_SEED) -> list:
    rng = np.random.Generator(np.random.PCG64(seed))
    n_r = rng.choice(np.array([65, 129, 257]), size=n)
    lo, hi = math.log10(2.0), math.log10(50.0)
    ra_factor = 10.0 ** rng.uniform(lo, hi, size=n)
    return [_wl(f"ensemble_{i}_{3 * (int(n_r[i]) - 1)}x{int(n_r[i])}_E1e-5",
                1e-5, float(ra_factor[i]), 3 * (int(n_r[i]) - 1), int(n_r[i]),
                "cnab2", 1e-6, 200, "theta_smooth", 400 + i)
            for i in range(n)]

# Amplitudes of the random initial states (fixed constants of the recipe).
#   theta_noise:  theta ~ A_TH_NOISE N(0,1)(1+i) on every (m, n)
#   theta_smooth: the same times e^{-n/n_d}, n_d = K/32 (a radial
#                 dissipation range: the last kept coefficient is ~1e-14 of
#                 the first, so the state is resolved to FP64)
#   decaying:     Psi ~ A_PSI_DEC e^{-m/64} e^{-n/64} N(0,1)(1+i),
#                 theta ~ A_TH_DEC e^{-m/64} e^{-n/64} N(0,1)(1+i)
#   kolmogorov:   |a_mn| = A k^{-5/3} for k <= K_R = 20 and
#                 A K_R^{-5/3} (k/K_R)^{-5} beyond (the m^{-5/3} range and the
#                 steeper m^{-5} range past the Rhines scale m ~ 20 that
#                 Sect. 6.2 reports for turbulent QG convection), k =
#                 max(1, sqrt(m^2+n^2)), times e^{-n/n_d}, n_d = K/32, with
#                 random phases.  A_PSI_KOL gives Re = 1e4 and A_TH_KOL an rms
#                 theta of 1e-2 alpha at 3072 x 1025 (K = 682).
A_TH_NOISE = 1.0e-4
A_PSI_DEC = 6.02e-4
A_TH_DEC = 1.35e-5
A_PSI_KOL = 445.018
A_TH_KOL = 1.62955e-3
K_RHINES = 20.0
N_DISS = 32.0


def _gamma(n):
    """Appendix B coefficients gamma_0..gamma_4 of phi_n (gamma_0 = 1)."""
    n = np.asarray(n, dtype=np.float64)
    d = 2 * n**4 + 20 * n**3 + 78 * n**2 + 140 * n + 95
    g1 = 8 * (n + 1) * (n**2 + 4 * n + 5) / d
    g2 = (-2 * (n + 2) * (2 * n**4 + 16 * n**3 + 58 * n**2 + 104 * n + 75)
          / ((n + 3) * d))
    g4 = ((n + 1) * (2 * n**4 + 12 * n**3 + 30 * n**2 + 36 * n + 15)
          / ((n + 3) * d))
    return np.stack([np.ones_like(n), g1, g2, -g1, g4])


def psi_from_basis(c: np.ndarray, K: int) -> np.ndarray:
    """Chebyshev coefficients (..., K) of sum_n c_n phi_n, n < K - 4."""
    nb = K - 4
    g = _gamma(np.arange(nb))
    out = np.zeros(c.shape[:-1] + (K,), np.result_type(c, np.float64))
    for i in range(5):
        out[..., i:i + nb] += c[..., :nb] * g[i]
    return out


def dirichlet_from_basis(c: np.ndarray, K: int) -> np.ndarray:
    """Chebyshev coefficients (..., K) of sum_n c_n (T_{n+2} - T_n)."""
    nb = K - 2
    out = np.zeros(c.shape[:-1] + (K,), np.result_type(c, np.float64))
    out[..., 2:] += c[..., :nb]
    out[..., :nb] -= c[..., :nb]
    return out


@dataclasses.dataclass
class State:
    psi: np.ndarray    # (M, K) complex128, row m = 0 identically zero
    theta: np.ndarray  # (M, K) complex128, row m = 0 real
    uphi0: np.ndarray  # (K,) float64


def make_state(M: int, K: int, ic: str, seed: int) -> State:
    """Seeded initial state of shape (M, K) with the given recipe."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = np.arange(M, dtype=np.float64)[:, None]
    n = np.arange(K, dtype=np.float64)[None, :]
    if ic in ("theta_noise", "theta_smooth"):
        # Psi = 0, zonal flow = 0, theta basis coefficients N(0, 1e-4)
        # (theta_smooth: with the radial dissipation range).
        xi = rng.standard_normal((2, M, K))
        cp = np.zeros((M, K), np.complex128)
        ct = A_TH_NOISE * (xi[0] + 1j * xi[1])
        if ic == "theta_smooth":
            ct = ct * np.exp(-n / (K / N_DISS))
    elif ic == "decaying":
        env = np.exp(-m / 64.0) * np.exp(-n / 64.0)
        xp = rng.standard_normal((2, M, K))
        xt = rng.standard_normal((2, M, K))
        cp = A_PSI_DEC * env * (xp[0] + 1j * xp[1])
        ct = A_TH_DEC * env * (xt[0] + 1j * xt[1])
    elif ic == "kolmogorov":
        k = np.maximum(1.0, np.sqrt(m**2 + n**2))
        env = np.where(k <= K_RHINES, k ** (-5.0 / 3.0),
                       K_RHINES ** (-5.0 / 3.0) * (k / K_RHINES) ** (-5.0))
        env = env * np.exp(-n / (K / N_DISS))
        ph_p = rng.uniform(0.0, 2.0 * math.pi, (M, K))
        ph_t = rng.uniform(0.0, 2.0 * math.pi, (M, K))
        cp = A_PSI_KOL * env * np.exp(1j * ph_p)
        ct = A_TH_KOL * env * np.exp(1j * ph_t)
    else:
        raise ValueError(f"unknown initial-condition recipe {ic!r}")
    cp[0, :] = 0
    ct[0, :] = ct[0, :].real
    psi = psi_from_basis(cp, K)
    theta = dirichlet_from_basis(ct, K)
    return State(psi=np.ascontiguousarray(psi),
                 theta=np.ascontiguousarray(theta), uphi0=np.zeros(K))


def make_direction(M: int, K: int, seed: int) -> np.ndarray:
    """Unit-norm random direction in the free theta coefficients (n >= 2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xi = rng.standard_normal((2, M, K))
    d = xi[0] + 1j * xi[1]
    d[:, :2] = 0
    d[0, :] = d[0, :].real
    return d / np.linalg.norm(d)


def workload_state(w: Workload) -> State:
    return make_state(w.M, w.n_c, w.ic, w.seed)
