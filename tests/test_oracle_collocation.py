"""Integration-method oracle against an independent collocation DNS.

The paper validates its sparse Chebyshev-integration scheme (Sect. 3.2,
Appendix A) against the Chebyshev-collocation scheme (Sect. 3.1) on the
same physical problem.  The two discretise the radial direction
differently: tau rows and integrated operators against boundary rows and a
dense differentiation matrix, truncated (dealiased) radial products against
collocated ones.  Started from one smooth, nonlinear, buoyancy-driven state
and advanced with the same CNAB2 steps, the two trajectories therefore differ
only by the radial truncation error, which must fall quickly as N_r grows.
A wrong sign, a missing term or a wrong boundary condition in either
stepper leaves an O(1) difference that does not fall with N_r.
"""
import numpy as np
import pytest

from oracle import transforms as tr
from oracle.collocation import CollocationCNAB2
from oracle.step import QGOracle
from paper_1902_07092_amd import inputs

E, PR, ETA, N_PHI = 1e-3, 1.0, 0.35, 48


def _state(K, amp=1.0, k0=6, mmax=8, seed=5):
    """A smooth state: k0 radial basis functions per field, m < mmax,
    amplitudes falling like exp(-(m + n)/1.5)."""
    M = N_PHI // 3 + 1
    rng = np.random.default_rng(seed)
    m = np.arange(M)[:, None]
    n = np.arange(k0)[None, :]
    env = np.exp(-(m + n) / 1.5)
    cp = np.zeros((M, K), complex)
    ct = np.zeros((M, K), complex)
    cu = np.zeros(K)
    cp[:, :k0] = env * (rng.standard_normal((M, k0)) + 1j * rng.standard_normal((M, k0)))
    ct[:, :k0] = env * (rng.standard_normal((M, k0)) + 1j * rng.standard_normal((M, k0)))
    cp[0] = 0.0
    ct[0] = ct[0].real
    cp[mmax:] = 0.0
    ct[mmax:] = 0.0
    cu[:k0] = np.exp(-np.arange(k0) / 1.5) * rng.standard_normal(k0)
    return (inputs.psi_from_basis(amp * cp, K),
            inputs.dirichlet_from_basis(amp * ct, K),
            inputs.dirichlet_from_basis(amp * cu, K))


def _differences(n_r, Ra, amp, dt, nsteps, plant=None):
    o = QGOracle(E, Ra, PR, ETA, N_PHI, n_r)
    if plant is not None:
        plant(o)
    psi, th, u = _state(o.K, amp)
    o.set_state(psi, th, u)
    c = CollocationCNAB2(E, Ra, PR, ETA, N_PHI, n_r)
    c.set_state(tr.cheb_to_grid(psi, n_r), tr.cheb_to_grid(th, n_r),
                tr.cheb_to_grid(u, n_r))
    o.step(dt, "cnab2", nsteps)
    for _ in range(nsteps):
        c.step(dt)
    out = {}
    for f, a, b in (("psi", tr.cheb_to_grid(o.psi, n_r), c.Psi),
                    ("theta", tr.cheb_to_grid(o.theta, n_r), c.theta),
                    ("uphi", tr.cheb_to_grid(o.uphi, n_r), c.u)):
        assert np.isfinite(a).all() and np.isfinite(b).all(), f
        out[f] = float(np.abs(a - b).max() / np.abs(a).max())
    return out


def test_linear_steps_agree_spectrally():
    """Tiny amplitude, Ra = 0: viscous decay, Coriolis coupling and the
    boundary conditions alone."""
    d33 = _differences(33, 0.0, 1e-6, 1e-3, 5)
    d97 = _differences(97, 0.0, 1e-6, 1e-3, 5)
    # measured at the time of writing: psi 9.3e-4 -> 2.9e-6,
    # theta 1.7e-4 -> 1.8e-9, uphi 4.1e-4 -> 1.8e-12
    for f in d33:
        assert d97[f] < d33[f] / 100.0, (f, d33, d97)
    assert max(d97.values()) < 1e-5, d97


def test_nonlinear_convection_steps_agree():
    """Ra = 1e5, order-one amplitudes: psi grows tenfold in ten steps under
    buoyancy; the advection terms, the zonal forcing and the buoyancy
    coupling all act."""
    d33 = _differences(33, 1e5, 1.0, 2e-4, 10)
    d97 = _differences(97, 1e5, 1.0, 2e-4, 10)
    # measured at the time of writing: psi 7.8e-4 -> 3.6e-5,
    # theta 7.0e-4 -> 1.1e-6, uphi 4.5e-2 -> 6.8e-5
    for f in d33:
        assert d97[f] < d33[f] / 10.0, (f, d33, d97)
    assert d97["psi"] < 2e-4 and d97["theta"] < 1e-5 and d97["uphi"] < 5e-4, d97


def _flip_buoyancy(o):
    """Buoyancy enters only E_psi, linearly in theta: E_psi at -theta."""
    orig = o.explicit

    def explicit(psi, theta, uphi):
        Ep, _, _ = orig(psi, -theta, uphi)
        _, Et, Eu = orig(psi, theta, uphi)
        return Ep, Et, Eu
    o.explicit = explicit


def _flip_coriolis(o):
    """E enters the oracle only through the (2/E) i m term of B_m."""
    o.E = -o.E


def _drop_zonal_forcing(o):
    orig = o.explicit

    def explicit(psi, theta, uphi):
        Ep, Et, Eu = orig(psi, theta, uphi)
        return Ep, Et, 0.0 * Eu
    o.explicit = explicit


@pytest.mark.parametrize("plant", [_flip_buoyancy, _flip_coriolis,
                                   _drop_zonal_forcing])
def test_planted_mistake_is_caught(plant):
    """The comparison is sensitive: one planted mistake in the integration
    oracle leaves a difference far above the truncation error at N_r = 65."""
    d = _differences(65, 1e5, 1.0, 2e-4, 10, plant)
    assert max(d.values()) > 1e-2, d
