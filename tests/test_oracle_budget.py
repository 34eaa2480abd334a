"""Energy budgets of the CNAB2 step (oracle, CPU).

The powers of every term of the semi-discrete equations (oracle/budget.py)
sum to the energies' rates, so the budget of one time step,

    r = (E(y^{n+1}) - E(y^n)) / dt - (P(y^n) + P(y^{n+1})) / 2,

is the time discretisation's error: O(dt^2) for CNAB2 (Sect. 4,
eq. multistep1).  Measured on the second step (the first one starts with
E^{-1} := E^0) of a resolved nonlinear 96 x 33 state, for kinetic and
thermal energy.  The dt range resolves the fastest (Rossby) waves of
E = 1e-3; with steps near the CFL bound the kinetic budget converges more
slowly, as the scheme's error constant for the unresolved waves is large.

Planted mistakes, each in a copy of the oracle (never in the oracle):
  * Adams-Bashforth weights (1, 0) instead of (3/2, -1/2) in the step: the
    residual falls as O(dt) only (ratio 2 per halving);
  * the background advection u_s dT_c/ds with the wrong sign in the
    step's explicit terms: the thermal budget no longer closes;
  * the buoyancy dropped from the step: the kinetic budget no longer
    closes.
"""
import numpy as np
import pytest

from oracle import budget as bd
from oracle.step import QGOracle
from paper_1902_07092_amd import inputs

W = inputs.SMALL
DTS = (2e-6, 1e-6, 5e-7, 2.5e-7)


def _state():
    """A resolved nonlinear state: coefficients decaying like e^{-1.5 n}
    (the last of 21 about 1e-13), Re ~ 10, theta ~ 0.1."""
    rng = np.random.default_rng(5)
    M, K = W.M, W.n_c
    env = np.exp(-1.5 * np.arange(K))[None, :] * np.exp(-np.arange(M) / 4.0)[:, None]
    cp = (rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))) * env
    ct = (rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))) * env
    cp[0] = 0
    ct[0] = ct[0].real
    psi = inputs.psi_from_basis(cp, K)
    psi *= 2.0 / np.abs(psi).max()
    theta = inputs.dirichlet_from_basis(ct, K)
    theta *= 0.1 / np.abs(theta).max()
    uphi = inputs.dirichlet_from_basis(np.exp(-1.5 * np.arange(K)), K).real * 0.5
    return psi, theta, uphi


def _residuals(cls, dt):
    o = cls(W.E, W.Ra, W.Pr, W.eta, W.n_phi, W.n_r, W.n_c)
    o.set_state(*_state())
    o.step(dt, "cnab2", 1)
    y1 = (o.psi.copy(), o.theta.copy(), o.uphi.copy())
    p1 = bd.powers(o, *y1)
    o.step(dt, "cnab2", 1)
    y2 = (o.psi, o.theta, o.uphi)
    p2 = bd.powers(o, *y2)
    out = {}
    for kind, energy in (("kinetic", lambda y: bd.kinetic_energy(o, y[0], y[2])),
                         ("thermal", lambda y: bd.thermal_energy(o, y[1]))):
        rate = (energy(y2) - energy(y1)) / dt
        mean = 0.5 * (sum(p1[kind].values()) + sum(p2[kind].values()))
        out[kind] = (rate - mean, rate, p1[kind])
    return out


def _orders(cls):
    res = [_residuals(cls, dt) for dt in DTS]
    out = {}
    for kind in ("kinetic", "thermal"):
        r = [abs(x[kind][0]) for x in res]
        rate = abs(res[-1][kind][1])
        out[kind] = ([r[i] / r[i + 1] for i in range(len(r) - 1)], r[-1] / rate,
                     res[-1][kind][2])
    return out


def test_cnab2_budgets_are_second_order():
    out = _orders(QGOracle)
    for kind, (ratios, rel, terms) in out.items():
        print(kind, "ratios", [f"{x:.3f}" for x in ratios], f"last rel {rel:.2e}",
              {k: f"{v:.3e}" for k, v in terms.items()})
        assert all(3.6 < x < 4.4 for x in ratios), (kind, ratios)
        assert rel < 1e-5, (kind, rel)
    # signs the physics fixes: viscosity and diffusion remove energy
    assert out["kinetic"][2]["viscous"] < 0 and out["thermal"][2]["diffusion"] < 0


class _EulerExtrapolation(QGOracle):
    def step_cnab2(self, dt):
        self._hist = None          # E^{n-1} := E^n every step: weights (1, 0)
        super().step_cnab2(dt)


class _WrongBackground(QGOracle):
    def advection_grid(self, psi, theta, uphi):
        a = super().advection_grid(psi, theta, uphi)
        a["n_th"] = a["n_th"] - 2 * a["us"] * self.dtc[:, None]
        return a


class _NoBuoyancy(QGOracle):
    def explicit(self, psi, theta, uphi):
        Ra = self.Ra
        self.Ra = 0.0
        try:
            return super().explicit(psi, theta, uphi)
        finally:
            self.Ra = Ra


@pytest.mark.parametrize("cls,kind", [(_EulerExtrapolation, "kinetic"),
                                      (_EulerExtrapolation, "thermal"),
                                      (_WrongBackground, "thermal"),
                                      (_NoBuoyancy, "kinetic")])
def test_planted_mistakes_break_the_budget(cls, kind):
    ratios, rel, _ = _orders(cls)[kind]
    print(cls.__name__, kind, [f"{x:.3f}" for x in ratios], f"{rel:.2e}")
    assert not (all(3.6 < x < 4.4 for x in ratios) and rel < 1e-5)
