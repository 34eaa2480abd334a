"""Pins of the oracle's implicit buoyancy (Sect. 4: the buoyancy term of
the vorticity equation treated implicitly, the temperature advanced first):

  * the sequential solve (theta, then Psi with the new theta's buoyancy)
    equals a dense solve of the coupled 2K x 2K tau system;
  * a run started from the m = 12 eigenmode of Sect. 6.1 grows and drifts
    at the eigenvalue (a sign or scale error in the moved term would not);
  * the schemes keep their orders (Fig. 2), converging to the same
    solution as with explicit buoyancy.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import eigen
from oracle.operators import bordered_lhs, tau_rows_dirichlet, tau_rows_psi
from oracle.step import QGOracle
from paper_1902_07092_amd import inputs


def test_sequential_solve_equals_dense_coupled_solve():
    o = QGOracle(1e-3, 8e4, 1.0, 0.35, 48, 33, buoyancy="implicit")
    K, a = o.K, 0.37e-3
    rng = np.random.default_rng(3)
    rp = rng.standard_normal((o.M, K)) + 1j * rng.standard_normal((o.M, K))
    rt = rng.standard_normal((o.M, K)) + 1j * rng.standard_normal((o.M, K))
    rt[0] = rt[0].real
    ru = rng.standard_normal(K)
    psi, th, _ = o.solve(a, rp, rt, ru)
    free = QGOracle(1e-3, 8e4, 1.0, 0.35, 48, 33).solve(a, rp, rt, ru)[0]
    ops = o.ops
    for m in (1, 4, o.M - 1):
        g = 1j * m * (o.Ra / o.Pr) / o.s_o
        top = np.hstack([bordered_lhs(tau_rows_psi(K), ops.A(m) - a * ops.B(m, o.E)),
                         np.vstack([np.zeros((4, K)), -a * g * ops.C[4:]])])
        bot = np.hstack([np.zeros((K, K)),
                         bordered_lhs(tau_rows_dirichlet(K),
                                      ops.D - a * ops.F(m) / o.Pr)])
        S = np.vstack([top, bot])
        f = np.concatenate([rp[m], rt[m]])
        f[:4] = 0
        f[K:K + 2] = 0
        x = sla.solve(S, f)
        # the dense system's condition number is ~1e12: the two solves
        # agree to ~1e-12 (measured 3e-12 at m = 4), while dropping the
        # coupling moves Psi by ~4e-3
        assert np.abs(psi[m] - x[:K]).max() < 1e-10 * np.abs(x[:K]).max()
        assert np.abs(th[m] - x[K:]).max() < 1e-12 * np.abs(x[K:]).max()
        assert np.abs(free[m] - x[:K]).max() > 1e-4 * np.abs(x[:K]).max()


@pytest.mark.parametrize("scheme,dt,n,tol", [("bpr353", 1e-6, 30, 3e-7),
                                             ("cnab2", 1e-7, 120, 1e-6)])
def test_eigenmode_growth_with_implicit_buoyancy(scheme, dt, n, tol):
    K, m = 64, 12
    o = QGOracle(3e-6, 1e7, 0.025, 0.35, 39, 97, K, buoyancy="implicit")
    A, B = eigen.integration_operator(o.E, o.Ra, o.Pr, o.eta, m, K)
    sc = 1 / np.maximum(np.abs(A).max(1), np.abs(B).max(1))
    lam, V = sla.eig(A * sc[:, None], B * sc[:, None])
    ok = np.isfinite(lam)
    i = np.flatnonzero(ok)[np.argmax(lam[ok].real)]
    v = V[:, i] * 1e-8 / np.abs(V[:, i]).max()
    psi = np.zeros((o.M, K), complex)
    th = np.zeros_like(psi)
    psi[m], th[m] = v[:K], v[K:]
    o.set_state(psi, th, np.zeros(K))
    o.step(dt, scheme, n)
    y1 = np.concatenate([o.psi[m], o.theta[m]])
    o.step(dt, scheme, n)
    y2 = np.concatenate([o.psi[m], o.theta[m]])
    got = np.log(np.vdot(y1, y2) / np.vdot(y1, y1)) / (n * dt)
    assert abs(got - lam[i]) / abs(lam[i]) < tol, (got, lam[i])


def _run(scheme, dt, T, buoyancy):
    o = QGOracle(1e-3, 8e4, 1.0, 0.35, 24, 17, 10, buoyancy=buoyancy)
    st = inputs.make_state(o.M, o.K, "decaying", 5)
    o.set_state(100 * st.psi, 1e3 * st.theta, np.zeros(o.K))
    o.step(dt, scheme, int(round(T / dt)))
    return np.concatenate([o.psi.ravel(), o.theta.ravel(), o.uphi])


@pytest.fixture(scope="module")
def reference():
    T = 2e-3
    return T, _run("bpr353", T / 1280, T, "explicit")


@pytest.mark.parametrize("scheme,order", [("cnab2", 2), ("bpr353", 3),
                                          ("ars222", 2), ("sbdf3", 3)])
def test_temporal_order_with_implicit_buoyancy(scheme, order, reference):
    T, ref = reference
    errs = [np.linalg.norm(_run(scheme, T / n, T, "implicit") - ref)
            for n in (20, 40, 80)]
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(slopes > order - 0.3), slopes
    # and it is a different discretisation than the explicit one
    e = np.linalg.norm(_run(scheme, T / 20, T, "explicit") - ref)
    assert abs(e - errs[0]) > 1e-3 * e
