"""Reverse mode on the GPU (qg_adjoint_explicit, qg_gradient) through the C
ABI, against the oracle's discrete adjoint (oracle.adjoint, dense per-m
transposes built from the oracle's own maps), the GPU's own tangent-linear
model (dot-product test) and central differences of the GPU's forward
energy integral at 768 x 257 over 200 CNAB2 steps (Sect. 4 eq. multistep1,
Appendix A, Sect. 6.2).
"""
import sys

import numpy as np
import pytest

from oracle.adjoint import CNAB2Adjoint, dirichlet_free_to_full
from oracle.step import QGOracle
from paper_1902_07092_amd import inputs

pytestmark = pytest.mark.gpu

E, RA, PR, ETA, N_PHI, N_R = 1e-3, 2.0e5, 1.0, 0.35, 48, 17
DT, N = 1e-4, 8


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def qg():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    from paper_1902_07092_amd import qg as mod
    mod.load()
    return mod


def _np(t):
    return t.detach().cpu().numpy()


def _ip(a, b):
    return sum(float(np.sum((np.conj(x) * y).real)) for x, y in zip(a, b))


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _bc_state(M, K, seed):
    r = np.random.default_rng(seed)
    cp = r.standard_normal((M, K)) + 1j * r.standard_normal((M, K))
    ct = r.standard_normal((M, K)) + 1j * r.standard_normal((M, K))
    cp[0] = 0
    ct[0] = ct[0].real
    return (inputs.psi_from_basis(cp, K), inputs.dirichlet_from_basis(ct, K),
            inputs.dirichlet_from_basis(r.standard_normal(K), K).real)


@pytest.fixture(scope="module")
def case():
    """48 x 17 in the nonlinear regime (the tangent tests' case): a state
    with every field and the zonal flow nonzero."""
    o = QGOracle(E, RA, PR, ETA, N_PHI, N_R)
    st = inputs.make_state(o.M, o.K, "decaying", 5)
    u = inputs.dirichlet_from_basis(
        1e-2 * np.random.default_rng(3).standard_normal(o.K), o.K)
    y0 = (st.psi * 40.0, st.theta * 40.0, u)
    return o, y0


def _solver(qg, o):
    return qg.QGSolver(E, RA, PR, ETA, N_PHI, N_R, o.K)


def test_adjoint_explicit_matches_oracle(qg, case):
    """E'(y)^H eb + kappa grad E_K(y) at a stepped (nonlinear) state on
    random co-states, against the oracle's transposed explicit terms."""
    o, y0 = case
    o.set_state(*y0)
    o.step(DT, "cnab2", 3)
    y = (o.psi.copy(), o.theta.copy(), o.uphi.copy())
    adj = CNAB2Adjoint(o)
    rng = np.random.default_rng(31)
    eb = [rng.standard_normal((o.M, o.K)) + 1j * rng.standard_normal((o.M, o.K)),
          rng.standard_normal((o.M, o.K)) + 1j * rng.standard_normal((o.M, o.K)),
          rng.standard_normal(o.K)]
    # the co-states the reverse sweep feeds in have zero tau rows (the
    # transposed solve zeroes them; the step replaces those rows of E)
    eb[0][0] = 0.0
    eb[0][:, :4] = 0.0
    eb[1][:, :2] = 0.0
    eb[2][:2] = 0.0
    kappa = 0.37
    s = _solver(qg, o)
    for kap in (0.0, kappa):
        ref = adj.explicit_T(y, *eb)
        if kap:
            gk = adj.grad_EK(y)
            ref = tuple(a + kap * b for a, b in zip(ref, gk))
        got = [_np(t) for t in s.adjoint_explicit(y, eb, kap)]
        err = {"psi": _rel(got[0][1:], ref[0][1:]), "theta": _rel(got[1], ref[1]),
               "uphi": _rel(got[2], ref[2])}
        _say(f"[adjoint explicit] kappa {kap}: rel err {err}")
        assert not got[0][0].any()
        assert max(err.values()) < 1e-11, err


def test_gradient_matches_oracle_adjoint(qg, case):
    """J and dJ/dy^0 over 8 CNAB2 steps against the oracle's reverse
    sweep; the gradient does not depend on the checkpoint interval (the
    recomputed trajectory is the stored one, bit for bit), and the context
    ends where qg_step leaves it."""
    o, y0 = case
    J_ref, gth_ref = CNAB2Adjoint(o).gradient(y0, DT, N)
    out = {}
    for interval in (1, 3, 8):
        s = _solver(qg, o)
        s.set_state(*y0)
        J, g = s.gradient(DT, N, interval)
        out[interval] = (J, [_np(t) for t in g])
        if interval == 3:
            plain = _solver(qg, o)
            plain.set_state(*y0)
            plain.step(DT, "cnab2", N)
            for a, b in zip(s.get_state(), plain.get_state()):
                assert np.array_equal(a, b)
            # the history continues as after qg_step
            s.step(DT, "cnab2", 2)
            plain.step(DT, "cnab2", 2)
            for a, b in zip(s.get_state(), plain.get_state()):
                assert np.array_equal(a, b)
    J, g = out[3]
    errJ = abs(J - J_ref) / abs(J_ref)
    errg = _rel(g[1], gth_ref)
    _say(f"[gradient] J {J:.15e} oracle {J_ref:.15e} (rel {errJ:.2e}); "
         f"dJ/dtheta rel err {errg:.2e}")
    assert errJ < 1e-12 and errg < 1e-11, (errJ, errg)
    for interval in (1, 8):
        assert out[interval][0] == J
        for a, b in zip(out[interval][1], g):
            assert np.array_equal(a, b), interval


def test_gradient_dot_product_with_tangent(qg, case):
    """<w, J v> from the GPU tangent-linear model (qg_step_tangent) and
    <J^T w, v> from the reverse sweep with terminal co-state w and no
    energy term: the derivative of N steps and its transpose, computed by
    different GPU code paths, agree to rounding."""
    o, y0 = case
    v = _bc_state(o.M, o.K, 11)
    rng = np.random.default_rng(13)
    w = (rng.standard_normal((o.M, o.K)) + 1j * rng.standard_normal((o.M, o.K)),
         rng.standard_normal((o.M, o.K)) + 1j * rng.standard_normal((o.M, o.K)),
         rng.standard_normal(o.K))
    w[0][0] = 0.0
    s = _solver(qg, o)
    s.set_state(*y0)
    s.tangent_set(*v)
    s.step_tangent(DT, N)
    lhs = _ip(w, s.tangent_get())
    s2 = _solver(qg, o)
    s2.set_state(*y0)
    _, g = s2.gradient(DT, N, 3, energy_weight=0.0, terminal=w)
    rhs = _ip([_np(t) for t in g], v)
    rel = abs(lhs - rhs) / abs(rhs)
    _say(f"[gradient] <w, J v> tangent {lhs:.15e}, <J^T w, v> reverse {rhs:.15e}, "
         f"rel {rel:.2e}")
    assert rel < 1e-12, (lhs, rhs)


def test_energy_gradient_autograd(qg, case):
    """The torch.autograd.Function wrapper: J.backward() gives the
    library's gradient."""
    import torch
    o, y0 = case
    s = _solver(qg, o)
    th = torch.tensor(y0[1], dtype=torch.complex128, device=s.device, requires_grad=True)
    J = qg.energy_integral(th, s, y0[0], y0[2], DT, N, 4)
    J.backward()
    s2 = _solver(qg, o)
    s2.set_state(*y0)
    J2, g = s2.gradient(DT, N, 4)
    assert float(J) == J2
    assert torch.equal(th.grad, g[1])


def test_gradient_errors(qg, case):
    o, y0 = case
    s = qg.QGSolver(E, RA, PR, ETA, N_PHI, N_R, o.K, precision=1)
    s.set_state(*y0)
    with pytest.raises(qg.QGError) as e:
        s.gradient(DT, 2)
    assert e.value.status == qg.QG_EUNSUPPORTED
    s = qg.QGSolver(E, RA, PR, ETA, N_PHI, N_R, o.K, pivoting=1)
    s.set_state(*y0)
    with pytest.raises(qg.QGError) as e:
        s.gradient(DT, 2)
    assert e.value.status == qg.QG_EUNSUPPORTED
    # J alone needs no adjoint solve
    J = s.energy_integral(DT, 2)
    assert J > 0


def test_gradient_central_differences_768x257():
    """dJ/dtheta^0 at 768 x 257 over 200 CNAB2 steps (the adjoint
    workload) against central differences of the GPU's forward J in 16
    random admissible directions (seeds 500 .. 515): <= 1e-6 relative.
    The difference quotient is the fourth-order one,
    (J(-2h) - 8 J(-h) + 8 J(h) - J(2h)) / 12h, at h = 1e-3 of max |theta|:
    J carries the FP64 rounding of the step at this size (the oracle
    itself loses 1e-11 of Psi per step here), which with the two-point
    quotient gave 2e-7 at h = 1e-4, 3e-6 at 1e-5 and 5e-5 at 1e-6
    (measured), so the step must stay large and the quotient's own
    truncation small."""
    import torch
    from paper_1902_07092_amd import qg
    qg.load()
    assert torch.cuda.is_available()
    w = inputs.ADJOINT
    st = inputs.workload_state(w)
    s = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c)
    s.set_state(st.psi, st.theta, st.uphi0)
    J0, g = s.gradient(w.dt, w.steps, 20)
    gth = _np(g[1])
    scale = float(np.abs(st.theta).max())
    worst = 0.0
    for seed in range(500, 516):
        d = inputs.make_direction(w.M, w.n_c, seed)
        v = dirichlet_free_to_full(d[:, 2:])
        h = 1e-3 * scale / float(np.abs(v).max())
        Js = {}
        for k in (-2, -1, 1, 2):
            s.set_state(st.psi, st.theta + k * h * v, st.uphi0)
            Js[k] = s.energy_integral(w.dt, w.steps)
        fd = (Js[-2] - 8.0 * Js[-1] + 8.0 * Js[1] - Js[2]) / (12.0 * h)
        ad = float(np.sum((np.conj(gth) * v).real))
        rel = abs(fd - ad) / abs(ad)
        worst = max(worst, rel)
        _say(f"[gradient 768x257] seed {seed}: adjoint {ad:.12e}, central "
             f"difference {fd:.12e}, rel {rel:.2e}")
    assert worst <= 1e-6, worst
