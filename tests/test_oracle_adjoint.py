"""Pins of the oracle's discrete adjoint (oracle/adjoint.py): every
transposed piece passes the dot-product test <A x, y> = <x, A^T y> against
the forward oracle function it transposes, and the gradient of the
time-integrated kinetic energy matches central finite differences."""
import numpy as np
import pytest

from oracle.adjoint import CNAB2Adjoint, dirichlet_free_to_full, full_to_free_T
from oracle.step import QGOracle
from oracle import transforms as tr
from paper_1902_07092_amd import inputs


def _ip(a, b):
    return sum(float(np.sum((np.conj(x) * y).real)) for x, y in zip(a, b))


@pytest.fixture(scope="module")
def setup():
    o = QGOracle(1e-3, 2.0e5, 1.0, 0.35, 48, 17)
    st = inputs.make_state(o.M, o.K, "decaying", 5)
    y = (st.psi * 40.0, st.theta * 40.0, np.zeros(o.K))
    u = inputs.dirichlet_from_basis(
        1e-2 * np.random.default_rng(3).standard_normal(o.K), o.K)
    y = (y[0], y[1], u)
    return o, CNAB2Adjoint(o), y


def _rand_state(o, seed):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal((o.M, o.K)) + 1j * rng.standard_normal((o.M, o.K))
    t = rng.standard_normal((o.M, o.K)) + 1j * rng.standard_normal((o.M, o.K))
    p[0] = 0
    t[0] = t[0].real
    return p, t, rng.standard_normal(o.K)


def test_transform_transposes(setup):
    o, adj, _ = setup
    rng = np.random.default_rng(1)
    c = rng.standard_normal((o.M, o.n_r)) + 1j * rng.standard_normal((o.M, o.n_r))
    g = rng.standard_normal((o.n_r, o.n_phi))
    lhs = float(np.sum(tr.phi_to_grid(c.T, o.n_phi) * g))
    assert np.isclose(lhs, _ip([c], [adj.to_grid_T(g)]), rtol=1e-12)
    X = rng.standard_normal((o.M, o.K)) + 1j * rng.standard_normal((o.M, o.K))
    spec = tr.grid_to_cheb(tr.grid_to_phi(g, o.M).T, o.K)
    assert np.isclose(_ip([spec], [X]), float(np.sum(g * adj.to_spec_T(X))),
                      rtol=1e-12)


def test_field_map_transpose(setup):
    o, adj, _ = setup
    y = _rand_state(o, 2)
    f = o.spectral_fields(*y)
    rng = np.random.default_rng(4)
    fb = {k: rng.standard_normal(v.shape) + 1j * rng.standard_normal(v.shape)
          for k, v in f.items()}
    lhs = _ip([fb[k] for k in f], [f[k] for k in f])
    yb = adj.fields_T(fb)
    assert np.isclose(lhs, _ip(yb, y), rtol=1e-12)


def test_solve_and_operator_transposes(setup):
    o, adj, _ = setup
    r = _rand_state(o, 5)
    xb = _rand_state(o, 6)
    adt = 0.5e-4
    x = o.solve(adt, *r)
    assert np.isclose(_ip(xb, x), _ip(adj.solve_T(adt, xb), r), rtol=1e-10)
    y = _rand_state(o, 7)
    my, ly = o.mass(*y), o.linear(*y)
    fwd = [a + 0.5e-4 * b for a, b in zip(my, ly)]
    fwd[0][0] = 0.0
    assert np.isclose(_ip(xb, fwd), _ip(adj.mass_lin_T(0.5e-4, xb), y), rtol=1e-10)


def test_explicit_transpose(setup):
    """E is quadratic, so (E(y + v) - E(y - v)) / 2 is its exact
    linearisation at y applied to v."""
    o, adj, y = setup
    v = _rand_state(o, 8)
    v = tuple(1e-3 * a for a in v)
    ep = o.explicit(*[a + b for a, b in zip(y, v)])
    em = o.explicit(*[a - b for a, b in zip(y, v)])
    jv = [(a - b) / 2 for a, b in zip(ep, em)]
    w = _rand_state(o, 9)
    assert np.isclose(_ip(w, jv), _ip(adj.explicit_T(y, *w), v), rtol=1e-9)


def test_gradient_matches_finite_differences(setup):
    o, adj, y = setup
    dt, n = 1e-4, 12
    free0 = y[1][:, 2:]

    def J(free):
        th = dirichlet_free_to_full(free)
        th[0] = th[0].real
        o.set_state(y[0], th, y[2])
        J_, _ = adj.gradient((y[0], th, y[2]), dt, n)
        return J_
    J0, g_full = adj.gradient((y[0], dirichlet_free_to_full(free0), y[2]), dt, n)
    g = full_to_free_T(g_full)
    g[0] = g[0].real                 # theta_0 is real: no imaginary direction
    rng = np.random.default_rng(11)
    for _ in range(3):
        d = rng.standard_normal(free0.shape) + 1j * rng.standard_normal(free0.shape)
        d[0] = d[0].real
        d /= np.linalg.norm(d)
        h = 1e-5 * np.linalg.norm(free0)
        fd = (J(free0 + h * d) - J(free0 - h * d)) / (2 * h)
        an = float(np.sum((np.conj(g) * d).real))
        assert abs(fd - an) <= 1e-7 * abs(an) + 1e-14 * abs(J0), (fd, an)


def _bc_state(o, seed):
    """A random state that satisfies the boundary conditions."""
    r = np.random.default_rng(seed)
    cp = r.standard_normal((o.M, o.K)) + 1j * r.standard_normal((o.M, o.K))
    ct = r.standard_normal((o.M, o.K)) + 1j * r.standard_normal((o.M, o.K))
    cp[0] = 0
    ct[0] = ct[0].real
    return (inputs.psi_from_basis(cp, o.K), inputs.dirichlet_from_basis(ct, o.K),
            inputs.dirichlet_from_basis(r.standard_normal(o.K), o.K).real)


def test_transposed_step_map_matches_finite_differences(setup):
    """J^T w of the 8-step map y^0 -> y^8 (transpose_map): <J^T w, v>
    equals <w, (Phi(y + h v) - Phi(y - h v)) / 2h> to O(h^2) (measured at
    the time of writing: 2.1e-7 at h = 1e-4, 2.1e-9 at h = 1e-5)."""
    from oracle.adjoint import transpose_map
    o, adj, y0 = setup
    v, w = _bc_state(o, 11), _bc_state(o, 12)
    dt, n = 1e-4, 8
    rhs = _ip(transpose_map(adj, y0, dt, n, w), v)

    def phi(y):
        o.set_state(*y)
        o.step(dt, "cnab2", n)
        return (o.psi.copy(), o.theta.copy(), o.uphi.copy())
    errs = []
    for h in (1e-4, 1e-5):
        fp = phi(tuple(a + h * b for a, b in zip(y0, v)))
        fm = phi(tuple(a - h * b for a, b in zip(y0, v)))
        lhs = _ip(w, [(a - b) / (2 * h) for a, b in zip(fp, fm)])
        errs.append(abs(lhs - rhs) / abs(rhs))
    assert errs[1] < 1e-8 and errs[0] / errs[1] > 50, errs
