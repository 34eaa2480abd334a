"""qg_create_static: the allocation-free entry point (its workspace is the
library's static device array), against qg_create with a caller-allocated
workspace, through the C ABI: the same steps give the same state bit for
bit, on two contexts in a row, the second one smaller; the array is held by
one context per device at a time, and sizes beyond it are refused."""
import sys

import numpy as np
import pytest

from paper_1902_07092_amd import inputs

pytestmark = pytest.mark.gpu


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


def _run(qg, w, static, scheme, n):
    s = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c,
                    static_workspace=static)
    st = inputs.make_state(w.M, w.n_c, "decaying", 21)
    st.psi *= 10.0
    st.theta *= 1e3
    s.set_state(st.psi, st.theta, st.uphi0)
    s.step(w.dt, scheme, n)
    out = s.get_state()
    d = s.diagnostics()
    return s, out, d


def test_static_workspace_equals_allocated_workspace(qg):
    big = [w for w in inputs.ensemble_workloads() if w.n_r == 129][0]
    small = inputs.SMALL
    for w, scheme, n in ((big, "cnab2", 6), (small, "bpr353", 4)):
        _say(f"[no-alloc] {w.n_phi}x{w.n_r} {scheme} x{n}")
        s, a, da = _run(qg, w, True, scheme, n)
        # while it lives, the static array is not handed out again
        with pytest.raises(qg.QGError) as e:
            qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c,
                        static_workspace=True)
        assert e.value.status == qg.QG_EINVAL
        del s
        _, b, db = _run(qg, w, False, scheme, n)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        assert da["E_kin"] == db["E_kin"] and da["step"] == db["step"] == n


def test_static_workspace_refuses_large_sizes(qg):
    w = inputs.MEDIUM
    s = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c)
    del s
    with pytest.raises(qg.QGError) as e:
        qg.QGSolver(1e-8, 1e12, 1.0, 0.35, 3072, 1025, static_workspace=True)
    assert e.value.status == qg.QG_ENOMEM
    assert "static workspace" in str(e.value)
