"""The radial transforms on the FP64 matrix cores (qg_params.dct = 2:
eq. cheb and icheb as dense products per m, 2 (N_r - 1) <= 512) through
the C ABI: against the oracle at the parity bar, against the FFT
transforms of the same library, against the extended-precision reference
at 768 x 257, with Ekman pumping and in an ensemble."""
import sys

import numpy as np
import pytest

import refcheck
from oracle.step import QGOracle
from paper_1902_07092_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-11


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


def _rel(a, b):
    scale = np.abs(b).max()
    return float(np.abs(a - b).max() / scale) if scale > 0 else float(
        np.abs(a).max())


def _state(M, K, strong=False):
    """The radial-size tests' state (decaying seed 7, theta x 100), or a
    strongly nonlinear one with a zonal flow (strong=True: FP64 itself
    loses ~1e-11 on it at 384 x 193, the FFT and matrix-core transforms
    alike, measured 1.1e-11 and 3e-12 apart)."""
    if not strong:
        st = inputs.make_state(M, K, "decaying", 7)
        st.theta *= 1e2
        return st
    st = inputs.make_state(M, K, "decaying", 21)
    st.psi *= 10.0
    st.theta *= 1e3
    st.uphi0 = inputs.dirichlet_from_basis(np.linspace(1.0, 0.1, K), K).real * 0.5
    return st


@pytest.mark.parametrize("n_phi,n_r", [(48, 17), (96, 33), (96, 49), (192, 65),
                                       (384, 129), (384, 193)])
def test_mfma_dct_parity(qg, n_phi, n_r):
    w = inputs.SMALL
    K = (2 * (n_r - 1)) // 3
    M = n_phi // 3 + 1
    st = _state(M, K)
    _say(f"[mfma dct] {n_phi}x{n_r} K={K}")
    runs = {}
    for dct in ("mfma", "fft"):
        s = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, n_phi, n_r, K, dct=dct)
        s.set_state(st.psi, st.theta, st.uphi0)
        s.step(w.dt, "cnab2", 3)
        s.step(w.dt, "bpr353", 1)
        runs[dct] = s.get_state()
    o = QGOracle(w.E, w.Ra, w.Pr, w.eta, n_phi, n_r, K)
    o.set_state(st.psi, st.theta, st.uphi0)
    o.step(w.dt, "cnab2", 3)
    o.step(w.dt, "bpr353", 1)
    err = {f: _rel(a, b) for f, a, b in zip(refcheck.FIELDS, runs["mfma"],
                                            (o.psi, o.theta, o.uphi))}
    d = {f: _rel(a, b) for f, a, b in zip(refcheck.FIELDS, runs["mfma"], runs["fft"])}
    _say(f"  against the oracle {err}; against the FFT transforms {d}")
    assert max(err.values()) < TOL, err
    assert max(d.values()) < TOL, d


def test_mfma_dct_medium_reference(qg):
    """768 x 257, 2 BPR353 steps: the reference criterion of refcheck."""
    w = inputs.MEDIUM
    s = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c, dct="mfma")
    st = inputs.workload_state(w)
    s.set_state(st.psi, st.theta, st.uphi0)
    s.step(w.dt, "bpr353", 2)
    ref = refcheck.load("medium_bpr353_2")
    err, _ = refcheck.check(ref, s.get_state())
    _say(f"[mfma dct] medium 2 steps vs reference: {refcheck.report(ref, err)}")


def test_mfma_dct_with_pumping_and_ensemble(qg):
    w = inputs.SMALL
    st = _state(w.M, w.n_c, strong=True)
    s = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c,
                    ekman_eps=1e-2, dct="mfma")
    o = QGOracle(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c, ekman_eps=1e-2)
    for x in (s, o):
        x.set_state(st.psi, st.theta, st.uphi0)
    s.step(w.dt, "cnab2", 4)
    o.step(w.dt, "cnab2", 4)
    err = {f: _rel(a, b) for f, a, b in zip(refcheck.FIELDS, s.get_state(),
                                            (o.psi, o.theta, o.uphi))}
    _say(f"[mfma dct] pumping: {err}")
    assert max(err.values()) < TOL, err
    mem = inputs.ensemble_workloads()[7]
    members = [dict(E=mem.E, Ra=mem.Ra * f, Pr=mem.Pr, eta=mem.eta, n_phi=mem.n_phi,
                    n_r=mem.n_r, n_c=mem.n_c, dct=d)
               for f, d in ((1.0, "mfma"), (2.0, "mfma"), (1.0, "fft"))]
    ens = qg.QGEnsemble(members)
    st7 = inputs.workload_state(mem)
    for i in range(3):
        ens.set_state(i, st7.psi, st7.theta, st7.uphi0)
    ens.step(mem.dt, "cnab2", 10)
    got = ens.get_state(0)
    ref = refcheck.load("ensemble7_cnab2_10")
    e, _ = refcheck.check(ref, got)
    _say(f"[mfma dct] ensemble member 7: {refcheck.report(ref, e)}")
    d = {f: _rel(a, b) for f, a, b in zip(refcheck.FIELDS, got, ens.get_state(2))}
    _say(f"  against the FFT member {d}")
    assert max(d.values()) < TOL, d


def test_mfma_dct_statuses(qg):
    w = inputs.LARGE
    with pytest.raises(qg.QGError) as e:
        qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c, dct="mfma")
    assert e.value.status == qg.QG_EUNSUPPORTED
    w = inputs.SMALL
    with pytest.raises(qg.QGError) as e:
        qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c, dct="mfma",
                    precision=1)
    assert e.value.status == qg.QG_EUNSUPPORTED
