"""Mixed precision (FP32 transforms and advection products, FP64 solves,
state and diagnostics) against the FP64 oracle, through the C ABI.

The bound per field is 30 x the oracle's own spread under FP32-level
rounding noise in every transform (tests/golden/make_tolerances.py,
u = 2^-24); the measured errors are printed.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle.diagnostics import diagnostics as oracle_diagnostics
from oracle.step import QGOracle
from paper_1902_07092_amd import inputs

pytestmark = pytest.mark.gpu

_TOLS = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "parity_tolerances.json")))


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


@pytest.mark.parametrize("wname,scheme,nsteps,case", [
    ("SMALL", "cnab2", 50, "mixed_small_cnab2_50"),
    ("MEDIUM", "bpr353", 1, "mixed_medium_bpr353_1"),
    ("LARGE", "cnab2", 1, "mixed_large_cnab2_1")])
def test_mixed_precision_error_per_field(qg, wname, scheme, nsteps, case):
    w = getattr(inputs, wname)
    _say(f"[mixed] {w.n_phi}x{w.n_r} {scheme} x{nsteps}")
    st = inputs.workload_state(w)
    s = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c,
                    precision=1)
    s.set_state(st.psi, st.theta, st.uphi0)
    s.step(w.dt, scheme, nsteps)
    o = QGOracle(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c)
    o.set_state(st.psi, st.theta, st.uphi0)
    o.step(w.dt, scheme, nsteps)
    psi, th, up = s.get_state()
    err = dict(psi=_rel(psi, o.psi), theta=_rel(th, o.theta),
               uphi=_rel(up, o.uphi))
    dg, do = s.diagnostics(), oracle_diagnostics(o)
    err_ek = abs(dg["E_kin"] - do["E_kin"]) / abs(do["E_kin"])
    tol = _TOLS[case]["tol"]
    _say(f"  rel err {err}, E_kin {err_ek:.2e}; bound {tol}")
    for f in err:
        assert err[f] <= tol[f], (f, err[f], tol[f])
    # diagnostics are computed in FP64 from the (FP64) state
    assert err_ek <= max(10 * err["psi"], 1e-9), err_ek


def test_mixed_and_fp64_share_the_solves(qg):
    """A zero state stays zero and the factor choice is the same in both
    precisions (the band LU and solves are FP64 in both)."""
    w = inputs.SMALL
    st = inputs.workload_state(w)
    for prec in (0, 1):
        s = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c,
                        precision=prec)
        s.set_state(np.zeros_like(st.psi), np.zeros_like(st.theta),
                    np.zeros_like(st.uphi0))
        s.step(w.dt, "cnab2", 3)
        p, t, u = s.get_state()
        assert not p.any() and not t.any() and not u.any()
        assert s.diagnostics()["pivoted"] == 0


def _sample_errors(s, ref):
    """max |gpu - oracle| over the stored rows / max |oracle| over the whole
    field, per field (tests/golden/large_cnab2_50_samples.json)."""
    psi, th, up = s.get_state()
    out = {}
    for f, arr in (("psi", psi), ("theta", th)):
        d = 0.0
        for m, row in ref[f].items():
            r = np.array(row)
            d = max(d, float(np.abs(arr[int(m)] - (r[:, 0] + 1j * r[:, 1])).max()))
        out[f] = d / ref["max_abs"][f]
    out["uphi"] = float(np.abs(up - np.array(ref["uphi"])).max()
                        / ref["max_abs"]["uphi"])
    return out


@pytest.mark.parametrize("precision,case", [(0, "large_cnab2_50"),
                                            (1, "mixed_large_cnab2_50")])
def test_large_after_50_steps(qg, precision, case):
    """50 CNAB2 steps at 3072 x 1025 in FP64 and in mixed precision against
    the oracle's state after the same steps (sampled rows), in the launch
    configuration the benchmark times: the first 21 steps run the
    band-product autotuner, the rest use its choice."""
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "large_cnab2_50_samples.json")))
    w = inputs.LARGE
    assert ref["workload"] == w.name and ref["dt"] == w.dt
    _say(f"[large 50] precision {precision}")
    st = inputs.workload_state(w)
    s = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c,
                    precision=precision)
    s.set_state(st.psi, st.theta, st.uphi0)
    pick = s.step_autotune(w.dt, w.scheme, 21)
    s.step(w.dt, w.scheme, ref["steps"] - 21)
    err = _sample_errors(s, ref)
    _say(f"  band systems per thread {pick}")
    tol = _TOLS[case]["tol"]
    _say(f"  rel err {err}; bound {tol}")
    for f in err:
        assert err[f] <= max(1e-11, tol[f]), (f, err[f], tol[f])
