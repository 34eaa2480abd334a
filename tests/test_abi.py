"""Host-side checks of the C ABI library (no GPU needed): every symbol of
include/qg.h is exported, parameter validation, and the host-built
integration operators against the oracle's."""
import os
import re

import numpy as np
import pytest

from oracle.operators import IntegrationOperators

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qg.h")


@pytest.fixture(scope="module")
def qg():
    from paper_1902_07092_amd import qg as mod
    mod.load()
    return mod


def test_header_symbols_exported(qg):
    text = open(HEADER).read()
    names = set(re.findall(r"^(?:qg_status|void|const char \*)\s*\*?\s*"
                           r"(qg_[a-z_]+)\s*\(", text, flags=re.M))
    assert {"qg_create", "qg_step", "qg_diagnostics", "qg_set_state",
            "qg_get_state", "qg_destroy", "qg_workspace_size",
            "qg_last_error", "qg_operator_band"} <= names
    lib = qg.load()
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("bad", [
    dict(n_phi=95), dict(n_phi=12), dict(eta=1.2), dict(eta=0.0),
    dict(n_c=33), dict(n_c=5), dict(precision=2), dict(E=0.0),
    dict(Pr=-1.0), dict(n_r=9), dict(pivoting=2), dict(pivoting=-1),
    dict(ekman=2), dict(ekman=1, eps=0.0), dict(ekman=1, eps=float("inf"))])
def test_workspace_size_rejects_invalid(qg, bad):
    p = dict(E=1e-3, Ra=8e4, Pr=1.0, eta=0.35, n_phi=96, n_r=33, n_c=0,
             precision=0, pivoting=0)
    p.update(bad)
    with pytest.raises(qg.QGError) as e:
        qg.qg_workspace_size(qg.qg_params(**p))
    assert e.value.status == qg.QG_EINVAL


def test_workspace_size_grows_with_problem(qg):
    small = qg.qg_workspace_size(qg.qg_params(1e-3, 8e4, 1, .35, 96, 33, 0, 0))
    large = qg.qg_workspace_size(qg.qg_params(1e-8, 1e12, 1, .35, 3072, 1025,
                                              0, 0))
    assert 0 < small < large < 2 * 1024**3


def test_ensemble_workspace_groups_members(qg):
    """Members that differ only in Ra share one group (operators, tables,
    factors); the per-run arrays scale with the group size.  A single-run
    context holds more than a one-member group: the second state slot of
    its discardable steps and the tangent-linear arrays."""
    a = qg.qg_params(1e-5, 2e7, 1.0, 0.35, 192, 65, 0, 0, 0)
    a2 = qg.qg_params(1e-5, 3e8, 1.0, 0.35, 192, 65, 0, 0, 0)
    b = qg.qg_params(1e-5, 5e7, 1.0, 0.35, 96, 33, 0, 0, 0)
    solo_a = qg.qg_workspace_size(a)
    one_a = qg.qg_ensemble_workspace_size([a])
    one_b = qg.qg_ensemble_workspace_size([b])
    assert one_a < solo_a
    pair = qg.qg_ensemble_workspace_size([a, a2])
    assert one_a < pair < 2 * one_a          # shared factors and tables
    mixed = qg.qg_ensemble_workspace_size([a, b, a2])
    assert mixed == qg.qg_ensemble_workspace_size([b, a2, a])
    assert mixed == pair + one_b
    bad = qg.qg_params(1e-5, 2e7, 1.0, 0.35, 95, 65, 0, 0, 0)
    with pytest.raises(qg.QGError):
        qg.qg_ensemble_workspace_size([a, bad])
    with pytest.raises(qg.QGError):
        qg.qg_ensemble_workspace_size([])


@pytest.mark.parametrize("K", [12, 21, 170])
def test_host_operators_match_oracle(qg, K):
    o = IntegrationOperators(0.35, K)
    names = ["A0", "A2", "B0", "B2", "B4", "C", "D", "F0", "F2"]
    for which, nm in enumerate(names):
        band = qg.qg_operator_band(0.35, K, which)
        q = 4 if nm[0] in "ABC" else 2
        full = np.zeros((K, K))
        for k in range(q, K):
            for off in range(-8, 9):
                if 0 <= k + off < K:
                    full[k, k + off] = band[k, off + 8]
        ref = getattr(o, nm)
        assert np.abs(band[:q]).max() == 0.0
        err = np.abs(full[q:] - ref[q:]).max() / np.abs(ref[q:]).max()
        assert err < 1e-13, (nm, err)
