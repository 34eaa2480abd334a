"""Write tests/golden/reference/<case>.json: extended-precision reference
states of the parity workloads, and the FP64 oracle's distance from them.

For every case the seeded initial state is stepped twice by the oracle:
in FP64 and in long double (oracle.step.QGOracle(dtype=np.longdouble):
every product, transform and operator in long double, bordered solves
refined to long-double accuracy).  The file holds the long-double state
(rounded to binary64) on the sampled rows, the maxima of the full fields,
and the FP64 oracle's error against it, over the full fields and over the
sampled entries, also per sampled row, and the same errors of a second
binary64 implementation of the step (the oracle with band LUs without row
interchanges, pivot=False).  Where added (--add-galerkin), the errors of
the two FP64 Galerkin implementations (oracle method="galerkin", with and
without row interchanges) are stored as well: the Galerkin bases solve for
the same Chebyshev coefficients, so the same reference serves both
formulations.  The GPU parity tests (tests/refcheck.py) hold the HIP path
to the same reference.

The 12288 x 4097 case (mixed precision on the GPU only) stores the FP64
oracle's state as its reference: its rounding is far below the FP32
transforms' that case measures.

Calls only the oracle and the seeded input generators.  Usage:
    python tests/golden/make_reference.py [case ...]     (default: all)
    python tests/golden/make_reference.py --add-variant case ...
    python tests/golden/make_reference.py --add-galerkin case ...
(the second form adds the unpivoted run's errors to existing files, the
third the two Galerkin runs' errors).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.step import QGOracle  # noqa: E402
from paper_1902_07092_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "reference")
SMALL_RUNS = [("cnab2", 1), ("cnab2", 20), ("bpr353", 5), ("ars222", 6),
              ("ars443", 5), ("sbdf2", 8), ("sbdf3", 8), ("sbdf4", 8),
              ("cnab2", 100)]
MED_ROWS = (0, 1, 2, 8, 32, 64, 128, 192, 256)
LARGE_ROWS = (0, 1, 2, 20, 100, 256, 512, 855, 1024)


def _cases():
    c = {}
    for scheme, n in SMALL_RUNS:
        c[f"small_{scheme}_{n}"] = dict(w="SMALL", scheme=scheme, steps=n,
                                        rows=None, stride=1)
    for n in (2, 20, 500):
        c[f"medium_bpr353_{n}"] = dict(w="MEDIUM", scheme="bpr353", steps=n,
                                       rows=MED_ROWS, stride=1)
    for n in (2, 50):
        c[f"large_cnab2_{n}"] = dict(w="LARGE", scheme="cnab2", steps=n,
                                     rows=LARGE_ROWS, stride=2)
    c["mid_cnab2_2"] = dict(w="LARGE_MID", scheme="cnab2", steps=2,
                            rows=(0, 1, 20, 1024, 2048), stride=4)
    c["top_cnab2_1"] = dict(w="LARGE_TOP", scheme="cnab2", steps=1,
                            rows=(0, 1, 20, 2048, 4096), stride=8, fp64_ref=True)
    # member 7 of the seeded 64-run ensemble (192 x 65, Ra = 4.02 Ra_c)
    c["ensemble7_cnab2_10"] = dict(w="ensemble:7", scheme="cnab2", steps=10,
                                   rows=None, stride=1)
    return c


CASES = _cases()


def _sample(a, rows, stride):
    return a if rows is None else a[list(rows), ::stride]


def _cplx(a):
    return [[float(v.real), float(v.imag)] for v in a]


def make(name):
    spec = CASES[name]
    w = (inputs.ensemble_workloads()[int(spec["w"].split(":")[1])]
         if spec["w"].startswith("ensemble:") else getattr(inputs, spec["w"]))
    st = inputs.workload_state(w)
    runs = {}
    kinds = (np.float64,) if spec.get("fp64_ref") else (np.float64, np.longdouble)
    for dt_ in kinds:
        t0 = time.time()
        o = QGOracle(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c, dtype=dt_)
        o.set_state(st.psi, st.theta, st.uphi0)
        o.step(w.dt, spec["scheme"], spec["steps"])
        runs[dt_] = o
        print(f"[{name}] {dt_.__name__}: {spec['steps']} {spec['scheme']} steps "
              f"in {time.time() - t0:.0f} s", flush=True)
    ref = runs[kinds[-1]]
    orc = runs[np.float64]
    rows, stride = spec["rows"], spec["stride"]
    fields = ("psi", "theta", "uphi")
    out = dict(case=name, workload=w.name, n_phi=w.n_phi, n_r=w.n_r,
               n_c=w.n_c, E=w.E, Ra=w.Ra, Pr=w.Pr, eta=w.eta,
               scheme=spec["scheme"], dt=w.dt, steps=spec["steps"],
               initial_state=f"{w.ic}, seed {w.seed}",
               reference=("FP64 oracle" if spec.get("fp64_ref") else
                          "oracle in long double, refined solves"),
               rows=list(rows) if rows is not None else None, stride=stride)
    if not spec.get("fp64_ref"):
        floor = max((r for _, r in ref.refine_its), default=0.0)
        out["refine_floor"] = floor
    out["max_abs"] = {f: float(np.abs(getattr(ref, f)).max()) for f in fields}
    out["ref"] = {}
    out["oracle_err"] = {}
    out["oracle_err_sampled"] = {}
    out["oracle_row_err"] = {}
    for f in fields:
        R = getattr(ref, f)
        X = getattr(orc, f)
        scale = out["max_abs"][f]
        if f == "uphi":
            out["ref"][f] = [float(v) for v in R[::stride]]
            d = np.abs(X - R)
            out["oracle_err"][f] = float(d.max() / scale) if scale else 0.0
            out["oracle_err_sampled"][f] = (float(d[::stride].max() / scale)
                                            if scale else 0.0)
            continue
        Rs, Xs = _sample(R, rows, stride), _sample(X, rows, stride)
        mlist = list(rows) if rows is not None else list(range(R.shape[0]))
        out["ref"][f] = {str(m): _cplx(Rs[i]) for i, m in enumerate(mlist)}
        out["oracle_err"][f] = float(np.abs(X - R).max() / scale) if scale else 0.0
        out["oracle_err_sampled"][f] = (float(np.abs(Xs - Rs).max() / scale)
                                        if scale else 0.0)
        out["oracle_row_err"][f] = {
            str(m): float(np.abs(Xs[i] - Rs[i]).max()) for i, m in enumerate(mlist)}
    if not spec.get("fp64_ref"):
        _variant(name, w, st, spec, out)
    _write(name, out)


def _write(name, out):
    os.makedirs(OUT, exist_ok=True)
    path = os.path.join(OUT, f"{name}.json")
    with open(path + ".tmp", "w") as fh:
        json.dump(out, fh, separators=(",", ":"))
    os.replace(path + ".tmp", path)
    print(f"[{name}] wrote {path} ({os.path.getsize(path)} bytes); FP64 oracle "
          f"error {out['oracle_err_sampled']}; unpivoted "
          f"{out.get('variant_err_sampled')}; Galerkin "
          f"{out.get('galerkin_err_sampled')}, {out.get('galerkin_np_err_sampled')}",
          flush=True)


# Further FP64 implementations: key prefix -> oracle options.
IMPLS = {"variant": dict(pivot=False),
         "galerkin": dict(method="galerkin"),
         "galerkin_np": dict(method="galerkin", pivot=False)}


def _variant(name, w, st, spec, out, key="variant"):
    """Another FP64 implementation (IMPLS[key]) against the stored
    reference entries."""
    t0 = time.time()
    v = QGOracle(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c, **IMPLS[key])
    v.set_state(st.psi, st.theta, st.uphi0)
    v.step(w.dt, spec["scheme"], spec["steps"])
    print(f"[{name}] {key} float64: {spec['steps']} {spec['scheme']} steps "
          f"in {time.time() - t0:.0f} s", flush=True)
    stride = out["stride"]
    out[f"{key}_err_sampled"], out[f"{key}_row_err"] = {}, {}
    for f in ("psi", "theta", "uphi"):
        scale = out["max_abs"][f]
        a = np.asarray(getattr(v, f))
        if f == "uphi":
            d = np.abs(a[::stride] - np.array(out["ref"][f]))
            out[f"{key}_err_sampled"][f] = float(d.max() / scale) if scale else 0.0
            continue
        rows = {}
        for m, r in out["ref"][f].items():
            r = np.array([complex(x, y) for x, y in r])
            rows[m] = float(np.abs(a[int(m), ::stride] - r).max())
        out[f"{key}_row_err"][f] = rows
        out[f"{key}_err_sampled"][f] = (max(rows.values()) / scale) if scale else 0.0


def add_variant(name, keys=("variant",)):
    """Adds further FP64 implementations' errors to an existing reference
    file."""
    spec = CASES[name]
    with open(os.path.join(OUT, f"{name}.json")) as fh:
        out = json.load(fh)
    w = (inputs.ensemble_workloads()[int(spec["w"].split(":")[1])]
         if spec["w"].startswith("ensemble:") else getattr(inputs, spec["w"]))
    assert out["workload"] == w.name and out["steps"] == spec["steps"]
    for key in keys:
        _variant(name, w, inputs.workload_state(w), spec, out, key)
    _write(name, out)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--add-variant":
        for name in args[1:]:
            add_variant(name)
    elif args and args[0] == "--add-galerkin":
        for name in args[1:]:
            add_variant(name, ("galerkin", "galerkin_np"))
    else:
        for name in (args or list(CASES)):
            make(name)
