"""Write tests/golden/large_cnab2_50_samples.json: the oracle's state after
50 CNAB2 steps of the 3072 x 1025 workload, sampled (whole Chebyshev rows
of a few wavenumbers, the zonal flow), with the full-field maxima that the
relative error measure divides by.  The GPU tests compare the FP64 and the
mixed-precision runs against it; a live oracle run of 50 steps at this size
takes minutes.

Calls only the oracle and the seeded input generators.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.step import QGOracle  # noqa: E402
from paper_1902_07092_amd import inputs  # noqa: E402

ROWS = (0, 1, 20, 256, 1024)
STEPS = 50


def main():
    w = inputs.LARGE
    st = inputs.workload_state(w)
    o = QGOracle(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c)
    o.set_state(st.psi, st.theta, st.uphi0)
    o.step(w.dt, w.scheme, STEPS)

    def cplx(a):
        return [[float(v.real), float(v.imag)] for v in a]
    out = {"workload": w.name, "scheme": w.scheme, "dt": w.dt,
           "steps": STEPS, "rows": list(ROWS),
           "max_abs": {"psi": float(np.abs(o.psi).max()),
                       "theta": float(np.abs(o.theta).max()),
                       "uphi": float(np.abs(o.uphi).max())},
           "psi": {str(m): cplx(o.psi[m]) for m in ROWS if m > 0},
           "theta": {str(m): cplx(o.theta[m]) for m in ROWS},
           "uphi": [float(v) for v in o.uphi]}
    path = os.path.join(HERE, "large_cnab2_50_samples.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("wrote", path, os.path.getsize(path), "bytes")


if __name__ == "__main__":
    main()
