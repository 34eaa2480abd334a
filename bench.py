#!/usr/bin/env python
"""Benchmark of the FP64 IMEX step of spherical QG convection on one GPU.

Workload (default): 3072 x 1025 grid (N_m = 1024, N_c = 682), E = 1e-8,
Pr = 1, Ra = 20 Ra_c, CNAB2, dt = 2.5e-10, seeded turbulent-like initial
state (k^-5/3 spectrum steepening past m ~ 20, random phases, Re = 1e4).
Beside it: the same steps with FP32 transforms and products, the cost of
one step of every other time scheme of Table 1 relative to CNAB2, the cost
of a tangent-linear step against a forward step at 768 x 257, and the
batched ensemble of 64 runs of uneven size and Ra.  A step is one CNAB2 step of the
whole hot path: Chebyshev synthesis, azimuthal FFTs and products, radial
analysis, explicit terms, right-hand sides and the bordered solves of every
m.  The state is resident in HBM before the timed region; the time-step
factorisation is done once before it (as in the paper's timings), and so
are the library's autotuner steps (launch shape of the band products).

Prints one JSON line (metric, value = grid-point-steps/s, roofline of the
dominant kernel measured with HIP events on the solver's stream, CPU
baseline of the oracle on the host cores).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point-steps/s FP64 vs mixed/batched; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0


def alg_bytes(kernel, M, R, K, nterm=2, mixed=False):
    """Compulsory HBM bytes of one launch: the kernel's own inputs and
    outputs, factor re-reads excluded.  Spectral arrays are FP64 complex
    (16 B); the exchange arrays X and NL are too, or FP32 complex (8 B) in
    the mixed-precision step."""
    c = 16
    x = 8 if mixed else 16
    return {
        "synth": 2 * M * K * c + 6 * R * M * x,
        "ring": 8 * R * M * x + 8 * R,
        "analysis": 2 * R * M * x + 8 * R + 3 * M * K * c,
        "solve": 2 * 2 * M * K * c,
        "rhs": (2 + nterm) * 2 * M * K * c,
    }[kernel]


def factor_bytes(kernel, M, K, pad=48):
    """Bytes of the stored band-LU factors one solve launch streams
    (unpivoted layout: L, U scaled, 1/U_jj padded to whole batches of
    `pad` steps; W, C, Minv)."""
    if kernel != "solve":
        return 0
    n4, n2 = K - 4, K - 2
    q4, q2 = (n4 + pad - 1) // pad * pad, (n2 + pad - 1) // pad * pad
    psi = (M - 1) * (q4 * (8 + 8 + 1) * 16 + 4 * n4 * 16 + (32 + 16) * 16)
    real = (M + 1) * (q2 * (4 + 4 + 1) * 8 + 2 * n2 * 8 + (8 + 4) * 8)
    return psi + real


def kernel_source_hash():
    """Hash of every device source: counter-measured traffic is reported
    only for the kernels it was measured on."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1902_07092_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel, workload):
    """Counter-measured HBM bytes per launch from profiles/, if they were
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
        rec = data[workload][kernel]
        if rec.get("source_hash") != kernel_source_hash():
            return None
        return rec["bytes_per_launch"]
    except (KeyError, ValueError, TypeError):
        return None


def cpu_baseline(w, state, steps):
    """The oracle, as it stands, on the host cores: init (operators and
    factorisation) untimed, then `steps` full steps timed."""
    from oracle.step import QGOracle
    o = QGOracle(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c)
    o.set_state(state.psi, state.theta, state.uphi0)
    o.factor(0.5 * w.dt)
    t0 = time.perf_counter()
    o.step(w.dt, w.scheme, steps)
    dt = time.perf_counter() - t0
    return {"value": w.grid_points * steps / dt, "unit": "grid-point-steps/s",
            "cores": os.cpu_count(), "kind": "oracle",
            "sample": f"{steps} full {w.scheme.upper()} step(s) of "
                      f"{w.name}, oracle init untimed, {dt:.1f} s"}


def copy_calibration(torch, mb, steps):
    """A plain copy of known size: FETCH_SIZE and WRITE_SIZE of its
    dispatches, against the bytes it must move, give the factor that turns
    the counters of the step's kernels into HBM bytes."""
    n = mb * (1 << 20)
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        dst.copy_(src)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n,
                      "ms_per_copy": ms, "GBps": 2 * n / ms / 1e6}),
          flush=True)


def timed_steps(torch, solver, w, steps):
    stream = solver.stream
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    solver.step(w.dt, w.scheme, steps)
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop)


def mixed_run(qg, torch, w, state, args, fp64_solver):
    """The same sequence of steps with FP32 transforms and products (FP64
    solves, state and history); its state is compared with the FP64 run's
    after the same steps."""
    import numpy as np
    s = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c,
                    device="cuda:0", precision=1)
    s.set_state(state.psi, state.theta, state.uphi0)
    s.step(w.dt, w.scheme, 0)
    tuned = (s.step_autotune(w.dt, w.scheme, args.tune_steps)
             if args.tune_steps else None)
    s.step(w.dt, w.scheme, args.warmup)
    ms = timed_steps(torch, s, w, args.steps) / args.steps
    kern = s.step_timed(w.dt, w.scheme, args.steps)
    a, b = s.get_state(), fp64_solver.get_state()
    rel = {f: float(np.abs(x - y).max() / max(np.abs(y).max(), 1e-300))
           for f, x, y in zip(("psi", "theta", "uphi"), a, b)}
    return {"value": w.grid_points / (ms * 1e-3), "unit": "grid-point-steps/s",
            "ms_per_step": ms, "precision": "FP32 transforms and products, "
            "FP64 solves/state/diagnostics",
            "rel_diff_vs_fp64_run": rel,
            "rel_diff_after_steps": args.tune_steps + args.warmup + 2 * args.steps,
            "band_systems_per_thread": tuned,
            "kernels": {k: {"avg_launch_us": v[0] / max(1, v[1]) * 1e3,
                            "launches": v[1]} for k, v in kern.items()}}


# Cost of one step relative to CNAB2, Table 1 of the paper (its own
# CPU runs, integration + Galerkin at 1025 x 682 x 1280): context only.
TABLE1_COST = {"sbdf4": 1.01, "sbdf3": 0.97, "sbdf2": 0.96, "cnab2": 1.0,
               "bpr353": 3.24, "ars443": 3.66, "ars222": 1.81}


def schemes_run(qg, torch, w, state, args):
    """Every time scheme of Table 1 (except LZ232) on the same workload:
    a fresh start per scheme, warm-up steps past the SBDF start-up and the
    refactorisation, then args.scheme_steps timed steps."""
    s = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c,
                    device="cuda:0")
    out = {}
    for name in ("cnab2", "sbdf2", "sbdf3", "sbdf4", "bpr353", "ars222",
                 "ars443"):
        s.set_state(state.psi, state.theta, state.uphi0)
        s.step(w.dt, name, 4)
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record(s.stream)
        s.step(w.dt, name, args.scheme_steps)
        stop.record(s.stream)
        torch.cuda.synchronize()
        out[name] = {"ms_per_step": start.elapsed_time(stop) / args.scheme_steps}
    for name, v in out.items():
        v["cost_vs_cnab2"] = v["ms_per_step"] / out["cnab2"]["ms_per_step"]
        v["table1_cost_vs_cnab2"] = TABLE1_COST[name]
    return out


def variants_run(qg, torch, w, state, args):
    """The method variants on the headline workload: the Galerkin bases
    (Sect. 3.2.2) and implicit buoyancy (Sect. 4), each from a fresh start,
    warm-up steps past the factorisation, then args.steps timed steps
    (median of 3 repeats) with the solve's launch time."""
    out = {}
    for name, kw in (("galerkin", dict(method="galerkin")),
                     ("implicit_buoyancy", dict(buoyancy="implicit"))):
        s = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c,
                        device="cuda:0", **kw)
        s.set_state(state.psi, state.theta, state.uphi0)
        s.step(w.dt, w.scheme, args.warmup)
        reps = [timed_steps(torch, s, w, args.steps) / args.steps for _ in range(3)]
        ms = _median(reps)
        kern = s.step_timed(w.dt, w.scheme, args.steps)
        out[name] = {"ms_per_step": ms, "repeats_ms_per_step": reps,
                     "value": w.grid_points / (ms * 1e-3),
                     "unit": "grid-point-steps/s",
                     "solve_avg_launch_us": kern["solve"][0] / kern["solve"][1] * 1e3,
                     "solve_launches_per_step": kern["solve"][1] / args.steps}
    return out


def tangent_run(qg, torch, inputs, args):
    """The 768 x 257 adjoint-study workload (E = 1e-6, Ra = 5 Ra_c, CNAB2):
    forward steps against tangent-linear steps (state and perturbation
    advanced together), both timed on the solver's stream."""
    import numpy as np
    w = inputs.ADJOINT
    st = inputs.workload_state(w)
    rng = np.random.default_rng(500)
    cth = (rng.standard_normal((w.M, w.n_c))
           + 1j * rng.standard_normal((w.M, w.n_c)))
    cth[0] = cth[0].real
    d = (np.zeros_like(st.psi), inputs.dirichlet_from_basis(cth, w.n_c),
         np.zeros(w.n_c))
    s = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c,
                    device="cuda:0")
    out = {}
    for mode in ("forward", "tangent"):
        s.set_state(st.psi, st.theta, st.uphi0)
        if mode == "tangent":
            s.tangent_set(*d)
        run = (lambda n: s.step(w.dt, "cnab2", n)) if mode == "forward" \
            else (lambda n: s.step_tangent(w.dt, n))
        run(args.warmup)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s.stream)
        run(args.ens_steps)
        b.record(s.stream)
        torch.cuda.synchronize()
        out[mode] = a.elapsed_time(b) / args.ens_steps
    return {"workload": w.name, "ms_per_forward_step": out["forward"],
            "ms_per_tangent_step": out["tangent"],
            "tangent_vs_forward": out["tangent"] / out["forward"],
            "perturbation": "random initial-temperature coefficients, seed 500"}


def _median(v):
    v = sorted(v)
    n = len(v)
    return v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])


def _timed(torch, stream, fn):
    """Milliseconds of fn() between events on `stream` (fn may synchronise
    itself; the host time it spends between launches counts)."""
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b)


def adjoint_run(qg, torch, inputs, args, repeats=5):
    """The adjoint workload (768 x 257, E = 1e-6, Ra = 5 Ra_c, CNAB2, 200
    steps): the forward run against the gradient of the time-integrated
    kinetic energy with respect to the initial state (qg_gradient:
    forward pass with a checkpoint every 20 steps, then recomputation and
    the reverse sweep), median of `repeats` runs each."""
    w = inputs.ADJOINT
    st = inputs.workload_state(w)
    s = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c,
                    device="cuda:0")
    s.set_state(st.psi, st.theta, st.uphi0)
    s.gradient(w.dt, 20, 20)                  # factorisation, first launches
    fwd, grad = [], []
    for _ in range(repeats):
        s.set_state(st.psi, st.theta, st.uphi0)
        fwd.append(_timed(torch, s.stream, lambda: s.step(w.dt, "cnab2", w.steps)))
        s.set_state(st.psi, st.theta, st.uphi0)
        grad.append(_timed(torch, s.stream, lambda: s.gradient(w.dt, w.steps, 20)))
    return {"workload": w.name, "steps": w.steps, "checkpoint_interval": 20,
            "ms_forward": _median(fwd), "ms_gradient": _median(grad),
            "adjoint_vs_forward": _median(grad) / _median(fwd),
            "repeats": repeats, "ms_forward_all": fwd, "ms_gradient_all": grad,
            "gradient": "J = dt sum w_n E_K(y^n) and dJ/dy^0, forward pass "
                        "included"}


def config_lines(qg, torch, inputs, args, repeats=5):
    """GPU throughput of the 96 x 33 CNAB2 workload (100 steps) and of the
    768 x 257 BPR353 workload (500 steps), median of `repeats` runs."""
    out = {}
    for w in (inputs.SMALL, inputs.MEDIUM):
        st = inputs.workload_state(w)
        s = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c,
                        device="cuda:0")
        s.set_state(st.psi, st.theta, st.uphi0)
        s.step(w.dt, w.scheme, 2)            # factorisation, first launches
        ms = []
        for _ in range(repeats):
            s.set_state(st.psi, st.theta, st.uphi0)
            ms.append(_timed(torch, s.stream, lambda: s.step(w.dt, w.scheme, w.steps)))
        med = _median(ms)
        out[w.name] = {"steps": w.steps, "scheme": w.scheme, "ms_total": med,
                       "ms_per_step": med / w.steps,
                       "grid_point_steps_per_s": w.grid_points * w.steps / (med * 1e-3),
                       "repeats_ms": ms}
    return out


def cpu_model():
    try:
        import subprocess
        txt = subprocess.run(["lscpu"], capture_output=True, text=True,
                             timeout=10).stdout
        for line in txt.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_legs(inputs):
    """The oracle on the host cores for the other configurations: 96 x 33
    CNAB2 (100 steps), 768 x 257 BPR353 with the integration method and
    the collocation cross-check (one step each), 768 x 257 CNAB2 forward of
    the adjoint workload (two steps).  Init untimed."""
    from oracle import transforms as tr
    from oracle.collocation import CollocationCNAB2
    from oracle.step import QGOracle
    legs = {}

    def leg(name, w, scheme, steps, colloc=False):
        st = inputs.workload_state(w)
        if colloc:
            o = CollocationCNAB2(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r)
            grid = [tr.cheb_to_grid(a, w.n_r) for a in (st.psi, st.theta, st.uphi0)]
            load = lambda: o.set_state(*grid)
            run = lambda n: [o.step(w.dt) for _ in range(n)]
        else:
            o = QGOracle(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c)
            load = lambda: o.set_state(st.psi, st.theta, st.uphi0)
            run = lambda n: o.step(w.dt, scheme, n)
        load()
        run(1)                               # factorisation untimed
        load()
        t0 = time.perf_counter()
        run(steps)
        dt = time.perf_counter() - t0
        legs[name] = {"value": w.grid_points * steps / dt,
                      "unit": "grid-point-steps/s", "steps": steps,
                      "scheme": scheme, "seconds": dt}

    leg(inputs.SMALL.name, inputs.SMALL, "cnab2", 100)
    leg(inputs.MEDIUM.name, inputs.MEDIUM, "bpr353", 1)
    leg(inputs.MEDIUM.name + "_collocation", inputs.MEDIUM, "cnab2", 1,
        colloc=True)
    leg(inputs.ADJOINT.name, inputs.ADJOINT, "cnab2", 2)
    return legs


def ensemble_run(qg, torch, inputs, args):
    """The batched ensemble: 64 runs of uneven size and Ra stepped together
    (one launch per kernel and size group, graph replay), against the same
    runs stepped one context after another."""
    ws = inputs.ensemble_workloads()
    members = [dict(E=w.E, Ra=w.Ra, Pr=w.Pr, eta=w.eta, n_phi=w.n_phi,
                    n_r=w.n_r, n_c=w.n_c) for w in ws]
    states = [inputs.workload_state(w) for w in ws]
    ens = qg.QGEnsemble(members)
    for i, st in enumerate(states):
        ens.set_state(i, st.psi, st.theta, st.uphi0)
    dt = ws[0].dt
    ens.step(dt, "cnab2", args.warmup)
    tuned = None
    if args.ens_tune_steps:
        picks = ens.step_autotune(dt, "cnab2", args.ens_tune_steps)
        _, grp = ens.groups()
        tuned = {f"{ws[i].n_phi}x{ws[i].n_r}": picks[grp[i]]
                 for i in range(len(ws))}
    def timed(e):
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record(e.stream)
        e.step(dt, "cnab2", args.ens_steps)
        stop.record(e.stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / args.ens_steps
    reps = [timed(ens) for _ in range(5)]
    ms = _median(reps)
    gp = sum(w.grid_points for w in ws)
    # the same ensemble with the radial transforms on the matrix cores
    mf = qg.QGEnsemble([dict(m, dct="mfma") for m in members])
    for i, st in enumerate(states):
        mf.set_state(i, st.psi, st.theta, st.uphi0)
    mf.step(dt, "cnab2", args.warmup)
    if args.ens_tune_steps:
        mf.step_autotune(dt, "cnab2", args.ens_tune_steps)
    mf_reps = [timed(mf) for _ in range(3)]
    del mf
    bad = [i for i in range(len(ws)) if ens.diagnostics(i)["nonfinite"]]
    # the same runs, one single-run context after another
    solos = []
    for w, st in zip(ws, states):
        s = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c,
                        device="cuda:0")
        s.set_state(st.psi, st.theta, st.uphi0)
        s.step(dt, "cnab2", args.warmup)
        solos.append(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in solos:
        s.step(dt, "cnab2", args.ens_steps)
    torch.cuda.synchronize()
    solo_ms = (time.perf_counter() - t0) * 1e3 / args.ens_steps
    sizes = {}
    for w in ws:
        sizes[f"{w.n_phi}x{w.n_r}"] = sizes.get(f"{w.n_phi}x{w.n_r}", 0) + 1
    return {"value": gp / (ms * 1e-3), "unit": "grid-point-steps/s",
            "ms_per_step": ms, "repeats_ms_per_step": reps,
            "mfma_dct_ms_per_step": _median(mf_reps),
            "mfma_dct_repeats_ms_per_step": mf_reps,
            "members": len(ws), "sizes": sizes,
            "grid_points_per_step": gp, "steps": args.ens_steps,
            "band_systems_per_thread": tuned,
            "nonfinite_members": bad,
            "one_context_after_another": {
                "value": gp / (solo_ms * 1e-3), "ms_per_step": solo_ms,
                "timing": "host clock around all contexts' steps"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large_3072x1025_E1e-8_cnab2")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision run")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the batched-ensemble run")
    ap.add_argument("--ens-steps", type=int, default=20)
    ap.add_argument("--no-schemes", action="store_true",
                    help="skip the per-scheme step costs")
    ap.add_argument("--scheme-steps", type=int, default=10)
    ap.add_argument("--tune-steps", type=int, default=21,
                    help="untimed steps of the band-product autotuner "
                    "before the warm-up (0: compiled default shape)")
    ap.add_argument("--ens-tune-steps", type=int, default=21)
    ap.add_argument("--adjoint-only", action="store_true",
                    help="print only the adjoint workload's forward and "
                         "gradient times")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="only the batched-ensemble run (for profiling it)")
    ap.add_argument("--method", choices=("tau", "galerkin"), default="tau",
                    help="boundary conditions of the headline run: tau rows "
                         "(default) or the Galerkin bases")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64",
                    help="precision of the headline run (mixed also runs the "
                         "12288 x 4097 workload, which FP64 does not fit)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run a plain device-to-device copy of MB MiB "
                         "(steps times), the reference for HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the step's per-m and per-ring "
              "kernels run on a single device; --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        copy_calibration(torch, args.copy_calibration, args.steps)
        return

    from paper_1902_07092_amd import inputs, qg
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_run(qg, torch, inputs, args)}),
              flush=True)
        return
    if args.ensemble_only:
        print(json.dumps({"batched": ensemble_run(qg, torch, inputs, args)}),
              flush=True)
        return
    w = inputs.WORKLOADS[args.workload]
    state = inputs.workload_state(w)
    prec = 1 if args.precision == "mixed" else 0
    solver = qg.QGSolver(w.E, w.Ra, w.Pr, w.eta, w.n_phi, w.n_r, w.n_c,
                         device="cuda:0", precision=prec, method=args.method)
    solver.set_state(state.psi, state.theta, state.uphi0)
    solver.step(w.dt, w.scheme, 0)            # factorise (untimed)
    # band-product launch shape picked by the library's autotuner (untimed
    # steps; the results do not depend on the shape)
    tuned = (solver.step_autotune(w.dt, w.scheme, args.tune_steps)
             if args.tune_steps else None)
    solver.step(w.dt, w.scheme, args.warmup)
    stream = solver.stream
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    solver.step(w.dt, w.scheme, args.steps)
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    ms_per_step = total_ms / args.steps
    value = w.grid_points * args.steps / (total_ms * 1e-3)

    # per-kernel durations over the same number of steps, HIP events on
    # the solver's stream around every launch
    kern = solver.step_timed(w.dt, w.scheme, args.steps)
    M, R, K = w.M, w.n_r, w.n_c
    dominant = max(kern, key=lambda k: kern[k][0])
    ms_tot, launches = kern[dominant]
    avg_s = ms_tot / launches * 1e-3
    ab = alg_bytes(dominant, M, R, K, mixed=prec == 1)
    achieved = ab / avg_s / 1e9
    # counters were taken on the FP64 kernels only
    traffic = traffic_for(dominant, w.name) if prec == 0 else None
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": traffic, "kernel": dominant,
                "alg_bytes_per_launch": ab,
                "avg_launch_us": avg_s * 1e6}
    kernels = {k: {"avg_launch_us": v[0] / max(1, v[1]) * 1e3,
                   "launches": v[1],
                   "alg_GBps": alg_bytes(k, M, R, K, mixed=prec == 1)
                   / (v[0] / max(1, v[1])
                                                        * 1e-3) / 1e9,
                   "factor_bytes_per_launch": factor_bytes(k, M, K)}
               for k, v in kern.items()}
    out = {"metric": METRIC, "value": value, "unit": "grid-point-steps/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_per_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": w.name, "n_phi": w.n_phi, "n_r": w.n_r,
                      "n_c": w.n_c, "E": w.E, "Ra": w.Ra, "Pr": w.Pr,
                      "eta": w.eta, "scheme": w.scheme, "dt": w.dt,
                      "method": args.method,
                      "band_systems_per_thread": tuned,
                      "parallelism": "single GPU"},
           "roofline": roofline, "kernels": kernels}
    print(f"[bench] gpu done: {ms_per_step:.4f} ms/step", file=sys.stderr,
          flush=True)
    if prec == 1:
        out["dtype"] = "f32+f64"
    if not args.no_mixed and prec == 0:
        out["mixed"] = mixed_run(qg, torch, w, state, args, solver)
        print(f"[bench] mixed done: {out['mixed']['ms_per_step']:.4f} ms/step",
              file=sys.stderr, flush=True)
    if not args.no_schemes and prec == 0:
        out["schemes"] = schemes_run(qg, torch, w, state, args)
        print("[bench] schemes done", file=sys.stderr, flush=True)
    if not args.no_schemes and prec == 0:
        out["variants"] = variants_run(qg, torch, w, state, args)
        print("[bench] variants done", file=sys.stderr, flush=True)
    if not args.no_schemes and prec == 0:
        out["tangent_linear"] = tangent_run(qg, torch, inputs, args)
        print("[bench] tangent done", file=sys.stderr, flush=True)
    if not args.no_schemes and prec == 0:
        out["adjoint"] = adjoint_run(qg, torch, inputs, args)
        print(f"[bench] adjoint done: {out['adjoint']['adjoint_vs_forward']:.2f} "
              "x forward", file=sys.stderr, flush=True)
        out["configs"] = config_lines(qg, torch, inputs, args)
        print("[bench] config lines done", file=sys.stderr, flush=True)
    if not args.no_ensemble and prec == 0:
        out["batched"] = ensemble_run(qg, torch, inputs, args)
        print(f"[bench] ensemble done: {out['batched']['ms_per_step']:.4f} "
              "ms/step", file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, state, args.cpu_steps)
        out["cpu_baseline"]["model"] = cpu_model()
        if not args.no_schemes:
            out["cpu_baseline"]["other_configs"] = cpu_legs(inputs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
