"""Thin Python binding of libqg.so (argument marshalling only).

Every step of the solver runs in the HIP library; PyTorch provides the
device workspace and the stream.  Functions carry the C ABI names of
include/qg.h; QGSolver wraps one context.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqg.so")

QG_OK, QG_EINVAL, QG_ENOMEM, QG_EDEVICE = 0, -1, -2, -3
QG_ENONFINITE, QG_ESTATE, QG_EUNSUPPORTED = -4, -5, -6
SCHEMES = {"cnab2": 0, "bpr353": 1, "ars222": 2, "ars443": 3,
           "sbdf2": 4, "sbdf3": 5, "sbdf4": 6}
STATUS_NAMES = {0: "QG_OK", -1: "QG_EINVAL", -2: "QG_ENOMEM",
                -3: "QG_EDEVICE", -4: "QG_ENONFINITE", -5: "QG_ESTATE",
                -6: "QG_EUNSUPPORTED"}


class qg_params(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double), ("Ra", ctypes.c_double),
                ("Pr", ctypes.c_double), ("eta", ctypes.c_double),
                ("n_phi", ctypes.c_int), ("n_r", ctypes.c_int),
                ("n_c", ctypes.c_int), ("precision", ctypes.c_int),
                ("pivoting", ctypes.c_int), ("ekman", ctypes.c_int),
                ("eps", ctypes.c_double), ("method", ctypes.c_int),
                ("buoyancy", ctypes.c_int), ("dct", ctypes.c_int)]

# qg_params.method: boundary conditions by tau rows or Galerkin bases
QG_TAU, QG_GALERKIN = 0, 1
METHODS = {"tau": QG_TAU, "galerkin": QG_GALERKIN}
# qg_params.buoyancy
BUOYANCY = {"explicit": 0, "implicit": 1}
# qg_params.dct: radial transforms
DCT = {"default": 0, "fft": 1, "mfma": 2}


class qg_diag(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("E_kin", ctypes.c_double),
                ("E_zon", ctypes.c_double), ("E_therm", ctypes.c_double),
                ("enstrophy", ctypes.c_double), ("Re", ctypes.c_double),
                ("Ro", ctypes.c_double), ("dt_cfl", ctypes.c_double),
                ("step", ctypes.c_longlong), ("nonfinite", ctypes.c_int),
                ("pivoted", ctypes.c_int), ("growth", ctypes.c_double)]


class QGError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")


_lib = None


def load():
    """Load libqg.so; fails loudly when the HIP library is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"HIP library {LIB_PATH} is missing; run __graft_entry__.build() "
            "(or python -m paper_1902_07092_amd.build)")
    # torch first: the library must bind to the HIP runtime that owns the
    # workspace and the streams torch hands over, not load a second copy
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "qg_workspace_size": (i, [ctypes.POINTER(qg_params),
                                  ctypes.POINTER(ctypes.c_size_t)]),
        "qg_create": (i, [ctypes.POINTER(vp), ctypes.POINTER(qg_params), vp,
                          ctypes.c_size_t, vp]),
        "qg_create_static": (i, [ctypes.POINTER(vp), ctypes.POINTER(qg_params),
                                 vp]),
        "qg_set_state": (i, [vp, vp, vp, vp, i]),
        "qg_get_state": (i, [vp, vp, vp, vp, i]),
        "qg_step": (i, [vp, d, i, i]),
        "qg_diagnostics": (i, [vp, ctypes.POINTER(qg_diag)]),
        "qg_last_error": (ctypes.c_char_p, [vp]),
        "qg_destroy": (None, [vp]),
        "qg_operator_band": (i, [d, i, i, vp]),
        "qg_step_timed": (i, [vp, d, i, i, vp, vp]),
        "qg_step_autotune": (i, [vp, d, i, i, ctypes.POINTER(i)]),
        "qg_tangent_set": (i, [vp, vp, vp, vp, i]),
        "qg_tangent_get": (i, [vp, vp, vp, vp, i]),
        "qg_step_tangent": (i, [vp, d, i]),
        "qg_adjoint_solve": (i, [vp, d, vp, vp, vp, i]),
        "qg_adjoint_mass_lin": (i, [vp, d, vp, vp, vp, i]),
        "qg_gradient_workspace_size": (i, [vp, i, i,
                                           ctypes.POINTER(ctypes.c_size_t)]),
        "qg_gradient": (i, [vp, d, i, i, d, vp, vp, vp, vp, vp, vp,
                            ctypes.POINTER(d), vp, ctypes.c_size_t]),
        "qg_adjoint_explicit": (i, [vp, vp, vp, vp, vp, vp, vp, d, vp,
                                    ctypes.c_size_t]),
        "qg_checkpoint_size": (i, [vp, ctypes.POINTER(ctypes.c_size_t)]),
        "qg_checkpoint_save": (i, [vp, vp, ctypes.c_size_t, i]),
        "qg_checkpoint_load": (i, [vp, vp, ctypes.c_size_t, i]),
        "qg_ensemble_workspace_size": (i, [vp, i,
                                           ctypes.POINTER(ctypes.c_size_t)]),
        "qg_ensemble_create": (i, [ctypes.POINTER(vp), vp, i, vp,
                                   ctypes.c_size_t, vp]),
        "qg_ensemble_set_state": (i, [vp, i, vp, vp, vp, i]),
        "qg_ensemble_get_state": (i, [vp, i, vp, vp, vp, i]),
        "qg_ensemble_step": (i, [vp, d, i, i]),
        "qg_ensemble_step_autotune": (i, [vp, d, i, i, ctypes.POINTER(i)]),
        "qg_ensemble_groups": (i, [vp, ctypes.POINTER(i), ctypes.POINTER(i)]),
        "qg_ensemble_diagnostics": (i, [vp, i, ctypes.POINTER(qg_diag)]),
        "qg_ensemble_last_error": (ctypes.c_char_p, [vp]),
        "qg_ensemble_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


# ---------------------------------------------------------------- C ABI names
def qg_workspace_size(params: qg_params) -> int:
    n = ctypes.c_size_t(0)
    st = load().qg_workspace_size(ctypes.byref(params), ctypes.byref(n))
    if st != QG_OK:
        raise QGError(st, "invalid parameters")
    return n.value


def qg_operator_band(eta: float, n_c: int, which: int) -> np.ndarray:
    out = np.zeros((n_c, 17), np.float64)
    st = load().qg_operator_band(eta, n_c, which,
                                 out.ctypes.data_as(ctypes.c_void_p))
    if st != QG_OK:
        raise QGError(st, "qg_operator_band")
    return out


def _check(ctx, st):
    if st != QG_OK:
        msg = load().qg_last_error(ctx)
        raise QGError(st, msg.decode() if msg else "")


def qg_create(params, workspace_ptr, nbytes, stream_ptr):
    ctx = ctypes.c_void_p()
    st = load().qg_create(ctypes.byref(ctx), ctypes.byref(params),
                          ctypes.c_void_p(workspace_ptr), nbytes,
                          ctypes.c_void_p(stream_ptr))
    if st != QG_OK:
        raise QGError(st, "qg_create")
    return ctx


def qg_create_static(params, stream_ptr):
    """qg_create with the library's static device workspace (no device
    allocation by anyone); one such context per device at a time."""
    ctx = ctypes.c_void_p()
    st = load().qg_create_static(ctypes.byref(ctx), ctypes.byref(params),
                                 ctypes.c_void_p(stream_ptr))
    if st != QG_OK:
        raise QGError(st, qg_last_error(None))
    return ctx


def qg_set_state(ctx, psi_ptr, theta_ptr, uphi_ptr, on_device):
    _check(ctx, load().qg_set_state(ctx, psi_ptr, theta_ptr, uphi_ptr,
                                    int(on_device)))


def qg_get_state(ctx, psi_ptr, theta_ptr, uphi_ptr, on_device):
    _check(ctx, load().qg_get_state(ctx, psi_ptr, theta_ptr, uphi_ptr,
                                    int(on_device)))


def qg_step(ctx, dt, scheme, nsteps):
    _check(ctx, load().qg_step(ctx, float(dt), int(scheme), int(nsteps)))


KERNEL_CLASSES = ("synth", "ring", "analysis", "solve", "rhs")


def qg_step_timed(ctx, dt, scheme, nsteps):
    ms = (ctypes.c_double * 5)()
    n = (ctypes.c_int * 5)()
    _check(ctx, load().qg_step_timed(ctx, float(dt), int(scheme), int(nsteps),
                                     ctypes.cast(ms, ctypes.c_void_p),
                                     ctypes.cast(n, ctypes.c_void_p)))
    return {k: (ms[i], n[i]) for i, k in enumerate(KERNEL_CLASSES) if n[i]}


def qg_step_autotune(ctx, dt, scheme, nsteps) -> int:
    """Returns the chosen systems per thread of the band products."""
    out = ctypes.c_int(0)
    _check(ctx, load().qg_step_autotune(ctx, float(dt), int(scheme),
                                        int(nsteps), ctypes.byref(out)))
    return out.value


def qg_diagnostics(ctx) -> dict:
    d = qg_diag()
    _check(ctx, load().qg_diagnostics(ctx, ctypes.byref(d)))
    return {name: getattr(d, name) for name, _ in qg_diag._fields_}


def qg_last_error(ctx) -> str:
    msg = load().qg_last_error(ctx)
    return msg.decode() if msg else ""


def qg_destroy(ctx):
    load().qg_destroy(ctx)


def _params_array(members):
    arr = (qg_params * len(members))(*members)
    return arr


def qg_ensemble_workspace_size(members) -> int:
    arr = _params_array(members)
    n = ctypes.c_size_t(0)
    st = load().qg_ensemble_workspace_size(ctypes.cast(arr, ctypes.c_void_p),
                                           len(members), ctypes.byref(n))
    if st != QG_OK:
        raise QGError(st, "invalid member parameters")
    return n.value


def _echeck(ens, st):
    if st != QG_OK:
        msg = load().qg_ensemble_last_error(ens)
        raise QGError(st, msg.decode() if msg else "")


def qg_ensemble_create(members, workspace_ptr, nbytes, stream_ptr):
    arr = _params_array(members)
    ens = ctypes.c_void_p()
    st = load().qg_ensemble_create(ctypes.byref(ens),
                                   ctypes.cast(arr, ctypes.c_void_p),
                                   len(members), ctypes.c_void_p(workspace_ptr),
                                   nbytes, ctypes.c_void_p(stream_ptr))
    if st != QG_OK:
        raise QGError(st, "qg_ensemble_create")
    return ens


def qg_ensemble_set_state(ens, member, psi_ptr, theta_ptr, uphi_ptr,
                          on_device):
    _echeck(ens, load().qg_ensemble_set_state(ens, int(member), psi_ptr,
                                              theta_ptr, uphi_ptr,
                                              int(on_device)))


def qg_ensemble_get_state(ens, member, psi_ptr, theta_ptr, uphi_ptr,
                          on_device):
    _echeck(ens, load().qg_ensemble_get_state(ens, int(member), psi_ptr,
                                              theta_ptr, uphi_ptr,
                                              int(on_device)))


def qg_ensemble_step(ens, dt, scheme, nsteps):
    _echeck(ens, load().qg_ensemble_step(ens, float(dt), int(scheme),
                                         int(nsteps)))


def qg_ensemble_groups(ens, n_members):
    """(number of size groups, group of each member)."""
    ng = ctypes.c_int(0)
    gm = (ctypes.c_int * max(1, n_members))()
    _echeck(ens, load().qg_ensemble_groups(ens, ctypes.byref(ng), gm))
    return ng.value, list(gm)[:n_members]


def qg_ensemble_step_autotune(ens, dt, scheme, nsteps, ngroups) -> list:
    """Returns the chosen systems per thread of each size group."""
    out = (ctypes.c_int * max(1, ngroups))()
    _echeck(ens, load().qg_ensemble_step_autotune(ens, float(dt), int(scheme),
                                                  int(nsteps), out))
    return list(out)[:ngroups]


def qg_ensemble_diagnostics(ens, member) -> dict:
    d = qg_diag()
    _echeck(ens, load().qg_ensemble_diagnostics(ens, int(member),
                                                ctypes.byref(d)))
    return {name: getattr(d, name) for name, _ in qg_diag._fields_}


def qg_ensemble_destroy(ens):
    load().qg_ensemble_destroy(ens)


# ---------------------------------------------------------------- wrapper
class QGSolver:
    """One solver context on a HIP device, workspace allocated by torch."""

    def __init__(self, E, Ra, Pr, eta, n_phi, n_r, n_c=0, device="cuda:0",
                 stream=None, pivoting=0, precision=0, ekman_eps=None,
                 static_workspace=False, method="tau", buoyancy="explicit",
                 dct="default"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.params = qg_params(E, Ra, Pr, eta, n_phi, n_r, n_c, precision,
                                pivoting, 0 if ekman_eps is None else 1,
                                0.0 if ekman_eps is None else ekman_eps,
                                METHODS[method], BUOYANCY[buoyancy], DCT[dct])
        self.M = n_phi // 3 + 1
        self.K = n_c if n_c else (2 * (n_r - 1)) // 3
        nbytes = qg_workspace_size(self.params)
        with torch.cuda.device(self.device):
            self.stream = stream or torch.cuda.current_stream(self.device)
            if static_workspace:
                self.workspace = None
                self.ctx = qg_create_static(self.params,
                                            self.stream.cuda_stream)
            else:
                self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8,
                                             device=self.device)
                base = self.workspace.data_ptr()
                aligned = (base + 255) // 256 * 256
                self.ctx = qg_create(self.params, aligned, nbytes,
                                     self.stream.cuda_stream)
        self.nbytes = nbytes

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            self.ctx = None
            try:
                qg_destroy(ctx)
            except TypeError:   # interpreter shutdown: module already torn down
                pass

    def _arrays(self, psi, theta, uphi):
        torch = self.torch
        if isinstance(psi, torch.Tensor):
            ps = psi.to(self.device, torch.complex128).contiguous()
            th = theta.to(self.device, torch.complex128).contiguous()
            up = uphi.to(self.device, torch.float64).contiguous()
            return (ps, th, up), (ps.data_ptr(), th.data_ptr(),
                                  up.data_ptr()), 1
        ps = np.ascontiguousarray(psi, np.complex128)
        th = np.ascontiguousarray(theta, np.complex128)
        up = np.ascontiguousarray(uphi, np.float64)
        return (ps, th, up), (ps.ctypes.data, th.ctypes.data,
                              up.ctypes.data), 0

    def set_state(self, psi, theta, uphi):
        keep, ptrs, dev = self._arrays(psi, theta, uphi)
        if keep[0].shape != (self.M, self.K) or keep[1].shape != (
                self.M, self.K) or keep[2].shape != (self.K,):
            raise ValueError("state arrays must be (M, K), (M, K), (K,)")
        qg_set_state(self.ctx, *[ctypes.c_void_p(p) for p in ptrs], dev)

    def get_state(self, on_device=False):
        torch = self.torch
        if on_device:
            ps = torch.empty((self.M, self.K), dtype=torch.complex128,
                             device=self.device)
            th = torch.empty_like(ps)
            up = torch.empty(self.K, dtype=torch.float64, device=self.device)
            ptrs = (ps.data_ptr(), th.data_ptr(), up.data_ptr())
        else:
            ps = np.empty((self.M, self.K), np.complex128)
            th = np.empty_like(ps)
            up = np.empty(self.K)
            ptrs = (ps.ctypes.data, th.ctypes.data, up.ctypes.data)
        qg_get_state(self.ctx, *[ctypes.c_void_p(p) for p in ptrs],
                     int(on_device))
        return ps, th, up

    def step(self, dt, scheme="cnab2", n=1):
        qg_step(self.ctx, dt, SCHEMES[scheme], n)

    def checkpoint(self):
        """qg_checkpoint_save into a host buffer: the state and the
        multistep history of the current scheme (numpy uint8 array)."""
        n = ctypes.c_size_t(0)
        _check(self.ctx, load().qg_checkpoint_size(self.ctx, ctypes.byref(n)))
        buf = np.zeros(n.value, np.uint8)
        _check(self.ctx, load().qg_checkpoint_save(
            self.ctx, ctypes.c_void_p(buf.ctypes.data), n.value, 0))
        return buf

    def restore(self, buf):
        """qg_checkpoint_load from a host buffer written by checkpoint()
        (or a device tensor holding one)."""
        torch = self.torch
        if isinstance(buf, torch.Tensor):
            _check(self.ctx, load().qg_checkpoint_load(
                self.ctx, ctypes.c_void_p(buf.data_ptr()), buf.numel(), 1))
            return
        b = np.ascontiguousarray(buf, np.uint8)
        _check(self.ctx, load().qg_checkpoint_load(
            self.ctx, ctypes.c_void_p(b.ctypes.data), b.size, 0))

    def checkpoint_device(self):
        """qg_checkpoint_save into a device tensor (uint8)."""
        torch = self.torch
        n = ctypes.c_size_t(0)
        _check(self.ctx, load().qg_checkpoint_size(self.ctx, ctypes.byref(n)))
        buf = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        _check(self.ctx, load().qg_checkpoint_save(
            self.ctx, ctypes.c_void_p(buf.data_ptr()), n.value, 1))
        return buf

    def step_timed(self, dt, scheme="cnab2", n=1):
        """Returns {kernel class: (total ms, launches)}."""
        return qg_step_timed(self.ctx, dt, SCHEMES[scheme], n)

    def tangent_set(self, dpsi, dtheta, duphi):
        """Perturbation of the current state for qg_step_tangent (host
        arrays, the layout of set_state)."""
        import numpy as np
        a = [np.ascontiguousarray(x, dtype=t) for x, t in
             ((dpsi, np.complex128), (dtheta, np.complex128), (duphi, np.float64))]
        _check(self.ctx, load().qg_tangent_set(
            self.ctx, *[ctypes.c_void_p(x.ctypes.data) for x in a], 0))

    def step_tangent(self, dt, n=1):
        _check(self.ctx, load().qg_step_tangent(self.ctx, float(dt), int(n)))

    def adjoint_solve(self, dt, psi, theta, uphi):
        """qg_adjoint_solve on host arrays (copies; returns the result)."""
        import numpy as np
        ps = np.array(psi, dtype=np.complex128, order="C")
        th = np.array(theta, dtype=np.complex128, order="C")
        up = np.array(uphi, dtype=np.float64, order="C")
        _check(self.ctx, load().qg_adjoint_solve(
            self.ctx, float(dt), ctypes.c_void_p(ps.ctypes.data),
            ctypes.c_void_p(th.ctypes.data), ctypes.c_void_p(up.ctypes.data), 0))
        return ps, th, up

    def adjoint_mass_lin(self, c, psi, theta, uphi):
        """qg_adjoint_mass_lin on host arrays (copies; returns the result)."""
        import numpy as np
        ps = np.array(psi, dtype=np.complex128, order="C")
        th = np.array(theta, dtype=np.complex128, order="C")
        up = np.array(uphi, dtype=np.float64, order="C")
        _check(self.ctx, load().qg_adjoint_mass_lin(
            self.ctx, float(c), ctypes.c_void_p(ps.ctypes.data),
            ctypes.c_void_p(th.ctypes.data), ctypes.c_void_p(up.ctypes.data), 0))
        return ps, th, up

    def tangent_get(self):
        import numpy as np
        ps = np.empty((self.M, self.K), np.complex128)
        th = np.empty_like(ps)
        up = np.empty(self.K)
        _check(self.ctx, load().qg_tangent_get(
            self.ctx, ctypes.c_void_p(ps.ctypes.data),
            ctypes.c_void_p(th.ctypes.data), ctypes.c_void_p(up.ctypes.data), 0))
        return ps, th, up

    # ------------------------------------------------------ reverse mode
    def _work(self, nsteps, interval):
        torch = self.torch
        n = ctypes.c_size_t(0)
        _check(self.ctx, load().qg_gradient_workspace_size(
            self.ctx, int(nsteps), int(interval), ctypes.byref(n)))
        buf = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        base = (buf.data_ptr() + 255) // 256 * 256
        return buf, base, n.value

    def _dev_state(self, psi, theta, uphi):
        torch = self.torch
        return (torch.as_tensor(psi, dtype=torch.complex128, device=self.device).contiguous(),
                torch.as_tensor(theta, dtype=torch.complex128, device=self.device).contiguous(),
                torch.as_tensor(uphi, dtype=torch.float64, device=self.device).contiguous())

    def gradient(self, dt, nsteps, interval=20, energy_weight=1.0,
                 terminal=None, want_grad=True):
        """qg_gradient from the current state: returns (J, (gpsi, gtheta,
        guphi)) with device tensors (None without want_grad); terminal:
        an optional co-state (psi, theta, uphi) of y^N.  The context ends
        at y^N."""
        torch = self.torch
        buf, base, nbytes = self._work(nsteps, interval)
        adj = self._dev_state(*terminal) if terminal is not None else None
        if want_grad:
            g = (torch.empty((self.M, self.K), dtype=torch.complex128, device=self.device),
                 torch.empty((self.M, self.K), dtype=torch.complex128, device=self.device),
                 torch.empty(self.K, dtype=torch.float64, device=self.device))
        J = ctypes.c_double(0.0)
        ap = [ctypes.c_void_p(a.data_ptr()) for a in adj] if adj else [None] * 3
        gp = [ctypes.c_void_p(a.data_ptr()) for a in g] if want_grad else [None] * 3
        _check(self.ctx, load().qg_gradient(
            self.ctx, float(dt), int(nsteps), int(interval), float(energy_weight),
            *ap, *gp, ctypes.byref(J), ctypes.c_void_p(base), nbytes))
        del buf
        return J.value, (g if want_grad else None)

    def energy_integral(self, dt, nsteps):
        """J = dt sum_n w_n E_K(y^n) over nsteps CNAB2 steps (forward only)."""
        return self.gradient(dt, nsteps, interval=max(1, nsteps),
                             want_grad=False)[0]

    def adjoint_explicit(self, state, costate, kappa=0.0):
        """qg_adjoint_explicit: E'(y)^H costate + kappa grad E_K(y) for a
        state y = (psi, theta, uphi); returns device tensors."""
        buf, base, nbytes = self._work(0, 1)
        y = self._dev_state(*state)
        b = [x.clone() for x in self._dev_state(*costate)]
        _check(self.ctx, load().qg_adjoint_explicit(
            self.ctx, *[ctypes.c_void_p(x.data_ptr()) for x in y],
            *[ctypes.c_void_p(x.data_ptr()) for x in b], float(kappa),
            ctypes.c_void_p(base), nbytes))
        del buf
        return tuple(b)

    def step_autotune(self, dt, scheme="cnab2", n=9):
        """n steps while timing the band-product shapes; returns the
        chosen systems per thread."""
        return qg_step_autotune(self.ctx, dt, SCHEMES[scheme], n)

    def diagnostics(self):
        return qg_diagnostics(self.ctx)


def _energy_gradient_function():
    import torch

    class EnergyGradient(torch.autograd.Function):
        """J(theta^0) = dt sum_n w_n E_K(y^n) over nsteps CNAB2 steps from
        (psi0, theta^0, uphi0), as a differentiable function of the initial
        temperature coefficients theta^0 ((M, K) complex tensor on the
        solver's device; it must meet the boundary conditions, as for
        set_state).  Forward and backward run in the HIP library
        (qg_gradient): the forward pass computes the gradient as well and
        keeps it for backward.  PyTorch's complex convention matches the
        library's (dJ/dRe + i dJ/dIm)."""

        @staticmethod
        def forward(ctx, theta0, solver, psi0, uphi0, dt, nsteps, interval):
            solver.set_state(*solver._dev_state(psi0, theta0.detach(), uphi0))
            J, g = solver.gradient(dt, nsteps, interval)
            ctx.save_for_backward(g[1])
            return torch.tensor(J, dtype=torch.float64, device=theta0.device)

        @staticmethod
        def backward(ctx, gJ):
            (gth,) = ctx.saved_tensors
            return gJ * gth, None, None, None, None, None, None

    return EnergyGradient


def energy_integral(theta0, solver, psi0, uphi0, dt, nsteps, interval=20):
    """Differentiable J(theta^0) (see _energy_gradient_function)."""
    global _EG
    if _EG is None:
        _EG = _energy_gradient_function()
    return _EG.apply(theta0, solver, psi0, uphi0, dt, nsteps, interval)


_EG = None


class QGEnsemble:
    """Many runs stepped together (qg_ensemble_*); members is a list of
    dicts with the QGSolver parameters E, Ra, Pr, eta, n_phi, n_r and
    optionally n_c, precision, pivoting, ekman_eps, method ("tau" or
    "galerkin"), buoyancy ("explicit" or "implicit"), dct ("default",
    "fft" or "mfma").  The ensemble gets a stream of its own (graph capture
    needs one)."""

    def __init__(self, members, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.params = [qg_params(m["E"], m["Ra"], m["Pr"], m["eta"],
                                 m["n_phi"], m["n_r"], m.get("n_c", 0),
                                 m.get("precision", 0), m.get("pivoting", 0),
                                 0 if m.get("ekman_eps") is None else 1,
                                 m.get("ekman_eps") or 0.0,
                                 METHODS[m.get("method", "tau")],
                                 BUOYANCY[m.get("buoyancy", "explicit")],
                                 DCT[m.get("dct", "default")])
                       for m in members]
        self.shapes = [(p.n_phi // 3 + 1,
                        p.n_c if p.n_c else (2 * (p.n_r - 1)) // 3)
                       for p in self.params]
        nbytes = qg_ensemble_workspace_size(self.params)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8,
                                         device=self.device)
            aligned = (self.workspace.data_ptr() + 255) // 256 * 256
            self.stream = torch.cuda.Stream(self.device)
            self.ens = qg_ensemble_create(self.params, aligned, nbytes,
                                          self.stream.cuda_stream)
        self.nbytes = nbytes

    def __len__(self):
        return len(self.params)

    def __del__(self):
        ens = getattr(self, "ens", None)
        if ens:
            self.ens = None
            try:
                qg_ensemble_destroy(ens)
            except TypeError:   # interpreter shutdown: module already torn down
                pass

    def set_state(self, member, psi, theta, uphi):
        M, K = self.shapes[member]
        ps = np.ascontiguousarray(psi, np.complex128)
        th = np.ascontiguousarray(theta, np.complex128)
        up = np.ascontiguousarray(uphi, np.float64)
        if ps.shape != (M, K) or th.shape != (M, K) or up.shape != (K,):
            raise ValueError("state arrays must be (M, K), (M, K), (K,)")
        qg_ensemble_set_state(self.ens, member,
                              ctypes.c_void_p(ps.ctypes.data),
                              ctypes.c_void_p(th.ctypes.data),
                              ctypes.c_void_p(up.ctypes.data), 0)

    def get_state(self, member):
        M, K = self.shapes[member]
        ps = np.empty((M, K), np.complex128)
        th = np.empty_like(ps)
        up = np.empty(K)
        qg_ensemble_get_state(self.ens, member,
                              ctypes.c_void_p(ps.ctypes.data),
                              ctypes.c_void_p(th.ctypes.data),
                              ctypes.c_void_p(up.ctypes.data), 0)
        return ps, th, up

    def step(self, dt, scheme="cnab2", n=1):
        qg_ensemble_step(self.ens, dt, SCHEMES[scheme], n)

    def groups(self):
        """(number of size groups, group of each member)."""
        return qg_ensemble_groups(self.ens, len(self.shapes))

    def step_autotune(self, dt, scheme="cnab2", n=21):
        """n steps while each size group times the band-product shapes;
        returns the chosen systems per thread of each group."""
        return qg_ensemble_step_autotune(self.ens, dt, SCHEMES[scheme], n,
                                         self.groups()[0])

    def diagnostics(self, member):
        return qg_ensemble_diagnostics(self.ens, member)
