"""Direct solve of a bordered (almost-banded) matrix (oracle; test infra).

Paper Appendix A.  The K x K tau matrix is split as
    [ A  B ] [psi_1]   [g]
    [ C  D ] [psi_2] = [h],
A: p x p, B: p x (K-p) dense boundary rows, C: (K-p) x p sparse, D: band.
Solve D x = h and D y = C (band LU, LAPACK ?gbtrf/?gbtrs), form the Schur
complement M = A - B y, solve M psi_1 = g - B x, then psi_2 = x - y psi_1.
"""
import numpy as np
import scipy.linalg as sla
from scipy.linalg import lapack


def _bandwidths(D, tol=0.0):
    nz = np.argwhere(np.abs(D) > tol)
    d = nz[:, 1] - nz[:, 0]
    return max(0, -d.min()), max(0, d.max())


def _to_lapack_band(D, kl, ku):
    n = D.shape[0]
    ab = np.zeros((2 * kl + ku + 1, n), D.dtype)
    for j in range(n):
        lo, hi = max(0, j - ku), min(n, j + kl + 1)
        ab[kl + ku + np.arange(lo, hi) - j, j] = D[lo:hi, j]
    return ab


class BorderedSolver:
    """Factor once (init or on a dt change), then solve many right-hand
    sides; matrix real or complex, right-hand sides complex or real."""

    def __init__(self, L, p):
        L = np.asarray(L)
        self.p = p
        self.cplx = np.iscomplexobj(L)
        self.A = L[:p, :p].copy()        # copies: the dense L is not kept
        self.B = L[:p, p:].copy()
        C = L[p:, :p]
        D = L[p:, p:]
        self.kl, self.ku = _bandwidths(D)
        ab = _to_lapack_band(D, self.kl, self.ku)
        if self.cplx:
            self._trf, self._trs = lapack.zgbtrf, lapack.zgbtrs
        else:
            self._trf, self._trs = lapack.dgbtrf, lapack.dgbtrs
        self.lu, self.piv, info = self._trf(ab, self.kl, self.ku)
        if info != 0:
            raise np.linalg.LinAlgError(f"band LU failed, info={info}")
        self.y = self._band_solve(C)
        self.M = self.A - self.B @ self.y
        self.Mlu = sla.lu_factor(self.M)

    def _band_solve(self, rhs):
        rhs = np.asarray(rhs)
        if not self.cplx and np.iscomplexobj(rhs):
            return (self._band_solve(rhs.real)
                    + 1j * self._band_solve(rhs.imag))
        x, info = self._trs(self.lu, self.kl, self.ku, rhs, self.piv)
        if info != 0:
            raise np.linalg.LinAlgError(f"band solve failed, info={info}")
        return x

    def solve(self, f):
        """f: (K,) or (K, nrhs)."""
        f = np.asarray(f)
        g, h = f[:self.p], f[self.p:]
        x = self._band_solve(h)
        rhs1 = g - self.B @ x
        if not self.cplx and np.iscomplexobj(rhs1):
            psi1 = (sla.lu_solve(self.Mlu, rhs1.real)
                    + 1j * sla.lu_solve(self.Mlu, rhs1.imag))
        else:
            psi1 = sla.lu_solve(self.Mlu, rhs1)
        psi2 = x - self.y @ psi1
        return np.concatenate([psi1, psi2], axis=0)
