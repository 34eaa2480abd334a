"""Direct solve of a bordered (almost-banded) matrix (oracle; test infra).

Paper Appendix A.  The K x K tau matrix is split as
    [ A  B ] [psi_1]   [g]
    [ C  D ] [psi_2] = [h],
A: p x p, B: p x (K-p) dense boundary rows, C: (K-p) x p sparse, D: band.
Solve D x = h and D y = C (band LU, LAPACK ?gbtrf/?gbtrs), form the Schur
complement M = A - B y, solve M psi_1 = g - B x, then psi_2 = x - y psi_1.

BandLU is the band factorisation alone (also the whole solve of the pure
band systems of the Galerkin bases, oracle.galerkin).

pivot=False replaces the LAPACK band LU by a plain band LU without row
interchanges (Doolittle, written out below).  The appendix does not fix
the elimination order; the two are equally valid binary64 implementations
of the same solve, and their difference measures how much the rounding
of the solve alone moves a step's result.
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


class BandLU:
    """LU of a band matrix D (kl sub-, ku super-diagonals taken from its
    nonzero pattern): LAPACK ?gbtrf/?gbtrs with partial pivoting, or with
    pivot=False the plain band LU without row interchanges below."""

    def __init__(self, D, pivot=True):
        D = np.asarray(D)
        self.pivot = pivot
        self.cplx = np.iscomplexobj(D)
        self.n = D.shape[0]
        self.kl, self.ku = _bandwidths(D)
        self.dmax = float(np.abs(D).max())
        if not pivot:
            self._factor_plain(D)
            return
        ab = _to_lapack_band(D, self.kl, self.ku)
        if self.cplx:
            self._trf, self._trs = lapack.zgbtrf, lapack.zgbtrs
        else:
            self._trf, self._trs = lapack.dgbtrf, lapack.dgbtrs
        self.lu, self.piv, info = self._trf(ab, self.kl, self.ku)
        if info != 0:
            raise np.linalg.LinAlgError(f"band LU failed, info={info}")

    def _factor_plain(self, D):
        """Band LU without row interchanges: column j's multipliers
        l_ij = a_ij / u_jj (i = j+1..j+kl), then row i -= l_ij row j over
        the band; L and U overwrite a copy of the band."""
        n, kl, ku = D.shape[0], self.kl, self.ku
        a = np.array(D, dtype=np.complex128 if self.cplx else np.float64)
        for j in range(n):
            piv = a[j, j]
            if piv == 0:
                raise np.linalg.LinAlgError(f"zero pivot at step {j}")
            lo, hi = j + 1, min(n, j + kl + 1)
            ce = min(n, j + ku + 1)
            a[lo:hi, j] /= piv
            a[lo:hi, lo:ce] -= np.outer(a[lo:hi, j], a[j, lo:ce])
        self._plain = a

    def growth(self):
        """max |U| / max |D| of the plain factorisation (pivot=False)."""
        return float(np.abs(np.triu(self._plain)).max()) / self.dmax

    def _plain_solve(self, rhs):
        a, kl, ku = self._plain, self.kl, self.ku
        n = a.shape[0]
        x = np.array(rhs, dtype=np.result_type(a, rhs), copy=True)
        for j in range(n):                      # L z = rhs (unit diagonal)
            hi = min(n, j + kl + 1)
            x[j + 1:hi] -= np.multiply.outer(a[j + 1:hi, j], x[j])
        for j in range(n - 1, -1, -1):          # U x = z
            x[j] = x[j] / a[j, j]
            lo = max(0, j - ku)
            x[lo:j] -= np.multiply.outer(a[lo:j, j], x[j])
        return x

    def solve(self, rhs):
        rhs = np.asarray(rhs)
        if not self.pivot:
            return self._plain_solve(rhs)
        if not self.cplx and np.iscomplexobj(rhs):
            return self.solve(rhs.real) + 1j * self.solve(rhs.imag)
        x, info = self._trs(self.lu, self.kl, self.ku, rhs, self.piv)
        if info != 0:
            raise np.linalg.LinAlgError(f"band solve failed, info={info}")
        return x


class BorderedSolver:
    """Factor once (init or on a dt change), then solve many right-hand
    sides; matrix real or complex, right-hand sides complex or real."""

    def __init__(self, L, p, pivot=True):
        L = np.asarray(L)
        self.p = p
        self.pivot = pivot
        self.cplx = np.iscomplexobj(L)
        self.A = L[:p, :p].copy()        # copies: the dense L is not kept
        self.B = L[:p, p:].copy()
        C = L[p:, :p]
        self.band = BandLU(L[p:, p:], pivot)
        self.kl, self.ku = self.band.kl, self.band.ku
        self.y = self._band_solve(C)
        self.M = self.A - self.B @ self.y
        self.Mlu = sla.lu_factor(self.M)

    def _band_solve(self, rhs):
        return self.band.solve(rhs)

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
