"""Chebyshev-integration operators and tau rows (oracle; test infrastructure).

Paper Sect. 3.2 ("Spectral equations using a Chebyshev integration method").

Regularised streamfunction (Sect. 3.2.1): psi = h^2 Psi, h^2 = s_o^2 - s^2,
    u_s = (h^2/s) dPsi/dphi,  u_phi = <u_phi> - h^2 dPsi/ds + 3 s Psi,
    omega = (1/s) d(s <u_phi>)/ds - L_I Psi,
    L_I Psi = Lap(h^2 Psi) - (1/s) d(s^2 Psi)/ds,
    Lap_m = d^2/ds^2 + (1/s) d/ds - m^2/s^2.

Integrated operators (eq. psi_int, uphi_int, temp_int):
    A_m = int^4 s^4 L_I,  B_m = int^4 s^4 (Lap_m L_I + (2/E) i m),  C = int^4 s^4,
    D = int^2 s^2,  E = s^2 - 3 int s  (= int^2 s^2 (Lap_1)),
    F_m = int^2 s^2 Lap_m.
Each differential term is integrated by parts until no derivative is left
(the construction the paper describes below eq. psiint), leaving sums of
int^j (polynomial x f); those are products of the sparse Chebyshev
integration matrix of eq. (int1) and the multiplication-by-s matrix
(x T_n = (T_{n-1}+T_{n+1})/2).  The products are formed on a basis padded
by 16 modes and truncated to K x K (reading: intermediate truncation must
not clip the band).  Only rows k >= q are meaningful (paper: "for k>4",
"for k>2", 1-based); rows 0..q-1 carry the tau boundary rows instead.

Coefficients depend on m through m^2 only, apart from the Coriolis term, so
every operator is stored as its m^0, m^2, m^4 parts.

Arithmetic is in the floating type `dtype` (FP64 by default; long double
for the extended-precision reference), with eta taken as the exact value of
the binary64 number passed in.
"""
from math import comb

import numpy as np
import scipy.sparse as sp

from .grid import radii

# ----------------------------------------------------------------------------
# Laurent polynomials in s with an extra formal variable mu = m^2:
# dict {(e, k): c} meaning sum c s^e mu^k.


def lp_add(a, b, sb=1.0):
    out = dict(a)
    for key, c in b.items():
        out[key] = out.get(key, 0.0) + sb * c
    return {k: v for k, v in out.items() if v != 0}


def lp_mul(a, b):
    out = {}
    for (e1, k1), c1 in a.items():
        for (e2, k2), c2 in b.items():
            key = (e1 + e2, k1 + k2)
            out[key] = out.get(key, 0.0) + c1 * c2
    return {k: v for k, v in out.items() if v != 0}


def lp_ds(a):
    out = {}
    for (e, k), c in a.items():
        if e != 0:
            out[(e - 1, k)] = out.get((e - 1, k), 0.0) + e * c
    return {k: v for k, v in out.items() if v != 0}


def lp_ds_n(a, n):
    for _ in range(n):
        a = lp_ds(a)
    return a


def mono(e, c=1.0, k=0):
    return {(e, k): c}


# Differential operators: dict {p: laurent poly} meaning sum a_p(s) d^p/ds^p.
def op_add(A, B, sb=1.0):
    out = dict(A)
    for p, b in B.items():
        out[p] = lp_add(out.get(p, {}), b, sb)
    return {p: v for p, v in out.items() if v}


def op_compose(A, B):
    """(A o B) f = sum_p a_p d^p [ sum_r b_r d^r f ] by the Leibniz rule."""
    out = {}
    for p, a in A.items():
        for r, b in B.items():
            for j in range(p + 1):
                term = lp_mul(a, lp_ds_n(b, j))
                if not term:
                    continue
                key = p - j + r
                out[key] = lp_add(out.get(key, {}), lp_mul(
                    {(0, 0): float(comb(p, j))}, term))
    return {p: v for p, v in out.items() if v}


def mult(poly):
    return {0: dict(poly)}


D1 = {1: {(0, 0): 1.0}}


def laplacian_m(m2=None):
    """Lap_m = d^2 + s^-1 d - m^2 s^-2 (m^2 formal unless a number is
    given)."""
    third = mono(-2, -1.0, 1) if m2 is None else mono(-2, -float(m2))
    return {2: mono(0), 1: mono(-1), 0: third}


def qg_operators(eta, dtype=np.float64):
    """The polynomial-coefficient differential operators of Sect. 3.2."""
    s_i, s_o = radii(dtype(eta))
    h2 = {(0, 0): s_o**2, (2, 0): dtype(-1)}
    lap = laplacian_m()
    L_I = op_add(op_compose(lap, mult(h2)),
                 op_compose(mult(mono(-1)), op_compose(D1, mult(mono(2)))),
                 -1.0)
    s4LI = op_compose(mult(mono(4)), L_I)
    s4LapLI = op_compose(mult(mono(4)), op_compose(lap, L_I))
    s2Lap = op_compose(mult(mono(2)), lap)
    s2Lap1 = op_compose(mult(mono(2)), laplacian_m(1))
    return dict(L_I=L_I, s4LI=s4LI, s4LapLI=s4LapLI, s2Lap=s2Lap,
                s2Lap1=s2Lap1, h2=h2)


def assert_polynomial(op):
    for p, a in op.items():
        for (e, k), c in a.items():
            if e < 0 and abs(c) > 1e-12:
                raise ValueError(f"negative power s^{e} in d^{p} coefficient")


def integrate_by_parts(op, q):
    """int^q (sum_p a_p d^p) -> {j: b_j} with int^q ... = sum_j int^j b_j
    (up to a polynomial of degree < q, i.e. rows < q), using
    int^j (a f^(p)) = int^(j-1) (a f^(p-1)) - int^j (a' f^(p-1))."""
    assert_polynomial(op)
    terms = {}
    work = [(q, p, {k: v for k, v in a.items() if k[0] >= 0})
            for p, a in op.items()]
    while work:
        j, p, a = work.pop()
        if not a:
            continue
        if p == 0:
            terms[j] = lp_add(terms.get(j, {}), a)
            continue
        assert j >= 1
        work.append((j - 1, p - 1, a))
        work.append((j, p - 1, lp_add({}, lp_ds(a), -1.0)))
    return {j: b for j, b in terms.items() if b}


# ----------------------------------------------------------------------------
# Sparse Chebyshev matrices on a padded basis of size N.

def int_matrix_x(N, dtype=np.float64):
    """eq. (int1): int T_n dx = (T_{n+1}/(n+1) - T_{n-1}/(n-1))/2, n > 1,
    with int T_0 = T_1 and int T_1 = T_2/4 (+const).  Row 0 (the constant)
    is left zero."""
    rows, cols, vals = [], [], []
    one = dtype(1)
    for k in range(1, N):
        cprev = 2 * one if k == 1 else one
        rows.append(k), cols.append(k - 1), vals.append(cprev / (2 * k))
        if k + 1 < N:
            rows.append(k), cols.append(k + 1), vals.append(-one / (2 * k))
    return sp.csr_matrix((np.array(vals, dtype), (rows, cols)), shape=(N, N))


def mulx_matrix(N, dtype=np.float64):
    """x T_0 = T_1, x T_n = (T_{n-1} + T_{n+1})/2."""
    rows, cols, vals = [1], [0], [1.0]
    for n in range(1, N):
        rows.append(n - 1), cols.append(n), vals.append(0.5)
        if n + 1 < N:
            rows.append(n + 1), cols.append(n), vals.append(0.5)
    return sp.csr_matrix((np.array(vals, dtype), (rows, cols)), shape=(N, N))


class ChebAlgebra:
    """Integration in s and multiplication by s on the padded basis
    (s = x/2 + c, ds = dx/2)."""

    def __init__(self, eta, N, dtype=np.float64):
        s_i, s_o = radii(dtype(eta))
        self.N = N
        self.dtype = dtype
        half_gap = (s_o - s_i) / 2
        c = (s_o + s_i) / 2
        self.I = (half_gap * int_matrix_x(N, dtype)).tocsr()
        self.S = (half_gap * mulx_matrix(N, dtype)
                  + c * sp.identity(N, dtype=dtype)).tocsr()
        self._spow = [sp.identity(N, dtype=dtype, format="csr")]

    def spow(self, e):
        while len(self._spow) <= e:
            self._spow.append((self.S @ self._spow[-1]).tocsr())
        return self._spow[e]

    def mul_poly(self, poly_by_power):
        out = sp.csr_matrix((self.N, self.N), dtype=self.dtype)
        for e, c in poly_by_power.items():
            out = out + c * self.spow(e)
        return out

    def ipow(self, j):
        out = sp.identity(self.N, dtype=self.dtype, format="csr")
        for _ in range(j):
            out = (self.I @ out).tocsr()
        return out

    def integrated(self, op, q):
        """Matrices {k: int^q (op) restricted to the mu^k part}."""
        terms = integrate_by_parts(op, q)
        by_k = {}
        for j, b in terms.items():
            for (e, k), c in b.items():
                by_k.setdefault(k, {}).setdefault(j, {})
                by_k[k][j][e] = by_k[k][j].get(e, 0.0) + c
        mats = {}
        for k, per_j in by_k.items():
            out = sp.csr_matrix((self.N, self.N), dtype=self.dtype)
            for j, poly in per_j.items():
                out = out + self.ipow(j) @ self.mul_poly(poly)
            mats[k] = out.tocsr()
        return mats


PAD = 16


class IntegrationOperators:
    """K x K dense parts of the integration-method operators (m-split)."""

    def __init__(self, eta, K, dtype=np.float64):
        self.eta, self.K = eta, K
        self.dtype = dtype
        N = K + PAD
        alg = ChebAlgebra(eta, N, dtype)
        ops = qg_operators(eta, dtype)

        def dense(mats):
            return {k: np.asarray(m[:K, :K].todense()) for k, m in
                    mats.items()}
        a = dense(alg.integrated(ops["s4LI"], 4))
        b = dense(alg.integrated(ops["s4LapLI"], 4))
        c = dense(alg.integrated(mult(mono(4)), 4))
        d = dense(alg.integrated(mult(mono(2)), 2))
        f = dense(alg.integrated(ops["s2Lap"], 2))
        e = dense(alg.integrated(ops["s2Lap1"], 2))
        z = np.zeros((K, K), dtype)
        self.A0, self.A2 = a.get(0, z), a.get(1, z)
        self.B0, self.B2, self.B4 = b.get(0, z), b.get(1, z), b.get(2, z)
        self.C = c[0]
        self.D = d[0]
        self.F0, self.F2 = f.get(0, z), f.get(1, z)
        self.E = e[0]

    def A(self, m):
        return self.A0 + m * m * self.A2

    def B(self, m, E):
        """B_m including the implicit Coriolis term (2/E) i m C."""
        dt = self.dtype
        m2 = dt(m * m)
        return (self.B0 + m2 * self.B2 + m2 * m2 * self.B4
                + (1j * (dt(2) * m / dt(E))) * self.C)

    def F(self, m):
        return self.F0 + self.dtype(m * m) * self.F2


# ----------------------------------------------------------------------------
# Tau rows, paper eq. (bcs_coll_dirichlet), (bcs_coll_neumann), (bc_d3psi_coll)
# written on standard coefficients: they are the boundary evaluations
# f(s_o) = sum a_n, f(s_i) = sum (-1)^n a_n, f'''(s_o) ~ sum T_n'''(1) a_n,
# f'(s_i) ~ sum T_n'(-1) a_n.  Row order: Dirichlet s_o, Dirichlet s_i,
# third derivative at s_o, Neumann at s_i (Sect. 3.2.2, Fig. 1b).

def tau_rows_psi(K, dtype=np.float64):
    n = np.arange(K, dtype=dtype)
    return np.array([np.ones(K, dtype), (-1) ** n,
                     n**2 * (n**2 - 1) * (n**2 - 4) / 15,
                     (-1) ** (n + 1) * n**2])


def tau_rows_dirichlet(K, dtype=np.float64):
    n = np.arange(K, dtype=dtype)
    return np.array([np.ones(K, dtype), (-1) ** n])


def bordered_lhs(bc_rows, op_rows):
    """Full K x K tau matrix: boundary rows on top, operator rows k >= p."""
    p = bc_rows.shape[0]
    L = np.array(op_rows, dtype=np.result_type(op_rows, np.float64),
                 copy=True)
    L[:p, :] = bc_rows
    return L


# ----------------------------------------------------------------------------
def evaluate_op(op, m, derivs, s):
    """sum_p a_p(s; m^2) f^(p)(s) on a grid; derivs[p] holds f^(p)(s);
    m and s broadcast against each other."""
    m2 = np.asarray(m, dtype=np.result_type(np.asarray(s).real, np.float64)) ** 2
    out = 0.0
    for p, a in op.items():
        coef = 0.0
        for (e, k), c in a.items():
            coef = coef + c * s**e * m2**k
        out = out + coef * derivs[p]
    return out
