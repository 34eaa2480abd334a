// Host-side operator construction and bordered band factorisation.
//
// Operators (Gastine 2019, Sect. 3.2, eqs. psi_int, uphi_int, temp_int):
//   A_m = int^4 s^4 L_I,  B_m = int^4 s^4 Lap_m L_I (+ Coriolis, added per m),
//   C = int^4 s^4,  D = int^2 s^2,  F_m = int^2 s^2 Lap_m  (E = F_1).
// The differential operators are written with polynomial coefficients in s
// (expanded by hand from L_I Psi = Lap_m(h^2 Psi) - (1/s) d(s^2 Psi)/ds,
// h^2 = a - s^2, a = s_o^2), every term int^q (c(s) d^p) is integrated by
// parts until no derivative remains (the construction described below
// eq. psiint), and each remaining int^j (polynomial x f) is applied to the
// Chebyshev basis vectors with the integration recurrence of eq. (int1)
// and the multiplication-by-s recurrence, on a padded basis.
#include "host_ops.h"

#include <cmath>
#include <map>

namespace qg {

namespace {

using Poly = std::vector<double>;  // coefficients of s^0, s^1, ...

Poly pderiv(const Poly& a) {
  Poly d(a.size() > 1 ? a.size() - 1 : 1, 0.0);
  for (size_t e = 1; e < a.size(); ++e) d[e - 1] = e * a[e];
  return d;
}

void padd(Poly& acc, const Poly& b, double sc) {
  if (acc.size() < b.size()) acc.resize(b.size(), 0.0);
  for (size_t e = 0; e < b.size(); ++e) acc[e] += sc * b[e];
}

// d^p coefficients -> {j: b_j} with int^q sum_p c_p d^p = sum_j int^j b_j
// (modulo a polynomial of degree < q), via
//   int^j (c f^(p)) = int^(j-1) (c f^(p-1)) - int^j (c' f^(p-1)).
std::map<int, Poly> reduce(const std::vector<Poly>& by_p, int q) {
  struct T { int j, p; Poly c; };
  std::vector<T> work;
  for (int p = 0; p < (int)by_p.size(); ++p)
    if (!by_p[p].empty()) work.push_back({q, p, by_p[p]});
  std::map<int, Poly> out;
  while (!work.empty()) {
    T t = work.back();
    work.pop_back();
    bool zero = true;
    for (double v : t.c) zero = zero && v == 0.0;
    if (zero) continue;
    if (t.p == 0) { padd(out[t.j], t.c, 1.0); continue; }
    work.push_back({t.j - 1, t.p - 1, t.c});
    Poly d = pderiv(t.c);
    for (double& v : d) v = -v;
    work.push_back({t.j, t.p - 1, d});
  }
  return out;
}

struct Basis {
  int N;        // padded size
  double half;  // (s_o - s_i)/2
  double mid;   // (s_o + s_i)/2
  // multiply by s = half x + mid
  void mul_s(const std::vector<double>& v, std::vector<double>& r) const {
    r.assign(N, 0.0);
    for (int k = 0; k < N; ++k) {
      double xv = 0.0;
      if (k + 1 < N) xv += 0.5 * v[k + 1];
      if (k == 1) xv += v[0];
      else if (k >= 2) xv += 0.5 * v[k - 1];
      r[k] = mid * v[k] + half * xv;
    }
  }
  // integrate in s: eq. (int1), row 0 left zero
  void integ(const std::vector<double>& v, std::vector<double>& r) const {
    r.assign(N, 0.0);
    for (int k = 1; k < N; ++k) {
      double prev = (k == 1 ? 2.0 : 1.0) * v[k - 1];
      double next = (k + 1 < N) ? v[k + 1] : 0.0;
      r[k] = half * (prev - next) / (2.0 * k);
    }
  }
};

// Band of rows q..K-1 of sum_j int^j M_{b_j} on the K first basis vectors.
std::vector<double> band_of(const std::map<int, Poly>& terms, int q, int K,
                            const Basis& B) {
  std::vector<double> band((size_t)K * BANDW, 0.0);
  std::vector<double> e(B.N), acc(B.N), t1(B.N), t2(B.N);
  for (int n = 0; n < K; ++n) {
    std::fill(acc.begin(), acc.end(), 0.0);
    for (const auto& jt : terms) {
      const Poly& b = jt.second;
      // Horner: r = sum_e b_e s^e e_n
      std::fill(e.begin(), e.end(), 0.0);
      e[n] = 1.0;
      std::vector<double> r(B.N, 0.0);
      for (int ex = (int)b.size() - 1; ex >= 0; --ex) {
        B.mul_s(r, t1);
        for (int k = 0; k < B.N; ++k) r[k] = t1[k] + b[ex] * e[k];
      }
      for (int j = 0; j < jt.first; ++j) {
        B.integ(r, t2);
        r.swap(t2);
      }
      for (int k = 0; k < B.N; ++k) acc[k] += r[k];
    }
    for (int k = q; k < K; ++k) {
      int off = n - k;
      if (off >= -BANDC && off <= BANDC) band[(size_t)k * BANDW + off + BANDC] = acc[k];
    }
  }
  return band;
}

Poly P(std::initializer_list<std::pair<int, double>> mon) {
  Poly p;
  for (auto& m : mon) {
    if ((int)p.size() <= m.first) p.resize(m.first + 1, 0.0);
    p[m.first] += m.second;
  }
  return p;
}

}  // namespace

Operators build_operators(double eta, int K) {
  const double s_i = eta / (1.0 - eta), s_o = 1.0 / (1.0 - eta);
  const double a = s_o * s_o;
  Basis B{K + 24, 0.5 * (s_o - s_i), 0.5 * (s_o + s_i)};
  Operators o;
  o.K = K;
  // s^4 L_I = s^4 h^2 d^2 + (s^3 h^2 - 5 s^5) d - (6 s^4 + m^2 s^2 h^2)
  std::vector<Poly> a0 = {P({{4, -6.0}}), P({{3, a}, {5, -6.0}}),
                          P({{4, a}, {6, -1.0}})};
  std::vector<Poly> a2 = {P({{2, -a}, {4, 1.0}})};
  // s^4 Lap_m L_I = s^2 G'' - 3 s G' + (4 - m^2) G,  G = s^2 L_I Psi
  std::vector<Poly> b0 = {Poly{}, P({{1, a}, {3, -12.0}}),
                          P({{2, -a}, {4, -28.0}}), P({{3, 2 * a}, {5, -11.0}}),
                          P({{4, a}, {6, -1.0}})};
  std::vector<Poly> b2 = {P({{0, -4 * a}, {2, 6.0}}), P({{1, 2 * a}, {3, 7.0}}),
                          P({{2, -2 * a}, {4, 2.0}})};
  std::vector<Poly> b4 = {P({{0, a}, {2, -1.0}})};
  std::vector<Poly> c = {P({{4, 1.0}})};
  std::vector<Poly> d = {P({{2, 1.0}})};
  // s^2 Lap_m = s^2 d^2 + s d - m^2
  std::vector<Poly> f0 = {Poly{}, P({{1, 1.0}}), P({{2, 1.0}})};
  std::vector<Poly> f2 = {P({{0, -1.0}})};
  o.A0 = band_of(reduce(a0, 4), 4, K, B);
  o.A2 = band_of(reduce(a2, 4), 4, K, B);
  o.B0 = band_of(reduce(b0, 4), 4, K, B);
  o.B2 = band_of(reduce(b2, 4), 4, K, B);
  o.B4 = band_of(reduce(b4, 4), 4, K, B);
  o.C = band_of(reduce(c, 4), 4, K, B);
  o.D = band_of(reduce(d, 2), 2, K, B);
  o.F0 = band_of(reduce(f0, 2), 2, K, B);
  o.F2 = band_of(reduce(f2, 2), 2, K, B);
  return o;
}

void tau_row(int which, int K, double* row) {
  for (int n = 0; n < K; ++n) {
    double dn = n, sg = (n % 2) ? -1.0 : 1.0;
    switch (which) {
      case 0: row[n] = 1.0; break;                                     // f(s_o)
      case 1: row[n] = sg; break;                                      // f(s_i)
      case 2: row[n] = dn * dn * (dn * dn - 1) * (dn * dn - 4) / 15.0; break;
      default: row[n] = -sg * dn * dn; break;                          // f'(s_i)
    }
  }
}

namespace {
template <typename T> double mag(const T& v) { return std::abs(v); }
}  // namespace

template <typename T>
bool factor_bordered(const std::vector<T>& full, int K, int p, int kl, int ku, bool pivot,
                     BorderedFactor<T>& f) {
  const int n = K - p;
  f.p = p; f.n = n; f.kl = kl; f.ku = ku;
  const int kut = pivot ? kl + ku : ku;   // U bandwidth (with the pivoting fill)
  f.kut = kut;
  const int ld = 2 * kl + ku + 1;      // LAPACK band storage
  std::vector<T> ab((size_t)ld * n, T(0));
  auto A = [&](int i, int j) -> T& { return ab[(size_t)j * ld + (kl + ku + i - j)]; };
  auto Dfull = [&](int i, int j) { return full[(size_t)(p + i) * K + (p + j)]; };
  double dmax = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = std::max(0, j - ku); i <= std::min(n - 1, j + kl); ++i) {
      A(i, j) = Dfull(i, j);
      dmax = std::max(dmax, mag(A(i, j)));
    }
  std::vector<int> ipiv(n);
  for (int j = 0; j < n; ++j) {
    int last = std::min(n - 1, j + kl);
    int jp = j;
    double best = mag(A(j, j));
    if (pivot)
      for (int i = j + 1; i <= last; ++i)
        if (mag(A(i, j)) > best) { best = mag(A(i, j)); jp = i; }
    ipiv[j] = jp;
    if (best == 0.0) return false;
    int cend = std::min(n - 1, j + kut);
    if (jp != j)
      for (int cc = j; cc <= cend; ++cc) std::swap(A(j, cc), A(jp, cc));
    T inv = T(1) / A(j, j);
    for (int i = j + 1; i <= last; ++i) A(i, j) *= inv;
    for (int cc = j + 1; cc <= cend; ++cc) {
      T u = A(j, cc);
      if (u == T(0)) continue;
      for (int i = j + 1; i <= last; ++i) A(i, cc) -= A(i, j) * u;
    }
  }
  double umax = 0.0;
  for (int j = 0; j < n; ++j)
    for (int e = 0; e <= kut && j - e >= 0; ++e) umax = std::max(umax, mag(A(j - e, j)));
  f.growth = dmax > 0.0 ? umax / dmax : 0.0;
  f.piv.assign(n, 0);
  f.Lc.assign((size_t)n * kl, T(0));
  f.Uc.assign((size_t)n * (kut + 1), T(0));
  for (int j = 0; j < n; ++j) {
    f.piv[j] = ipiv[j] - j;
    for (int d = 0; d < kl; ++d)
      if (j + 1 + d < n) f.Lc[(size_t)j * kl + d] = A(j + 1 + d, j);
    f.Uc[(size_t)j * (kut + 1)] = T(1) / A(j, j);
    for (int e = 1; e <= kut; ++e)
      if (j - e >= 0) f.Uc[(size_t)j * (kut + 1) + e] = A(j - e, j);
  }
  // w_i = B_i D^-1, i.e. D^T w_i^T = B_i^T (plain transpose).
  f.W.assign((size_t)p * n, T(0));
  std::vector<T> u(n);
  for (int i = 0; i < p; ++i) {
    for (int j = 0; j < n; ++j) u[j] = full[(size_t)i * K + p + j];
    // U^T u = b (forward)
    for (int j = 0; j < n; ++j) {
      T s = u[j];
      for (int e = 1; e <= kut && j - e >= 0; ++e) s -= A(j - e, j) * u[j - e];
      u[j] = s / A(j, j);
    }
    // apply the transposed elimination steps in reverse order
    for (int j = n - 1; j >= 0; --j) {
      T s = u[j];
      for (int d = 0; d < kl && j + 1 + d < n; ++d) s -= A(j + 1 + d, j) * u[j + 1 + d];
      u[j] = s;
      if (ipiv[j] != j) std::swap(u[j], u[ipiv[j]]);
    }
    for (int j = 0; j < n; ++j) f.W[(size_t)i * n + j] = u[j];
  }
  f.Cb.assign((size_t)kl * p, T(0));
  for (int r = 0; r < kl && r < n; ++r)
    for (int i = 0; i < p; ++i) f.Cb[(size_t)r * p + i] = full[(size_t)(p + r) * K + i];
  // M = A - w C, inverted by Gauss-Jordan with partial pivoting
  std::vector<T> M((size_t)p * p), I((size_t)p * p, T(0));
  for (int i = 0; i < p; ++i) {
    I[(size_t)i * p + i] = T(1);
    for (int k = 0; k < p; ++k) {
      T s = full[(size_t)i * K + k];
      for (int r = 0; r < kl && r < n; ++r) s -= f.W[(size_t)i * n + r] * f.Cb[(size_t)r * p + k];
      M[(size_t)i * p + k] = s;
    }
  }
  for (int col = 0; col < p; ++col) {
    int piv = col;
    for (int r = col + 1; r < p; ++r)
      if (mag(M[(size_t)r * p + col]) > mag(M[(size_t)piv * p + col])) piv = r;
    if (mag(M[(size_t)piv * p + col]) == 0.0) return false;
    for (int k = 0; k < p; ++k) {
      std::swap(M[(size_t)col * p + k], M[(size_t)piv * p + k]);
      std::swap(I[(size_t)col * p + k], I[(size_t)piv * p + k]);
    }
    T inv = T(1) / M[(size_t)col * p + col];
    for (int k = 0; k < p; ++k) { M[(size_t)col * p + k] *= inv; I[(size_t)col * p + k] *= inv; }
    for (int r = 0; r < p; ++r) {
      if (r == col) continue;
      T fct = M[(size_t)r * p + col];
      for (int k = 0; k < p; ++k) {
        M[(size_t)r * p + k] -= fct * M[(size_t)col * p + k];
        I[(size_t)r * p + k] -= fct * I[(size_t)col * p + k];
      }
    }
  }
  f.Minv = I;
  return true;
}

void galerkin_gamma(int j, long double g[5]) {
  const long double n = j;
  const long double n2 = n * n, n3 = n2 * n, n4 = n3 * n;
  const long double q = 2 * n4 + 20 * n3 + 78 * n2 + 140 * n + 95;
  g[0] = 1.0L;
  g[1] = 8 * (n + 1) * (n2 + 4 * n + 5) / q;
  g[2] = -2 * (n + 2) * (2 * n4 + 16 * n3 + 58 * n2 + 104 * n + 75) / ((n + 3) * q);
  g[3] = -g[1];
  g[4] = (n + 1) * (2 * n4 + 12 * n3 + 30 * n2 + 36 * n + 15) / ((n + 3) * q);
}

template <typename T>
void galerkin_matrix(const std::vector<T>& full, int K, int q, std::vector<T>& G) {
  const int n = K - q;
  G.assign((size_t)n * n, T(0));
  // column j of S: rows j..j+4 (gamma_i^j) or rows j (-1) and j+2 (+1)
  for (int j = 0; j < n; ++j) {
    long double s[5] = {0, 0, 0, 0, 0};
    int ns;
    if (q == 4) {
      galerkin_gamma(j, s);
      ns = 5;
    } else {
      s[0] = -1.0L;
      s[2] = 1.0L;
      ns = 3;
    }
    // rows i of P_q Op with a nonzero in columns j..j+ns-1: the operator
    // band reaches 8 columns either side of its row q + i
    const int lo = std::max(0, j - 8 - q), hi = std::min(n - 1, j + ns - 1 + 8 - q);
    for (int i = lo; i <= hi; ++i) {
      T acc(0);
      for (int r = 0; r < ns && j + r < K; ++r)
        if (s[r] != 0.0L) acc += full[(size_t)(q + i) * K + j + r] * T(s[r]);
      G[(size_t)i * n + j] = acc;
    }
  }
}

template void galerkin_matrix<long double>(const std::vector<long double>&, int, int,
                                           std::vector<long double>&);
template void galerkin_matrix<cplxl>(const std::vector<cplxl>&, int, int, std::vector<cplxl>&);

template bool factor_bordered<double>(const std::vector<double>&, int, int, int, int, bool,
                                      BorderedFactor<double>&);
template bool factor_bordered<cplx>(const std::vector<cplx>&, int, int, int, int, bool,
                                    BorderedFactor<cplx>&);
template bool factor_bordered<long double>(const std::vector<long double>&, int, int, int, int,
                                           bool, BorderedFactor<long double>&);
template bool factor_bordered<cplxl>(const std::vector<cplxl>&, int, int, int, int, bool,
                                     BorderedFactor<cplxl>&);

}  // namespace qg
