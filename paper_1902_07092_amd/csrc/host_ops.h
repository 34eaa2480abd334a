// Host-side construction of the Chebyshev-integration operators and of the
// per-wavenumber bordered factorisations (run once per time-step size).
#pragma once
#include <complex>
#include <cstdint>
#include <vector>

namespace qg {

using cplx = std::complex<double>;
using cplxl = std::complex<long double>;

// Width of every stored operator band: offsets -8..+8 around the diagonal.
constexpr int BANDW = 17;
constexpr int BANDC = 8;  // centre index of a stored band row

// m-independent banded operators, rows k = 0..K-1, entry [k*BANDW + (n-k+8)]
// (rows below the number of tau rows are meaningless and stored as zero).
struct Operators {
  int K = 0;
  std::vector<double> A0, A2;            // int^4 s^4 L_I = A0 + m^2 A2
  std::vector<double> B0, B2, B4;        // int^4 s^4 Lap_m L_I
  std::vector<double> C;                 // int^4 s^4
  std::vector<double> D;                 // int^2 s^2
  std::vector<double> F0, F2;            // int^2 s^2 Lap_m = F0 + m^2 F2
};

Operators build_operators(double eta, int K);

// Factorisation of one bordered system (p tau rows on top of a band with
// kl sub- and ku super-diagonals).  Band LU of the band block D (positions
// 0..n-1, n = K - p), with partial pivoting or without row interchanges,
// and the Schur data for the border.
template <typename T>
struct BorderedFactor {
  int p = 0, n = 0, kl = 0, ku = 0;
  int kut = 0;                // stored U super-diagonals: kl + ku pivoted, ku unpivoted
  double growth = 0.0;        // max |U| / max |D| over the band
  std::vector<int32_t> piv;   // [n] pivot offset (row swapped with j at step j)
  std::vector<T> Lc;          // [n][kl] multipliers of column j, rows j+1..j+kl
  std::vector<T> Uc;          // [n][kut+1] e=0: 1/U(j,j); e>=1: U(j-e, j)
  std::vector<T> W;           // [p][n]  w = B D^-1
  std::vector<T> Cb;          // [kl][p] first kl rows of the border column C
  std::vector<T> Minv;        // [p][p]  (A - w C)^-1
};

// Full bordered K x K matrix given as dense rows; builds the factor.
// Instantiated for double, complex<double> and their long-double
// counterparts (the factorisation in extended precision, every entry then
// rounded once to binary64 when the device layout is packed).
template <typename T>
bool factor_bordered(const std::vector<T>& full, int K, int p, int kl, int ku, bool pivot,
                     BorderedFactor<T>& out);


// Galerkin bases (Sect. 3.2.2, Appendix B).  gamma_0..4 of the Psi basis
// function phi_j = sum_i gamma_i^j T_{j+i} (gamma_0 = 1), from the closed
// forms of Appendix B.
void galerkin_gamma(int j, long double g[5]);

// P_q Op S: the (K - q) x (K - q) Galerkin system (dense rows) from the
// full K x K operator `full` (rows q.. used): S the Psi stencil (q = 4) or
// the Dirichlet stencil T_{n+2} - T_n (q = 2).  A band with 8 / 12 (q = 4)
// or 4 / 6 (q = 2) sub- / super-diagonals.
template <typename T>
void galerkin_matrix(const std::vector<T>& full, int K, int q, std::vector<T>& G);

// Tau rows: Dirichlet at s_o, Dirichlet at s_i, third derivative at s_o,
// Neumann at s_i (first p of them).
void tau_row(int which, int K, double* row);

}  // namespace qg
