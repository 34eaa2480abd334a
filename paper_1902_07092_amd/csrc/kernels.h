// Kernel interfaces of the QG step (gfx950, FP64).
#pragma once
#include <hip/hip_runtime.h>

namespace qg {

// In-LDS Stockham FFT plan: n = product of radices (2, 3 or 4), twiddles
// tw[k] = exp(-2 pi i k / n), k < n.
struct FftPlan {
  int n;
  int npass;
  int radix[24];
  const double2* tw;   // tw[k * tw_stride] = exp(-2 pi i k / n)
  int tw_stride;
};

struct Geom {
  int M, K, R, nphi;
  double s_o, s_i, mid, half;   // s = half * x + mid
  double dtc_coef;              // dT_c/ds = dtc_coef / s
  double Ra_Pr, inv_Pr, two_over_E;
  const double* xk;             // Gauss-Lobatto nodes, x_0 = +1
  const double* wq;             // Clenshaw-Curtis weight * half * s_k
  const double* dsk;            // local radial spacing (CFL)
  FftPlan dct;                  // length 2 (R - 1)
  FftPlan phi;                  // length nphi
  FftPlan phi_half;             // length nphi / 2 (real transforms)
};

struct Bands {  // [17][K] each (offset-major): entry (k, n) at [(n - k + 8) * K + k]
  const double *A0, *A2, *B0, *B2, *B4, *C, *D, *F0, *F2;
};

// Factors of all bordered systems of one kind (see host_ops.h layout).
template <typename TF>
struct FactorSet {
  const int* piv;     // [S][n]
  const TF* Lc;       // [S][n][kl]
  const TF* Uc;       // [S][n][kl+ku+1]
  const TF* W;        // [S][p][n]
  const TF* Cb;       // [S][kl][p]
  const TF* Minv;     // [S][p][p]
};

constexpr int MAX_TERMS = 8;

// Right-hand side of one implicit solve:
//   rhs = (Mass + cL * Lin) y_base + sum_q coef_q * slot_q     (rows >= p)
struct RhsSpec {
  const double2* base_psi;   // [M][K] (row m = 0 holds the zonal flow)
  const double2* base_th;    // [M][K]
  double cL;
  int nterm;
  const double2* term_psi[MAX_TERMS];
  const double2* term_th[MAX_TERMS];
  double coef[MAX_TERMS];
  double2* out_psi;          // new state
  double2* out_th;
  double2* lin_psi;          // optional: Lin y_new (nullptr: not needed)
  double2* lin_th;
};

}  // namespace qg
