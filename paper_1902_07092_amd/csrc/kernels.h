// Kernel interfaces of the QG step (gfx950, FP64).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

namespace qg {

struct Geom {
  int M, K, R, nphi;
  double s_o, s_i, mid, half;   // s = half * x + mid
  double dtc_coef;              // dT_c/ds = dtc_coef / s
  double Ra_Pr, inv_Pr, two_over_E;
  const double* xk;             // Gauss-Lobatto nodes, x_0 = +1
  const double* wq;             // Clenshaw-Curtis weight * half * s_k
  const double* dsk;            // local radial spacing (CFL)
  const double2* tw_dct;        // plan twiddles, length 2 (R - 1) (fft.h layout)
  const double2* tw_phi;        // plan twiddles, length nphi
  const double2* tw_half;       // plan twiddles, length nphi / 2
  const double2* w_phi;         // exp(-2 pi i m / nphi), m <= nphi / 2
  const float2* tw_dct32;       // the same tables in FP32 (mixed precision)
  const float2* tw_phi32;
  const float2* tw_half32;
  const float2* w_phi32;
  // Runs stepped together (an ensemble of one size): every launch takes
  // the run as its grid y (band products: part of z).  Per-run arrays are
  // run-major with strides M K ([M][K] arrays), 2 M K (right-hand sides),
  // 6 M R and 2 M R (X, NL), R (zonal, rate) and 8 M (diag).  ra_pr: Ra/Pr
  // of each run (nullptr: Ra_Pr for all).
  int nmem;
  const double* ra_pr;
  // Ekman pumping (nullptr: none): per run [M][R], the synthesis writes
  // F_eps(Psi_m)(s_k) for m >= 1 and Upsilon_eps u (1 + (E/2) omega_0) at
  // m = 0; the analysis subtracts it from N_omega (adds it to the zonal
  // forcing).  Upsilon_eps = pump_ups / h_eps^{3/2}, h_eps^2 = pump_so2e - s^2.
  double2* pump;
  double pump_ups, pump_so2e, half_E;
  // Non-finite guard of a single run (nullptr: none).  The solves set it
  // to the step's tag when a new state holds NaN or Inf; while it is set,
  // every kernel of the step sequence returns at once, so that nothing
  // after the failing step overwrites the last finite state or history.
  int* nf;
  // Implicit buoyancy (Sect. 4): the analysis leaves C[(Ra/Pr)(i m/s_o)
  // theta] out of E_psi, the band products put it into Lin, and the solve
  // advances theta before Psi.
  int buoy_implicit;
  // Radial transforms as dense products on the FP64 matrix cores (nullptr:
  // FFT of the even extension).  dct_s [KP][RP]: T_n(x_k) = cos(pi n k / N)
  // for the synthesis (KP = K rounded up to 4, RP = R rounded up to 16);
  // dct_a [R4][K16]: the forward DCT-I weights (1/N)(1/2 at n = 0)(1 at
  // k = 0, N else 2) cos(pi n k / N) for the analysis (R4 = R rounded up to
  // 4, K16 = K rounded up to 16); zero outside n < K, k <= N.
  const double* dct_s;
  const double* dct_a;
};

// True when the non-finite guard is set: the kernel must return.
__device__ __forceinline__ bool nf_stop(const int* nf) {
  return nf && *reinterpret_cast<const volatile int*>(nf) != 0;
}

// Records a non-finite output (any lane of the wavefront) under `tag`.
__device__ __forceinline__ void nf_mark(int* nf, bool bad, int tag) {
  if (nf && __any(bad) && (threadIdx.x & 63) == 0) atomicCAS(nf, 0, tag);
}

struct Bands {  // [17][K] each (offset-major): entry (k, n) at [(n - k + 8) * K + k]
  const double *A0, *A2, *B0, *B2, *B4, *C, *D, *F0, *F2;
};

// Factors of all bordered systems of one kind.  With row interchanges
// (pivoted solve): piv, Lc, Uc in the host_ops.h layout, steps padded to
// whole 16-step batches.  Without (unpivoted solve): L, U, ui, steps padded
// to q rows (a multiple of solve_np_pad()).  W, Cb and Minv serve both.
template <typename TF>
struct FactorSet {
  const int* piv;     // [S][npad] row-interchange offsets
  const TF* Lc;       // [S][npad][kl]
  const TF* Uc;       // [S][npad][kut+1]  e=0: 1/U(j,j); e>=1: U(j-e, j)
  const TF* W;        // [S][p][n]
  const TF* Cb;       // [S][kl][p]
  const TF* Minv;     // [S][p][p]
  const TF* L;        // [S][q][kl]  multipliers of column j, rows j+1..j+kl
  const TF* U;        // [S][q][ku]  U(j-e, j) / U(j-e, j-e), e = 1..ku
  const TF* ui;       // [S][q]      1 / U(j, j)
  // Galerkin bases (unpivoted layout, no border): gamma_i^j of the Psi
  // stencil, [n][5] (nullptr with tau rows)
  const double* gam;
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
  int tag;                   // non-finite tag of this step (Geom::nf)
  double buoy_adt;           // implicit buoyancy: a dt of the solve (Psi gets
                             // a dt C[(Ra/Pr)(i m/s_o) theta_new]); else 0
};

// A linear combination of up to MAX_LEVELS arrays (multistep levels).
constexpr int MAX_LEVELS = 4;
struct Combine {
  int nb;
  const double2* in[MAX_LEVELS];
  double c[MAX_LEVELS];
};

// Transform kernels (transforms.hip), FP64 or, with `mixed`, FP32 for the
// transforms and products (exchange arrays X and NL in float2).  The
// launchers return false for a size without a compiled plan.
bool transform_sizes_ok(int n2, int nphi, bool mixed);
// Largest 2 (N_r - 1) with matrix-core radial transforms (FP64 only).
constexpr int MFMA_DCT_MAX_N2 = 512;
size_t mfma_dct_table_bytes(int R, int K, bool analysis);
void mfma_dct_tables(int R, int K, std::vector<double>& syn, std::vector<double>& ana);
size_t transform_lds_bytes(int n2, int nphi, int K, bool mixed);
std::vector<double2> plan_twiddles(int n);
bool launch_synth(const Geom& g, const double2* psi, const double2* th, void* X, double* diag,
                  bool mixed, hipStream_t st);
bool launch_ring(const Geom& g, const void* X, void* NL, double* zonal, double* rate, bool mixed,
                 hipStream_t st, double* G = nullptr);
bool launch_analysis(const Geom& g, const Bands& b, const void* NL, const double* zonal,
                     const double2* th_state, double2* Epsi, double2* Eth, bool mixed,
                     hipStream_t st);

}  // namespace qg
