// Adjoint of the bordered solves of the implicit step (Appendix A), FP64,
// gfx950, with the stored factors of the unpivoted band LU.
//
// A bordered system S = [A B; C D] (p tau rows on top, D the band block,
// D = L U, W = B D^-1, Minv = (A - W C)^-1) is solved forward by the step.
// Its adjoint in the real inner product is S^-H (S^-T for the real
// systems):
//   z   = D^-H f_b = L^-H U^-H f_b     (a forward sweep with U^H, then a
//                                        backward sweep with L^H)
//   y_a = Minv^H (f_a - C^H z),   y_b = z - W^H y_a,
// since D^-H B^H = (B D^-1)^H = W^H.  With the tau-row zeroing of the
// right-hand side (its own adjoint) y_a is then set to zero, and theta at
// m = 0 takes real inputs (the adjoint of keeping theta_0 real).  One
// thread per system: this is the transposition of the step's solve for
// gradients, not a tuned kernel.  The band products of the step's
// right-hand side are transposed here as well.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace qg {

namespace {

__device__ __forceinline__ double2 cj_mul(double2 a, double2 b) {   // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cj_mul(double a, double2 b) { return make_double2(a * b.x, a * b.y); }
__device__ __forceinline__ double2 sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// x: the K entries of one system, f on entry, y = S^-H f (tau rows zeroed)
// on exit.  Factors of system s at the offsets of the step's solve.
template <typename TF, int P, int KL, int KU>
__device__ void solve_adjoint_one(const FactorSet<TF>& F, size_t s, int K, int q, double2* x) {
  const int n = K - P;
  const TF* L = F.L + s * q * KL;
  const TF* U = F.U + s * q * KU;
  const TF* ui = F.ui + s * q;
  const TF* W = F.W + s * P * n;
  const TF* Cb = F.Cb + s * KL * P;
  const TF* Mi = F.Minv + s * P * P;
  double2* fb = x + P;
  // U^H r = f_b with U = diag(U_jj) Uhat: Uhat^H r' = f_b, then r = r' conj(1/U_jj)
  for (int j = 0; j < n; ++j) {
    double2 acc = fb[j];
    for (int e = 1; e <= KU; ++e)
      if (j - e >= 0) acc = sub(acc, cj_mul(U[(size_t)j * KU + (e - 1)], fb[j - e]));
    fb[j] = acc;
  }
  for (int j = 0; j < n; ++j) fb[j] = cj_mul(ui[j], fb[j]);
  // L^H z = r (L unit lower, multipliers of column j in rows j+1..j+KL)
  for (int j = n - 1; j >= 0; --j) {
    double2 acc = fb[j];
    for (int d = 0; d < KL; ++d)
      if (j + 1 + d < n) acc = sub(acc, cj_mul(L[(size_t)j * KL + d], fb[j + 1 + d]));
    fb[j] = acc;
  }
  double2 t[P], ya[P];
  for (int c = 0; c < P; ++c) {
    double2 acc = x[c];
    for (int r = 0; r < KL && r < n; ++r) acc = sub(acc, cj_mul(Cb[r * P + c], fb[r]));
    t[c] = acc;
  }
  for (int i = 0; i < P; ++i) {
    double2 acc = make_double2(0.0, 0.0);
    for (int c = 0; c < P; ++c) acc = add(acc, cj_mul(Mi[c * P + i], t[c]));
    ya[i] = acc;
  }
  for (int j = 0; j < n; ++j) {
    double2 acc = fb[j];
    for (int i = 0; i < P; ++i) acc = sub(acc, cj_mul(W[(size_t)i * n + j], ya[i]));
    fb[j] = acc;
  }
  for (int i = 0; i < P; ++i) x[i] = make_double2(0.0, 0.0);
}

// Systems: Psi of m = 1..M-1 (rows 1..M-1 of psi), then the real systems:
// the zonal flow (row 0 of psi) and theta of m = 0..M-1.
__global__ __launch_bounds__(64) void solve_adjoint_kernel(FactorSet<double2> Fp,
                                                           FactorSet<double> Fr, int M, int K,
                                                           int q4, int q2, double2* psi,
                                                           double2* th) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < M - 1) {
    solve_adjoint_one<double2, 4, 8, 8>(Fp, (size_t)idx, K, q4, psi + (size_t)(idx + 1) * K);
  } else if (idx < 2 * M) {
    const int s = idx - (M - 1);   // 0: zonal flow, 1 + m: theta of m
    double2* x = (s == 0) ? psi : th + (size_t)(s - 1) * K;
    if (s <= 1)                     // real inputs: the zonal flow, theta at m = 0
      for (int k = 0; k < K; ++k) x[k].y = 0.0;
    solve_adjoint_one<double, 2, 4, 4>(Fr, (size_t)s, K, q2, x);
  }
}

// out = (Mass + c Lin)^H mu per system, column n of the band operators
// (entry (k, n) at [(n - k + 8) K + k], rows k >= p: the tau rows of mu are
// zero): Psi (A_m + c B_m, with the Coriolis part (2/E) i m C conjugated),
// the zonal flow (D + c E, E = F at m = 1) and theta (D + c F_m / Pr).
// blockIdx.y: 0..M-2 Psi of m = y + 1, M-1 the zonal flow, M + m theta.
__global__ __launch_bounds__(64) void band_adjoint_kernel(Geom g, Bands b, double c,
                                                          const double2* __restrict__ mu_psi,
                                                          const double2* __restrict__ mu_th,
                                                          double2* __restrict__ out_psi,
                                                          double2* __restrict__ out_th) {
  const int K = g.K, M = g.M;
  const int n = blockIdx.x * 64 + threadIdx.x;
  const int sys = blockIdx.y;
  if (n >= K) return;
  double2 acc = make_double2(0.0, 0.0);
  if (sys < M - 1) {
    const int m = sys + 1;
    const double dm = (double)m, m2 = dm * dm;
    const double2* mu = mu_psi + (size_t)m * K;
    for (int o = 0; o < 17; ++o) {
      const int k = n - o + 8;
      if (k < 4 || k >= K) continue;
      const size_t i = (size_t)o * K + k;
      const double re = b.A0[i] + m2 * b.A2[i] + c * (b.B0[i] + m2 * (b.B2[i] + m2 * b.B4[i]));
      const double im = c * g.two_over_E * dm * b.C[i];
      const double2 v = mu[k];
      acc.x += re * v.x + im * v.y;
      acc.y += re * v.y - im * v.x;
    }
    out_psi[(size_t)m * K + n] = acc;
  } else {
    const bool zonal = (sys == M - 1);
    const int m = zonal ? 0 : sys - M;
    const double s1 = zonal ? c : c * g.inv_Pr;
    const double s2 = zonal ? c : c * g.inv_Pr * (double)m * (double)m;
    const double2* mu = zonal ? mu_psi : mu_th + (size_t)m * K;
    for (int o = 0; o < 17; ++o) {
      const int k = n - o + 8;
      if (k < 2 || k >= K) continue;
      const size_t i = (size_t)o * K + k;
      const double re = b.D[i] + s1 * b.F0[i] + s2 * b.F2[i];
      acc.x += re * mu[k].x;
      acc.y += re * mu[k].y;
    }
    (zonal ? out_psi : out_th + (size_t)m * K)[n] = acc;
  }
}

}  // namespace

void launch_band_adjoint(const Geom& g, const Bands& b, double c, const double2* mu_psi,
                         const double2* mu_th, double2* out_psi, double2* out_th, hipStream_t st) {
  hipLaunchKernelGGL(band_adjoint_kernel, dim3((g.K + 63) / 64, 2 * g.M), dim3(64), 0, st, g, b,
                     c, mu_psi, mu_th, out_psi, out_th);
}

void launch_solve_adjoint(const Geom& g, const FactorSet<double2>& Fp, const FactorSet<double>& Fr,
                          int q4, int q2, double2* psi, double2* th, hipStream_t st) {
  const int systems = (g.M - 1) + (g.M + 1);
  hipLaunchKernelGGL(solve_adjoint_kernel, dim3((systems + 63) / 64), dim3(64), 0, st, Fp, Fr,
                     g.M, g.K, q4, q2, psi, th);
}

}  // namespace qg
