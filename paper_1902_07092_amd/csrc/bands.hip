// Banded products of the implicit stage, FP64, gfx950:
//   out = (alpha Mass + cL Lin) y + sum_q coef_q slot_q     (rows k >= p)
// for every system: Psi (m >= 1, eq. psi_int: Mass = A_m, Lin = B_m), the
// zonal flow (eq. uphi_int: Mass = D, Lin = E) and theta (eq. temp_int:
// Mass = D, Lin = F_m / Pr).  alpha = 1 gives the right-hand side of an
// implicit solve (CNAB2, BPR353 stages); alpha = 0, cL = 1 the product
// Lin y of a new stage value (BPR353).  With implicit buoyancy (Sect. 4)
// Lin of Psi also carries C[(Ra/Pr)(i m/s_o) theta] (BUOY).
//
// The operators split in powers of m (A_m = A0 + m^2 A2, B_m = B0 + m^2 B2
// + m^4 B4 + (2/E) i m C, F_m = F0 + m^2 F2), so a thread keeps the
// m-independent combinations of its row's 17 band entries in registers and
// runs over a chunk of MCH systems: the bands are read once per (row,
// chunk) instead of once per system.  MCH trades band reuse against
// parallelism; it is chosen per context (4, 8, 16 or 32; qg_step_autotune
// times them).  Every output entry is computed by one thread in the same
// order whatever MCH is, so the results do not depend on it.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace qg {

namespace {

constexpr int BW = 17;    // band entries per row (offsets -8..8)
constexpr int RB = 64;    // rows per block

__device__ __forceinline__ double2 ld(const double2* p, int i, int K) {
  return (i >= 0 && i < K) ? p[i] : make_double2(0.0, 0.0);
}

}  // namespace

// blockIdx.x: rows [RB x, RB x + RB); blockIdx.y: chunk of MCH systems;
// blockIdx.z = 2 run + kind, kind 0 = Psi (m = 1 + MCH y + i), 1 = zonal
// flow and theta (u = MCH y + i: u = 0 the zonal flow, u >= 1 theta of
// m = u - 1).
// sys_out: out rows are system indices (Psi m -> m - 1, zonal -> M - 1,
// theta m -> M + m) in out_psi; else out_psi[m] (Psi, zonal at m = 0) and
// out_th[m].
template <int MCH, bool BUOY>
__global__ __launch_bounds__(64) void band_kernel(Geom g, Bands b, RhsSpec rs, double alpha,
                                                  double2* __restrict__ out_psi,
                                                  double2* __restrict__ out_th, int sys_out) {
  const int K = g.K, M = g.M;
  const int k = blockIdx.x * RB + threadIdx.x;
  const int kind = blockIdx.z & 1;
  const int u0 = blockIdx.y * MCH;
  if (k >= K || nf_stop(g.nf)) return;
  const double cL = rs.cL;
  const size_t mem = blockIdx.z >> 1, mk = (size_t)M * K;
  const size_t moff = mem * mk;
  out_psi += sys_out ? 2 * moff : moff;
  if (!sys_out) out_th += moff;
  if (kind == 0) {
    double P0[BW], P1[BW], P2[BW], P3[BW], PC[BUOY ? BW : 1];
#pragma unroll
    for (int o = 0; o < BW; ++o) {
      const size_t i = (size_t)o * K + k;
      P0[o] = alpha * b.A0[i] + cL * b.B0[i];
      P1[o] = alpha * b.A2[i] + cL * b.B2[i];
      P2[o] = cL * b.B4[i];
      P3[o] = cL * g.two_over_E * b.C[i];
      if constexpr (BUOY) PC[o] = cL * b.C[i];
    }
    const double ra_pr = g.ra_pr ? g.ra_pr[mem] : g.Ra_Pr;
    for (int i = 0; i < MCH; ++i) {
      const int m = 1 + u0 + i;
      if (m >= M) break;
      double2 acc = make_double2(0.0, 0.0);
      if (k >= 4) {
        const double dm = (double)m, m2 = dm * dm;
        const double2* y = rs.base_psi + moff + (size_t)m * K;
#pragma unroll
        for (int o = 0; o < BW; ++o) {
          const double re = P0[o] + m2 * (P1[o] + m2 * P2[o]);
          const double im = dm * P3[o];
          const double2 v = ld(y, k + o - 8, K);
          acc.x += re * v.x - im * v.y;
          acc.y += re * v.y + im * v.x;
        }
        if constexpr (BUOY) {   // cL C[(Ra/Pr)(i m/s_o) theta]
          const double2* th = rs.base_th + moff + (size_t)m * K;
          double2 cb = make_double2(0.0, 0.0);
#pragma unroll
          for (int o = 0; o < BW; ++o) {
            const double2 v = ld(th, k + o - 8, K);
            cb.x += PC[o] * v.x;
            cb.y += PC[o] * v.y;
          }
          const double gb = ra_pr * dm / g.s_o;
          acc.x -= gb * cb.y;
          acc.y += gb * cb.x;
        }
        for (int q = 0; q < rs.nterm; ++q) {
          const double2 v = rs.term_psi[q][moff + (size_t)m * K + k];
          acc.x += rs.coef[q] * v.x;
          acc.y += rs.coef[q] * v.y;
        }
      }
      double2* o = sys_out ? out_psi + (size_t)(m - 1) * K : out_psi + (size_t)m * K;
      o[k] = acc;
    }
  } else {
    double D[BW], F0[BW], F2[BW];
#pragma unroll
    for (int o = 0; o < BW; ++o) {
      const size_t i = (size_t)o * K + k;
      D[o] = alpha * b.D[i];
      F0[o] = b.F0[i];
      F2[o] = b.F2[i];
    }
    for (int i = 0; i < MCH; ++i) {
      const int u = u0 + i;
      if (u > M) break;
      const bool zonal = (u == 0);
      const int m = zonal ? 0 : u - 1;
      const double s1 = zonal ? cL : cL * g.inv_Pr;
      const double s2 = zonal ? cL : cL * g.inv_Pr * (double)m * (double)m;
      double2 acc = make_double2(0.0, 0.0);
      if (k >= 2) {
        const double2* y = (zonal ? rs.base_psi : rs.base_th) + moff + (size_t)m * K;
#pragma unroll
        for (int o = 0; o < BW; ++o) {
          const double re = D[o] + s1 * F0[o] + s2 * F2[o];
          const double2 v = ld(y, k + o - 8, K);
          acc.x += re * v.x;
          acc.y += re * v.y;
        }
        for (int q = 0; q < rs.nterm; ++q) {
          const double2 v = (zonal ? rs.term_psi[q] : rs.term_th[q])[moff + (size_t)m * K + k];
          acc.x += rs.coef[q] * v.x;
          acc.y += rs.coef[q] * v.y;
        }
      }
      double2* o = sys_out ? out_psi + (size_t)(zonal ? M - 1 : M + m) * K
                           : (zonal ? out_psi : out_th) + (size_t)m * K;
      o[k] = acc;
    }
  }
}

namespace {
dim3 band_grid(const Geom& g, int mch) {
  const int chunks = (g.M + 1 + mch - 1) / mch;   // covers M - 1 Psi and M + 1 real systems
  return dim3((g.K + RB - 1) / RB, chunks, 2 * g.nmem);
}

template <bool BUOY>
void launch_band_t(const Geom& g, const Bands& b, const RhsSpec& rs, double alpha, double2* o1,
                   double2* o2, int sys_out, int mch, hipStream_t st) {
  const dim3 grid = band_grid(g, mch);
  switch (mch) {
    case 4:
      hipLaunchKernelGGL((band_kernel<4, BUOY>), grid, dim3(RB), 0, st, g, b, rs, alpha, o1, o2,
                         sys_out);
      break;
    case 8:
      hipLaunchKernelGGL((band_kernel<8, BUOY>), grid, dim3(RB), 0, st, g, b, rs, alpha, o1, o2,
                         sys_out);
      break;
    case 32:
      hipLaunchKernelGGL((band_kernel<32, BUOY>), grid, dim3(RB), 0, st, g, b, rs, alpha, o1, o2,
                         sys_out);
      break;
    default:
      hipLaunchKernelGGL((band_kernel<16, BUOY>), grid, dim3(RB), 0, st, g, b, rs, alpha, o1, o2,
                         sys_out);
      break;
  }
}

void launch_band(const Geom& g, const Bands& b, const RhsSpec& rs, double alpha, double2* o1,
                 double2* o2, int sys_out, int mch, hipStream_t st) {
  if (g.buoy_implicit)
    launch_band_t<true>(g, b, rs, alpha, o1, o2, sys_out, mch, st);
  else
    launch_band_t<false>(g, b, rs, alpha, o1, o2, sys_out, mch, st);
}
}  // namespace

bool band_mch_ok(int mch) { return mch == 4 || mch == 8 || mch == 16 || mch == 32; }

// out = sum_{b < nb} c_b in_b over n complex entries: the combination of
// past states whose mass product a multistep right-hand side needs
// (M applied once to the combination instead of once per level).
__global__ __launch_bounds__(256) void combine_kernel(Combine cb, double2* __restrict__ out,
                                                      size_t n, const int* nf) {
  if (nf_stop(nf)) return;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double2 acc = make_double2(0.0, 0.0);
    for (int q = 0; q < cb.nb; ++q) {
      const double2 v = cb.in[q][i];
      acc.x += cb.c[q] * v.x;
      acc.y += cb.c[q] * v.y;
    }
    out[i] = acc;
  }
}

void launch_combine(const Combine& cb, double2* out, size_t n, const int* nf, hipStream_t st) {
  const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(combine_kernel, dim3((unsigned)std::max<size_t>(blocks, 1)), dim3(256), 0,
                     st, cb, out, n, nf);
}

// out = in over n complex entries (a stored multistep level), skipped
// while the non-finite guard is set.
__global__ __launch_bounds__(256) void copy_kernel(const double2* __restrict__ in,
                                                   double2* __restrict__ out, size_t n,
                                                   const int* nf) {
  if (nf_stop(nf)) return;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = in[i];
}

void launch_copy(const double2* in, double2* out, size_t n, const int* nf, hipStream_t st) {
  const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)std::max<size_t>(blocks, 1)), dim3(256), 0, st,
                     in, out, n, nf);
}

void launch_rhs(const Geom& g, const Bands& b, const RhsSpec& rs, double2* rhs, int mch,
                hipStream_t st) {
  launch_band(g, b, rs, 1.0, rhs, nullptr, 1, mch, st);
}

// rhs += sum_q coef_q term_q on the rows k >= p of every system (system
// layout of the band products' sys_out), with the same operations in the
// same order as band_kernel's term loop: a band product stored by
// band_kernel with no terms and completed here equals band_kernel with
// the terms, bit for bit.  blockIdx.y: system row (Psi m -> m - 1, zonal
// flow -> M - 1, theta m -> M + m), blockIdx.z: run.
__global__ __launch_bounds__(256) void rhs_terms_kernel(Geom g, RhsSpec rs,
                                                        double2* __restrict__ rhs) {
  const int K = g.K, M = g.M;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (k >= K || nf_stop(g.nf)) return;
  const size_t moff = (size_t)blockIdx.z * M * K;
  const bool psi_row = r < M - 1, zonal = r == M - 1;
  if (k < (psi_row ? 4 : 2)) return;
  const int m = psi_row ? r + 1 : (zonal ? 0 : r - M);
  const size_t src = moff + (size_t)m * K + k;
  double2* o = rhs + 2 * moff + (size_t)r * K + k;
  double2 acc = *o;
  for (int q = 0; q < rs.nterm; ++q) {
    const double2 v = (r < M ? rs.term_psi[q] : rs.term_th[q])[src];
    acc.x += rs.coef[q] * v.x;
    acc.y += rs.coef[q] * v.y;
  }
  *o = acc;
}

void launch_rhs_terms(const Geom& g, const RhsSpec& rs, double2* rhs, hipStream_t st) {
  const dim3 grid((g.K + 255) / 256, 2 * g.M, g.nmem);
  hipLaunchKernelGGL(rhs_terms_kernel, grid, dim3(256), 0, st, g, rs, rhs);
}

void launch_lin(const Geom& g, const Bands& b, const double2* ypsi, const double2* yth,
                double2* lpsi, double2* lth, int mch, hipStream_t st) {
  RhsSpec rs{};
  rs.base_psi = ypsi;
  rs.base_th = yth;
  rs.cL = 1.0;
  rs.nterm = 0;
  launch_band(g, b, rs, 0.0, lpsi, lth, 0, mch, st);
}

}  // namespace qg
