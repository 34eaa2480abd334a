// Reverse mode of the explicit terms of the QG step (FP64, gfx950): the
// adjoint of the map y -> E(y) = (E_psi, E_theta, E_u) of eq. psi_int,
// temp_int and uphi_int, linearised about a state y, applied to a co-state
// (Ebar_psi, Ebar_theta, Ebar_u), plus kappa times the gradient of the
// kinetic energy E_K(y) (Sect. 6.2).  The forward map is
//   synth (per m)  -> X[6][k][m]  -> ring (per s_k) -> NL[2][m][k], zonal[k]
//                  -> analysis (per m) -> E,
// and its transpose runs backwards through three kernels of the same
// shapes:
//   analysis_T_kernel  per m:   transposed band products C^T and -D^T and
//                               the transposed forward DCT-I (eq. icheb)
//   ring_T_kernel      per s_k: the products' co-state on the grid, the
//                               products linearised about the forward
//                               fields (recomputed from X), the transposed
//                               inverse real FFTs (eq. fft), the zonal
//                               forcing and the energy gradient
//   synth_T_kernel     per m:   transposed field assembly, transposed
//                               inverse DCT-I (eq. cheb) and transposed
//                               Chebyshev derivative recurrences (Horner)
//
// Inner product: real, sum Re(conj(a) b) over every complex entry; the
// co-state of a complex entry z is dJ/dRe z + i dJ/dIm z, so a complex-
// linear map A has the adjoint A^H.  The Ekman pumping terms and the FP32
// transforms have no reverse mode here.
#include <hip/hip_runtime.h>

#include "fft.h"
#include "kernels.h"
#include "transform_util.h"

namespace qg {

namespace {

__device__ __forceinline__ double2 shfl_up2(double2 v, int off) {
  return make_double2(__shfl_up(v.x, off), __shfl_up(v.y, off));
}

// In-place transpose of the Chebyshev derivative d/ds (cheb_deriv_inplace):
// that map is b_n = w_n sum_{j > n, j - n odd} j a_j with w_0 = 2, else 4,
// so its transpose is a'_j = j sum_{n < j, j - n odd} w_n b_n: prefix sums
// of the weighted entries of opposite parity.  Each thread takes a run of
// (even, odd) pairs; the sums over earlier threads come from a wavefront
// scan and one LDS exchange.  Ends with a barrier.
template <int T>
__device__ void cheb_deriv_T_inplace(double2* c, int K, double2* wred) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int npair = (K + 1) / 2;
  const int ch = (npair + T - 1) / T;
  const int p0 = min(npair, t * ch), p1 = min(npair, p0 + ch);
  double2 se = z2(), so = z2();
  for (int p = p0; p < p1; ++p) {
    const int je = 2 * p, jo = je + 1;
    se = add2(se, scl2(je == 0 ? 2.0 : 4.0, c[je]));
    if (jo < K) so = add2(so, scl2(4.0, c[jo]));
  }
  // inclusive scan over the lanes, then shifted by one lane (exclusive)
  double2 ie = se, io = so;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double2 ue = shfl_up2(ie, off), uo = shfl_up2(io, off);
    if (lane >= off) {
      ie = add2(ie, ue);
      io = add2(io, uo);
    }
  }
  double2 re = shfl_up2(ie, 1), ro = shfl_up2(io, 1);
  if (lane == 0) re = ro = z2();
  if (lane == 63) {
    wred[2 * w] = ie;
    wred[2 * w + 1] = io;
  }
  __syncthreads();
  for (int w2 = 0; w2 < w; ++w2) {
    re = add2(re, wred[2 * w2]);
    ro = add2(ro, wred[2 * w2 + 1]);
  }
  for (int p = p0; p < p1; ++p) {
    const int je = 2 * p, jo = je + 1;
    const double2 be = c[je];
    const double2 bo = (jo < K) ? c[jo] : z2();
    c[je] = scl2((double)je, ro);            // sum over odd n < je
    re = add2(re, scl2(je == 0 ? 2.0 : 4.0, be));
    if (jo < K) c[jo] = scl2((double)jo, re);   // sum over even n < jo
    ro = add2(ro, scl2(4.0, bo));
  }
  __syncthreads();
}

}  // namespace

// ------------------------------------------------------------ analysis_T
// Forward (analysis_kernel): c = DCT(NL_f row), c_n = (h_n / N) FFT(e)_n
// with the even extension e of the N + 1 grid values, h_0 = 1/2, else 1;
// then E_psi = C (c + i (Ra/Pr)(m/s_o) theta) on rows k >= 4 (m >= 1),
// E_u = -D c on rows k >= 2 (m = 0, c from the zonal forcing) and
// E_theta = -D c on rows k >= 2.  Transposed: cbar = C^T Ebar (or -D^T Ebar),
// thetabar = -i (Ra/Pr)(m/s_o) cbar, and the grid co-state
//   fbar_k = (eps_k / N) sum_n h_n cbar_n cos(pi n k / N),
// eps_0 = eps_N = 1, else 2 (the even extension counts interior points
// twice) -- an inverse DCT-I of cbar / 2 (e_0 = b_0, e_n = b_n / 2 with
// b_0 = cbar_0 / 2, b_n = cbar_n).  With mu, the same band loop also gives
// ml = (Mass + cmu Lin)^H mu, the transposed band products of a step's
// right-hand side (Sect. 4 eq. multistep1; rows below the tau rows, which
// the transposed solve leaves zero).
template <int N2, int T>
__global__ __launch_bounds__(T) void analysis_T_kernel(Geom g, Bands b,
                                                       const double2* __restrict__ Ea,
                                                       const double2* __restrict__ Eb2,
                                                       double ca, double cb,
                                                       const double2* __restrict__ mu,
                                                       double cmu, size_t mk,
                                                       double2* __restrict__ NLb,
                                                       double* __restrict__ zb,
                                                       double2* __restrict__ thb,
                                                       double2* __restrict__ ml, int split) {
  extern __shared__ double2 sm[];
  constexpr int N = N2 / 2;
  constexpr int E = out_count<N2, T>();
  const int K = g.K, R = g.R, M = g.M;
  const int t = threadIdx.x;
  // split: blocks [0, B) take field 0 of their m, blocks [B, 2B) field 1
  // (B = 8 ceil(M / 8)); otherwise one block takes both
  int only = -1, bid = blockIdx.x;
  if (split) {
    const int B = 8 * ((M + 7) >> 3);
    only = bid < B ? 0 : 1;
    if (bid >= B) bid -= B;
  }
  const int m = xcd_index_of(bid, M);
  if (m >= M || nf_stop(g.nf)) return;
  double2* fb = sm;
  double2* c = reinterpret_cast<double2*>(reinterpret_cast<char*>(sm) +
                                          coef_offset<double2>(lds_slots(N2)));
  // the co-state rows of E (e) and of the right-hand side (u) sit in the
  // transform buffer until the transform (2 K <= N2 slots)
  double2* e = fb;
  double2* u = fb + K;
  const double invN = 1.0 / N;
  const double dm = (double)m, m2 = dm * dm;
  const double bcoef = g.Ra_Pr * dm / g.s_o;
#pragma unroll 1
  for (int f = 0; f < 2; ++f) {
    if (only >= 0 && f != only) continue;
    // co-state of E: ca Ea + cb Eb2 (Eb2 optional; Ea null: zero)
    const size_t off = (size_t)f * mk + (size_t)m * K;
    for (int k = t; k < K; k += T) {
      double2 v = Ea ? scl2(ca, Ea[off + k]) : z2();
      if (Eb2) v = add2(v, scl2(cb, Eb2[off + k]));
      e[k] = v;
      if (mu) u[k] = mu[off + k];
    }
    __syncthreads();
    const bool cband = (f == 0 && m > 0);
    // real systems: zonal flow D + c E (E = F at m = 1), theta D + (c/Pr) F_m
    const double s1 = (f == 0) ? cmu : cmu * g.inv_Pr;
    const double s2 = (f == 0) ? cmu : cmu * g.inv_Pr * m2;
    for (int n = t; n < K; n += T) {
      double2 acc = z2(), mv = z2();
#pragma unroll
      for (int o = 0; o < 17; ++o) {
        const int k = n - o + 8;   // entry (k, n) of the band at [o][k]
        const size_t i = (size_t)o * K + k;
        if (cband) {
          if (k >= 4 && k < K) {
            acc = add2(acc, scl2(b.C[i], e[k]));
            if (mu) {   // (A_m + c B_m)^H, Coriolis part (2/E) i m C conjugated
              const double re = b.A0[i] + m2 * b.A2[i] +
                                cmu * (b.B0[i] + m2 * (b.B2[i] + m2 * b.B4[i]));
              const double im = cmu * g.two_over_E * dm * b.C[i];
              const double2 v = u[k];
              mv.x += re * v.x + im * v.y;
              mv.y += re * v.y - im * v.x;
            }
          }
        } else {
          if (k >= 2 && k < K) {
            acc = sub2(acc, scl2(b.D[i], e[k]));
            if (mu) mv = add2(mv, scl2(b.D[i] + s1 * b.F0[i] + s2 * b.F2[i], u[k]));
          }
        }
      }
      c[n] = acc;
      if (f == 0) thb[(size_t)m * K + n] = cband ? make_double2(bcoef * acc.y, -bcoef * acc.x) : z2();
      if (mu) ml[off + n] = mv;
    }
    __syncthreads();
    auto ext = [&](int i) -> double2 {
      const int nn = (i <= N) ? i : N2 - i;
      return nn < K ? scl2(0.5, c[nn]) : z2();
    };
    double2 o[E];
    fft_out<N2, T, -1>(ext, fb, g.tw_dct, o);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int k = t + i * T;
      if (k > N) continue;
      const double2 v = scl2(((k == 0 || k == N) ? 1.0 : 2.0) * invN, o[i]);
      if (f == 0 && m == 0) {   // the zonal forcing replaced N_omega's m = 0 row
        zb[k] = v.x;
        NLb[k] = z2();
      } else {
        NLb[((size_t)f * M + m) * R + k] = v;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- ring_T
// Forward (ring_kernel) at s_k: real grid fields g_f(phi) = X_f,0 +
// 2 Re sum_{m >= 1} X_f,m e^{i m phi} (real part of X_f,0), the products
//   N_omega = g0 g2 + g1 g3,   N_theta = g0 g4 + g1 g5,
// NL_f,m = (1/N_phi) sum_j N_f(phi_j) e^{-i m phi_j} for m < M (m = 0 real),
// and zonal = 2 (h^2/s) sum_{m >= 1} Im(conj(X0_m) X3_m) / m.
// Transposed: Nbar_f(phi_j) = (1/N_phi) sum_m Re(NLbar_f,m e^{i m phi_j})
// (a real synthesis of the half spectrum Re NLbar_0, NLbar_m / 2), the
// product co-states
//   gbar0 = Nw g2 + Nt g4, gbar1 = Nw g3 + Nt g5, gbar2 = Nw g0,
//   gbar3 = Nw g1,         gbar4 = Nt g0,         gbar5 = Nt g1,
// Xbar_f,m = 2 sum_j gbar_f(phi_j) e^{-i m phi_j} (m >= 1), sum_j gbar_f
// (m = 0, real), and from the zonal forcing (co-state zb)
//   Xbar0_m += -2 i (h^2/s) zb X3_m / m,  Xbar3_m += 2 i (h^2/s) zb X0_m / m.
// The energy E_K = pi sum_k wq_k sum_m c_m ((h^2/s)^2 |X0_m|^2 + s^2 |X1_m|^2)
// (c_0 = 1 with the real zonal part, else 2) adds kappa times its gradient
// to Xbar0 and Xbar1.  Two real fields share each complex FFT.
template <int NPHI, int T>
__global__ __launch_bounds__(T) void ring_T_kernel(Geom g, const double2* __restrict__ X,
                                                   const double* __restrict__ G,
                                                   const double2* __restrict__ NLb,
                                                   const double* __restrict__ zb, double kappa,
                                                   double2* __restrict__ Xb) {
  extern __shared__ double2 sm[];
  double2* fb = sm;
  constexpr int E = out_count<NPHI, T>();
  const int R = g.R, M = g.M;
  const int t = threadIdx.x;
  const int k = xcd_index(R);
  if (k >= R || nf_stop(g.nf)) return;
  const double s = g.half * g.xk[k] + g.mid;
  const double h2s = (g.s_o * g.s_o - s * s) / s;
  // products' co-state on the grid: N_omega in the real part, N_theta in
  // the imaginary part of one complex synthesis
  double nbw[E], nbt[E];
  {
    auto half = [&](int f, int mm) -> double2 {
      const double2 v = NLb[((size_t)f * M + mm) * R + k];
      return mm == 0 ? make_double2(v.x, 0.0) : scl2(0.5, v);
    };
    auto get = [&](int i) -> double2 {
      if (i < M) {
        const double2 a = half(0, i), b = half(1, i);
        return (i == 0) ? make_double2(a.x, b.x) : make_double2(a.x - b.y, a.y + b.x);
      }
      if (i > NPHI - M) {
        const double2 a = half(0, NPHI - i), b = half(1, NPHI - i);
        return make_double2(a.x + b.y, b.x - a.y);
      }
      return z2();
    };
    double2 z[E];
    fft_out<NPHI, T, +1>(get, fb, g.tw_phi, z);
    const double inv = 1.0 / NPHI;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      nbw[i] = z[i].x * inv;
      nbt[i] = z[i].y * inv;
    }
  }
  // forward grid fields: stored by the forward ring (G), else three
  // complex syntheses of two fields each
  double gf[6][E];
  if (G) {
#pragma unroll
    for (int f = 0; f < 6; ++f)
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int j = t + i * T;
        gf[f][i] = (j < NPHI) ? G[((size_t)f * R + k) * NPHI + j] : 0.0;
      }
  } else {
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double2* A = X + ((size_t)(2 * q) * R + k) * M;
    const double2* B = X + ((size_t)(2 * q + 1) * R + k) * M;
    auto get = [&](int i) -> double2 {
      if (i < M) {
        const double2 a = A[i], b = B[i];
        return (i == 0) ? make_double2(a.x, b.x) : make_double2(a.x - b.y, a.y + b.x);
      }
      if (i > NPHI - M) {
        const double2 a = A[NPHI - i], b = B[NPHI - i];
        return make_double2(a.x + b.y, b.x - a.y);
      }
      return z2();
    };
    double2 z[E];
    fft_out<NPHI, T, +1>(get, fb, g.tw_phi, z);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      gf[2 * q][i] = z[i].x;
      gf[2 * q + 1][i] = z[i].y;
    }
  }
  }
  const double ek = kappa * 2.0 * 3.14159265358979323846 * g.wq[k];
  const double zk = 2.0 * h2s * zb[k];
  const double2* X0 = X + (size_t)k * M;
  const double2* X1 = X + ((size_t)R + k) * M;
  const double2* X3 = X + ((size_t)3 * R + k) * M;
#pragma unroll 1
  for (int p = 0; p < 3; ++p) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int j = t + i * T;
      if (j >= NPHI) continue;
      double a, b;
      if (p == 0) {
        a = nbw[i] * gf[2][i] + nbt[i] * gf[4][i];
        b = nbw[i] * gf[3][i] + nbt[i] * gf[5][i];
      } else if (p == 1) {
        a = nbw[i] * gf[0][i];
        b = nbw[i] * gf[1][i];
      } else {
        a = nbt[i] * gf[0][i];
        b = nbt[i] * gf[1][i];
      }
      fb[j] = make_double2(a, b);
    }
    __syncthreads();
    fft_to_lds<NPHI, T, -1>([&](int ii) { return fb[ii]; }, fb, g.tw_phi);
    for (int m = t; m < M; m += T) {
      const double2 Zm = fb[lds_pad(m)];
      double2 Zc = fb[lds_pad((NPHI - m) % NPHI)];
      Zc.y = -Zc.y;
      double2 A = scl2(0.5, add2(Zm, Zc));
      const double2 dd = sub2(Zm, Zc);
      double2 B = make_double2(0.5 * dd.y, -0.5 * dd.x);
      if (m == 0) {
        A.y = 0.0;
        B.y = 0.0;
      } else {
        A = scl2(2.0, A);
        B = scl2(2.0, B);
      }
      const double im = m > 0 ? 1.0 / (double)m : 0.0;
      if (p == 0) {
        if (m > 0) {
          A = add2(A, ix(-zk * im, X3[m]));                    // -2 i (h^2/s) zb X3 / m
          A = add2(A, scl2(2.0 * ek * h2s * h2s, X0[m]));
          B = add2(B, scl2(2.0 * ek * s * s, X1[m]));
        } else {
          B.x += ek * s * s * X1[0].x;
        }
      } else if (p == 1 && m > 0) {
        B = add2(B, ix(zk * im, X0[m]));                       // 2 i (h^2/s) zb X0 / m
      }
      Xb[((size_t)(2 * p) * R + k) * M + m] = A;
      Xb[((size_t)(2 * p + 1) * R + k) * M + m] = B;
    }
  }
}

// --------------------------------------------------------------- synth_T
// Forward (synth_kernel), with P_d the d-th s-derivative of Psi_m on the
// grid (inverse DCT-I of D^d psi_m), h2 = s_o^2 - s^2, h2s = h2 / s,
// mh = m^2 h2 / s^2:
//   X0 = i m P0,  X1 = 3 P0 - h2s P1,
//   omega = (6 + mh) P0 - (h2s - 5 s) P1 - h2 P2,  X3 = i m omega,
//   X2 = a0 P0 + a1 P1 + a2 P2 + a3 P3 with
//        a0 = 6 + mh - 2 m^2 s_o^2 h2s / s^3,
//        a1 = 5 s - h2s + h2s (s_o^2 / s^2 + 12 + mh),
//        a2 = -(h2 + h2s (h2s - 7 s)),  a3 = -h2s h2;
//   m = 0 (zonal flow u, P_d its derivatives): X1 = P0 / s,
//        X2 = (1/s - h2s/s^2) P0 + (1 + h2s/s) P1 + h2s P2;
//   theta: X5 = i m T0, X4 = h2s (T1 + dTc/ds at m = 0).
// Transposed: Pbar_d = sum_f conj(coefficient) Xbar_f pointwise; the
// transposed inverse DCT-I S_n = sum_{k=0}^{N} Pbar(k) cos(pi n k / N) is an
// FFT of the even extension with half weight at the interior points; and
// psibar = S_0 + D^T (S_1 + D^T (S_2 + D^T S_3)) (Horner).  thetabar adds
// the buoyancy co-state of analysis_T.
template <int N2, int T>
__global__ __launch_bounds__(T) void synth_T_kernel(Geom g, const double2* __restrict__ Xb,
                                                    const double2* __restrict__ thb0,
                                                    const double2* __restrict__ add,
                                                    size_t mk, double2* __restrict__ psib,
                                                    double2* __restrict__ thb, int split) {
  extern __shared__ double2 sm[];
  __shared__ double2 wred[2 * (T / 64)];
  constexpr int N = N2 / 2;
  constexpr int E = out_count<N2, T>();
  const int K = g.K, R = g.R, M = g.M;
  const int t = threadIdx.x;
  // split: blocks [0, B) take Psi (or the zonal flow) of their m, blocks
  // [B, 2B) theta (B = 8 ceil(M / 8)); otherwise one block takes both
  int only = -1, bid = blockIdx.x;
  if (split) {
    const int B = 8 * ((M + 7) >> 3);
    only = bid < B ? 0 : 1;
    if (bid >= B) bid -= B;
  }
  const int m = xcd_index_of(bid, M);
  if (m >= M || nf_stop(g.nf)) return;
  double2* fb = sm;
  double2* acc = reinterpret_cast<double2*>(reinterpret_cast<char*>(sm) +
                                            coef_offset<double2>(lds_slots(N2)));
  const double dm = (double)m, m2 = dm * dm, so2 = g.s_o * g.s_o;
  auto xb = [&](int f, int kk) { return Xb[((size_t)f * R + kk) * M + m]; };
  // co-state of derivative d of field fld (0: Psi or the zonal flow, 1:
  // theta) at radial point kk
  auto pbar = [&](int fld, int d, int kk) -> double2 {
    const double s = g.half * g.xk[kk] + g.mid;
    const double is = 1.0 / s, h2 = so2 - s * s, h2s = h2 * is;
    if (fld == 1) {
      if (d == 1) return scl2(h2s, xb(4, kk));
      return m > 0 ? ix(-dm, xb(5, kk)) : z2();
    }
    const double2 x2 = xb(2, kk);
    if (m == 0) {
      if (d == 0) return add2(scl2(is, xb(1, kk)), scl2(is - h2s * is * is, x2));
      if (d == 1) return scl2(1.0 + h2s * is, x2);
      return scl2(h2s, x2);
    }
    const double mh = m2 * h2 * is * is;
    const double2 wb = ix(-dm, xb(3, kk));   // co-state of omega
    if (d == 0) {
      const double a0 = 6.0 + mh - h2s * 2.0 * m2 * so2 * is * is * is;
      return add2(add2(ix(-dm, xb(0, kk)), scl2(3.0, xb(1, kk))),
                  add2(scl2(6.0 + mh, wb), scl2(a0, x2)));
    }
    if (d == 1) {
      const double a1 = -(h2s - 5.0 * s) + h2s * (so2 * is * is + 12.0 + mh);
      return add2(add2(scl2(-h2s, xb(1, kk)), scl2(-(h2s - 5.0 * s), wb)), scl2(a1, x2));
    }
    if (d == 2) return add2(scl2(-h2, wb), scl2(-(h2 + h2s * (h2s - 7.0 * s)), x2));
    return scl2(-h2s * h2, x2);
  };
#pragma unroll 1
  for (int fld = 0; fld < 2; ++fld) {
    if (only >= 0 && fld != only) continue;
    const int nd = fld == 1 ? 2 : (m > 0 ? 4 : 3);
#pragma unroll 1
    for (int d = nd - 1; d >= 0; --d) {
      if (d < nd - 1) cheb_deriv_T_inplace<T>(acc, K, wred);
      auto get = [&](int i) -> double2 {
        const int kk = (i <= N) ? i : N2 - i;
        return scl2((kk == 0 || kk == N) ? 1.0 : 0.5, pbar(fld, d, kk));
      };
      double2 o[E];
      fft_out<N2, T, -1>(get, fb, g.tw_dct, o);
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int n = t + i * T;
        if (n < K) acc[n] = (d == nd - 1) ? o[i] : add2(acc[n], o[i]);
      }
      __syncthreads();
    }
    for (int n = t; n < K; n += T) {
      const size_t i = (size_t)m * K + n;
      double2 v = (fld == 0) ? ((m == 0) ? make_double2(acc[n].x, 0.0) : acc[n])
                             : add2(acc[n], thb0[i]);
      if (add) v = add2(v, add[(size_t)fld * mk + i]);
      (fld == 0 ? psib : thb)[i] = v;
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------- helpers
namespace {

// J = c sum_{n=0}^{N} w_n sum_m diag[n][8 m] (kinetic energies of the
// syntheses of y^0 .. y^N), w_n = 1/2 at both ends, else 1.
__global__ __launch_bounds__(256) void energy_total_kernel(const double* __restrict__ diag, int M,
                                                           int N, double c,
                                                           double* __restrict__ J) {
  __shared__ double red[4];
  double v = 0.0;
  for (int n = 0; n <= N; ++n) {
    double e = 0.0;
    for (int m = threadIdx.x; m < M; m += 256) e += diag[((size_t)n * M + m) * 8];
    v += (n == 0 || n == N) ? 0.5 * e : e;
  }
  const double tot = block_sum(v, red);
  if (threadIdx.x == 0) *J = c * tot;
}

// Co-state layouts: the library's arrays keep the zonal flow in row 0 of
// the Psi array (as a real entry); the C ABI has Psi with its row 0 and
// the zonal flow separate.
__global__ void to_internal_kernel(int M, int K, const double2* __restrict__ psi,
                                   const double2* __restrict__ th,
                                   const double* __restrict__ u, double2* __restrict__ dp,
                                   double2* __restrict__ dt) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t MK = (size_t)M * K;
  if (i >= MK) return;
  dp[i] = (i < (size_t)K) ? make_double2(u ? u[i] : 0.0, 0.0) : (psi ? psi[i] : z2());
  dt[i] = th ? th[i] : z2();
}

__global__ void to_api_kernel(int M, int K, const double2* __restrict__ sp,
                              const double2* __restrict__ st, double2* __restrict__ psi,
                              double2* __restrict__ th, double* __restrict__ u) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t MK = (size_t)M * K;
  if (i >= MK) return;
  if (i < (size_t)K) {
    psi[i] = z2();
    u[i] = sp[i].x;
  } else {
    psi[i] = sp[i];
  }
  th[i] = st[i];
}

// Threads per block of the reverse kernels: twice the forward kernels'
// (capped at 256); the reverse kernels carry more work per block.
constexpr int threads_rdct(int n2) { return clampi(n2 / 4, 64, 256); }
constexpr int threads_rphi(int nphi) { return clampi(nphi / 6, 64, 256); }

template <int N2>
void analysis_T_n(const Geom& g, const Bands& b, const double2* Ea, const double2* Eb,
                  double ca, double cb, const double2* mu, double cmu, size_t mk,
                  double2* NLb, double* zb, double2* thb, double2* ml, hipStream_t st) {
  constexpr int T = threads_rdct(N2);
  const size_t shm = dct_lds<double2>(N2, g.K);
  allow_lds(analysis_T_kernel<N2, T>, shm);
  hipLaunchKernelGGL((analysis_T_kernel<N2, T>), dim3(2 * xcd_grid(g.M)), dim3(T), shm, st, g, b,
                     Ea, Eb, ca, cb, mu, cmu, mk, NLb, zb, thb, ml, 1);
}

template <int NPHI>
void ring_T_n(const Geom& g, const double2* X, const double* G, const double2* NLb,
              const double* zb, double kappa, double2* Xb, hipStream_t st) {
  constexpr int T = threads_rphi(NPHI);
  const size_t shm = phi_lds<double2>(NPHI);
  allow_lds(ring_T_kernel<NPHI, T>, shm);
  hipLaunchKernelGGL((ring_T_kernel<NPHI, T>), dim3(xcd_grid(g.R)), dim3(T), shm, st, g, X, G,
                     NLb, zb, kappa, Xb);
}

template <int N2>
void synth_T_n(const Geom& g, const double2* Xb, const double2* thb0, const double2* add,
               size_t mk, double2* psib, double2* thb, hipStream_t st) {
  constexpr int T = threads_rdct(N2);
  const size_t shm = dct_lds<double2>(N2, g.K);
  allow_lds(synth_T_kernel<N2, T>, shm);
  hipLaunchKernelGGL((synth_T_kernel<N2, T>), dim3(2 * xcd_grid(g.M)), dim3(T), shm, st, g, Xb,
                     thb0, add, mk, psib, thb, 1);
}

#define QG_RDCT(X) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) \
  X(1024) X(1536) X(2048) X(3072) X(4096) X(6144)
#define QG_RPHI(X) X(24) X(48) X(96) X(192) X(384) X(768) X(1536) X(3072) X(6144)

}  // namespace

// The transposed explicit terms at the state whose forward fields X the
// caller has synthesised (launch_synth, FP64; G: its grid fields from the
// forward ring, or null):
//   (psib, thb) = E'(y)^H (ca Ea + cb Eb) + kappa grad E_K(y)
//                 + (Mass + cmu Lin)^H mu  (with mu)  or  + add  (without),
// co-state pairs (Psi block, theta block mk entries later); Ea, Eb, add
// and mu may be null (zero).  NLb [2][M][R], zb [R], thb0 [M][K], ml (a
// pair) and Xb [6][R][M] are scratch.  False: no kernel for these sizes.
bool launch_explicit_T(const Geom& g, const Bands& b, const double2* X, const double* G,
                       const double2* Ea, const double2* Eb, double ca, double cb, size_t mk,
                       double kappa, double2* NLb, double* zb, double2* thb0, double2* Xb,
                       const double2* add, const double2* mu, double cmu, double2* ml,
                       double2* psib, double2* thb, hipStream_t st) {
  const int n2 = 2 * (g.R - 1);
  bool ok = false;
  if (mu) add = ml;
  switch (n2) {
#define QG_CASE(n) case n: analysis_T_n<n>(g, b, Ea, Eb, ca, cb, mu, cmu, mk, NLb, zb, thb0, ml, st); ok = true; break;
    QG_RDCT(QG_CASE)
#undef QG_CASE
    default: break;
  }
  if (!ok) return false;
  ok = false;
  switch (g.nphi) {
#define QG_CASE(n) case n: ring_T_n<n>(g, X, G, NLb, zb, kappa, Xb, st); ok = true; break;
    QG_RPHI(QG_CASE)
#undef QG_CASE
    default: break;
  }
  if (!ok) return false;
  switch (n2) {
#define QG_CASE(n) case n: synth_T_n<n>(g, Xb, thb0, add, mk, psib, thb, st); return true;
    QG_RDCT(QG_CASE)
#undef QG_CASE
    default: return false;
  }
}

void launch_energy_total(const double* diag, int M, int N, double c, double* J,
                         hipStream_t st) {
  hipLaunchKernelGGL(energy_total_kernel, dim3(1), dim3(256), 0, st, diag, M, N, c, J);
}

void launch_to_internal(int M, int K, const double2* psi, const double2* th, const double* u,
                        double2* dp, double2* dt, hipStream_t st) {
  const size_t MK = (size_t)M * K;
  hipLaunchKernelGGL(to_internal_kernel, dim3((unsigned)((MK + 255) / 256)), dim3(256), 0, st, M,
                     K, psi, th, u, dp, dt);
}

void launch_to_api(int M, int K, const double2* sp, const double2* sth, double2* psi,
                   double2* th, double* u, hipStream_t st) {
  const size_t MK = (size_t)M * K;
  hipLaunchKernelGGL(to_api_kernel, dim3((unsigned)((MK + 255) / 256)), dim3(256), 0, st, M, K,
                     sp, sth, psi, th, u);
}

}  // namespace qg
