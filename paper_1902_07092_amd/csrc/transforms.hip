// Transform kernels of one IMEX step of spherical quasi-geostrophic
// convection (FP64, gfx950):
//
//   synth_kernel     per m:    Chebyshev derivative recurrences and inverse
//                              DCT-I (eq. cheb) of Psi, Psi', Psi'', Psi''',
//                              theta, theta'; the six products' factors in
//                              physical s and spectral phi
//   ring_kernel      per s_k:  c2r FFTs (eq. fft), advection products,
//                              r2c FFTs (eq. ifft), zonal forcing
//   analysis_kernel  per m:    forward DCT-I (eq. icheb) with radial
//                              dealiasing, explicit terms C[..], -D[..]
//
// Layout: X[f][k][m] (m fastest, written per m, read per ring) and
// NL[f][m][k] (k fastest, written per ring, read per m): every kernel
// reads contiguous rows and scatters only its stores.  Blocks go to the
// eight XCDs round robin; the kernels map consecutive m (or k) to the same
// XCD so that the 16-byte scattered stores of neighbouring blocks share L2
// lines.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>
#include <vector>

#include "fft.h"
#include "kernels.h"
#include "transform_util.h"

namespace qg {

// ----------------------------------------------- radial transforms on MFMA
// At small N_r the radial transforms are short dense products: per m the
// six coefficient series of the synthesis (Psi and its first three
// derivatives, theta, theta') go to the grid as one [R x K] x [K x 12]
// product, the two fields of the analysis to coefficients as one
// [K x R] x [R x 4] product, on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64: A[r][k] from lane 16 k + r, B[k][c] from lane
// 16 k + c, D[r][c] in lane 16 (r mod 4) + c, register r / 4).  The tables
// (Geom::dct_s, dct_a) are built on the host in long double.
typedef double v4d __attribute__((ext_vector_type(4)));

template <int N2>
constexpr int threads_mf() { return clampi(N2 / 2, 64, 256); }

__host__ __device__ constexpr int mf_kp(int K) { return (K + 3) & ~3; }
__host__ __device__ constexpr int mf_rp(int R) { return (R + 15) & ~15; }
__host__ __device__ constexpr int mf_r4(int R) { return (R + 3) & ~3; }
__host__ __device__ constexpr int mf_k16(int K) { return (K + 15) & ~15; }

// Synthesis: levels 0..3 of Psi_m and 0..1 of theta_m (Chebyshev
// derivatives by the same in-place recurrence as the FFT path) into LDS,
// then P[d][k] = sum_n T_n(x_k) c_d[n] for all six levels at once.
// Returns P, [6][RP] in LDS (levels 4, 5: theta, theta').
template <int T>
__device__ const double2* mf_synth_levels(const Geom& g, const double2* __restrict__ pm,
                                          const double2* __restrict__ tm, double2* sm,
                                          double2* wred) {
  const int K = g.K, t = threadIdx.x;
  const int KP = mf_kp(K), RP = mf_rp(g.R);
  double2* Cl = sm;            // [6][KP] coefficient levels
  double2* Pl = sm + 6 * KP;   // [6][RP] grid values
  for (int nn = t; nn < KP; nn += T) {
    Cl[nn] = nn < K ? pm[nn] : z2();
    Cl[4 * KP + nn] = nn < K ? tm[nn] : z2();
  }
  __syncthreads();
  for (int d = 1; d < 6; ++d) {
    if (d == 4) continue;
    for (int nn = t; nn < KP; nn += T) Cl[d * KP + nn] = Cl[(d - 1) * KP + nn];
    __syncthreads();
    cheb_deriv_inplace<T>(Cl + d * KP, K, wred);   // ends with a barrier
  }
  constexpr int NW = T / 64;
  const int lane = t & 63, w = t >> 6, r16 = lane & 15, kq = lane >> 4;
  const int dc = r16 >> 1, comp = r16 & 1;   // B column: level, real or imaginary part
  const double* cl = reinterpret_cast<const double*>(Cl);
  double* pl = reinterpret_cast<double*>(Pl);
  for (int rt = w; rt < RP / 16; rt += NW) {
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    const double* ta = g.dct_s + 16 * rt + r16;
#pragma unroll 4
    for (int kb = 0; kb < KP / 4; ++kb) {
      const int n = 4 * kb + kq;
      const double a = ta[(size_t)n * RP];
      const double b = (dc < 6) ? cl[2 * (dc * KP + n) + comp] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    if (dc < 6) {
#pragma unroll
      for (int i = 0; i < 4; ++i) pl[2 * (dc * RP + 16 * rt + 4 * i + kq) + comp] = acc[i];
    }
  }
  __syncthreads();
  return Pl;
}

// Grid values of level d at this thread's points k = t + i T.
template <int N2, int T, typename C>
__device__ __forceinline__ void mf_read(const double2* Pl, int R, int d,
                                        C (&P)[out_count<N2, T>()]) {
  const int RP = mf_rp(R);
#pragma unroll
  for (int i = 0; i < out_count<N2, T>(); ++i) {
    const int k = threadIdx.x + i * T;
    P[i] = (k < RP) ? to_c<C>(Pl[d * RP + k]) : zc<C>();
  }
}

// Analysis: the two fields (their grid values, [2][R4] in LDS, zero past
// k = N) to their Chebyshev coefficients, [2][K16] in LDS.
template <int T>
__device__ void mf_analysis_gemm(const Geom& g, const double2* Fl, double2* Cw) {
  const int R4 = mf_r4(g.R), K16 = mf_k16(g.K), t = threadIdx.x;
  constexpr int NW = T / 64;
  const int lane = t & 63, w = t >> 6, r16 = lane & 15, kq = lane >> 4;
  const int fc = r16 >> 1, comp = r16 & 1;   // B column: field, real or imaginary part
  const double* fl = reinterpret_cast<const double*>(Fl);
  double* cw = reinterpret_cast<double*>(Cw);
  for (int rt = w; rt < K16 / 16; rt += NW) {
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    const double* ta = g.dct_a + 16 * rt + r16;
#pragma unroll 4
    for (int kb = 0; kb < R4 / 4; ++kb) {
      const int k = 4 * kb + kq;
      const double a = ta[(size_t)k * K16];
      const double b = (fc < 2) ? fl[2 * (fc * R4 + k) + comp] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    if (fc < 2) {
#pragma unroll
      for (int i = 0; i < 4; ++i) cw[2 * (fc * K16 + 16 * rt + 4 * i + kq) + comp] = acc[i];
    }
  }
  __syncthreads();
}

// Waves per SIMD for the register allocator (lds_waves): the synthesis
// holds one transform buffer and the coefficients (K <= N2 / 3 + 1), the
// ring one transform buffer.  Only the FP64 kernels of 256-thread blocks
// are constrained: with the 64-thread blocks of the ensemble sizes the
// spills cost more than the extra wave gives (64 runs of N_r = 65 .. 257:
// 0.759 -> 0.794 ms per step), and the FP32 kernels fit unconstrained.
template <int N2, int T, typename C>
constexpr int synth_waves() {
  if (T < 256 || sizeof(C) != sizeof(double2)) return 1;
  return lds_waves(coef_offset<C>(lds_slots(N2)) + sizeof(double2) * (N2 / 3 + 1) + 256, T);
}
template <int NPHI, int T, typename C>
constexpr int ring_waves() {
  if (T < 256 || sizeof(C) != sizeof(double2)) return 1;
  return lds_waves(sizeof(C) * lds_slots(NPHI) + 256, T);
}

// -------------------------------------------------------------- synth
// Fields (Fourier coefficient m at s_k), written X[f][k][m]:
//   0: dPsi/dphi = i m Psi          1: v = u_phi / s
//   2: c_w = omega + (h^2/s) d_s omega   3: d omega/dphi = i m omega
//   4: c_t = (h^2/s)(d_s theta + dTc/ds [m=0])   5: d theta/dphi
// with u_phi = -h^2 Psi' + 3 s Psi (+ zonal flow at m = 0), omega = -L_I Psi
// (m >= 1) and omega_0 = u' + u/s (Sect. 3.2.1).  The inverse DCT-I of a
// coefficient row a_n (n < K) is the FFT of the even extension e_0 = a_0,
// e_n = e_{2N-n} = a_n / 2 (eq. cheb).  Thread t owns the radial points
// k = t + i T, and the fields are accumulated derivative by derivative.
template <int N2, int T, typename C, bool PUMP, bool MF = false>
__global__ __launch_bounds__(T, (synth_waves<N2, T, C>())) void synth_kernel(Geom g, const double2* __restrict__ psi,
                                                  const double2* __restrict__ th,
                                                  C* __restrict__ X,
                                                  double* __restrict__ diag, int split) {
  extern __shared__ double2 sm[];
  __shared__ double2 wred[2 * (T / 64)];
  __shared__ double red[T / 64];
  constexpr int N = N2 / 2;
  constexpr int E = out_count<N2, T>();
  constexpr int NP = (N / T + 1) < E ? (N / T + 1) : E;   // registers holding k <= N
  const int K = g.K, R = g.R, M = g.M;
  const int t = threadIdx.x;
  // split: blocks [0, B) take the Psi part of their m (fields 0..3), blocks
  // [B, 2B) the theta part (fields 4, 5), B = 8 ceil(M / 8); the Psi parts
  // (about 2/3 of the work) are dispatched first, and the short theta
  // parts fill the last round.  Otherwise one block does both.
  int part = 0, bid = blockIdx.x;
  if (split) {
    const int B = 8 * ((M + 7) >> 3);
    part = bid < B ? 1 : 2;
    if (bid >= B) bid -= B;
  }
  const int m = xcd_index_of(bid, M);
  if (m >= M || nf_stop(g.nf)) return;
  double2* pump = g.pump;
  {
    const size_t mem = blockIdx.y;
    psi += mem * M * K;
    th += mem * M * K;
    X += mem * 6 * R * M;
    if (diag) diag += mem * 8 * M;
    if (PUMP) pump += mem * M * R + (size_t)m * R;
  }
  // Ekman pumping, eq. approx_pump, accumulated in this block's row of
  // g.pump (each entry by the thread that owns its radial point):
  //   d = 0: -(3 s^2/(2 h_e^2) + m^2 + 5 i m s_o/(2 h_e)) Psi
  //   d = 1: + (s/2) Psi'            d = 2: + L_I Psi = -omega, times Upsilon_e
  // and at m = 0 Upsilon_e u (1 + (E/2) omega_0) once omega_0 is known.
  auto ups_e = [&](double s, double& he2, double& he) {
    he2 = g.pump_so2e - s * s;
    he = sqrt(he2);
    return g.pump_ups / (he * sqrt(he));
  };
  C* fb = reinterpret_cast<C*>(sm);
  double2* c = reinterpret_cast<double2*>(reinterpret_cast<char*>(sm) + coef_offset<C>(lds_slots(N2)));
  auto ext = [&](int i) -> C {
    const int nn = (i <= N) ? i : N2 - i;
    if (nn >= K) return zc<C>();
    const double2 v = c[nn];
    return to_c<C>(nn == 0 ? v : scl2(0.5, v));
  };
  auto store = [&](int f, int k, double2 v) { X[((size_t)f * R + k) * M + m] = to_c<C>(v); };

  const double dm = (double)m, m2 = dm * dm, so2 = g.s_o * g.s_o;
  double sk[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const int k = t + i * T;
    sk[i] = (k <= N) ? g.half * g.xk[k] + g.mid : 1.0;
  }
  double2 a1[NP], a2[NP], a3[NP];   // m > 0: u_phi, omega, c_w accumulators
  double ek = 0.0, et = 0.0, ens = 0.0, ez = 0.0;

  [[maybe_unused]] const double2* Pl = nullptr;   // MF: grid values of all six levels
  if constexpr (MF) Pl = mf_synth_levels<T>(g, psi + (size_t)m * K, th + (size_t)m * K, sm, wred);
  if (part != 2) {   // Psi (or, at m = 0, the zonal flow): fields 0..3
  if constexpr (!MF) {
    for (int nn = t; nn < K; nn += T) c[nn] = psi[(size_t)m * K + nn];
    __syncthreads();
  }
  const int nder = (m > 0) ? 4 : 3;
#pragma unroll 1
  for (int d = 0; d < nder; ++d) {
    C P[E];
    if constexpr (MF) {
      mf_read<N2, T>(Pl, R, d, P);
    } else {
      if (d > 0) cheb_deriv_inplace<T>(c, K, wred);
      fft_out<N2, T, -1>(ext, fb, Tw<C>::dct(g), P);
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      int k = t + i * T;
      if (k > N) continue;
      double s = sk[i];
      opaque(s, k);
      const double is = 1.0 / s, h2 = so2 - s * s, h2s = h2 * is;
      const double2 p = to_d2(P[i]);
      if (m > 0) {
        const double mh = m2 * h2 * is * is;
        if (d == 0) {
          store(0, k, ix(dm, p));
          if constexpr (PUMP) {
            double he2, he;
            (void)ups_e(s, he2, he);
            const double cr = 1.5 * s * s / he2 + m2, ci = 2.5 * dm * g.s_o / he;
            pump[k] = make_double2(-(cr * p.x - ci * p.y), -(cr * p.y + ci * p.x));
          }
          a1[i] = scl2(3.0 * s, p);
          a2[i] = scl2(6.0 + mh, p);
          a3[i] = scl2(6.0 + mh - h2s * 2.0 * m2 * so2 * is * is * is, p);
          if (diag) ek += 2.0 * g.wq[k] * h2s * h2s * m2 * abs2(p);
        } else if (d == 1) {
          const double2 uph = sub2(a1[i], scl2(h2, p));
          store(1, k, scl2(is, uph));
          if constexpr (PUMP) pump[k] = add2(pump[k], scl2(0.5 * s, p));
          if (diag) ek += 2.0 * g.wq[k] * abs2(uph);
          a2[i] = sub2(a2[i], scl2(h2s - 5.0 * s, p));
          a3[i] = add2(a3[i], scl2(-(h2s - 5.0 * s) + h2s * (so2 * is * is + 12.0 + mh), p));
        } else if (d == 2) {
          const double2 om = sub2(a2[i], scl2(h2, p));
          store(3, k, ix(dm, om));
          if constexpr (PUMP) {
            double he2, he;
            const double ue = ups_e(s, he2, he);
            pump[k] = scl2(ue, sub2(pump[k], om));
          }
          if (diag) ens += 2.0 * g.wq[k] * abs2(om);
          a3[i] = sub2(a3[i], scl2(h2 + h2s * (h2s - 7.0 * s), p));
        } else {
          store(2, k, sub2(a3[i], scl2(h2s * h2, p)));
        }
      } else {
        // zonal flow u = P0, u' = P1, u'' = P2 (real)
        if (d == 0) {
          store(0, k, z2());
          store(1, k, scl2(is, p));
          store(3, k, z2());
          a1[i] = p;
          a2[i] = scl2(is, p);                                   // omega
          a3[i] = sub2(scl2(is, p), scl2(h2s * is * is, p));     // c_w
          if (diag) {
            ek += g.wq[k] * p.x * p.x;
            ez += g.wq[k] * p.x * p.x;
          }
        } else if (d == 1) {
          a2[i] = add2(a2[i], p);
          a3[i] = add2(a3[i], scl2(1.0 + h2s * is, p));
          if constexpr (PUMP) {
            double he2, he;
            const double ue = ups_e(s, he2, he);
            pump[k] = make_double2(ue * a1[i].x * (1.0 + g.half_E * a2[i].x), 0.0);
          }
          if (diag) ens += g.wq[k] * a2[i].x * a2[i].x;
        } else {
          store(2, k, add2(a3[i], scl2(h2s, p)));
        }
      }
    }
  }
  }   // Psi part
  // theta, theta'
  if (part != 1) {
  if constexpr (!MF) {
    __syncthreads();
    for (int nn = t; nn < K; nn += T) c[nn] = th[(size_t)m * K + nn];
    __syncthreads();
  }
#pragma unroll 1
  for (int d = 0; d < 2; ++d) {
    C P[E];
    if constexpr (MF) {
      mf_read<N2, T>(Pl, R, 4 + d, P);
    } else {
      if (d > 0) cheb_deriv_inplace<T>(c, K, wred);
      fft_out<N2, T, -1>(ext, fb, Tw<C>::dct(g), P);
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      int k = t + i * T;
      if (k > N) continue;
      double s = sk[i];
      opaque(s, k);
      const double is = 1.0 / s, h2s = (so2 - s * s) * is;
      const double2 p = to_d2(P[i]);
      if (d == 0) {
        store(5, k, ix(dm, p));
        if (diag) et += (m > 0 ? 2.0 : 1.0) * g.wq[k] * (m > 0 ? abs2(p) : p.x * p.x);
      } else {
        double2 v = p;
        if (m == 0) v.x += g.dtc_coef * is;
        store(4, k, scl2(h2s, v));
      }
    }
  }
  }   // theta part
  // diagnostics of this block's part: slots 0, 1, 3 and the non-finite flag
  // of Psi in 4 (Psi part), slot 2 and the flag of theta in 5 (theta part)
  if (diag) {
    const double pi = 3.14159265358979323846;
    double bad = 0.0, badt = 0.0;
    for (int nn = t; nn < K; nn += T) {
      if (part != 2) {
        const double2 a = psi[(size_t)m * K + nn];
        if (!isfinite(a.x) || !isfinite(a.y)) bad = 1.0;
      }
      if (part != 1) {
        const double2 b = th[(size_t)m * K + nn];
        if (!isfinite(b.x) || !isfinite(b.y)) badt = 1.0;
      }
    }
    const double s0 = block_sum(ek, red);
    const double s1 = block_sum(ez, red);
    const double s2 = block_sum(et, red);
    const double s3 = block_sum(ens, red);
    const double s4 = block_max(bad, red);
    const double s5 = block_max(badt, red);
    if (t == 0) {
      if (part != 2) {
        diag[m * 8 + 0] = pi * s0;
        diag[m * 8 + 1] = pi * s1;
        diag[m * 8 + 3] = 2.0 * pi * s3;
        diag[m * 8 + 4] = s4;
      }
      if (part != 1) {
        diag[m * 8 + 2] = pi * s2;
        diag[m * 8 + 5] = s5;
      }
    }
  }
}

// ---------------------------------------------------------------- ring
// Per radial level: three complex inverse FFTs of length N_phi (each
// carries two real fields of similar size: z = A + i B from the half
// spectra), the products
//   N_omega = dPsi/dphi c_w + v d omega/dphi,
//   N_theta = dPsi/dphi c_t + v d theta/dphi,
// then the two real forward FFTs (eq. ifft) as one batch of two complex
// FFTs of length N_phi/2 of z_j = x_2j + i x_2j+1:
//   X_m = (Z_m + Z*_{N/2-m})/2 - (i/2) w^m (Z_m - Z*_{N/2-m}),  w = e^{-2 pi i/N},
// scaled by 1/N_phi and truncated to m <= N_m (N_omega can exceed N_theta by
// many orders of magnitude, so the two never share one complex transform).
// Zonal forcing: mean(u_s omega) = 2 sum_{m>=1} Re(u_s,m conj(omega_m)) with
// u_s,m = (h^2/s) X0_m and omega_m = X3_m / (i m).  G (optional, FP64
// single runs): the six grid fields g_f(phi_j) out, [6][R][N_phi], for the
// reverse mode.
template <int NPHI, int T, typename C>
__global__ __launch_bounds__(T, (ring_waves<NPHI, T, C>())) void ring_kernel(Geom g, const C* __restrict__ X,
                                                 C* __restrict__ NL,
                                                 double* __restrict__ zonal,
                                                 double* __restrict__ rate,
                                                 double* __restrict__ G) {
  using RT = fftd::real_t<C>;
  extern __shared__ double2 sm[];
  C* fb = reinterpret_cast<C*>(sm);
  __shared__ double red[T / 64];
  constexpr int E = out_count<NPHI, T>();
  constexpr int NH = NPHI / 2;
  const int R = g.R, M = g.M;
  const int t = threadIdx.x;
  const int k = xcd_index(R);
  if (k >= R || nf_stop(g.nf)) return;
  {
    const size_t mem = blockIdx.y;
    X += mem * 6 * R * M;
    NL += mem * 2 * M * R;
    zonal += mem * R;
    if (rate) rate += mem * R;
  }
  const double s = g.half * g.xk[k] + g.mid;
  const double h2s = (g.s_o * g.s_o - s * s) / s;
  const C* X0 = X + (size_t)k * M;
  C z1[E];
  RT nw[E], nt[E];
  double zs = 0.0, rmax = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const C* A = X + ((size_t)(2 * q) * R + k) * M;
    const C* B = X + ((size_t)(2 * q + 1) * R + k) * M;
    auto get = [&](int i) -> C {
      if (i < M) {
        const C a = A[i], b = B[i];
        if (q == 1 && i > 0) {
          const C x0 = X0[i];
          zs += ((double)x0.y * b.x - (double)x0.x * b.y) / (double)i;
        }
        return (i == 0) ? fftd::mk<C>(a.x, b.x) : fftd::mk<C>(a.x - b.y, a.y + b.x);
      }
      if (i > NPHI - M) {
        const C a = A[NPHI - i], b = B[NPHI - i];
        return fftd::mk<C>(a.x + b.y, b.x - a.y);
      }
      return zc<C>();
    };
    C z[E];
    fft_out<NPHI, T, +1>(get, fb, Tw<C>::phi(g), z);
    if (G) {
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int j = t + i * T;
        if (j < NPHI) {
          G[((size_t)(2 * q) * R + k) * NPHI + j] = (double)z[i].x;
          G[((size_t)(2 * q + 1) * R + k) * NPHI + j] = (double)z[i].y;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < E; ++i) {
      if (q == 0) {
        z1[i] = z[i];
        if (rate)
          rmax = fmax(rmax, fmax(h2s * fabs((double)z[i].x) / g.dsk[k],
                                 fabs((double)z[i].y) * NPHI / (2.0 * 3.14159265358979323846)));
      } else if (q == 1) {
        nw[i] = z1[i].x * z[i].x + z1[i].y * z[i].y;
      } else {
        nt[i] = z1[i].x * z[i].x + z1[i].y * z[i].y;
      }
    }
  }
  // real products: N_omega at [0, NPHI), N_theta at [NPHI, 2 NPHI) (reals)
  __syncthreads();
  RT* fr = reinterpret_cast<RT*>(fb);
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int j = t + i * T;
    if (j < NPHI) {
      fr[j] = nw[i];
      fr[NPHI + j] = nt[i];
    }
  }
  __syncthreads();
  const C* zin = fb;
  fft_to_lds<NH, T, -1, 2>([&](int ii) { return zin[ii]; }, fb, Tw<C>::half(g));
  const RT inv = (RT)1.0 / (RT)NPHI;
  for (int m = t; m < M; m += T) {
    const C w = Tw<C>::w(g)[m];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      C zk = fb[lds_pad(f * NH + m)];
      C zc_ = fb[lds_pad(f * NH + (NH - m) % NH)];
      zc_.y = -zc_.y;
      const C e = fftd::scl((RT)0.5, fftd::add(zk, zc_));
      const C dd = fftd::sub(zk, zc_);
      const C o = fftd::mk<C>((RT)0.5 * dd.y, (RT)-0.5 * dd.x);   // (Z_m - Z*)/(2i)
      C xm = fftd::add(e, fftd::mul(w, o));
      if (m == 0) xm.y = 0;
      NL[((size_t)f * M + m) * R + k] = fftd::scl(inv, xm);
    }
  }
  const double tot = block_sum(zs, red);
  if (t == 0) zonal[k] = -2.0 * h2s * tot;
  if (rate) {
    const double rm = block_max(rmax, red);
    if (t == 0) rate[k] = rm;
  }
}

// ------------------------------------------------------------ analysis
// Explicit right-hand sides at a stage state:
//   m >= 1: E_psi = C [ (Ra/Pr)(i m/s_o) theta + N_omega ]   (eq. psi_int)
//   m = 0:  E_u   = -D [ mean(u_s omega) ]                   (eq. uphi_int)
//   all m:  E_th  = -D [ N_theta ]                           (eq. temp_int)
// Forward DCT-I (eq. icheb): a_n = (h_n / N) FFT(e)_n with the even
// extension e_i = f_{|i|}, h_0 = 1/2, else 1, kept for n < K.
template <int N2, int T, typename C, bool MF = false>
__global__ __launch_bounds__(T) void analysis_kernel(Geom g, Bands b,
                                                     const C* __restrict__ NL,
                                                     const double* __restrict__ zonal,
                                                     const double2* __restrict__ th_state,
                                                     double2* __restrict__ Epsi,
                                                     double2* __restrict__ Eth, int split) {
  extern __shared__ double2 sm[];
  constexpr int N = N2 / 2;
  constexpr int E = out_count<N2, T>();
  const int K = g.K, R = g.R, M = g.M;
  const int t = threadIdx.x;
  // split: blocks [0, B) transform field 0 (E_psi, or E_u at m = 0) of
  // their m, blocks [B, 2B) field 1 (E_theta), B = 8 ceil(M / 8): two equal
  // halves, so that the last round of resident blocks is half as long.
  // Otherwise one block does both.
  int only = -1, bid = blockIdx.x;
  if (split) {
    const int B = 8 * ((M + 7) >> 3);
    only = bid < B ? 0 : 1;
    if (bid >= B) bid -= B;
  }
  const int m = xcd_index_of(bid, M);
  if (m >= M || nf_stop(g.nf)) return;
  const size_t mem = blockIdx.y;
  NL += mem * 2 * M * R;
  zonal += mem * R;
  const double2* pump = g.pump ? g.pump + mem * M * R + (size_t)m * R : nullptr;
  th_state += mem * M * K;
  Epsi += mem * M * K;
  Eth += mem * M * K;
  C* fb = reinterpret_cast<C*>(sm);
  // the coefficients take the transform buffer's place once the transform
  // is done (analysis_lds: the larger of the two, not their sum)
  double2* c = sm;
  const double invN = 1.0 / N;
  const double2* thm = th_state + (size_t)m * K;
  const double ra_pr = g.ra_pr ? g.ra_pr[mem] : g.Ra_Pr;
  // (Ra/Pr)(m/s_o), times i; zero when the buoyancy is implicit (then it
  // belongs to the implicit operator)
  const double bcoef = g.buoy_implicit ? 0.0 : ra_pr * (double)m / g.s_o;
  // the field transformed for f (0: N_omega less the pumping term, or the
  // zonal forcing at m = 0; 1: N_theta) at radial point kk
  auto field = [&](int f, int kk) -> C {
    if (f == 0 && m == 0)
      return to_c<C>(make_double2(zonal[kk] + (pump ? pump[kk].x : 0.0), 0.0));
    if (f == 0 && pump) return to_c<C>(sub2(to_d2(NL[(size_t)m * R + kk]), pump[kk]));
    return NL[((size_t)f * M + m) * R + kk];
  };
  [[maybe_unused]] double2* Cw = nullptr;   // MF: coefficients of both fields, [2][K16]
  if constexpr (MF) {
    const int R4 = mf_r4(R);
    double2* Fl = sm;
    Cw = sm + 2 * R4;
    for (int kk = t; kk < R4; kk += T) {
      Fl[kk] = kk < R ? to_d2(field(0, kk)) : z2();
      Fl[R4 + kk] = kk < R ? to_d2(field(1, kk)) : z2();
    }
    __syncthreads();
    mf_analysis_gemm<T>(g, Fl, Cw);
  }
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    if (only >= 0 && f != only) continue;
    if constexpr (MF) {
      c = Cw + f * mf_k16(K);
    } else {
      auto get = [&](int i) -> C { return field(f, (i <= N) ? i : N2 - i); };
      C o[E];
      fft_out<N2, T, -1>(get, fb, Tw<C>::dct(g), o);
      __syncthreads();   // every read of fb is done before c overwrites it
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int nn = t + i * T;
        if (nn < K) c[nn] = scl2(nn == 0 ? 0.5 * invN : invN, to_d2(o[i]));
      }
      __syncthreads();
    }
    // band rows: fixed 17 terms (entries outside the matrix are stored as
    // zeros), so that every load of a row is issued at once
    for (int k = t; k < K; k += T) {
      double2 acc = z2();
      if (f == 0 && m > 0) {
        if (k >= 4) {
#pragma unroll
          for (int o = 0; o < 17; ++o) {
            const int nn = min(max(k + o - 8, 0), K - 1);
            const double cc = b.C[(size_t)o * K + k];
            acc = add2(acc, scl2(cc, add2(c[nn], ix(bcoef, thm[nn]))));
          }
        }
        Epsi[(size_t)m * K + k] = acc;
      } else {
        if (k >= 2) {
#pragma unroll
          for (int o = 0; o < 17; ++o) {
            const int nn = min(max(k + o - 8, 0), K - 1);
            acc = sub2(acc, scl2(b.D[(size_t)o * K + k], c[nn]));
          }
        }
        (f == 0 ? Epsi : Eth)[(size_t)m * K + k] = acc;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ launchers
namespace {

template <int N2, typename C, bool PUMP>
void synth_np(const Geom& g, const double2* psi, const double2* th, void* X, double* diag,
              hipStream_t st) {
  if constexpr (std::is_same<C, double2>::value && N2 <= MFMA_DCT_MAX_N2) {
    if (g.dct_s) {   // radial transform on the matrix cores
      constexpr int T = threads_mf<N2>();
      const size_t shm = sizeof(double2) * 6 * (mf_kp(g.K) + mf_rp(g.R));
      allow_lds(synth_kernel<N2, T, C, PUMP, true>, shm);
      hipLaunchKernelGGL((synth_kernel<N2, T, C, PUMP, true>), dim3(xcd_grid(g.M), g.nmem),
                         dim3(T), shm, st, g, psi, th, static_cast<C*>(X), diag, 0);
      return;
    }
  }
  constexpr int T = threads_dct(N2);
  const size_t shm = dct_lds<C>(N2, g.K);
  allow_lds(synth_kernel<N2, T, C, PUMP>, shm);
  hipLaunchKernelGGL((synth_kernel<N2, T, C, PUMP>), dim3(2 * xcd_grid(g.M), g.nmem), dim3(T), shm,
                     st, g, psi, th, static_cast<C*>(X), diag, 1);
}

// The pumping terms are a separate instantiation: without them the kernel
// carries no pumping code (and no extra registers).
template <int N2, typename C>
void synth_n(const Geom& g, const double2* psi, const double2* th, void* X, double* diag,
             hipStream_t st) {
  if (g.pump)
    synth_np<N2, C, true>(g, psi, th, X, diag, st);
  else
    synth_np<N2, C, false>(g, psi, th, X, diag, st);
}

template <int NPHI, typename C>
void ring_n(const Geom& g, const void* X, void* NL, double* zonal, double* rate, double* G,
            hipStream_t st) {
  constexpr int T = threads_phi(NPHI);
  const size_t shm = phi_lds<C>(NPHI);
  allow_lds(ring_kernel<NPHI, T, C>, shm);
  hipLaunchKernelGGL((ring_kernel<NPHI, T, C>), dim3(xcd_grid(g.R), g.nmem), dim3(T), shm, st, g,
                     static_cast<const C*>(X), static_cast<C*>(NL), zonal, rate, G);
}

template <int N2, typename C>
void analysis_n(const Geom& g, const Bands& b, const void* NL, const double* zonal,
                const double2* th, double2* Ep, double2* Et, hipStream_t st) {
  if constexpr (std::is_same<C, double2>::value && N2 <= MFMA_DCT_MAX_N2) {
    if (g.dct_a) {   // radial transform on the matrix cores
      constexpr int T = threads_mf<N2>();
      const size_t shm = sizeof(double2) * 2 * (mf_r4(g.R) + mf_k16(g.K));
      allow_lds(analysis_kernel<N2, T, C, true>, shm);
      hipLaunchKernelGGL((analysis_kernel<N2, T, C, true>), dim3(xcd_grid(g.M), g.nmem),
                         dim3(T), shm, st, g, b, static_cast<const C*>(NL), zonal, th, Ep, Et, 0);
      return;
    }
  }
  constexpr int T = threads_dct(N2);
  const size_t shm = analysis_lds<C>(N2, g.K);
  allow_lds(analysis_kernel<N2, T, C>, shm);
  hipLaunchKernelGGL((analysis_kernel<N2, T, C>), dim3(2 * xcd_grid(g.M), g.nmem), dim3(T), shm, st,
                     g, b, static_cast<const C*>(NL), zonal, th, Ep, Et, 1);
}

// Compiled lengths: 2 (N_r - 1) = 2^a or 3 * 2^a (the paper's radial
// resolutions 193, 769 and 3073 are of the second kind), FP64 up to 6144
// (the LDS bound of the FP64 radial transforms), FP32 up to 12288;
// N_phi = 3 * 2^a, FP64 up to 6144 (the LDS bound of the FP64 rings),
// FP32 up to 12288.
#define QG_DCT64(X) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) \
  X(1024) X(1536) X(2048) X(3072) X(4096) X(6144)
#define QG_PHI64(X) X(24) X(48) X(96) X(192) X(384) X(768) X(1536) X(3072) X(6144)
#define QG_DCT32(X) QG_DCT64(X) X(8192) X(12288)
#define QG_PHI32(X) QG_PHI64(X) X(12288)

}  // namespace

bool transform_sizes_ok(int n2, int nphi, bool mixed) {
  bool a = false, b = false;
#define QG_CASE(n) a = a || (n2 == n);
  if (mixed) { QG_DCT32(QG_CASE) } else { QG_DCT64(QG_CASE) }
#undef QG_CASE
#define QG_CASE(n) b = b || (nphi == n);
  if (mixed) { QG_PHI32(QG_CASE) } else { QG_PHI64(QG_CASE) }
#undef QG_CASE
  return a && b;
}

size_t transform_lds_bytes(int n2, int nphi, int K, bool mixed) {
  const size_t d = mixed ? dct_lds<float2>(n2, K) : dct_lds<double2>(n2, K);
  const size_t p = mixed ? phi_lds<float2>(nphi) : phi_lds<double2>(nphi);
  return d > p ? d : p;
}

size_t mfma_dct_table_bytes(int R, int K, bool analysis) {
  return sizeof(double) * (analysis ? (size_t)mf_r4(R) * mf_k16(K) : (size_t)mf_kp(K) * mf_rp(R));
}

// cos(pi n k / N) in long double with the argument reduced mod 2N, rounded
// once; the analysis table carries the forward DCT-I weights.
void mfma_dct_tables(int R, int K, std::vector<double>& syn, std::vector<double>& ana) {
  const int N = R - 1, KP = mf_kp(K), RP = mf_rp(R), R4 = mf_r4(R), K16 = mf_k16(K);
  const long double pi = 3.14159265358979323846264338327950288L;
  auto cs = [&](int n, int k) {
    const long long a = ((long long)n * k) % (2LL * N);
    return cosl(pi * (long double)a / (long double)N);
  };
  syn.assign((size_t)KP * RP, 0.0);
  ana.assign((size_t)R4 * K16, 0.0);
  for (int n = 0; n < K; ++n)
    for (int k = 0; k <= N; ++k) {
      syn[(size_t)n * RP + k] = (double)cs(n, k);
      const long double wn = (n == 0 ? 0.5L : 1.0L) / (long double)N;
      const long double wk = (k == 0 || k == N) ? 1.0L : 2.0L;
      ana[(size_t)k * K16 + n] = (double)(wn * wk * cs(n, k));
    }
}

std::vector<double2> plan_twiddles(int n) {
  const RadixPlan pl = radix_plan(n);
  std::vector<double2> tw(n > 1 ? n - 1 : 1, make_double2(1.0, 0.0));
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int s = 0; s < pl.np; ++s) {
    const int R = pl.r[s], Ns = plan_ns(pl, s);
    for (int r = 1; r < R; ++r)
      for (int k = 0; k < Ns; ++k) {
        const long double a = -2.0L * pi * (long double)(k * r) / (long double)(Ns * R);
        tw[(Ns - 1) + (r - 1) * Ns + k] = make_double2((double)cosl(a), (double)sinl(a));
      }
  }
  return tw;
}

bool launch_synth(const Geom& g, const double2* psi, const double2* th, void* X, double* diag,
                  bool mixed, hipStream_t st) {
  const int n2 = 2 * (g.R - 1);
  if (mixed) {
    switch (n2) {
#define QG_CASE(n) case n: synth_n<n, float2>(g, psi, th, X, diag, st); return true;
      QG_DCT32(QG_CASE)
#undef QG_CASE
      default: return false;
    }
  }
  switch (n2) {
#define QG_CASE(n) case n: synth_n<n, double2>(g, psi, th, X, diag, st); return true;
    QG_DCT64(QG_CASE)
#undef QG_CASE
    default: return false;
  }
}

bool launch_ring(const Geom& g, const void* X, void* NL, double* zonal, double* rate, bool mixed,
                 hipStream_t st, double* G) {
  if (mixed) {
    if (G) return false;
    switch (g.nphi) {
#define QG_CASE(n) case n: ring_n<n, float2>(g, X, NL, zonal, rate, nullptr, st); return true;
      QG_PHI32(QG_CASE)
#undef QG_CASE
      default: return false;
    }
  }
  switch (g.nphi) {
#define QG_CASE(n) case n: ring_n<n, double2>(g, X, NL, zonal, rate, G, st); return true;
    QG_PHI64(QG_CASE)
#undef QG_CASE
    default: return false;
  }
}

bool launch_analysis(const Geom& g, const Bands& b, const void* NL, const double* zonal,
                     const double2* th_state, double2* Epsi, double2* Eth, bool mixed,
                     hipStream_t st) {
  const int n2 = 2 * (g.R - 1);
  if (mixed) {
    switch (n2) {
#define QG_CASE(n) case n: analysis_n<n, float2>(g, b, NL, zonal, th_state, Epsi, Eth, st); return true;
      QG_DCT32(QG_CASE)
#undef QG_CASE
      default: return false;
    }
  }
  switch (n2) {
#define QG_CASE(n) case n: analysis_n<n, double2>(g, b, NL, zonal, th_state, Epsi, Eth, st); return true;
    QG_DCT64(QG_CASE)
#undef QG_CASE
    default: return false;
  }
}

}  // namespace qg
