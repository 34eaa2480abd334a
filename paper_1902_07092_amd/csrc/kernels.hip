// HIP kernels of one IMEX step of spherical quasi-geostrophic convection
// (Chebyshev-integration / tau radial scheme, Fourier in azimuth), FP64.
//
//   synth_kernel     per m:    Chebyshev derivatives, inverse DCT-I
//                              (eq. cheb), six spectral-in-phi fields
//   ring_kernel      per s_k:  c2r FFTs (eq. fft), advection products,
//                              r2c FFT (eq. ifft), zonal forcing
//   analysis_kernel  per m:    forward DCT-I (eq. icheb), radial dealiasing,
//                              explicit right-hand sides C[..], -D[..]
//   solve_kernel     per system: IMEX right-hand side and bordered band
//                              solve (Appendix A), one wavefront each
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace qg {

__device__ __forceinline__ double2 operator+(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 operator-(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 operator*(double a, double2 b) { return make_double2(a * b.x, a * b.y); }
__device__ __forceinline__ double2& operator+=(double2& a, double2 b) { a.x += b.x; a.y += b.y; return a; }
__device__ __forceinline__ double2& operator-=(double2& a, double2 b) { a.x -= b.x; a.y -= b.y; return a; }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 mulf(double a, double2 b) { return a * b; }
__device__ __forceinline__ double2 mulf(double2 a, double2 b) { return cmul(a, b); }
__device__ __forceinline__ double2 times_i(double2 a) { return make_double2(-a.y, a.x); }
__device__ __forceinline__ double2 zero2() { return make_double2(0.0, 0.0); }

template <typename T> __device__ __forceinline__ T tzero();
template <> __device__ __forceinline__ double tzero<double>() { return 0.0; }
template <> __device__ __forceinline__ double2 tzero<double2>() { return zero2(); }

__device__ __forceinline__ double readlane_d(double v, int lane) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double2 readlane2(double2 v, int lane) {
  return make_double2(readlane_d(v.x, lane), readlane_d(v.y, lane));
}

// ------------------------------------------------------------------ FFT
// In-place Stockham FFT in LDS: every pass loads its butterfly inputs into
// registers, synchronises, and writes the outputs back to the same buffer.
// sgn = -1: X_k = sum_j x_j e^{-2 pi i jk/n}; sgn = +1: the e^{+} sum.
template <int MAXB>
__device__ void fft_lds(double2* buf, const FftPlan& P, int sgn) {
  const int n = P.n;
  const int T = blockDim.x, t = threadIdx.x;
  int Ns = 1;
  for (int s = 0; s < P.npass; ++s) {
    const int R = P.radix[s];
    const int nb = n / R;
    const int tws = n / (Ns * R);
    double2 v[MAXB][4];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
      int j = t + i * T;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        v[i][r] = (j < nb && r < R) ? buf[j + r * nb] : zero2();
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
      int j = t + i * T;
      if (j >= nb) continue;
      int k = j % Ns;
#pragma unroll
      for (int r = 1; r < 4; ++r) {
        if (r < R) {
          double2 w = P.tw[k * r * tws * P.tw_stride];
          if (sgn > 0) w.y = -w.y;
          v[i][r] = cmul(v[i][r], w);
        }
      }
      double2 y0, y1, y2, y3;
      if (R == 2) {
        y0 = v[i][0] + v[i][1];
        y1 = v[i][0] - v[i][1];
        y2 = y3 = zero2();
      } else if (R == 4) {
        double2 a = v[i][0] + v[i][2], b = v[i][0] - v[i][2];
        double2 c = v[i][1] + v[i][3], d = v[i][1] - v[i][3];
        double2 id = times_i(d);
        if (sgn < 0) id = make_double2(-id.x, -id.y);   // (sgn i) d
        y0 = a + c;
        y1 = b + id;
        y2 = a - c;
        y3 = b - id;
      } else {  // R == 3
        const double h3 = 0.86602540378443864676;   // sqrt(3)/2
        double2 t1 = v[i][1] + v[i][2], t2 = v[i][1] - v[i][2];
        double2 base = v[i][0] - 0.5 * t1;
        double2 rot = (sgn * h3) * times_i(t2);
        y0 = v[i][0] + t1;
        y1 = base + rot;
        y2 = base - rot;
        y3 = zero2();
      }
      int o = (j / Ns) * Ns * R + k;
      buf[o] = y0;
      buf[o + Ns] = y1;
      if (R > 2) buf[o + 2 * Ns] = y2;
      if (R > 3) buf[o + 3 * Ns] = y3;
    }
    __syncthreads();
    Ns *= R;
  }
}

// ------------------------------------------------------------ reductions
__device__ double block_sum(double v, double* red) {
  const int t = threadIdx.x, T = blockDim.x;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (t == 0)
    for (int w = 0; w < (T + 63) / 64; ++w) s += red[w];
  __syncthreads();
  return s;  // valid on thread 0
}

__device__ double block_max(double v, double* red) {
  const int t = threadIdx.x, T = blockDim.x;
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (t == 0)
    for (int w = 0; w < (T + 63) / 64; ++w) s = fmax(s, red[w]);
  __syncthreads();
  return s;
}

// ------------------------------------------------- Chebyshev derivative
// dst_n = (4/c_n) sum_{j > n, j - n odd} j src_j (c_0 = 2, else 1): the
// coefficients of d/ds on the unit gap (ds = dx/2).  Parallel suffix sums
// of j src_j over each parity class.
__device__ void cheb_deriv(const double2* src, double2* dst, int K, double2* scan) {
  const int T = blockDim.x, t = threadIdx.x;
  const int npair = (K + 1) / 2;
  const int ch = (npair + T - 1) / T;
  const int p0 = min(npair, t * ch), p1 = min(npair, p0 + ch);
  double2 se = zero2(), so = zero2();
  for (int pp = p0; pp < p1; ++pp) {
    int je = 2 * pp, jo = je + 1;
    se += (double)je * src[je];
    if (jo < K) so += (double)jo * src[jo];
  }
  scan[t] = se;
  scan[T + t] = so;
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {
    double2 ae = zero2(), ao = zero2();
    if (t + off < T) { ae = scan[t + off]; ao = scan[T + t + off]; }
    __syncthreads();
    scan[t] += ae;
    scan[T + t] += ao;
    __syncthreads();
  }
  double2 re = (t + 1 < T) ? scan[t + 1] : zero2();
  double2 ro = (t + 1 < T) ? scan[T + t + 1] : zero2();
  for (int pp = p1 - 1; pp >= p0; --pp) {
    int je = 2 * pp, jo = je + 1;
    if (jo < K) {
      dst[jo] = 4.0 * re;            // S_{jo+1} = S_{je+2}
      ro += (double)jo * src[jo];    // S_{jo}
    }
    dst[je] = (je == 0 ? 2.0 : 4.0) * ro;
    re += (double)je * src[je];      // S_{je}
  }
  __syncthreads();
}

// Inverse DCT-I (eq. cheb, standard coefficients): f_k = sum_{n<K} a_n
// cos(pi n k / N), N = R - 1, through the FFT of the even extension
// e_0 = 2 a_0, e_n = e_{2N-n} = a_n; f_k = FFT(e)_k / 2.  Each thread keeps
// the values at k = t + i T.
template <int MAXB, int MAXP>
__device__ void dct_inverse(const double2* coef, int K, double2* fb, const Geom& g,
                            double2 (&out)[MAXP]) {
  const int N = g.R - 1, T = blockDim.x, t = threadIdx.x;
  for (int i = t; i < 2 * N; i += T) {
    int n = (i <= N) ? i : 2 * N - i;
    double2 v = (n < K) ? coef[n] : zero2();
    if (i == 0) v = 2.0 * v;
    fb[i] = v;
  }
  __syncthreads();
  fft_lds<MAXB>(fb, g.dct, -1);
#pragma unroll
  for (int i = 0; i < MAXP; ++i) {
    int k = t + i * T;
    out[i] = (k < g.R) ? 0.5 * fb[k] : zero2();
  }
  __syncthreads();
}

// Forward DCT-I (eq. icheb, standard coefficients), keeping n < K (radial
// dealiasing): a_n = (h_n / N) [f_0 + (-1)^n f_N + 2 sum f_k cos(pi nk/N)],
// h_0 = h_N = 1/2.  Values are read through get(k).
template <int MAXB, typename Get>
__device__ void dct_forward(Get get, double2* coef, int K, double2* fb, const Geom& g) {
  const int N = g.R - 1, T = blockDim.x, t = threadIdx.x;
  for (int i = t; i < 2 * N; i += T) fb[i] = get((i <= N) ? i : 2 * N - i);
  __syncthreads();
  fft_lds<MAXB>(fb, g.dct, -1);
  const double invN = 1.0 / N;
  for (int n = t; n < K; n += T) coef[n] = ((n == 0) ? 0.5 * invN : invN) * fb[n];
  __syncthreads();
}

// -------------------------------------------------------------- synth
// Fields (Fourier coefficient m at s_k), written X[f][k][m]:
//   0: dPsi/dphi = i m Psi          1: v = u_phi / s
//   2: c_w = omega + (h^2/s) d_s omega   3: d omega/dphi = i m omega
//   4: c_t = (h^2/s)(d_s theta + dTc/ds [m=0])   5: d theta/dphi
// with u_phi = -h^2 Psi' + 3 s Psi (+ zonal flow at m = 0), omega = -L_I Psi
// (m >= 1) and omega_0 = u' + u/s (Sect. 3.2.1).
template <int MAXB, int MAXP>
__global__ void synth_kernel(Geom g, const double2* __restrict__ psi,
                             const double2* __restrict__ th, double2* __restrict__ X,
                             double* __restrict__ diag) {
  extern __shared__ double2 sm[];
  __shared__ double red[16];
  const int K = g.K, R = g.R, M = g.M, N = R - 1;
  const int T = blockDim.x, t = threadIdx.x;
  const int m = blockIdx.x;
  double2* ca = sm;
  double2* cb = sm + K;
  double2* fb = sm + 2 * K;
  double2* scan = fb + 2 * N;

  for (int n = t; n < K; n += T) ca[n] = psi[(size_t)m * K + n];
  __syncthreads();
  double2 P0[MAXP], P1[MAXP], P2[MAXP], P3[MAXP], T0[MAXP], T1[MAXP];
  dct_inverse<MAXB, MAXP>(ca, K, fb, g, P0);
  cheb_deriv(ca, cb, K, scan);
  dct_inverse<MAXB, MAXP>(cb, K, fb, g, P1);
  cheb_deriv(cb, ca, K, scan);
  dct_inverse<MAXB, MAXP>(ca, K, fb, g, P2);
  if (m > 0) {
    cheb_deriv(ca, cb, K, scan);
    dct_inverse<MAXB, MAXP>(cb, K, fb, g, P3);
  } else {
#pragma unroll
    for (int i = 0; i < MAXP; ++i) P3[i] = zero2();
  }
  for (int n = t; n < K; n += T) ca[n] = th[(size_t)m * K + n];
  __syncthreads();
  dct_inverse<MAXB, MAXP>(ca, K, fb, g, T0);
  cheb_deriv(ca, cb, K, scan);
  dct_inverse<MAXB, MAXP>(cb, K, fb, g, T1);

  const double dm = (double)m, m2 = dm * dm, so2 = g.s_o * g.s_o;
  double ek = 0.0, et = 0.0, ens = 0.0, ez = 0.0;
#pragma unroll
  for (int i = 0; i < MAXP; ++i) {
    const int k = t + i * T;
    if (k >= R) continue;
    const double s = g.half * g.xk[k] + g.mid;
    const double is = 1.0 / s;
    const double h2 = so2 - s * s;
    const double h2s = h2 * is;
    double2 F[6];
    double2 om;
    if (m > 0) {
      double2 LI = h2 * P2[i] + (h2s - 5.0 * s) * P1[i] - (6.0 + m2 * h2 * is * is) * P0[i];
      double2 dLI = h2 * P3[i] + (h2s - 7.0 * s) * P2[i]
                  - (so2 * is * is + 12.0 + m2 * h2 * is * is) * P1[i]
                  + (2.0 * m2 * so2 * is * is * is) * P0[i];
      om = make_double2(-LI.x, -LI.y);
      double2 dom = make_double2(-dLI.x, -dLI.y);
      double2 uph = (3.0 * s) * P0[i] - h2 * P1[i];
      F[0] = dm * times_i(P0[i]);
      F[1] = is * uph;
      F[2] = om + h2s * dom;
      F[3] = dm * times_i(om);
      F[4] = h2s * T1[i];
      F[5] = dm * times_i(T0[i]);
      if (diag) {
        const double w = g.wq[k];
        double us2 = h2s * h2s * m2 * (P0[i].x * P0[i].x + P0[i].y * P0[i].y);
        ek += 2.0 * w * (us2 + uph.x * uph.x + uph.y * uph.y);
        et += 2.0 * w * (T0[i].x * T0[i].x + T0[i].y * T0[i].y);
        ens += 2.0 * w * (om.x * om.x + om.y * om.y);
      }
    } else {
      // zonal flow u = P0, u' = P1, u'' = P2 (real)
      om = P1[i] + is * P0[i];
      double2 dom = P2[i] + is * P1[i] - (is * is) * P0[i];
      F[0] = zero2();
      F[1] = is * P0[i];
      F[2] = om + h2s * dom;
      F[3] = zero2();
      F[4] = h2s * (T1[i] + make_double2(g.dtc_coef * is, 0.0));
      F[5] = zero2();
      if (diag) {
        const double w = g.wq[k];
        ek += w * P0[i].x * P0[i].x;
        ez += w * P0[i].x * P0[i].x;
        et += w * T0[i].x * T0[i].x;
        ens += w * om.x * om.x;
      }
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) X[((size_t)f * R + k) * M + m] = F[f];
  }
  if (diag) {
    const double pi = 3.14159265358979323846;
    double bad = 0.0;
    for (int n = t; n < K; n += T) {
      double2 a = psi[(size_t)m * K + n], b = th[(size_t)m * K + n];
      if (!isfinite(a.x) || !isfinite(a.y) || !isfinite(b.x) || !isfinite(b.y)) bad = 1.0;
    }
    double s0 = block_sum(ek, red);
    double s1 = block_sum(ez, red);
    double s2 = block_sum(et, red);
    double s3 = block_sum(ens, red);
    double s4 = block_max(bad, red);
    if (t == 0) {
      diag[m * 8 + 0] = pi * s0;
      diag[m * 8 + 1] = pi * s1;
      diag[m * 8 + 2] = pi * s2;
      diag[m * 8 + 3] = 2.0 * pi * s3;
      diag[m * 8 + 4] = s4;
    }
  }
}

// ---------------------------------------------------------------- ring
// Per radial level: three complex inverse FFTs of length N_phi (each
// carries two real fields of similar size), the products
//   N_omega = dPsi/dphi c_w + v d omega/dphi,
//   N_theta = dPsi/dphi c_t + v d theta/dphi,
// then one real forward FFT per product (eq. ifft; N_omega can exceed
// N_theta by many orders of magnitude, so the two never share a complex
// transform), scaled by 1/N_phi and truncated to m <= N_m, and the zonal
// forcing mean(u_s omega) = 2 sum_{m>=1} Re(u_s,m conj(omega_m)).
// A real sequence x of length N goes through a complex FFT of length N/2 of
// z_j = x_2j + i x_2j+1:  X_k = (Z_k + Z*_{N/2-k})/2 - (i/2) w^k (Z_k - Z*_{N/2-k}),
// w = exp(-2 pi i / N).
template <int MAXB, int MAXJ>
__global__ void ring_kernel(Geom g, const double2* __restrict__ X, double2* __restrict__ NL,
                            double* __restrict__ zonal, double* __restrict__ rate) {
  extern __shared__ double2 fb[];
  __shared__ double red[16];
  const int R = g.R, M = g.M, nphi = g.nphi, nh = nphi / 2;
  const int T = blockDim.x, t = threadIdx.x;
  const int k = blockIdx.x;
  const double s = g.half * g.xk[k] + g.mid;
  const double h2s = (g.s_o * g.s_o - s * s) / s;
  double2 z1[MAXJ];
  double nw[MAXJ], nt[MAXJ];
  double rmax = 0.0;
  for (int q = 0; q < 3; ++q) {
    const double2* A = X + ((size_t)(2 * q) * R + k) * M;
    const double2* B = X + ((size_t)(2 * q + 1) * R + k) * M;
    for (int i = t; i < nphi; i += T) {
      double2 z = zero2();
      if (i < M) {
        double2 a = A[i], b = B[i];
        z = (i == 0) ? make_double2(a.x, b.x) : make_double2(a.x - b.y, a.y + b.x);
      } else if (i > nphi - M) {
        double2 a = A[nphi - i], b = B[nphi - i];
        z = make_double2(a.x + b.y, b.x - a.y);
      }
      fb[i] = z;
    }
    __syncthreads();
    fft_lds<MAXB>(fb, g.phi, +1);
#pragma unroll
    for (int i = 0; i < MAXJ; ++i) {
      int j = t + i * T;
      if (j >= nphi) continue;
      double2 z = fb[j];
      if (q == 0) {
        z1[i] = z;
        if (rate) rmax = fmax(rmax, fmax(h2s * fabs(z.x) / g.dsk[k], fabs(z.y) * nphi / (2.0 * 3.14159265358979323846)));
      } else if (q == 1) {
        nw[i] = z1[i].x * z.x + z1[i].y * z.y;
      } else {
        nt[i] = z1[i].x * z.x + z1[i].y * z.y;
      }
    }
    __syncthreads();
  }
  // real products, N_omega in doubles [0, nphi), N_theta in [nphi, 2 nphi)
  double* fr = reinterpret_cast<double*>(fb);
#pragma unroll
  for (int i = 0; i < MAXJ; ++i) {
    int j = t + i * T;
    if (j >= nphi) continue;
    fr[j] = nw[i];
    fr[nphi + j] = nt[i];
  }
  __syncthreads();
  fft_lds<MAXB>(fb, g.phi_half, -1);
  fft_lds<MAXB>(fb + nh, g.phi_half, -1);
  const double inv = 1.0 / nphi;
  for (int m = t; m < M; m += T) {
    const double2 w = g.phi.tw[m];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const double2* Z = fb + f * nh;
      double2 zk = Z[m % nh];
      double2 zc = Z[(nh - m % nh) % nh];
      zc.y = -zc.y;
      double2 e = 0.5 * (zk + zc);
      double2 d = zk - zc;
      double2 o = make_double2(0.5 * d.y, -0.5 * d.x);   // (Z_k - Z*)/(2i)
      double2 xm = e + cmul(w, o);
      if (m == 0) xm.y = 0.0;
      NL[((size_t)f * R + k) * M + m] = inv * xm;
    }
  }
  // zonal forcing from the spectral fields: u_s,m = (h^2/s) X0_m,
  // omega_m = X3_m / (i m)  =>  Re(u_s,m conj(omega_m)) = -(h^2/s) Im(X0 conj X3)/m
  const double2* A0 = X + ((size_t)0 * R + k) * M;
  const double2* A3 = X + ((size_t)3 * R + k) * M;
  double zs = 0.0;
  for (int m = 1 + t; m < M; m += T) {
    double2 a = A0[m], b = A3[m];
    zs += (a.y * b.x - a.x * b.y) / (double)m;
  }
  double tot = block_sum(zs, red);
  if (t == 0) zonal[k] = -2.0 * h2s * tot;
  if (rate) {
    double rm = block_max(rmax, red);
    if (t == 0) rate[k] = rm;
  }
}

// ------------------------------------------------------------ analysis
// Explicit right-hand sides at a stage state:
//   m >= 1: E_psi = C [ (Ra/Pr)(i m/s_o) theta + N_omega ]   (eq. psi_int)
//   m = 0:  E_u   = -D [ mean(u_s omega) ]                   (eq. uphi_int)
//   all m:  E_th  = -D [ N_theta ]                           (eq. temp_int)
template <int MAXB>
__global__ void analysis_kernel(Geom g, Bands b, const double2* __restrict__ NL,
                                const double* __restrict__ zonal,
                                const double2* __restrict__ th_state,
                                double2* __restrict__ Epsi, double2* __restrict__ Eth) {
  extern __shared__ double2 sm[];
  const int K = g.K, R = g.R, M = g.M, N = R - 1;
  const int T = blockDim.x, t = threadIdx.x;
  const int m = blockIdx.x;
  double2* ca = sm;
  double2* cb = sm + K;
  double2* fb = sm + 2 * K;
  if (m == 0)
    dct_forward<MAXB>([&](int kk) { return make_double2(zonal[kk], 0.0); }, ca, K, fb, g);
  else
    dct_forward<MAXB>([&](int kk) { return NL[((size_t)0 * R + kk) * M + m]; }, ca, K, fb, g);
  dct_forward<MAXB>([&](int kk) { return NL[((size_t)1 * R + kk) * M + m]; }, cb, K, fb, g);
  const double2* thm = th_state + (size_t)m * K;
  const double bcoef = g.Ra_Pr * (double)m / g.s_o;   // (Ra/Pr)(m/s_o), times i
  for (int k = t; k < K; k += T) {
    double2 ep = zero2(), et = zero2();
    const int lo = max(0, k - 8), hi = min(K - 1, k + 8);
    if (m > 0) {
      if (k >= 4)
        for (int n = lo; n <= hi; ++n) {
          double c = b.C[(size_t)(n - k + 8) * K + k];
          double2 v = ca[n] + bcoef * times_i(thm[n]);
          ep += c * v;
        }
    } else if (k >= 2) {
      for (int n = lo; n <= hi; ++n) ep -= b.D[(size_t)(n - k + 8) * K + k] * ca[n];
    }
    if (k >= 2)
      for (int n = lo; n <= hi; ++n) et -= b.D[(size_t)(n - k + 8) * K + k] * cb[n];
    Epsi[(size_t)m * K + k] = ep;
    Eth[(size_t)m * K + k] = et;
  }
}

// ----------------------------------------------------------------- rhs
// Right-hand side of one implicit solve, rows k >= p of every system:
//   rhs = (Mass + cL Lin) y_base + sum_q coef_q slot_q.
// Thread per (system, row); bands are offset-major ([17][K]).  System
// index: s < M - 1 is Psi of m = s + 1, s = M - 1 the zonal flow, s > M - 1
// theta of m = s - M.  Output rhs[s][K] (rows < p left zero).
__global__ void rhs_kernel(Geom g, Bands b, RhsSpec rs, double2* __restrict__ rhs) {
  const int K = g.K, M = g.M;
  const int s = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int kind = (s < M - 1) ? 0 : (s == M - 1 ? 1 : 2);
  const int m = (kind == 0) ? s + 1 : (kind == 1 ? 0 : s - M);
  const int P = (kind == 0) ? 4 : 2;
  double2 acc = zero2();
  if (k >= P) {
    const double2* yb = (kind == 2 ? rs.base_th : rs.base_psi) + (size_t)m * K;
    const double dm = (double)m, m2 = dm * dm, cL = rs.cL;
#pragma unroll
    for (int o = 0; o < 17; ++o) {
      const int nn = k + o - 8;
      if (nn < 0 || nn >= K) continue;
      const size_t idx = (size_t)o * K + k;
      double re, im = 0.0;
      if (kind == 0) {
        re = b.A0[idx] + m2 * b.A2[idx] + cL * (b.B0[idx] + m2 * b.B2[idx] + m2 * m2 * b.B4[idx]);
        im = cL * g.two_over_E * dm * b.C[idx];
      } else if (kind == 1) {
        re = b.D[idx] + cL * (b.F0[idx] + b.F2[idx]);
      } else {
        re = b.D[idx] + cL * g.inv_Pr * (b.F0[idx] + m2 * b.F2[idx]);
      }
      acc += cmul(make_double2(re, im), yb[nn]);
    }
#pragma unroll
    for (int q = 0; q < MAX_TERMS; ++q) {
      if (q < rs.nterm) {
        const double2* src = (kind == 2 ? rs.term_th[q] : rs.term_psi[q]) + (size_t)m * K;
        acc += rs.coef[q] * src[k];
      }
    }
  }
  rhs[(size_t)s * K + k] = acc;
}

// --------------------------------------------------------------- solve
// One wavefront per bordered system (same system index as rhs_kernel):
// psi_1 = -Minv (w . h), h <- h - C psi_1, then the band LU solve with row
// interchanges (forward, LAPACK gbtrs order) and back substitution.
//
// Lane t holds position q = t (mod 64) of a 64-wide window of the
// right-hand side.  Each step reads the pivot row with readlane, swaps with
// writelane, and updates the lanes below (above) it with one FMA.  Factor
// columns are staged in LDS in double-buffered batches of B steps (factor
// arrays padded to whole batches with identity steps), and the window is
// refilled from global memory with loads issued a batch ahead.  KUT is the
// number of stored U super-diagonals (ku plus the largest pivot offset).
constexpr int SOLVE_BATCH = 16;

template <typename TF, int N>
struct Regs { TF v[N]; };

// The AMDGPU writelane intrinsic (lane `lane` of v takes the uniform value
// x), reached through its LLVM name since this clang has no builtin for it.
__device__ int llvm_amdgcn_writelane(int x, int lane, int v) __asm("llvm.amdgcn.writelane.i32");
__device__ __forceinline__ int writelane_i(int v, int x, int lane) {
  return llvm_amdgcn_writelane(x, lane, v);
}
__device__ __forceinline__ double writelane_d(double v, double x, int lane) {
  long long bv = __double_as_longlong(v), bx = __double_as_longlong(x);
  int lo = writelane_i((int)(bv & 0xffffffffLL), (int)(bx & 0xffffffffLL), lane);
  int hi = writelane_i((int)(bv >> 32), (int)(bx >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double2 writelane2(double2 v, double2 x, int lane) {
  return make_double2(writelane_d(v.x, x.x, lane), writelane_d(v.y, x.y, lane));
}

template <typename TF, int P, int KL, int KUT>
__device__ void solve_system(const Geom& g, const FactorSet<TF>& F, double2* rhs,
                             const RhsSpec& rs, int kind, int sys, int so, double2* sm) {
  constexpr int WU = KUT + 1;
  constexpr int B = SOLVE_BATCH;
  constexpr int LPL = (B * KL + 63) / 64;
  constexpr int UPL = (B * WU + 63) / 64;
  const int K = g.K, M = g.M, n = K - P;
  const int npad = (n + B - 1) / B * B;
  const int t = threadIdx.x;
  const int m = (kind == 0) ? sys + 1 : (kind == 1 ? 0 : sys - M);
  TF* Lst = reinterpret_cast<TF*>(sm);            // [2][B*KL]
  TF* Ust = Lst + 2 * B * KL;                     // [2][B*WU]
  double2* hg = rhs + (size_t)sys * K + P;        // h, then y, then x (n entries)
  auto hat = [&](int q) { return (q >= 0 && q < n) ? hg[q] : zero2(); };

  // Schur complement for the p boundary unknowns
  double2 wh[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    double2 acc = zero2();
    const TF* wr = F.W + ((size_t)so * P + i) * n;
    for (int j = t; j < n; j += 64) acc += mulf(wr[j], hg[j]);
    for (int off = 32; off > 0; off >>= 1) {
      acc.x += __shfl_xor(acc.x, off);
      acc.y += __shfl_xor(acc.y, off);
    }
    wh[i] = acc;
  }
  double2 psi1[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    double2 acc = zero2();
#pragma unroll
    for (int i2 = 0; i2 < P; ++i2) acc -= mulf(F.Minv[((size_t)so * P + i) * P + i2], wh[i2]);
    psi1[i] = acc;
  }
  double2 bw = hat(t);
  if (t < KL) {
#pragma unroll
    for (int i = 0; i < P; ++i) bw -= mulf(F.Cb[((size_t)so * KL + t) * P + i], psi1[i]);
  }

  const int* piv = F.piv + (size_t)so * npad;
  const TF* Lc = F.Lc + (size_t)so * npad * KL;
  const TF* Uc = F.Uc + (size_t)so * npad * WU;
  const int nb = npad / B;

  // ---- forward elimination
  Regs<TF, LPL> lr;
#pragma unroll
  for (int i = 0; i < LPL; ++i) {
    const int idx = t + 64 * i;
    if (idx < B * KL) Lst[idx] = Lc[idx];
  }
  int pv_cur = (t < B) ? piv[t] : 0;
  // window refill prefetch: the lane retiring at the end of batch bi
  // holds position q = j0 + ((t - j0) & 63) < j0 + B and takes q + 64
  double2 hn = hat(t + 64);   // used by the lanes retiring after batch 0
  __syncthreads();
  for (int bi = 0; bi < nb; ++bi) {
    const int j0 = bi * B;
    const TF* Lcur = Lst + (bi & 1) * B * KL;
    int pv_next = 0;
    if (bi + 1 < nb) {
#pragma unroll
      for (int i = 0; i < LPL; ++i) {
        const int idx = t + 64 * i;
        lr.v[i] = (idx < B * KL) ? Lc[(size_t)(j0 + B) * KL + idx] : tzero<TF>();
      }
      pv_next = (t < B) ? piv[j0 + B + t] : 0;
    }
#pragma unroll
    for (int jj = 0; jj < B; ++jj) {
      const int j = j0 + jj;
      const int p = __builtin_amdgcn_readlane(pv_cur, jj);
      const int src = j & 63;
      const int dst = (j + p) & 63;
      const int d = ((t - j) & 63) - 1;
      const bool act = (d >= 0 && d < KL);
      const TF l = Lcur[jj * KL + (act ? d : 0)];
      const double2 a = readlane2(bw, src);
      const double2 bj = readlane2(bw, dst);
      bw = writelane2(bw, a, dst);
      bw = writelane2(bw, bj, src);
      if (act) bw -= mulf(l, bj);
    }
    // positions j0..j0+B-1 are final
    const int q = j0 + ((t - j0) & 63);
    const bool retire = (q < j0 + B);
    if (retire && q < n) hg[q] = bw;
    if (retire) bw = hn;
    // the lanes retiring after the next batch prefetch their new position
    const int q2 = j0 + B + ((t - j0 - B) & 63);
    if (q2 < j0 + 2 * B) hn = hat(q2 + 64);
    if (bi + 1 < nb) {
      TF* Lnext = Lst + ((bi + 1) & 1) * B * KL;
#pragma unroll
      for (int i = 0; i < LPL; ++i) {
        const int idx = t + 64 * i;
        if (idx < B * KL) Lnext[idx] = lr.v[i];
      }
    }
    pv_cur = pv_next;
    __syncthreads();
  }

  // ---- back substitution (column oriented), batches from the bottom
  Regs<TF, UPL> ur;
#pragma unroll
  for (int i = 0; i < UPL; ++i) {
    const int idx = t + 64 * i;
    if (idx < B * WU) Ust[idx] = Uc[(size_t)(npad - B) * WU + idx];
  }
  // y was written to global memory by other lanes: make it visible
  __threadfence();
  {
    const int top = npad - 1;
    const int q0 = top - ((top - t) & 63);
    bw = hat(q0);
    hn = hat(q0 - 64);   // used by the lanes retiring after batch 0
  }
  __syncthreads();
  for (int bi = 0; bi < nb; ++bi) {
    const int c0 = npad - (bi + 1) * B;   // first column of this batch
    const TF* Ucur = Ust + (bi & 1) * B * WU;
    if (bi + 1 < nb) {
#pragma unroll
      for (int i = 0; i < UPL; ++i) {
        const int idx = t + 64 * i;
        ur.v[i] = (idx < B * WU) ? Uc[(size_t)(c0 - B) * WU + idx] : tzero<TF>();
      }
    }
#pragma unroll
    for (int jj = B - 1; jj >= 0; --jj) {
      const int j = c0 + jj;
      const int src = j & 63;
      const int e = (j - t) & 63;
      const bool act = (e >= 1 && e <= KUT);
      const TF* urow = Ucur + jj * WU;
      const TF uj = urow[act ? e : 0];
      const double2 xj = mulf(urow[0], readlane2(bw, src));
      bw = writelane2(bw, xj, src);
      if (act) bw -= mulf(uj, xj);
    }
    const int j1 = c0 + B - 1;
    const int q = j1 - ((j1 - t) & 63);
    const bool retire = (q >= c0);
    if (retire && q < n) hg[q] = bw;
    if (retire) bw = hn;
    const int q2 = (c0 - 1) - ((c0 - 1 - t) & 63);   // retiring after the next batch
    if (q2 >= c0 - B) hn = hat(q2 - 64);
    if (bi + 1 < nb) {
      TF* Unext = Ust + ((bi + 1) & 1) * B * WU;
#pragma unroll
      for (int i = 0; i < UPL; ++i) {
        const int idx = t + 64 * i;
        if (idx < B * WU) Unext[idx] = ur.v[i];
      }
    }
    __syncthreads();
  }

  // ---- new state
  __threadfence();
  double2* out = (kind == 2 ? rs.out_th : rs.out_psi) + (size_t)m * K;
  const bool real_row = (kind != 0 && m == 0);   // zonal flow and theta_0
  for (int k = t; k < K; k += 64) {
    double2 v = zero2();
#pragma unroll
    for (int i = 0; i < P; ++i)
      if (k == i) v = psi1[i];
    if (k >= P) v = hg[k - P];
    if (real_row) v.y = 0.0;
    out[k] = v;
  }
}

template <int KUTP, int KUTR>
__global__ __launch_bounds__(64) void solve_all_kernel(Geom g, FactorSet<double2> Fp,
                                                       FactorSet<double> Fr, double2* rhs,
                                                       RhsSpec rs) {
  extern __shared__ double2 sm[];
  const int blk = blockIdx.x, M = g.M;
  if (blk < M - 1) solve_system<double2, 4, 8, KUTP>(g, Fp, rhs, rs, 0, blk, blk, sm);
  else solve_system<double, 2, 4, KUTR>(g, Fr, rhs, rs, blk == M - 1 ? 1 : 2, blk,
                                        blk - (M - 1), sm);
}

// Lin y_new for BPR353 stages (rows >= p), thread per (system, row).
__global__ void lin_kernel(Geom g, Bands b, const double2* __restrict__ ypsi,
                           const double2* __restrict__ yth, double2* __restrict__ lpsi,
                           double2* __restrict__ lth) {
  const int K = g.K, M = g.M;
  const int s = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int kind = (s < M - 1) ? 0 : (s == M - 1 ? 1 : 2);
  const int m = (kind == 0) ? s + 1 : (kind == 1 ? 0 : s - M);
  const int P = (kind == 0) ? 4 : 2;
  const double2* y = (kind == 2 ? yth : ypsi) + (size_t)m * K;
  double2 acc = zero2();
  if (k >= P) {
    const double dm = (double)m, m2 = dm * dm;
#pragma unroll
    for (int o = 0; o < 17; ++o) {
      const int nn = k + o - 8;
      if (nn < 0 || nn >= K) continue;
      const size_t idx = (size_t)o * K + k;
      double re, im = 0.0;
      if (kind == 0) {
        re = b.B0[idx] + m2 * b.B2[idx] + m2 * m2 * b.B4[idx];
        im = g.two_over_E * dm * b.C[idx];
      } else if (kind == 1) {
        re = b.F0[idx] + b.F2[idx];
      } else {
        re = g.inv_Pr * (b.F0[idx] + m2 * b.F2[idx]);
      }
      acc += cmul(make_double2(re, im), y[nn]);
    }
  }
  (kind == 2 ? lth : lpsi)[(size_t)m * K + k] = acc;
}

// ------------------------------------------------------------ launchers
template <int MAXB, int MAXP>
void launch_synth_t(const Geom& g, const double2* psi, const double2* th, double2* X,
                    double* diag, int threads, hipStream_t st) {
  size_t shm = sizeof(double2) * (2 * g.K + 2 * (g.R - 1) + 2 * threads);
  hipLaunchKernelGGL((synth_kernel<MAXB, MAXP>), dim3(g.M), dim3(threads), shm, st, g, psi, th, X,
                     diag);
}

void launch_synth(const Geom& g, const double2* psi, const double2* th, double2* X, double* diag,
                  int threads, hipStream_t st) {
  if (threads <= 256) launch_synth_t<4, 5>(g, psi, th, X, diag, threads, st);
  else launch_synth_t<4, 5>(g, psi, th, X, diag, threads, st);
}

void launch_ring(const Geom& g, const double2* X, double2* NL, double* zonal, double* rate,
                 int threads, hipStream_t st) {
  size_t shm = sizeof(double2) * g.nphi;
  hipLaunchKernelGGL((ring_kernel<4, 16>), dim3(g.R), dim3(threads), shm, st, g, X, NL, zonal, rate);
}

void launch_analysis(const Geom& g, const Bands& b, const double2* NL, const double* zonal,
                     const double2* th_state, double2* Epsi, double2* Eth, int threads,
                     hipStream_t st) {
  size_t shm = sizeof(double2) * (2 * g.K + 2 * (g.R - 1));
  hipLaunchKernelGGL((analysis_kernel<4>), dim3(g.M), dim3(threads), shm, st, g, b, NL, zonal,
                     th_state, Epsi, Eth);
}

size_t solve_lds_bytes(const Geom& g, int kutp, int kutr) {
  const int B = SOLVE_BATCH;
  const size_t psi = sizeof(double2) * 2 * B * (8 + kutp + 1);
  const size_t real = sizeof(double) * 2 * B * (4 + kutr + 1);
  return psi > real ? psi : real;
}

int solve_batch() { return SOLVE_BATCH; }

void launch_rhs(const Geom& g, const Bands& b, const RhsSpec& rs, double2* rhs, hipStream_t st) {
  dim3 grid((g.K + 255) / 256, 2 * g.M);
  hipLaunchKernelGGL(rhs_kernel, grid, dim3(256), 0, st, g, b, rs, rhs);
}

void launch_lin(const Geom& g, const Bands& b, const double2* ypsi, const double2* yth,
                double2* lpsi, double2* lth, hipStream_t st) {
  dim3 grid((g.K + 255) / 256, 2 * g.M);
  hipLaunchKernelGGL(lin_kernel, grid, dim3(256), 0, st, g, b, ypsi, yth, lpsi, lth);
}

bool launch_solve(const Geom& g, const FactorSet<double2>& Fp, const FactorSet<double>& Fr,
                  double2* rhs, const RhsSpec& rs, int kutp, int kutr, hipStream_t st) {
  const size_t shm = solve_lds_bytes(g, kutp, kutr);
  const dim3 grid(2 * g.M), block(64);
  if (kutp == 12 && kutr == 4)
    hipLaunchKernelGGL((solve_all_kernel<12, 4>), grid, block, shm, st, g, Fp, Fr, rhs, rs);
  else if (kutp == 16 && kutr == 8)
    hipLaunchKernelGGL((solve_all_kernel<16, 8>), grid, block, shm, st, g, Fp, Fr, rhs, rs);
  else
    return false;
  return true;
}

}  // namespace qg
