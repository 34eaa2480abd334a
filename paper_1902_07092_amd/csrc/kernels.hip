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
          double c = b.C[k * 17 + (n - k + 8)];
          double2 v = ca[n] + bcoef * times_i(thm[n]);
          ep += c * v;
        }
    } else if (k >= 2) {
      for (int n = lo; n <= hi; ++n) ep -= b.D[k * 17 + (n - k + 8)] * ca[n];
    }
    if (k >= 2)
      for (int n = lo; n <= hi; ++n) et -= b.D[k * 17 + (n - k + 8)] * cb[n];
    Epsi[(size_t)m * K + k] = ep;
    Eth[(size_t)m * K + k] = et;
  }
}

// --------------------------------------------------------------- solve
// One wavefront per bordered system.  kind 0: Psi of m = blockIdx.x + 1
// (complex matrix A_m - a dt B_m, p = 4, band 8/8).  kind 1: blockIdx.x = 0
// is the zonal flow (D - a dt E), blockIdx.x = 1 + m is theta of m
// (D - a dt F_m / Pr); real matrices, p = 2, band 4/4.
template <typename TF, int P, int KL, int KU>
__global__ __launch_bounds__(64) void solve_kernel(Geom g, Bands b, FactorSet<TF> F,
                                                   RhsSpec rs, int kind) {
  constexpr int KUT = KL + KU;
  constexpr int WU = KUT + 1;
  constexpr int BATCH = 32;
  extern __shared__ double2 sm[];
  const int K = g.K, n = K - P;
  const int t = threadIdx.x;
  const int sys = blockIdx.x;
  int m;
  bool is_psi_row;   // state row lives in the psi array (Psi or zonal flow)
  if (kind == 0) { m = sys + 1; is_psi_row = true; }
  else if (sys == 0) { m = 0; is_psi_row = true; }
  else { m = sys - 1; is_psi_row = false; }
  const bool zonal = (kind == 1 && sys == 0);
  double2* yb = sm;                 // K: base state, later the new state
  double2* hb = sm + K;             // n: right-hand side / solution
  TF* Lst = reinterpret_cast<TF*>(hb + n);
  TF* Ust = Lst + BATCH * KL;
  int* pst = reinterpret_cast<int*>(Ust + BATCH * WU);

  const double2* ybase = (is_psi_row ? rs.base_psi : rs.base_th) + (size_t)m * K;
  for (int k = t; k < K; k += 64) yb[k] = ybase[k];
  __syncthreads();

  const double dm = (double)m, m2 = dm * dm;
  // banded coefficient of (Mass + c Lin) at (k, n); Psi has an imaginary
  // Coriolis part (2 m / E) C in Lin.
  auto coef = [&](int k, int off, double c, double& re, double& im) {
    const int idx = k * 17 + off + 8;
    if (kind == 0) {
      re = b.A0[idx] + m2 * b.A2[idx] + c * (b.B0[idx] + m2 * b.B2[idx] + m2 * m2 * b.B4[idx]);
      im = c * g.two_over_E * dm * b.C[idx];
    } else if (zonal) {
      re = b.D[idx] + c * (b.F0[idx] + b.F2[idx]);
      im = 0.0;
    } else {
      re = b.D[idx] + c * g.inv_Pr * (b.F0[idx] + m2 * b.F2[idx]);
      im = 0.0;
    }
  };
  // right-hand side, rows k >= P
  for (int k = P + t; k < K; k += 64) {
    double2 acc = zero2();
    const int lo = max(0, k - 8), hi = min(K - 1, k + 8);
    for (int nn = lo; nn <= hi; ++nn) {
      double re, im;
      coef(k, nn - k, rs.cL, re, im);
      acc += cmul(make_double2(re, im), yb[nn]);
    }
    for (int q = 0; q < rs.nterm; ++q) {
      const double2* src = (is_psi_row ? rs.term_psi[q] : rs.term_th[q]) + (size_t)m * K;
      acc += rs.coef[q] * src[k];
    }
    hb[k - P] = acc;
  }
  __syncthreads();

  const size_t so = (size_t)sys;
  // Schur complement for the p boundary unknowns: psi_1 = -Minv (w . h)
  double2 wh[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    double2 acc = zero2();
    const TF* wr = F.W + (so * P + i) * n;
    for (int j = t; j < n; j += 64) acc += mulf(wr[j], hb[j]);
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
    for (int i2 = 0; i2 < P; ++i2) acc -= mulf(F.Minv[(so * P + i) * P + i2], wh[i2]);
    psi1[i] = acc;
  }
  if (t < KL && t < n) {
    double2 acc = hb[t];
#pragma unroll
    for (int i = 0; i < P; ++i) acc -= mulf(F.Cb[(so * KL + t) * P + i], psi1[i]);
    hb[t] = acc;
  }
  __syncthreads();

  // ---- forward elimination with row interchanges (LAPACK gbtrs order)
  const int* piv = F.piv + so * n;
  const TF* Lc = F.Lc + so * n * KL;
  const TF* Uc = F.Uc + so * n * WU;
  double2 bw = (t < n) ? hb[t] : zero2();
  for (int j0 = 0; j0 < n; j0 += BATCH) {
    const int jend = min(BATCH, n - j0);
    for (int idx = t; idx < BATCH * KL; idx += 64) {
      int jj = idx / KL;
      Lst[idx] = (jj < jend) ? Lc[(size_t)(j0 + jj) * KL + (idx % KL)] : tzero<TF>();
    }
    if (t < BATCH) pst[t] = (t < jend) ? piv[j0 + t] : 0;
    __syncthreads();
    for (int jj = 0; jj < jend; ++jj) {
      const int j = j0 + jj;
      const int p = __builtin_amdgcn_readfirstlane(pst[jj]);
      const int src = j & 63;
      if (p != 0) {
        const int dst = (j + p) & 63;
        double2 a = readlane2(bw, src), c = readlane2(bw, dst);
        if (t == src) bw = c;
        else if (t == dst) bw = a;
      }
      const double2 bj = readlane2(bw, src);
      const int d = ((t - j) & 63) - 1;
      if (d >= 0 && d < KL && j + 1 + d < n) bw -= mulf(Lst[jj * KL + d], bj);
    }
    const int q = j0 + ((t - j0) & 63);
    if (q < j0 + BATCH && q < n) {
      hb[q] = bw;
      const int q2 = q + 64;
      bw = (q2 < n) ? hb[q2] : zero2();
    }
    __syncthreads();
  }

  // ---- back substitution with U (column oriented)
  {
    const int top = n - 1;
    const int q0 = top - ((top - t) & 63);
    bw = (q0 >= 0) ? hb[q0] : zero2();
  }
  for (int j1 = n - 1; j1 >= 0; j1 -= BATCH) {
    const int jend = min(BATCH, j1 + 1);
    for (int idx = t; idx < BATCH * WU; idx += 64) {
      int jj = idx / WU;
      Ust[idx] = (jj < jend) ? Uc[(size_t)(j1 - jj) * WU + (idx % WU)] : tzero<TF>();
    }
    __syncthreads();
    for (int jj = 0; jj < jend; ++jj) {
      const int j = j1 - jj;
      const int src = j & 63;
      const double2 xj = mulf(Ust[jj * WU], readlane2(bw, src));
      if (t == src) bw = xj;
      const int e = (j - t) & 63;
      if (e >= 1 && e <= KUT && j - e >= 0) bw -= mulf(Ust[jj * WU + e], xj);
    }
    const int q = j1 - ((j1 - t) & 63);
    if (q > j1 - BATCH && q >= 0) {
      hb[q] = bw;
      const int q2 = q - 64;
      bw = (q2 >= 0) ? hb[q2] : zero2();
    }
    __syncthreads();
  }

  // ---- new state
  double2* out = (is_psi_row ? rs.out_psi : rs.out_th) + (size_t)m * K;
  const bool real_row = (kind == 1 && m == 0);   // zonal flow and theta_0
  for (int k = t; k < K; k += 64) {
    double2 v = (k < P) ? psi1[k] : hb[k - P];
    if (real_row) v.y = 0.0;
    yb[k] = v;
    out[k] = v;
  }
  double2* lin = is_psi_row ? rs.lin_psi : rs.lin_th;
  if (lin) {
    __syncthreads();
    lin += (size_t)m * K;
    for (int k = t; k < K; k += 64) {
      double2 acc = zero2();
      if (k >= P) {
        const int lo = max(0, k - 8), hi = min(K - 1, k + 8);
        for (int nn = lo; nn <= hi; ++nn) {
          double re0, im0, re1, im1;
          coef(k, nn - k, 0.0, re0, im0);
          coef(k, nn - k, 1.0, re1, im1);
          acc += cmul(make_double2(re1 - re0, im1 - im0), yb[nn]);
        }
      }
      lin[k] = acc;
    }
  }
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

void launch_solve_psi(const Geom& g, const Bands& b, const FactorSet<double2>& F,
                      const RhsSpec& rs, hipStream_t st) {
  const int n = g.K - 4;
  size_t shm = sizeof(double2) * (g.K + n) + sizeof(double2) * 32 * (8 + 17) + sizeof(int) * 32;
  hipLaunchKernelGGL((solve_kernel<double2, 4, 8, 8>), dim3(g.M - 1), dim3(64), shm, st, g, b, F, rs,
                     0);
}

void launch_solve_real(const Geom& g, const Bands& b, const FactorSet<double>& F,
                       const RhsSpec& rs, hipStream_t st) {
  const int n = g.K - 2;
  size_t shm = sizeof(double2) * (g.K + n) + sizeof(double) * 32 * (4 + 9) + sizeof(int) * 32;
  hipLaunchKernelGGL((solve_kernel<double, 2, 4, 4>), dim3(g.M + 1), dim3(64), shm, st, g, b, F, rs,
                     1);
}

}  // namespace qg
