// Device helpers shared by the transform kernels of the step
// (transforms.hip) and their transposes (reverse.hip): complex arithmetic,
// launch geometry, the register-output FFT wrapper, the in-place Chebyshev
// derivative and block reductions; and the host-side launch helpers.
#pragma once
#include <hip/hip_runtime.h>

#include "fft.h"
#include "kernels.h"

namespace qg {
namespace {
__device__ __forceinline__ double2 add2(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 sub2(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 scl2(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 ix(double m, double2 a) { return make_double2(-m * a.y, m * a.x); }  // i m a
__device__ __forceinline__ double2 z2() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double abs2(double2 a) { return a.x * a.x + a.y * a.y; }

constexpr int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
constexpr int threads_dct(int n2) { return clampi(n2 / 8, 64, 256); }
constexpr int threads_phi(int nphi) { return clampi(nphi / 12, 64, 256); }

// Waves per SIMD asked of the register allocator for a kernel of T-thread
// blocks that hold `lds` bytes of LDS each: as many as the CU's 160 KiB of
// LDS lets run at once, at most 3.  Fewer registers than the allocator
// would pick unconstrained cost a few spills, and the third wave per SIMD
// hides more of the latency of the barriers and memory accesses between
// the transform passes (3072 x 1025: synthesis 96 -> 86 us, ring 111 ->
// 98 us, bit for bit the same results).  Where one block fills the LDS the
// allocator stays unconstrained.
constexpr int lds_waves(size_t lds, int T) {
  const int blocks = (int)((160 * 1024) / lds);
  return clampi(blocks * (T / 64) / 4, 1, 3);
}

// Block -> m: XCD x = block mod 8 takes the contiguous range [x per, (x+1) per).
__device__ __forceinline__ int xcd_index_of(int b, int count) {
  const int per = (count + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}
__device__ __forceinline__ int xcd_index(int count) { return xcd_index_of(blockIdx.x, count); }
inline int xcd_grid(int count) { return 8 * ((count + 7) / 8); }

// Hides a value from the optimiser for one use: the per-point factors of
// the derivative loops would otherwise be hoisted out of those loops for all
// points at once and held in registers for the whole kernel.
__device__ __forceinline__ void opaque(double& s, int& k) {
  asm volatile("" : "+v"(s), "+v"(k));
}

// FP64 <-> transform precision
template <typename C> __device__ __forceinline__ C to_c(double2 v);
template <> __device__ __forceinline__ double2 to_c<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 to_c<float2>(double2 v) {
  return make_float2((float)v.x, (float)v.y);
}
__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }
template <typename C> __device__ __forceinline__ C zc() { return to_c<C>(make_double2(0.0, 0.0)); }

// Twiddle tables of the transform precision.
template <typename C> struct Tw;
template <> struct Tw<double2> {
  static __device__ __forceinline__ const double2* dct(const Geom& g) { return g.tw_dct; }
  static __device__ __forceinline__ const double2* phi(const Geom& g) { return g.tw_phi; }
  static __device__ __forceinline__ const double2* half(const Geom& g) { return g.tw_half; }
  static __device__ __forceinline__ const double2* w(const Geom& g) { return g.w_phi; }
};
template <> struct Tw<float2> {
  static __device__ __forceinline__ const float2* dct(const Geom& g) { return g.tw_dct32; }
  static __device__ __forceinline__ const float2* phi(const Geom& g) { return g.tw_phi32; }
  static __device__ __forceinline__ const float2* half(const Geom& g) { return g.tw_half32; }
  static __device__ __forceinline__ const float2* w(const Geom& g) { return g.w_phi32; }
};

// Byte offset of the FP64 coefficient buffer after n transform slots.
template <typename C>
constexpr size_t coef_offset(int slots) {
  return ((size_t)slots * sizeof(C) + 15) / 16 * 16;
}

__device__ __forceinline__ double2 shfl_down2(double2 v, int off) {
  return make_double2(__shfl_down(v.x, off), __shfl_down(v.y, off));
}

// Transform with outputs in registers, out[i] = X_{t + i T} (zero past n).
template <int n, int T>
constexpr int out_count() { return (n + T - 1) / T; }

template <int n, int T, int SGN, typename C, typename Get>
__device__ __forceinline__ void fft_out(Get get, C* buf, const C* __restrict__ tw,
                                        C (&out)[out_count<n, T>()]) {
  if constexpr (reg_out_ok<n, T>()) {
    fft_to_regs<n, T, SGN>(get, buf, tw, out);
  } else {
    fft_to_lds<n, T, SGN>(get, buf, tw);
#pragma unroll
    for (int i = 0; i < out_count<n, T>(); ++i) {
      const int k = threadIdx.x + i * T;
      out[i] = (k < n) ? buf[lds_pad(k)] : zc<C>();
    }
  }
}

// In-place Chebyshev derivative d/ds on the unit gap (ds = dx / 2):
// c'_n = (4 / c_n) sum_{j > n, j - n odd} j c_j, c_0 = 2, else 1.  Each
// thread takes a run of (even, odd) index pairs; the suffix sums over the
// runs of later threads come from a wavefront scan and one LDS exchange.
// Ends with a barrier.
template <int T>
__device__ void cheb_deriv_inplace(double2* c, int K, double2* wred) {
  constexpr int NW = T / 64;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int npair = (K + 1) / 2;
  const int ch = (npair + T - 1) / T;
  const int p0 = min(npair, t * ch), p1 = min(npair, p0 + ch);
  double2 se = z2(), so = z2();
  for (int p = p0; p < p1; ++p) {
    const int je = 2 * p, jo = je + 1;
    se = add2(se, scl2((double)je, c[je]));
    if (jo < K) so = add2(so, scl2((double)jo, c[jo]));
  }
  // exclusive suffix sums over the lanes above this one
  double2 xe = shfl_down2(se, 1), xo = shfl_down2(so, 1);
  if (lane == 63) xe = xo = z2();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double2 ue = shfl_down2(xe, off), uo = shfl_down2(xo, off);
    if (lane + off < 64) {
      xe = add2(xe, ue);
      xo = add2(xo, uo);
    }
  }
  if (lane == 0) {
    wred[2 * w] = add2(xe, se);
    wred[2 * w + 1] = add2(xo, so);
  }
  __syncthreads();
  double2 re = xe, ro = xo;
  for (int w2 = w + 1; w2 < NW; ++w2) {
    re = add2(re, wred[2 * w2]);
    ro = add2(ro, wred[2 * w2 + 1]);
  }
  for (int p = p1 - 1; p >= p0; --p) {
    const int je = 2 * p, jo = je + 1;
    const double2 ae = c[je];
    const double2 ao = (jo < K) ? c[jo] : z2();
    if (jo < K) c[jo] = scl2(4.0, re);       // S_even(p + 1)
    ro = add2(ro, scl2((double)jo, ao));     // S_odd(p)
    c[je] = scl2(je == 0 ? 2.0 : 4.0, ro);
    re = add2(re, scl2((double)je, ae));     // S_even(p)
  }
  __syncthreads();
}

__device__ inline double block_sum(double v, double* red) {
  const int t = threadIdx.x, T = blockDim.x;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (T + 63) / 64; ++w) s += red[w];
  return s;
}

__device__ inline double block_max(double v, double* red) {
  const int t = threadIdx.x, T = blockDim.x;
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  __syncthreads();
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (T + 63) / 64; ++w) s = fmax(s, red[w]);
  return s;
}

template <typename Kern>
void allow_lds(Kern k, size_t bytes) {
  if (bytes > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename C>
size_t dct_lds(int n2, int K) { return coef_offset<C>(lds_slots(n2)) + sizeof(double2) * K; }
template <typename C>
size_t phi_lds(int nphi) { return sizeof(C) * lds_slots(nphi); }
// The analysis writes its coefficients over the transform buffer.
template <typename C>
size_t analysis_lds(int n2, int K) {
  const size_t a = sizeof(C) * lds_slots(n2), b = sizeof(double2) * K;
  return a > b ? a : b;
}

}  // namespace
}  // namespace qg
