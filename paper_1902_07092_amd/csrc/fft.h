// Block-wide FFTs in LDS for the transforms of the QG step (eq. fft,
// eq. ifft in azimuth; the even extension behind eq. cheb / eq. icheb in
// radius), FP64 (double2) or FP32 (float2), compile-time radix plans for
// gfx950.
//
// A length-n transform runs as Stockham passes of radix 16, 8, 4, 3 or 2.
// A pass reads its butterfly inputs x[j + r n/R] into registers, applies
// the twiddles w_{Ns R}^{(j mod Ns) r}, does the R-point DFT in registers
// and writes y[(j / Ns) Ns R + (j mod Ns) + r Ns].  The first pass takes
// its inputs from a caller functor (global memory or another LDS array),
// and the last pass can leave its outputs in registers: thread t then owns
// the outputs k = t + i T, i < n / T.  LDS slots are permuted within each
// aligned group of eight (lds_pad) so that both the contiguous reads and
// the strided first-pass writes spread over the banks.
//
// Twiddle tables: pass s (Ns = product of the radices before it) reads
// tw[(Ns - 1) + (r - 1) Ns + k] = exp(-2 pi i k r / (Ns R)), k < Ns,
// 1 <= r < R; a whole plan needs n - 1 entries.
#pragma once
#include <hip/hip_runtime.h>

namespace qg {

struct RadixPlan {
  int np;
  int r[8];
};

// n = 2^a or 3 * 2^a: radix 8 passes, one 16 (a = 1 mod 3) or 4
// (a = 2 mod 3) pass, and the factor 3 as the last pass.
constexpr RadixPlan radix_plan(int n) {
  RadixPlan p{0, {0, 0, 0, 0, 0, 0, 0, 0}};
  const int three = (n % 3 == 0) ? 1 : 0;
  const int m = three ? n / 3 : n;
  int a = 0;
  while ((1 << a) < m) ++a;
  int q = a / 3;
  const int rem = a % 3;
  if (rem == 1) {
    if (q >= 1) {
      p.r[p.np++] = 16;
      q -= 1;
    } else {
      p.r[p.np++] = 2;
    }
  }
  for (int i = 0; i < q; ++i) p.r[p.np++] = 8;
  if (rem == 2) p.r[p.np++] = 4;
  if (three) p.r[p.np++] = 3;
  return p;
}

constexpr int plan_ns(const RadixPlan& p, int s) {
  int ns = 1;
  for (int i = 0; i < s; ++i) ns *= p.r[i];
  return ns;
}

constexpr bool plan_valid(int n) {
  const RadixPlan p = radix_plan(n);
  return p.np > 0 && plan_ns(p, p.np) == n;
}

// LDS slot of transform element i.  gfx950 serves a 16-byte LDS read in
// phases of 16 lanes and a 16-byte write in phases of 8 lanes; a phase is
// free of bank conflicts when its slots differ modulo 16 (reads) or 8
// (writes).  The low three bits of i are XORed with a function of bits 3..6
// that is one-to-one both in bits 3..5 and in bits 4..6: contiguous runs
// stay a permutation of their aligned groups (reads and the writes of
// passes with Ns >= 8), and the first pass's writes at stride 8 (radix 8)
// or 16 (radix 16) land on eight different slots modulo 8.  A padding of
// one slot per eight, used before, cost a two-way conflict on every
// contiguous read.
__host__ __device__ constexpr int lds_pad(int i) { return i ^ (((i >> 3) ^ (i >> 4)) & 7); }
// LDS elements of `count` transforms of length n laid end to end
__host__ __device__ constexpr int lds_slots(int n, int count = 1) { return (n * count + 7) & ~7; }

#ifdef __HIPCC__
namespace fftd {

template <typename C> struct Real;
template <> struct Real<double2> { using type = double; };
template <> struct Real<float2> { using type = float; };
template <typename C> using real_t = typename Real<C>::type;

template <typename C>
__device__ __forceinline__ C mk(real_t<C> x, real_t<C> y);
template <>
__device__ __forceinline__ double2 mk<double2>(double x, double y) { return make_double2(x, y); }
template <>
__device__ __forceinline__ float2 mk<float2>(float x, float y) { return make_float2(x, y); }
template <typename C>
__device__ __forceinline__ C add(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C>
__device__ __forceinline__ C sub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C>
__device__ __forceinline__ C scl(real_t<C> s, C a) { return mk<C>(s * a.x, s * a.y); }
template <typename C>
__device__ __forceinline__ C mul(C a, C b) {
  return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// SGN * i * a
template <int SGN, typename C>
__device__ __forceinline__ C rot(C a) {
  return SGN > 0 ? mk<C>(-a.y, a.x) : mk<C>(a.y, -a.x);
}

// e^{SGN 2 pi i e / 16} * a for the constant exponents of the 16-point DFT
template <int SGN, int E, typename C>
__device__ __forceinline__ C w16(C a) {
  using R = real_t<C>;
  constexpr double c1 = 0.92387953251128675613;  // cos(pi/8)
  constexpr double s1 = 0.38268343236508977173;  // sin(pi/8)
  constexpr double c2 = 0.70710678118654752440;  // cos(pi/4)
  constexpr int e = E % 16;
  if constexpr (e == 0) return a;
  else if constexpr (e == 4) return rot<SGN>(a);
  else if constexpr (e == 8) return mk<C>(-a.x, -a.y);
  else if constexpr (e == 12) return rot<-SGN>(a);
  else {
    constexpr double ang[16][2] = {{1, 0}, {c1, s1}, {c2, c2}, {s1, c1}, {0, 1}, {-s1, c1},
                                   {-c2, c2}, {-c1, s1}, {-1, 0}, {-c1, -s1}, {-c2, -c2},
                                   {-s1, -c1}, {0, -1}, {s1, -c1}, {c2, -c2}, {c1, -s1}};
    return mul(a, mk<C>((R)ang[e][0], (R)(SGN * ang[e][1])));
  }
}

template <int SGN, typename C>
__device__ __forceinline__ void dft4(C& x0, C& x1, C& x2, C& x3) {
  const C a = add(x0, x2), b = sub(x0, x2);
  const C c = add(x1, x3), d = rot<SGN>(sub(x1, x3));
  x0 = add(a, c);
  x1 = add(b, d);
  x2 = sub(a, c);
  x3 = sub(b, d);
}

// y_q = sum_r x_r e^{SGN 2 pi i r q / R}, in place
template <int R, int SGN, typename C>
__device__ __forceinline__ void dft(C* v) {
  using RT = real_t<C>;
  if constexpr (R == 2) {
    const C t = sub(v[0], v[1]);
    v[0] = add(v[0], v[1]);
    v[1] = t;
  } else if constexpr (R == 3) {
    const RT h3 = (RT)0.86602540378443864676;  // sqrt(3)/2
    const C t1 = add(v[1], v[2]), t2 = sub(v[1], v[2]);
    const C base = sub(v[0], scl((RT)0.5, t1));
    const C r = scl(h3, rot<SGN>(t2));
    v[0] = add(v[0], t1);
    v[1] = add(base, r);
    v[2] = sub(base, r);
  } else if constexpr (R == 4) {
    dft4<SGN>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    // 4-point DFTs of the even and odd samples, then one radix-2 stage
    C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<SGN>(e0, e1, e2, e3);
    dft4<SGN>(o0, o1, o2, o3);
    o1 = w16<SGN, 2>(o1);
    o2 = w16<SGN, 4>(o2);
    o3 = w16<SGN, 6>(o3);
    v[0] = add(e0, o0); v[4] = sub(e0, o0);
    v[1] = add(e1, o1); v[5] = sub(e1, o1);
    v[2] = add(e2, o2); v[6] = sub(e2, o2);
    v[3] = add(e3, o3); v[7] = sub(e3, o3);
  } else if constexpr (R == 16) {
    // r = u + 4 s, q = q1 + 4 q2: DFT4 over s, twiddle w16^{u q1}, DFT4 over u
    C a[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u][0] = v[u]; a[u][1] = v[u + 4]; a[u][2] = v[u + 8]; a[u][3] = v[u + 12];
      dft4<SGN>(a[u][0], a[u][1], a[u][2], a[u][3]);
    }
    a[1][1] = w16<SGN, 1>(a[1][1]); a[1][2] = w16<SGN, 2>(a[1][2]); a[1][3] = w16<SGN, 3>(a[1][3]);
    a[2][1] = w16<SGN, 2>(a[2][1]); a[2][2] = w16<SGN, 4>(a[2][2]); a[2][3] = w16<SGN, 6>(a[2][3]);
    a[3][1] = w16<SGN, 3>(a[3][1]); a[3][2] = w16<SGN, 6>(a[3][2]); a[3][3] = w16<SGN, 9>(a[3][3]);
#pragma unroll
    for (int q1 = 0; q1 < 4; ++q1) {
      C b0 = a[0][q1], b1 = a[1][q1], b2 = a[2][q1], b3 = a[3][q1];
      dft4<SGN>(b0, b1, b2, b3);
      v[q1] = b0; v[q1 + 4] = b1; v[q1 + 8] = b2; v[q1 + 12] = b3;
    }
  }
}

// One Stockham pass over BATCH transforms of length n held end to end.
// Inputs come from `get(global index)`, outputs go to `put(global index,
// value)` (the index space is batch * n + position).
template <int n, int T, int BATCH, int S, int SGN, typename C, typename Get, typename Put>
__device__ __forceinline__ void pass(Get get, Put put, const C* tw) {
  // An opaque copy of the table pointer keeps the compiler from hoisting
  // the twiddle loads of every pass out of the caller's loops (that would
  // hold all of them in registers for the whole kernel).
  // The thread index is made opaque too, so that the LDS and twiddle
  // offsets are recomputed per pass instead of being kept live.
  int t = threadIdx.x;
  asm volatile("" : "+s"(tw), "+v"(t));
  constexpr RadixPlan pl = radix_plan(n);
  constexpr int R = pl.r[S];
  constexpr int Ns = plan_ns(pl, S);
  constexpr int nb = n / R;
  constexpr int NB = nb * BATCH;
  constexpr int NBT = (NB + T - 1) / T;
  C v[NBT][R];
#pragma unroll
  for (int b = 0; b < NBT; ++b) {
    const int g = t + b * T;
    if (NB % T == 0 || g < NB) {
      const int bt = g / nb, j = g - bt * nb;
      if constexpr (Ns > 1) {
        const int k = j % Ns;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C w = tw[(Ns - 1) + (r - 1) * Ns + k];
          if (SGN > 0) w.y = -w.y;
          v[b][r] = w;
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const C x = get(bt * n + j + r * nb);
        if constexpr (Ns > 1) {
          if (r > 0) v[b][r] = mul(x, v[b][r]);
          else v[b][r] = x;
        } else {
          v[b][r] = x;
        }
      }
      dft<R, SGN>(v[b]);
    }
  }
  put.begin();
#pragma unroll
  for (int b = 0; b < NBT; ++b) {
    const int g = t + b * T;
    if (NB % T == 0 || g < NB) {
      const int bt = g / nb, j = g - bt * nb;
      const int k = j % Ns;
      const int o = bt * n + (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) put(o + r * Ns, v[b][r], b, r);
    }
  }
  put.end();
}

// Writes into the padded LDS buffer; begin/end are the barriers that keep
// the in-place passes race free.
template <typename C>
struct LdsPut {
  C* buf;
  __device__ __forceinline__ void begin() const { __syncthreads(); }
  __device__ __forceinline__ void end() const { __syncthreads(); }
  __device__ __forceinline__ void operator()(int i, C x, int, int) const { buf[lds_pad(i)] = x; }
};

// Keeps the last pass's outputs in registers: out[b + r NBT] holds element
// t + (b + r NBT) T of the (single) transform.
template <int NBT, int E, typename C>
struct RegPut {
  C (&out)[E];
  __device__ __forceinline__ void begin() const {}
  __device__ __forceinline__ void end() const {}
  __device__ __forceinline__ void operator()(int, C x, int b, int r) const { out[b + r * NBT] = x; }
};

template <typename C>
struct LdsGet {
  const C* buf;
  __device__ __forceinline__ C operator()(int i) const { return buf[lds_pad(i)]; }
};

// Passes S .. np - 1; the last one writes to LDS or (REGS) to registers.
template <int n, int T, int BATCH, int S, int SGN, bool REGS, typename C, typename Get,
          typename Out>
__device__ __forceinline__ void chain(Get get, C* buf, const C* __restrict__ tw, Out& out) {
  constexpr RadixPlan pl = radix_plan(n);
  constexpr bool last = (S + 1 == pl.np);
  constexpr int NBT = (n / pl.r[S]) * BATCH / T;
  if constexpr (S == 0) {
    if constexpr (last && REGS) pass<n, T, BATCH, S, SGN>(get, RegPut<NBT, n / T, C>{out}, tw);
    else pass<n, T, BATCH, S, SGN>(get, LdsPut<C>{buf}, tw);
  } else {
    if constexpr (last && REGS)
      pass<n, T, BATCH, S, SGN>(LdsGet<C>{buf}, RegPut<NBT, n / T, C>{out}, tw);
    else pass<n, T, BATCH, S, SGN>(LdsGet<C>{buf}, LdsPut<C>{buf}, tw);
  }
  if constexpr (!last) chain<n, T, BATCH, S + 1, SGN, REGS>(get, buf, tw, out);
}

}  // namespace fftd

// Number of registers per thread for the register-output form.
template <int n, int T>
constexpr int reg_out_count() { return n / T; }

// True when the last pass of the plan divides evenly over T threads, which
// the register-output form needs.
template <int n, int T>
constexpr bool reg_out_ok() {
  constexpr RadixPlan pl = radix_plan(n);
  return (n / pl.r[pl.np - 1]) % T == 0 && n % T == 0;
}

// Transform with the result in LDS (natural order, padded indices).
// Starts and ends with a barrier.  C is double2 or float2.
template <int n, int T, int SGN, int BATCH = 1, typename C, typename Get>
__device__ __forceinline__ void fft_to_lds(Get get, C* buf, const C* __restrict__ tw) {
  static_assert(plan_valid(n), "unsupported transform length");
  C none[1];
  fftd::chain<n, T, BATCH, 0, SGN, false>(get, buf, tw, none);
}

// Transform with the result in registers: out[i] = X_{t + i T}.  `buf` is
// scratch for the intermediate passes; the first pass starts with a
// barrier, so `buf` may still be read before the call, and the caller
// needs a barrier before writing `buf` afterwards.
template <int n, int T, int SGN, typename C, typename Get>
__device__ __forceinline__ void fft_to_regs(Get get, C* buf, const C* __restrict__ tw,
                                            C (&out)[n / T]) {
  static_assert(plan_valid(n), "unsupported transform length");
  static_assert(reg_out_ok<n, T>(), "last pass does not divide over the block");
  fftd::chain<n, T, 1, 0, SGN, true>(get, buf, tw, out);
}

#endif  // __HIPCC__

}  // namespace qg
