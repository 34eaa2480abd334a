// Bordered band solve with row interchanges (Appendix A), FP64: the
// fallback used when an unpivoted band LU would grow (see solve.hip for the
// unpivoted solve).  One wavefront per system.
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

// --------------------------------------------------------------- solve
// One wavefront per bordered system (system index: s < M - 1 is Psi of
// m = s + 1, s = M - 1 the zonal flow, s > M - 1 theta of m = s - M):
// psi_1 = -Minv (w . h), h <- h - C psi_1, then the band LU solve with row
// interchanges (forward, LAPACK gbtrs order) and back substitution.
//
// Lane t holds position q = t (mod 64) of a 64-wide window of the
// right-hand side.  Each step reads the pivot row with readlane (and, with
// row interchanges, swaps it in with writelane), and updates the lanes below
// (above) it with one FMA.  Factor
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

template <typename TF, int P, int KL, int KUT, bool PIV>
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
  int pv_cur = (PIV && t < B) ? piv[t] : 0;
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
      if (PIV) pv_next = (t < B) ? piv[j0 + B + t] : 0;
    }
#pragma unroll
    for (int jj = 0; jj < B; ++jj) {
      const int j = j0 + jj;
      const int src = j & 63;
      const int d = ((t - j) & 63) - 1;
      const bool act = (d >= 0 && d < KL);
      const TF l = Lcur[jj * KL + (act ? d : 0)];
      if constexpr (PIV) {
        const int p = __builtin_amdgcn_readlane(pv_cur, jj);
        const int dst = (j + p) & 63;
        const double2 a = readlane2(bw, src);
        const double2 bj = readlane2(bw, dst);
        bw = writelane2(bw, a, dst);
        bw = writelane2(bw, bj, src);
        if (act) bw -= mulf(l, bj);
      } else {
        // no interchanges: row j is final, the KL rows below take it
        const double2 bj = readlane2(bw, src);
        if (act) bw -= mulf(l, bj);
      }
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
  bool bad = false;
  for (int k = t; k < K; k += 64) {
    double2 v = zero2();
#pragma unroll
    for (int i = 0; i < P; ++i)
      if (k == i) v = psi1[i];
    if (k >= P) v = hg[k - P];
    if (real_row) v.y = 0.0;
    out[k] = v;
    bad = bad || !isfinite(v.x) || !isfinite(v.y);
  }
  nf_mark(g.nf, bad, rs.tag);
}

template <int KUTP, int KUTR, bool PIV>
__global__ __launch_bounds__(64) void solve_all_kernel(Geom g, FactorSet<double2> Fp,
                                                       FactorSet<double> Fr, double2* rhs,
                                                       RhsSpec rs) {
  extern __shared__ double2 sm[];
  if (nf_stop(g.nf)) return;
  const int blk = blockIdx.x, M = g.M;
  const size_t moff = (size_t)blockIdx.y * M * g.K;   // run of an ensemble
  rhs += 2 * moff;
  rs.out_psi += moff;
  rs.out_th += moff;
  if (blk < M - 1) solve_system<double2, 4, 8, KUTP, PIV>(g, Fp, rhs, rs, 0, blk, blk, sm);
  else solve_system<double, 2, 4, KUTR, PIV>(g, Fr, rhs, rs, blk == M - 1 ? 1 : 2, blk,
                                             blk - (M - 1), sm);
}

// ------------------------------------------------------------ launchers
size_t solve_lds_bytes(const Geom& g, int kutp, int kutr) {
  const int B = SOLVE_BATCH;
  const size_t psi = sizeof(double2) * 2 * B * (8 + kutp + 1);
  const size_t real = sizeof(double) * 2 * B * (4 + kutr + 1);
  return psi > real ? psi : real;
}

int solve_batch() { return SOLVE_BATCH; }

bool launch_solve(const Geom& g, const FactorSet<double2>& Fp, const FactorSet<double>& Fr,
                  double2* rhs, const RhsSpec& rs, int kutp, int kutr, bool pivoted,
                  hipStream_t st) {
  const size_t shm = solve_lds_bytes(g, kutp, kutr);
  const dim3 grid(2 * g.M, g.nmem), block(64);
  if (!pivoted && kutp == 8 && kutr == 4)
    hipLaunchKernelGGL((solve_all_kernel<8, 4, false>), grid, block, shm, st, g, Fp, Fr, rhs, rs);
  else if (pivoted && kutp == 12 && kutr == 4)
    hipLaunchKernelGGL((solve_all_kernel<12, 4, true>), grid, block, shm, st, g, Fp, Fr, rhs, rs);
  else if (pivoted && kutp == 16 && kutr == 8)
    hipLaunchKernelGGL((solve_all_kernel<16, 8, true>), grid, block, shm, st, g, Fp, Fr, rhs, rs);
  else
    return false;
  return true;
}

}  // namespace qg
