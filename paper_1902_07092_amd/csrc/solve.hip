// Bordered band solves of every system (Appendix A) with band LUs that have
// no row interchanges, FP64, gfx950.
//
// A wavefront carries four systems, sixteen lanes each.  Lane l of a
// system holds rows q = l (mod 16) of a sixteen-row window.  Elimination
// step j broadcasts the final row j inside each 16-lane row with DPP
// (row_newbcast), and the rows below it (forward, multipliers of L) or above
// it (backward, U scaled to a unit diagonal) take one complex FMA each.
// Every eight steps the eight finished lanes store their row and take the
// row sixteen further on, loaded three batches ahead.  The factor columns
// of a batch of sixteen steps are loaded three batches ahead into
// registers and staged through a two-slot LDS ring.
//
// Per system: h = rhs rows p.. ; Schur part psi_1 = -Minv (w . h),
// h <- h - C psi_1 (first kl rows); forward L y = h with y' = y / U_jj
// stored over h; backward U' x = y'; the new state [psi_1, x] is written.
//
// Galerkin bases (Sect. 3.2.2, eq. psiint_galerkin, uphi_galerkin,
// temp_galerkin): the systems are pure bands (no border) on the Galerkin
// coefficients x~, with 8 sub- and 12 super-diagonals for Psi and 4 and 6
// for the Dirichlet systems; the right-hand side is the same rows p.. .
// The backward sweep of a 12-wide U' stores and refills lanes every four
// steps instead of eight (the 16-row window must hold the pivot and the 12
// rows above it).  x~ goes over h, then the Chebyshev coefficients
// y = S x~ (the stencil: Appendix B's gamma_i^n for Psi, T_{n+2} - T_n for
// the Dirichlet systems) are written as the new state.
#include <hip/hip_runtime.h>

#include <utility>

#include "kernels.h"

namespace qg {

namespace {

#ifndef QG_SOLVE_NSET
#define QG_SOLVE_NSET 3
#endif
constexpr int SB = 16;     // steps per batch = lanes per system
constexpr int NSET = QG_SOLVE_NSET;   // factor batches in flight (the batch loop is unrolled by NSET)

__device__ __forceinline__ double2 z2() { return make_double2(0.0, 0.0); }

// Value of lane LANE of each 16-lane row.
template <int LANE>
__device__ __forceinline__ double bcast(double v) {
  // one 64-bit DPP move (row_newbcast was made for FP64 operands); every
  // lane has a source, so the "old" value is never used
  return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + LANE, 0xF, 0xF, true);
}
template <int LANE>
__device__ __forceinline__ double2 bcast2(double2 v) {
  return make_double2(bcast<LANE>(v.x), bcast<LANE>(v.y));
}

// bw -= l a
__device__ __forceinline__ void fms(double2& bw, double l, double2 a) {
  bw.x = fma(-l, a.x, bw.x);
  bw.y = fma(-l, a.y, bw.y);
}
__device__ __forceinline__ void fms(double2& bw, double2 l, double2 a) {
  bw.x = fma(-l.x, a.x, bw.x);
  bw.x = fma(l.y, a.y, bw.x);
  bw.y = fma(-l.x, a.y, bw.y);
  bw.y = fma(-l.y, a.x, bw.y);
}
__device__ __forceinline__ double2 mul(double l, double2 a) { return make_double2(l * a.x, l * a.y); }
__device__ __forceinline__ double2 mul(double2 l, double2 a) {
  return make_double2(l.x * a.x - l.y * a.y, l.x * a.y + l.y * a.x);
}

template <typename TF> __device__ __forceinline__ TF tz();
template <> __device__ __forceinline__ double tz<double>() { return 0.0; }
template <> __device__ __forceinline__ double2 tz<double2>() { return z2(); }

// One kind of system (P boundary rows, KL sub- and KU super-diagonals of
// the band, factor type TF; GAL: Galerkin band without border) for the
// four systems of this wavefront.
template <typename TF, int P, int KL, int KU = KL, bool GAL = false>
struct Solver4 {
  static_assert(KL <= 8 && KU <= 12, "band wider than the 16-row window");
  static_assert(GAL || KL == KU, "bordered systems have a symmetric band");
  static constexpr int KW = KL > KU ? KL : KU;                 // widest factor column
  template <int W>
  static constexpr int cps() { return SB * W * (int)sizeof(TF) / 16; }   // 16-byte chunks per system batch
  template <int W>
  static constexpr int nch() { return 4 * cps<W>() / 64; }              // chunks per lane per batch
  static_assert(nch<KL>() * 64 == 4 * cps<KL>() && nch<KU>() * 64 == 4 * cps<KU>(),
                "batch does not divide over the wavefront");

  // (plain copies: references to the kernel's by-value arguments would
  // place those structures in scratch memory)
  FactorSet<TF> F;
  double2* out_psi;
  double2* out_th;
  int M, K;
  int kind, nsys, sys0, so0;   // kind of system; valid count; first global / factor index
  int n, q, nb;                // band rows, padded rows (multiple of NSET * SB), batches
  TF* ring;                    // LDS [2][4][SB KW + pad]
  int t, lane, grp;
  bool valid;
  int so;                      // factor index of this lane's system (clamped)
  double2* hg;                 // this system's h / y' (rhs rows p..)
  bool bad = false;            // a stored entry of the new state is not finite

  // a batch of factor columns of width W (KL for L, KU for U')
  template <int W>
  struct Batch {
    double2 v[nch<W>()];
  };
  // chunk I of this lane: wave chunk c = t + 64 I, system c / CPS
  template <int W, int I>
  __device__ __forceinline__ double2 load_chunk(const TF* base, int b) const {
    constexpr int CPS = cps<W>();
    const int c = t + 64 * I;
    const int gs = c / CPS, e = c - gs * CPS;
    const int s = min(so0 + gs, so0 + nsys - 1);
    return reinterpret_cast<const double2*>(base + ((size_t)s * q + (size_t)b * SB) * W)[e];
  }
  template <int W, int... I>
  __device__ __forceinline__ Batch<W> load_batch(const TF* base, int b,
                                                 std::integer_sequence<int, I...>) const {
    return Batch<W>{{load_chunk<W, I>(base, b)...}};
  }
  template <int W>
  __device__ __forceinline__ Batch<W> load_batch(const TF* base, int b) const {
    return load_batch<W>(base, b, std::make_integer_sequence<int, nch<W>()>{});
  }
  // LDS ring slot: [4 systems][SB][W], each system's block followed by a
  // 16-byte pad so that the four systems' reads fall in different banks
  static constexpr int SYS_CH = cps<KW>() + 1;   // 16-byte chunks per system block (room for either width)
  template <int W, int... I>
  __device__ __forceinline__ void stage(int slot, const Batch<W>& r,
                                        std::integer_sequence<int, I...>) const {
    constexpr int CPS = cps<W>();
    double2* dst = reinterpret_cast<double2*>(ring) + (size_t)slot * 4 * SYS_CH;
    if constexpr (CPS + 1 == SYS_CH)   // chunk c of system c / CPS
      ((dst[(t + 64 * I) + (t + 64 * I) / CPS] = r.v[I]), ...);
    else
      ((dst[((t + 64 * I) / CPS) * SYS_CH + (t + 64 * I) % CPS] = r.v[I]), ...);
  }
  template <int W>
  __device__ __forceinline__ void stage(int slot, const Batch<W>& r) const {
    stage<W>(slot, r, std::make_integer_sequence<int, nch<W>()>{});
  }
  template <int W>
  __device__ __forceinline__ TF coef(int slot, int jj, int d) const {   // d in [1, W]
    const TF* blk = reinterpret_cast<const TF*>(reinterpret_cast<const double2*>(ring) +
                                                (size_t)(slot * 4 + grp) * SYS_CH);
    return blk[jj * W + (d - 1)];
  }
  __device__ __forceinline__ double2 hrow(int r) const { return (r < n) ? hg[r] : z2(); }
  __device__ __forceinline__ TF uirow(int r) const {
    return F.ui[(size_t)so * q + min(r, q - 1)];
  }

  // ---------------------------------------------------------- forward
  // The coefficients of a group of steps are read from LDS before its
  // first step (the compiler barrier keeps the reads together), so that the
  // elimination chain never waits on LDS.
  template <int JJ>
  __device__ __forceinline__ TF fcoef(int slot) const {   // this lane's L entry at step JJ
    const int d = (lane - JJ) & 15;
    const bool act = (d >= 1 && d <= KL);
    const TF l = coef<KL>(slot, JJ, act ? d : 1);
    return act ? l : tz<TF>();
  }
  template <int JJ>
  __device__ __forceinline__ TF bcoef(int slot) const {   // this lane's U' entry at column JJ
    const int e = (JJ - lane) & 15;
    const bool act = (e >= 1 && e <= KU);
    const TF u = coef<KU>(slot, JJ, act ? e : 1);
    return act ? u : tz<TF>();
  }
  template <int J0, int... J>
  __device__ __forceinline__ void fhalf(double2& bw, int slot, std::integer_sequence<int, J...>)
      const {
    TF c[sizeof...(J)] = {fcoef<J0 + J>(slot)...};
    asm volatile("" ::: "memory");
    ((fms(bw, c[J], bcast2<J0 + J>(bw))), ...);
  }
  // backward: columns J0 + G - 1 - J, J = 0..G-1 (G = 8 or 4 steps)
  template <int J0, int... J>
  __device__ __forceinline__ void bgroup(double2& bw, int slot, std::integer_sequence<int, J...>)
      const {
    constexpr int G = sizeof...(J);
    TF c[G] = {bcoef<J0 + G - 1 - J>(slot)...};
    asm volatile("" ::: "memory");
    ((fms(bw, c[J], bcast2<J0 + G - 1 - J>(bw))), ...);
  }

  __device__ __forceinline__ void run(double2* out_state) {
    if constexpr (GAL) {
      run_galerkin(out_state);
      return;
    } else {
      run_bordered(out_state);
    }
  }

  __device__ __forceinline__ void run_bordered(double2* out_state) {
    // ---- Schur part for the p border unknowns
    double2 wh[P];
#pragma unroll
    for (int i = 0; i < P; ++i) wh[i] = z2();
    const TF* Wr = F.W + (size_t)so * P * n;
    // four rows per lane per chunk, two chunks in flight: the loads of the
    // next chunk are issued before the current one is summed (every lane
    // still adds its rows in increasing order)
    constexpr int U = 4;
    double2 hA[U], hB[U];
    TF wA[U][P], wB[U][P];
    auto load = [&](int j0, double2 (&h)[U], TF (&w)[U][P]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = min(j0 + u * SB + lane, n - 1);
        h[u] = hg[j];
#pragma unroll
        for (int i = 0; i < P; ++i) w[u][i] = Wr[(size_t)i * n + j];
      }
    };
    auto add = [&](int j0, const double2 (&h)[U], const TF (&w)[U][P]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (j0 + u * SB + lane < n) {
#pragma unroll
          for (int i = 0; i < P; ++i) {
            const double2 v = mul(w[u][i], h[u]);
            wh[i].x += v.x;
            wh[i].y += v.y;
          }
        }
      }
    };
    load(0, hA, wA);
    for (int j0 = 0; j0 < n; j0 += 2 * U * SB) {
      load(j0 + U * SB, hB, wB);
      add(j0, hA, wA);
      load(j0 + 2 * U * SB, hA, wA);
      add(j0 + U * SB, hB, wB);
    }
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) {
        wh[i].x += __shfl_xor(wh[i].x, off, 16);
        wh[i].y += __shfl_xor(wh[i].y, off, 16);
      }
    double2 psi1[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      double2 acc = z2();
#pragma unroll
      for (int i2 = 0; i2 < P; ++i2) fms(acc, F.Minv[((size_t)so * P + i) * P + i2], wh[i2]);
      psi1[i] = acc;
    }

    // ---- forward: L y = h, y' = y / U_jj over h
    double2 bw = hrow(lane);
    if (lane < KL) {
#pragma unroll
      for (int i = 0; i < P; ++i) fms(bw, F.Cb[((size_t)so * KL + lane) * P + i], psi1[i]);
    }
    sweep<true>(bw);
    __threadfence();

    // ---- backward: U' x = y'
    bw = hrow((nb - 1) * SB + lane);
    sweep<false>(bw);

    // ---- border unknowns
    if (valid && lane < P) {
      double2 v = psi1[0];
#pragma unroll
      for (int i = 1; i < P; ++i)
        if (lane == i) v = psi1[i];
      if (kind != 0 && (kind == 1 || sys0 + grp == M)) v.y = 0.0;
      out_state[lane] = v;
      bad = bad || !isfinite(v.x) || !isfinite(v.y);
    }
  }

  // Galerkin band: forward and backward sweeps with x~ written over h, then
  // the K Chebyshev coefficients y = S x~ of the new state.
  __device__ __forceinline__ void run_galerkin(double2* out_state) {
    double2 bw = hrow(lane);
    sweep<true>(bw);
    __threadfence();
    bw = hrow((nb - 1) * SB + lane);
    sweep<false>(bw);
    __threadfence();   // x~ rows of the other lanes of the group
    // Row k = lane + 16 t needs x~_{k-i}, i <= 4: lane (lane - i) mod 16
    // holds it, in this chunk of 16 rows or (lane < i) in the previous one.
    // Each lane loads only its own rows, eight chunks per round with every
    // load in flight before the first is used; the neighbours come by
    // shuffles within the 16-lane group.
    const bool real_row = (kind == 1) || (kind == 2 && sys0 + grp == M);
    constexpr int U = 8;
    double2 prev = z2();
    for (int k0 = 0; k0 < K; k0 += U * SB) {
      double2 x[U];
      double gm[U][P == 4 ? 5 : 1];   // gamma_i^{k-i} of this lane's rows, loaded up front
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + u * SB + lane;
        x[u] = (k < n) ? hg[min(k, n - 1)] : z2();
        if constexpr (P == 4) {
#pragma unroll
          for (int i = 0; i < 5; ++i) {
            const int j = k - i;
            gm[u][i] = (j >= 0 && j < n) ? F.gam[(size_t)j * 5 + i] : 0.0;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + u * SB + lane;
        auto nb_row = [&](int i) {   // x~_{k-i}
          const int src = (lane - i) & 15;
          const double2 a = make_double2(__shfl(x[u].x, src, 16), __shfl(x[u].y, src, 16));
          const double2 b = make_double2(__shfl(prev.x, src, 16), __shfl(prev.y, src, 16));
          return lane >= i ? a : b;
        };
        double2 v;
        if constexpr (P == 4) {   // Psi: y_k = sum_i gamma_i^{k-i} x~_{k-i}
          v = z2();
#pragma unroll
          for (int i = 0; i < 5; ++i) {
            const double2 xi = i ? nb_row(i) : x[u];
            v.x = fma(gm[u][i], xi.x, v.x);
            v.y = fma(gm[u][i], xi.y, v.y);
          }
        } else {                  // Dirichlet: y_k = x~_{k-2} - x~_k
          const double2 x2 = nb_row(2);
          v = make_double2(x2.x - x[u].x, x2.y - x[u].y);
        }
        if (real_row) v.y = 0.0;
        if (valid && k < K) {
          out_state[k] = v;
          bad = bad || !isfinite(v.x) || !isfinite(v.y);
        }
        prev = x[u];
      }
    }
  }

  // One full sweep; FWD: batches 0..nb-1 (factor columns of width KL),
  // else nb-1..0 (width KU).
  template <bool FWD>
  __device__ __forceinline__ void sweep(double2& bw) {
    constexpr int W = FWD ? KL : KU;
    const TF* base = FWD ? F.L : F.U;
    const bool real_row = (kind == 1) || (kind == 2 && sys0 + grp == M);
    // the bordered solve writes x below the border rows of the state; the
    // Galerkin solve writes x~ over h
    double2* xo = GAL ? hg : out_ptr() + P;
    auto bidx = [&](int i) { return FWD ? i : nb - 1 - i; };
    // sets[k] holds a batch i = k (mod NSET) ahead of its use; hs / us
    // the refill rows and 1 / U(j, j) of batches k (mod NSET)
    Batch<W> sets[NSET];
    double2 hs[NSET];
    TF us[NSET];
    {   // batch 0 to the ring, batches 1..NSET in flight (loads past the
        // last batch re-read it)
      stage<W>(0, load_batch<W>(base, bidx(0)));
      prologue<FWD>(sets, hs, us, std::make_integer_sequence<int, NSET>{});
    }
    for (int i0 = 0; i0 < nb; i0 += NSET)   // nb is a multiple of NSET
      batches<FWD>(bw, i0, base, real_row, xo, sets, hs, us,
                   std::make_integer_sequence<int, NSET>{});
  }

  template <bool FWD, int... KK>
  __device__ __forceinline__ void prologue(Batch<FWD ? KL : KU> (&sets)[NSET],
                                           double2 (&hs)[NSET], TF (&us)[NSET],
                                           std::integer_sequence<int, KK...>) {
    constexpr int W = FWD ? KL : KU;
    // batch k + 1 goes to sets[(k + 1) mod NSET]
    ((sets[(KK + 1) % NSET] = load_batch<W>(
          base_of<FWD>(), FWD ? min(KK + 1, nb - 1) : nb - 1 - min(KK + 1, nb - 1))),
     ...);
    ((hs[KK] = refill_row<FWD>(KK)), ...);
    if (FWD) ((us[KK] = uirow(KK * SB + lane)), ...);
  }
  template <bool FWD>
  __device__ __forceinline__ const TF* base_of() const { return FWD ? F.L : F.U; }
  template <bool FWD>
  __device__ __forceinline__ double2 refill_row(int k) const {   // used in batch k
    const int rr = FWD ? (k + 1) * SB + lane : (nb - 2 - k) * SB + lane;
    return (rr >= 0 && rr < q) ? hrow(rr) : z2();
  }
  template <bool FWD, int... KK>
  __device__ __forceinline__ void batches(double2& bw, int i0, const TF* base, bool real_row,
                                          double2* xo, Batch<FWD ? KL : KU> (&sets)[NSET],
                                          double2 (&hs)[NSET], TF (&us)[NSET],
                                          std::integer_sequence<int, KK...>) {
    (batch<FWD>(bw, i0 + KK, base, real_row, xo, sets[(KK + 1) % NSET], hs[KK], us[KK]), ...);
  }

  // Row `row` of lanes [L0, L0 + G) is final: store it (backward: the
  // solution, real rows with zero imaginary part) and take the refill row.
  template <bool FWD, int L0, int G>
  __device__ __forceinline__ void retire(double2& bw, int row, bool real_row, double2* xo,
                                         double2 hr, TF ur) {
    if (lane >= L0 && lane < L0 + G) {
      if (valid && row < n) {
        if (FWD) {
          hg[row] = mul(ur, bw);
        } else {
          double2 v = bw;
          if (real_row && !GAL) v.y = 0.0;
          xo[row] = v;
          if (!GAL) bad = bad || !isfinite(v.x) || !isfinite(v.y);
        }
      }
      bw = hr;
    }
  }

  // Batch i of a sweep.  nxt holds batch i + 1 (staged to the ring now)
  // and is reloaded with batch i + 1 + NSET; hr / ur are this batch's
  // refill rows and scalings, reloaded for batch i + NSET.
  template <bool FWD>
  __device__ __forceinline__ void batch(double2& bw, int i, const TF* base, bool real_row,
                                        double2* xo, Batch<FWD ? KL : KU>& nxt, double2& hr,
                                        TF& ur) {
    constexpr int W = FWD ? KL : KU;
    const int b = FWD ? i : nb - 1 - i;
    const int slot = i & 1;
    // next batch to the ring, and the batch NSET after it in flight
    if (i + 1 < nb) stage<W>((i + 1) & 1, nxt);
    {
      const int inext = min(i + 1 + NSET, nb - 1);
      nxt = load_batch<W>(base, FWD ? inext : nb - 1 - inext);
    }
    const int row = b * SB + lane;          // this lane's row in batch b
    if (FWD) {
      fhalf<0>(bw, slot, std::make_integer_sequence<int, 8>{});
      retire<true, 0, 8>(bw, row, real_row, xo, hr, ur);      // rows b SB + 0..7 are final
      fhalf<8>(bw, slot, std::make_integer_sequence<int, 8>{});
      retire<true, 8, 8>(bw, row, real_row, xo, hr, ur);
      // refills and scalings of batch i + NSET
      const int rn = (b + NSET + 1) * SB + lane;
      hr = (rn < q) ? hrow(rn) : z2();
      ur = uirow((b + NSET) * SB + lane);
    } else {
      if constexpr (KU <= 8) {   // two groups of eight columns
        bgroup<8>(bw, slot, std::make_integer_sequence<int, 8>{});   // columns 15..8
        retire<false, 8, 8>(bw, row, real_row, xo, hr, ur);          // rows b SB + 8..15 are final
        bgroup<0>(bw, slot, std::make_integer_sequence<int, 8>{});   // columns 7..0
        retire<false, 0, 8>(bw, row, real_row, xo, hr, ur);
      } else {                   // four groups of four columns
        bgroup<12>(bw, slot, std::make_integer_sequence<int, 4>{});
        retire<false, 12, 4>(bw, row, real_row, xo, hr, ur);
        bgroup<8>(bw, slot, std::make_integer_sequence<int, 4>{});
        retire<false, 8, 4>(bw, row, real_row, xo, hr, ur);
        bgroup<4>(bw, slot, std::make_integer_sequence<int, 4>{});
        retire<false, 4, 4>(bw, row, real_row, xo, hr, ur);
        bgroup<0>(bw, slot, std::make_integer_sequence<int, 4>{});
        retire<false, 0, 4>(bw, row, real_row, xo, hr, ur);
      }
      const int rn = (b - NSET - 1) * SB + lane;
      hr = (rn >= 0) ? hrow(rn) : z2();
    }
  }
  __device__ __forceinline__ double2* out_ptr() const {
    const int m = (kind == 0) ? sys0 + grp + 1 : (kind == 1 ? 0 : sys0 + grp - M);
    return (kind == 2 ? out_th : out_psi) + (size_t)max(m, 0) * K;
  }

  // ---------------------------------------------------------- adjoint
  // y = S^-H f for the bordered system S = [A B; C D], D = L U, in the
  // real inner product (Appendix A transposed): z = D^-H f_b by the two
  // sweeps above run on the factors of D^H = (U^H)(L^H) (F holds them:
  // L the unit-lower U^H scaled, ui = conj(1 / U_jj), U the unit-upper
  // L^H), then y_a = Minv^H (f_a - C^H z), y_b = z - W^H y_a, and the tau
  // rows of y are zero (the adjoint of zeroing the tau rows of a
  // right-hand side).  Real systems take real inputs (the adjoint of
  // keeping theta_0 and the zonal flow real).  fa: rows 0..P-1 of f.
  __device__ __forceinline__ void run_adjoint(const double2* fa) {
    const bool real_row = (kind == 1) || (kind == 2 && sys0 + grp == M);
    if (real_row && valid)
      for (int r = lane; r < n; r += SB) hg[r].y = 0.0;
    __syncthreads();
    double2 bw = hrow(lane);
    sweep<true>(bw);
    __threadfence();
    bw = hrow((nb - 1) * SB + lane);
    sweep<false>(bw);
    __syncthreads();
    // the groups past the last system (valid = false) only kept the sweeps
    // in step; their output rows do not exist
    double2 ya[P];
    if (valid) {
      const double2* xo = out_ptr() + P;
      double2 tc[P];
#pragma unroll
      for (int c = 0; c < P; ++c) {
        tc[c] = fa[c];
        if (real_row) tc[c].y = 0.0;
        for (int r = 0; r < KW && r < n; ++r)
          tc[c] = sub_cj(tc[c], F.Cb[((size_t)so * KW + r) * P + c], xo[r]);
      }
#pragma unroll
      for (int i = 0; i < P; ++i) {
        double2 acc = z2();
#pragma unroll
        for (int c = 0; c < P; ++c) acc = add_cj(acc, F.Minv[((size_t)so * P + c) * P + i], tc[c]);
        ya[i] = acc;
      }
    }
    __syncthreads();
    if (valid) {
      double2* xs = out_ptr();
      double2* xo = xs + P;
      const TF* Wr = F.W + (size_t)so * P * n;
      for (int j = lane; j < n; j += SB) {
        double2 v = xo[j];
#pragma unroll
        for (int i = 0; i < P; ++i) v = sub_cj(v, Wr[(size_t)i * n + j], ya[i]);
        if (real_row) v.y = 0.0;
        xo[j] = v;
        bad = bad || !isfinite(v.x) || !isfinite(v.y);
      }
      if (lane < P) xs[lane] = z2();
    }
  }
  // a - conj(c) b, a + conj(c) b
  static __device__ __forceinline__ double2 sub_cj(double2 a, double2 c, double2 b) {
    return make_double2(a.x - (c.x * b.x + c.y * b.y), a.y - (c.x * b.y - c.y * b.x));
  }
  static __device__ __forceinline__ double2 sub_cj(double2 a, double c, double2 b) {
    return make_double2(a.x - c * b.x, a.y - c * b.y);
  }
  static __device__ __forceinline__ double2 add_cj(double2 a, double2 c, double2 b) {
    return make_double2(a.x + (c.x * b.x + c.y * b.y), a.y + (c.x * b.y - c.y * b.x));
  }
  static __device__ __forceinline__ double2 add_cj(double2 a, double c, double2 b) {
    return make_double2(a.x + c * b.x, a.y + c * b.y);
  }
};

template <typename T> __device__ __forceinline__ T cj(T v);
template <> __device__ __forceinline__ double cj<double>(double v) { return v; }
template <> __device__ __forceinline__ double2 cj<double2>(double2 v) { return make_double2(v.x, -v.y); }

// Factors of D^H from those of D (unpivoted layout, q padded steps, KW
// sub- and super-diagonals): D = L diag(d) U' (U' unit upper stored by
// columns, U[j][e-1] = U'(j-e, j); ui[j] = 1/d_j), so D^H = U'^H
// diag(conj d) L^H with
//   LT[j][e-1] = conj(U'(j, j+e)) = conj(U[j+e][e-1])     (j + e < n)
//   UT[j][e-1] = conj(L(j, j-e))  = conj(L[j-e][e-1])     (j < n, j >= e)
//   uiT[j] = conj(ui[j]);
// the padding steps stay identity steps.
template <typename TF, int KW>
__global__ __launch_bounds__(256) void transpose_factors_kernel(const TF* __restrict__ L,
                                                                const TF* __restrict__ U,
                                                                const TF* __restrict__ ui, int S,
                                                                int n, int q, TF* __restrict__ LT,
                                                                TF* __restrict__ UT,
                                                                TF* __restrict__ uiT) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)S * q) return;
  const size_t s = idx / q;
  const int j = (int)(idx - s * q);
  const TF* Ls = L + s * q * KW;
  const TF* Us = U + s * q * KW;
#pragma unroll
  for (int e = 1; e <= KW; ++e) {
    LT[idx * KW + (e - 1)] = (j + e < n) ? cj(Us[(size_t)(j + e) * KW + (e - 1)]) : tz<TF>();
    UT[idx * KW + (e - 1)] = (j < n && j >= e) ? cj(Ls[(size_t)(j - e) * KW + (e - 1)]) : tz<TF>();
  }
  uiT[idx] = cj(ui[idx]);
}

}  // namespace

// Block: one wavefront, four systems.  System blocks [0, nbp) take the Psi
// systems (m = 1..M-1), the rest the real systems (zonal flow, theta of
// every m).  The runs of an ensemble share the factors: the 1D grid puts
// system block b of every run on the same XCD (the hardware hands block
// ids to the eight XCDs round robin) and back to back, so each XCD reads
// a factor batch from HBM once for all runs:
//   id = ((b / 8) nmem + run) 8 + b % 8,   b < nb (padded ids exit).
// GAL: the Galerkin bands (8 / 12 and 4 / 6 diagonals, no border).
// part 0: every system; 1: the real systems only; 2: the Psi systems only,
// whose right-hand sides first take rs.buoy_adt C[(Ra/Pr)(i m/s_o) theta]
// of the new theta when rs.buoy_adt != 0 (implicit buoyancy: part 1, then
// part 2).
template <bool GAL>
__global__ __launch_bounds__(64) void solve_np_kernel(Geom g, Bands bd, FactorSet<double2> Fp,
                                                      FactorSet<double> Fr, double2* rhs,
                                                      RhsSpec rs, int qp, int qr, int part) {
  using SolverP = Solver4<double2, 4, 8, GAL ? 12 : 8, GAL>;
  using SolverR = Solver4<double, 2, 4, GAL ? 6 : 4, GAL>;
  __shared__ double2 ring_mem[2 * 4 * SolverP::SYS_CH];
  static_assert(SolverR::SYS_CH <= SolverP::SYS_CH, "ring too small for the real systems");
  const int M = g.M, K = g.K;
  const int nbp = (M - 1 + 3) / 4;
  const int nb = (part == 1 ? 0 : nbp) + (part == 2 ? 0 : (M + 1 + 3) / 4);
  const int id = blockIdx.x, rest = id >> 3;
  const int run = rest % g.nmem;
  int b = (rest / g.nmem) * 8 + (id & 7);   // system block
  if (b >= nb || nf_stop(g.nf)) return;
  if (part == 1) b += nbp;                   // real systems only
  const int t = threadIdx.x, lane = t & 15, grp = t >> 4;
  const size_t moff = (size_t)run * M * K;   // run of an ensemble
  rhs += 2 * moff;
  rs.out_psi += moff;
  rs.out_th += moff;
  if (b < nbp) {
    SolverP s{Fp, rs.out_psi, rs.out_th, M, K};
    s.kind = 0;
    s.sys0 = 4 * b;
    s.so0 = s.sys0;
    s.nsys = min(4, M - 1 - s.sys0);
    s.n = K - 4; s.q = qp; s.nb = qp / SB;
    s.ring = ring_mem;
    s.t = t; s.lane = lane; s.grp = grp;
    s.valid = grp < s.nsys;
    s.so = s.so0 + min(grp, s.nsys - 1);
    s.hg = rhs + (size_t)(s.sys0 + min(grp, s.nsys - 1)) * K + 4;
    if (rs.buoy_adt != 0.0 && s.valid) {
      // h_k += a dt (Ra/Pr)(i m/s_o) sum_n C_kn theta_n, rows k >= 4; each
      // lane updates the rows it reads first in the sweeps
      const int m = s.sys0 + grp + 1;
      const double ra_pr = g.ra_pr ? g.ra_pr[run] : g.Ra_Pr;
      const double gb = rs.buoy_adt * ra_pr * (double)m / g.s_o;
      const double2* th = rs.out_th + (size_t)m * K;
      for (int k = 4 + lane; k < K; k += SB) {
        double2 cb = z2();
#pragma unroll
        for (int o = 0; o < 17; ++o) {
          const int n = k + o - 8;
          const double c = bd.C[(size_t)o * K + k];
          const double2 v = (n >= 0 && n < K) ? th[min(max(n, 0), K - 1)] : z2();
          cb.x = fma(c, v.x, cb.x);
          cb.y = fma(c, v.y, cb.y);
        }
        double2 h = s.hg[k - 4];
        h.x -= gb * cb.y;
        h.y += gb * cb.x;
        s.hg[k - 4] = h;
      }
      __threadfence();
    }
    s.run(s.out_ptr());
    nf_mark(g.nf, s.bad, rs.tag);
  } else {
    SolverR s{Fr, rs.out_psi, rs.out_th, M, K};
    const int r0 = 4 * (b - nbp);              // first real-system index
    s.kind = (r0 == 0) ? 1 : 2;                // the zonal flow leads the first block
    s.sys0 = (M - 1) + r0;
    s.so0 = r0;
    s.nsys = min(4, M + 1 - r0);
    s.n = K - 2; s.q = qr; s.nb = qr / SB;
    s.ring = reinterpret_cast<double*>(ring_mem);
    s.t = t; s.lane = lane; s.grp = grp;
    s.valid = grp < s.nsys;
    s.so = s.so0 + min(grp, s.nsys - 1);
    s.hg = rhs + (size_t)(s.sys0 + min(grp, s.nsys - 1)) * K + 2;
    // system kind per group: only group 0 of block 0 is the zonal flow
    if (r0 == 0 && grp > 0) s.kind = 2;
    s.run(s.out_ptr());
    nf_mark(g.nf, s.bad, rs.tag);
  }
}

// y = S^-H f for every system of a step (the transposed solves of a
// reverse sweep): the block layout of solve_np_kernel; the factor sets
// carry the factors of D^H (transpose_factors_kernel) with the border data
// of D.  f and y are co-state arrays [M][K] (Psi of m in row m, the zonal
// flow in row 0 of f_psi / y_psi, theta of m in row m); f is overwritten.
__global__ __launch_bounds__(64) void solve_adjoint_np_kernel(Geom g, FactorSet<double2> Fp,
                                                              FactorSet<double> Fr,
                                                              double2* f_psi, double2* f_th,
                                                              double2* y_psi, double2* y_th,
                                                              int qp, int qr) {
  __shared__ double2 ring_mem[2 * 4 * (SB * 8 + 1)];
  const int M = g.M, K = g.K;
  const int nbp = (M - 1 + 3) / 4;
  const int nb = nbp + (M + 1 + 3) / 4;
  const int id = blockIdx.x;
  const int b = (id >> 3) * 8 + (id & 7);
  if (b >= nb) return;
  const int t = threadIdx.x, lane = t & 15, grp = t >> 4;
  if (b < nbp) {
    Solver4<double2, 4, 8> s{Fp, y_psi, y_th, M, K};
    s.kind = 0;
    s.sys0 = 4 * b;
    s.so0 = s.sys0;
    s.nsys = min(4, M - 1 - s.sys0);
    s.n = K - 4; s.q = qp; s.nb = qp / SB;
    s.ring = ring_mem;
    s.t = t; s.lane = lane; s.grp = grp;
    s.valid = grp < s.nsys;
    s.so = s.so0 + min(grp, s.nsys - 1);
    const int m = s.sys0 + min(grp, s.nsys - 1) + 1;
    s.hg = f_psi + (size_t)m * K + 4;
    s.run_adjoint(f_psi + (size_t)m * K);
  } else {
    Solver4<double, 2, 4> s{Fr, y_psi, y_th, M, K};
    const int r0 = 4 * (b - nbp);
    s.kind = (r0 == 0) ? 1 : 2;
    s.sys0 = (M - 1) + r0;
    s.so0 = r0;
    s.nsys = min(4, M + 1 - r0);
    s.n = K - 2; s.q = qr; s.nb = qr / SB;
    s.ring = reinterpret_cast<double*>(ring_mem);
    s.t = t; s.lane = lane; s.grp = grp;
    s.valid = grp < s.nsys;
    s.so = s.so0 + min(grp, s.nsys - 1);
    if (r0 == 0 && grp > 0) s.kind = 2;
    const int r = r0 + min(grp, s.nsys - 1);          // 0: zonal flow, 1 + m: theta of m
    double2* f = (r == 0) ? f_psi : f_th + (size_t)(r - 1) * K;
    s.hg = f + 2;
    s.run_adjoint(f);
  }
}

void launch_transpose_factors(const FactorSet<double2>& Fp, const FactorSet<double>& Fr, int Sp,
                              int Sr, int n4, int n2, int qp, int qr, double2* pLT, double2* pUT,
                              double2* puiT, double* rLT, double* rUT, double* ruiT,
                              hipStream_t st) {
  const size_t np = (size_t)Sp * qp, nr = (size_t)Sr * qr;
  hipLaunchKernelGGL((transpose_factors_kernel<double2, 8>), dim3((unsigned)((np + 255) / 256)),
                     dim3(256), 0, st, Fp.L, Fp.U, Fp.ui, Sp, n4, qp, pLT, pUT, puiT);
  hipLaunchKernelGGL((transpose_factors_kernel<double, 4>), dim3((unsigned)((nr + 255) / 256)),
                     dim3(256), 0, st, Fr.L, Fr.U, Fr.ui, Sr, n2, qr, rLT, rUT, ruiT);
}

bool launch_solve_adjoint_np(const Geom& g, const FactorSet<double2>& FpT,
                             const FactorSet<double>& FrT, int qp, int qr, double2* f_psi,
                             double2* f_th, double2* y_psi, double2* y_th, hipStream_t st) {
  if (qp % (NSET * SB) || qr % (NSET * SB)) return false;
  const int nb = (g.M - 1 + 3) / 4 + (g.M + 1 + 3) / 4;
  const int blocks = 8 * ((nb + 7) / 8);
  hipLaunchKernelGGL(solve_adjoint_np_kernel, dim3(blocks), dim3(64), 0, st, g, FpT, FrT, f_psi,
                     f_th, y_psi, y_th, qp, qr);
  return true;
}

bool launch_solve_np(const Geom& g, const Bands& bd, const FactorSet<double2>& Fp,
                     const FactorSet<double>& Fr, double2* rhs, const RhsSpec& rs, int qp, int qr,
                     bool galerkin, hipStream_t st) {
  if (qp % (NSET * SB) || qr % (NSET * SB)) return false;
  if (galerkin && !Fp.gam) return false;
  const int nbp = (g.M - 1 + 3) / 4, nbr = (g.M + 1 + 3) / 4;
  auto go = [&](int part, int nb) {
    const int blocks = 8 * ((nb + 7) / 8) * g.nmem;
    if (galerkin)
      hipLaunchKernelGGL(solve_np_kernel<true>, dim3(blocks), dim3(64), 0, st, g, bd, Fp, Fr, rhs,
                         rs, qp, qr, part);
    else
      hipLaunchKernelGGL(solve_np_kernel<false>, dim3(blocks), dim3(64), 0, st, g, bd, Fp, Fr,
                         rhs, rs, qp, qr, part);
  };
  if (rs.buoy_adt != 0.0) {   // theta first, then Psi with the new theta's buoyancy
    go(1, nbr);
    go(2, nbp);
  } else {
    go(0, nbp + nbr);
  }
  return true;
}

int solve_np_pad() { return NSET * SB; }

}  // namespace qg
