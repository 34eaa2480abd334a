// C ABI of the QG step: context, workspace layout, host-side factorisation,
// and the kernel sequences of the time schemes (CNAB2, SBDF2-4, BPR353,
// ARS222, ARS443).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "../../include/qg.h"
#include "host_ops.h"
#include "kernels.h"

namespace qg {
size_t solve_lds_bytes(const Geom& g, int kutp, int kutr);
void launch_rhs(const Geom& g, const Bands& b, const RhsSpec& rs, double2* rhs, int mch,
                hipStream_t st);
void launch_lin(const Geom& g, const Bands& b, const double2* ypsi, const double2* yth,
                double2* lpsi, double2* lth, int mch, hipStream_t st);
void launch_rhs_terms(const Geom& g, const RhsSpec& rs, double2* rhs, hipStream_t st);
bool band_mch_ok(int mch);
void launch_combine(const Combine& cb, double2* out, size_t n, const int* nf, hipStream_t st);
void launch_copy(const double2* in, double2* out, size_t n, const int* nf, hipStream_t st);
void launch_solve_adjoint(const Geom& g, const FactorSet<double2>& Fp, const FactorSet<double>& Fr,
                          int q4, int q2, double2* psi, double2* th, hipStream_t st);
void launch_band_adjoint(const Geom& g, const Bands& b, double c, const double2* mu_psi,
                         const double2* mu_th, double2* out_psi, double2* out_th, hipStream_t st);
bool launch_solve(const Geom& g, const FactorSet<double2>& Fp, const FactorSet<double>& Fr,
                  double2* rhs, const RhsSpec& rs, int kutp, int kutr, bool pivoted,
                  hipStream_t st);
int solve_batch();
bool launch_solve_np(const Geom& g, const Bands& bd, const FactorSet<double2>& Fp,
                     const FactorSet<double>& Fr, double2* rhs, const RhsSpec& rs, int qp, int qr,
                     bool galerkin, hipStream_t st);
int solve_np_pad();
bool launch_explicit_T(const Geom& g, const Bands& b, const double2* X, const double* G,
                       const double2* Ea, const double2* Eb, double ca, double cb, size_t mk,
                       double kappa, double2* NLb, double* zb, double2* thb0, double2* Xb,
                       const double2* add, const double2* mu, double cmu, double2* ml,
                       double2* psib, double2* thb, hipStream_t st);
void launch_energy_total(const double* diag, int M, int N, double c, double* J,
                         hipStream_t st);
void launch_transpose_factors(const FactorSet<double2>& Fp, const FactorSet<double>& Fr, int Sp,
                              int Sr, int n4, int n2, int qp, int qr, double2* pLT, double2* pUT,
                              double2* puiT, double* rLT, double* rUT, double* ruiT,
                              hipStream_t st);
bool launch_solve_adjoint_np(const Geom& g, const FactorSet<double2>& FpT,
                             const FactorSet<double>& FrT, int qp, int qr, double2* f_psi,
                             double2* f_th, double2* y_psi, double2* y_th, hipStream_t st);
void launch_to_internal(int M, int K, const double2* psi, const double2* th, const double* u,
                        double2* dp, double2* dt, hipStream_t st);
void launch_to_api(int M, int K, const double2* sp, const double2* sth, double2* psi,
                   double2* th, double* u, hipStream_t st);
}  // namespace qg

using namespace qg;

namespace {

// Stiffly accurate SDIRK schemes with an explicit first stage (paper
// Sect. 4, eq. dirks; Table 1): s stages, a_ii = diag for i >= 1, the last
// stage is the new state.
struct Dirk {
  int s;
  double diag;
  double AE[5][5];
  double AI[5][5];
};

// BPR353: Boscarino, Pareschi & Russo (2013), Sect. 8.3.
const Dirk BPR353 = {5,
                     0.5,
                     {{0, 0, 0, 0, 0},
                      {1, 0, 0, 0, 0},
                      {4.0 / 9, 2.0 / 9, 0, 0, 0},
                      {0.25, 0, 0.75, 0, 0},
                      {0.25, 0, 0.75, 0, 0}},
                     {{0, 0, 0, 0, 0},
                      {0.5, 0.5, 0, 0, 0},
                      {5.0 / 18, -1.0 / 9, 0.5, 0, 0},
                      {0.5, 0, 0, 0.5, 0},
                      {0.25, 0, 0.75, -0.5, 0.5}}};

// ARS222: Ascher, Ruuth & Spiteri (1997), Sect. 2.6, with
// gamma = 1 - 1/sqrt 2 and delta = 1 - 1/(2 gamma).
const double ARS_G = 1.0 - 1.0 / std::sqrt(2.0);
const double ARS_D = 1.0 - 1.0 / (2.0 * ARS_G);
const Dirk ARS222 = {3,
                     ARS_G,
                     {{0, 0, 0}, {ARS_G, 0, 0}, {ARS_D, 1.0 - ARS_D, 0}},
                     {{0, 0, 0}, {0, ARS_G, 0}, {0, 1.0 - ARS_G, ARS_G}}};

// ARS443: the same paper, Sect. 2.8.
const Dirk ARS443 = {5,
                     0.5,
                     {{0, 0, 0, 0, 0},
                      {0.5, 0, 0, 0, 0},
                      {11.0 / 18, 1.0 / 18, 0, 0, 0},
                      {5.0 / 6, -5.0 / 6, 0.5, 0, 0},
                      {0.25, 1.75, 0.75, -1.75, 0}},
                     {{0, 0, 0, 0, 0},
                      {0, 0.5, 0, 0, 0},
                      {0, 1.0 / 6, 0.5, 0, 0},
                      {0, -0.5, 0.5, 0.5, 0},
                      {0, 1.5, -1.5, 0.5, 0.5}}};

// SBDFk (Table 1): sum_{j=0}^{k} a_j y^{n+1-j} = dt (L y^{n+1}
// + sum_{j=1}^{k} b_j E^{n+1-j}), the mass matrix on every y.
struct Sbdf {
  int k;
  double a[5];
  double b[4];
};
const Sbdf SBDF2 = {2, {1.5, -2.0, 0.5}, {2.0, -1.0}};
const Sbdf SBDF3 = {3, {11.0 / 6, -3.0, 1.5, -1.0 / 3}, {3.0, -3.0, 1.0}};
const Sbdf SBDF4 = {4, {25.0 / 12, -4.0, 3.0, -4.0 / 3, 0.25}, {4.0, -6.0, 4.0, -1.0}};

const Dirk* dirk_of(int scheme) {
  switch (scheme) {
    case QG_BPR353: return &BPR353;
    case QG_ARS222: return &ARS222;
    case QG_ARS443: return &ARS443;
    default: return nullptr;
  }
}

const Sbdf* sbdf_of(int scheme) {
  switch (scheme) {
    case QG_SBDF2: return &SBDF2;
    case QG_SBDF3: return &SBDF3;
    case QG_SBDF4: return &SBDF4;
    default: return nullptr;
  }
}

struct Layout {
  size_t total = 0;
  size_t take(size_t bytes) {
    size_t off = total;
    total += (bytes + 255) / 256 * 256;
    return off;
  }
};

// qg_params.dct = 0: the radial transforms of FP64 contexts with
// 2 (N_r - 1) <= MFMA_DCT_MAX_N2 run on the matrix cores when this is set.
constexpr bool MFMA_DCT_DEFAULT = false;

struct Sizes {
  int M, K, R, nphi, n4, n2, Sr;
  bool pump;    // Ekman pumping terms
  bool gal;     // Galerkin bases (qg_params.method = 1)
  bool mfdct;   // radial transforms on the matrix cores (qg_params.dct)
  int p4, p2;   // n4, n2 padded to whole 16-step batches (pivoted solve)
  int q4, q2;   // n4, n2 padded to whole groups of solve batches (unpivoted solve)
};

bool sizes_of(const qg_params* p, Sizes& z, std::string& why) {
  if (!p) { why = "null parameters"; return false; }
  if (!(p->E > 0 && p->Ra > 0 && p->Pr > 0)) { why = "E, Ra and Pr must be positive"; return false; }
  if (!(p->eta > 0 && p->eta < 1)) { why = "eta must lie in (0, 1)"; return false; }
  if (p->n_phi % 3 || p->n_phi < 24) { why = "n_phi must be a multiple of 3, >= 24"; return false; }
  if (p->n_r < 17) { why = "n_r must be >= 17"; return false; }
  int K = p->n_c ? p->n_c : (2 * (p->n_r - 1)) / 3;
  if (K < 8 || K >= p->n_r) { why = "n_c must satisfy 8 <= n_c < n_r"; return false; }
  if (p->precision != 0 && p->precision != 1) { why = "precision must be 0 or 1"; return false; }
  if (p->pivoting != 0 && p->pivoting != 1) { why = "pivoting must be 0 or 1"; return false; }
  if (p->ekman != 0 && p->ekman != 1) { why = "ekman must be 0 or 1"; return false; }
  if (p->method != 0 && p->method != 1) { why = "method must be 0 (tau) or 1 (Galerkin)"; return false; }
  if (p->buoyancy != 0 && p->buoyancy != 1) { why = "buoyancy must be 0 (explicit) or 1 (implicit)"; return false; }
  if (p->dct < 0 || p->dct > 2) { why = "dct must be 0 (default), 1 (FFT) or 2 (matrix cores)"; return false; }
  if (p->ekman && !(p->eps > 0 && std::isfinite(p->eps))) {
    why = "eps must be positive with Ekman pumping";
    return false;
  }
  z.pump = p->ekman == 1;
  z.gal = p->method == 1;
  {
    const bool mf_ok = p->precision == 0 && 2 * (p->n_r - 1) <= MFMA_DCT_MAX_N2;
    z.mfdct = mf_ok && (p->dct == 2 || (p->dct == 0 && MFMA_DCT_DEFAULT));
  }
  z.M = p->n_phi / 3 + 1;
  z.K = K;
  z.R = p->n_r;
  z.nphi = p->n_phi;
  z.n4 = K - 4;
  z.n2 = K - 2;
  z.p4 = (z.n4 + 15) / 16 * 16;   // whole solve batches (16 steps)
  z.p2 = (z.n2 + 15) / 16 * 16;
  const int qpad = solve_np_pad();   // unpivoted solve: whole groups of prefetched batches
  z.q4 = (z.n4 + qpad - 1) / qpad * qpad;
  z.q2 = (z.n2 + qpad - 1) / qpad * qpad;
  z.Sr = z.M + 1;
  return true;
}

struct WsMap {
  size_t ra, flag;
  size_t state, ybuf, eslot, lslot, mE, mY, pump, tan, X, NL, zonal, rate, diag, xk, wq, dsk, twd, twp, twh, wphi,
      twd32, twp32, twh32, wphi32, bands, rhs;
  size_t p_piv, p_L, p_U, p_W, p_C, p_Mi, p_ui, p_gam;
  size_t dct_s, dct_a;   // matrix-core radial transform tables
  size_t r_piv, r_L, r_U, r_W, r_C, r_Mi, r_ui;
  size_t total;
};

// Per-run arrays are sized for nmem runs (run-major inside each array, see
// Geom); operators, tables and factors are shared by the runs.
WsMap map_workspace(const Sizes& z, int nmem, bool single) {
  Layout L;
  WsMap w;
  const size_t nm = (size_t)nmem;
  const size_t MK = nm * z.M * z.K * sizeof(double2);
  const size_t RM = nm * z.R * z.M * sizeof(double2);
  const size_t Sp = z.M - 1;
  w.ra = L.take(nm * sizeof(double));
  w.flag = L.take(sizeof(int));
  // single runs keep two state slots: a step writes the other one, so that
  // a step that produces a non-finite state can be discarded
  w.state = L.take((single ? 4 : 2) * MK);
  w.ybuf = L.take(4 * MK);
  w.eslot = L.take(8 * MK);   // DIRK explicit stages (4)
  w.lslot = L.take(8 * MK);   // DIRK implicit stage products (4)
  w.mE = L.take(8 * MK);      // SBDF explicit terms E^n .. E^{n-3}
  w.mY = L.take(6 * MK);      // SBDF past states y^{n-1} .. y^{n-3}
  w.pump = L.take(z.pump ? RM : 0);   // Ekman pumping terms [M][R] per run
  w.tan = L.take(single ? 10 * MK : 0);   // tangent state, its E history, y +- c d
  w.X = L.take(6 * RM);
  w.NL = L.take(2 * RM);
  w.zonal = L.take(nm * z.R * sizeof(double));
  w.rate = L.take(nm * z.R * sizeof(double));
  w.diag = L.take(nm * z.M * 8 * sizeof(double));
  w.xk = L.take(z.R * sizeof(double));
  w.wq = L.take(z.R * sizeof(double));
  w.dsk = L.take(z.R * sizeof(double));
  w.twd = L.take((size_t)2 * (z.R - 1) * sizeof(double2));
  w.twp = L.take((size_t)z.nphi * sizeof(double2));
  w.twh = L.take((size_t)z.nphi / 2 * sizeof(double2));
  w.wphi = L.take((size_t)(z.nphi / 2 + 1) * sizeof(double2));
  w.twd32 = L.take((size_t)2 * (z.R - 1) * sizeof(float2));
  w.twp32 = L.take((size_t)z.nphi * sizeof(float2));
  w.twh32 = L.take((size_t)z.nphi / 2 * sizeof(float2));
  w.wphi32 = L.take((size_t)(z.nphi / 2 + 1) * sizeof(float2));
  w.bands = L.take((size_t)9 * z.K * BANDW * sizeof(double));
  w.rhs = L.take(2 * MK);
  w.p_piv = L.take(Sp * z.p4 * sizeof(int));
  w.p_L = L.take(Sp * std::max(z.p4, z.q4) * 8 * sizeof(double2));
  // U: pivoted 17 columns, unpivoted 8 (tau) or 12 (Galerkin)
  w.p_U = L.take(Sp * std::max(z.p4 * 17, z.q4 * (z.gal ? 12 : 8)) * sizeof(double2));
  w.p_ui = L.take(Sp * z.q4 * sizeof(double2));
  w.p_W = L.take(Sp * 4 * z.n4 * sizeof(double2));
  w.p_C = L.take(Sp * 8 * 4 * sizeof(double2));
  w.p_Mi = L.take(Sp * 16 * sizeof(double2));
  const size_t Sr = z.Sr;
  w.r_piv = L.take(Sr * z.p2 * sizeof(int));
  w.r_L = L.take(Sr * std::max(z.p2, z.q2) * 4 * sizeof(double));
  w.r_U = L.take(Sr * std::max(z.p2 * 9, z.q2 * (z.gal ? 6 : 4)) * sizeof(double));
  w.r_ui = L.take(Sr * z.q2 * sizeof(double));
  w.r_W = L.take(Sr * 2 * z.n2 * sizeof(double));
  w.r_C = L.take(Sr * 4 * 2 * sizeof(double));
  w.r_Mi = L.take(Sr * 4 * sizeof(double));
  w.p_gam = L.take(z.gal ? (size_t)z.n4 * 5 * sizeof(double) : 0);   // Galerkin stencil of Psi
  w.dct_s = L.take(z.mfdct ? mfma_dct_table_bytes(z.R, z.K, false) : 0);
  w.dct_a = L.take(z.mfdct ? mfma_dct_table_bytes(z.R, z.K, true) : 0);
  w.total = L.total;
  return w;
}

}  // namespace

struct qg_ctx {
  qg_params p;
  Sizes z;
  WsMap w;
  int nmem = 1;              // runs stepped together (an ensemble group)
  bool single = true;        // a qg_create context (not an ensemble group)
  int static_dev = -1;       // device whose static workspace this context holds
  char* ws = nullptr;
  hipStream_t st = nullptr;
  Operators ops;
  Geom g;
  Bands b;
  FactorSet<double2> Fp;
  FactorSet<double> Fr;
  int kutp = 16, kutr = 8;   // stored U super-diagonals (Psi, real systems)
  int band_mch = 16;         // systems per thread of the band products
  bool pivoted = true;       // band LU with row interchanges in use
  bool galerkin = false;     // Galerkin bases (pure band systems, no border)
  bool mixed = false;        // FP32 transforms and products (qg_params.precision = 1)
  bool diag64 = true;        // FP64 transform kernels exist for the diagnostics
  double growth = 0.0;       // largest growth factor of the band LUs in use
  double factored_adt = -1.0;
  int have_prev = 0, cur = 0;   // CNAB2 history
  int ms_n = 0;                 // SBDF levels stored since the history began
  int t_set = 0, t_have_prev = 0, t_cur = 0;   // tangent-linear run (qg_step_tangent)
  double t_scale = 1.0;                        // c of the difference quotient
  int last_scheme = -1;         // scheme and dt of the history
  double last_dt = 0.0;
  double t = 0.0;
  long long step = 0;
  std::string err;
  // A second stream of a single run (default priority), held for the
  // duration of one stepping call: the band product of a CNAB2 right-hand
  // side, which needs only y^n, runs there beside the synthesis, ring and
  // analysis.  A stream kept between calls would take one of the process's
  // few hardware queues from other work (measured: a 64-run ensemble
  // stepped 10% slower beside an idle context that held one).
  hipStream_t st2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // per-kernel timing (qg_step_timed): events recorded around each launch
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_marks;
  double2* ptr2(size_t off) { return reinterpret_cast<double2*>(ws + off); }
  double* ptrd(size_t off) { return reinterpret_cast<double*>(ws + off); }
  size_t mk() const { return (size_t)nmem * z.M * z.K; }   // one field of every run
  int sidx = 0;               // state slot of a single run (two slots)
  int tag = 0;                // step number within the current call (non-finite flag)
  double2* psi() { return ptr2(w.state) + (size_t)(2 * sidx) * mk(); }
  double2* th() { return psi() + mk(); }
  // where a step writes the new state: the other slot of a single run,
  // in place for the runs of an ensemble group (their graphs capture the
  // pointers)
  double2* nxt_psi() { return single ? ptr2(w.state) + (size_t)(2 * (1 - sidx)) * mk() : psi(); }
  double2* nxt_th() { return nxt_psi() + mk(); }
  void flip() { if (single) sidx ^= 1; }
  int* nf_flag() { return reinterpret_cast<int*>(ws + w.flag); }
  double2* slot(size_t base, int i, int field) {
    return ptr2(base) + ((size_t)(2 * i + field)) * mk();
  }
  // tangent region: [0] the tangent state d (Psi/u, theta), [1], [2] its
  // explicit-term history, [3] y + c d, [4] y - c d; each 2 mk entries
  double2* tng(int i) { return ptr2(w.tan) + (size_t)(2 * i) * mk(); }
};

#define HIPCHK(expr)                                                           \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);            \
      return QG_EDEVICE;                                                       \
    }                                                                          \
  } while (0)

namespace {

qg_status fail(qg_ctx* ctx, qg_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

std::vector<double2> twiddles(int n) {
  std::vector<double2> tw(n);
  for (int k = 0; k < n; ++k) {
    long double a = -2.0L * 3.14159265358979323846264338327950288L * k / n;
    tw[k] = make_double2((double)cosl(a), (double)sinl(a));
  }
  return tw;
}

// Clenshaw-Curtis weights on x_k = cos(pi k / N), k = 0..N.
std::vector<double> cc_weights(int nr) {
  const int N = nr - 1;
  std::vector<double> w(nr, 0.0);
  const double pi = 3.14159265358979323846;
  for (int k = 0; k <= N; ++k) {
    double th = pi * k / N, v = 1.0;
    for (int j = 1; j <= N / 2; ++j) {
      double bj = (2 * j == N) ? 1.0 : 2.0;
      v -= bj * std::cos(2.0 * j * th) / (4.0 * j * j - 1.0);
    }
    double ck = (k == 0 || k == N) ? 1.0 : 2.0;
    w[k] = ck * v / N;
  }
  return w;
}

// Full K x K tau matrix of one system, dense rows (host), from the bands.
template <typename T>
void assemble(const qg_ctx* ctx, int kind, int m, double adt, std::vector<T>& full, int& p) {
  const int K = ctx->z.K;
  const Operators& o = ctx->ops;
  full.assign((size_t)K * K, T(0));
  p = (kind == 0) ? 4 : 2;
  std::vector<double> row(K);
  for (int r = 0; r < p; ++r) {
    tau_row(r, K, row.data());
    for (int n = 0; n < K; ++n) full[(size_t)r * K + n] = T(row[n]);
  }
  const double m2 = (double)m * m;
  for (int k = p; k < K; ++k)
    for (int off = -8; off <= 8; ++off) {
      int n = k + off;
      if (n < 0 || n >= K) continue;
      size_t i = (size_t)k * BANDW + off + BANDC;
      T v;
      if (kind == 0) {
        double re = o.A0[i] + m2 * o.A2[i] - adt * (o.B0[i] + m2 * o.B2[i] + m2 * m2 * o.B4[i]);
        double im = -adt * (2.0 * m / ctx->p.E) * o.C[i];
        if constexpr (std::is_same<T, cplx>::value) v = cplx(re, im);
        else v = T(re);
      } else if (kind == 1) {  // zonal flow: D - a dt E, E = F0 + F2
        v = T(o.D[i] - adt * (o.F0[i] + o.F2[i]));
      } else {                 // theta: D - a dt F_m / Pr
        v = T(o.D[i] - adt * (o.F0[i] + m2 * o.F2[i]) / ctx->p.Pr);
      }
      full[(size_t)k * K + n] = v;
    }
}

// Largest row-interchange offset of a factorisation.
template <typename T>
int max_pivot(const BorderedFactor<T>& f) {
  int mx = 0;
  for (int v : f.piv) mx = std::max(mx, v);
  return mx;
}

// A host factor entry (long double, real or complex) rounded to the
// device type.
template <typename D2, typename T>
D2 to_dev(const T& v) {
  if constexpr (std::is_same<D2, double2>::value)
    return make_double2((double)std::real(v), (double)std::imag(v));
  else
    return (double)std::real(v);
}

// Device layout of one system: steps padded to npad with identity steps
// (no interchange, zero multipliers, U = 1), U truncated to wu columns
// (the dropped fill is checked to be exactly zero).
template <typename T, typename D2>
bool pack(const BorderedFactor<T>& f, size_t s, int kl, int wu, int p, int npad, int* piv, D2* L,
          D2* U, D2* W, D2* C, D2* Mi) {
  const int n = f.n, wfull = f.kut + 1;
  auto cvt = [](const T& v) -> D2 { return to_dev<D2>(v); };
  const T one(1.0);
  for (int j = 0; j < npad; ++j) {
    piv[s * npad + j] = (j < n) ? f.piv[j] : 0;
    for (int d = 0; d < kl; ++d)
      L[(s * npad + j) * kl + d] = cvt(j < n ? f.Lc[(size_t)j * kl + d] : T(0));
    for (int e = 0; e < wu; ++e)
      U[(s * npad + j) * wu + e] = cvt(j < n ? f.Uc[(size_t)j * wfull + e] : (e == 0 ? one : T(0)));
    if (j < n)
      for (int e = wu; e < wfull; ++e)
        if (f.Uc[(size_t)j * wfull + e] != T(0)) return false;
  }
  for (size_t i = 0; i < (size_t)p * n; ++i) W[s * p * n + i] = cvt(f.W[i]);
  for (size_t i = 0; i < (size_t)kl * p; ++i) C[s * kl * p + i] = cvt(f.Cb[i]);
  for (size_t i = 0; i < (size_t)p * p; ++i) Mi[s * p * p + i] = cvt(f.Minv[i]);
  return true;
}

// Unpivoted layout of one system: multipliers L [q][kl], U scaled to a
// unit diagonal by rows, column-wise [q][ku], and 1/U(j,j) [q]; steps past
// n are identity steps (zero multipliers, unit diagonal).
template <typename T, typename D2>
void pack_np(const BorderedFactor<T>& f, size_t s, int kl, int ku, int p, int q, D2* L, D2* U,
             D2* ui, D2* W, D2* C, D2* Mi) {
  const int n = f.n, wf = f.kut + 1;
  auto cvt = [](const T& v) -> D2 { return to_dev<D2>(v); };
  for (int j = 0; j < q; ++j) {
    for (int d = 0; d < kl; ++d)
      L[(s * q + j) * kl + d] = cvt(j < n ? f.Lc[(size_t)j * kl + d] : T(0));
    for (int e = 1; e <= ku; ++e) {
      T v(0);
      if (j < n && j - e >= 0) v = f.Uc[(size_t)j * wf + e] * f.Uc[(size_t)(j - e) * wf];
      U[(s * q + j) * ku + (e - 1)] = cvt(v);
    }
    ui[s * q + j] = cvt(j < n ? f.Uc[(size_t)j * wf] : T(1));
  }
  for (size_t i = 0; i < (size_t)p * n; ++i) W[s * p * n + i] = cvt(f.W[i]);
  for (size_t i = 0; i < (size_t)kl * p; ++i) C[s * kl * p + i] = cvt(f.Cb[i]);
  for (size_t i = 0; i < (size_t)p * p; ++i) Mi[s * p * p + i] = cvt(f.Minv[i]);
}

template <typename F>
void parallel_for(int count, F fn) {
  unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (unsigned w = 0; w < hw; ++w)
    th.emplace_back([&, w] {
      for (int i = (int)w; i < count; i += (int)hw) fn(i);
    });
  for (auto& x : th) x.join();
}

// Unpivoted band LUs are used when every system's growth factor stays
// below this bound (their solve then needs no row interchanges); otherwise
// all systems are refactored with partial pivoting.
constexpr double MAX_UNPIVOTED_GROWTH = 1e4;

// Galerkin bases (Sect. 3.2.2): for every system P_q (mass - a dt L) S,
// formed and factored without row interchanges in long double, every
// factor entry then rounded once to binary64 (as for the tau systems); the
// Psi stencil's gamma_i^j rounded the same way for the device's y = S x~.
qg_status refactor_galerkin(qg_ctx* ctx, double adt) {
  const Sizes& z = ctx->z;
  const size_t Sp = z.M - 1, Sr = z.Sr;
  std::vector<BorderedFactor<cplxl>> fp(Sp);
  std::vector<BorderedFactor<long double>> fr(Sr);
  std::vector<int> ok(Sp + Sr, 1);
  // G must vanish outside its stated band (the factorisation reads only
  // the band)
  auto banded = [](const auto& G, int n, int kl, int ku) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        if ((j - i > ku || i - j > kl) && G[(size_t)i * n + j] != decltype(G[0])(0)) return false;
    return true;
  };
  parallel_for((int)(Sp + Sr), [&](int idx) {
    int p;
    if (idx < (int)Sp) {
      std::vector<cplx> full;
      assemble<cplx>(ctx, 0, idx + 1, adt, full, p);
      std::vector<cplxl> fl(full.begin(), full.end()), G;
      galerkin_matrix<cplxl>(fl, z.K, 4, G);
      ok[idx] = banded(G, z.n4, 8, 12) &&
                factor_bordered<cplxl>(G, z.n4, 0, 8, 12, false, fp[idx]);
    } else {
      const int s = idx - (int)Sp;
      std::vector<double> full;
      assemble<double>(ctx, s == 0 ? 1 : 2, s == 0 ? 0 : s - 1, adt, full, p);
      std::vector<long double> fl(full.begin(), full.end()), G;
      galerkin_matrix<long double>(fl, z.K, 2, G);
      ok[idx] = banded(G, z.n2, 4, 6) &&
                factor_bordered<long double>(G, z.n2, 0, 4, 6, false, fr[s]);
    }
  });
  double growth = 0.0;
  for (auto& f : fp) growth = std::max(growth, f.growth);
  for (auto& f : fr) growth = std::max(growth, f.growth);
  ctx->growth = growth;
  for (int v : ok)
    if (!v) return fail(ctx, QG_EINVAL, "singular Galerkin matrix (dt too large or bad parameters)");
  if (growth > MAX_UNPIVOTED_GROWTH)
    return fail(ctx, QG_EUNSUPPORTED,
                "Galerkin band LU without row interchanges grew by " + std::to_string(growth));
  const WsMap& w = ctx->w;
  auto up = [&](size_t off, const void* src, size_t bytes) {
    return hipMemcpyAsync(ctx->ws + off, src, bytes, hipMemcpyHostToDevice, ctx->st);
  };
  std::vector<double2> pL(Sp * z.q4 * 8), pU(Sp * z.q4 * 12), pui(Sp * z.q4);
  std::vector<double> rL(Sr * z.q2 * 4), rU(Sr * z.q2 * 6), rui(Sr * z.q2);
  double2 d2;
  double d1;
  parallel_for((int)(Sp + Sr), [&](int idx) {
    if (idx < (int)Sp)
      pack_np<cplxl, double2>(fp[idx], idx, 8, 12, 0, z.q4, pL.data(), pU.data(), pui.data(),
                             &d2, &d2, &d2);
    else
      pack_np<long double, double>(fr[idx - Sp], idx - Sp, 4, 6, 0, z.q2, rL.data(), rU.data(),
                                  rui.data(), &d1, &d1, &d1);
  });
  std::vector<double> gam((size_t)z.n4 * 5);
  for (int j = 0; j < z.n4; ++j) {
    long double g[5];
    galerkin_gamma(j, g);
    for (int i = 0; i < 5; ++i) gam[(size_t)j * 5 + i] = (double)g[i];
  }
  HIPCHK(up(w.p_L, pL.data(), pL.size() * sizeof(double2)));
  HIPCHK(up(w.p_U, pU.data(), pU.size() * sizeof(double2)));
  HIPCHK(up(w.p_ui, pui.data(), pui.size() * sizeof(double2)));
  HIPCHK(up(w.r_L, rL.data(), rL.size() * sizeof(double)));
  HIPCHK(up(w.r_U, rU.data(), rU.size() * sizeof(double)));
  HIPCHK(up(w.r_ui, rui.data(), rui.size() * sizeof(double)));
  HIPCHK(up(w.p_gam, gam.data(), gam.size() * sizeof(double)));
  HIPCHK(hipStreamSynchronize(ctx->st));
  ctx->pivoted = false;
  ctx->galerkin = true;
  ctx->factored_adt = adt;
  return QG_OK;
}

qg_status refactor(qg_ctx* ctx, double adt) {
  if (ctx->z.gal) return refactor_galerkin(ctx, adt);
  const Sizes& z = ctx->z;
  const size_t Sp = z.M - 1, Sr = z.Sr;
  std::vector<BorderedFactor<cplxl>> fp(Sp);
  std::vector<BorderedFactor<long double>> fr(Sr);
  std::vector<int> ok(Sp + Sr, 1);
  bool pivot = ctx->p.pivoting != 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    // each factorisation runs in long double (the band LU, the border data
    // w = B D^-1 with its long recurrences, and M^-1), then every entry is
    // rounded once to FP64: the stored factors are accurate to the last bit
    // and only the device's substitutions round in FP64
    parallel_for((int)(Sp + Sr), [&](int idx) {
      int p;
      if (idx < (int)Sp) {
        std::vector<cplx> full;
        assemble<cplx>(ctx, 0, idx + 1, adt, full, p);
        std::vector<cplxl> fl(full.begin(), full.end());
        ok[idx] = factor_bordered<cplxl>(fl, z.K, 4, 8, 8, pivot, fp[idx]);
      } else {
        const int s = idx - (int)Sp;
        std::vector<double> full;
        assemble<double>(ctx, s == 0 ? 1 : 2, s == 0 ? 0 : s - 1, adt, full, p);
        std::vector<long double> fl(full.begin(), full.end());
        ok[idx] = factor_bordered<long double>(fl, z.K, 2, 4, 4, pivot, fr[s]);
      }
    });
    double growth = 0.0;
    bool good = true;
    for (int v : ok) good = good && v;
    for (auto& f : fp) growth = std::max(growth, f.growth);
    for (auto& f : fr) growth = std::max(growth, f.growth);
    ctx->growth = growth;
    if (pivot || (good && growth <= MAX_UNPIVOTED_GROWTH)) break;
    pivot = true;   // unpivoted elimination broke down or grew: pivot everywhere
    std::fill(ok.begin(), ok.end(), 1);
  }
  for (int v : ok)
    if (!v) return fail(ctx, QG_EINVAL, "singular tau matrix (dt too large or bad parameters)");
  int mp = 0, mr = 0;
  for (auto& f : fp) mp = std::max(mp, max_pivot(f));
  for (auto& f : fr) mr = std::max(mr, max_pivot(f));
  const int kutp = !pivot ? 8 : ((8 + mp <= 12) ? 12 : 16);
  const int kutr = !pivot ? 4 : ((4 + mr <= 4) ? 4 : 8);
  const WsMap& w = ctx->w;
  auto up = [&](size_t off, const void* src, size_t bytes) {
    return hipMemcpyAsync(ctx->ws + off, src, bytes, hipMemcpyHostToDevice, ctx->st);
  };
  std::vector<double2> pW(Sp * 4 * z.n4), pC(Sp * 32), pM(Sp * 16);
  std::vector<double> rW(Sr * 2 * z.n2), rC(Sr * 8), rM(Sr * 4);
  if (pivot) {
    std::vector<int> ppiv(Sp * z.p4), rpiv(Sr * z.p2);
    std::vector<double2> pL(Sp * z.p4 * 8), pU(Sp * z.p4 * (kutp + 1));
    std::vector<double> rL(Sr * z.p2 * 4), rU(Sr * z.p2 * (kutr + 1));
    parallel_for((int)(Sp + Sr), [&](int idx) {
      if (idx < (int)Sp)
        ok[idx] = pack<cplxl, double2>(fp[idx], idx, 8, kutp + 1, 4, z.p4, ppiv.data(), pL.data(),
                                      pU.data(), pW.data(), pC.data(), pM.data());
      else
        ok[idx] = pack<long double, double>(fr[idx - Sp], idx - Sp, 4, kutr + 1, 2, z.p2, rpiv.data(),
                                       rL.data(), rU.data(), rW.data(), rC.data(), rM.data());
    });
    for (int v : ok)
      if (!v) return fail(ctx, QG_EINVAL, "internal: band fill beyond the stored width");
    HIPCHK(up(w.p_piv, ppiv.data(), ppiv.size() * sizeof(int)));
    HIPCHK(up(w.p_L, pL.data(), pL.size() * sizeof(double2)));
    HIPCHK(up(w.p_U, pU.data(), pU.size() * sizeof(double2)));
    HIPCHK(up(w.r_piv, rpiv.data(), rpiv.size() * sizeof(int)));
    HIPCHK(up(w.r_L, rL.data(), rL.size() * sizeof(double)));
    HIPCHK(up(w.r_U, rU.data(), rU.size() * sizeof(double)));
    HIPCHK(hipStreamSynchronize(ctx->st));
  } else {
    std::vector<double2> pL(Sp * z.q4 * 8), pU(Sp * z.q4 * 8), pui(Sp * z.q4);
    std::vector<double> rL(Sr * z.q2 * 4), rU(Sr * z.q2 * 4), rui(Sr * z.q2);
    parallel_for((int)(Sp + Sr), [&](int idx) {
      if (idx < (int)Sp)
        pack_np<cplxl, double2>(fp[idx], idx, 8, 8, 4, z.q4, pL.data(), pU.data(), pui.data(),
                               pW.data(), pC.data(), pM.data());
      else
        pack_np<long double, double>(fr[idx - Sp], idx - Sp, 4, 4, 2, z.q2, rL.data(), rU.data(),
                                rui.data(), rW.data(), rC.data(), rM.data());
    });
    HIPCHK(up(w.p_L, pL.data(), pL.size() * sizeof(double2)));
    HIPCHK(up(w.p_U, pU.data(), pU.size() * sizeof(double2)));
    HIPCHK(up(w.p_ui, pui.data(), pui.size() * sizeof(double2)));
    HIPCHK(up(w.r_L, rL.data(), rL.size() * sizeof(double)));
    HIPCHK(up(w.r_U, rU.data(), rU.size() * sizeof(double)));
    HIPCHK(up(w.r_ui, rui.data(), rui.size() * sizeof(double)));
    HIPCHK(hipStreamSynchronize(ctx->st));
  }
  HIPCHK(up(w.p_W, pW.data(), pW.size() * sizeof(double2)));
  HIPCHK(up(w.p_C, pC.data(), pC.size() * sizeof(double2)));
  HIPCHK(up(w.p_Mi, pM.data(), pM.size() * sizeof(double2)));
  HIPCHK(up(w.r_W, rW.data(), rW.size() * sizeof(double)));
  HIPCHK(up(w.r_C, rC.data(), rC.size() * sizeof(double)));
  HIPCHK(up(w.r_Mi, rM.data(), rM.size() * sizeof(double)));
  HIPCHK(hipStreamSynchronize(ctx->st));
  ctx->kutp = kutp;
  ctx->kutr = kutr;
  ctx->pivoted = pivot;
  ctx->factored_adt = adt;
  return QG_OK;
}

// Kernel classes timed by qg_step_timed.
enum { K_SYNTH = 0, K_RING = 1, K_ANALYSIS = 2, K_SOLVE = 3, K_RHS = 4, K_COUNT = 5 };

hipEvent_t next_event(qg_ctx* ctx) {
  if (ctx->ev_used == ctx->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->ev_pool.push_back(e);
  }
  return ctx->ev_pool[ctx->ev_used++];
}

template <typename F>
void timed(qg_ctx* ctx, int cls, F launch) {
  if (!ctx->prof) { launch(); return; }
  hipEvent_t a = next_event(ctx), b = next_event(ctx);
  if (a) (void)hipEventRecord(a, ctx->st);
  launch();
  if (b) (void)hipEventRecord(b, ctx->st);
  if (a && b) ctx->ev_marks.push_back({cls, {a, b}});
}

// E(y) into (Ep, Et); diag (optional): the synthesis's per-m diagnostics
// of y (kinetic energy and the rest, see synth_kernel).
// X: where the synthesis writes the fields (default: the workspace's); G:
// the ring's grid fields out (reverse mode, optional); NL, zonal: the
// exchange arrays (default: the workspace's).
qg_status explicit_terms(qg_ctx* ctx, const double2* psi, const double2* th, double2* Ep,
                         double2* Et, double* diag = nullptr, double2* X = nullptr,
                         double* G = nullptr, double2* NL = nullptr, double* zonal = nullptr) {
  bool ok = true;
  if (!X) X = ctx->ptr2(ctx->w.X);
  if (!NL) NL = ctx->ptr2(ctx->w.NL);
  if (!zonal) zonal = ctx->ptrd(ctx->w.zonal);
  timed(ctx, K_SYNTH, [&] {
    ok = launch_synth(ctx->g, psi, th, X, diag, ctx->mixed, ctx->st) && ok;
  });
  timed(ctx, K_RING, [&] {
    ok = launch_ring(ctx->g, X, NL, zonal, nullptr, ctx->mixed, ctx->st, G) && ok;
  });
  timed(ctx, K_ANALYSIS, [&] {
    ok = launch_analysis(ctx->g, ctx->b, NL, zonal, th, Ep, Et, ctx->mixed, ctx->st) && ok;
  });
  if (!ok) return fail(ctx, QG_EUNSUPPORTED, "no transform kernel for these sizes");
  HIPCHK(hipGetLastError());
  return QG_OK;
}

// rhs: the right-hand side buffer (default: the workspace's); rhs_done:
// the caller has already formed it.
qg_status implicit_solve(qg_ctx* ctx, const RhsSpec& rs_in, double2* rhs = nullptr,
                         bool rhs_done = false) {
  RhsSpec rs = rs_in;
  rs.tag = ctx->tag;
  rs.buoy_adt = ctx->g.buoy_implicit ? ctx->factored_adt : 0.0;
  if (ctx->g.buoy_implicit && ctx->pivoted)
    return fail(ctx, QG_EUNSUPPORTED,
                "implicit buoyancy needs the unpivoted factors (growth factor above the bound)");
  if (!rhs) rhs = ctx->ptr2(ctx->w.rhs);
  if (!rhs_done)
    timed(ctx, K_RHS, [&] { launch_rhs(ctx->g, ctx->b, rs, rhs, ctx->band_mch, ctx->st); });
  bool ok = true;
  timed(ctx, K_SOLVE, [&] {
    ok = ctx->pivoted
             ? launch_solve(ctx->g, ctx->Fp, ctx->Fr, rhs, rs, ctx->kutp, ctx->kutr, true,
                            ctx->st)
             : launch_solve_np(ctx->g, ctx->b, ctx->Fp, ctx->Fr, rhs, rs, ctx->z.q4, ctx->z.q2, ctx->galerkin,
                               ctx->st);
  });
  if (!ok) return fail(ctx, QG_EUNSUPPORTED, "no solve kernel for this band width");
  if (rs.lin_psi)
    launch_lin(ctx->g, ctx->b, rs.out_psi, rs.out_th, rs.lin_psi, rs.lin_th, ctx->band_mch,
               ctx->st);
  HIPCHK(hipGetLastError());
  return QG_OK;
}

// True when a CNAB2 step of this context may put its band product on the
// second stream: a single run with a workspace of its own (the static
// workspace's callers create no streams), not timed per kernel, on a
// stream that no graph is capturing.
bool overlap_rhs(qg_ctx* ctx) {
  if (!ctx->single || ctx->static_dev >= 0 || ctx->prof) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(ctx->st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return false;
  if (ctx->st2 && ctx->ev_fork && ctx->ev_join) return true;
  // the stream and events belong to the device of the context's stream,
  // whichever device is current
  int dev = 0, prev = 0;
  if (hipStreamGetDevice(ctx->st, &dev) != hipSuccess || hipGetDevice(&prev) != hipSuccess ||
      hipSetDevice(dev) != hipSuccess)
    return false;
  bool ok = true;
  if (!ctx->ev_fork &&
      hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) != hipSuccess) {
    ctx->ev_fork = nullptr;
    ok = false;
  }
  if (ok && !ctx->ev_join &&
      hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) != hipSuccess) {
    ctx->ev_join = nullptr;
    ok = false;
  }
  if (ok && !ctx->st2 &&
      hipStreamCreateWithFlags(&ctx->st2, hipStreamNonBlocking) != hipSuccess) {
    ctx->st2 = nullptr;
    ok = false;
  }
  (void)hipSetDevice(prev);
  return ok;
}

// Ends a stepping call: the second stream goes (its queued work still
// completes; the context's stream already waits for it through ev_join).
struct SideStreamRelease {
  qg_ctx* ctx;
  ~SideStreamRelease() {
    if (ctx && ctx->st2) {
      (void)hipStreamDestroy(ctx->st2);
      ctx->st2 = nullptr;
    }
  }
};

// The band product of a CNAB2 right-hand side, (A + (dt/2) L) y^n with no
// explicit term, into rhs on the second stream once the context's stream
// has reached this point (y^n written).
qg_status fork_band(qg_ctx* ctx, const double2* psi, const double2* th, double dt,
                    double2* rhs) {
  RhsSpec band{};
  band.base_psi = psi;
  band.base_th = th;
  band.cL = 0.5 * dt;
  band.nterm = 0;
  HIPCHK(hipEventRecord(ctx->ev_fork, ctx->st));
  HIPCHK(hipStreamWaitEvent(ctx->st2, ctx->ev_fork, 0));
  launch_rhs(ctx->g, ctx->b, band, rhs, ctx->band_mch, ctx->st2);
  HIPCHK(hipEventRecord(ctx->ev_join, ctx->st2));
  return QG_OK;
}

// The context's stream waits for the band product and adds the explicit
// terms of rs to it (the band kernel's term loop: the one-stream result
// bit for bit).
qg_status join_terms(qg_ctx* ctx, const RhsSpec& rs, double2* rhs) {
  HIPCHK(hipStreamWaitEvent(ctx->st, ctx->ev_join, 0));
  launch_rhs_terms(ctx->g, rs, rhs, ctx->st);
  return QG_OK;
}

qg_status step_cnab2(qg_ctx* ctx, double dt) {
  const int cur = ctx->cur, prev = 1 - cur;
  double2 *Ep = ctx->slot(ctx->w.eslot, cur, 0), *Et = ctx->slot(ctx->w.eslot, cur, 1);
  // (A + (dt/2) L) y^n needs no explicit term: on the second stream it
  // runs beside the transforms, and the terms are added after them.
  const bool ovl = overlap_rhs(ctx);
  double2* rhs = ctx->ptr2(ctx->w.rhs);
  if (ovl) {
    const qg_status f = fork_band(ctx, ctx->psi(), ctx->th(), dt, rhs);
    if (f != QG_OK) return f;
  }
  qg_status s = explicit_terms(ctx, ctx->psi(), ctx->th(), Ep, Et);
  if (s != QG_OK) {
    if (ovl) (void)hipStreamWaitEvent(ctx->st, ctx->ev_join, 0);
    return s;
  }
  RhsSpec rs{};
  rs.base_psi = ctx->psi();
  rs.base_th = ctx->th();
  rs.cL = 0.5 * dt;
  rs.nterm = 2;
  rs.term_psi[0] = Ep;
  rs.term_th[0] = Et;
  rs.coef[0] = 1.5 * dt;
  rs.term_psi[1] = ctx->have_prev ? ctx->slot(ctx->w.eslot, prev, 0) : Ep;
  rs.term_th[1] = ctx->have_prev ? ctx->slot(ctx->w.eslot, prev, 1) : Et;
  rs.coef[1] = -0.5 * dt;
  rs.out_psi = ctx->nxt_psi();
  rs.out_th = ctx->nxt_th();
  if (ovl) {
    s = join_terms(ctx, rs, rhs);
    if (s != QG_OK) return s;
  }
  s = implicit_solve(ctx, rs, rhs, ovl);
  if (s != QG_OK) return s;
  ctx->have_prev = 1;
  ctx->cur = prev;
  return QG_OK;
}

// One step of the tangent-linear CNAB2 model about the current state y^n
// (before y^n itself is stepped): with T^n = E'(y^n) d^n,
//   (M - dt/2 L) d^{n+1} = (M + dt/2 L) d^n + dt (3/2 T^n - 1/2 T^{n-1}),
// tau rows and projections as in the step.  E is quadratic in the state,
// so T^n = (E(y + c d) - E(y - c d)) / (2c) exactly in exact arithmetic;
// c ~ max|y| / max|d| balances the two roundings.  The first tangent step
// takes T^{-1} := T^0 if the state's own history starts there as well
// (E^{-1} := E^0, a function of y^0), else T^{-1} := 0 (the history is
// not perturbed).
qg_status step_tangent(qg_ctx* ctx, double dt) {
  const size_t mk = ctx->mk(), n2 = 2 * mk;
  const double cs = ctx->t_scale;
  Combine cb{};
  cb.nb = 2;
  cb.in[0] = ctx->psi();
  cb.in[1] = ctx->tng(0);
  cb.c[0] = 1.0;
  cb.c[1] = cs;
  launch_combine(cb, ctx->tng(3), n2, ctx->g.nf, ctx->st);
  cb.c[1] = -cs;
  launch_combine(cb, ctx->tng(4), n2, ctx->g.nf, ctx->st);
  double2* Ea = ctx->slot(ctx->w.eslot, 2, 0);   // E(y + c d), E(y - c d): DIRK
  double2* Eb = ctx->slot(ctx->w.eslot, 3, 0);   // stage slots, unused by CNAB2
  qg_status s = explicit_terms(ctx, ctx->tng(3), ctx->tng(3) + mk, Ea, Ea + mk);
  if (s == QG_OK) s = explicit_terms(ctx, ctx->tng(4), ctx->tng(4) + mk, Eb, Eb + mk);
  if (s != QG_OK) return s;
  const int cur = ctx->t_cur, prev = 1 - cur;
  Combine dq{};
  dq.nb = 2;
  dq.in[0] = Ea;
  dq.in[1] = Eb;
  dq.c[0] = 0.5 / cs;
  dq.c[1] = -0.5 / cs;
  launch_combine(dq, ctx->tng(1 + cur), n2, ctx->g.nf, ctx->st);
  RhsSpec rs{};
  rs.base_psi = ctx->tng(0);
  rs.base_th = ctx->tng(0) + mk;
  rs.cL = 0.5 * dt;
  rs.nterm = 1;
  rs.term_psi[0] = ctx->tng(1 + cur);
  rs.term_th[0] = ctx->tng(1 + cur) + mk;
  rs.coef[0] = 1.5 * dt;
  const double2* pe = ctx->t_have_prev ? ctx->tng(1 + prev)
                                       : (ctx->have_prev ? nullptr : ctx->tng(1 + cur));
  if (pe) {
    rs.term_psi[1] = pe;
    rs.term_th[1] = pe + mk;
    rs.coef[1] = -0.5 * dt;
    rs.nterm = 2;
  }
  rs.out_psi = ctx->tng(0);
  rs.out_th = ctx->tng(0) + mk;
  s = implicit_solve(ctx, rs);
  if (s != QG_OK) return s;
  ctx->t_have_prev = 1;
  ctx->t_cur = prev;
  return QG_OK;
}

qg_status step_dirk(qg_ctx* ctx, double dt, const Dirk& T) {
  // y_1 = y_n (explicit first stage); stages i = 2..s solve
  // (M - a_ii dt L) y_i = M y_n + dt sum_{j<i} (aE_ij E_j + aI_ij L y_j);
  // y_{n+1} = y_s.
  const int S = T.s;
  const double2* y0p = ctx->psi();
  const double2* y0t = ctx->th();
  const double2* yp[5] = {y0p, nullptr, nullptr, nullptr, nullptr};
  const double2* yt[5] = {y0t, nullptr, nullptr, nullptr, nullptr};
  for (int i = 1; i < S; ++i) {
    const int j = i - 1;
    bool need_e = false;
    for (int r = 0; r < S; ++r) need_e = need_e || T.AE[r][j] != 0.0;
    if (need_e) {
      qg_status s = explicit_terms(ctx, yp[j], yt[j], ctx->slot(ctx->w.eslot, j, 0),
                                   ctx->slot(ctx->w.eslot, j, 1));
      if (s != QG_OK) return s;
    }
    RhsSpec rs{};
    rs.base_psi = y0p;
    rs.base_th = y0t;
    rs.cL = dt * T.AI[i][0];
    rs.nterm = 0;
    for (int jj = 0; jj < i; ++jj) {
      if (T.AE[i][jj] != 0.0) {
        rs.term_psi[rs.nterm] = ctx->slot(ctx->w.eslot, jj, 0);
        rs.term_th[rs.nterm] = ctx->slot(ctx->w.eslot, jj, 1);
        rs.coef[rs.nterm++] = dt * T.AE[i][jj];
      }
      if (jj >= 1 && T.AI[i][jj] != 0.0) {
        rs.term_psi[rs.nterm] = ctx->slot(ctx->w.lslot, jj, 0);
        rs.term_th[rs.nterm] = ctx->slot(ctx->w.lslot, jj, 1);
        rs.coef[rs.nterm++] = dt * T.AI[i][jj];
      }
    }
    double2 *op, *ot;
    if (i == S - 1) {
      op = ctx->nxt_psi();
      ot = ctx->nxt_th();
    } else {
      int b = (i - 1) % 2;
      op = ctx->slot(ctx->w.ybuf, b, 0);
      ot = ctx->slot(ctx->w.ybuf, b, 1);
    }
    rs.out_psi = op;
    rs.out_th = ot;
    bool need_l = false;
    for (int r = i + 1; r < S; ++r) need_l = need_l || T.AI[r][i] != 0.0;
    rs.lin_psi = need_l ? ctx->slot(ctx->w.lslot, i, 0) : nullptr;
    rs.lin_th = need_l ? ctx->slot(ctx->w.lslot, i, 1) : nullptr;
    qg_status s = implicit_solve(ctx, rs);
    if (s != QG_OK) return s;
    yp[i] = op;
    yt[i] = ot;
  }
  return QG_OK;
}

// Autotuner candidates: systems per thread of the band products.
constexpr int TUNE_N = 4;
const int TUNE_MCH[TUNE_N] = {4, 8, 16, 32};

// The factorisation (mass - adt L) is refactored when adt changes
// (synchronises the stream).
qg_status prepare(qg_ctx* ctx, double adt) {
  if (adt != ctx->factored_adt) return refactor(ctx, adt);
  return QG_OK;
}

qg_status step_sbdf(qg_ctx* ctx, double dt, const Sbdf& S) {
  // Level n: E^n into ring slot n % 4, y^n into ring slot n % 3 (after
  // the combination has read y^{n-3} from that slot).  While fewer than k
  // levels exist the step is a BPR353 step (start-up).
  const int n = ctx->ms_n, k = S.k;
  qg_status s = explicit_terms(ctx, ctx->psi(), ctx->th(), ctx->slot(ctx->w.mE, n % 4, 0),
                               ctx->slot(ctx->w.mE, n % 4, 1));
  if (s != QG_OK) return s;
  double2* Yn = ctx->slot(ctx->w.mY, n % 3, 0);
  const size_t count = 2 * ctx->mk();
  if (n + 1 < k) {
    launch_copy(ctx->psi(), Yn, count, ctx->g.nf, ctx->st);
    s = prepare(ctx, BPR353.diag * dt);
    if (s == QG_OK) s = step_dirk(ctx, dt, BPR353);
  } else {
    s = prepare(ctx, dt / S.a[0]);
    if (s != QG_OK) return s;
    // (M - dt/a_0 L) y^{n+1} = M [sum_j (-a_{j+1}/a_0) y^{n-j}]
    //                          + dt/a_0 sum_j b_{j+1} E^{n-j}
    Combine cb{};
    cb.nb = k;
    cb.in[0] = ctx->psi();
    cb.c[0] = -S.a[1] / S.a[0];
    for (int j = 1; j < k; ++j) {
      cb.in[j] = ctx->slot(ctx->w.mY, (n - j) % 3, 0);
      cb.c[j] = -S.a[j + 1] / S.a[0];
    }
    double2* yc = ctx->slot(ctx->w.ybuf, 0, 0);
    launch_combine(cb, yc, 2 * ctx->mk(), ctx->g.nf, ctx->st);
    launch_copy(ctx->psi(), Yn, count, ctx->g.nf, ctx->st);
    RhsSpec rs{};
    rs.base_psi = yc;
    rs.base_th = ctx->slot(ctx->w.ybuf, 0, 1);
    rs.cL = 0.0;
    rs.nterm = k;
    for (int j = 0; j < k; ++j) {
      rs.term_psi[j] = ctx->slot(ctx->w.mE, (n - j) % 4, 0);
      rs.term_th[j] = ctx->slot(ctx->w.mE, (n - j) % 4, 1);
      rs.coef[j] = dt * S.b[j] / S.a[0];
    }
    rs.out_psi = ctx->nxt_psi();
    rs.out_th = ctx->nxt_th();
    s = implicit_solve(ctx, rs);
  }
  if (s != QG_OK) return s;
  ctx->ms_n = n + 1;
  return QG_OK;
}

// a_ii dt (or b_0 dt) of the scheme's implicit solves; SBDF start-up steps
// use BPR353's.
double scheme_adt(int scheme, double dt) {
  if (const Dirk* T = dirk_of(scheme)) return T->diag * dt;
  if (const Sbdf* S = sbdf_of(scheme)) return dt / S->a[0];
  return 0.5 * dt;   // CNAB2
}

// One step of any scheme; the new state goes to the other slot, which
// becomes the current one.
qg_status step_scheme(qg_ctx* ctx, double dt, int scheme) {
  qg_status s;
  if (const Dirk* T = dirk_of(scheme)) s = step_dirk(ctx, dt, *T);
  else if (const Sbdf* S = sbdf_of(scheme)) s = step_sbdf(ctx, dt, *S);
  else s = step_cnab2(ctx, dt);
  if (s == QG_OK) ctx->flip();
  return s;
}

// A multistep history belongs to the scheme and dt that made it.
void begin_history(qg_ctx* ctx, double dt, int scheme) {
  if (scheme != ctx->last_scheme || dt != ctx->last_dt) {
    ctx->have_prev = 0;
    ctx->ms_n = 0;
    ctx->last_scheme = scheme;
    ctx->last_dt = dt;
  }
}

}  // namespace

extern "C" {

qg_status qg_workspace_size(const qg_params* p, size_t* bytes) {
  Sizes z;
  std::string why;
  if (!bytes || !sizes_of(p, z, why)) return QG_EINVAL;
  *bytes = map_workspace(z, 1, true).total;
  return QG_OK;
}

}  // extern "C"

namespace {

// A context for nmem runs of one size that differ only in Ra (ra[i]; all
// runs use p->Ra when ra is null).  nmem = 1 is the single-run context.
qg_status create_ctx(qg_ctx** out, const qg_params* p, int nmem, const double* ra,
                     void* workspace, size_t workspace_bytes, void* stream, bool single) {
  if (!out) return QG_EINVAL;
  *out = nullptr;
  Sizes z;
  std::string why;
  if (!sizes_of(p, z, why) || nmem < 1) return QG_EINVAL;
  const bool mixed = p->precision == 1;
  if (z.nphi % 6 || !transform_sizes_ok(2 * (z.R - 1), z.nphi, mixed)) return QG_EUNSUPPORTED;
  if (z.gal && p->pivoting) return QG_EUNSUPPORTED;   // Galerkin bands: no row interchanges
  if (p->dct == 2 && !z.mfdct) return QG_EUNSUPPORTED;   // matrix-core DCT: FP64, small N_r
  if (p->buoyancy && p->pivoting) return QG_EUNSUPPORTED;   // the coupled solve is unpivoted
  if (!workspace || ((uintptr_t)workspace & 255)) return QG_EINVAL;
  WsMap w = map_workspace(z, nmem, single);
  if (workspace_bytes < w.total) return QG_ENOMEM;
  std::vector<double> ra_pr(nmem);
  for (int i = 0; i < nmem; ++i) {
    const double r = ra ? ra[i] : p->Ra;
    if (!(r > 0) || !std::isfinite(r)) return QG_EINVAL;
    ra_pr[i] = r / p->Pr;
  }

  qg_ctx* ctx = new qg_ctx();
  ctx->p = *p;
  ctx->p.n_c = z.K;
  ctx->z = z;
  ctx->w = w;
  ctx->nmem = nmem;
  ctx->single = single;
  ctx->ws = static_cast<char*>(workspace);
  ctx->st = static_cast<hipStream_t>(stream);

  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete ctx;
    return QG_EDEVICE;
  }
  const size_t lds_fft = transform_lds_bytes(2 * (z.R - 1), z.nphi, z.K, mixed) + 1024;
  ctx->g.K = z.K;
  const size_t lds_solve = solve_lds_bytes(ctx->g, 16, 8);
  ctx->mixed = mixed;
  // diagnostics stay FP64 whenever the FP64 transform kernels fit
  ctx->diag64 = transform_sizes_ok(2 * (z.R - 1), z.nphi, false) &&
                transform_lds_bytes(2 * (z.R - 1), z.nphi, z.K, false) + 1024 <=
                    (size_t)prop.sharedMemPerBlock;
  if (std::max(lds_fft, lds_solve) > (size_t)prop.sharedMemPerBlock) {
    delete ctx;
    return QG_EUNSUPPORTED;
  }

  ctx->ops = build_operators(p->eta, z.K);
  const double s_i = p->eta / (1 - p->eta), s_o = 1 / (1 - p->eta);
  // host tables
  std::vector<double> xk(z.R), wq(z.R), dsk(z.R);
  std::vector<double> cc = cc_weights(z.R);
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < z.R; ++k) xk[k] = std::cos(pi * k / (z.R - 1));
  for (int k = 0; k < z.R; ++k) {
    double s = 0.5 * (s_o - s_i) * xk[k] + 0.5 * (s_o + s_i);
    wq[k] = cc[k] * 0.5 * (s_o - s_i) * s;
  }
  for (int k = 0; k < z.R; ++k) {
    auto sk = [&](int i) { return 0.5 * (s_o - s_i) * xk[i] + 0.5 * (s_o + s_i); };
    double a = (k > 0) ? std::fabs(sk(k - 1) - sk(k)) : 1e300;
    double b = (k + 1 < z.R) ? std::fabs(sk(k) - sk(k + 1)) : 1e300;
    dsk[k] = std::min(a, b);
  }
  std::vector<double2> twd = plan_twiddles(2 * (z.R - 1)), twp = plan_twiddles(z.nphi),
                       twh = plan_twiddles(z.nphi / 2), wphi = twiddles(z.nphi);
  wphi.resize(z.nphi / 2 + 1);
  auto to32 = [](const std::vector<double2>& v) {
    std::vector<float2> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = make_float2((float)v[i].x, (float)v[i].y);
    return o;
  };
  const std::vector<float2> twd32 = to32(twd), twp32 = to32(twp), twh32 = to32(twh),
                            wphi32 = to32(wphi);
  std::vector<double> dct_s, dct_a;
  if (z.mfdct) mfma_dct_tables(z.R, z.K, dct_s, dct_a);
  std::vector<double> bandbuf((size_t)9 * z.K * BANDW);
  const std::vector<double>* bl[9] = {&ctx->ops.A0, &ctx->ops.A2, &ctx->ops.B0,
                                      &ctx->ops.B2, &ctx->ops.B4, &ctx->ops.C,
                                      &ctx->ops.D,  &ctx->ops.F0, &ctx->ops.F2};
  for (int i = 0; i < 9; ++i)   // device layout: offset-major [17][K]
    for (int k = 0; k < z.K; ++k)
      for (int o = 0; o < BANDW; ++o)
        bandbuf[(size_t)i * z.K * BANDW + (size_t)o * z.K + k] = (*bl[i])[(size_t)k * BANDW + o];
  auto up = [&](size_t off, const void* src, size_t bytes) {
    return hipMemcpyAsync(ctx->ws + off, src, bytes, hipMemcpyHostToDevice, ctx->st);
  };
  if (up(w.xk, xk.data(), xk.size() * 8) != hipSuccess ||
      up(w.wq, wq.data(), wq.size() * 8) != hipSuccess ||
      up(w.dsk, dsk.data(), dsk.size() * 8) != hipSuccess ||
      up(w.twd, twd.data(), twd.size() * 16) != hipSuccess ||
      up(w.twp, twp.data(), twp.size() * 16) != hipSuccess ||
      up(w.twh, twh.data(), twh.size() * 16) != hipSuccess ||
      up(w.wphi, wphi.data(), wphi.size() * 16) != hipSuccess ||
      up(w.twd32, twd32.data(), twd32.size() * 8) != hipSuccess ||
      up(w.twp32, twp32.data(), twp32.size() * 8) != hipSuccess ||
      up(w.twh32, twh32.data(), twh32.size() * 8) != hipSuccess ||
      up(w.wphi32, wphi32.data(), wphi32.size() * 8) != hipSuccess ||
      up(w.bands, bandbuf.data(), bandbuf.size() * 8) != hipSuccess ||
      up(w.ra, ra_pr.data(), ra_pr.size() * 8) != hipSuccess ||
      (z.mfdct && (up(w.dct_s, dct_s.data(), dct_s.size() * 8) != hipSuccess ||
                   up(w.dct_a, dct_a.data(), dct_a.size() * 8) != hipSuccess)) ||
      hipMemsetAsync(ctx->ws + w.state, 0, (single ? 4 : 2) * ctx->mk() * sizeof(double2),
                     ctx->st) != hipSuccess ||
      hipMemsetAsync(ctx->ws + w.flag, 0, sizeof(int), ctx->st) != hipSuccess ||
      hipStreamSynchronize(ctx->st) != hipSuccess) {
    delete ctx;
    return QG_EDEVICE;
  }
  Geom& g = ctx->g;
  g.M = z.M; g.K = z.K; g.R = z.R; g.nphi = z.nphi;
  g.s_o = s_o; g.s_i = s_i;
  g.mid = 0.5 * (s_o + s_i); g.half = 0.5 * (s_o - s_i);
  const double r = std::sqrt(1 - p->eta * p->eta);
  const double alpha = p->eta / (1 - p->eta) * (std::asinh(r / p->eta) / r - 1.0);
  g.dtc_coef = alpha / std::log(p->eta);
  g.Ra_Pr = p->Ra / p->Pr;
  g.inv_Pr = 1.0 / p->Pr;
  g.two_over_E = 2.0 / p->E;
  g.nmem = nmem;
  g.pump = z.pump ? ctx->ptr2(w.pump) : nullptr;
  g.pump_ups = std::sqrt(s_o / p->E);
  g.pump_so2e = z.pump ? (s_o + p->eps) * (s_o + p->eps) : 0.0;
  g.half_E = 0.5 * p->E;
  g.nf = single ? ctx->nf_flag() : nullptr;
  g.buoy_implicit = p->buoyancy == 1;
  g.dct_s = z.mfdct ? ctx->ptrd(w.dct_s) : nullptr;
  g.dct_a = z.mfdct ? ctx->ptrd(w.dct_a) : nullptr;
  g.ra_pr = ctx->ptrd(w.ra);
  g.xk = ctx->ptrd(w.xk);
  g.wq = ctx->ptrd(w.wq);
  g.dsk = ctx->ptrd(w.dsk);
  g.tw_dct = ctx->ptr2(w.twd);
  g.tw_phi = ctx->ptr2(w.twp);
  g.tw_half = ctx->ptr2(w.twh);
  g.w_phi = ctx->ptr2(w.wphi);
  g.tw_dct32 = reinterpret_cast<const float2*>(ctx->ws + w.twd32);
  g.tw_phi32 = reinterpret_cast<const float2*>(ctx->ws + w.twp32);
  g.tw_half32 = reinterpret_cast<const float2*>(ctx->ws + w.twh32);
  g.w_phi32 = reinterpret_cast<const float2*>(ctx->ws + w.wphi32);
  const double* bd = ctx->ptrd(w.bands);
  const size_t bs = (size_t)z.K * BANDW;
  ctx->b = Bands{bd, bd + bs, bd + 2 * bs, bd + 3 * bs, bd + 4 * bs,
                 bd + 5 * bs, bd + 6 * bs, bd + 7 * bs, bd + 8 * bs};
  ctx->Fp = FactorSet<double2>{reinterpret_cast<const int*>(ctx->ws + w.p_piv), ctx->ptr2(w.p_L),
                               ctx->ptr2(w.p_U), ctx->ptr2(w.p_W), ctx->ptr2(w.p_C),
                               ctx->ptr2(w.p_Mi), ctx->ptr2(w.p_L), ctx->ptr2(w.p_U),
                               ctx->ptr2(w.p_ui), z.gal ? ctx->ptrd(w.p_gam) : nullptr};
  ctx->Fr = FactorSet<double>{reinterpret_cast<const int*>(ctx->ws + w.r_piv), ctx->ptrd(w.r_L),
                              ctx->ptrd(w.r_U), ctx->ptrd(w.r_W), ctx->ptrd(w.r_C),
                              ctx->ptrd(w.r_Mi), ctx->ptrd(w.r_L), ctx->ptrd(w.r_U),
                              ctx->ptrd(w.r_ui)};
  *out = ctx;
  return QG_OK;
}

// State of run `mem` in (resets the time, step counter and multistep
// history of the whole context) and out.
// Validates a caller's state (finite, boundary conditions) and uploads it
// to dst_psi (row 0 := zonal flow) and dst_th; *amax = its largest entry.
qg_status load_state(qg_ctx* ctx, const double* psi, const double* theta, const double* uphi,
                     int on_device, double2* dst_psi, double2* dst_th, double* amax) {
  if (!psi || !theta || !uphi) return fail(ctx, QG_EINVAL, "null state pointer");
  const Sizes& z = ctx->z;
  const size_t MK = (size_t)z.M * z.K;
  std::vector<double2> hp(MK), ht(MK);
  std::vector<double> hu(z.K);
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
  HIPCHK(hipMemcpyAsync(hp.data(), psi, MK * 16, kind, ctx->st));
  HIPCHK(hipMemcpyAsync(ht.data(), theta, MK * 16, kind, ctx->st));
  HIPCHK(hipMemcpyAsync(hu.data(), uphi, z.K * 8, kind, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  for (size_t i = 0; i < MK; ++i)
    if (!std::isfinite(hp[i].x) || !std::isfinite(hp[i].y) || !std::isfinite(ht[i].x) ||
        !std::isfinite(ht[i].y))
      return fail(ctx, QG_ENONFINITE, "non-finite value in the state");
  for (int n = 0; n < z.K; ++n)
    if (!std::isfinite(hu[n])) return fail(ctx, QG_ENONFINITE, "non-finite zonal flow");
  // boundary conditions (tau rows) per row
  std::vector<double> rows(4 * z.K);
  for (int r = 0; r < 4; ++r) tau_row(r, z.K, rows.data() + r * z.K);
  auto check = [&](const double2* a, int p, bool real_only) {
    for (int r = 0; r < p; ++r) {
      double sr = 0, si = 0, mr = 0, mi = 0;
      for (int n = 0; n < z.K; ++n) {
        double c = rows[r * z.K + n];
        sr += c * a[n].x; si += c * a[n].y;
        mr += std::fabs(c * a[n].x); mi += std::fabs(c * a[n].y);
      }
      if (std::fabs(sr) > 1e-10 * mr + 1e-300 || std::fabs(si) > 1e-10 * mi + 1e-300) return false;
    }
    if (real_only)
      for (int n = 0; n < z.K; ++n)
        if (a[n].y != 0.0) return false;
    return true;
  };
  for (int m = 1; m < z.M; ++m)
    if (!check(&hp[(size_t)m * z.K], 4, false))
      return fail(ctx, QG_ESTATE, "Psi violates the boundary conditions at m=" + std::to_string(m));
  for (int m = 0; m < z.M; ++m)
    if (!check(&ht[(size_t)m * z.K], 2, m == 0))
      return fail(ctx, QG_ESTATE,
                  "theta violates the boundary conditions (or is complex) at m=" + std::to_string(m));
  std::vector<double2> hu2(z.K);
  for (int n = 0; n < z.K; ++n) hu2[n] = make_double2(hu[n], 0.0);
  if (!check(hu2.data(), 2, true))
    return fail(ctx, QG_ESTATE, "zonal flow violates the boundary conditions");
  for (int n = 0; n < z.K; ++n) hp[n] = hu2[n];  // row 0 of the psi array holds the zonal flow
  double mx = 0.0;
  for (size_t i = 0; i < MK; ++i)
    mx = std::max(mx, std::max(std::hypot(hp[i].x, hp[i].y), std::hypot(ht[i].x, ht[i].y)));
  if (amax) *amax = mx;
  HIPCHK(hipMemcpyAsync(dst_psi, hp.data(), MK * 16, hipMemcpyHostToDevice, ctx->st));
  HIPCHK(hipMemcpyAsync(dst_th, ht.data(), MK * 16, hipMemcpyHostToDevice, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  return QG_OK;
}

qg_status set_state_run(qg_ctx* ctx, int mem, const double* psi, const double* theta,
                        const double* uphi, int on_device) {
  if (!ctx) return QG_EINVAL;
  if (mem < 0 || mem >= ctx->nmem) return fail(ctx, QG_EINVAL, "no such run");
  const size_t MK = (size_t)ctx->z.M * ctx->z.K;
  qg_status s = load_state(ctx, psi, theta, uphi, on_device, ctx->psi() + mem * MK,
                           ctx->th() + mem * MK, nullptr);
  if (s != QG_OK) return s;
  ctx->t_set = 0;
  ctx->t = 0.0;
  ctx->step = 0;
  ctx->have_prev = 0;
  ctx->cur = 0;
  ctx->ms_n = 0;
  ctx->last_scheme = -1;
  ctx->err.clear();
  return QG_OK;
}

// Copies a state out of the workspace (row 0 of src_psi holds the zonal
// flow; the psi output gets zeros there).
qg_status read_state(qg_ctx* ctx, const double2* src_psi, const double2* src_th, double* psi,
                     double* theta, double* uphi, int on_device) {
  if (!psi || !theta || !uphi) return fail(ctx, QG_EINVAL, "null state pointer");
  const Sizes& z = ctx->z;
  const size_t MK = (size_t)z.M * z.K;
  std::vector<double2> hp(MK);
  HIPCHK(hipMemcpyAsync(hp.data(), src_psi, MK * 16, hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  std::vector<double> hu(z.K);
  for (int n = 0; n < z.K; ++n) {
    hu[n] = hp[n].x;
    hp[n] = make_double2(0.0, 0.0);
  }
  const hipMemcpyKind k1 = on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost;
  const hipMemcpyKind k2 = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  HIPCHK(hipMemcpyAsync(psi, hp.data(), MK * 16, k1, ctx->st));
  HIPCHK(hipMemcpyAsync(theta, src_th, MK * 16, k2, ctx->st));
  HIPCHK(hipMemcpyAsync(uphi, hu.data(), z.K * 8, k1, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  return QG_OK;
}

qg_status get_state_run(qg_ctx* ctx, int mem, double* psi, double* theta, double* uphi,
                        int on_device) {
  if (!ctx) return QG_EINVAL;
  if (mem < 0 || mem >= ctx->nmem) return fail(ctx, QG_EINVAL, "no such run");
  const size_t MK = (size_t)ctx->z.M * ctx->z.K;
  return read_state(ctx, ctx->psi() + mem * MK, ctx->th() + mem * MK, psi, theta, uphi,
                    on_device);
}

qg_status check_step_args(qg_ctx* ctx, double dt, int scheme, int nsteps) {
  if (!(dt > 0) || !std::isfinite(dt)) return fail(ctx, QG_EINVAL, "dt must be positive");
  if (scheme < QG_CNAB2 || scheme > QG_SBDF4) return fail(ctx, QG_EINVAL, "unknown scheme");
  if (nsteps < 0) return fail(ctx, QG_EINVAL, "nsteps must be >= 0");
  return QG_OK;
}

// Host-side position of a single run at a step boundary: what a step that
// turns out non-finite must restore (its device state and history are
// left untouched by the guarded kernels, see Geom::nf).
struct Mark {
  int sidx, cur, have_prev, ms_n, t_cur, t_have_prev;
  double t;
  long long step;
};
Mark mark_of(const qg_ctx* c) {
  return Mark{c->sidx, c->cur, c->have_prev, c->ms_n, c->t_cur, c->t_have_prev, c->t, c->step};
}

// After a run of steps: reads the non-finite flag (synchronises).  If step
// i of the run (tag i + 1) produced a non-finite value, the run is rolled
// back to the boundary before it: marks[i] holds that boundary.
qg_status check_finite(qg_ctx* ctx, const std::vector<Mark>& marks) {
  int tag = 0;
  HIPCHK(hipMemcpyAsync(&tag, ctx->nf_flag(), sizeof(int), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  if (tag == 0) return QG_OK;
  const int i = tag - 1;
  if (i < 0 || i >= (int)marks.size())
    return fail(ctx, QG_EDEVICE, "internal: non-finite flag out of range");
  const Mark& m = marks[i];
  ctx->sidx = m.sidx;
  ctx->cur = m.cur;
  ctx->have_prev = m.have_prev;
  ctx->ms_n = m.ms_n;
  ctx->t_cur = m.t_cur;
  ctx->t_have_prev = m.t_have_prev;
  ctx->t = m.t;
  ctx->step = m.step;
  const int zero = 0;
  HIPCHK(hipMemcpyAsync(ctx->nf_flag(), &zero, sizeof(int), hipMemcpyHostToDevice, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  return fail(ctx, QG_ENONFINITE,
              "non-finite state produced by step " + std::to_string(m.step + 1) +
                  "; the state is the last finite one (step " + std::to_string(m.step) + ")");
}

qg_status step_ctx(qg_ctx* ctx, double dt, int scheme, int nsteps) {
  if (!ctx) return QG_EINVAL;
  qg_status s0 = check_step_args(ctx, dt, scheme, nsteps);
  if (s0 != QG_OK) return s0;
  if (nsteps == 0) return QG_OK;
  SideStreamRelease release{ctx};
  begin_history(ctx, dt, scheme);
  if (!sbdf_of(scheme)) {   // SBDF steps pick their factorisation per step
    s0 = prepare(ctx, scheme_adt(scheme, dt));
    if (s0 != QG_OK) return s0;
  }
  std::vector<Mark> marks;
  if (ctx->single) marks.reserve(nsteps);
  for (int i = 0; i < nsteps; ++i) {
    if (ctx->single) marks.push_back(mark_of(ctx));
    ctx->tag = i + 1;
    qg_status s = step_scheme(ctx, dt, scheme);
    if (s != QG_OK) return s;
    ctx->t += dt;
    ctx->step += 1;
  }
  return ctx->single ? check_finite(ctx, marks) : QG_OK;
}

// One autotuner candidate: `per` steps with band-product shape mch, the
// band-product launches timed with events on the context's stream
// (synchronises); *ms = mean duration of one right-hand-side launch.
qg_status tune_candidate(qg_ctx* ctx, double dt, int scheme, int per, int mch, double* ms) {
  ctx->band_mch = mch;
  ctx->prof = true;
  ctx->ev_used = 0;
  ctx->ev_marks.clear();
  qg_status s = step_ctx(ctx, dt, scheme, per);
  ctx->prof = false;
  if (s != QG_OK) return s;
  HIPCHK(hipStreamSynchronize(ctx->st));
  double tot = 0.0;
  int n = 0;
  for (auto& mk : ctx->ev_marks) {
    if (mk.first != K_RHS) continue;
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, mk.second.first, mk.second.second));
    tot += t;
    ++n;
  }
  ctx->ev_marks.clear();
  *ms = n ? tot / n : 0.0;
  return QG_OK;
}

// Runs warm + TUNE_N * per steps of ctx (untimed warm-up, then every
// candidate) and keeps the shape with the shortest band-product launches.
qg_status tune_ctx(qg_ctx* ctx, double dt, int scheme, int warm, int per) {
  qg_status s = step_ctx(ctx, dt, scheme, warm);
  if (s != QG_OK) return s;
  double best = 0.0;
  int pick = ctx->band_mch;
  for (int c = 0; c < TUNE_N; ++c) {
    double ms = 0.0;
    s = tune_candidate(ctx, dt, scheme, per, TUNE_MCH[c], &ms);
    if (s != QG_OK) return s;
    if (c == 0 || ms < best) {
      best = ms;
      pick = TUNE_MCH[c];
    }
  }
  ctx->band_mch = pick;
  return QG_OK;
}

// Diagnostics of run `mem` (the kernels evaluate every run of the context).
qg_status diagnostics_run(qg_ctx* ctx, int mem, qg_diag* out) {
  if (!ctx || !out) return QG_EINVAL;
  if (mem < 0 || mem >= ctx->nmem) return fail(ctx, QG_EINVAL, "no such run");
  const Sizes& z = ctx->z;
  const bool mixed = !ctx->diag64;   // FP64 diagnostics whenever those kernels fit
  if (!launch_synth(ctx->g, ctx->psi(), ctx->th(), ctx->ptr2(ctx->w.X), ctx->ptrd(ctx->w.diag),
                    mixed, ctx->st) ||
      !launch_ring(ctx->g, ctx->ptr2(ctx->w.X), ctx->ptr2(ctx->w.NL), ctx->ptrd(ctx->w.zonal),
                   ctx->ptrd(ctx->w.rate), mixed, ctx->st))
    return fail(ctx, QG_EUNSUPPORTED, "no transform kernel for these sizes");
  HIPCHK(hipGetLastError());
  std::vector<double> d((size_t)z.M * 8), rate(z.R);
  HIPCHK(hipMemcpyAsync(d.data(), ctx->ptrd(ctx->w.diag) + (size_t)mem * z.M * 8, d.size() * 8,
                        hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(hipMemcpyAsync(rate.data(), ctx->ptrd(ctx->w.rate) + (size_t)mem * z.R,
                        rate.size() * 8, hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  double ek = 0, ez = 0, et = 0, en = 0, bad = 0, rmax = 0;
  for (int m = 0; m < z.M; ++m) {
    ek += d[m * 8 + 0];
    ez += d[m * 8 + 1];
    et += d[m * 8 + 2];
    en += d[m * 8 + 3];
    bad = std::max(bad, std::max(d[m * 8 + 4], d[m * 8 + 5]));
  }
  for (int k = 0; k < z.R; ++k) rmax = std::max(rmax, rate[k]);
  const double s_o = ctx->g.s_o, s_i = ctx->g.s_i, pi = 3.14159265358979323846;
  out->t = ctx->t;
  out->E_kin = ek;
  out->E_zon = ez;
  out->E_therm = et;
  out->enstrophy = en;
  out->Re = std::sqrt(2.0 * ek / (pi * (s_o * s_o - s_i * s_i)));
  out->Ro = out->Re * ctx->p.E;
  out->dt_cfl = rmax > 0 ? 1.0 / rmax : INFINITY;
  out->step = ctx->step;
  out->nonfinite = bad > 0 ? 1 : 0;
  out->pivoted = (ctx->factored_adt >= 0.0 && ctx->pivoted) ? 1 : 0;
  out->growth = ctx->factored_adt >= 0.0 ? ctx->growth : 0.0;
  return QG_OK;
}

}  // namespace

extern "C" {

qg_status qg_create(qg_ctx** out, const qg_params* p, void* workspace, size_t workspace_bytes,
                    void* stream) {
  return create_ctx(out, p, 1, nullptr, workspace, workspace_bytes, stream, true);
}

qg_status qg_set_state(qg_ctx* ctx, const double* psi, const double* theta, const double* uphi,
                       int on_device) {
  return set_state_run(ctx, 0, psi, theta, uphi, on_device);
}

qg_status qg_get_state(qg_ctx* ctx, double* psi, double* theta, double* uphi, int on_device) {
  return get_state_run(ctx, 0, psi, theta, uphi, on_device);
}

qg_status qg_step(qg_ctx* ctx, double dt, int scheme, int nsteps) {
  return step_ctx(ctx, dt, scheme, nsteps);
}

qg_status qg_tangent_set(qg_ctx* ctx, const double* dpsi, const double* dtheta,
                         const double* duphi, int on_device) {
  if (!ctx) return QG_EINVAL;
  if (ctx->g.buoy_implicit)
    return fail(ctx, QG_EUNSUPPORTED, "tangent and adjoint runs need explicit buoyancy");
  if (ctx->nmem != 1) return fail(ctx, QG_EINVAL, "tangent runs need a single-run context");
  double dmax = 0.0;
  qg_status s = load_state(ctx, dpsi, dtheta, duphi, on_device, ctx->tng(0), ctx->tng(0) + ctx->mk(),
                           &dmax);
  if (s != QG_OK) return s;
  const size_t MK = (size_t)ctx->z.M * ctx->z.K;
  std::vector<double2> hp(MK), ht(MK);
  HIPCHK(hipMemcpyAsync(hp.data(), ctx->psi(), MK * 16, hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(hipMemcpyAsync(ht.data(), ctx->th(), MK * 16, hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  double ymax = 0.0;
  for (size_t i = 0; i < MK; ++i)
    ymax = std::max(ymax, std::max(std::hypot(hp[i].x, hp[i].y), std::hypot(ht[i].x, ht[i].y)));
  ctx->t_scale = (ymax > 0.0 && dmax > 0.0) ? ymax / dmax : 1.0;
  ctx->t_set = 1;
  ctx->t_have_prev = 0;
  ctx->t_cur = 0;
  return QG_OK;
}

qg_status qg_adjoint_solve(qg_ctx* ctx, double dt, double* psi, double* theta, double* uphi,
                           int on_device) {
  if (!ctx) return QG_EINVAL;
  if (ctx->nmem != 1) return fail(ctx, QG_EINVAL, "adjoint solves need a single-run context");
  if (!psi || !theta || !uphi) return fail(ctx, QG_EINVAL, "null pointer");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(ctx, QG_EINVAL, "dt must be positive");
  qg_status s = prepare(ctx, 0.5 * dt);
  if (s != QG_OK) return s;
  if (ctx->pivoted)
    return fail(ctx, QG_EUNSUPPORTED, "adjoint solves use the unpivoted factors");
  if (ctx->galerkin)
    return fail(ctx, QG_EUNSUPPORTED, "adjoint solves need the tau formulation");
  if (ctx->g.buoy_implicit)
    return fail(ctx, QG_EUNSUPPORTED, "tangent and adjoint runs need explicit buoyancy");
  const Sizes& z = ctx->z;
  const size_t MK = (size_t)z.M * z.K;
  std::vector<double2> hp(MK);
  std::vector<double> hu(z.K);
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
  HIPCHK(hipMemcpyAsync(hp.data(), psi, MK * 16, kind, ctx->st));
  HIPCHK(hipMemcpyAsync(hu.data(), uphi, z.K * 8, kind, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  for (int n = 0; n < z.K; ++n) hp[n] = make_double2(hu[n], 0.0);   // row 0: the zonal flow
  double2* bp = ctx->tng(3);
  double2* bt = ctx->tng(3) + ctx->mk();
  HIPCHK(hipMemcpyAsync(bp, hp.data(), MK * 16, hipMemcpyHostToDevice, ctx->st));
  HIPCHK(hipMemcpyAsync(bt, theta, MK * 16,
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, ctx->st));
  launch_solve_adjoint(ctx->g, ctx->Fp, ctx->Fr, z.q4, z.q2, bp, bt, ctx->st);
  HIPCHK(hipGetLastError());
  return read_state(ctx, bp, bt, psi, theta, uphi, on_device);
}

qg_status qg_adjoint_mass_lin(qg_ctx* ctx, double c, double* psi, double* theta,
                              double* uphi, int on_device) {
  if (!ctx) return QG_EINVAL;
  if (ctx->g.buoy_implicit)
    return fail(ctx, QG_EUNSUPPORTED, "tangent and adjoint runs need explicit buoyancy");
  if (ctx->nmem != 1) return fail(ctx, QG_EINVAL, "adjoint products need a single-run context");
  if (!psi || !theta || !uphi) return fail(ctx, QG_EINVAL, "null pointer");
  if (!std::isfinite(c)) return fail(ctx, QG_EINVAL, "c must be finite");
  const Sizes& z = ctx->z;
  const size_t MK = (size_t)z.M * z.K;
  std::vector<double2> hp(MK);
  std::vector<double> hu(z.K);
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
  HIPCHK(hipMemcpyAsync(hp.data(), psi, MK * 16, kind, ctx->st));
  HIPCHK(hipMemcpyAsync(hu.data(), uphi, z.K * 8, kind, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  for (int n = 0; n < z.K; ++n) hp[n] = make_double2(hu[n], 0.0);   // row 0: the zonal flow
  double2 *ip = ctx->tng(3), *it = ctx->tng(3) + ctx->mk();
  double2 *op = ctx->tng(4), *ot = ctx->tng(4) + ctx->mk();
  HIPCHK(hipMemcpyAsync(ip, hp.data(), MK * 16, hipMemcpyHostToDevice, ctx->st));
  HIPCHK(hipMemcpyAsync(it, theta, MK * 16,
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, ctx->st));
  launch_band_adjoint(ctx->g, ctx->b, c, ip, it, op, ot, ctx->st);
  HIPCHK(hipGetLastError());
  return read_state(ctx, op, ot, psi, theta, uphi, on_device);
}

qg_status qg_tangent_get(qg_ctx* ctx, double* dpsi, double* dtheta, double* duphi,
                         int on_device) {
  if (!ctx) return QG_EINVAL;
  if (!ctx->t_set) return fail(ctx, QG_ESTATE, "no tangent state (qg_tangent_set)");
  return read_state(ctx, ctx->tng(0), ctx->tng(0) + ctx->mk(), dpsi, dtheta, duphi, on_device);
}

qg_status qg_step_tangent(qg_ctx* ctx, double dt, int nsteps) {
  if (!ctx) return QG_EINVAL;
  if (ctx->g.buoy_implicit)
    return fail(ctx, QG_EUNSUPPORTED, "tangent and adjoint runs need explicit buoyancy");
  qg_status s = check_step_args(ctx, dt, QG_CNAB2, nsteps);
  if (s != QG_OK) return s;
  if (!ctx->t_set) return fail(ctx, QG_ESTATE, "no tangent state (qg_tangent_set)");
  if (nsteps == 0) return QG_OK;
  SideStreamRelease release{ctx};
  const bool fresh = ctx->last_scheme != QG_CNAB2 || ctx->last_dt != dt;
  begin_history(ctx, dt, QG_CNAB2);
  if (fresh) ctx->t_have_prev = 0;
  s = prepare(ctx, 0.5 * dt);
  if (s != QG_OK) return s;
  std::vector<Mark> marks;
  marks.reserve(nsteps);
  for (int i = 0; i < nsteps; ++i) {
    marks.push_back(mark_of(ctx));
    ctx->tag = i + 1;
    s = step_tangent(ctx, dt);
    if (s == QG_OK) s = step_cnab2(ctx, dt);
    if (s != QG_OK) return s;
    ctx->flip();
    ctx->t += dt;
    ctx->step += 1;
  }
  s = check_finite(ctx, marks);
  if (s == QG_ENONFINITE) ctx->t_set = 0;   // the tangent was updated in place
  return s;
}

qg_status qg_diagnostics(qg_ctx* ctx, qg_diag* out) { return diagnostics_run(ctx, 0, out); }

}  // extern "C"

// ---------------------------------------------------------- checkpoints
namespace {

// Fixed header of a checkpoint, followed by `narr` arrays of 2 M K
// complex entries: the state (Psi with the zonal flow in row 0, theta),
// then the stored explicit terms E^{n-1}, .., E^{n-nE}, then the stored
// states y^{n-1}, .., y^{n-nY} (multistep levels).
struct CkptHeader {
  char magic[8];
  int version, n_phi, n_r, n_c, precision, ekman;
  double E, Ra, Pr, eta, eps;
  int scheme;          // scheme of the history (-1: none)
  int have_prev;       // CNAB2: E^{n-1} stored
  int ms_n;            // SBDF: levels since the history began
  int nE, nY;          // arrays of explicit terms and of past states
  int pad;
  double dt, t;
  long long step;
  char reserved[256 - 8 - 6 * 4 - 5 * 8 - 6 * 4 - 2 * 8 - 8];
};
static_assert(sizeof(CkptHeader) == 256, "checkpoint header size");
const char CKPT_MAGIC[8] = {'Q', 'G', 'C', 'K', 'P', 'T', '0', '1'};

// Arrays the current history needs (CNAB2: E^{n-1}; SBDFk: up to three
// levels of E and y; the SDIRK schemes keep none).
void ckpt_levels(const qg_ctx* c, int& nE, int& nY) {
  nE = nY = 0;
  if (c->last_scheme == QG_CNAB2 && c->have_prev) nE = 1;
  if (sbdf_of(c->last_scheme)) nE = nY = std::min(c->ms_n, 3);
}

size_t ckpt_bytes(const qg_ctx* c) {
  int nE, nY;
  ckpt_levels(c, nE, nY);
  return sizeof(CkptHeader) + (size_t)(1 + nE + nY) * 2 * c->mk() * sizeof(double2);
}

// Workspace location of array a of a checkpoint (see CkptHeader).
double2* ckpt_array(qg_ctx* c, int a, int nE) {
  if (a == 0) return c->psi();
  const int n = c->ms_n;
  if (a <= nE) {
    const int j = a;   // E^{n-j}
    if (c->last_scheme == QG_CNAB2) return c->slot(c->w.eslot, 1 - c->cur, 0);
    return c->slot(c->w.mE, ((n - j) % 4 + 4) % 4, 0);
  }
  const int j = a - nE;   // y^{n-j}
  return c->slot(c->w.mY, ((n - j) % 3 + 3) % 3, 0);
}

}  // namespace

extern "C" {

qg_status qg_checkpoint_size(const qg_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return QG_EINVAL;
  if (!ctx->single) return QG_EINVAL;
  *bytes = ckpt_bytes(ctx);
  return QG_OK;
}

qg_status qg_checkpoint_save(qg_ctx* ctx, void* buf, size_t bytes, int on_device) {
  if (!ctx) return QG_EINVAL;
  if (!ctx->single) return fail(ctx, QG_EINVAL, "checkpoints need a single-run context");
  if (!buf) return fail(ctx, QG_EINVAL, "null checkpoint buffer");
  if (bytes < ckpt_bytes(ctx)) return fail(ctx, QG_EINVAL, "checkpoint buffer too small");
  CkptHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, CKPT_MAGIC, 8);
  h.version = 1;
  h.n_phi = ctx->p.n_phi; h.n_r = ctx->p.n_r; h.n_c = ctx->z.K;
  h.precision = ctx->p.precision; h.ekman = ctx->p.ekman;
  h.E = ctx->p.E; h.Ra = ctx->p.Ra; h.Pr = ctx->p.Pr; h.eta = ctx->p.eta;
  h.eps = ctx->p.ekman ? ctx->p.eps : 0.0;
  h.scheme = ctx->last_scheme;
  h.have_prev = ctx->have_prev;
  h.ms_n = ctx->ms_n;
  ckpt_levels(ctx, h.nE, h.nY);
  h.dt = ctx->last_dt; h.t = ctx->t; h.step = ctx->step;
  const size_t arr = 2 * ctx->mk() * sizeof(double2);
  char* dst = static_cast<char*>(buf);
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (on_device) HIPCHK(hipMemcpyAsync(dst, &h, sizeof(h), hipMemcpyHostToDevice, ctx->st));
  else std::memcpy(dst, &h, sizeof(h));
  for (int a = 0; a < 1 + h.nE + h.nY; ++a)
    HIPCHK(hipMemcpyAsync(dst + sizeof(h) + a * arr, ckpt_array(ctx, a, h.nE), arr, k, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  return QG_OK;
}

qg_status qg_checkpoint_load(qg_ctx* ctx, const void* buf, size_t bytes, int on_device) {
  if (!ctx) return QG_EINVAL;
  if (!ctx->single) return fail(ctx, QG_EINVAL, "checkpoints need a single-run context");
  if (!buf || bytes < sizeof(CkptHeader)) return fail(ctx, QG_EINVAL, "checkpoint too short");
  CkptHeader h;
  const char* src = static_cast<const char*>(buf);
  if (on_device) {
    HIPCHK(hipMemcpyAsync(&h, src, sizeof(h), hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
  } else {
    std::memcpy(&h, src, sizeof(h));
  }
  if (std::memcmp(h.magic, CKPT_MAGIC, 8) != 0 || h.version != 1)
    return fail(ctx, QG_EINVAL, "not a checkpoint of this library");
  const qg_params& p = ctx->p;
  if (h.n_phi != p.n_phi || h.n_r != p.n_r || h.n_c != ctx->z.K || h.precision != p.precision ||
      h.ekman != p.ekman || h.E != p.E || h.Ra != p.Ra || h.Pr != p.Pr || h.eta != p.eta ||
      (p.ekman && h.eps != p.eps))
    return fail(ctx, QG_EINVAL, "checkpoint of a different problem (sizes or parameters)");
  if (h.nE < 0 || h.nE > 3 || h.nY < 0 || h.nY > 3 || h.ms_n < 0)
    return fail(ctx, QG_EINVAL, "corrupt checkpoint header");
  const size_t arr = 2 * ctx->mk() * sizeof(double2);
  if (bytes < sizeof(h) + (size_t)(1 + h.nE + h.nY) * arr)
    return fail(ctx, QG_EINVAL, "checkpoint truncated");
  // host position first: the array locations depend on it
  ctx->last_scheme = h.scheme;
  ctx->last_dt = h.dt;
  ctx->t = h.t;
  ctx->step = h.step;
  ctx->have_prev = h.have_prev;
  ctx->cur = 0;
  ctx->ms_n = h.ms_n;
  ctx->t_set = 0;
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  for (int a = 0; a < 1 + h.nE + h.nY; ++a)
    HIPCHK(hipMemcpyAsync(ckpt_array(ctx, a, h.nE), src + sizeof(h) + a * arr, arr, k, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  ctx->err.clear();
  return QG_OK;
}

qg_status qg_step_autotune(qg_ctx* ctx, double dt, int scheme, int nsteps,
                           int* systems_per_thread) {
  if (!ctx || !systems_per_thread) return QG_EINVAL;
  qg_status s = check_step_args(ctx, dt, scheme, nsteps);
  if (s != QG_OK) return s;
  const Sbdf* sb = sbdf_of(scheme);
  const int warm = sb ? sb->k : 1;   // start-up and factorisation, untimed
  const int per = (nsteps - warm) / TUNE_N;
  if (per < 1) return fail(ctx, QG_EINVAL, "autotune needs 4 timed steps after the warm-up");
  s = tune_ctx(ctx, dt, scheme, warm, per);
  if (s != QG_OK) return s;
  *systems_per_thread = ctx->band_mch;
  return step_ctx(ctx, dt, scheme, nsteps - warm - TUNE_N * per);
}

qg_status qg_step_timed(qg_ctx* ctx, double dt, int scheme, int nsteps, double* kernel_ms,
                        int* launches) {
  if (!ctx || !kernel_ms || !launches) return QG_EINVAL;
  // factorise first so that the refactorisation is outside the timing
  if (dt > 0 && std::isfinite(dt) && scheme >= QG_CNAB2 && scheme <= QG_SBDF4) {
    qg_status s = prepare(ctx, scheme_adt(scheme, dt));
    if (s != QG_OK) return s;
  }
  ctx->prof = true;
  ctx->ev_used = 0;
  ctx->ev_marks.clear();
  qg_status s = qg_step(ctx, dt, scheme, nsteps);
  ctx->prof = false;
  if (s != QG_OK) return s;
  HIPCHK(hipStreamSynchronize(ctx->st));
  for (int c = 0; c < K_COUNT; ++c) { kernel_ms[c] = 0.0; launches[c] = 0; }
  for (auto& mk : ctx->ev_marks) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, mk.second.first, mk.second.second));
    kernel_ms[mk.first] += ms;
    launches[mk.first] += 1;
  }
  ctx->ev_marks.clear();
  return QG_OK;
}

}  // extern "C"

// ---------------------------------------------------------- reverse mode
// Gradient of the time-integrated kinetic energy through CNAB2 steps
// (eq. multistep1 with E^{-1} := E^0, Sect. 4), by the discrete adjoint:
// with y^{n+1} = P S^-1 Z r^n, S = M - (dt/2) L, r^n = (M + (dt/2) L) y^n +
// dt (c_n E(y^n) - (1/2) E(y^{n-1})), c_0 = 1/2 + 1/2 (E^{-1} := E^0),
// else 3/2, the co-states run backwards as
//   rb^{n-1} = Z S^-H P ybar^n,
//   ybar^n   = kappa_n grad E_K(y^n) + (M + (dt/2) L)^H rb^n
//              + E'(y^n)^H (c_n dt rb^n - (1/2) dt rb^{n+1}),
// kappa_n = w_E dt w_n (trapezoid weights w_n, 1/2 at both ends), and
// ybar^N adds the caller's terminal co-state.  The forward trajectory is
// kept at every `interval`-th step (state and E^{n-1}); each block but the
// last is recomputed from its checkpoint before its reverse steps, and the
// synthesised fields X of a block's states are kept for the transposed
// explicit terms.
namespace {

struct GradMap {
  size_t ck, blk, Xs, Gs, E2, NL2, zonal2, rhs2, Xb, thb0, ml, rb, acc, adj, tmp, diag, J;
  size_t pLT, pUT, puiT, rLT, rUT, ruiT;   // factors of D^H (transposed solves)
  size_t total;
};

int grad_slots(int nsteps, int interval) {   // states (and X fields) kept per block
  return std::max(3, std::min(interval, std::max(nsteps, 0)) + 1);
}

GradMap map_gradient(const qg_ctx* c, int nsteps, int interval) {
  Layout L;
  GradMap w;
  const size_t S = 2 * c->mk() * sizeof(double2);   // a (Psi and u, theta) pair
  const size_t XS = (size_t)6 * c->z.R * c->z.M * sizeof(double2);
  const int nblk = nsteps > 0 ? (nsteps + interval - 1) / interval : 0;
  const int slots = grad_slots(nsteps, interval);
  // two sets of block storage: one block is swept backwards while the
  // next one is recomputed on a second stream
  w.ck = L.take((size_t)nblk * 2 * S);    // y^{n0} and E^{n0-1} of each block
  w.blk = L.take((size_t)2 * slots * S);  // the states of a block
  w.Xs = L.take((size_t)2 * slots * XS);  // their synthesised fields
  w.Gs = L.take((size_t)2 * slots * 6 * c->z.R * c->z.nphi * sizeof(double));   // grid fields
  w.E2 = L.take(2 * S);                   // explicit terms of the recomputation
  w.NL2 = L.take((size_t)2 * c->z.R * c->z.M * sizeof(double2));   // its exchange arrays
  w.zonal2 = L.take((size_t)c->z.R * sizeof(double));
  w.rhs2 = L.take(S);
  w.Xb = L.take(XS);
  w.thb0 = L.take(c->mk() * sizeof(double2));
  w.ml = L.take(S);
  w.rb = L.take(2 * S);
  w.acc = L.take(S);
  w.adj = L.take(S);
  w.tmp = L.take(S);
  w.diag = L.take((size_t)(std::max(nsteps, 0) + 1) * c->z.M * 8 * sizeof(double));
  w.J = L.take(sizeof(double));
  const Sizes& z = c->z;
  const size_t Sp = z.M - 1, Sr = z.Sr;
  w.pLT = L.take(Sp * z.q4 * 8 * sizeof(double2));
  w.pUT = L.take(Sp * z.q4 * 8 * sizeof(double2));
  w.puiT = L.take(Sp * z.q4 * sizeof(double2));
  w.rLT = L.take(Sr * z.q2 * 4 * sizeof(double));
  w.rUT = L.take(Sr * z.q2 * 4 * sizeof(double));
  w.ruiT = L.take(Sr * z.q2 * sizeof(double));
  w.total = L.total;
  return w;
}

struct Pair {
  double2* p;   // Psi of m >= 1, the zonal flow in row 0
  double2* t;   // theta
};

Pair pair_at(char* base, size_t off, size_t i, size_t mk) {
  double2* p = reinterpret_cast<double2*>(base + off) + 2 * i * mk;
  return {p, p + mk};
}

qg_status reverse_ok(qg_ctx* ctx) {
  if (ctx->nmem != 1 || !ctx->single)
    return fail(ctx, QG_EINVAL, "reverse mode needs a single-run context");
  if (ctx->mixed) return fail(ctx, QG_EUNSUPPORTED, "reverse mode runs in FP64 only");
  if (ctx->z.pump) return fail(ctx, QG_EUNSUPPORTED, "reverse mode has no Ekman pumping terms");
  if (ctx->g.buoy_implicit)
    return fail(ctx, QG_EUNSUPPORTED, "reverse mode transposes the explicit buoyancy");
  return QG_OK;
}

// One CNAB2 step y -> out with E(y) into En and E^{n-1} in Ep (nullptr:
// E^{-1} := E^n); diag: the synthesis's diagnostics of y; X, G: where the
// fields of y go (nullptr: the workspace; no grid fields).
struct Scratch {   // exchange arrays and right-hand side of a step (null: the workspace's)
  double2* NL = nullptr;
  double* zonal = nullptr;
  double2* rhs = nullptr;
};

// overlap: the band product on the second stream, as in step_cnab2 (the
// same trajectory bit for bit).
qg_status cnab2_into(qg_ctx* ctx, double dt, Pair y, Pair En, const Pair* Ep, Pair out,
                     double* diag, double2* X, double* G, const Scratch& sc = Scratch{},
                     bool overlap = false) {
  double2* rhs = sc.rhs ? sc.rhs : ctx->ptr2(ctx->w.rhs);
  const bool ovl = overlap && overlap_rhs(ctx);
  if (ovl) {
    const qg_status f = fork_band(ctx, y.p, y.t, dt, rhs);
    if (f != QG_OK) return f;
  }
  qg_status s = explicit_terms(ctx, y.p, y.t, En.p, En.t, diag, X, G, sc.NL, sc.zonal);
  if (s != QG_OK) {
    if (ovl) (void)hipStreamWaitEvent(ctx->st, ctx->ev_join, 0);
    return s;
  }
  RhsSpec rs{};
  rs.base_psi = y.p;
  rs.base_th = y.t;
  rs.cL = 0.5 * dt;
  rs.nterm = 2;
  rs.term_psi[0] = En.p;
  rs.term_th[0] = En.t;
  rs.coef[0] = 1.5 * dt;
  rs.term_psi[1] = Ep ? Ep->p : En.p;
  rs.term_th[1] = Ep ? Ep->t : En.t;
  rs.coef[1] = -0.5 * dt;
  rs.out_psi = out.p;
  rs.out_th = out.t;
  if (ovl) {
    s = join_terms(ctx, rs, rhs);
    if (s != QG_OK) return s;
  }
  return implicit_solve(ctx, rs, rhs, ovl);
}

// A second stream and the events of the overlapped reverse sweep, released
// on every return path.
struct SweepStreams {
  hipStream_t st2 = nullptr;
  std::vector<hipEvent_t> ev;
  ~SweepStreams() {
    if (st2) {
      (void)hipStreamSynchronize(st2);
      (void)hipStreamDestroy(st2);
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  hipEvent_t event() {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    ev.push_back(e);
    return e;
  }
};

// out = E'(y)^H (ca Ea + cb Eb) + kappa grad E_K(y) + add
//       + (Mass + cmu Lin)^H mu, with X the synthesised fields of y (pairs
// may be null: zero).
qg_status explicit_T(qg_ctx* ctx, const double2* X, const double* G, const double2* Ea,
                     const double2* Eb, double ca, double cb, double kappa, const double2* add,
                     const double2* mu, double cmu, char* base, const GradMap& w, Pair out) {
  if (!launch_explicit_T(ctx->g, ctx->b, X, G, Ea, Eb, ca, cb, ctx->mk(), kappa,
                         ctx->ptr2(ctx->w.NL), ctx->ptrd(ctx->w.zonal),
                         reinterpret_cast<double2*>(base + w.thb0),
                         reinterpret_cast<double2*>(base + w.Xb), add, mu, cmu,
                         reinterpret_cast<double2*>(base + w.ml), out.p, out.t, ctx->st))
    return fail(ctx, QG_EUNSUPPORTED, "no reverse transform kernel for these sizes");
  HIPCHK(hipGetLastError());
  return QG_OK;
}

qg_status gradient_run(qg_ctx* ctx, double dt, int N, int C, double ew, const double* adj_psi,
                       const double* adj_th, const double* adj_u, double* g_psi, double* g_th,
                       double* g_u, double* J, char* base, const GradMap& w) {
  SideStreamRelease release{ctx};
  const size_t mk = ctx->mk();
  const int M = ctx->z.M, K = ctx->z.K;
  const bool grad = g_psi != nullptr;
  qg_status s = prepare(ctx, 0.5 * dt);
  if (s != QG_OK) return s;
  if (grad && ctx->pivoted)
    return fail(ctx, QG_EUNSUPPORTED, "the adjoint solves use the unpivoted factors");
  if (grad && ctx->galerkin)
    return fail(ctx, QG_EUNSUPPORTED, "the adjoint solves need the tau formulation");
  if (grad && ctx->g.buoy_implicit)
    return fail(ctx, QG_EUNSUPPORTED, "tangent and adjoint runs need explicit buoyancy");
  const size_t XS = (size_t)6 * ctx->z.R * M;   // entries of one X
  const size_t GS = (size_t)6 * ctx->z.R * ctx->z.nphi;
  const int slots = grad_slots(N, C);
  // slot `slot` of storage set `set` (states, fields, grid fields)
  auto Yb = [&](int set, int slot) { return pair_at(base, w.blk, (size_t)(set * slots + slot), mk); };
  auto Xsb = [&](int set, int slot) {
    return reinterpret_cast<double2*>(base + w.Xs) + (size_t)(set * slots + slot) * XS;
  };
  auto Gsb = [&](int set, int slot) {
    return reinterpret_cast<double*>(base + w.Gs) + (size_t)(set * slots + slot) * GS;
  };
  auto Y = [&](int slot) { return Yb(0, slot); };
  auto Xs = [&](int slot) { return Xsb(0, slot); };
  auto Gs = [&](int slot) { return Gsb(0, slot); };
  std::vector<char> has_g[2] = {std::vector<char>(slots, 0), std::vector<char>(slots, 0)};
  auto ck = [&](int b, int a) { return pair_at(base, w.ck, 2 * (size_t)b + a, mk); };
  double* diag = reinterpret_cast<double*>(base + w.diag);
  double* Jd = reinterpret_cast<double*>(base + w.J);
  HIPCHK(hipMemsetAsync(ctx->nf_flag(), 0, sizeof(int), ctx->st));
  const int nblk = N > 0 ? (N + C - 1) / C : 0;
  const int nl = nblk > 0 ? (nblk - 1) * C : 0;   // first step of the last block
  // ---- forward pass: a checkpoint per block; the last block keeps its
  // states and fields; E_K of every state for J
  Pair E2[2] = {pair_at(base, w.E2, 0, mk), pair_at(base, w.E2, 1, mk)};
  // slot of y^n in the forward pass: the last block keeps y^nl .. y^N in
  // slots 0 .. N - nl; before it the states take slots 1 and 2 in turn
  auto slot_of = [&](int n) { return n >= nl ? n - nl : 1 + n % 2; };
  launch_copy(ctx->psi(), Y(slot_of(0)).p, 2 * mk, nullptr, ctx->st);
  for (int n = 0; n < N; ++n) {
    Pair y = Y(slot_of(n)), En = E2[n % 2], Ep = E2[(n + 1) % 2];
    if (n % C == 0) {
      launch_copy(y.p, ck(n / C, 0).p, 2 * mk, nullptr, ctx->st);
      if (n > 0) launch_copy(Ep.p, ck(n / C, 1).p, 2 * mk, nullptr, ctx->st);
    }
    ctx->tag = n + 1;
    s = cnab2_into(ctx, dt, y, En, n > 0 ? &Ep : nullptr, Y(slot_of(n + 1)),
                   diag + (size_t)n * M * 8, n >= nl ? Xs(n - nl) : nullptr,
                   n >= nl ? Gs(n - nl) : nullptr, Scratch{}, true);
    if (s != QG_OK) return s;
    if (n >= nl) has_g[0][n - nl] = 1;
  }
  {
    Pair yN = Y(slot_of(N));
    if (!launch_synth(ctx->g, yN.p, yN.t, Xs(N - nl), diag + (size_t)N * M * 8, false, ctx->st))
      return fail(ctx, QG_EUNSUPPORTED, "no transform kernel for these sizes");
    launch_energy_total(diag, M, N, ew * dt, Jd, ctx->st);
  }
  HIPCHK(hipGetLastError());
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, ctx->nf_flag(), sizeof(int), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(hipMemcpyAsync(J, Jd, sizeof(double), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  if (flag) {
    HIPCHK(hipMemsetAsync(ctx->nf_flag(), 0, sizeof(int), ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    return fail(ctx, QG_ENONFINITE, "non-finite state at step " + std::to_string(flag) +
                                        " of the forward pass; the state is unchanged");
  }
  // the context continues from y^N with its CNAB2 history, as after
  // qg_step(dt, CNAB2, N) from a fresh history
  if (N > 0) {
    launch_copy(Y(slot_of(N)).p, ctx->psi(), 2 * mk, nullptr, ctx->st);
    ctx->last_scheme = QG_CNAB2;
    ctx->last_dt = dt;
    ctx->cur = 0;
    ctx->have_prev = 1;
    launch_copy(E2[(N - 1) % 2].p, ctx->slot(ctx->w.eslot, 1, 0), 2 * mk, nullptr, ctx->st);
    ctx->ms_n = 0;
    ctx->t += N * dt;
    ctx->step += N;
    ctx->t_set = 0;
  }
  if (!grad) {
    HIPCHK(hipStreamSynchronize(ctx->st));
    return QG_OK;
  }
  // ---- reverse pass
  Pair rb[2] = {pair_at(base, w.rb, 0, mk), pair_at(base, w.rb, 1, mk)};
  Pair acc = pair_at(base, w.acc, 0, mk), adj = pair_at(base, w.adj, 0, mk);
  Pair tmp = pair_at(base, w.tmp, 0, mk);
  FactorSet<double2> FpT = ctx->Fp;
  FactorSet<double> FrT = ctx->Fr;
  double2* pLT = reinterpret_cast<double2*>(base + w.pLT);
  double2* pUT = reinterpret_cast<double2*>(base + w.pUT);
  double2* puiT = reinterpret_cast<double2*>(base + w.puiT);
  double* rLT = reinterpret_cast<double*>(base + w.rLT);
  double* rUT = reinterpret_cast<double*>(base + w.rUT);
  double* ruiT = reinterpret_cast<double*>(base + w.ruiT);
  FpT.L = pLT; FpT.U = pUT; FpT.ui = puiT;
  FrT.L = rLT; FrT.U = rUT; FrT.ui = ruiT;
  launch_transpose_factors(ctx->Fp, ctx->Fr, M - 1, ctx->z.Sr, K - 4, K - 2, ctx->z.q4,
                           ctx->z.q2, pLT, pUT, puiT, rLT, rUT, ruiT, ctx->st);
  int cur = 0;   // rb[cur] = rb^n, rb[1 - cur] = rb^{n+1}
  const bool has_adj = adj_psi || adj_th || adj_u;
  if (has_adj)   // the terminal co-state, added at n = N
    launch_to_internal(M, K, reinterpret_cast<const double2*>(adj_psi),
                       reinterpret_cast<const double2*>(adj_th), adj_u, adj.p, adj.t, ctx->st);
  auto reverse_step = [&](int n, const double2* X, const double* G) -> qg_status {
    const double kappa = ew * dt * ((n == 0 || n == N) ? 0.5 : 1.0);
    Pair out = (n > 0) ? tmp : acc;
    qg_status st;
    if (n < N) {
      st = explicit_T(ctx, X, G, rb[cur].p, n + 1 < N ? rb[1 - cur].p : nullptr,
                      (n == 0 ? 1.0 : 1.5) * dt, -0.5 * dt, kappa, nullptr, rb[cur].p,
                      0.5 * dt, base, w, out);
    } else {
      st = explicit_T(ctx, X, G, nullptr, nullptr, 0.0, 0.0, kappa, has_adj ? adj.p : nullptr,
                      nullptr, 0.0, base, w, out);
    }
    if (st != QG_OK) return st;
    if (n > 0) {   // rb^{n-1} over rb^{n+1}, which is no longer needed
      if (!launch_solve_adjoint_np(ctx->g, FpT, FrT, ctx->z.q4, ctx->z.q2, tmp.p, tmp.t,
                                   rb[1 - cur].p, rb[1 - cur].t, ctx->st))
        return fail(ctx, QG_EUNSUPPORTED, "no transposed solve for this padding");
      cur = 1 - cur;
    }
    HIPCHK(hipGetLastError());
    return QG_OK;
  };
  // Blocks are swept backwards from the last one (storage set 0, filled by
  // the forward pass).  While block b is swept on the caller's stream,
  // block b - 1 is recomputed from its checkpoint into the other set on a
  // second stream; events order the two.
  const int last = std::max(nblk, 1) - 1;
  auto set_of = [&](int b) { return (last - b) & 1; };
  SweepStreams ss;
  if (last > 0) {
    int dev = 0;
    HIPCHK(hipStreamGetDevice(ctx->st, &dev));
    int prev = 0;
    HIPCHK(hipGetDevice(&prev));
    HIPCHK(hipSetDevice(dev));
    const hipError_t e = hipStreamCreateWithFlags(&ss.st2, hipStreamNonBlocking);
    HIPCHK(hipSetDevice(prev));
    HIPCHK(e);
  }
  std::vector<hipEvent_t> rec_done(std::max(nblk, 1), nullptr), rev_done(std::max(nblk, 1), nullptr);
  hipEvent_t fwd_done = nullptr;
  if (last > 0) {
    fwd_done = ss.event();
    if (!fwd_done) return fail(ctx, QG_EDEVICE, "event creation failed");
    HIPCHK(hipEventRecord(fwd_done, ctx->st));
  }
  const Scratch sc2{reinterpret_cast<double2*>(base + w.NL2),
                    reinterpret_cast<double*>(base + w.zonal2),
                    reinterpret_cast<double2*>(base + w.rhs2)};
  // y^{n0+1} .. y^{top} of block b and the fields of y^{n0} .. y^{top}, on st2
  auto recompute = [&](int b) -> qg_status {
    const int n0 = b * C, top = n0 + C - 1, set = set_of(b);
    hipStream_t main_st = ctx->st;
    ctx->st = ss.st2;
    qg_status r = QG_OK;
    launch_copy(ck(b, 0).p, Yb(set, 0).p, 2 * mk, nullptr, ctx->st);
    if (n0 > 0) launch_copy(ck(b, 1).p, E2[1].p, 2 * mk, nullptr, ctx->st);
    std::fill(has_g[set].begin(), has_g[set].end(), 0);
    for (int n = n0; n < top && r == QG_OK; ++n) {
      const int j = n - n0;
      Pair Ep = E2[(j + 1) % 2];
      r = cnab2_into(ctx, dt, Yb(set, j), E2[j % 2], n > 0 ? &Ep : nullptr, Yb(set, j + 1),
                     nullptr, Xsb(set, j), Gsb(set, j), sc2);
      has_g[set][j] = 1;
    }
    if (r == QG_OK) {
      Pair yt = Yb(set, top - n0);
      if (!launch_synth(ctx->g, yt.p, yt.t, Xsb(set, top - n0), nullptr, false, ctx->st))
        r = fail(ctx, QG_EUNSUPPORTED, "no transform kernel for these sizes");
    }
    ctx->st = main_st;
    return r;
  };
  for (int b = last; b >= 0; --b) {
    const int n0 = b * C, set = set_of(b);
    const int top = (b == last) ? N : n0 + C - 1;   // highest state of this block
    if (b > 0) {   // recompute block b - 1 into the set block b + 1 used
      HIPCHK(hipStreamWaitEvent(ss.st2, fwd_done, 0));
      if (b + 1 <= last) HIPCHK(hipStreamWaitEvent(ss.st2, rev_done[b + 1], 0));
      s = recompute(b - 1);
      if (s != QG_OK) return s;
      rec_done[b - 1] = ss.event();
      if (!rec_done[b - 1]) return fail(ctx, QG_EDEVICE, "event creation failed");
      HIPCHK(hipEventRecord(rec_done[b - 1], ss.st2));
    }
    if (b < last) HIPCHK(hipStreamWaitEvent(ctx->st, rec_done[b], 0));
    for (int n = top; n >= n0; --n) {
      s = reverse_step(n, Xsb(set, n - n0), has_g[set][n - n0] ? Gsb(set, n - n0) : nullptr);
      if (s != QG_OK) return s;
    }
    if (b > 1) {
      rev_done[b] = ss.event();
      if (!rev_done[b]) return fail(ctx, QG_EDEVICE, "event creation failed");
      HIPCHK(hipEventRecord(rev_done[b], ctx->st));
    }
  }
  launch_to_api(M, K, acc.p, acc.t, reinterpret_cast<double2*>(g_psi),
                reinterpret_cast<double2*>(g_th), g_u, ctx->st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->st));
  return QG_OK;
}

}  // namespace

extern "C" {

qg_status qg_gradient_workspace_size(const qg_ctx* ctx, int nsteps, int interval,
                                     size_t* bytes) {
  if (!ctx || !bytes || nsteps < 0 || interval < 1) return QG_EINVAL;
  *bytes = map_gradient(ctx, nsteps, interval).total;
  return QG_OK;
}

qg_status qg_gradient(qg_ctx* ctx, double dt, int nsteps, int interval, double energy_weight,
                      const double* adj_psi, const double* adj_theta, const double* adj_uphi,
                      double* grad_psi, double* grad_theta, double* grad_uphi, double* J,
                      void* work, size_t work_bytes) {
  if (!ctx) return QG_EINVAL;
  qg_status s = reverse_ok(ctx);
  if (s != QG_OK) return s;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(ctx, QG_EINVAL, "dt must be positive");
  if (nsteps < 0 || interval < 1) return fail(ctx, QG_EINVAL, "nsteps >= 0, interval >= 1");
  if (!std::isfinite(energy_weight)) return fail(ctx, QG_EINVAL, "energy_weight must be finite");
  if (!J) return fail(ctx, QG_EINVAL, "null J");
  const bool any_g = grad_psi || grad_theta || grad_uphi;
  if (any_g && !(grad_psi && grad_theta && grad_uphi))
    return fail(ctx, QG_EINVAL, "gradient outputs: all three or none");
  const GradMap w = map_gradient(ctx, nsteps, interval);
  if (!work || work_bytes < w.total) return fail(ctx, QG_EINVAL, "gradient workspace too small");
  if (reinterpret_cast<uintptr_t>(work) % 256)
    return fail(ctx, QG_EINVAL, "gradient workspace must be 256-byte aligned");
  s = gradient_run(ctx, dt, nsteps, interval, energy_weight, adj_psi, adj_theta, adj_uphi,
                   grad_psi, grad_theta, grad_uphi, J, static_cast<char*>(work), w);
  if (s == QG_OK) ctx->err.clear();
  return s;
}

qg_status qg_adjoint_explicit(qg_ctx* ctx, const double* psi, const double* theta,
                              const double* uphi, double* bar_psi, double* bar_theta,
                              double* bar_uphi, double kappa, void* work, size_t work_bytes) {
  if (!ctx) return QG_EINVAL;
  qg_status s = reverse_ok(ctx);
  if (s != QG_OK) return s;
  if (!psi || !theta || !uphi || !bar_psi || !bar_theta || !bar_uphi)
    return fail(ctx, QG_EINVAL, "null pointer");
  if (!std::isfinite(kappa)) return fail(ctx, QG_EINVAL, "kappa must be finite");
  const GradMap w = map_gradient(ctx, 0, 1);
  if (!work || work_bytes < w.total) return fail(ctx, QG_EINVAL, "workspace too small");
  if (reinterpret_cast<uintptr_t>(work) % 256)
    return fail(ctx, QG_EINVAL, "workspace must be 256-byte aligned");
  char* base = static_cast<char*>(work);
  const size_t mk = ctx->mk();
  const int M = ctx->z.M, K = ctx->z.K;
  Pair y = pair_at(base, w.blk, 0, mk), eb = pair_at(base, w.tmp, 0, mk);
  Pair out = pair_at(base, w.acc, 0, mk);
  double2* X = reinterpret_cast<double2*>(base + w.Xs);
  HIPCHK(hipMemsetAsync(ctx->nf_flag(), 0, sizeof(int), ctx->st));
  launch_to_internal(M, K, reinterpret_cast<const double2*>(psi),
                     reinterpret_cast<const double2*>(theta), uphi, y.p, y.t, ctx->st);
  launch_to_internal(M, K, reinterpret_cast<const double2*>(bar_psi),
                     reinterpret_cast<const double2*>(bar_theta), bar_uphi, eb.p, eb.t, ctx->st);
  if (!launch_synth(ctx->g, y.p, y.t, X, nullptr, false, ctx->st))
    return fail(ctx, QG_EUNSUPPORTED, "no transform kernel for these sizes");
  s = explicit_T(ctx, X, nullptr, eb.p, nullptr, 1.0, 0.0, kappa, nullptr, nullptr, 0.0, base, w,
                 out);
  if (s != QG_OK) return s;
  launch_to_api(M, K, out.p, out.t, reinterpret_cast<double2*>(bar_psi),
                reinterpret_cast<double2*>(bar_theta), bar_uphi, ctx->st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->st));
  return QG_OK;
}

}  // extern "C"

// ------------------------------------------------------------ ensembles
#ifndef QG_ENSEMBLE_GRAPH
#define QG_ENSEMBLE_GRAPH 1   // replay captured steps (0: every step eager)
#endif

struct qg_ensemble {
  std::vector<qg_ctx*> groups;   // one context per size class
  std::vector<int> grp, run;     // member -> (group, run within the group)
  hipStream_t st = nullptr;
  bool own_stream = false;
  // each group runs on a stream of its own, forked from and joined back to
  // st around every step, so that the groups' kernels overlap
  std::vector<hipStream_t> gst;
  std::vector<hipEvent_t> gev;
  hipEvent_t fork = nullptr;
  std::string err;
  // captured steps, one single-stream graph per group (replayed on the
  // group's stream between the fork and the join)
  std::vector<hipGraphExec_t> exec;
  double g_dt = 0.0;
  int g_scheme = -1, g_cur = -1, g_steps = 0;
  std::vector<int> g_mch;   // band-product shape of each group at capture
  double t = 0.0;
  long long step = 0;
};

namespace {

qg_status efail(qg_ensemble* e, qg_status s, const std::string& msg) {
  if (e) e->err = msg;
  return s;
}

// Members that share every parameter but Ra form one group (they share the
// operators, tables and LU factors).
bool same_group(const qg_params& a, const qg_params& b, const Sizes& za, const Sizes& zb) {
  return a.E == b.E && a.Pr == b.Pr && a.eta == b.eta && za.nphi == zb.nphi && za.R == zb.R &&
         za.K == zb.K && a.precision == b.precision && a.pivoting == b.pivoting &&
         a.ekman == b.ekman && (!a.ekman || a.eps == b.eps) && a.method == b.method &&
         a.buoyancy == b.buoyancy && za.mfdct == zb.mfdct;
}

struct Grouping {
  std::vector<int> first;              // first member of each group
  std::vector<std::vector<int>> mem;   // members of each group
  std::vector<int> grp, run;
  std::vector<size_t> off;             // workspace offset of each group
  size_t total = 0;
};

bool group_members(const qg_params* ps, int n, Grouping& G) {
  if (!ps || n < 1) return false;
  std::vector<Sizes> zs(n);
  std::string why;
  G.grp.assign(n, -1);
  G.run.assign(n, -1);
  for (int i = 0; i < n; ++i) {
    if (!sizes_of(&ps[i], zs[i], why)) return false;
    int g = -1;
    for (size_t j = 0; j < G.first.size(); ++j)
      if (same_group(ps[G.first[j]], ps[i], zs[G.first[j]], zs[i])) { g = (int)j; break; }
    if (g < 0) {
      g = (int)G.first.size();
      G.first.push_back(i);
      G.mem.emplace_back();
    }
    G.grp[i] = g;
    G.run[i] = (int)G.mem[g].size();
    G.mem[g].push_back(i);
  }
  Layout L;
  for (size_t j = 0; j < G.first.size(); ++j)
    G.off.push_back(L.take(map_workspace(zs[G.first[j]], (int)G.mem[j].size(), false).total));
  G.total = L.total;
  return true;
}

qg_status step_groups(qg_ensemble* e, double dt, int scheme) {
  if (hipEventRecord(e->fork, e->st) != hipSuccess)
    return efail(e, QG_EDEVICE, "hipEventRecord failed");
  for (size_t j = 0; j < e->groups.size(); ++j) {
    qg_ctx* c = e->groups[j];
    if (hipStreamWaitEvent(e->gst[j], e->fork, 0) != hipSuccess)
      return efail(e, QG_EDEVICE, "hipStreamWaitEvent failed");
    qg_status s = step_scheme(c, dt, scheme);
    if (s != QG_OK) return efail(e, s, c->err);
    if (hipEventRecord(e->gev[j], e->gst[j]) != hipSuccess ||
        hipStreamWaitEvent(e->st, e->gev[j], 0) != hipSuccess)
      return efail(e, QG_EDEVICE, "group join failed");
  }
  return QG_OK;
}

void account(qg_ensemble* e, double dt, int n) {
  for (qg_ctx* c : e->groups) {
    c->t += dt * n;
    c->step += n;
  }
  e->t += dt * n;
  e->step += n;
}

void drop_graph(qg_ensemble* e) {
  if (!e->exec.empty()) {
    (void)hipStreamSynchronize(e->st);   // no replay may be in flight
    for (hipStream_t gs : e->gst) (void)hipStreamSynchronize(gs);
    for (hipGraphExec_t x : e->exec)
      if (x) (void)hipGraphExecDestroy(x);
  }
  e->exec.clear();
  e->g_scheme = -1;
}

// Capture `steps` steps of each group on its own stream (no launch happens
// during capture; the host-side step state is restored afterwards).
qg_status capture(qg_ensemble* e, double dt, int scheme, int steps) {
  drop_graph(e);
  for (size_t j = 0; j < e->groups.size(); ++j) {
    qg_ctx* c = e->groups[j];
    const int cur = c->cur, have_prev = c->have_prev;
    if (hipStreamBeginCapture(e->gst[j], hipStreamCaptureModeRelaxed) != hipSuccess) {
      drop_graph(e);
      return efail(e, QG_EDEVICE, "hipStreamBeginCapture failed");
    }
    qg_status s = QG_OK;
    for (int i = 0; i < steps && s == QG_OK; ++i)
      s = step_scheme(c, dt, scheme);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(e->gst[j], &graph);
    c->cur = cur;
    c->have_prev = have_prev;
    if (s != QG_OK || ec != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      drop_graph(e);
      return s != QG_OK ? efail(e, s, c->err) : efail(e, QG_EDEVICE, "hipStreamEndCapture failed");
    }
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      drop_graph(e);
      return efail(e, QG_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    e->exec.push_back(x);
  }
  e->g_dt = dt;
  e->g_scheme = scheme;
  e->g_cur = e->groups[0]->cur;
  e->g_steps = steps;
  e->g_mch.clear();
  for (qg_ctx* c : e->groups) e->g_mch.push_back(c->band_mch);
  return QG_OK;
}

bool same_shapes(const qg_ensemble* e) {
  if (e->g_mch.size() != e->groups.size()) return false;
  for (size_t j = 0; j < e->groups.size(); ++j)
    if (e->g_mch[j] != e->groups[j]->band_mch) return false;
  return true;
}

// One replay of every group's graph, forked from and joined back to e->st.
qg_status replay(qg_ensemble* e) {
  if (hipEventRecord(e->fork, e->st) != hipSuccess)
    return efail(e, QG_EDEVICE, "hipEventRecord failed");
  for (size_t j = 0; j < e->groups.size(); ++j) {
    if (hipStreamWaitEvent(e->gst[j], e->fork, 0) != hipSuccess ||
        hipGraphLaunch(e->exec[j], e->gst[j]) != hipSuccess ||
        hipEventRecord(e->gev[j], e->gst[j]) != hipSuccess ||
        hipStreamWaitEvent(e->st, e->gev[j], 0) != hipSuccess)
      return efail(e, QG_EDEVICE, "graph replay failed");
  }
  return QG_OK;
}

}  // namespace

extern "C" {

qg_status qg_ensemble_workspace_size(const qg_params* members, int n, size_t* bytes) {
  Grouping G;
  if (!bytes || !group_members(members, n, G)) return QG_EINVAL;
  *bytes = G.total;
  return QG_OK;
}

qg_status qg_ensemble_create(qg_ensemble** out, const qg_params* members, int n,
                             void* workspace, size_t workspace_bytes, void* stream) {
  if (!out) return QG_EINVAL;
  *out = nullptr;
  Grouping G;
  if (!group_members(members, n, G)) return QG_EINVAL;
  if (!workspace || ((uintptr_t)workspace & 255)) return QG_EINVAL;
  if (workspace_bytes < G.total) return QG_ENOMEM;
  qg_ensemble* e = new qg_ensemble();
  e->st = static_cast<hipStream_t>(stream);
  if (!e->st) {   // the legacy default stream cannot be captured
    if (hipStreamCreateWithFlags(&e->st, hipStreamNonBlocking) != hipSuccess) {
      delete e;
      return QG_EDEVICE;
    }
    e->own_stream = true;
  }
  e->grp = G.grp;
  e->run = G.run;
  if (hipEventCreateWithFlags(&e->fork, hipEventDisableTiming) != hipSuccess) {
    qg_ensemble_destroy(e);
    return QG_EDEVICE;
  }
  for (size_t j = 0; j < G.first.size(); ++j) {
    hipStream_t gs = nullptr;
    hipEvent_t ge = nullptr;
    if (hipStreamCreateWithFlags(&gs, hipStreamNonBlocking) != hipSuccess) {
      qg_ensemble_destroy(e);
      return QG_EDEVICE;
    }
    e->gst.push_back(gs);
    if (hipEventCreateWithFlags(&ge, hipEventDisableTiming) != hipSuccess) {
      qg_ensemble_destroy(e);
      return QG_EDEVICE;
    }
    e->gev.push_back(ge);
    std::vector<double> ra;
    for (int i : G.mem[j]) ra.push_back(members[i].Ra);
    qg_ctx* c = nullptr;
    const size_t next = (j + 1 < G.off.size()) ? G.off[j + 1] : G.total;
    // set-up work on the caller's stream must precede the group's
    if (hipStreamSynchronize(e->st) != hipSuccess) {
      qg_ensemble_destroy(e);
      return QG_EDEVICE;
    }
    qg_status s = create_ctx(&c, &members[G.first[j]], (int)ra.size(), ra.data(),
                             static_cast<char*>(workspace) + G.off[j], next - G.off[j], gs,
                             false);
    if (s != QG_OK) {
      qg_ensemble_destroy(e);
      return s;
    }
    e->groups.push_back(c);
  }
  *out = e;
  return QG_OK;
}

qg_status qg_ensemble_set_state(qg_ensemble* e, int member, const double* psi,
                                const double* theta, const double* uphi, int on_device) {
  if (!e) return QG_EINVAL;
  if (member < 0 || member >= (int)e->grp.size()) return efail(e, QG_EINVAL, "no such member");
  qg_ctx* c = e->groups[e->grp[member]];
  qg_status s = set_state_run(c, e->run[member], psi, theta, uphi, on_device);
  if (s != QG_OK) return efail(e, s, c->err);
  for (qg_ctx* g : e->groups) {   // the ensemble restarts as a whole
    g->t = 0.0;
    g->step = 0;
    g->have_prev = 0;
    g->cur = 0;
    g->ms_n = 0;
    g->last_scheme = -1;
  }
  e->t = 0.0;
  e->step = 0;
  e->err.clear();
  return QG_OK;
}

qg_status qg_ensemble_get_state(qg_ensemble* e, int member, double* psi, double* theta,
                                double* uphi, int on_device) {
  if (!e) return QG_EINVAL;
  if (member < 0 || member >= (int)e->grp.size()) return efail(e, QG_EINVAL, "no such member");
  qg_ctx* c = e->groups[e->grp[member]];
  qg_status s = get_state_run(c, e->run[member], psi, theta, uphi, on_device);
  return s == QG_OK ? s : efail(e, s, c->err);
}

qg_status qg_ensemble_step(qg_ensemble* e, double dt, int scheme, int nsteps) {
  if (!e) return QG_EINVAL;
  for (qg_ctx* c : e->groups) {
    qg_status s = check_step_args(c, dt, scheme, nsteps);
    if (s != QG_OK) return efail(e, s, c->err);
  }
  if (nsteps == 0) return QG_OK;
  for (qg_ctx* c : e->groups) begin_history(c, dt, scheme);
  if (sbdf_of(scheme)) {
    // SBDF steps run eagerly: start-up steps refactor, and the history
    // ring turns every step
    drop_graph(e);
    for (int i = 0; i < nsteps; ++i) {
      qg_status s = step_groups(e, dt, scheme);
      if (s != QG_OK) return s;
      account(e, dt, 1);
    }
    return QG_OK;
  }
  for (qg_ctx* c : e->groups) {
    const double before = c->factored_adt;
    qg_status s = prepare(c, scheme_adt(scheme, dt));
    if (s != QG_OK) return efail(e, s, c->err);
    if (c->factored_adt != before) drop_graph(e);
  }
  int left = nsteps;
  // CNAB2's first step after a restart has no history: run it eagerly
  while (left > 0 && scheme == QG_CNAB2 && !e->groups[0]->have_prev) {
    qg_status s = step_groups(e, dt, scheme);
    if (s != QG_OK) return s;
    account(e, dt, 1);
    --left;
  }
  // CNAB2 alternates its two history slots: a graph holds two steps
  const int per = (scheme == QG_CNAB2) ? 2 : 1;
  if (QG_ENSEMBLE_GRAPH && left >= per) {
    if (e->exec.empty() || e->g_dt != dt || e->g_scheme != scheme || e->g_cur != e->groups[0]->cur ||
        e->g_steps != per || !same_shapes(e)) {
      qg_status s = capture(e, dt, scheme, per);
      if (s != QG_OK) return s;
    }
    for (; left >= per; left -= per) {
      qg_status sr = replay(e);
      if (sr != QG_OK) return sr;
      for (qg_ctx* c : e->groups) c->have_prev = 1;
      account(e, dt, per);
    }
  }
  for (; left > 0; --left) {
    qg_status s = step_groups(e, dt, scheme);
    if (s != QG_OK) return s;
    account(e, dt, 1);
  }
  return QG_OK;
}

qg_status qg_ensemble_step_autotune(qg_ensemble* e, double dt, int scheme, int nsteps,
                                    int* systems_per_thread) {
  if (!e || !systems_per_thread) return QG_EINVAL;
  for (qg_ctx* c : e->groups) {
    qg_status s = check_step_args(c, dt, scheme, nsteps);
    if (s != QG_OK) return efail(e, s, c->err);
  }
  const Sbdf* sb = sbdf_of(scheme);
  const int warm = sb ? sb->k : 1;
  const int per = (nsteps - warm) / TUNE_N;
  if (per < 1) return efail(e, QG_EINVAL, "autotune needs 4 timed steps after the warm-up");
  // each group in turn, alone on its stream, eagerly (no graph): its own
  // shape from its own band-product timings; every group takes the same
  // steps, so the ensemble stays in step.  Work queued on the ensemble's
  // stream comes first.
  if (hipStreamSynchronize(e->st) != hipSuccess) return efail(e, QG_EDEVICE, "sync failed");
  drop_graph(e);
  for (size_t j = 0; j < e->groups.size(); ++j) {
    qg_ctx* c = e->groups[j];
    qg_status s = tune_ctx(c, dt, scheme, warm, per);
    if (s != QG_OK) return efail(e, s, c->err);
    systems_per_thread[j] = c->band_mch;
  }
  e->t += dt * (warm + TUNE_N * per);
  e->step += warm + TUNE_N * per;
  return qg_ensemble_step(e, dt, scheme, nsteps - warm - TUNE_N * per);
}

qg_status qg_ensemble_groups(const qg_ensemble* e, int* ngroups, int* group_of_member) {
  if (!e || !ngroups) return QG_EINVAL;
  *ngroups = (int)e->groups.size();
  if (group_of_member)
    for (size_t i = 0; i < e->grp.size(); ++i) group_of_member[i] = e->grp[i];
  return QG_OK;
}

qg_status qg_ensemble_diagnostics(qg_ensemble* e, int member, qg_diag* out) {
  if (!e || !out) return QG_EINVAL;
  if (member < 0 || member >= (int)e->grp.size()) return efail(e, QG_EINVAL, "no such member");
  qg_ctx* c = e->groups[e->grp[member]];
  qg_status s = diagnostics_run(c, e->run[member], out);
  return s == QG_OK ? s : efail(e, s, c->err);
}

const char* qg_ensemble_last_error(const qg_ensemble* e) {
  return e ? e->err.c_str() : "null ensemble";
}

void qg_ensemble_destroy(qg_ensemble* e) {
  if (!e) return;
  if (e->st) (void)hipStreamSynchronize(e->st);
  for (hipStream_t gs : e->gst) (void)hipStreamSynchronize(gs);
  drop_graph(e);
  for (qg_ctx* c : e->groups) qg_destroy(c);
  for (hipEvent_t ge : e->gev) (void)hipEventDestroy(ge);
  for (hipStream_t gs : e->gst) (void)hipStreamDestroy(gs);
  if (e->fork) (void)hipEventDestroy(e->fork);
  if (e->own_stream && e->st) (void)hipStreamDestroy(e->st);
  delete e;
}

}  // extern "C"

// ------------------------------------------------- static workspace
// The workspace of qg_create_static: a device array that the library holds
// on every device it runs on until the process ends.  In host code its
// name is only a handle; its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
constexpr size_t STATIC_WS_BYTES = (size_t)128 << 20;
static __device__ __align__(256) char scratch[STATIC_WS_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex static_mu;
void* static_ptr[MAX_DEVICES] = {};     // device address of `scratch`
bool static_busy[MAX_DEVICES] = {};     // held by a live context
thread_local std::string create_err;    // message of the last failed create
}  // namespace

extern "C" {

qg_status qg_create_static(qg_ctx** out, const qg_params* p, void* stream) {
  if (!out) return QG_EINVAL;
  *out = nullptr;
  Sizes z;
  std::string why;
  if (!sizes_of(p, z, why)) {
    create_err = "invalid parameters: " + why;
    return QG_EINVAL;
  }
  const size_t need = map_workspace(z, 1, true).total;
  if (need > STATIC_WS_BYTES) {
    create_err = "these parameters need " + std::to_string(need) +
                 " workspace bytes; the static workspace holds " +
                 std::to_string(STATIC_WS_BYTES) + " (use qg_create)";
    return QG_ENOMEM;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
    create_err = "no current HIP device";
    return QG_EDEVICE;
  }
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(static_mu);
    if (static_busy[dev]) {
      create_err = "the static workspace of device " + std::to_string(dev) +
                   " is held by another context (destroy it first)";
      return QG_EINVAL;
    }
    if (!static_ptr[dev]) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) {
        create_err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
        return QG_EDEVICE;
      }
      static_ptr[dev] = ptr;
    }
    ws = static_ptr[dev];
    static_busy[dev] = true;
  }
  const qg_status s = create_ctx(out, p, 1, nullptr, ws, STATIC_WS_BYTES, stream, true);
  if (s != QG_OK) {
    std::lock_guard<std::mutex> lock(static_mu);
    static_busy[dev] = false;
    create_err = "context creation failed";
    return s;
  }
  (*out)->static_dev = dev;
  create_err.clear();
  return QG_OK;
}

const char* qg_last_error(const qg_ctx* ctx) { return ctx ? ctx->err.c_str() : create_err.c_str(); }

void qg_destroy(qg_ctx* ctx) {
  if (!ctx) return;
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->st2) {
    (void)hipStreamSynchronize(ctx->st2);
    (void)hipStreamDestroy(ctx->st2);
  }
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->static_dev >= 0) {
    (void)hipStreamSynchronize(ctx->st);   // no kernel may still use the array
    std::lock_guard<std::mutex> lock(static_mu);
    static_busy[ctx->static_dev] = false;
  }
  delete ctx;
}

qg_status qg_operator_band(double eta, int n_c, int which, double* out) {
  if (!(eta > 0 && eta < 1) || n_c < 8 || which < 0 || which > 8 || !out) return QG_EINVAL;
  Operators o = build_operators(eta, n_c);
  const std::vector<double>* bl[9] = {&o.A0, &o.A2, &o.B0, &o.B2, &o.B4, &o.C, &o.D, &o.F0, &o.F2};
  std::copy(bl[which]->begin(), bl[which]->end(), out);
  return QG_OK;
}

}  // extern "C"
