/*
 * qg.h - C ABI of the MI355X one-step solver for spherical quasi-geostrophic
 * convection (Gastine, "pizza", arXiv:1902.07092).
 *
 * The method (paper Sect. 2-4): the regularised streamfunction Psi
 * (psi = h^2 Psi, Sect. 3.2.1), the temperature perturbation theta and the
 * axisymmetric zonal flow <u_phi> are expanded in Fourier modes m = 0..N_m in
 * azimuth (N_phi = 3 N_m grid points, eq. fft/ifft) and in N_c Chebyshev
 * polynomials on N_r Gauss-Lobatto points in radius (eq. cheb/icheb).  The
 * equations are multiplied by s^4 (Psi) or s^2 (theta, zonal flow) and
 * integrated four or two times (eq. psi_int, uphi_int, temp_int), giving
 * banded operators; boundary conditions are imposed as tau rows on top
 * (eq. bc_d3psi_coll and Fig. 1b), and every m is solved as a bordered
 * band system (Appendix A).  Nonlinear advection is pseudo-spectral.  Time
 * stepping is IMEX with explicit buoyancy: the multistep schemes CNAB2
 * (eq. multistep1) and SBDF2/3/4, and the stiffly accurate SDIRK schemes
 * BPR353, ARS222 and ARS443 (Table 1, eq. dirks).  Ekman pumping is
 * optional (qg_params.ekman: the approximated F_eps of eq. approx_pump,
 * explicit).
 *
 * Conventions shared by every entry point
 *   - Coefficients are standard Chebyshev coefficients a_n, f(x) =
 *     sum_n a_n T_n(x), x = +1 at the outer radius s_o, with
 *     s_o = 1/(1-eta), s_i = eta/(1-eta) (unit gap).
 *   - psi, theta: M x N_c complex128 (interleaved re, im doubles), row
 *     m = 0..M-1, M = N_phi/3 + 1.  Row m = 0 of psi is ignored on input and
 *     returned as zeros (Psi carries the non-axisymmetric motions only).
 *     Row 0 of theta must be real.
 *   - uphi: N_c real doubles, the zonal flow <u_phi>.
 *   - Pointers flagged on_device = 1 are device pointers on the context's
 *     device; on_device = 0 means host memory.  The caller owns them; the
 *     library copies in or out and keeps nothing.
 *   - Calls that step a single-run context (qg_step and its timed and
 *     autotuned forms, qg_step_tangent) queue their kernels on the
 *     context's stream and synchronise it once at the end, to read the
 *     non-finite flag the solves set (see qg_step).  Calls that return host
 *     data (qg_get_state into host memory, qg_diagnostics, checkpoints)
 *     or refactor (a change of dt) synchronise as well.  Ensemble steps
 *     are asynchronous.
 *   - Errors are returned as qg_status; qg_last_error gives a message.
 *     Nothing is thrown across the ABI.  A context must not be used from
 *     two threads at once; distinct contexts are independent.
 */
#ifndef QG_H
#define QG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qg_ctx qg_ctx;

typedef enum {
  QG_OK = 0,
  QG_EINVAL = -1,       /* bad parameter, size or pointer */
  QG_ENOMEM = -2,       /* workspace too small */
  QG_EDEVICE = -3,      /* a HIP call failed */
  QG_ENONFINITE = -4,   /* NaN or Inf in a state */
  QG_ESTATE = -5,       /* state violates the boundary conditions */
  QG_EUNSUPPORTED = -6  /* valid for the method, not for this build's kernels */
} qg_status;

/* IMEX time schemes of Table 1 (Sect. 4), explicit buoyancy:
 *   QG_CNAB2   Crank-Nicolson / Adams-Bashforth 2 (multistep, order 2)
 *   QG_BPR353  Boscarino-Pareschi-Russo SDIRK, 5 stages (order 3)
 *   QG_ARS222  Ascher-Ruuth-Spiteri SDIRK (2,2,2) (order 2)
 *   QG_ARS443  Ascher-Ruuth-Spiteri SDIRK (4,4,3) (order 3)
 *   QG_SBDF2..4  semi-implicit backward differences (multistep, order
 *              2..4); not self-starting: while fewer than k levels are
 *              stored, SBDFk takes BPR353 steps (their factorisation is
 *              rebuilt on the switch, synchronously).
 * Multistep histories belong to the scheme and dt that made them: a step
 * with another scheme or dt restarts the history. */
typedef enum {
  QG_CNAB2 = 0,
  QG_BPR353 = 1,
  QG_ARS222 = 2,
  QG_ARS443 = 3,
  QG_SBDF2 = 4,
  QG_SBDF3 = 5,
  QG_SBDF4 = 6
} qg_scheme;

typedef struct {
  double E;      /* Ekman number  nu / (Omega d^2)            (eq. controls) */
  double Ra;     /* Rayleigh number                          (eq. controls) */
  double Pr;     /* Prandtl number                           (eq. controls) */
  double eta;    /* radius ratio s_i / s_o, 0 < eta < 1      (Sect. 2) */
  int n_phi;     /* azimuthal grid points, multiple of 3; this build needs
                    n_phi = 3 * 2^a >= 24 */
  int n_r;       /* radial Gauss-Lobatto points; this build needs
                    n_r - 1 = 2^a >= 16 or 3 * 2^a >= 24, with
                    2 (n_r - 1) <= 6144 (FP64) or 12288 (mixed).  Sizes
                    whose per-workgroup LDS needs exceed the device limit
                    give QG_EUNSUPPORTED */
  int n_c;       /* Chebyshev modes kept, 8 <= n_c < n_r; 0 selects
                    floor(2 (n_r - 1) / 3) (radial dealiasing, Sect. 3.2.1) */
  int precision; /* 0 = FP64 throughout.  1 = mixed: the transforms and
                    advection products (synthesis outputs, azimuthal FFTs
                    and products, the input of the forward radial
                    transform) in FP32 with FP32 accumulation; Chebyshev
                    recurrences, explicit-term band products, right-hand
                    sides, band LU factors, solves, state, history and
                    diagnostics in FP64 (the diagnostics use the FP64
                    transforms whenever those fit the device, i.e. up to
                    n_phi = 6144, n_r = 2049).  Mixed also accepts
                    n_phi = 12288 and n_r = 4097. */
  int pivoting;  /* band LU of the bordered systems (Appendix A):
                    0 = without row interchanges when every system's growth
                        factor max|U| / max|D| stays <= 1e4, else with
                        partial pivoting (the choice is made at each
                        factorisation and reported in qg_diag);
                    1 = always with partial pivoting */
  int ekman;     /* 1: Ekman pumping, explicit like the advection (Sect. 3.2):
                    the approximated F_eps of eq. approx_pump in the Psi
                    equation, and Upsilon_eps u (1 + (E/2) omega_0) in the
                    zonal-flow equation (its pumping term, eq. uphi, and the
                    zonal wind's self-interaction in N_uphi); 0: none */
  double eps;    /* eps of F_eps (h_eps^2 = (s_o + eps)^2 - s^2); > 0 and
                    finite when ekman = 1, ignored otherwise */
  int method;    /* boundary conditions of the integration method
                    (Sect. 3.2.2):
                    0 = tau rows on top of every operator, bordered solves
                        (Appendix A);
                    1 = Galerkin bases (eq. psiint_galerkin, uphi_galerkin,
                        temp_galerkin; Appendix B): Psi on
                        phi_n = sum_i gamma_i^n T_{n+i}, zonal flow and
                        temperature on T_{n+2} - T_n, pure band systems
                        (8 sub- and 12 super-diagonals for Psi, 4 and 6 for
                        the others) solved without row interchanges.  The
                        state stays in Chebyshev coefficients.  Needs
                        pivoting = 0 (QG_EUNSUPPORTED otherwise, and from a
                        factorisation whose growth factor exceeds 1e4); the
                        reverse-mode entries (qg_gradient,
                        qg_adjoint_explicit, qg_adjoint_solve) return
                        QG_EUNSUPPORTED. */
  int buoyancy;  /* buoyancy term of the vorticity equation (Sect. 4):
                    0 = explicit, with the advection (E_psi carries
                        C[(Ra/Pr)(i m/s_o) theta]);
                    1 = implicit: the term belongs to the implicit operator
                        (Crank-Nicolson in CNAB2, the implicit tableau in a
                        DIRK stage, b_0 in SBDF) and every implicit solve
                        advances theta first, then Psi with a dt C[(Ra/Pr)
                        (i m/s_o) theta_new] added to its right-hand side.
                        Needs the unpivoted factors (pivoting = 1, or a
                        factorisation that falls back to pivoting, gives
                        QG_EUNSUPPORTED); the tangent-linear and
                        reverse-mode entries return QG_EUNSUPPORTED. */
  int dct;       /* radial transforms (eq. cheb, icheb) of the synthesis and
                    the analysis: 0 = the library's choice for the size;
                    1 = FFTs of the even extension (every size);
                    2 = dense products on the FP64 matrix cores (per m one
                        [N_r x N_c] x [N_c x 12] product for the six
                        synthesised series, one [N_c x N_r] x [N_r x 4]
                        for the two analysed fields), FP64 only and
                        2 (n_r - 1) <= 512, else QG_EUNSUPPORTED. */
} qg_params;

typedef struct {
  double t;         /* simulated time since the last qg_set_state */
  double E_kin;     /* (1/2) <u_s^2 + u_phi^2>              (Sect. 6.2) */
  double E_zon;     /* (1/2) <<u_phi>^2>                     (Sect. 6.2) */
  double E_therm;   /* (1/2) <theta^2> */
  double enstrophy; /* <omega^2>                            (Sect. 4) */
  double Re;        /* [2 E_kin / (pi (s_o^2 - s_i^2))]^1/2  (Sect. 6.3) */
  double Ro;        /* Re E                                  (Sect. 6.3) */
  double dt_cfl;    /* right side of eq. (cfl) with alpha = 1 */
  long long step;   /* steps taken since the last qg_set_state */
  int nonfinite;    /* 1 if the state holds NaN or Inf */
  int pivoted;      /* 1 if the band LUs in use have row interchanges */
  double growth;    /* largest growth factor max|U| / max|D| of those LUs
                       (0 before the first factorisation) */
} qg_diag;

/* Device bytes the caller must provide to qg_create for these parameters.
 * Returns QG_EINVAL for invalid or unsupported parameters. */
qg_status qg_workspace_size(const qg_params *p, size_t *bytes);

/* Create a context on the current HIP device.  workspace: device memory
 * of at least qg_workspace_size bytes, 256-byte aligned, owned by the
 * caller and kept alive until qg_destroy.  stream: a hipStream_t (NULL =
 * default stream).  Builds the integration operators on the host
 * (Sect. 3.2) and uploads them.  The state starts at zero. */
qg_status qg_create(qg_ctx **ctx, const qg_params *p, void *workspace,
                    size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * qg_create with the workspace in a static device array of 128 MiB that the
 * library holds on each device it runs on until the process ends (enough
 * for every size up to n_phi x n_r = 768 x 257).  The library allocates no
 * device memory in this call or later ones; the caller passes only the
 * stream.  The array is shared by every call on the device, so at most one
 * such context per device exists at a time: a second one gets QG_EINVAL
 * until the first is destroyed (overlapping use would race).  Parameters
 * whose workspace exceeds the array give QG_ENOMEM.  On failure
 * qg_last_error(NULL) gives the message.  Otherwise as qg_create. */
qg_status qg_create_static(qg_ctx **ctx, const qg_params *p, void *stream);

/* Copy a state in.  Host inputs are checked: non-finite values give
 * QG_ENONFINITE, boundary-condition residuals above 1e-10 relative give
 * QG_ESTATE (tau conditions, Sect. 3.2.2).  Resets t, the step counter and
 * the multistep history. */
qg_status qg_set_state(qg_ctx *ctx, const double *psi, const double *theta,
                       const double *uphi, int on_device);

/* Copy the current state out (row m = 0 of psi is written as zeros). */
qg_status qg_get_state(qg_ctx *ctx, double *psi, double *theta, double *uphi,
                       int on_device);

/* Advance nsteps steps of size dt with the given scheme (qg_scheme).  The
 * bordered LU factors of every m are rebuilt on the host (synchronously)
 * whenever the implicit coefficient a_ii dt changes (Sect. 3.1:
 * factorisation at start-up and on a time-step change).  CNAB2 uses
 * E^{n-1} := E^n on the first step of its history.  QG_EINVAL for an
 * unknown scheme, dt <= 0 or nsteps < 0.
 *
 * Non-finite values: every solve checks the new state it writes.  A step
 * whose new state (or a stage of it) holds NaN or Inf is discarded: the
 * call returns QG_ENONFINITE, the context keeps the state, multistep
 * history, time and step count from before that step (steps before it in
 * the same call are kept), and qg_last_error names the step.  The steps
 * queued after it do nothing.  The call synchronises the stream once at
 * its end to read the flag.
 *
 * Streams: a context of qg_create stepping CNAB2 puts the band product of
 * each right-hand side on a second HIP stream that the call creates
 * (default priority, non-blocking) and destroys before it returns; events
 * order it after the context's stream and the rest of the step after it,
 * so that the caller sees one stream.  The results equal the one-stream
 * sequence bit for bit.  Ensemble groups, qg_create_static contexts,
 * qg_step_timed and a stream under graph capture use the context's
 * stream alone. */
qg_status qg_step(qg_ctx *ctx, double dt, int scheme, int nsteps);

/* Checkpoints of a single-run context: the state and the multistep history
 * of the scheme in use (CNAB2's stored E^{n-1}; for SBDFk the stored
 * explicit terms and states, at most three levels each; the SDIRK
 * schemes keep none), with the time, step count, scheme and dt.  A run
 * resumed with qg_checkpoint_load (into this or another context with the
 * same parameters) and stepped on with the same scheme and dt equals the
 * uninterrupted run bit for bit.  The buffer is the caller's, host memory
 * or (on_device = 1) device memory, at least qg_checkpoint_size bytes
 * (which depends on the history held when it is asked).  qg_checkpoint_load
 * returns QG_EINVAL for a buffer that is too short, not a checkpoint, or
 * one of a problem with other sizes or parameters; it resets a tangent
 * run.  Both synchronise the stream. */
qg_status qg_checkpoint_size(const qg_ctx *ctx, size_t *bytes);
qg_status qg_checkpoint_save(qg_ctx *ctx, void *buf, size_t bytes, int on_device);
qg_status qg_checkpoint_load(qg_ctx *ctx, const void *buf, size_t bytes, int on_device);

/* qg_step with per-kernel timing, for benchmarks: HIP events are recorded
 * on the context's stream around every kernel launch.  On return (stream
 * synchronised) kernel_ms[c] holds the summed duration in milliseconds and
 * launches[c] the number of launches of kernel class c:
 *   0 synthesis (inverse DCT + fields, per m)   1 azimuthal transforms and
 *   products (per radial level)   2 analysis (forward DCT + explicit terms,
 *   per m)   3 bordered solves of every system (one launch)   4 right-hand
 *   sides of every system (one launch).
 * A dt or scheme change refactorises before the timed steps (SBDF
 * start-up steps refactorise inside them). */
qg_status qg_step_timed(qg_ctx *ctx, double dt, int scheme, int nsteps,
                        double *kernel_ms, int *launches);

/* qg_step with an autotuner for the launch shape of the band-product
 * kernel (right-hand sides and stage products, Sect. 4 with the operators
 * of Sect. 3.2): after an untimed warm-up (1 step; k steps for SBDFk, which
 * covers its start-up), the steps are split evenly over the candidate
 * shapes of 4, 8, 16 and 32 systems per thread, each candidate's steps
 * timed with HIP events on the context's stream; the fastest shape is kept
 * for this and later calls and written to *systems_per_thread.  Every
 * entry of a product is computed by one thread in the same order for
 * every shape, so the run is exactly that of qg_step with the same
 * arguments.  Synchronises once.  QG_EINVAL if fewer than 4 steps remain
 * after the warm-up, or for qg_step's invalid arguments. */
qg_status qg_step_autotune(qg_ctx *ctx, double dt, int scheme, int nsteps,
                           int *systems_per_thread);

/* Tangent-linear runs (toward the adjoint of the time-integrated kinetic
 * energy; single-run contexts): qg_tangent_set loads a perturbation d of
 * the current state (same layout and checks as qg_set_state: it must meet
 * the homogeneous boundary conditions); qg_step_tangent advances the state
 * and d together by CNAB2 steps, d by the derivative of the step at the
 * current state,
 *   (M - dt/2 L) d^{n+1} = (M + dt/2 L) d^n + dt (3/2 T^n - 1/2 T^{n-1}),
 *   T^n = E'(y^n) d^n = (E(y^n + c d^n) - E(y^n - c d^n)) / (2c)
 * (exact for the quadratic explicit terms E of Sect. 3.2, c = max|y| /
 * max|d| at qg_tangent_set), with qg_step's rules for dt and the history
 * (T^{-1} := T^0 when the state's history starts at the same step, else
 * 0); qg_tangent_get copies d out.  Each tangent step costs two explicit
 * evaluations, one band product and one solve more than a CNAB2 step.
 * QG_ESTATE if no tangent state was set (qg_set_state clears it).  A
 * non-finite state or tangent discards the step as in qg_step and clears
 * the tangent (it is updated in place). */
qg_status qg_tangent_set(qg_ctx *ctx, const double *dpsi, const double *dtheta,
                         const double *duphi, int on_device);
qg_status qg_step_tangent(qg_ctx *ctx, double dt, int nsteps);
qg_status qg_tangent_get(qg_ctx *ctx, double *dpsi, double *dtheta,
                         double *duphi, int on_device);

/* The adjoint (in the real inner product) of the implicit solve of a
 * CNAB2 step of size dt, Appendix A: per system, r = Z S^-H P x, S the
 * bordered tau matrix (S^-T for the real theta and zonal-flow systems), P
 * the projection that keeps theta at m = 0 real, Z the zeroing of the tau
 * rows of the right-hand side; computed with the stored band-LU factors
 * (refactorised first if dt differs, synchronously).  In place on arrays
 * in the state layout (psi row 0 is written as zeros, the zonal flow is
 * uphi).  The first piece of a reverse sweep; single-run contexts only.
 * QG_EUNSUPPORTED when the factors use row interchanges (qg_params.pivoting
 * or a growth factor above the unpivoted bound). */
qg_status qg_adjoint_solve(qg_ctx *ctx, double dt, double *psi, double *theta,
                           double *uphi, int on_device);

/* The adjoint of the band products of a step's right-hand side (Sect. 4,
 * eq. multistep1): x <- (Mass + c Lin)^H x per system (Psi: A_m + c B_m;
 * theta: D + c F_m / Pr; zonal flow: D + c E), the rows below the tau rows
 * of x only (those of the solve's adjoint are zero).  In place, state
 * layout as qg_adjoint_solve; single-run contexts only. */
qg_status qg_adjoint_mass_lin(qg_ctx *ctx, double c, double *psi,
                              double *theta, double *uphi, int on_device);

/* Reverse mode (discrete adjoint of the CNAB2 step, Sect. 4 eq. multistep1
 * with E^{-1} := E^0, through the bordered solves of Appendix A).
 *
 * qg_gradient runs nsteps CNAB2 steps of size dt from the current state
 * y^0 (its CNAB2 history restarts there, as after qg_set_state) and
 * returns
 *   J = energy_weight * dt * sum_{n=0}^{N} w_n E_K(y^n)
 *       (w_n trapezoid weights, 1/2 at n = 0 and N; E_K the kinetic energy
 *       of Sect. 6.2 as in qg_diagnostics)
 * in *J (host), and, when the three grad_* pointers are given, the
 * gradient of J + <ybar_N, y^N> with respect to y^0 in grad_* (ybar_N the
 * terminal co-state adj_*, or zero when those three are NULL): the
 * co-state of each complex entry z is dJ/dRe z + i dJ/dIm z, so that for a
 * perturbation d of y^0, dJ = sum Re(conj(grad) d).  The reverse sweep
 * keeps the forward state and E^{n-1} at every interval-th step and
 * recomputes each block of `interval` steps (but the last) from it; the
 * recomputation of the next block runs on a second stream of the same
 * device, created and destroyed by the call, while the current block is
 * swept backwards on the context's stream.
 * All arrays are device memory in the state layout of qg_set_state (psi
 * [M][K] complex with its row 0 unused, theta [M][K] complex, uphi [K]).
 * work: device memory of at least qg_gradient_workspace_size bytes,
 * 256-byte aligned, owned by the caller and free again on return.  The
 * context ends at y^N with the CNAB2 history of that run (qg_step may
 * continue it).  Synchronous.  Single-run FP64 contexts without Ekman
 * pumping (else QG_EINVAL / QG_EUNSUPPORTED); the gradient needs the
 * unpivoted band LU (QG_EUNSUPPORTED otherwise; J alone does not).  A
 * non-finite forward state returns QG_ENONFINITE with the context
 * unchanged; the reverse sweep itself is not checked. */
qg_status qg_gradient_workspace_size(const qg_ctx *ctx, int nsteps,
                                     int interval, size_t *bytes);
qg_status qg_gradient(qg_ctx *ctx, double dt, int nsteps, int interval,
                      double energy_weight, const double *adj_psi,
                      const double *adj_theta, const double *adj_uphi,
                      double *grad_psi, double *grad_theta, double *grad_uphi,
                      double *J, void *work, size_t work_bytes);

/* The transposed explicit terms at a state y (Sect. 3.2, eq. psi_int,
 * temp_int, uphi_int): bar <- E'(y)^H bar + kappa grad E_K(y), in place on
 * the co-state bar; y and bar are device arrays in the state layout, y
 * need not be the context's state.  work: as for qg_gradient with
 * nsteps = 0, interval = 1.  The piece of the reverse sweep that holds the
 * transforms; for checking it against a reference.  Synchronous; the same
 * contexts as qg_gradient. */
qg_status qg_adjoint_explicit(qg_ctx *ctx, const double *psi,
                              const double *theta, const double *uphi,
                              double *bar_psi, double *bar_theta,
                              double *bar_uphi, double kappa, void *work,
                              size_t work_bytes);

/* Diagnostics of the current state (synchronises the stream). */
qg_status qg_diagnostics(qg_ctx *ctx, qg_diag *out);

/* Message of the last error on this context ("" if none); with ctx =
 * NULL, the message of this thread's last failed qg_create_static. */
const char *qg_last_error(const qg_ctx *ctx);

/* Release the context (not the caller's workspace). */
void qg_destroy(qg_ctx *ctx);

/* ---------------------------------------------------------------------
 * Ensembles: many runs of the step advanced together (runs of uneven size
 * and Rayleigh number, as in the paper's range of problem sizes, Sect. 5).
 * Members that share every parameter except Ra form a group: one launch of
 * each kernel advances every run of a group (the run is a grid dimension),
 * and the runs of a group share operators, twiddle tables and LU factors
 * (the bordered matrices do not depend on Ra, Sect. 3.2 and Appendix A).
 * Each group runs on a stream of its own, forked from and joined back to
 * the ensemble's stream around every step, so that groups overlap.  Steps
 * after the first are captured once per (dt, scheme) into one HIP graph
 * per group (on the group's stream) and replayed (CNAB2 and the SDIRK
 * schemes; SBDF steps run eagerly); each member's arithmetic
 * is exactly that of a single-run context with its parameters, so results
 * are identical to stepping it alone.  An ensemble must not be used from
 * two threads at once.
 */
typedef struct qg_ensemble qg_ensemble;

/* Device bytes for an ensemble of n members with parameters members[0..n-1]
 * (each valid for qg_workspace_size).  QG_EINVAL on an invalid member. */
qg_status qg_ensemble_workspace_size(const qg_params *members, int n,
                                     size_t *bytes);

/* Create an ensemble on the current device.  workspace: at least
 * qg_ensemble_workspace_size bytes, 256-byte aligned, caller-owned until
 * qg_ensemble_destroy.  stream: a hipStream_t; NULL makes the ensemble
 * create (and later destroy) a stream of its own, since graph capture
 * needs a stream other than the legacy default one.  States start at
 * zero. */
qg_status qg_ensemble_create(qg_ensemble **e, const qg_params *members,
                             int n, void *workspace, size_t workspace_bytes,
                             void *stream);

/* Copy member `member`'s state in, with the checks of qg_set_state.  The
 * ensemble restarts as a whole: time, step counter and the CNAB2 history of
 * every member are reset, so set every member before stepping. */
qg_status qg_ensemble_set_state(qg_ensemble *e, int member, const double *psi,
                                const double *theta, const double *uphi,
                                int on_device);

/* Copy member `member`'s current state out (as qg_get_state). */
qg_status qg_ensemble_get_state(qg_ensemble *e, int member, double *psi,
                                double *theta, double *uphi, int on_device);

/* Advance every member nsteps steps of size dt with the given scheme
 * (qg_step's rules: refactorisation on a change of a_ii dt, synchronous;
 * the multistep history rules).  Asynchronous on the ensemble's stream
 * otherwise. */
qg_status qg_ensemble_step(qg_ensemble *e, double dt, int scheme, int nsteps);

/* Number of size groups of the ensemble, and (if group_of_member is not
 * NULL) the group of each member (an array of n ints). */
qg_status qg_ensemble_groups(const qg_ensemble *e, int *ngroups,
                             int *group_of_member);

/* qg_ensemble_step with the band-product autotuner of qg_step_autotune,
 * per size group: after work queued on the ensemble's stream, each group in
 * turn runs the warm-up and candidate steps alone on its own stream,
 * eagerly, timing its band-product launches; it keeps its fastest shape
 * (systems_per_thread[g] for group g: an array of at least ngroups ints).
 * Every group takes the same steps; the remaining steps follow as in
 * qg_ensemble_step (graphs captured for the new shapes).  The members'
 * results equal those of qg_ensemble_step.  QG_EINVAL if fewer than 4
 * steps remain after the warm-up. */
qg_status qg_ensemble_step_autotune(qg_ensemble *e, double dt, int scheme,
                                    int nsteps, int *systems_per_thread);

/* Diagnostics of member `member` (synchronises the stream). */
qg_status qg_ensemble_diagnostics(qg_ensemble *e, int member, qg_diag *out);

/* Message of the last error on this ensemble ("" if none). */
const char *qg_ensemble_last_error(const qg_ensemble *e);

/* Release the ensemble (not the caller's workspace). */
void qg_ensemble_destroy(qg_ensemble *e);

/* Host-only: the banded integration operators qg_create builds for radius
 * ratio eta and n_c modes (eq. psi_int, uphi_int, temp_int), for checking
 * against a reference without a device.  which = 0..8 selects A0, A2, B0,
 * B2, B4, C, D, F0, F2 with A_m = A0 + m^2 A2 (int^4 s^4 L_I),
 * B_m = B0 + m^2 B2 + m^4 B4 (int^4 s^4 Lap_m L_I, Coriolis term excluded),
 * C = int^4 s^4, D = int^2 s^2, F_m = F0 + m^2 F2 (int^2 s^2 Lap_m).
 * out: host array of n_c x 17 doubles, entry [k][n - k + 8]; rows below
 * the tau rows (k < 4 for A, B, C; k < 2 for D, F) are zero. */
qg_status qg_operator_band(double eta, int n_c, int which, double *out);

#ifdef __cplusplus
}
#endif

#endif /* QG_H */
