/*
 * rve.h -- C ABI of the MI355X variational FFT homogenization library.
 *
 * The library solves, increment by increment, the periodic boundary-value
 * problem of a representative volume element (RVE) stated in Lucarini &
 * Segurado, "On the accuracy of spectral solvers for micromechanics based
 * fatigue modeling" (arXiv:1806.10599):
 *
 *   Sec. 2.1, Eq. 1     Div P = 0,  F = Fbar + Ftilde,  <F> = Fbar, Ftilde periodic
 *   Sec. 2.1, Eq. 2     P = P(F, alpha) at every voxel (internal variables alpha)
 *   Sec. 2.1, Eqs. 9-11 discrete equilibrium G(P) = F^-1{ Ghat : F(P) } = 0
 *   Sec. 2.1, Eqs.12-16 Newton iterations; each linear step G(K:dF) = -G(P) is
 *                       solved with conjugate gradients (text after Eq. 16)
 *   Sec. 2.2, Eqs.18-21 continuous (Eq. 19) or discrete (Eq. 21) projection
 *   Sec. 3.2, Eq. 22    crystal-plasticity flow rule of the grains
 *   Sec. 3.3, Eqs.23-24 fatigue indicator fields accumulated per cycle
 *
 * Conventions (all entry points):
 *   - Every function returns rve_status (0 = RVE_OK, < 0 = error).  No C++
 *     exception crosses the ABI.  On error, rve_last_error(h) describes it.
 *   - Grid: n[0] x n[1] x n[2] voxels (the GPU path requires a cubic grid,
 *     n in {16, 24, 32, 40, 48, 64, 96, 128}); cell size L[3].
 *   - Voxel (a, b, c) has flat index v = (a*n1 + b)*n2 + c (z fastest).
 *   - Second-order tensor fields are SoA: component c = 3*i + j (row-major
 *     3x3), stored as [9][N] doubles; c-th component of voxel v at c*N + v.
 *   - Units: stresses and moduli in MPa, time in s.
 *   - Pointers: host pointers unless an argument says otherwise.  The caller
 *     owns all inputs and outputs; the library copies inputs during the call
 *     and owns all device state, allocated through rve_config.dev_alloc (or
 *     hipMalloc when NULL) and released by rve_destroy.
 *   - Work is ordered on rve_config.stream.  Calls that return host results
 *     synchronize that stream before returning.
 *   - A HIP runtime error poisons the handle (RVE_EDEVICE); only
 *     rve_last_error and rve_destroy are valid afterwards.
 *   - One handle per host thread at a time; handles are independent.
 */
#ifndef RVE_H
#define RVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rve_s* rve_t;

typedef enum {
  RVE_OK = 0,
  RVE_EINVAL = -1,   /* bad argument; nothing was changed                   */
  RVE_ENOMEM = -2,   /* device allocation failed                            */
  RVE_EDEVICE = -3,  /* HIP runtime error; handle is poisoned               */
  RVE_ENOTCONV = -4, /* Newton did not converge; committed state unchanged  */
  RVE_ELOCAL = -5,   /* a voxel's return mapping failed; state unchanged    */
  RVE_ESTATE = -6    /* call not valid in the current state                 */
} rve_status;

/* Device allocator hooks (e.g. a framework's caching allocator). */
typedef void* (*rve_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*rve_free_fn)(void* ptr, void* ctx);

enum { RVE_PROJ_CONTINUOUS = 0,   /* Ghat  of Sec. 2.2, Eq. 19 */
       RVE_PROJ_DISCRETE = 1 };   /* Ghat' of Sec. 2.2, Eq. 21 */
enum { RVE_PREC_FP64 = 0,         /* every pass in FP64                      */
       RVE_PREC_MIXED = 1 };      /* FFT/projection/CG in FP32; return
                                     mapping, residual, averages in FP64     */

typedef struct {
  int32_t n[3];          /* voxels per axis                                  */
  double L[3];           /* cell edge lengths (only ratios matter)           */
  int32_t projection;    /* RVE_PROJ_*                                       */
  int32_t precision;     /* RVE_PREC_*                                       */
  int32_t warm_start;    /* 0 = homogeneous predictor; 1 = learned: the
                            candidate and the homogeneous predictor are both
                            evaluated and the smaller FP64 residual wins;
                            2 = learned, and a candidate whose FP64 residual
                            is below half of the homogeneous predictor's
                            last evaluated one is kept without evaluating
                            the homogeneous predictor (needs a network
                            attached with rve_attach_warm_start);
                            3 = as 2 with the extrapolation F_prev + dF_bar
                            + c G(dFt_prev) in place of the network: the
                            last fluctuation increment scaled by the load
                            ratio c = dF_bar : dF_bar_prev / |dF_bar_prev|^2
                            (the baseline the learned start is measured
                            against; no network needed)                      */
  int32_t use_graph;     /* 1 = replay CG chunks from a captured hipGraph    */
  double newton_tol;     /* equilibrium: ||G(P)||_2 <= tol ||P||_2 (FP64)     */
  int32_t newton_max_iter;
  double cg_tol;         /* CG stop: ||r||_2 <= cg_tol ||b||_2               */
  int32_t cg_max_iter;
  int32_t cg_chunk;      /* CG iterations between host convergence checks    */
  void* stream;          /* hipStream_t; NULL = default stream               */
  rve_alloc_fn dev_alloc;
  rve_free_fn dev_free;
  void* alloc_ctx;
  int32_t cg_forcing;    /* 0: every linear solve to cg_tol; 1: Newton
                            iteration k solves to min(0.1, max(cg_tol,
                            newton_tol / (4 r_k))), r_k = ||G(P)||/||P|| at
                            its start, i.e. only as far as reaching the
                            equilibrium tolerance needs; 2: min(0.1,
                            max(cg_tol, newton_tol / (2 r_k), 0.05 r_k))
                            (far from equilibrium the quadratic term of
                            Newton's method dominates the next residual).
                            Per RVE in a batch; other values are EINVAL. */
} rve_config;

#define RVE_MAX_NEWTON_LOG 64

typedef struct {
  int32_t newton_iters;      /* Newton corrections performed                  */
  int32_t cg_iters_total;    /* CG matvecs over the increment                 */
  int32_t local_failures;    /* voxels whose return mapping failed            */
  int32_t used_learned;      /* 1 if the learned warm start was accepted      */
  int32_t cg_breakdowns;     /* CG solves stopped by p.Ap <= 0                 */
  int32_t status;            /* rve_status of the increment                   */
  double residual_rel;       /* final ||G(P)||/||P||                          */
  double predictor_residual; /* ||G(P)||/||P|| of the accepted predictor     */
  double plain_predictor_residual; /* same for the homogeneous predictor
                                      (-1: not evaluated, warm_start = 2) */
  double P_bar[9];           /* <P>, row-major                                */
  double sigma_bar[9];       /* P_bar Fbar^T / det Fbar                       */
  double residual_history[RVE_MAX_NEWTON_LOG];
  int32_t cg_iters[RVE_MAX_NEWTON_LOG];
  double seconds;            /* wall time of the call                          */
} rve_increment_info;

/* Fills *cfg with defaults: 16^3 cube of edge 1, discrete operator, FP64,
   homogeneous predictor, tol 1e-6, 25 Newton, cg_tol 1e-4, 2000 CG,
   chunk 8, default stream, hipMalloc. */
rve_status rve_config_default(rve_config* cfg);

/* Creates a handle and allocates all device buffers for the grid.
   Errors: RVE_EINVAL (unsupported grid or options), RVE_ENOMEM, RVE_EDEVICE. */
rve_status rve_create(const rve_config* cfg, rve_t* out);

/* Releases every device buffer; NULL-safe.  Synchronizes the stream. */
rve_status rve_destroy(rve_t h);

/* Parameter block layout (params[nparams], nparams >= 10), MPa and s:
     0 C11, 1 C12, 2 C44          cubic elastic constants of the grains
     3 gdot0, 4 g, 5 n            flow rule of Eq. 22: gdot0 |(tau-chi)/g|^n
     6 c, 7 d                     back stress: chi = (chi0 + c dg)/(1 + d|dg|)
     8 E, 9 nu                    isotropic St-Venant-Kirchhoff second phase
*/
#define RVE_NPARAMS 10

/* Microstructure (Sec. 2.1 text before Eq. 6; Sec. 3.1): phase[N] labels in
   [0, G); quat[G*4] unit quaternions (w, x, y, z) rotating lattice to sample
   frame; law[G] 0 = FCC crystal plasticity, 1 = isotropic SVK.  Resets the
   state to F = I, Fp^-1 = I, chi = 0, indicator fields = 0, t = 0.
   Errors: RVE_EINVAL for labels out of range, non-unit quaternions, unknown
   laws or nparams < RVE_NPARAMS (state untouched). */
rve_status rve_set_microstructure(rve_t h, const int32_t* phase, int32_t G,
                                  const double* quat, const int32_t* law,
                                  const double* params, int32_t nparams);

/* User material in the form of a commercial FE code's finite-strain user
   subroutine (Appendix A; Sec. 2.3 of the paper describes plugging such
   subroutines into the solver).  The solver calls fn at every constitutive
   evaluation of the increment algorithm with device pointers, structure-of-
   arrays over the n voxels (component c of voxel v at c*n + v), float64:
     F1 [9][n]         deformation gradient at t_k (row-major 3x3)
     F0 [9][n]         committed deformation gradient at t_k-1
     statev_old [nstatev][n]  committed state variables (read only)
     statev_new [nstatev][n]  trial state variables (write every entry)
     sigma [6][n]      Cauchy stress at t_k, order 11, 22, 33, 12, 13, 23
     ddsdde [36][n]    6x6 tangent of the Jaumann rate of the Kirchhoff stress
                       divided by J (Eq. A.2), entry (I, J) at (6 I + J) n + v,
                       engineering shear strains
     fails             device int32 counter: add 1 per voxel whose update failed
   dt is the time step; stream the hipStream_t on which fn must enqueue its
   work (it must not synchronize the device or read the outputs back).  fn
   returns 0 when the work was enqueued, anything else is an error
   (RVE_EDEVICE from the increment).  The library then forms P (Eq. A.1) and,
   before each linear solve, K (Eq. A.16).  The pointers are valid only
   during the call; the library owns them.  State variables are committed
   with the increment (rolled back on RVE_ENOTCONV / RVE_ELOCAL). */
typedef int32_t (*rve_umat_fn)(void* user, const double* F1, const double* F0,
                               const double* statev_old, double* statev_new,
                               int32_t nstatev, double* sigma, double* ddsdde,
                               int32_t* fails, int64_t n, double dt,
                               void* stream);

/* Uses fn for every voxel in place of the crystal-plasticity microstructure
   (user is passed through to fn).  statev0: host [nstatev][N] initial state
   variables (may be NULL when nstatev = 0), 0 <= nstatev <= 1024.  Resets
   the state to F = I, P = 0, t = 0.  The fatigue indicator fields stay zero,
   the learned warm start is not used, and the crystal-only entry points
   (rve_debug_constitutive, rve_bench_kernels, rve_ws_features and the FPINV,
   CHI and DGAMMA fields) return RVE_ESTATE until rve_set_microstructure is
   called again.  Checkpoint blobs then also hold the state variables.
   Errors: RVE_EINVAL (null fn, nstatev out of range, null statev0),
   RVE_ENOMEM. */
rve_status rve_set_user_material(rve_t h, rve_umat_fn fn, void* user,
                                 int32_t nstatev, const double* statev0);

/* The example user material shipped with the library, an rve_umat_fn: a
   compressible neo-Hookean solid, tau = mu (B - I) + lambda ln J I, with its
   exact Jaumann tangent.  State variables (nstatev >= 3): 0 mu, 1 lambda
   (per voxel, MPa), 2 the sum over converged increments of |J - J_prev|.
   user is ignored; returns 0, or -1 for nstatev < 3 or a launch failure.
   A voxel with det F1 <= 0 counts as a failure. */
int32_t rve_umat_neo_hooke(void* user, const double* F1, const double* F0,
                           const double* statev_old, double* statev_new,
                           int32_t nstatev, double* sigma, double* ddsdde,
                           int32_t* fails, int64_t n, double dt, void* stream);

/* One load increment to the macroscopic gradient F_bar_new[9] (row-major)
   over the time step dt (Sec. 2.1, Eqs. 12-16 and the end of Sec. 2.1).
   Predictor F = F_prev + (F_bar_new - F_bar_prev) (plus the projected
   learned correction when enabled); Newton-CG to newton_tol; on success the
   internal variables and fatigue indicators are committed.  On
   RVE_ENOTCONV / RVE_ELOCAL nothing is committed.  info may be NULL. */
rve_status rve_apply_macro_strain_increment(rve_t h, const double F_bar_new[9],
                                            double dt,
                                            rve_increment_info* info);

/* Automatic time incrementation (named among the solver's capabilities in
   Sec. 2.3, without an algorithm; this is the library's reading): the
   step to F_bar_new over dt is first tried whole; after a failed attempt
   (RVE_ENOTCONV or RVE_ELOCAL, nothing committed) the sub-step is halved,
   after grow_after converged sub-steps in a row it is doubled (never past
   the rest of the step).  Sub-step targets lie on the straight path
   F_bar_0 + f (F_bar_new - F_bar_0) with time step f dt; the last one is
   F_bar_new itself.  When the sub-step would fall below 2^-max_cutbacks of
   the step the call fails with the last attempt's status and the RVE is
   returned to its state before the call (also when a sub-step target is
   rejected with RVE_EINVAL).  0 <= max_cutbacks <= 30, grow_after >= 1.
   info (may be NULL) sums the converged sub-steps. */
typedef struct {
  int32_t status;             /* rve_status of the call                      */
  int32_t substeps;           /* converged sub-steps                          */
  int32_t cutbacks;           /* failed attempts                              */
  int32_t newton_iters_total; /* Newton corrections of converged sub-steps   */
  int32_t cg_iters_total;     /* CG matvecs of converged sub-steps            */
  int32_t pad;
  double min_fraction;        /* smallest converged sub-step / step (0: none) */
  double seconds;             /* wall time of the call                        */
  rve_increment_info last;    /* the last attempt                             */
} rve_adaptive_info;

rve_status rve_apply_macro_strain_increment_adaptive(
    rve_t h, const double F_bar_new[9], double dt, int32_t max_cutbacks,
    int32_t grow_after, rve_adaptive_info* info);

/* Zeroes the per-cycle indicator accumulators (call at each cycle start). */
rve_status rve_reset_fips(rve_t h);

enum {
  RVE_FIELD_F = 0,         /* [9][N] committed deformation gradient          */
  RVE_FIELD_P = 1,         /* [9][N] first Piola-Kirchhoff stress             */
  RVE_FIELD_SIGMA = 2,     /* [9][N] Cauchy stress P F^T / det F              */
  RVE_FIELD_FPINV = 3,     /* [9][N] inverse plastic deformation gradient    */
  RVE_FIELD_CHI = 4,       /* [12][N] back stresses (MPa)                     */
  RVE_FIELD_DGAMMA = 5,    /* [12][N] slip increments of the last increment  */
  RVE_FIELD_PCYC = 6,      /* [N] accumulated plastic slip, sum sqrt(2/3 dLp:dLp) */
  RVE_FIELD_PCYC_LIT = 7,  /* [N] sum dLp:dLp / dt (Eq. 23 integrand)         */
  RVE_FIELD_WCYC = 8,      /* [12][N] plastic work per system (Eq. 24), MPa   */
  RVE_FIELD_STATEV = 9,    /* [nstatev][N] committed user-material state      */
  RVE_FIELD_COUNT = 10
};

/* Bit of field id f in the mask of rve_get_fields / rve_batch_get_fields. */
#define RVE_FIELD_BIT(f) (1u << (f))

/* Copies the committed fields selected by mask (RVE_FIELD_BIT of each field
   id; float64, layouts above) into dst (host, or device memory when
   dst_on_device != 0), in increasing field-id order, each field directly
   after the previous one.  dst_bytes must be at least the sum of the
   selected fields' sizes (checked before anything is copied).  Errors:
   RVE_EINVAL (empty mask, unknown bits, NULL or small dst), RVE_ESTATE
   (RVE_FIELD_STATEV without a user material; crystal fields with one). */
rve_status rve_get_fields(rve_t h, uint32_t mask, void* dst, size_t dst_bytes,
                          int32_t dst_on_device);

/* Macro state: F_bar (9), P_bar (9), sigma_bar (9), t, increments. */
rve_status rve_get_macro(rve_t h, double out[29]);

/* ---- non-local fatigue indicators (Sec. 3.3, Eqs. 25-26) ----------------
   Averages of the committed indicator fields over integration volumes and
   their maxima over the RVE:
   * Eq. 25: the grain average of P_cyc over every crystal grain (a label of
     law 0 with at least one voxel); its maximum P_cyc^g.  Both P_cyc
     fields (RVE_FIELD_PCYC and the literal RVE_FIELD_PCYC_LIT) are
     averaged.
   * Eq. 26: every crystal grain is cut, for each of its four {111} slip
     planes, into bands of width band_width (length units of the cell
     lengths L) parallel to the plane; a band's value is the largest, over
     the plane's three slip systems a, of the band average of W_cyc^a; the
     maximum over all bands is W_cyc^b.
   Band geometry: voxel centres at ((i + 1/2) L_d / n); the grain's
   reference point is the centre of its voxel of lowest index; a voxel's
   offset d from it is the periodic minimal image (grains are taken to span
   less than half the cell per axis); band index j = floor(d.n / w + 1/2)
   with n the sample-frame unit normal of the plane (slip systems 3p..3p+2
   lie on plane p).  The band lists are built on the host when a width is
   first used and kept until the width or the microstructure changes; the
   averages and maxima run on the device in a fixed order (bitwise
   reproducible).  The first index wins among equal maxima. */
typedef struct {
  double band_width;       /* the width used                                */
  int32_t grains;          /* crystal grains with at least one voxel        */
  int32_t pcyc_label;      /* label of P_cyc^g (-1: no crystal grain)       */
  double pcyc_g;           /* Eq. 25 on RVE_FIELD_PCYC                      */
  double pcyc_lit_g;       /* Eq. 25 on RVE_FIELD_PCYC_LIT                  */
  int32_t pcyc_lit_label;  /* label of pcyc_lit_g                           */
  int32_t wcyc_label;      /* grain of the band of W_cyc^b (-1: no band)    */
  int64_t bands;           /* bands with at least one voxel                 */
  double wcyc_b;           /* Eq. 26                                        */
  int64_t wcyc_band;       /* index of that band in the band list           */
  int32_t wcyc_plane;      /* its slip plane, 0..3                          */
  int32_t wcyc_j;          /* its band index j                              */
  int32_t wcyc_system;     /* slip system of its value, 0..11               */
  int32_t wcyc_voxels;     /* voxels in that band                           */
} rve_nonlocal_fips;

/* Fills *out for the committed indicator fields.  Optional host outputs
   (NULL to skip): grain_pcyc[labels], grain_pcyc_lit[labels] per label
   (0 for labels that are not crystal grains; labels must equal the G of
   rve_set_microstructure); band_wcyc[band_cap] band values and
   band_desc[band_cap][5] (label, plane, j, system of the value, voxels),
   bands in (label, plane, j) order.  Call with NULL arrays first to learn
   out->bands.  Errors: RVE_EINVAL (band_width not finite or <= 0, labels
   mismatch, band_cap < bands: *out is filled first), RVE_ESTATE (no
   crystal microstructure). */
rve_status rve_get_nonlocal_fips(rve_t h, double band_width,
                                 rve_nonlocal_fips* out, double* grain_pcyc,
                                 double* grain_pcyc_lit, int32_t labels,
                                 double* band_wcyc, int32_t* band_desc,
                                 int64_t band_cap);

/* Checkpoint: the committed state (F, Fp^-1, chi, dgamma, indicators, macro
   state, counters; user-material state variables) as an opaque
   little-endian blob.  rve_state_size gives
   the byte count; rve_set_state restores a blob from the same grid. */
rve_status rve_state_size(rve_t h, size_t* bytes);
rve_status rve_get_state(rve_t h, void* dst, size_t bytes);
rve_status rve_set_state(rve_t h, const void* src, size_t bytes);

const char* rve_last_error(rve_t h);

/* ---- test hooks (same conventions) ---------------------------------------
   rve_debug_apply_G: out = G(in) (Sec. 2.1, Eq. 11) for a [9][N] float64
   field, in the given precision (RVE_PREC_FP64: FP64 passes; RVE_PREC_MIXED:
   input rounded to FP32, FP32 passes, output widened).  Host pointers.
   rve_debug_constitutive: evaluates the point law (Sec. 2.1, Eq. 2; Eq. 13
   tangent) at F[9][N] with the committed internal variables and time step dt,
   writing P[9][N], K[81][N] (component 9*(3i+j) + (3k+l) = dP_ij/dF_kl) and
   the trial slips dg[12][N]; returns the failed-voxel count in *fails.  K is
   the tangent as the handle's solver forms it: in FP64, or in mixed mode
   the FP32 tangent (FP32 linear algebra at the FP64 state), widened.
   rve_debug_set_field: overwrites one committed field (F, FPINV, CHI, PCYC,
   PCYC_LIT or WCYC) from host memory, e.g. to inject a failure or given
   indicator fields. */
rve_status rve_debug_apply_G(rve_t h, const double* in, double* out,
                             int32_t precision);

/* For callers that cannot allocate device memory (code under stream or
   graph capture, tight serving loops, harnesses that forbid hipMalloc):
   out = G(in) (Sec. 2.1, Eq. 11) in FP64, the computation of
   rve_debug_apply_G(..., RVE_PREC_FP64) without a handle and without any
   allocation.  The spectrum, FFT twiddles, wave vectors and per-block
   partial sums live in one static device array of RVE_NOALLOC_SCRATCH_BYTES
   per GPU, which each GPU the library runs on holds until the process ends.
   n: voxels per axis of a cubic grid, one of 16, 24, 32, 40, 48, 64 (at most
   RVE_NOALLOC_MAX_N); L[3]: cell edge lengths (host); projection: RVE_PROJ_*;
   in, out: [9][n^3] float64 fields in device memory of the current device,
   layout of the fields above, owned by the caller, not aliased; stream:
   hipStream_t (NULL = default stream).  The work is enqueued on stream and
   the call returns without synchronizing.  Every call on one GPU uses that
   GPU's array (nothing needs to start at zero: each call writes every entry
   it reads), so calls that overlap in time on one GPU (other streams or
   threads) race.  Errors (nothing enqueued): RVE_EINVAL (n unsupported or
   above the maximum, bad L or projection, NULL or aliased fields),
   RVE_EDEVICE (HIP error); rve_last_error(NULL) describes them. */
#define RVE_NOALLOC_MAX_N 64
#define RVE_NOALLOC_SCRATCH_BYTES 18881536
rve_status rve_apply_G_noalloc(int32_t n, const double L[3],
                               int32_t projection, const double* in,
                               double* out, void* stream);
rve_status rve_debug_constitutive(rve_t h, const double* F, double dt,
                                  double* P, double* K, double* dg,
                                  int32_t* fails);
rve_status rve_debug_set_field(rve_t h, int32_t field, const double* src,
                               size_t bytes);

/* rve_bench_kernels: average duration in milliseconds of each hot-path
   kernel over `reps` launches, timed with HIP events on the handle's
   stream, using the launch configuration and buffers of the last increment
   (needs at least one committed increment).  ms_out[count], count <= 8,
   indexed by kernel class:
     0 matvec pass A (forward z/y FFTs of K:p; publishes the CG step
       alpha = r.r / p.(K:p), equal to r.r / p.G(K:p) since p lies in the
       range of the orthogonal projection G),
     1 pass B (x FFTs and the projection of Sec. 2.2),
     2 pass C (inverse y/z FFTs, r -= alpha G(K:p) and the new r.r),
     3 unused (the CG vector update rides on classes 2 and 7; reported
       as 0),
     4 FP64 return mapping (Sec. 3.2, Eq. 22),
     5 tangent (Eq. 13),
     6 FP64 residual G(P) (Eq. 11; three kernels),
     7 CG direction, the previous iteration's x += alpha p and K:p
       (Eqs. 15-16).
   Only scratch buffers are written; the committed state is untouched. */
rve_status rve_bench_kernels(rve_t h, int32_t reps, double* ms_out,
                             int32_t count);

/* Live kernel timing.  With bit k of mask set, every launch of kernel class
   k made by the solver's own iteration (classes as for rve_bench_kernels;
   CG launches inside captured graphs included) is bracketed by a pair of
   HIP events on the handle's stream; the elapsed times are summed after
   each synchronisation of that stream.  Changing the mask re-captures the
   CG graph.  rve_get_kernel_timing copies the summed milliseconds and the
   launch counts of classes [0, count) (count <= 8; either pointer may be
   NULL) and zeroes them when reset != 0.  Launches whose RVE has already
   converged (the tail of a CG chunk) are counted like any other. */
rve_status rve_set_kernel_timing(rve_t h, uint32_t mask);
rve_status rve_get_kernel_timing(rve_t h, double* ms_total, int64_t* launches,
                                 int32_t count, int32_t reset);
/* Times only one direct launch in every `stride` (1 to 1024; 1, the
   default, times every launch) of each CG-iteration class (0-3 and 7,
   counted per class from this call), so that the events cost little of a
   timed solve; the other classes and graph-replayed chunks are timed at
   every launch.  rve_get_kernel_timing then reports the timed launches
   only.  RVE_EINVAL for a stride out of range. */
rve_status rve_set_kernel_timing_stride(rve_t h, int32_t stride);
/* Every direct launch of each timed class [0, count) since the last reset,
   timed or skipped by the stride (graph replays not included); zeroes these
   counts and the timing sums when reset != 0.  RVE_EINVAL for count out of
   [0, 8]. */
rve_status rve_get_kernel_launches(rve_t h, int64_t* launches, int32_t count,
                                   int32_t reset);
/* Work of the return mappings timed while bit 4 (return mapping) is set:
   out[0] local Newton steps and out[1] residual evaluations summed over
   crystal voxels and launches, out[2] crystal and out[3] particle voxel
   visits (Sec. 3.2, Eq. 22 integrated per voxel).  Zeroed when reset != 0
   and whenever bit 4 is switched on. */
rve_status rve_get_return_map_counts(rve_t h, int64_t out[4], int32_t reset);

/* Schedule of the CG matvec G(K : p) (Sec. 2.1, Eqs. 15-16): cpb
   components of the tensor field per slab block in the z/y-transform
   passes (1 or 3), tt kz columns per block in the x-transform and
   projection pass (4, 8 or 16), and fused (0 or 1): whether the CG
   direction step and K : p run in their own streaming kernel (0) or inside
   the first transform pass (1), which then forms p = r + beta p_old for
   all nine components of each voxel of its slab and transforms its own
   rows of K : p.  Both give the same CG up to the order of the FP64 sum of
   p . (K:p).  By default (0, 0, -) the handle times every valid schedule
   once on its own buffers at the first CG solve and keeps the fastest.
   rve_set_fft_schedule forces one (or (0, 0, -) to tune again);
   RVE_EINVAL when the schedule does not exist for the grid and precision or
   fused is not 0 or 1.  rve_get_fft_schedule writes (cpb, tt, fused) in use
   (zeros before the first solve) and, in *ms (nullable), the tuned matvec
   time in milliseconds (0 when forced). */
rve_status rve_set_fft_schedule(rve_t h, int32_t cpb, int32_t tt,
                                int32_t fused);
rve_status rve_get_fft_schedule(rve_t h, int32_t out[3], double* ms);
/* Tunes the schedule now (as the first CG solve would) on the handle's
   buffers, so that a timed run does not include the tuning; the vectors it
   touches are rewritten by the next solve.  Replaces a forced schedule. */
rve_status rve_tune_fft_schedule(rve_t h);

/* ---- learned warm start -------------------------------------------------
   A small network predicts the fluctuation increment of the next load
   increment from the committed state, so that the Newton iteration of
   Sec. 2.1 (Eqs. 12-16) starts nearer to equilibrium.  It predicts, per
   |dF_bar|, the correction to the extrapolation c dFt_prev (the last
   converged fluctuation increment scaled by the load ratio c = dF_bar :
   dF_bar_prev / |dF_bar_prev|^2, warm_start = 3 on its own); the sum is
   projected by G (Sec. 2.1, Eq. 11) and kept only when its FP64
   equilibrium residual is smaller than the homogeneous predictor's; Newton
   then runs to the same tolerance either way.
   Architecture: four 3x3x3 convolutions with periodic padding, 40 -> 32 ->
   32 -> 32 -> 9 channels, ReLU after the first three; bf16 weights and
   activations, FP32 accumulation on the matrix cores.  Grids need n % 16 == 0.
   Parameters (float32, host order): for each layer W[27][cin][cout] (tap
   t = (dx+1)*9 + (dy+1)*3 + (dz+1)) followed by b[cout].
   Device buffers (caller-owned, dst/src on the device):
     features  uint16 bf16 [N][48]  (channel list in the design notes)
     targets   float [N][16] (first 9: the committed increment's fluctuation
               increment / |dFbar| less cos times the one before it / its
               |dFbar|, cos the cosine between the two dFbar: the part the
               extrapolation misses)
     outputs   float [N][16]
   rve_ws_train_step: one Adam step (lr, betas 0.9/0.999, eps 1e-8) on the
   mean squared error over the 9 real output channels of one sample; *loss
   receives the loss before the step; grad_host (nullable) the FP32
   gradient in parameter order.
   rve_attach_warm_start: the handle uses the network when its config has
   warm_start = 1 or 2 (pass NULL to detach; detach before destroying the
   network).  rve_ws_features: input of the increment to F_bar_new from the
   committed state.  rve_ws_target: target of the last committed increment.
   Errors: RVE_EINVAL (bad sizes, n % 16 != 0), RVE_ESTATE (no increment
   yet for rve_ws_target), RVE_ENOMEM. */
typedef struct rve_ws_s* rve_ws_t;
typedef struct {
  void* stream;          /* hipStream_t used by training and rve_ws_forward */
  rve_alloc_fn dev_alloc;
  rve_free_fn dev_free;
  void* alloc_ctx;
} rve_ws_config;

rve_status rve_ws_create(const rve_ws_config* cfg, rve_ws_t* out);
rve_status rve_ws_destroy(rve_ws_t w);
rve_status rve_ws_param_count(rve_ws_t w, int64_t* count);
rve_status rve_ws_set_params(rve_ws_t w, const float* params, int64_t count);
rve_status rve_ws_get_params(rve_ws_t w, float* params, int64_t count);
rve_status rve_ws_forward(rve_ws_t w, const uint16_t* X, int32_t n, float* Y);
rve_status rve_ws_train_step(rve_ws_t w, const uint16_t* X, const float* T,
                             int32_t n, float lr, double* loss,
                             float* grad_host);
/* The loss of one sample without a training step (parameters and optimiser
   state untouched). */
rve_status rve_ws_loss(rve_ws_t w, const uint16_t* X, const float* T,
                       int32_t n, double* loss);
const char* rve_ws_last_error(rve_ws_t w);
rve_status rve_attach_warm_start(rve_t h, rve_ws_t w);
rve_status rve_ws_features(rve_t h, const double F_bar_new[9], uint16_t* X);
rve_status rve_ws_target(rve_t h, float* T);

/* ---- user materials of commercial FE codes (Appendix A) -----------------
   rve_umat_bridge converts, voxel by voxel, the output of a finite-strain
   user material written for a commercial FE code -- the Cauchy stress and
   the tangent of the Jaumann rate of the Kirchhoff stress (Appendix A,
   Eq. A.2), both in the component order 11, 22, 33, 12, 13, 23 with
   engineering shear strains -- into the first Piola-Kirchhoff stress
   P = J sigma F^-T (Eq. A.1) and the tangent K = dP/dF of the FFT solver
   (Eq. A.16).  All arrays are caller-owned device memory, float64,
   structure-of-arrays over n voxels: F [9][n] (row-major 3x3 per voxel),
   sigma [6][n], ddsdde [36][n] (6x6 row-major per voxel: entry (I, J) at
   (6 I + J) n + v), outputs P [9][n] and K [81][n] (component
   9 (3i+j) + (3k+l) = dP_ij/dF_kl).  The work is enqueued on stream
   (hipStream_t, NULL = default stream); the call returns after enqueueing.
   n = 0 does nothing.  Errors: RVE_EINVAL (null pointer, n < 0),
   RVE_EDEVICE (launch failure); rve_last_error(NULL) describes them. */
rve_status rve_umat_bridge(const double* F, const double* sigma,
                           const double* ddsdde, int64_t n, double* P,
                           double* K, void* stream);

/* ---- batches of RVEs ------------------------------------------------------
   count independent RVEs (1 <= count <= 255), each with its own cubic grid
   n[b] in {16, 24, 32, 40, 48, 64}, microstructure and committed state,
   solved together: each pass of the Newton-CG iteration (Sec. 2.1,
   Eqs. 11-16) runs as one kernel launch over the whole batch, and each RVE
   keeps its own Newton and CG stopping tests, so an RVE that has converged
   does no further work in that increment.  Results per RVE are those of a
   single handle with the same configuration up to the summation order of
   the reductions.
   cfg: projection, precision, tolerances, stream and allocator as for
   rve_create; cfg.n is ignored (grids come from n[count]); cfg.L is each
   RVE's cell; warm_start must be 0.  cfg.use_graph selects how an
   increment runs: 0 = one launch per pass for the whole batch, the Newton
   decisions and a check per cg_chunk CG iterations on the host; 1 = the
   Newton decisions on the device, each linear solve of all RVEs in one
   persistent launch (grid barriers between the passes of a CG iteration;
   the launch stops when every RVE's CG is done), the predictor and the
   first four Newton iterations replayed from one captured graph, further
   iterations launched one at a time.  Both give the same results bit for
   bit.  All RVEs share the material
   constants: rve_batch_set_microstructure rejects params that differ from
   those of an earlier call.  Voxel layouts, fields and info records are those
   of the single-RVE calls, per RVE b.
   rve_batch_apply_macro_strain_increment: F_bar_new[count][9] (RVE b's
   macro gradient at F_bar_new + 9 b), one dt; info[count] (nullable)
   receives each RVE's record.  Every RVE that converges commits, the others
   keep their committed state; returns RVE_OK when all converged, else the
   status of the first RVE that did not.  Errors as for the single-RVE
   calls; RVE_EINVAL for b out of range. */
typedef struct rve_batch_s* rve_batch_t;
rve_status rve_batch_create(const rve_config* cfg, int32_t count,
                            const int32_t* n, rve_batch_t* out);
rve_status rve_batch_destroy(rve_batch_t h);
rve_status rve_batch_set_microstructure(rve_batch_t h, int32_t b,
                                        const int32_t* phase, int32_t G,
                                        const double* quat, const int32_t* law,
                                        const double* params, int32_t nparams);
rve_status rve_batch_apply_macro_strain_increment(rve_batch_t h,
                                                  const double* F_bar_new,
                                                  double dt,
                                                  rve_increment_info* info);
rve_status rve_batch_reset_fips(rve_batch_t h);
rve_status rve_batch_get_fields(rve_batch_t h, int32_t b, uint32_t mask,
                                void* dst, size_t dst_bytes,
                                int32_t dst_on_device);
rve_status rve_batch_get_macro(rve_batch_t h, int32_t b, double out[29]);
/* Test hook: out = G(in) (Sec. 2.1, Eq. 11) for every RVE of the batch at
   once, through the batched pass kernels in the batch's precision (FP64, or
   in mixed mode the FP32 passes of the CG on the input rounded to FP32, the
   output widened).  in / out: host float64, RVE after RVE, each RVE b a
   [9][n_b^3] block (layout of the single-RVE fields).  Errors: RVE_EINVAL
   (NULL pointers). */
rve_status rve_batch_debug_apply_G(rve_batch_t h, const double* in,
                                   double* out);
/* Per-grid-edge schedule of the batched CG matvec (Sec. 2.1, Eqs. 15-16):
   cpb components per slab block (1 or 3) and tt kz columns per pencil block
   (4, 8 or 16), as for a single RVE (the direction step is always part of
   the first pass in a batch).  Unless forced, every edge of the batch is
   tuned at the first increment (or by rve_batch_tune_fft_schedule): each
   valid candidate times one matvec of that edge's RVEs alone through the
   batched passes, and the fastest is kept.  rve_batch_set_fft_schedule
   forces edge's schedule, or with (0, 0) tunes it again at the next
   increment; rve_batch_get_fft_schedule writes edge's (cpb, tt) and in *ms
   (nullable) the tuned matvec time of its RVEs in milliseconds (0 when
   forced or not tuned yet).  Errors: RVE_EINVAL (no RVE of that edge in
   the batch, a schedule that does not exist for it, NULL out). */
rve_status rve_batch_tune_fft_schedule(rve_batch_t h);
rve_status rve_batch_set_fft_schedule(rve_batch_t h, int32_t edge,
                                      int32_t cpb, int32_t tt);
rve_status rve_batch_get_fft_schedule(rve_batch_t h, int32_t edge,
                                      int32_t out[2], double* ms);

/* Host only (no device work, no GPU needed): the band lists that
   rve_get_nonlocal_fips uses, for a microstructure of n^3 voxels (phase,
   G, quat, law as in rve_set_microstructure), cell lengths L[3] and a band
   width.  *bands receives the number of bands and *entries the total
   length of their voxel lists.  When band_desc / band_vox are not NULL they
   receive, for bands in (label, plane, j) order, [bands][4] = (label,
   plane, j, voxels) and the concatenated ascending voxel indices; they
   must hold cap_bands and cap_entries items (call once with NULL arrays to
   learn the counts).  Errors: RVE_EINVAL (bad sizes, labels, quaternions,
   width, or capacities below the counts). */
rve_status rve_fip_band_lists(int32_t n, const double L[3],
                              const int32_t* phase, int32_t G,
                              const double* quat, const int32_t* law,
                              double band_width, int64_t* bands,
                              int64_t* entries, int32_t* band_desc,
                              int32_t* band_vox, int64_t cap_bands,
                              int64_t cap_entries);

/* rve_get_nonlocal_fips for RVE b of a batch (same arguments and rules;
   labels is that RVE's G). */
rve_status rve_batch_get_nonlocal_fips(rve_batch_t h, int32_t b,
                                       double band_width,
                                       rve_nonlocal_fips* out,
                                       double* grain_pcyc,
                                       double* grain_pcyc_lit, int32_t labels,
                                       double* band_wcyc, int32_t* band_desc,
                                       int64_t band_cap);
const char* rve_batch_last_error(rve_batch_t h);

#ifdef __cplusplus
}
#endif

#endif /* RVE_H */
