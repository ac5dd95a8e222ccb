/* fornax_m1.h -- C interface of the MI355X (gfx950) multigroup M1 radiation-moment step.
 *
 * The library advances the group radiation energy density E_g and flux F_{g,k} of every zone
 * of a static medium by one step of the semi-explicit method of Skinner, Dolence, Burrows,
 * Radice & Vartanyan, "FORNAX: a Flexible Code for Multiphysics Astrophysical Simulations"
 * (ApJS 2019):
 *   - radiation moment equations with v = 0 (Formulation of the Equations, eq:rad_system,
 *     interaction terms eq:rad_mom_src), group-integrated (eq:rad_system2);
 *   - finite-volume update (eq:finite_vol) with linear reconstruction in the volume coordinate
 *     (Reconstruction, eq:recon_constraints with n = 1), M1 closure, HLL fluxes with the
 *     diffusion correction of the energy flux (Riemann Solvers, eq:hll, eq:epsilon) and the
 *     geometric source terms of the covariant form (Appendix: covariant form, connection
 *     coefficients, eq:angmom, eq:grad2P);
 *   - operator-split backward-Euler interaction update (Interaction Terms, eq:be_update and
 *     the flux update that follows it), Algorithmic Steps 1, 3 and 4 with matter held fixed,
 *     or with the matter temperature solved for (the outer update; photons, ideal gas).
 *
 * Conventions
 *   - Every array pointer is a DEVICE pointer (hipMalloc'd or a torch CUDA tensor's data).
 *     Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL = null stream).
 *     No call synchronises the host.
 *   - Zone-group layout: structure of arrays, one array per component, element
 *     ((k * n[1] + j) * n[0] + i) * ngroups + g  (group innermost, x fastest among zones).
 *   - Flux components are covariant, F_k = h_k F^_k with h_k the scale factors; on Cartesian
 *     grids they equal the physical components.
 *   - Element type: double for FORNAX_FP64 contexts, float for FORNAX_MIXED contexts, for
 *     states, coefficients and face fluxes.  Diagnostics and inflow values are always double.
 *   - Errors are negative return codes, checked before any launch; the arguments are not
 *     modified when a call fails.  Numerical trouble (non-realizable or non-positive states)
 *     is not an error: it is counted in the diagnostics.
 */
#ifndef FORNAX_M1_H
#define FORNAX_M1_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FORNAX_OK = 0,
  FORNAX_EINVAL = -1,       /* null/misaligned pointer, bad shape, bad option combination */
  FORNAX_ECFL = -2,         /* dt above fornax_m1_max_dt(ctx, 1.0) */
  FORNAX_EDEVICE = -3,      /* HIP error (launch, copy, no device) */
  FORNAX_ENOMEM = -4,       /* device allocation failed */
  FORNAX_EUNSUPPORTED = -5, /* option not implemented for this configuration */
  FORNAX_ESCRATCH = -6      /* fornax_m1_step_noalloc: the step's scratch exceeds the static array */
};

/* Size of the static device array that fornax_m1_step_noalloc keeps its scratch in (one per
 * device, held until the process ends). */
#define FORNAX_M1_NOALLOC_SCRATCH_BYTES (16u << 20)

/* Coordinates.  SPHERICAL_LOGR: x1 = ln r, x2 = theta, x3 = phi (metric of the Appendix,
 * general spherical metric, with r = e^{x1}, theta = x2). */
enum { FORNAX_CARTESIAN = 0, FORNAX_SPHERICAL_LOGR = 1 };

/* Boundary conditions (Implementation of the dendritic grid, Boundary Conditions):
 * OUTFLOW copies the edge zone; PERIODIC wraps; REFLECT mirrors and flips the normal flux;
 * INFLOW fills the ghosts with prescribed (E, physical F) per group (x1 only; on other axes
 * fornax_m1_create returns FORNAX_EUNSUPPORTED); AXIS is the polar-axis
 * copy across theta = 0 or pi with a shift of n[2]/2 zones in phi and sign flips of the theta
 * and phi flux components (spherical x2 only, n[2] even or 1). */
enum { FORNAX_BC_OUTFLOW = 0, FORNAX_BC_PERIODIC = 1, FORNAX_BC_REFLECT = 2, FORNAX_BC_INFLOW = 3,
       FORNAX_BC_AXIS = 4 };

/* Precision.  FP64: every operation in double.  MIXED: float storage, reconstruction, flux and
 * divergence in float; the closure in double where f >= f_fp64; the interaction update and
 * all accumulations (energy, dE_matter) in double. */
enum { FORNAX_FP64 = 0, FORNAX_MIXED = 1 };

/* Reconstruction (Reconstruction subsection).  MINMOD (the method's default here), MC: linear
 * profiles in the volume coordinate with limited slopes (eq:recon_constraints, n = 1); NONE:
 * piecewise constant; PPM: the paper's piecewise-parabolic reconstruction (n = 2): constant
 * where a zone's average is not between its neighbours', else the parabola with the three zones' averages
 * (eq:recon_system1), each face state reset where that parabola turns between the zone's and
 * its neighbour's centres (monotone there, zero slope at the neighbour's centre), and the face
 * state nearer to an extremum of the parabola through both face states and the average
 * (eq:recon_system2) reset to give that parabola zero slope at its face; in the volume
 * coordinate on spherical grids (moments of each zone from the volume element).  PPM is not
 * available in fornax_m1_adjoint. */
enum { FORNAX_LIMITER_MINMOD = 0, FORNAX_LIMITER_MC = 1, FORNAX_LIMITER_NONE = 2, FORNAX_LIMITER_PPM = 3 };
enum { FORNAX_CLOSURE_M1 = 0, FORNAX_CLOSURE_EDDINGTON = 1 };

/* Explicit integrator of the transport (Numerical Discretization: the paper integrates the
 * explicit terms with Shu & Osher's second-order TVD Runge-Kutta scheme; Algorithmic Steps
 * describe its first-order case, the Euler push).  EULER: U^- = U^n + dt L(U^n).  SSPRK2:
 * U* = U^n + dt L(U^n), U^- = (U^n + U* + dt L(U*)) / 2 (two launches of the step kernel,
 * U* in context scratch).  Either way the implicit interaction update then maps U^- to
 * U^{n+1} once per step, and dE_matter is taken against that U^-. */
enum { FORNAX_EULER = 0, FORNAX_SSPRK2 = 1 };

/* Wavespeed bounds of the HLL fluxes (Riemann Solvers subsection, eq:hll takes the speeds S_L,
 * S_R of the fastest waves moving left and right, with no formula for them).  LIGHT: S_L = -c,
 * S_R = +c, the bound of every M1 characteristic speed (the method's default here).  M1:
 * HLLE bounds S_L = min(0, l-(L), l-(R)), S_R = max(0, l+(L), l+(R)) from the eigenvalues of the
 * flux Jacobian of the one-dimensional M1 system at each face state, taken with the state's
 * normal reduced flux f = F^_d / (cE): l-+ = (c / s)(f -+ 2 (s - 1) / sqrt(3)),
 * s = sqrt(4 - 3 f^2) (+-c/sqrt(3) at f = 0, both c f at |f| = 1; +-c/sqrt(3) for the
 * Eddington closure; +-c where E <= 0).  Less numerical diffusion where the radiation is close
 * to isotropic.  fornax_m1_adjoint supports LIGHT only. */
enum { FORNAX_WAVESPEED_LIGHT = 0, FORNAX_WAVESPEED_M1 = 1 };

typedef struct {
  int32_t ndim;             /* active directions, 1..3 */
  int32_t n[3];             /* zones per direction; n[d] = 1 for d >= ndim */
  int32_t ngroups;          /* energy groups, >= 1 */
  int32_t coord;            /* FORNAX_CARTESIAN or FORNAX_SPHERICAL_LOGR */
  double lo[3], hi[3];      /* coordinate extents in x-space (uniform in each x^d) */
  int32_t bc_lo[3], bc_hi[3];
  int32_t limiter;          /* FORNAX_LIMITER_* (minmod is the method's default) */
  int32_t closure;          /* FORNAX_CLOSURE_* */
  int32_t precision;        /* FORNAX_FP64 or FORNAX_MIXED */
  double c;                 /* (reduced) speed of light, > 0 */
  double f_fp64;            /* MIXED only: closure evaluated in double where f >= f_fp64 */
  int32_t integrator;       /* FORNAX_EULER (the configurations' default) or FORNAX_SSPRK2 */
  int32_t wavespeed;        /* FORNAX_WAVESPEED_LIGHT (default) or FORNAX_WAVESPEED_M1 */
} fornax_m1_desc;

typedef struct fornax_m1_ctx fornax_m1_ctx;   /* opaque; owns geometry tables and scratch */

typedef struct { void *E, *F[3]; } fornax_m1_state;               /* F[k] unused for k >= ndim */
typedef struct { const void *kappa, *sigma, *B; } fornax_m1_coeffs; /* absorption, scattering,
                                                                       emission: j = c kappa B */
typedef struct {
  double *energy_total;     /* [1]  sum_i V_i sum_g E_g^{n+1} (coordinate volume V_i) */
  double *dE_matter;        /* [nzones] -sum_g (E_g^{n+1} - E_g^-): energy given to matter */
  double *max_f;            /* [1]  max |F^|/(c E) over zone-groups with E > 0 */
  int32_t *n_unrealizable;  /* [1]  #zone-groups with |F^| > c E (1 + 8u), u = unit roundoff */
  int32_t *n_nonpositive;   /* [1]  #zone-groups with E <= 0 */
} fornax_m1_diag;           /* any member may be NULL; the whole pointer may be NULL */

/* Build a context: validates the description, builds the geometry tables on the host in
 * double precision (volumes, face areas, volume centroids, scale factors and volume-averaged
 * connection coefficients with the paper's overrides) and uploads them to the current HIP
 * device.  Returns FORNAX_OK and *out, or an error with *out = NULL. */
int fornax_m1_create(const fornax_m1_desc *desc, fornax_m1_ctx **out);
int fornax_m1_destroy(fornax_m1_ctx *ctx);

/* Largest time step for a CFL number: cfl / max_i sum_d c / (h_d Delta x^d)_i (the light
 * crossing time of a zone sets the step, General Description).  Host only; < 0 on error. */
double fornax_m1_max_dt(const fornax_m1_ctx *ctx, double cfl);

/* One step U^n -> U^{n+1}: explicit transport (Algorithmic Steps, step 1, v = 0) followed by
 * the implicit interaction update (steps 3 and 4, matter fixed).  `in` and `out` must not
 * alias.  `inflow` is a device array [ngroups][1+ndim] of doubles (E and physical flux of the
 * inflow ghosts) required iff a boundary is FORNAX_BC_INFLOW, else NULL.  `diag` may be NULL;
 * its totals are summed on the device from per-block partials in a fixed order (deterministic)
 * in the context's scratch, so calls on one context must not overlap (as for every call).
 * Errors: EINVAL, ECFL (dt <= 0 or dt > max_dt(1)), EDEVICE. */
int fornax_m1_step(fornax_m1_ctx *ctx, const fornax_m1_state *in, fornax_m1_state *out,
                   const fornax_m1_coeffs *cf, const double *inflow, double dt,
                   const fornax_m1_diag *diag, void *stream);

/* fornax_m1_step for the callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and results,
 * with every scratch buffer of the step -- the per-block diagnostics partials, the dE_matter
 * partials of tiles that split a zone's groups, the SSP-RK2 stage -- in one static device array
 * of FORNAX_M1_NOALLOC_SCRATCH_BYTES per device instead of the context's scratch.  Calls no
 * allocating routine.  Every call on a device shares that device's array (it keeps the last
 * call's contents; every launch writes the parts it reads, so nothing needs clearing), so calls
 * that overlap on one device -- on any contexts or streams -- race.  FORNAX_ESCRATCH,
 * before any launch, when the scratch of this grid and these options exceeds the array (the
 * diagnostics partials take 24 bytes per block; dE_matter on tiles that split groups takes 8
 * bytes per zone and group block; SSP-RK2 takes one state).  Otherwise the arguments, errors and
 * results of fornax_m1_step. */
int fornax_m1_step_noalloc(fornax_m1_ctx *ctx, const fornax_m1_state *in, fornax_m1_state *out,
                           const fornax_m1_coeffs *cf, const double *inflow, double dt,
                           const fornax_m1_diag *diag, void *stream);

/* Numerical face fluxes of U (eq:hll, eq:epsilon) per direction d < ndim, as coordinate flux
 * densities (the face area is not applied): face_flux[d] is an array
 * [faces_d][ngroups][1+ndim], faces_d running over (k, j, i) with the d index in 0..n[d]
 * (face i-1/2 of zone i) and x fastest; component 0 is the energy flux, 1+k the flux of F_k.
 * Faces of zero area (polar axis) hold 0. */
int fornax_m1_flux(fornax_m1_ctx *ctx, const fornax_m1_state *in, const fornax_m1_coeffs *cf,
                   const double *inflow, void *face_flux[3], void *stream);

/* Implicit interaction update alone, in place (eq:be_update with j = c kappa B, and
 * F <- F / (1 + c dt (kappa + sigma))).  dE_matter (nullable): -sum_g (E^{n+1} - E) per zone. */
int fornax_m1_source(fornax_m1_ctx *ctx, fornax_m1_state *inout, const fornax_m1_coeffs *cf,
                     double dt, double *dE_matter, void *stream);

/* Adjoint of one step (vector-Jacobian product), for gradients of a loss of U^N:
 *   lam_n = (dU^{n+1}/dU^n)^T lam_np1,   dkappa_accum += (dU^{n+1}/dkappa)^T lam_np1.
 * Un is the state the step started from.  Unp1 (required) is the state fornax_m1_step produced
 * from Un with the same coefficients, inflow and dt (the opacity derivative of the interaction
 * update needs U^{n+1}); a caller without it runs fornax_m1_step first.  A Unp1 that is not
 * that step's result gives a wrong dkappa, with no error.  The call allocates nothing.
 * lam_np1, lam_n are states of the context's type (lam_n must not alias lam_np1, Un or Unp1);
 * dkappa_accum is a zone-group array of the context's type, accumulated into.  Non-smooth points (minmod, realizability fallback,
 * epsilon kink, f clamp) take the derivative of the branch the forward step takes.  Same
 * layout, error and stream rules as fornax_m1_step; FORNAX_EUNSUPPORTED for spherical grids
 * and for 3-D; EINVAL when Unp1 is NULL. */
int fornax_m1_adjoint(fornax_m1_ctx *ctx, const fornax_m1_state *Un, const fornax_m1_state *Unp1,
                      const fornax_m1_coeffs *cf, const double *inflow, double dt,
                      const fornax_m1_state *lam_np1, fornax_m1_state *lam_n, void *dkappa_accum,
                      void *stream);

/* Explicit transport alone (Algorithmic Steps, step 1 with v = 0): out = U^- = U^n + dt L(U^n)
 * (with the SSPRK2 integrator, U^- = (U^n + U* + dt L(U*)) / 2), without the interaction
 * update.  cf->B is not read and may be NULL.  Same rules and errors as fornax_m1_step. */
int fornax_m1_transport(fornax_m1_ctx *ctx, const fornax_m1_state *in, fornax_m1_state *out,
                        const fornax_m1_coeffs *cf, const double *inflow, double dt, void *stream);

/* ---- Radiation-matter energy exchange (Interaction Terms: the outer update; photons, one
 * equation for the matter temperature T) ----
 * Matter model: internal energy density u = cv T (ideal gas); absorption
 *   kappa_g(T) = kappa0 * kg[g] * T^(-1/2) * (1 - exp(-nu_c[g] / T))
 * (the frequency- and temperature-dependent opacity of the paper's multigroup pulse test, at
 * the group's frequency nu_c[g]; units with h = k_B = 1); emission j_g = c kappa_g B_g(T) with
 *   B_g(T) = a_rad T^4 (15/pi^4) int_{nu_edge[g]/T}^{nu_edge[g+1]/T} x^3/(e^x - 1) dx
 * (Kirchhoff's law with the group-integrated Planck function); scattering sigma_g per
 * zone-group, independent of T. */
typedef struct {
  int32_t ngroups;          /* must equal the context's ngroups (<= 64) */
  const double *nu_edge;    /* HOST array [ngroups + 1], increasing, >= 0; the last may be +inf */
  const double *nu_c;       /* HOST array [ngroups], > 0 */
  const double *kg;         /* HOST array [ngroups], >= 0 */
  double a_rad;             /* radiation constant, > 0 */
  double tol;               /* Newton ends when |T^{k+1} - T^k| <= tol T^{k+1} (the paper: 1e-6) */
  int32_t max_newton;       /* Newton iterations before bisection decides T (0: bisection only) */
} fornax_m1_matter_model;

typedef struct {
  const double *cv;         /* [nzones] heat capacity per volume, > 0 */
  const double *kappa0;     /* [nzones] opacity scale, >= 0 */
  double *T;                /* [nzones] matter temperature, > 0; in: T^-, out: T^{n+1} */
} fornax_m1_matter;         /* device arrays of doubles */

/* Copies the model's tables into the context (host call; synchronous with the null stream).
 * EINVAL for a bad table, EUNSUPPORTED for ngroups > 64. */
int fornax_m1_set_matter_model(fornax_m1_ctx *ctx, const fornax_m1_matter_model *model);

/* kappa_g(T) and B_g(T) of every zone-group into kappa_out and B_out (zone-group arrays of the
 * context's type), for the transport with the opacities at T^n.  EINVAL without a model. */
int fornax_m1_matter_coeffs(fornax_m1_ctx *ctx, const fornax_m1_matter *m, void *kappa_out, void *B_out,
                            void *stream);

/* The interaction update with the matter energy equation, in place, per zone (all groups of a
 * zone together): the outer solve of r(T) = cv (T - T^-) + sum_g (E_g(T) - E_g^-) = 0 by
 * Newton-Raphson from T^- (forward-difference derivative with step 1e-7 T, backtracking by
 * halving until |r| decreases, at most 10 halvings), bisection on (0, T^- + sum_g max(E_g^-, 0)
 * / cv] until the bracket is 1e-13 of its upper end when Newton fails or runs out of
 * iterations; each group's inner backward-Euler update E_g(T) = (E_g^- + dt c kappa_g B_g)
 * / (1 + c dt kappa_g) (eq:be_update) at the converged T; then F^{n+1} = F^- / (1 + c dt
 * (kappa_g(T^{n+1}) + sigma_g)).  Always computed in double (float states are read and
 * written as float).  dE_matter (nullable): u^{n+1} - u^- per zone; iters (nullable, int32):
 * Newton iterations, or -(bisection steps) where bisection decided T.  EINVAL without a model
 * or for bad pointers. */
int fornax_m1_matter_source(fornax_m1_ctx *ctx, fornax_m1_state *inout, const void *sigma,
                            const fornax_m1_matter *m, double dt, double *dE_matter, int32_t *iters,
                            void *stream);

/* ---- Velocity-dependent terms (prescribed velocity) ----
 * The comoving-frame moment equations to first order in v/c (Formulation of the Equations,
 * eq:rad_system), with the velocity given on the zone faces instead of by a hydrodynamics
 * solve.  v[d], d < ndim: DEVICE array of the context's element type holding the coordinate
 * (contravariant) components v^0..v^{ndim-1} on the d-faces, layout [ndim][faces_d] with faces_d
 * over (k, j, i), the d index in 0..n[d] (face i-1/2 of zone i), x fastest.  On spherical grids
 * v^1 = v_r / r (x1 = ln r), v^2 = v_theta / r, v^3 = v_phi / (r sin theta).  The caller owns
 * the arrays; they are read, never written. */
typedef struct { const void *v[3]; } fornax_m1_velocity;

/* Group edges in frequency for the intergroup fluxes of the velocity step: HOST array
 * [ngroups + 1], increasing, finite, nu_edge[0] >= 0 (only ratios matter), copied into the
 * context (synchronous).  EINVAL for a bad table, ENOMEM. */
int fornax_m1_set_group_edges(fornax_m1_ctx *ctx, const double *nu_edge);

/* One step U^n -> U^{n+1} with the velocity terms (Algorithmic Steps 1 to 4, Euler push, matter
 * fixed):
 *   Step 1: the transport of fornax_m1_step plus the advective fluxes (v E), (v F_k) on every
 *           face, v^d times the reconstructed state on the upwind side of the face's normal
 *           component (Riemann Solvers subsection), and in the flux rows the connection part of
 *           (v^i F_k)_{;i} and -<v^i_{;k}> F_i (eq:rad_mom2);
 *   Step 2: E_g <- E_g + dt (Phi_{g+1/2} - Phi_{g-1/2} - <v^i_{;j}> P^j_{g i}) (eq:freq_adv_system),
 *           Phi_{g-1/2} = nu_{g-1/2} (X-_{g-1} at its upper edge + X+_g at its lower edge), X-+
 *           the parts of sum_ij <v^i_{;j}> P^j_i / dnu_g with <v^i_{;j}> < 0 and >= 0, linear in
 *           nu across each group with minmod-limited slopes (zero in the first and last group),
 *           Phi = 0 at both ends of the frequency range; no intergroup term in the flux rows
 *           (no closure for the third moment);
 *   Steps 3, 4: the interaction update of fornax_m1_step on the state after Step 2.
 * <v^i_{;j}> = <v^i_{,j}> + <Gamma^i_{jk}> <v^k>, each coordinate component linear across the
 * zone (<v^k>: its value at the volume centroid).  dE_matter and the diagnostics as for
 * fornax_m1_step, against the state after Step 2.  Two launches, in place on `out` between
 * them.  Errors: EINVAL (also without group edges, or a null v[d]), ECFL, EUNSUPPORTED for the
 * SSPRK2 integrator, the PPM reconstruction, the M1 wavespeeds or ngroups > 256, EDEVICE.
 * Stable while dt |v| nu_{g+1/2} <~ dnu (frequency CFL, not checked) and |v| < c. */
int fornax_m1_step_velocity(fornax_m1_ctx *ctx, const fornax_m1_state *in, fornax_m1_state *out,
                            const fornax_m1_coeffs *cf, const double *inflow,
                            const fornax_m1_velocity *vel, double dt, const fornax_m1_diag *diag,
                            void *stream);

/* Group-summed radiation energy and flux of every zone in the laboratory frame to first order
 * in v/c: with the physical velocity v^_k = h_k <v^k> (cell-centred h, <v^k> as above),
 *   E_lab = sum_g (E_g + 2 v^ . F^_g / c^2),  F^_lab = sum_g (F^_g + v^ E_g + v^ . P^_g),
 * physical components (the transformation behind the lab-frame flux continuity at a
 * transparent shock).  E_lab [nzones], F_lab[k] [nzones] for k < ndim: device arrays of
 * doubles.  EINVAL for bad pointers. */
int fornax_m1_lab_frame(fornax_m1_ctx *ctx, const fornax_m1_state *in, const fornax_m1_velocity *vel,
                        double *E_lab, double *F_lab[3], void *stream);

/* Measurement utility (not part of the method): plain device-to-device copy of `nbytes`
 * (multiple of 16, 16-byte aligned pointers) with the library's own kernel, used to scale
 * hardware byte counters and to measure achievable HBM bandwidth. */
int fornax_m1_copy_probe(void *dst, const void *src, int64_t nbytes, void *stream);

const char *fornax_m1_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* FORNAX_M1_H */
