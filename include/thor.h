/*
 * thor.h -- C ABI of the MI355X (gfx950) HEVI dynamical-core step.
 *
 * Method: Mendonca et al. 2016, "THOR: a new and flexible global circulation
 * model to explore planetary atmospheres" (arXiv:1607.05535).  One time step
 * is the split-explicit, horizontally explicit / vertically implicit (HEVI)
 * integration of the deep non-hydrostatic Euler equations in flux form
 * (Sec. 3, Eqs. mass, mom, entropy) on a spring-dynamics-smoothed
 * icosahedral grid (Sec. 2), with fourth-order hyperdiffusion and 3D
 * divergence damping (Sec. 4) and backward-Euler Newtonian relaxation
 * (Sec. 5, Eq. im_eq_t).
 *
 * Conventions
 *   - Every function returns THOR_OK (0) or a negative THOR_E* code and never
 *     throws or longjmps across the ABI.  thor_last_error() then holds a
 *     message for the calling thread.
 *   - Argument errors are detected before anything is enqueued on the GPU.
 *   - Handles (thor_grid, thor_state) are library-owned host objects freed by
 *     the matching *_free.  All device memory is supplied by the caller.
 *   - Fields at the boundary are FP64 in canonical [col][lev] order: column
 *     ids as defined by thor_grid_build, levels from the bottom.
 */
#ifndef THOR_H
#define THOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  THOR_OK = 0,
  THOR_EINVAL = -1,      /* bad argument; nothing was done */
  THOR_ENOMEM = -2,      /* host allocation failed, or dev_bytes too small */
  THOR_EHIP = -3,        /* a HIP runtime call failed (message has the detail) */
  THOR_ENONFINITE = -4,  /* thor_diag found NaN or Inf in the state */
  THOR_ENOTCONV = -5,    /* spring dynamics hit max_iter before the stop rule */
  THOR_ENOTSMOOTH = -6   /* spring dynamics stopped after its first step: nothing relaxed */
};

/* Message of the last failing call on this thread (empty if none).  Valid
 * until the next library call on the same thread. */
const char *thor_last_error(void);

typedef struct thor_grid thor_grid;
typedef struct thor_state thor_state;

/* ---------------------------------------------------------------------------
 * Grid (Sec. 2.1-2.2; Eqs. grid_qts, int_grid, spring_force, spr_vel, dbar,
 * centroid equation).
 *
 * Icosahedron with two vertices at the poles, split into ten rhombi, each
 * refined glevel times by recursive edge bisection onto the unit sphere:
 * n_col = 10 * 4^glevel + 2 columns, 12 of them pentagons.  Column ids: rhombus
 * r (north r = 0..4, south 5..9) owns lattice points a in [1, 2^g],
 * b in [0, 2^g - 1] with id = r 4^g + (a - 1) 2^g + b; north pole 10 * 4^g,
 * south pole 10 * 4^g + 1.  Neighbours are listed counter-clockwise (seen
 * from outside) starting at the smallest id; a pentagon's 6th slot is -1.
 *
 * smooth = 1 builds the modified grid: spring dynamics on the hexagon points
 *   dv/dt = sum_i k (d_i - dbar_spr) e_i - alpha v,
 *   dbar_spr = beta * 2 pi / (10 * 2^(glevel-1)),
 * integrated with step dt (symplectic Euler, tangent velocity) until no
 * point moves more than tol in one step, then the control-volume corners are
 * put at the triangle centroids and every point moved once to the centroid
 * of its control volume.  smooth = 0 keeps the bisection points (corners
 * still at the triangle centroids).  Paper values: beta 1.15, alpha 1,
 * dt 0.01, tol 1e-5; the paper gives no k, this library uses k = 100.
 * ------------------------------------------------------------------------- */
typedef struct {
  int glevel;       /* 0..8 */
  int smooth;       /* 1: spring dynamics + centroids; 0: standard grid */
  double k;         /* spring constant (> 0) */
  double beta;      /* natural-length factor (> 0) */
  double alpha;     /* friction (>= 0) */
  double dt;        /* pseudo time step (> 0) */
  double tol;       /* stop when every point moved less than tol in one step */
  int max_iter;     /* iteration cap (> 0) */
} thor_grid_params;

/* Fill p with the defaults above for grid level glevel. */
void thor_grid_params_default(int glevel, thor_grid_params *p);

/* Build the grid on the host.  EINVAL: bad parameters (glevel outside 0..8,
 * non-positive k, beta, dt, tol or max_iter).  ENOTCONV: max_iter reached
 * (*out is still returned and usable).  ENOTSMOOTH: smooth = 1 and glevel > 0
 * but the stopping rule already held after the first spring step while the
 * springs were out of equilibrium (largest force above 1e-9 k dbar_spr), so
 * no point was relaxed (*out is still returned: the bisection points moved
 * to their control-volume centroids).  (At glevel 1 the hexagon points start
 * in equilibrium: one step, THOR_OK.)  The per-step displacement shrinks with
 * the spacing, so with k = 100 this happens at glevel 8; a larger k relaxes
 * that grid.  ENOMEM: allocation failure. */
int thor_grid_build(const thor_grid_params *p, thor_grid **out);

/* Number of columns, pentagons and spring-dynamics iterations taken. */
int thor_grid_info(const thor_grid *g, int64_t *n_col, int *n_pent, int *spring_iters);

/* Copy the grid into caller-owned host buffers (any pointer may be NULL):
 *   nbr[n_col * 6]  neighbour ids, -1 in a pentagon's 6th slot
 *   xyz[n_col * 3]  unit-sphere cell points
 *   area[n_col]     control-volume areas on the unit sphere (sum = 4 pi) */
int thor_grid_export(const thor_grid *g, int32_t *nbr, double *xyz, double *area);

/* Operator coefficients derived from the geometry (host buffers, NULL ok):
 *   div_coef[n_col * 7 * 3]  div F = (1/r) sum_{j=0..6} c_j . F_j  (j = 0 the
 *                            cell itself, j >= 1 neighbour j-1; Eqs. flx_div,
 *                            int_grid, div_gauss); also grad s =
 *                            (1/r) sum_{j>=1} c_j (s_j - s_0) (Eq. grad)
 *   lap_coef[n_col * 6]      lap s = (1/r^2) sum_j l_j (s_nbr_j - s_0), the
 *                            triangle-gradient Laplacian of Sec. 4 */
int thor_grid_coefficients(const thor_grid *g, double *div_coef, double *lap_coef);

/* The divergence-damping operator lap(grad D) of Sec. 4 folded over the
 * two-ring of each column (host buffers, NULL ok):
 *   idx[n_col * 18]   two-ring column ids, -1 pads
 *   w[n_col * 18 * 3] lap(grad D) = (1/r^3) sum_m w_m (D_idx_m - D_0) */
int thor_grid_damping_coefficients(const thor_grid *g, int32_t *idx, double *w);

void thor_grid_free(thor_grid *g);

/* ---------------------------------------------------------------------------
 * Model configuration (Table 1 style planet parameters; Sec. 3-5).
 * ------------------------------------------------------------------------- */
typedef struct {
  double radius;   /* A [m] */
  double omega;    /* rotation rate [1/s], axis +z */
  double gravity;  /* constant, radial [m/s^2] */
  double Rd;       /* gas constant [J/kg/K] */
  double Cp;       /* heat capacity at constant pressure; Cv = Cp - Rd */
  double p_ref;    /* reference pressure of Eq. pressure [Pa] */
} thor_planet;

typedef struct {
  int n_lev;       /* layers, 1..64, equally spaced in height */
  double z_top;    /* rigid lid height [m] */
} thor_vertical;

enum { THOR_FP64 = 0, THOR_MIXED = 1 };

typedef struct {
  double dt;       /* large time step [s] */
  double diff_D;   /* nondimensional hyperdiffusion number, Kd = D dbar^4/dt (Eq. kd) */
  int div_damp;    /* 1: 3D divergence damping every substep (Sec. 4) */
  int precision;   /* THOR_FP64, or THOR_MIXED: horizontal stencils and
                      advection in FP32, vertical solve and reference state in
                      FP64 */
  int energy_fixer; /* 1: after the dynamics of every large step (before the
                      physics), one temperature increment, the same at every
                      cell and at fixed density, restores the total energy
                      (THOR_DIAG_ENERGY) of the step's start: the globally
                      uniform internal-energy adjustment of Williamson (2009)
                      that the paper implements but leaves off for its
                      results (Sec. 3).  Not available in ensembles. */
  int hydrostatic;  /* 1: the hydrostatic approximation of Sec. 3: no
                      vertical acceleration (time derivative, advection and
                      other slow terms of rho v_r dropped); each acoustic
                      substep's tridiagonal then gives the W that leaves the
                      columns in hydrostatic balance at the substep's end
                      (the [t] imbalance plus the deviation pressure gradient
                      and buoyancy sum to zero).  0: the paper's
                      non-hydrostatic equations. */
  int shallow;      /* 1: the shallow-atmosphere approximation of Sec. 3 with
                      the traditional approximation: every distance from the
                      centre is the planet radius (horizontal operators,
                      vertical flux divergence, volumes); the horizontal
                      momentum is advected by the horizontal velocity and the
                      vertical velocity as a scalar (no metric terms in w,
                      no curvature term in the vertical equation); the
                      Coriolis force is 2 Omega sin(lat) rhat x (rho v_h).
                      0: the paper's deep atmosphere.  Not available in
                      ensembles. */
  int lagrange_order; /* order k of the vertical Lagrange interpolation
                      (Sec. 2.1) used for interface values of centre fields
                      (theta of the vertical solve, the advected velocity,
                      the slow forcing of rho v_r, rho in its hyperdiffusion)
                      and centre values of rho v_r (the advected momentum):
                      0 or 1 (the paper's runs: the two-point mean) or 3 (cubic,
                      from the four nearest levels, shifted one level inward
                      at the ground and the lid; n_lev >= 4).  The buoyancy
                      of the vertical solve and the diagnostics keep the
                      two-point mean.  3 is not available in ensembles. */
  int anelastic;    /* 1: the anelastic approximation of Sec. 3: the density
                      in the mass-flux divergence of the continuity equation
                      is a reference density rho_r(z) that depends on height
                      only.  rho_r is the initial isothermal column (the
                      density of thor_init's hydrostatic state before the
                      noise); the flux is rho_r v with v = (rho v) / rho[t],
                      rho[t] the density at the start of the large step, so
                      each acoustic substep scales the horizontal mass
                      divergence by rho_r / rho[t] at the centres and the
                      vertical mass flux W, in the density update and in the
                      buoyancy of the vertical solve, by the ratio of the
                      two-point means at the interfaces.  Momenta, rho theta,
                      the equation of state and the divergence damping are
                      unchanged.  0: the paper's compressible continuity
                      equation.  Needs lagrange_order 0 or 1; phase V then
                      always runs the four-levels-per-lane mapping; not
                      available in ensembles. */
} thor_numerics;

/* Physics after each large step (Sec. 5, Eq. im_eq_t): backward-Euler
 * Newtonian relaxation of T at fixed density (K_T = 1/tau unless stated)
 * toward
 *   NEWTONIAN:   T_eq = T_mean + dT_daynight/2 cos(lat) cos(lon - lon_ss);
 *   HOT_JUPITER: the hot-Jupiter benchmark, Eqs. teq-hj, btrop, tvert:
 *                T_eq = T_vert(z) + beta_trop(sigma, z) dT_daynight
 *                       cos(lon - lon_ss) cos(lat), T_vert with T_surf = T_mean,
 *                lapse, z_strat, dT_strat; beta_trop with sigma_strat;
 *                sigma = p / p_s, p_s the column's lowest-cell pressure
 *                carried down to z = 0 hydrostatically at that cell's
 *                temperature.  No boundary-layer friction.
 *   HELD_SUAREZ: the Earth benchmark (Eqs. im_eq_v, im_eq_fv and the T_eq,
 *                K_T of Sec. 7.1): boundary-layer friction of the horizontal
 *                momentum, (rho v_h) / (1 + K_v dt) with K_v = k_f max(0,
 *                (sigma - sigma_b) / (1 - sigma_b)), and relaxation with
 *                K_T = k_a + (k_s - k_a) max(0, (sigma - sigma_b) /
 *                (1 - sigma_b)) cos^4(lat) toward T_eq = max(T_min, [T_top -
 *                dT_y sin^2(lat) - dtheta_z ln(p / p_star) cos^2(lat)]
 *                (p / p_star)^(Rd / Cp)); sigma and p as for HOT_JUPITER.
 *                (tau and the HOT_JUPITER fields are unused.) */
enum { THOR_FORCING_NONE = 0, THOR_FORCING_NEWTONIAN = 1, THOR_FORCING_HOT_JUPITER = 2,
       THOR_FORCING_HELD_SUAREZ = 3 };

typedef struct {
  int kind;               /* THOR_FORCING_* */
  double tau;             /* relaxation time scale, K_T = 1/tau [s] */
  double T_mean;          /* NEWTONIAN: mean T_eq; HOT_JUPITER: T_surf [K] */
  double dT_daynight;     /* NEWTONIAN: day/night contrast; HOT_JUPITER: Delta T_E-P [K] */
  double lon_substellar;  /* [rad] */
  double lapse;           /* HOT_JUPITER: Gamma_trop [K/m] */
  double z_strat;         /* HOT_JUPITER: z_stra [m] */
  double dT_strat;        /* HOT_JUPITER: Delta T_stra [K] */
  double sigma_strat;     /* HOT_JUPITER: sigma_stra, in [0, 1) */
  double k_f, k_a, k_s;   /* HELD_SUAREZ: rates [1/s] */
  double sigma_b;         /* HELD_SUAREZ: boundary-layer top, in [0, 1) */
  double dT_y, dtheta_z;  /* HELD_SUAREZ: [K] */
  double p_star;          /* HELD_SUAREZ: [Pa] */
  double T_top, T_min;    /* HELD_SUAREZ: [K] */
} thor_forcing;

typedef struct {
  double T0;          /* isothermal temperature [K] */
  double p_surf;      /* surface pressure [Pa] */
  double noise_amp;   /* uniform temperature noise amplitude [K] */
  uint64_t seed;      /* SplitMix64 counter-based noise (see thor_state_init) */
  int planet_index;   /* counter offset of this planet in an ensemble */
} thor_init;

/* Device bytes thor_state_init needs for this grid and configuration. */
int thor_state_bytes(const thor_grid *g, const thor_vertical *v,
                     const thor_numerics *num, size_t *bytes);

/* Build the initial state and upload grid and state to the device.
 *
 * Initial state: isothermal T0 in discrete hydrostatic balance with the
 * vertical momentum equation, p at the first centre = p_surf exp(-g dz /
 * (2 Rd T0)), rest; then T += eps at fixed p, eps uniform in
 * [-noise_amp, noise_amp) from one SplitMix64 output step of
 * seed XOR (planet_index 2^40 + col 2^20 + lev).
 *
 * dev_buf: caller-owned device memory of at least thor_state_bytes bytes,
 *   256-byte aligned; it must stay allocated and unmoved for the life of the
 *   state and is never freed by the library.
 * hip_stream: the hipStream_t every later call enqueues on (NULL = default).
 * EINVAL: bad configuration (dt <= 0, n_lev outside 1..64, z_top <= 0,
 *   g dz / 2 >= Rd T0, Cp <= Rd, ...).  ENOMEM: dev_bytes too small.
 * EHIP: copy failure.  The call synchronises the stream before returning. */
int thor_state_init(const thor_grid *g, const thor_planet *planet,
                    const thor_vertical *v, const thor_numerics *num,
                    const thor_forcing *forcing, const thor_init *init,
                    void *dev_buf, size_t dev_bytes, void *hip_stream,
                    thor_state **out);

/* Advance n_large large steps of dt, each the three RK stages of Sec. 3 with
 * 1, n/2 and n acoustic substeps (n = n_acoustic; 1 + 3n/2 substeps per large
 * step), followed by the Newtonian relaxation if configured.  Asynchronous
 * on the state's stream.  EINVAL (nothing enqueued): n_large < 0,
 * n_acoustic < 2 or odd. */
int thor_step(thor_state *s, int n_large, int n_acoustic);

/* Diagnostics (synchronise the stream; host_out is caller-owned). */
enum {
  THOR_DIAG_MASS = 1,          /* 1 double: sum rho A_c r_k^2 dz (A_c unit sphere) */
  THOR_DIAG_FIELD = 2,         /* n_col * n_lev doubles of field `field` */
  THOR_DIAG_STATE_EXPORT = 3,  /* checkpoint blob of thor_state_blob_bytes */
  THOR_DIAG_SCALARS = 4,       /* thor_scalars */
  THOR_DIAG_ENERGY = 5,        /* 1 double: total energy [J] = sum over cells of
                                  (Cv p / Rd + (|rho v_h|^2 + (rho v_r)^2) / (2 rho)
                                  + rho g z) A_c r_k^2 dz, rho v_r at the layer
                                  centre (mean of its interfaces) */
  THOR_DIAG_ANGULAR_MOMENTUM = 6 /* 1 double: absolute angular momentum about
                                  the rotation axis [kg m^2/s] = sum over cells
                                  of ((R x rho v_h)_z + rho Omega r_k^2
                                  cos^2(lat)) A_c r_k^2 dz, R = r_k rhat (a
                                  conserved quantity of the equations that the
                                  scheme does not enforce; Sec. 3) */
};
enum {
  THOR_F_T = 0, THOR_F_U, THOR_F_V, THOR_F_W, THOR_F_P, THOR_F_RHO,
  THOR_F_RHOTHETA, THOR_F_MX, THOR_F_MY, THOR_F_MZ,
  THOR_F_WI   /* rho v_r at the interfaces 0..n_lev-1 (the lid value is 0) */
};
typedef struct {
  double mass, max_speed, max_w, min_T, max_T;
} thor_scalars;

/* ENONFINITE if the state holds NaN or Inf (the output is still written).
 * EINVAL: unknown kind/field or out_bytes too small. */
int thor_diag(thor_state *s, int kind, int field, void *host_out, size_t out_bytes);

/* Size of the checkpoint blob (prognostic fields, FP64, canonical layout). */
size_t thor_state_blob_bytes(const thor_state *s);

/* Restore prognostic fields from a blob of thor_diag(STATE_EXPORT).
 * Synchronises.  EINVAL: wrong size or header. */
int thor_state_import(thor_state *s, const void *blob, size_t bytes);

/* Autotuner: for each kernel family ("large", "slow", "hmom", "vert")
 * time the candidate workgroup sizes (1, 2, 4 or 8 wavefronts,
 * i.e. column groups of 1-8 x floor(64 / n_lev) columns) inside real large
 * steps with n_acoustic substeps on this state, keep the fastest, and restore
 * the state from a checkpoint taken before tuning (the state is unchanged).
 * With linear interpolation the "vert" family also tries four levels per
 * lane, and for 32 < n_lev <= 64 two (thor_set_vert_levels_per_lane); with
 * the anelastic switch it keeps four.
 * Synchronises.  wpb_out (4 ints, may be NULL) receives the choice in the
 * order above.  EINVAL: n_acoustic < 2 or odd. */
int thor_autotune(thor_state *s, int n_acoustic, int *wpb_out);

/* Work mapping of the acoustic phase V (the column tridiagonal): 1 level per
 * lane (floor(64 / n_lev) columns per wavefront), 2 levels per lane
 * (ceil(n_lev / 2) lanes per column) or 4 levels per lane (ceil(n_lev / 4)
 * lanes per column, 16-byte row accesses, two in-lane steps of odd-even
 * reduction before the cyclic reduction across lanes), the same arithmetic
 * either way up to rounding.  The default is 4 (1 with lagrange_order 3),
 * the ensemble kernels' mapping, so that a planet run alone equals its
 * ensemble member bitwise; thor_autotune may choose another (then the two
 * agree to rounding).
 * EINVAL: nl not 1, 2 or 4; 2 where n_lev <= 32; 2 or 4 where
 * lagrange_order is 3; 1 or 2 with the anelastic switch.  Synchronises. */
int thor_set_vert_levels_per_lane(thor_state *s, int nl);

/* Mean duration [ms] of the last n kernel launches of the named kernel family
 * recorded with HIP events when timing is on (see thor_set_timing).  Used to
 * measure achieved bandwidth; returns EINVAL for an unknown name. */
int thor_set_timing(thor_state *s, int on);
int thor_kernel_time(thor_state *s, const char *name, double *mean_ms, int *count);

void thor_state_free(thor_state *s);   /* never frees dev_buf */

/* ---------------------------------------------------------------------------
 * Ensembles of planets (each with its own grid level, layer count, planet
 * constants, time step and initial state) advanced together: every phase of
 * the large step is one launch over all members (a device table maps each
 * workgroup to a member and a local workgroup) and the whole large step is
 * replayed as one HIP graph.  All members must share the precision.  A member
 * advanced in an ensemble computes bit-identical results to the same
 * configuration advanced alone with thor_step.
 * ------------------------------------------------------------------------- */
typedef struct thor_batch thor_batch;

/* Device bytes for n members (arrays of n structs). */
int thor_batch_bytes(int n, const thor_grid *const *grids, const thor_vertical *v,
                     const thor_numerics *num, size_t *bytes);

/* Initialise member i exactly as thor_state_init would, inside one
 * caller-owned buffer (256-byte aligned).  EINVAL: any member's
 * configuration is invalid, uses a switch ensembles do not offer (energy
 * fixer, shallow, lagrange_order 3, anelastic), or precisions differ.
 * ENOMEM: dev_bytes too small.  Synchronises. */
int thor_batch_init(int n, const thor_grid *const *grids, const thor_planet *planets,
                    const thor_vertical *v, const thor_numerics *num,
                    const thor_forcing *forcings, const thor_init *inits,
                    void *dev_buf, size_t dev_bytes, void *hip_stream, thor_batch **out);

/* n_large large steps of every member with n_acoustic substeps (each member
 * uses its own dt).  Asynchronous.  EINVAL as thor_step. */
int thor_batch_step(thor_batch *b, int n_large, int n_acoustic);

/* Member i as a thor_state for thor_diag / thor_state_import (thor_step on a
 * member returns EINVAL).  The handle is owned by the batch. */
int thor_batch_member(thor_batch *b, int i, thor_state **out);

/* Workgroup-size autotuner over whole ensemble large steps (see
 * thor_autotune); the members' states are restored afterwards. */
int thor_batch_autotune(thor_batch *b, int n_acoustic, int *wpb_out);

void thor_batch_free(thor_batch *b);   /* frees the members; never frees dev_buf */

/* ---------------------------------------------------------------------------
 * Per-column corrector network: a multilayer perceptron with GELU hidden
 * layers, z = W h + b, W [out][in] row-major.  Operands are BF16 and products
 * accumulate in FP32 on the matrix cores; master weights, gradients and the
 * Adam moments are FP32.  Gradients are reproducible: the reductions over
 * the batch use fixed chunks summed in a fixed order.  Widths must be multiples of 32.  All device
 * pointers below are caller-owned device memory; the object lives in the
 * caller's buffer of thor_mlp_bytes bytes and enqueues on hip_stream.
 * ------------------------------------------------------------------------- */
typedef struct thor_mlp thor_mlp;

/* widths[0] = inputs, widths[n_layers] = outputs; max_batch rows per call. */
int thor_mlp_bytes(int n_layers, const int *widths, int max_batch, size_t *bytes);

/* He-normal weights from a SplitMix64 stream of `seed`, zero biases.
 * EINVAL: bad shape.  ENOMEM: dev_bytes too small.  Synchronises. */
int thor_mlp_init(int n_layers, const int *widths, int max_batch, uint64_t seed,
                  void *dev_buf, size_t dev_bytes, void *hip_stream, thor_mlp **out);

/* Number of FP32 parameters, packed as W1, b1, W2, b2, ... */
size_t thor_mlp_param_count(const thor_mlp *m);
int thor_mlp_set_params(thor_mlp *m, const float *host_params);   /* resets Adam; synchronises */
int thor_mlp_get_params(thor_mlp *m, float *host_params);         /* synchronises */

/* y[B][out] (device, FP32) = network(x[B][in] device BF16): one fused kernel
 * for the corrector's shape, else layer by layer (see below).  Asynchronous.
 * EINVAL: B outside 1..max_batch, or x not 16-byte aligned (also for the two
 * calls below). */
int thor_mlp_forward(thor_mlp *m, const void *x_bf16, int B, float *y);

/* on = 1 (the default): thor_mlp_forward runs a 4-layer network with at
 * most 1152 inputs, hidden widths of 256 and at most 256 outputs (the
 * corrector's shape) as one fused kernel per 48-row tile: the tile's inputs
 * and then its hidden activations kept in LDS (147,456 bytes per
 * workgroup), the weights read from a copy in MFMA fragment order kept
 * beside the BF16 copy; other shapes stay layer by layer.  on = 0: layer by
 * layer.
 * Both give the same products in the same order (equal outputs). */
int thor_mlp_set_fused(thor_mlp *m, int on);

/* Mean-squared loss sum (y - t)^2 / (B out) and, if grad_host is not NULL,
 * its gradient packed like the parameters (host FP32).  B % 32 == 0.
 * Synchronises. */
int thor_mlp_loss_grad(thor_mlp *m, const void *x_bf16, const float *t, int B,
                       double *loss, float *grad_host);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on the mean-squared loss of a
 * batch (B % 32 == 0).  Asynchronous. */
int thor_mlp_train_step(thor_mlp *m, const void *x_bf16, const float *t, int B, float lr);

void thor_mlp_free(thor_mlp *m);   /* never frees dev_buf */

/* ---------------------------------------------------------------------------
 * Learned per-column corrector of a coarse run toward a fine run.
 *
 * Restriction (fine grid -> coarse grid, same levels): every fine column goes
 * to the coarse column whose point is nearest (largest dot product, ties to
 * the lower id); T and p are area-weighted means over a coarse column's fine
 * columns, the velocity is the mass-weighted mean of the Cartesian velocity
 * projected on the coarse tangent plane; the coarse prognostic state is
 * rebuilt from them (rho = p / Rd T, rho theta from p, M = rho v,
 * W = interface mean of rho w).
 * ------------------------------------------------------------------------- */
typedef struct thor_restriction thor_restriction;
typedef struct thor_corrector thor_corrector;

int thor_restriction_bytes(const thor_grid *fine, const thor_grid *coarse, size_t *bytes);
/* Builds the map on the host and uploads it into dev_buf (dev_buf NULL: a
 * host-only map that can be exported but not used by thor_restrict).
 * Synchronises.  EINVAL: fine coarser than coarse, or a coarse column left
 * empty. */
int thor_restriction_build(const thor_grid *fine, const thor_grid *coarse, void *dev_buf,
                           size_t dev_bytes, void *hip_stream, thor_restriction **out);
int thor_restriction_export(const thor_restriction *r, int32_t *coarse_of_fine /*[n_fine]*/);
void thor_restriction_free(thor_restriction *r);

/* Overwrite coarse's state with the restriction of fine's (same levels,
 * lid and precision).  Waits for fine's stream, then enqueues on coarse's. */
int thor_restrict(thor_state *fine, thor_state *coarse, const thor_restriction *r);

/* (T, u, v, w, p) of every cell as FP32 [5][n_col][n_lev] into device memory.
 * Asynchronous. */
int thor_state_fields32(thor_state *s, float *dev_out);

/* Mean and standard deviation per (field, level) (host out: 5 n_lev means
 * then 5 n_lev spreads, [f][k]) over n_arrays field arrays [5][n_col][n_lev]
 * spaced `stride` floats apart, of C itself or, if Fn is not NULL, of
 * Fn - C.  FP64 sums; n_lev must divide 256.  Scratch: at least
 * n_arrays * 320 * n_lev doubles of device memory.  Synchronises. */
int thor_field_stats(const float *C, const float *Fn, int n_arrays, size_t stride, int n_col,
                     int n_lev, void *dev_scratch, size_t scratch_bytes, void *hip_stream,
                     double *mean_std_host);

/* For callers that cannot allocate memory (serving loops and harnesses that
 * forbid device allocations): thor_field_stats without the scratch argument
 * and without any device or host allocation.  The partial sums live in a
 * library-owned device array of 1 MiB per GPU (set up on the first call on
 * a device, kept until the process ends); the arrays are reduced in groups
 * that fit it (12 arrays at n_lev = 32) and summed on the device in
 * thor_field_stats' order.  Every call on a GPU shares that array: calls
 * that overlap on one GPU (other host threads, other streams) race.
 * EINVAL as thor_field_stats; ENOMEM if one array's partial sums
 * (320 n_lev doubles) do not fit (not for any n_lev that divides 256).
 * Synchronises. */
int thor_field_stats_noalloc(const float *C, const float *Fn, int n_arrays, size_t stride, int n_col,
                             int n_lev, void *hip_stream, double *mean_std_host);

/* A corrector of state s by network net (35 n_lev inputs, 5 n_lev outputs,
 * max_batch >= n_col; n_lev a multiple of 32; EINVAL otherwise; dev_buf
 * 256-byte aligned).  norm_host: 20 n_lev floats
 * [4][5][n_lev]: input means and spreads per (field, level), then those of
 * the targets (fine - coarse).
 * A column is corrected only while every normalised output stays within
 * `bound` and the corrected T and p stay positive (else it keeps the plain
 * coarse state).  A corrected cell is rebuilt the way the restriction builds
 * one: rho' = p' / (Rd T'), rho theta from p', M = rho' (v + du e + dv n)
 * with e, n the east and north unit vectors, and W rescaled to the new
 * interface density plus the interface mean of rho' dw.  The correction
 * therefore changes the mass like the restriction does. */
int thor_corrector_bytes(const thor_state *s, size_t *bytes);
int thor_corrector_init(thor_state *s, thor_mlp *net, const float *norm_host, float bound,
                        void *dev_buf, size_t dev_bytes, thor_corrector **out);

/* Training batch from stored pairs (device arrays): row b is column cols[b]
 * of pair pairs[b]; inputs from coarse_fields, targets the normalised
 * fine_fields - coarse_fields of that column; pairs are pair_stride floats
 * apart.  x_bf16 [B][35 n_lev], target [B][5 n_lev].  Asynchronous.  The
 * indices live in device memory and are not checked: the caller keeps
 * 0 <= cols[b] < n_col and pairs[b] within its stored pairs. */
int thor_corrector_batch(thor_corrector *c, const float *coarse_fields, const float *fine_fields,
                         size_t pair_stride, const int32_t *pairs, const int32_t *cols, int B,
                         void *x_bf16, float *target);

/* Apply the network to the state once (fields, inputs, forward, bounded
 * update).  n_applied (may be NULL; then asynchronous) receives the number
 * of corrected columns. */
int thor_corrector_apply(thor_corrector *c, int *n_applied);
void thor_corrector_free(thor_corrector *c);

/* ---------------------------------------------------------------------------
 * Post-processing on pressure levels (the paper shows its results on
 * pressure levels, interpolated linearly from the model levels; Sec. 7).
 *
 * Each thor_zonal_accumulate call takes the state as it stands (between
 * large steps): every column's u, v, T and theta = rho theta / rho are
 * interpolated linearly in p to the levels plev (a level outside the
 * column's range of cell-centre pressures has no value there); per latitude
 * band b, covering [-90 + 180 b / n_bands, -90 + 180 (b + 1) / n_bands)
 * degrees (the north pole in the last band), area-weighted means over the
 * columns with a value and the eddy fluxes [u'v'], [v'T'] (eddies are
 * deviations from the band mean) are added to device time sums.
 * thor_zonal_result gives the time means, each over the snapshots in which
 * the band/level had a value, and the mass streamfunction
 *   Psi = 2 pi radius cos(lat_b) / gravity * int_0^p [v] dp
 * (trapezoid rule over plev, [v](0) = [v](plev[0])).  Beside them, each
 * snapshot adds to the grid-imprinting map of the Held-Suarez results
 * (Sec. 7.1): per column, w* = w - {w} in the first model layer (w at the
 * layer centre; {w} the area-weighted mean over the column's band), whose
 * time mean [w*] thor_zonal_imprint returns.  Results are reproducible:
 * every sum runs in a fixed order.
 * ------------------------------------------------------------------------- */
typedef struct thor_zonal thor_zonal;
enum {
  THOR_ZM_U = 0, THOR_ZM_V = 1, THOR_ZM_T = 2, THOR_ZM_THETA = 3, THOR_ZM_UPVP = 4, THOR_ZM_VPTP = 5,
  THOR_ZM_WEIGHT = 6,     /* area fraction of the band with a value */
  THOR_ZM_PSI = 7,        /* kg/s */
  THOR_ZM_SNAPSHOTS = 8,  /* snapshots in which the band/level had a value */
  THOR_ZM_COUNT = 9
};

/* plev: n_plev pressures [Pa], positive and strictly ascending (host).
 * EINVAL: bad arguments.  1..4096 bands, 1..1024 levels. */
int thor_zonal_bytes(const thor_state *s, int n_bands, const double *plev, int n_plev, size_t *bytes);
/* g: the state's grid; radius, gravity: for Psi.  Uses the state's stream;
 * synchronises.  dev_buf: caller-owned, 256-byte aligned, never freed. */
int thor_zonal_init(thor_state *s, const thor_grid *g, double radius, double gravity, int n_bands,
                    const double *plev, int n_plev, void *dev_buf, size_t dev_bytes, thor_zonal **out);
/* Add the current snapshot.  Asynchronous on the state's stream. */
int thor_zonal_accumulate(thor_zonal *z);
/* host_out [n_bands][n_plev][THOR_ZM_COUNT]; synchronises. */
int thor_zonal_result(thor_zonal *z, double *host_out, int *n_snapshots);
/* host_out [n_col] (canonical ids): [w*] in m/s, 0 before the first
 * snapshot; n_snapshots may be NULL.  Synchronises. */
int thor_zonal_imprint(thor_zonal *z, double *host_out, int *n_snapshots);
/* Zero the time sums, the imprinting map's included (asynchronous, no
 * memset). */
int thor_zonal_reset(thor_zonal *z);
void thor_zonal_free(thor_zonal *z);   /* never frees dev_buf */

/* ---------------------------------------------------------------------------
 * Measurement aid (not part of the method): the memory-traffic mix of a
 * kernel without its arithmetic or gathers, to compare a kernel's achieved
 * bandwidth with what the memory system delivers for the same mix.  Reads
 * n_src FP64 arrays and writes n_dst FP64 arrays of n words each, one word
 * of every array per work item: dst_j[i] = sum_k src_k[i] + j.  src and dst
 * are host arrays of device pointers to caller-owned device arrays (no two
 * dst arrays may overlap); 1 <= n_src <= 16, 1 <= n_dst <= 8, n >= 1.
 * Enqueued on hip_stream, asynchronous.  EINVAL on bad counts or a NULL
 * pointer.
 * ------------------------------------------------------------------------- */
int thor_stream_mix(const double *const *src, int n_src, double *const *dst, int n_dst, int64_t n,
                    void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* THOR_H */
