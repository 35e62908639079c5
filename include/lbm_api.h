/*
 * lbm_api.h -- C ABI of the MI355X (gfx950) hybrid thermal pseudo-potential lattice
 * Boltzmann library, after Hu & Liu, "Study of boiling heat transfer on the wall with
 * an improved hybrid lattice Boltzmann model" (arXiv:1812.10375).
 *
 * One call of lbm_step advances the coupled system of Sec. 2 by one lattice time step
 * per step requested:
 *   - D2Q9 MRT collision and streaming (Eq. 1-5) with the pseudo-potential interaction
 *     force from the Peng-Robinson equation of state (Eq. 6, 7, 28), the Li-type forcing
 *     term (Eq. 8), buoyancy (Eq. 9) and wall adhesion with nucleation sites (Eq. 10,
 *     Sec. 4.2);
 *   - the temperature equation (Eq. 17) by classical RK4 (Eq. 18) with `n_sub`
 *     sub-steps (Eq. 27), finite-volume diffusion with harmonic-mean face
 *     conductivities (Eq. 22-26), isotropic gradients (Eq. 19), through the fluid and a
 *     conjugate heater below it (Sec. 4.2);
 *   - diagnostics: mass, stored energy, heat through the bottom, top and heater surface,
 *     and the running mean/variance of the bottom heat flux (Sec. 3.2, Sec. 4.3).
 *
 * Geometry.  Fluid nodes (x, y), 0 <= x < nx (periodic), 0 <= y < ny.  `heater_rows`
 * solid rows lie below fluid row 0; temperature lives on heater and fluid rows (T row
 * j = y + heater_rows).  The solid below fluid row 0 is a half-way bounce-back wall.
 * The top is a wall, a constant-pressure opening or a convective outlet.
 *
 * Memory.  The caller owns all device memory and the HIP stream.  lbm_init carves the
 * caller's workspace (lbm_workspace_bytes() bytes, 256-byte aligned device memory)
 * and copies the initial fields into it; the library never allocates device memory.
 * Host arrays passed in are copied before the call returns.  A context is used by one
 * host thread at a time.
 *
 * Errors.  Every entry point returns LBM_OK (0) or a negative status.  Argument errors
 * are reported at once.  Errors found on the device (non-finite values, density <= 0,
 * 1 - b rho <= 0, or a negative radicand under the square root of Eq. 7) are sticky:
 * lbm_observe reports LBM_ENONFINITE with the first bad step, and lbm_step refuses to
 * run afterwards (LBM_ESTATE).
 */
#ifndef LBM_API_H
#define LBM_API_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 2

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* bad argument or configuration                        */
  LBM_ENOMEM = -2,     /* workspace smaller than lbm_workspace_bytes()         */
  LBM_EHIP = -3,       /* a HIP runtime call failed                            */
  LBM_ENONFINITE = -4, /* the device flagged a bad state (see above)           */
  LBM_ESTATE = -5      /* call not allowed in the context's current state      */
};

enum { LBM_F32 = 0, LBM_F64 = 1 }; /* storage and arithmetic type of the fields   */
enum { LBM_TOP_WALL = 0, LBM_TOP_CONST_PRESSURE = 1, LBM_TOP_CONVECTIVE = 2 };
enum { LBM_TBC_DIRICHLET = 0, LBM_TBC_FLUX = 1, LBM_TBC_ZERO_GRAD = 2 };
enum {
  LBM_FREEZE_EOS_T = 1u,   /* EOS of Eq. 7 evaluated at T_sat (Sec. 3.2)          */
  LBM_NO_ADVECTION = 2u,   /* drop -u.grad T from Eq. 17                          */
  LBM_NO_LATENT = 4u,      /* drop the (dp/dT)_v div(u) term from Eq. 17          */
  LBM_DIFF_ISOTROPIC = 8u, /* diffusion by Eq. 20-21 (comparison scheme)          */
  LBM_TWO_LAUNCHES = 32u,  /* FP32 with n_sub = 1: run each step as a collide launch
                              followed by an energy launch ...                       */
  LBM_ONE_LAUNCH = 64u     /* ... or as one fused launch.  Without either flag the
                              library picks by grid size (fused when the collide tiles
                              fill the device's workgroup slots in one round).  A
                              performance knob: the results are identical.  Setting
                              both is an error.                                      */
};

/*
 * Configuration.  Set struct_size = sizeof(lbm_config) and abi_version =
 * LBM_ABI_VERSION.  Units are lattice units (c = dx = dt = 1).
 *   nx, ny, heater_rows   lattice size; nx, ny >= 1 (ny >= 2 with an open top); one field
 *                         of nx (ny + heater_rows) values must stay below 4 GiB (FP32: about
 *                         1.07e9 nodes, FP64: about 5.4e8)
 *   n_sub                 N of Eq. 27 (energy sub-steps per LB step), >= 1
 *   precision             LBM_F32 or LBM_F64 (the Peng-Robinson EOS of Eq. 7/28 and all
 *                         reductions are FP64 in both)
 *   a, b, R, omega        Peng-Robinson constants (Eq. 28, Sec. 3.1)
 *   T_sat                 saturation temperature (EOS temperature under FREEZE_EOS_T)
 *   G, sigma              Eq. 7 interaction strength (< 0) and Eq. 8 parameter
 *   tau_l, tau_v          viscous relaxation times of liquid and vapour (nu = (tau-1/2)/3);
 *                         tau varies linearly in density between rho_v and rho_l
 *   s_e, s_zeta, s_q      the other relaxation rates of Eq. 3
 *   rho_l, rho_v          coexistence densities (tau interpolation, constant-pressure top)
 *   cv, k                 fluid heat capacity and diffusivity: lambda = rho cv k
 *   rho_w, cv_w, lambda_w heater density, heat capacity, conductivity (Sec. 4.2)
 *   g                     gravity magnitude, acting along -y (Eq. 9)
 *   T_bottom, q_bottom    bottom thermal boundary: temperature of the Dirichlet ghost row
 *                         one spacing below the lowest T row, or heat flux into the domain
 *   T_top                 top Dirichlet temperature (bottom_tbc/top_tbc select the kind)
 *   Gw0, Gw_top           wall strengths of Eq. 10 at the bottom wall and a top wall
 *   n_sites, site_*       nucleation sites (Sec. 4.2): centre x, width, minimum strength;
 *                         host arrays of n_sites doubles (may be NULL when n_sites = 0)
 *   tile_rows             rows of temperature grid per energy tile, a performance knob.  In
 *                         FP64 and under LBM_DIFF_ISOTROPIC the fields do not depend on it.
 *                         The FP32 finite-volume path evaluates tiles whose rows are all
 *                         away from the boundaries in an all-fluid form of the same
 *                         coefficients (other rounding), so its fields follow the tile
 *                         shape in their last bits; so do the FP64 sums behind the
 *                         diagnostics, at any precision.  0 = automatic (one domain: tiles that fill
 *                         the device in one round; a batch: the tallest tiles), otherwise
 *                         clamped to [8, 48].  It sets the number of tile rows; the FP32
 *                         path (without LBM_DIFF_ISOTROPIC) then shortens the first and the
 *                         last tile row, whose tiles run the slower boundary code, and
 *                         raises the interior height to cover the grid (at most 48)
 */
typedef struct {
  uint32_t struct_size, abi_version;
  int32_t nx, ny, heater_rows, n_sub;
  int32_t precision, top_bc, bottom_tbc, top_tbc;
  uint32_t flags;
  int32_t tile_rows;
  double a, b, R, omega, T_sat, G, sigma;
  double tau_l, tau_v, s_e, s_zeta, s_q;
  double rho_l, rho_v;
  double cv, k, rho_w, cv_w, lambda_w;
  double g;
  double T_bottom, T_top, q_bottom;
  double Gw0, Gw_top;
  int32_t n_sites;
  const double *site_xc, *site_width, *site_gmin;
} lbm_config;

/*
 * Observation after the last completed step (all FP64):
 *   mass        sum of rho over the fluid, state after the step
 *   energy      sum of (rho c_v) T over heater and fluid (rho of the step's collision)
 *   rho_ave     domain-mean density that the next step's buoyancy uses (Eq. 9)
 *   q_bottom    heat entering through the bottom boundary per unit length and time,
 *               last step (RK-weighted over the Eq. 18 stages); q_bottom_mean/_var are
 *               its running mean and population variance over all steps
 *   q_surface   same through the heater/fluid surface (= q_bottom without a heater)
 *   *_cum       cumulative heat through bottom, top and surface; dE_cum is the
 *               cumulative sum of (rho c_v)(T^{n+1} - T^n)
 *   max_speed   largest |u| of the last collision
 */
typedef struct {
  int64_t step;
  double mass, energy, rho_ave;
  double q_bottom, q_bottom_mean, q_bottom_var, q_surface;
  double Q_bottom_cum, Q_top_cum, Q_surface_cum, dE_cum, max_speed;
  int32_t error_flags; /* LBM_ERR_* bits */
  int64_t first_bad_step;
} lbm_obs;

/* LBM_ERR_SYNC: in the fused FP32 step a workgroup waited too long (about a second) for
 * the collide tiles it depends on, for example because other work occupied the device
 * and delayed their dispatch; the step's results are not trustworthy. */
enum { LBM_ERR_RHO = 1, LBM_ERR_COVOLUME = 2, LBM_ERR_RADICAND = 4, LBM_ERR_NONFINITE = 8, LBM_ERR_SYNC = 16 };

/* Fields for lbm_read_field / lbm_write_field; element type is the context's precision.
 *   LBM_FIELD_F    9 x ny x nx pre-collision populations f^n (x fastest)   read/write
 *   LBM_FIELD_T    (heater_rows + ny) x nx temperature                     read/write
 *   LBM_FIELD_RHO  ny x nx density of the last collision                   read
 *   LBM_FIELD_UX/UY ny x nx Eq. 5 velocity of the last collision           read
 *   LBM_FIELD_GW   nx wall strength of each column of the bottom wall      read
 *   LBM_FIELD_STATE the rest of the state a run continues from, as an opaque record of
 *                  lbm_field_bytes() bytes (host memory only): the step count, the mass
 *                  carried by continuity and the last step's exchange through an open
 *                  top (which set rho_ave of the next step, Eq. 9), the cumulative heat
 *                  and energy sums, the running statistics of the bottom heat flux and
 *                  the sticky error state.                                     read/write
 * Checkpoint: lbm_read_field of F, T and STATE (reading STATE folds the pending
 * diagnostics as lbm_observe does).  Restart, in a context of the same configuration:
 * lbm_write_field of F, then T, then STATE (writing F resets the step count and the
 * carried mass; STATE, written last, restores them).  The run then continues bitwise
 * as if it had not been interrupted, its observations included.  A batch domain's STATE
 * can be read but not written (the domains of a batch share one step count). */
enum { LBM_FIELD_F = 0, LBM_FIELD_RHO = 1, LBM_FIELD_UX = 2, LBM_FIELD_UY = 3, LBM_FIELD_T = 4,
       LBM_FIELD_GW = 10, LBM_FIELD_STATE = 11 };

typedef struct lbm_ctx lbm_ctx;

/* Bytes of device workspace lbm_init needs for cfg; 0 if cfg is invalid.  Host only. */
size_t lbm_workspace_bytes(const lbm_config *cfg);

/* Create a context on the current HIP device.  d_workspace: device pointer to
 * ws_bytes bytes (>= lbm_workspace_bytes), 256-byte aligned, owned by the caller and
 * borrowed until lbm_destroy.  hip_stream: hipStream_t to enqueue on (NULL = default).
 * rho0_host: ny*nx initial densities (the populations start at equilibrium at rest);
 * T0_host: (heater_rows+ny)*nx initial temperatures.  Synchronises the stream. */
int lbm_init(const lbm_config *cfg, void *d_workspace, size_t ws_bytes, void *hip_stream,
             const double *rho0_host, const double *T0_host, lbm_ctx **out);

/* Enqueue nsteps (>= 0) complete steps on the context's stream; never synchronises.
 * Diagnostics of each step go to a device history of LBM_HISTORY_STEPS slots, folded
 * (two small kernels) at the end of the step that fills it and by lbm_observe.
 * Graph capture: every kernel argument repeats with period 2 steps except the history
 * slot, so a caller may capture a multiple of LBM_HISTORY_STEPS steps that starts with
 * an empty history (right after lbm_init, lbm_observe or lbm_write_field) into a HIP
 * graph and replay it on the context's stream; each replay folds its own diagnostics.
 * Replays advance the device's step counter only: call lbm_observe after them, before
 * any other call on the context (it takes the step count from the device).
 * Device memory written: the workspace only; no memset or host copy is enqueued. */
#define LBM_HISTORY_STEPS 256
int lbm_step(lbm_ctx *h, int64_t nsteps);

/* Use another stream from now on (for example a graph-capture stream).  The caller
 * orders the switch against work already enqueued on the old stream. */
int lbm_set_stream(lbm_ctx *h, void *hip_stream);

/* Synchronise the stream and fill *out; LBM_ENONFINITE if the device flagged an error. */
int lbm_observe(lbm_ctx *h, lbm_obs *out);

/* Copy a field to dst (host or device memory of `bytes` bytes, which must equal the
 * field's size).  Synchronises the stream for host destinations. */
int lbm_read_field(lbm_ctx *h, int field, void *dst, size_t bytes, int dst_is_device);

/* Overwrite the populations (LBM_FIELD_F, pre-collision), the temperature or the run
 * state (LBM_FIELD_STATE, host memory; LBM_EINVAL if the record does not belong to this
 * configuration). */
int lbm_write_field(lbm_ctx *h, int field, const void *src, size_t bytes, int src_is_device);

/* Size in bytes of a field of this context (0 for an unknown field). */
size_t lbm_field_bytes(lbm_ctx *h, int field);

/* Per-kernel timing for measurement.  While enabled, lbm_step records HIP events on
 * the context's stream around the collide kernel and around the energy kernel(s) of
 * every step.  lbm_kernel_times synchronises the stream, returns the summed durations
 * (milliseconds) and launch counts since timing was enabled or last read, and resets
 * them.  Disabled by default; enabling it adds two event records per kernel launch. */
int lbm_set_kernel_timing(lbm_ctx *h, int enable);
int lbm_kernel_times(lbm_ctx *h, double *collide_ms, int64_t *collide_launches,
                     double *energy_ms, int64_t *energy_launches);

/* Release the host-side context (the workspace stays the caller's). */
int lbm_destroy(lbm_ctx *h);

/*
 * Batches.  n independent domains (sizes, superheats, sites and boundaries may all
 * differ; precision, n_sub and the LBM_DIFF_ISOTROPIC flag must agree) advance together:
 * each lbm_batch_step launches one collide kernel and n_sub energy kernels whose
 * workgroups cover the tiles of every domain, so a batch of small domains fills the
 * device as one large domain would.  Each domain evolves exactly as it would alone with
 * the same tile_rows.  The workspace holds a device table of the domains followed by
 * each domain's own workspace; ownership, streams and errors are as for one domain.
 * lbm_batch_step has the same graph-capture property as lbm_step.  The per-step
 * diagnostics of all domains are folded together (two launches for the whole batch) at
 * the end of every 256th step and in lbm_batch_observe.
 */
typedef struct lbm_batch lbm_batch;

/* Bytes of device workspace for the batch; 0 if n < 1 or any cfg is invalid. */
size_t lbm_batch_workspace_bytes(const lbm_config *cfgs, int n);

/* rho0_host[i], T0_host[i]: initial fields of domain i as in lbm_init. */
int lbm_batch_init(const lbm_config *cfgs, int n, void *d_workspace, size_t ws_bytes, void *hip_stream,
                   const double *const *rho0_host, const double *const *T0_host, lbm_batch **out);
int lbm_batch_step(lbm_batch *b, int64_t nsteps);
int lbm_batch_set_stream(lbm_batch *b, void *hip_stream);

/* Synchronise and fill out[0..n-1]; LBM_ENONFINITE if any domain flagged an error (its
 * entry says which), after which lbm_batch_step returns LBM_ESTATE. */
int lbm_batch_observe(lbm_batch *b, lbm_obs *out);

/* Field access of domain i, as lbm_read_field / lbm_write_field. */
int lbm_batch_read_field(lbm_batch *b, int i, int field, void *dst, size_t bytes, int dst_is_device);
int lbm_batch_write_field(lbm_batch *b, int i, int field, const void *src, size_t bytes, int src_is_device);
int lbm_batch_destroy(lbm_batch *b);

/*
 * Tile-shape autotuner.  For the batch cfgs (n = 1 tunes one domain) it builds the batch
 * in the caller's workspace (lbm_batch_workspace_bytes bytes) once per candidate energy
 * tile height, times `steps` steps after `steps` warm-up steps with HIP events on the
 * stream, and returns the fastest height in *best_rows (pass it as tile_rows) and its
 * time per step in *best_ms.  Results are cached per process, keyed by the domain sizes,
 * precision, flags and n_sub; the workspace contents are scratch.  Synchronises.
 */
int lbm_autotune_tile_rows(const lbm_config *cfgs, int n, void *d_workspace, size_t ws_bytes,
                           void *hip_stream, const double *const *rho0_host,
                           const double *const *T0_host, int steps, int *best_rows, double *best_ms);

/*
 * Launch-shape autotuner, a superset of lbm_autotune_tile_rows (same workspace, inputs,
 * timing, caching and synchronisation).
 *   n >= 2: it times every candidate energy tile height for all domains together, then,
 *           taking the size classes (nx, ny, heater_rows) in order of their node count,
 *           every candidate height for one class with the others held at their best.
 *   n = 1:  it times the domain on its own path (lbm_init / lbm_step) at the automatic
 *           height (tile_rows = 0) and every candidate height; an FP32 domain with n_sub = 1 and the finite-volume faces is timed
 *           both as two launches per step and as the fused one-launch step.
 * rows[i] (n entries) receives domain i's tile_rows and flags[i] cfgs[i].flags with the
 * chosen launch mode (LBM_ONE_LAUNCH or LBM_TWO_LAUNCHES for a domain timed both ways,
 * neither otherwise); pass both back in the configurations.  *best_ms is the time per
 * step of that choice.  The choice changes results only as tile_rows does (above).
 */
int lbm_autotune(const lbm_config *cfgs, int n, void *d_workspace, size_t ws_bytes, void *hip_stream,
                 const double *const *rho0_host, const double *const *T0_host, int steps,
                 int32_t *rows, uint32_t *flags, double *best_ms);

/* Static description of a status code. */
const char *lbm_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif
