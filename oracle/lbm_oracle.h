/*
 * lbm_oracle.h -- plain FP64 CPU oracle of the hybrid thermal pseudo-potential
 * lattice Boltzmann step of Hu & Liu, "Study of boiling heat transfer on the wall
 * with an improved hybrid lattice Boltzmann model" (arXiv:1812.10375).
 *
 * TEST INFRASTRUCTURE.  This library exists only to check the GPU library against
 * the paper.  Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no source with the GPU library.
 *
 * Lattice: D2Q9, velocities e0=(0,0) e1=(1,0) e2=(0,1) e3=(-1,0) e4=(0,-1)
 * e5=(1,1) e6=(-1,1) e7=(-1,-1) e8=(1,-1); c = dx = dt = 1 (Sec. 3.1).
 * Fluid nodes (x,y), 0<=x<nx (periodic), 0<=y<ny.  A conjugate heater of
 * `heater_rows` solid rows sits below fluid row 0 (Sec. 4.2).  Temperature lives
 * on heater and fluid rows: T row j = y + heater_rows.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_TOP_WALL = 0, ORC_TOP_CONST_PRESSURE = 1, ORC_TOP_CONVECTIVE = 2 };
enum { ORC_TBC_DIRICHLET = 0, ORC_TBC_FLUX = 1, ORC_TBC_ZERO_GRAD = 2 };
enum {
  ORC_FREEZE_EOS_T = 1u,   /* EOS temperature held at T_sat (Sec. 3.2)            */
  ORC_NO_ADVECTION = 2u,   /* drop -u.grad T in Eq. 17                            */
  ORC_NO_LATENT = 4u,      /* drop the (dp/dT)_v div(u) term in Eq. 17            */
  ORC_DIFF_ISOTROPIC = 8u, /* diffusion by Eq. 20-21 instead of Eq. 22-26         */
  ORC_SIGMA_PLAIN = 16u    /* sigma term of Eq. 8 without the factor 12           */
};

typedef struct {
  int32_t nx, ny, heater_rows, n_sub;
  int32_t top_bc, bottom_tbc, top_tbc;
  uint32_t flags;
  double a, b, R, omega, T_sat, G, sigma;   /* Eq. 28, Eq. 7, Eq. 8            */
  double tau_l, tau_v, s_e, s_zeta, s_q;    /* Eq. 3 and the nu-tau relation    */
  double rho_l, rho_v;                      /* coexistence densities            */
  double cv, k, rho_w, cv_w, lambda_w;      /* Sec. 3.1, Sec. 4.2               */
  double g;                                 /* Eq. 9, acts along -y             */
  double T_bottom, T_top, q_bottom;         /* thermal boundary values          */
  double Gw0, Gw_top;                       /* Eq. 10 wall strengths            */
  int32_t n_sites;                          /* nucleation sites (Sec. 4.2)      */
  const double *site_xc, *site_width, *site_gmin;
} orc_params;

typedef struct {
  int64_t step;
  double mass, energy, rho_ave;
  double q_bottom, q_bottom_mean, q_bottom_var, q_surface;
  double Q_bottom_cum, Q_top_cum, Q_surface_cum, dE_cum, max_speed;
  int32_t error_flags;
  int64_t first_bad_step;
} orc_obs;

enum {
  ORC_FIELD_F = 0,     /* 9 x ny x nx, pre-collision populations f^n             */
  ORC_FIELD_RHO = 1,   /* ny x nx, density of the last collision                */
  ORC_FIELD_UX = 2,    /* ny x nx, Eq. 5 velocity of the last collision         */
  ORC_FIELD_UY = 3,
  ORC_FIELD_T = 4,     /* (heater_rows+ny) x nx                                 */
  ORC_FIELD_PSI = 5,   /* ny x nx                                               */
  ORC_FIELD_FX = 6,    /* ny x nx total force                                   */
  ORC_FIELD_FY = 7,
  ORC_FIELD_FMX = 8,   /* ny x nx interaction force (Eq. 6)                     */
  ORC_FIELD_FMY = 9,
  ORC_FIELD_GW = 10    /* nx, wall strength of each bottom solid column         */
};

enum { ORC_ERR_RHO = 1, ORC_ERR_COVOLUME = 2, ORC_ERR_RADICAND = 4, ORC_ERR_NONFINITE = 8 };

typedef struct orc_sim orc_sim;

orc_sim *orc_create(const orc_params *p, const double *rho0, const double *T0);
void orc_destroy(orc_sim *s);
int orc_step(orc_sim *s, int64_t nsteps);
void orc_observe(const orc_sim *s, orc_obs *out);
double *orc_field(orc_sim *s, int field);
int64_t orc_field_len(const orc_sim *s, int field);

/* Building blocks, exposed so that tests can pin them one by one. */
double orc_eos_p(const orc_params *p, double rho, double T);
double orc_psi(const orc_params *p, double rho, double T);
double orc_dpdT(const orc_params *p, double rho, double T);
double orc_Tc(const orc_params *p);
void orc_feq(double rho, double ux, double uy, double out[9]);
void orc_collide_node(const orc_params *p, const double f[9], double Fx, double Fy,
                      double Fmx, double Fmy, double psi, double fout[9], double *ux,
                      double *uy);
void orc_moments(orc_sim *s);                   /* rho, psi from f and T           */
void orc_forces(orc_sim *s);                    /* F_m + F_ads + F_b from psi, rho */
void orc_energy_rhs(orc_sim *s, const double *Y, double *K, double flux[3]);
void orc_energy_update(orc_sim *s);             /* N RK4 sub-steps of Eq. 17-18    */

#ifdef __cplusplus
}
#endif
#endif
