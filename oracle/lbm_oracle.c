/*
 * lbm_oracle.c -- plain FP64 CPU oracle of the hybrid thermal pseudo-potential
 * lattice Boltzmann step of Hu & Liu (arXiv:1812.10375).
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
 * the benchmark load this file's library; the GPU library never does, and the two
 * share no source.
 *
 * Everything is double precision and written node by node in the order the paper
 * states the method.  OpenMP splits independent node loops over rows only; every
 * reduction is a serial loop in a fixed index order, so results do not depend on
 * the thread count.  Where the paper is silent or misprinted, the reading taken is
 * stated at the point of use.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* D2Q9 velocity set in the order e0..e8 given in the header. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* Weights of the interaction force, Eq. 6: w(1) = 1/3, w(2) = 1/12. */
static const double WPSI[9] = {0.0,        1.0 / 3.0,  1.0 / 3.0,  1.0 / 3.0, 1.0 / 3.0,
                               1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0};

/*
 * Orthogonal D2Q9 moment matrix M of Eq. 2 (rows: rho, e, zeta, j_x, q_x, j_y, q_y,
 * p_xx, p_xy).  The paper does not print M; these rows are the ones for which
 * M f^eq reproduces the equilibrium moments of Eq. 4 (checked by the tests).
 */
static const double MM[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},         {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},     {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},      {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},      {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

struct orc_sim {
  orc_params p;
  double *site_store;
  int nx, ny, nh, nT;
  double Tc, kappa;
  double Minv[9][9];
  double *f, *fnew;                         /* 9 x ny x nx                     */
  double *rho, *psi, *ux, *uy, *Fx, *Fy, *Fmx, *Fmy;
  double *T, *Tn, *Y, *h1, *h2, *h3, *h4;   /* nT x nx                         */
  double *Gw;                               /* nx                              */
  double rho_ave;
  orc_obs obs;
  double welford_m2;
};

/* ------------------------------------------------------------------------- */
/* Peng-Robinson equation of state, Eq. 28 and Sec. 3.1.                      */
/* ------------------------------------------------------------------------- */

/* a = 0.45724 R^2 Tc^2 / pc and b = 0.0778 R Tc / pc give Tc = (a/b)(0.0778/0.45724)/R. */
double orc_Tc(const orc_params *p) { return (p->a / p->b) * (0.0778 / 0.45724) / p->R; }

static double pr_kappa(const orc_params *p) {
  return 0.37464 + 1.54226 * p->omega - 0.26992 * p->omega * p->omega;
}

/*
 * Temperature function of Eq. 28.  The printed form [1 + kappa sqrt(1 - T/Tc)]^2 is
 * read as the standard Peng-Robinson alpha function [1 + kappa (1 - sqrt(T/Tc))]^2:
 * only this form reproduces the coexistence densities quoted in Sec. 3.1.
 */
static double pr_phi(const orc_params *p, double T) {
  double s = 1.0 + pr_kappa(p) * (1.0 - sqrt(T / orc_Tc(p)));
  return s * s;
}

/* d(phi)/dT of the same function. */
static double pr_dphi(const orc_params *p, double T) {
  double Tc = orc_Tc(p), kap = pr_kappa(p);
  double s = 1.0 + kap * (1.0 - sqrt(T / Tc));
  return -kap * s / sqrt(T * Tc);
}

double orc_eos_p(const orc_params *p, double rho, double T) {
  double a = p->a, b = p->b;
  return rho * p->R * T / (1.0 - b * rho) -
         a * pr_phi(p, T) * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
}

/* (dp/dT) at constant specific volume, used by the latent-heat term of Eq. 17. */
double orc_dpdT(const orc_params *p, double rho, double T) {
  double a = p->a, b = p->b;
  return rho * p->R / (1.0 - b * rho) -
         a * pr_dphi(p, T) * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
}

/* Effective density from Eq. 7 with c = 1 and c_s^2 = 1/3: psi = sqrt(2 (p - rho/3) / G). */
double orc_psi(const orc_params *p, double rho, double T) {
  double pe = orc_eos_p(p, rho, T);
  return sqrt(2.0 * (pe - rho / 3.0) / p->G);
}

/* ------------------------------------------------------------------------- */
/* Equilibrium and MRT collision, Eq. 2-5 and Eq. 8.                          */
/* ------------------------------------------------------------------------- */

static void build_minv(double Minv[9][9]) {
  /* M is orthogonal with M M^T = diag(n_k), so M^-1 = M^T diag(1/n_k). */
  for (int k = 0; k < 9; ++k) {
    double nk = 0.0;
    for (int i = 0; i < 9; ++i) nk += MM[k][i] * MM[k][i];
    for (int i = 0; i < 9; ++i) Minv[i][k] = MM[k][i] / nk;
  }
}

static void equilibrium_moments(double rho, double ux, double uy, double meq[9]) {
  /* Eq. 4 */
  double usq = ux * ux + uy * uy;
  meq[0] = rho;
  meq[1] = rho * (-2.0 + 3.0 * usq);
  meq[2] = rho * (1.0 - 3.0 * usq);
  meq[3] = rho * ux;
  meq[4] = -rho * ux;
  meq[5] = rho * uy;
  meq[6] = -rho * uy;
  meq[7] = rho * (ux * ux - uy * uy);
  meq[8] = rho * ux * uy;
}

void orc_feq(double rho, double ux, double uy, double out[9]) {
  /* f^eq = M^-1 m^eq, with m^eq from Eq. 4. */
  double Minv[9][9], meq[9];
  build_minv(Minv);
  equilibrium_moments(rho, ux, uy, meq);
  for (int i = 0; i < 9; ++i) {
    double s = 0.0;
    for (int k = 0; k < 9; ++k) s += Minv[i][k] * meq[k];
    out[i] = s;
  }
}

/* Kinematic-viscosity relaxation time: the paper gives the bulk values only
 * (nu_l, nu_v in Sec. 3.1, nu = (tau - 1/2)/3 under Eq. 3); across the interface
 * tau is interpolated linearly in density between the two coexistence values. */
static double tau_nu(const orc_params *p, double rho) {
  double w = (rho - p->rho_v) / (p->rho_l - p->rho_v);
  if (w < 0.0) w = 0.0;
  if (w > 1.0) w = 1.0;
  return p->tau_v + (p->tau_l - p->tau_v) * w;
}

static void collide(const orc_params *p, const double Minv[9][9], const double f[9],
                    double Fx, double Fy, double Fmx, double Fmy, double psi, double fout[9],
                    double *uxo, double *uyo) {
  double m[9], meq[9], S[9], lam[9], ms[9];
  for (int k = 0; k < 9; ++k) {
    double s = 0.0;
    for (int i = 0; i < 9; ++i) s += MM[k][i] * f[i];
    m[k] = s;
  }
  double rho = m[0];
  /* Eq. 5: rho u = sum e f + F/2 (dt = 1); m[3], m[5] are sum e_x f, sum e_y f. */
  double ux = (m[3] + 0.5 * Fx) / rho;
  double uy = (m[5] + 0.5 * Fy) / rho;
  equilibrium_moments(rho, ux, uy, meq);

  /* Eq. 3: relaxation rates.  Only tau_nu is tied to the fluid by the paper; the
   * rates of rho and j do not change the result (the rho moment is conserved and
   * the post-collision j is rho u + F/2 for any rate); s_e, s_zeta, s_q are inputs. */
  double snu = 1.0 / tau_nu(p, rho);
  lam[0] = 1.0;
  lam[1] = p->s_e;
  lam[2] = p->s_zeta;
  lam[3] = 1.0;
  lam[4] = p->s_q;
  lam[5] = 1.0;
  lam[6] = p->s_q;
  lam[7] = snu;
  lam[8] = snu;

  /* Eq. 8, with the two misprints read as: |F_m|^2 = F_mx^2 + F_my^2 in the sigma
   * terms, and u_x F_y + u_y F_x as the last entry (the moment of the second-order
   * forcing term).  The sigma coefficient carries the factor 12 of the forcing scheme
   * the paper adopts unless ORC_SIGMA_PLAIN is set. */
  double tau_e = 1.0 / p->s_e, tau_z = 1.0 / p->s_zeta;
  double sig = (p->flags & ORC_SIGMA_PLAIN) ? p->sigma : 12.0 * p->sigma;
  double Fm2 = Fmx * Fmx + Fmy * Fmy;
  double uF = ux * Fx + uy * Fy;
  S[0] = 0.0;
  S[1] = 6.0 * uF + sig * Fm2 / (psi * psi * (tau_e - 0.5));
  S[2] = -6.0 * uF - sig * Fm2 / (psi * psi * (tau_z - 0.5));
  S[3] = Fx;
  S[4] = -Fx;
  S[5] = Fy;
  S[6] = -Fy;
  S[7] = 2.0 * (ux * Fx - uy * Fy);
  S[8] = ux * Fy + uy * Fx;

  /* Eq. 2: m* = m - Lambda (m - m^eq) + (I - Lambda/2) S, then f* = M^-1 m*. */
  for (int k = 0; k < 9; ++k) ms[k] = m[k] - lam[k] * (m[k] - meq[k]) + (1.0 - 0.5 * lam[k]) * S[k];
  for (int i = 0; i < 9; ++i) {
    double s = 0.0;
    for (int k = 0; k < 9; ++k) s += Minv[i][k] * ms[k];
    fout[i] = s;
  }
  *uxo = ux;
  *uyo = uy;
}

void orc_collide_node(const orc_params *p, const double f[9], double Fx, double Fy,
                      double Fmx, double Fmy, double psi, double fout[9], double *ux,
                      double *uy) {
  double Minv[9][9];
  build_minv(Minv);
  collide(p, Minv, f, Fx, Fy, Fmx, Fmy, psi, fout, ux, uy);
}

/* ------------------------------------------------------------------------- */
/* Simulation object                                                          */
/* ------------------------------------------------------------------------- */

static int wrapx(int x, int nx) { return ((x % nx) + nx) % nx; }

/* Nucleation sites (Sec. 4.2): the wall strength drops linearly from Gw0 at the
 * edge of a site to its minimum at the centre.  Column c has its centre at c + 1/2;
 * a site of width W centred at xc covers the columns whose centre lies within W/2
 * of xc (periodic in x). */
static void build_gw(orc_sim *s) {
  const orc_params *p = &s->p;
  for (int x = 0; x < s->nx; ++x) s->Gw[x] = p->Gw0;
  for (int k = 0; k < p->n_sites; ++k) {
    double xc = p->site_xc[k], half = 0.5 * p->site_width[k], gmin = p->site_gmin[k];
    for (int x = 0; x < s->nx; ++x) {
      double d = (x + 0.5) - xc;
      /* shortest periodic distance */
      d = d - s->nx * floor(d / s->nx + 0.5);
      double ad = fabs(d);
      if (ad < half) {
        double g = gmin + (p->Gw0 - gmin) * (ad / half);
        if (g < s->Gw[x]) s->Gw[x] = g;
      }
    }
  }
}

orc_sim *orc_create(const orc_params *p, const double *rho0, const double *T0) {
  if (p->nx < 1 || p->ny < 1 || p->heater_rows < 0 || p->n_sub < 1) return NULL;
  if (p->top_bc != ORC_TOP_WALL && p->ny < 2) return NULL;
  orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
  s->p = *p;
  s->nx = p->nx;
  s->ny = p->ny;
  s->nh = p->heater_rows;
  s->nT = p->heater_rows + p->ny;
  s->Tc = orc_Tc(p);
  s->kappa = pr_kappa(p);
  build_minv(s->Minv);
  if (p->n_sites > 0) {
    s->site_store = (double *)malloc(sizeof(double) * 3 * p->n_sites);
    memcpy(s->site_store, p->site_xc, sizeof(double) * p->n_sites);
    memcpy(s->site_store + p->n_sites, p->site_width, sizeof(double) * p->n_sites);
    memcpy(s->site_store + 2 * p->n_sites, p->site_gmin, sizeof(double) * p->n_sites);
    s->p.site_xc = s->site_store;
    s->p.site_width = s->site_store + p->n_sites;
    s->p.site_gmin = s->site_store + 2 * p->n_sites;
  }
  size_t N = (size_t)s->nx * s->ny, NT = (size_t)s->nx * s->nT;
  s->f = (double *)calloc(9 * N, sizeof(double));
  s->fnew = (double *)calloc(9 * N, sizeof(double));
  double **fields[] = {&s->rho, &s->psi, &s->ux, &s->uy, &s->Fx, &s->Fy, &s->Fmx, &s->Fmy};
  for (int k = 0; k < 8; ++k) *fields[k] = (double *)calloc(N, sizeof(double));
  double **tf[] = {&s->T, &s->Tn, &s->Y, &s->h1, &s->h2, &s->h3, &s->h4};
  for (int k = 0; k < 7; ++k) *tf[k] = (double *)calloc(NT, sizeof(double));
  s->Gw = (double *)calloc(s->nx, sizeof(double));
  build_gw(s);
  /* Initial populations: equilibrium at rest with the given density. */
  for (size_t n = 0; n < N; ++n) {
    double out[9];
    orc_feq(rho0[n], 0.0, 0.0, out);
    for (int i = 0; i < 9; ++i) s->f[i * N + n] = out[i];
    s->rho[n] = rho0[n];
  }
  memcpy(s->T, T0, NT * sizeof(double));
  s->obs.first_bad_step = -1;
  /* initial mass */
  double m = 0.0;
  for (size_t n = 0; n < N; ++n) {
    double r = 0.0;
    for (int i = 0; i < 9; ++i) r += s->f[i * N + n];
    m += r;
  }
  s->obs.mass = m;
  return s;
}

void orc_destroy(orc_sim *s) {
  if (!s) return;
  free(s->site_store);
  free(s->f);
  free(s->fnew);
  free(s->rho);
  free(s->psi);
  free(s->ux);
  free(s->uy);
  free(s->Fx);
  free(s->Fy);
  free(s->Fmx);
  free(s->Fmy);
  free(s->T);
  free(s->Tn);
  free(s->Y);
  free(s->h1);
  free(s->h2);
  free(s->h3);
  free(s->h4);
  free(s->Gw);
  free(s);
}

double *orc_field(orc_sim *s, int field) {
  switch (field) {
    case ORC_FIELD_F: return s->f;
    case ORC_FIELD_RHO: return s->rho;
    case ORC_FIELD_UX: return s->ux;
    case ORC_FIELD_UY: return s->uy;
    case ORC_FIELD_T: return s->T;
    case ORC_FIELD_PSI: return s->psi;
    case ORC_FIELD_FX: return s->Fx;
    case ORC_FIELD_FY: return s->Fy;
    case ORC_FIELD_FMX: return s->Fmx;
    case ORC_FIELD_FMY: return s->Fmy;
    case ORC_FIELD_GW: return s->Gw;
    default: return NULL;
  }
}

int64_t orc_field_len(const orc_sim *s, int field) {
  int64_t N = (int64_t)s->nx * s->ny;
  switch (field) {
    case ORC_FIELD_F: return 9 * N;
    case ORC_FIELD_T: return (int64_t)s->nx * s->nT;
    case ORC_FIELD_GW: return s->nx;
    default: return (field >= 1 && field <= 9) ? N : 0;
  }
}

void orc_observe(const orc_sim *s, orc_obs *out) { *out = s->obs; }

static void flag_error(orc_sim *s, int bits) {
  if (s->obs.error_flags == 0) s->obs.first_bad_step = s->obs.step;
  s->obs.error_flags |= bits;
}

/* ------------------------------------------------------------------------- */
/* Step part 1: density and effective density (Eq. 5, Eq. 7, Eq. 28).        */
/* ------------------------------------------------------------------------- */

void orc_moments(orc_sim *s) {
  const orc_params *p = &s->p;
  int nx = s->nx, ny = s->ny, nh = s->nh;
  size_t N = (size_t)nx * ny;
  int bad = 0;
#pragma omp parallel for reduction(| : bad)
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      size_t n = (size_t)y * nx + x;
      double r = 0.0;
      for (int i = 0; i < 9; ++i) r += s->f[i * N + n];
      s->rho[n] = r;
      double TE = (p->flags & ORC_FREEZE_EOS_T) ? p->T_sat : s->T[(size_t)(y + nh) * nx + x];
      if (!isfinite(r) || !isfinite(TE)) {
        bad |= ORC_ERR_NONFINITE;
        s->psi[n] = 0.0;
        continue;
      }
      if (r <= 0.0) bad |= ORC_ERR_RHO;
      if (1.0 - p->b * r <= 0.0) bad |= ORC_ERR_COVOLUME;
      double rad = 2.0 * (orc_eos_p(p, r, TE) - r / 3.0) / p->G;
      if (!(rad > 0.0)) {
        bad |= ORC_ERR_RADICAND;
        s->psi[n] = 0.0;
        continue;
      }
      s->psi[n] = sqrt(rad);
    }
  }
  if (bad) flag_error(s, bad);
}

/* ------------------------------------------------------------------------- */
/* Step part 2: forces, Eq. 6, Eq. 9, Eq. 10.                                 */
/* ------------------------------------------------------------------------- */

void orc_forces(orc_sim *s) {
  const orc_params *p = &s->p;
  int nx = s->nx, ny = s->ny;
  /* Eq. 9: rho_ave is the mean density of the fluid domain at this step. */
  double msum = 0.0;
  for (size_t n = 0; n < (size_t)nx * ny; ++n) msum += s->rho[n];
  s->rho_ave = msum / ((double)nx * ny);
#pragma omp parallel for
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      size_t n = (size_t)y * nx + x;
      double psic = s->psi[n];
      double sx = 0.0, sy = 0.0, ax = 0.0, ay = 0.0;
      for (int i = 1; i < 9; ++i) {
        int xx = wrapx(x + EX[i], nx), yy = y + EY[i];
        double pn, gw = 0.0;
        int solid = 0;
        if (yy < 0) {
          /* bottom wall / heater surface: a solid neighbour carries psi(x) in Eq. 6,
           * so that a uniform fluid next to a wall feels no interaction force */
          pn = psic;
          gw = s->Gw[xx];
          solid = 1;
        } else if (yy >= ny) {
          if (p->top_bc == ORC_TOP_WALL) {
            pn = psic;
            gw = p->Gw_top;
            solid = 1;
          } else {
            pn = s->psi[(size_t)(ny - 1) * nx + xx]; /* zero-gradient ghost row */
          }
        } else {
          pn = s->psi[(size_t)yy * nx + xx];
        }
        sx += WPSI[i] * pn * EX[i];
        sy += WPSI[i] * pn * EY[i];
        if (solid) {
          /* Eq. 10 weights: omega_a = w_a / 3 with w_a the Eq. 6 weights */
          ax += (WPSI[i] / 3.0) * gw * EX[i];
          ay += (WPSI[i] / 3.0) * gw * EY[i];
        }
      }
      /* Eq. 6 with the sign that makes it consistent with Eq. 7: F_m = -G psi sum w psi e */
      double fmx = -p->G * psic * sx, fmy = -p->G * psic * sy;
      /* Eq. 10: F_ads = G_w psi(x) sum omega S(x+e) e with S(x+e) = psi(x) s(x+e) and
       * omega = w/3 (1/9 axis, 1/36 diagonal); G_w is the strength of the solid
       * neighbour (it varies over the nucleation sites). */
      double fax = psic * psic * ax, fay = psic * psic * ay;
      /* Eq. 9: buoyancy, gravity along -y */
      double fbx = 0.0, fby = -(s->rho[n] - s->rho_ave) * p->g;
      s->Fmx[n] = fmx;
      s->Fmy[n] = fmy;
      s->Fx[n] = fmx + fax + fbx;
      s->Fy[n] = fmy + fay + fby;
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Step part 3: collision and streaming, Eq. 1-2, boundaries of Sec. 3.3, 4.2 */
/* ------------------------------------------------------------------------- */

static void collide_stream(orc_sim *s) {
  const orc_params *p = &s->p;
  int nx = s->nx, ny = s->ny;
  size_t N = (size_t)nx * ny;
#pragma omp parallel for
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      size_t n = (size_t)y * nx + x;
      double f[9], fp[9], ux, uy;
      for (int i = 0; i < 9; ++i) f[i] = s->f[i * N + n];
      collide(p, s->Minv, f, s->Fx[n], s->Fy[n], s->Fmx[n], s->Fmy[n], s->psi[n], fp, &ux, &uy);
      s->ux[n] = ux;
      s->uy[n] = uy;
      for (int i = 0; i < 9; ++i) {
        int xx = wrapx(x + EX[i], nx), yy = y + EY[i];
        if (yy < 0 || (yy >= ny && p->top_bc == ORC_TOP_WALL)) {
          /* half-way bounce-back: the population returns reversed to its node */
          s->fnew[OPP[i] * N + n] = fp[i];
        } else if (yy >= ny) {
          /* leaves through the open top */
        } else {
          s->fnew[i * N + (size_t)yy * nx + xx] = fp[i];
        }
      }
    }
  }
  if (p->top_bc != ORC_TOP_WALL) {
    /* The populations entering the top row from above (directions 4, 7, 8). */
    static const int IN[3] = {4, 7, 8};
    size_t top = (size_t)(ny - 1) * nx, below = (size_t)(ny - 2) * nx;
    if (p->top_bc == ORC_TOP_CONST_PRESSURE) {
      /* constant pressure (Sec. 3.3): equilibrium at rho_v with the velocity of the
       * row below */
      for (int x = 0; x < nx; ++x) {
        double fe[9];
        orc_feq(p->rho_v, s->ux[below + x], s->uy[below + x], fe);
        for (int k = 0; k < 3; ++k) s->fnew[IN[k] * N + top + x] = fe[IN[k]];
      }
    } else {
      /* convective outlet (Sec. 4.2): df/dt + U df/dy = 0 discretised implicitly,
       * f^{n+1}(top) = (f^n(top) + U f^{n+1}(top-1)) / (1 + U), with U the mean
       * outflow velocity of the row below (zero if that mean points inward). */
      double U = 0.0;
      for (int x = 0; x < nx; ++x) U += s->uy[below + x];
      U /= nx;
      if (U < 0.0) U = 0.0;
      for (int x = 0; x < nx; ++x)
        for (int k = 0; k < 3; ++k) {
          size_t i = IN[k];
          s->fnew[i * N + top + x] = (s->f[i * N + top + x] + U * s->fnew[i * N + below + x]) / (1.0 + U);
        }
    }
  }
  double *t = s->f;
  s->f = s->fnew;
  s->fnew = t;
}

/* ------------------------------------------------------------------------- */
/* Step part 4: energy equation, Eq. 17-27.                                   */
/* ------------------------------------------------------------------------- */

static double lam_at(const orc_sim *s, int j, int x) {
  /* lambda = rho c_v k in the fluid (Sec. 3.1); the heater has its own lambda_w. */
  if (j < s->nh) return s->p.lambda_w;
  return s->rho[(size_t)(j - s->nh) * s->nx + x] * s->p.cv * s->p.k;
}

static double rhoc_at(const orc_sim *s, int j, int x) {
  if (j < s->nh) return s->p.rho_w * s->p.cv_w;
  return s->rho[(size_t)(j - s->nh) * s->nx + x] * s->p.cv;
}

/* Eq. 25: harmonic-mean face conductivity (dx = 1). */
static double face_lambda(double lp, double ln) { return 2.0 / (1.0 / lp + 1.0 / ln); }

/* Temperature seen by a stencil at T row j (ghost rows below and above). */
static double T_at(const orc_sim *s, const double *Y, int j, int x) {
  const orc_params *p = &s->p;
  if (j < 0) {
    if (p->bottom_tbc == ORC_TBC_FLUX) return Y[x] + p->q_bottom / lam_at(s, 0, x);
    return p->T_bottom;
  }
  if (j >= s->nT) {
    if (p->top_tbc == ORC_TBC_DIRICHLET) return p->T_top;
    return Y[(size_t)(s->nT - 1) * s->nx + x];
  }
  return Y[(size_t)j * s->nx + x];
}

/* Velocity seen by the divergence stencil at fluid row y: zero on solids, a
 * zero-gradient ghost above an open top. */
static double u_at(const orc_sim *s, const double *u, int y, int x) {
  if (y < 0) return 0.0;
  if (y >= s->ny) {
    if (s->p.top_bc == ORC_TOP_WALL) return 0.0;
    y = s->ny - 1;
  }
  return u[(size_t)y * s->nx + x];
}

static double lam_ghost(const orc_sim *s, int j, int x) {
  if (j < 0) j = 0;
  if (j >= s->nT) j = s->nT - 1;
  return lam_at(s, j, x);
}

/* Eq. 19: isotropic central gradient of a field given by an accessor. */
typedef double (*acc_fn)(const orc_sim *, const double *, int, int);

static void grad19(const orc_sim *s, acc_fn F, const double *arr, int j, int x, double *gx,
                   double *gy) {
  int nx = s->nx;
  int xp = wrapx(x + 1, nx), xm = wrapx(x - 1, nx);
  double E = F(s, arr, j, xp), W = F(s, arr, j, xm), N = F(s, arr, j + 1, x), S = F(s, arr, j - 1, x);
  double NE = F(s, arr, j + 1, xp), SW = F(s, arr, j - 1, xm);
  double SE = F(s, arr, j - 1, xp), NW = F(s, arr, j + 1, xm);
  *gx = (E - W) / 3.0 + (NE - SW) / 12.0 + (SE - NW) / 12.0;
  *gy = (N - S) / 3.0 + (NE - SW) / 12.0 + (NW - SE) / 12.0;
}

static double T_acc(const orc_sim *s, const double *Y, int j, int x) { return T_at(s, Y, j, x); }
static double ux_acc(const orc_sim *s, const double *u, int j, int x) {
  (void)u;
  return u_at(s, s->ux, j - s->nh, x);
}
static double uy_acc(const orc_sim *s, const double *u, int j, int x) {
  (void)u;
  return u_at(s, s->uy, j - s->nh, x);
}
static double lam_acc(const orc_sim *s, const double *u, int j, int x) {
  (void)u;
  return lam_ghost(s, j, x);
}

/*
 * K(T) of Eq. 17 on every heater and fluid node for the stage field Y:
 *   K = -u.grad T + (1/(rho c_v)) div(lambda grad T) - (T/(rho c_v)) (dp/dT)_v div u
 * with the diffusion term by the finite-volume form Eq. 22-26 (or Eq. 20-21 when
 * ORC_DIFF_ISOTROPIC is set) and gradients by Eq. 19.  Heater nodes conduct only.
 * flux[0..2] receive the heat entering through the bottom boundary, the top boundary
 * and the heater/fluid surface, per unit time, summed over x.
 */
void orc_energy_rhs(orc_sim *s, const double *Y, double *K, double flux[3]) {
  const orc_params *p = &s->p;
  int nx = s->nx, nT = s->nT, nh = s->nh;
  int iso = (p->flags & ORC_DIFF_ISOTROPIC) != 0;
#pragma omp parallel for
  for (int j = 0; j < nT; ++j) {
    for (int x = 0; x < nx; ++x) {
      size_t P = (size_t)j * nx + x;
      double lp = lam_at(s, j, x), cp = rhoc_at(s, j, x), TP = Y[P];
      double D;
      if (!iso) {
        /* Eq. 22-26: heat entering the control volume through its four faces */
        int xp = wrapx(x + 1, nx), xm = wrapx(x - 1, nx);
        double qe = face_lambda(lp, lam_at(s, j, xp)) * (Y[(size_t)j * nx + xp] - TP);
        double qw = face_lambda(lp, lam_at(s, j, xm)) * (Y[(size_t)j * nx + xm] - TP);
        double qn, qs;
        if (j + 1 < nT) qn = face_lambda(lp, lam_at(s, j + 1, x)) * (Y[P + nx] - TP);
        else if (p->top_tbc == ORC_TBC_DIRICHLET) qn = lp * (p->T_top - TP); /* ghost at dx, face lambda = lambda_P */
        else qn = 0.0;                                                       /* zero gradient */
        if (j - 1 >= 0) qs = face_lambda(lp, lam_at(s, j - 1, x)) * (Y[P - nx] - TP);
        else if (p->bottom_tbc == ORC_TBC_FLUX) qs = p->q_bottom;
        else qs = lp * (p->T_bottom - TP);
        D = qe + qw + qn + qs;
      } else {
        /* Eq. 21 with Eq. 19-20: lambda Lap T + grad lambda . grad T */
        int xp = wrapx(x + 1, nx), xm = wrapx(x - 1, nx);
        double lap = (T_at(s, Y, j + 1, xp) + T_at(s, Y, j + 1, xm) + T_at(s, Y, j - 1, xp) +
                      T_at(s, Y, j - 1, xm) + 4.0 * T_at(s, Y, j, xp) + 4.0 * T_at(s, Y, j, xm) +
                      4.0 * T_at(s, Y, j + 1, x) + 4.0 * T_at(s, Y, j - 1, x) - 20.0 * TP) /
                     6.0;
        double tgx, tgy, lgx, lgy;
        grad19(s, T_acc, Y, j, x, &tgx, &tgy);
        grad19(s, lam_acc, NULL, j, x, &lgx, &lgy);
        D = lp * lap + (lgx * tgx + lgy * tgy);
      }
      double k = D / cp;
      if (j >= nh) {
        size_t n = (size_t)(j - nh) * nx + x;
        if (!(p->flags & ORC_NO_ADVECTION)) {
          double gx, gy;
          grad19(s, T_acc, Y, j, x, &gx, &gy);
          k += -(s->ux[n] * gx + s->uy[n] * gy);
        }
        if (!(p->flags & ORC_NO_LATENT)) {
          double dux, duy, dvx, dvy;
          grad19(s, ux_acc, NULL, j, x, &dux, &duy);
          grad19(s, uy_acc, NULL, j, x, &dvx, &dvy);
          double divu = dux + dvy;
          k += -(TP / cp) * orc_dpdT(p, s->rho[n], TP) * divu;
        }
      }
      K[P] = k;
    }
  }
  /* boundary heat, in a fixed order */
  double fb = 0.0, ft = 0.0, fs = 0.0;
  for (int x = 0; x < nx; ++x) {
    double lp = lam_at(s, 0, x), T0 = Y[x];
    fb += (p->bottom_tbc == ORC_TBC_FLUX) ? p->q_bottom : lp * (p->T_bottom - T0);
    if (p->top_tbc == ORC_TBC_DIRICHLET) {
      size_t P = (size_t)(nT - 1) * nx + x;
      ft += lam_at(s, nT - 1, x) * (p->T_top - Y[P]);
    }
    if (nh > 0) {
      /* heat from the top heater row into fluid row 0 through their common face */
      size_t Ph = (size_t)(nh - 1) * nx + x, Pf = (size_t)nh * nx + x;
      fs += face_lambda(lam_at(s, nh, x), lam_at(s, nh - 1, x)) * (Y[Ph] - Y[Pf]);
    }
  }
  if (nh == 0) fs = fb;
  flux[0] = fb;
  flux[1] = ft;
  flux[2] = fs;
}

/* Eq. 18 (classical RK4) applied N times with dt_T = dt/N (Eq. 27). */
void orc_energy_update(orc_sim *s) {
  const orc_params *p = &s->p;
  size_t NT = (size_t)s->nx * s->nT;
  double dt = 1.0 / p->n_sub;
  for (int sub = 0; sub < p->n_sub; ++sub) {
    double f1[3], f2[3], f3[3], f4[3];
    orc_energy_rhs(s, s->T, s->h1, f1);
    for (size_t P = 0; P < NT; ++P) s->Y[P] = s->T[P] + 0.5 * dt * s->h1[P];
    orc_energy_rhs(s, s->Y, s->h2, f2);
    for (size_t P = 0; P < NT; ++P) s->Y[P] = s->T[P] + 0.5 * dt * s->h2[P];
    orc_energy_rhs(s, s->Y, s->h3, f3);
    for (size_t P = 0; P < NT; ++P) s->Y[P] = s->T[P] + dt * s->h3[P];
    orc_energy_rhs(s, s->Y, s->h4, f4);
    double dE = 0.0;
    for (int j = 0; j < s->nT; ++j)
      for (int x = 0; x < s->nx; ++x) {
        size_t P = (size_t)j * s->nx + x;
        double Tn = s->T[P] + dt / 6.0 * (s->h1[P] + 2.0 * s->h2[P] + 2.0 * s->h3[P] + s->h4[P]);
        dE += rhoc_at(s, j, x) * (Tn - s->T[P]);
        s->Tn[P] = Tn;
      }
    double *t = s->T;
    s->T = s->Tn;
    s->Tn = t;
    double Qb = dt / 6.0 * (f1[0] + 2.0 * f2[0] + 2.0 * f3[0] + f4[0]);
    double Qt = dt / 6.0 * (f1[1] + 2.0 * f2[1] + 2.0 * f3[1] + f4[1]);
    double Qs = dt / 6.0 * (f1[2] + 2.0 * f2[2] + 2.0 * f3[2] + f4[2]);
    s->obs.Q_bottom_cum += Qb;
    s->obs.Q_top_cum += Qt;
    s->obs.Q_surface_cum += Qs;
    s->obs.dE_cum += dE;
    s->obs.q_bottom += Qb; /* per-LB-step accumulators, normalised in orc_step */
    s->obs.q_surface += Qs;
  }
}

/* ------------------------------------------------------------------------- */
/* One full step: moments, forces, collide-stream, energy, diagnostics.       */
/* ------------------------------------------------------------------------- */

int orc_step(orc_sim *s, int64_t nsteps) {
  int nx = s->nx, ny = s->ny;
  size_t N = (size_t)nx * ny;
  for (int64_t it = 0; it < nsteps; ++it) {
    if (s->obs.error_flags) return -4;
    orc_moments(s);
    if (s->obs.error_flags) return -4;
    orc_forces(s);
    collide_stream(s);
    /* the energy update of this step uses rho^n and u^n of this collision */
    s->obs.q_bottom = 0.0;
    s->obs.q_surface = 0.0;
    orc_energy_update(s);
    s->obs.q_bottom /= nx;
    s->obs.q_surface /= nx;
    /* diagnostics */
    double m = 0.0, vmax = 0.0;
    for (size_t n = 0; n < N; ++n) {
      double r = 0.0;
      for (int i = 0; i < 9; ++i) r += s->f[i * N + n];
      m += r;
      double sp = sqrt(s->ux[n] * s->ux[n] + s->uy[n] * s->uy[n]);
      if (sp > vmax) vmax = sp;
    }
    double E = 0.0;
    int nT = s->nT, bad = !isfinite(m);
    for (int j = 0; j < nT; ++j)
      for (int x = 0; x < nx; ++x) {
        double t = s->T[(size_t)j * nx + x];
        if (!isfinite(t)) bad = 1;
        E += rhoc_at(s, j, x) * t;
      }
    if (bad) {
      flag_error(s, ORC_ERR_NONFINITE);
      return -4;
    }
    s->obs.step += 1;
    s->obs.mass = m;
    s->obs.energy = E;
    s->obs.rho_ave = s->rho_ave;
    s->obs.max_speed = vmax;
    /* Welford running mean / population variance of the bottom heat flux */
    double cnt = (double)s->obs.step, q = s->obs.q_bottom;
    double d = q - s->obs.q_bottom_mean;
    s->obs.q_bottom_mean += d / cnt;
    s->welford_m2 += d * (q - s->obs.q_bottom_mean);
    s->obs.q_bottom_var = s->welford_m2 / cnt;
  }
  return 0;
}
