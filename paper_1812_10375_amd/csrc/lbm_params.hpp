// lbm_params.hpp -- kernel parameter block and device diagnostics record, shared by
// the kernels and the host code of the hybrid thermal pseudo-potential LB library.
#pragma once

namespace lbmk {


enum { TOP_WALL = 0, TOP_CONST_PRESSURE = 1, TOP_CONVECTIVE = 2 };
enum { TBC_DIRICHLET = 0, TBC_FLUX = 1, TBC_ZERO_GRAD = 2 };
enum { FREEZE_EOS_T = 1, NO_ADVECTION = 2, NO_LATENT = 4, DIFF_ISOTROPIC = 8 };
enum { ERR_RHO = 1, ERR_COVOLUME = 2, ERR_RADICAND = 4, ERR_NONFINITE = 8, ERR_SYNC = 16 };

constexpr int NT = 256;  // threads per block in every kernel

struct KParams {
  int nx, ny, nh, nT;
  int flags, top_bc, bottom_tbc, top_tbc;
  int ntxL, ntyL, nblkL, tyL;
  int ntxE, ntyE, nblkE, tyE, txE, tyE0;  // energy tiles: first tile row tyE0 rows, then tyE
  // equation of state (FP64)
  double a, b, R, G, Tc, inv_Tc, kappa, phi_sat, T_sat, inv3, two_G;
  // collision
  double rho_l, rho_v, inv_drho, tau_v, dtau;
  double s_e, s_z, s_q, c_e, c_z, c_q, sig_e, sig_z;
  double g, Gw_top;
  // energy
  double cv, k, cvk, rcw, inv_rcw, lambda_w, T_bottom, T_top, q_bottom;
  double sigma, tau_l, s_e_raw, s_z_raw;
  // FP32 energy kernel constants: 2k, R/c_v, a kappa^2/(T_c c_v), a kappa (1 + kappa)/(sqrt(T_c) c_v),
  // kappa^2/T_c, kappa (1 + kappa)/sqrt(T_c)
  float e_k2, e_g1a, e_g1b, e_g2a, e_kk2, e_kl2;
};

struct DevDiag {
  double mass, rho_ave, max_speed, energy, q_bottom, q_surface;
  double Q_bottom_cum, Q_top_cum, Q_surface_cum, dE_cum, q_mean, q_m2;
  long long nred;  // steps folded into the running statistics
  unsigned int err;
  int pad;
  unsigned long long first_bad;
};

// Byte offsets of the arrays carved out of a domain's workspace.
struct Layout {
  size_t f[2], T[2], rho, ux, uy, topin, gw, partL[2], pmin[2], mstate[2], dstep[2], hist, steps, diag, cdone, order,
      total;
};

// One domain of a batch, as the batched kernels see it (device memory).  tile0L and
// tile0E are the domain's first tile in the batch's collide and energy grids.
struct DomainDev {
  KParams P;
  Layout L;
  char* ws;
  int tile0L, tile0E;
};

}  // namespace lbmk
