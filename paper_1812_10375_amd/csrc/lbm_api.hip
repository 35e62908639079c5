// lbm_api.hip -- host side of the C ABI declared in include/lbm_api.h: validation,
// workspace carving, the wall profile, and the entry points.  Kernel launches live in
// lbm_f32.hip / lbm_f64.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <new>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "lbm_api.h"
#include "lbm_ctx.hpp"

using lbmk::DevDiag;
using lbmk::KParams;
using namespace lbmh;

namespace {

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

bool valid_config(const lbm_config* c) {
  if (!c) return false;
  if (c->struct_size != sizeof(lbm_config) || c->abi_version != LBM_ABI_VERSION) return false;
  if (c->nx < 1 || c->ny < 1 || c->heater_rows < 0 || c->n_sub < 1) return false;
  if (c->nx > (1 << 20) || c->ny > (1 << 20) || c->heater_rows > (1 << 20)) return false;
  if (c->precision != LBM_F32 && c->precision != LBM_F64) return false;
  // one field plane is addressed with 32-bit byte offsets
  const double vbytes = c->precision == LBM_F64 ? 8.0 : 4.0;
  if ((double)c->nx * (double)(c->ny + c->heater_rows) * vbytes >= 4294967296.0) return false;
  if (c->top_bc < LBM_TOP_WALL || c->top_bc > LBM_TOP_CONVECTIVE) return false;
  if (c->top_bc != LBM_TOP_WALL && c->ny < 2) return false;
  if (c->bottom_tbc != LBM_TBC_DIRICHLET && c->bottom_tbc != LBM_TBC_FLUX) return false;
  if (c->top_tbc != LBM_TBC_DIRICHLET && c->top_tbc != LBM_TBC_ZERO_GRAD) return false;
  if (c->flags & ~(15u | LBM_TWO_LAUNCHES | LBM_ONE_LAUNCH)) return false;
  if ((c->flags & LBM_TWO_LAUNCHES) && (c->flags & LBM_ONE_LAUNCH)) return false;
  if (c->tile_rows < 0) return false;
  if (!(c->a > 0 && c->b > 0 && c->R > 0 && c->T_sat > 0 && c->G < 0)) return false;
  if (!(c->tau_l > 0.5 && c->tau_v > 0.5 && c->s_e > 0 && c->s_e < 2 && c->s_zeta > 0 &&
        c->s_zeta < 2 && c->s_q > 0 && c->s_q < 2))
    return false;
  if (!(c->rho_l > c->rho_v && c->rho_v > 0)) return false;
  if (!(c->cv > 0 && c->k > 0)) return false;
  if (c->heater_rows > 0 && !(c->rho_w > 0 && c->cv_w > 0 && c->lambda_w > 0)) return false;
  if (c->n_sites < 0) return false;
  if (c->n_sites > 0 && (!c->site_xc || !c->site_width || !c->site_gmin)) return false;
  const double vals[] = {c->a, c->b, c->R, c->omega, c->T_sat, c->G, c->sigma, c->g,
                         c->T_bottom, c->T_top, c->q_bottom, c->Gw0, c->Gw_top};
  for (double v : vals)
    if (!std::isfinite(v)) return false;
  return true;
}

// Tile grids.  The collide tiles are fixed (64 x TY).  The energy tiles are as wide
// as the 64-lane LDS rows allow (56 + 8 halo) and, for a device with `ncu` compute
// units, as tall as possible while the tiles still fill every resident workgroup slot
// in one round (at least E_HMIN rows unless the grid is shorter).  ncu = 0 gives the
// largest tile count any device can use (for sizing the workspace).
struct Grids {
  int ntxL, ntyL, ntxE, ntyE, txE, tyE, tyE0;
};

// The FP32 register-row energy kernel runs tiles that reach within four rows of the
// bottom or the top of the temperature grid, or of the heater-fluid interface, through
// its general (per-row) code, about 1.3 times slower per row than the interior tiles.
// With `rows` tile rows, shorten the first and the last tile row to edge heights of
// about the cost of an interior tile, keeping the second tile row clear of the heater
// (first height >= nh + 4) and the second-to-last clear of the top (last height >= 4),
// and make the interior rows just tall enough to cover the grid.  Returns false
// (uniform tiles) when no interior height up to hmax allows this.
bool shape_edge_rows(int nT, int nh, int rows, int hmax, int& ty, int& ty0) {
  if (rows < 3) return false;
  for (int h = (nT + rows - 1) / rows; h <= hmax; ++h) {
    const int cap = std::max(E_HMIN, (10 * (h + 8)) / 13 - 8);
    if (nh + 4 > cap) continue;
    const int edge = nT - (rows - 2) * h;  // rows left for the first and the last tile row
    if (edge < nh + 8) return false;
    if (edge <= 2 * cap) {
      ty = h;
      ty0 = std::max(nh + 4, (edge + 1) / 2);
      return true;
    }
  }
  return false;
}

Grids grids(const lbm_config* c, int ncu) {
  Grids g{};
  const bool f64 = c->precision == LBM_F64;
  const int ty = f64 ? TY_F64 : TY_F32;
  const int nT = c->heater_rows + c->ny;
  g.ntxL = (c->nx + 63) / 64;
  g.ntyL = (c->ny + ty - 1) / ty;
  g.ntxE = (c->nx + E_TXMAX - 1) / E_TXMAX;
  g.txE = (c->nx + g.ntxE - 1) / g.ntxE;
  const int hmax = f64 ? E_HMAX : E_HMAX_F32;
  const int rows_min = (nT + hmax - 1) / hmax;
  const int rows_max = (nT + E_HMIN - 1) / E_HMIN;
  int rows = rows_max;
  if (ncu > 0 && c->tile_rows > 0) {
    // requested tile height, within the kernels' limits
    const int ty = std::min(std::max(c->tile_rows, E_HMIN), hmax);
    rows = std::max(rows_min, std::min(rows_max, (nT + ty - 1) / ty));
  } else if (ncu > 0) {
    const int slots = ncu * (f64 ? E_PER_CU_F64 : E_PER_CU_F32);
    rows = std::max(rows_min, std::min(rows_max, slots / g.ntxE));
  }
  g.tyE = (nT + rows - 1) / rows;
  g.ntyE = (nT + g.tyE - 1) / g.tyE;
  g.tyE0 = g.tyE;
  const bool row_kernel = !f64 && !(c->flags & LBM_DIFF_ISOTROPIC);
  int ty_in, ty_edge;
  if (ncu > 0 && row_kernel && shape_edge_rows(nT, c->heater_rows, g.ntyE, hmax, ty_in, ty_edge)) {
    g.tyE = ty_in;
    g.tyE0 = ty_edge;
  }
  return g;
}

Layout layout(const lbm_config* c) {
  Layout L{};
  const size_t R = c->precision == LBM_F64 ? 8 : 4;
  const size_t nx = c->nx, ny = c->ny, nT = (size_t)c->heater_rows + ny;
  const Grids g = grids(c, 0);  // upper bound on the energy tile count
  const int ntxL = g.ntxL, ntyL = g.ntyL, ntxE = g.ntxE, ntyE = g.ntyE;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.f[0] = take(9 * nx * ny * R);
  L.f[1] = take(9 * nx * ny * R);
  L.T[0] = take(nT * nx * R);
  L.T[1] = take(nT * nx * R);
  L.rho = take(nx * ny * R);
  L.ux = take(nx * ny * R);
  L.uy = take(nx * ny * R);
  L.topin = take(3 * nx * R);
  L.gw = take(nx * R);
  for (int k = 0; k < 2; ++k) L.partL[k] = take((size_t)ntxL * ntyL * 3 * sizeof(double));
  for (int k = 0; k < 2; ++k) L.pmin[k] = take((size_t)ntxE * sizeof(double));
  for (int k = 0; k < 2; ++k) L.mstate[k] = take(sizeof(double));
  for (int k = 0; k < 2; ++k) L.dstep[k] = take(sizeof(long long));
  L.hist = take((size_t)HIST * ntxE * ntyE * 5 * sizeof(double));
  L.steps = take((size_t)HIST * 5 * sizeof(double));
  L.diag = take(sizeof(DevDiag));
  L.cdone = take((size_t)ntxL * ntyL * sizeof(unsigned));
  L.order = take((size_t)((ntxL * ntyL + 1) / 2 + 1 + ntxE * ntyE) * sizeof(int));
  L.total = off;
  return L;
}

// Wall strength of each bottom-wall column (Eq. 10 with the nucleation sites of
// Sec. 4.2): a site of width W centred at xc lowers G_w linearly from Gw0 at its
// edges to its minimum at the centre; column c is centred at c + 1/2; x is periodic.
std::vector<double> wall_profile(const lbm_config* c) {
  std::vector<double> gw(c->nx, c->Gw0);
  for (int s = 0; s < c->n_sites; ++s) {
    const double half = 0.5 * c->site_width[s], gmin = c->site_gmin[s], xc = c->site_xc[s];
    for (int x = 0; x < c->nx; ++x) {
      double d = (x + 0.5) - xc;
      d -= c->nx * std::floor(d / c->nx + 0.5);
      const double ad = std::fabs(d);
      if (ad < half) gw[x] = std::min(gw[x], gmin + (c->Gw0 - gmin) * (ad / half));
    }
  }
  return gw;
}

KParams make_params(const lbm_config* c, int ncu) {
  KParams P{};
  P.nx = c->nx;
  P.ny = c->ny;
  P.nh = c->heater_rows;
  P.nT = c->heater_rows + c->ny;
  P.flags = (int)c->flags;
  P.top_bc = c->top_bc;
  P.bottom_tbc = c->bottom_tbc;
  P.top_tbc = c->top_tbc;
  const Grids g = grids(c, ncu);
  P.ntxL = g.ntxL;
  P.ntyL = g.ntyL;
  P.ntxE = g.ntxE;
  P.ntyE = g.ntyE;
  P.txE = g.txE;
  P.tyE = g.tyE;
  P.tyE0 = g.tyE0;
  P.nblkL = P.ntxL * P.ntyL;
  P.nblkE = P.ntxE * P.ntyE;
  P.tyL = c->precision == LBM_F64 ? TY_F64 : TY_F32;
  // Eq. 28 and Sec. 3.1: a = 0.45724 R^2 Tc^2 / pc, b = 0.0778 R Tc / pc
  const double Tc = (c->a / c->b) * (0.0778 / 0.45724) / c->R;
  const double kap = 0.37464 + 1.54226 * c->omega - 0.26992 * c->omega * c->omega;
  P.a = c->a;
  P.b = c->b;
  P.R = c->R;
  P.G = c->G;
  P.Tc = Tc;
  P.inv_Tc = 1.0 / Tc;
  P.kappa = kap;
  const double ssat = 1.0 + kap * (1.0 - std::sqrt(c->T_sat / Tc));
  P.phi_sat = ssat * ssat;
  P.T_sat = c->T_sat;
  P.inv3 = 1.0 / 3.0;
  P.two_G = 2.0 / c->G;
  P.rho_l = c->rho_l;
  P.rho_v = c->rho_v;
  P.inv_drho = 1.0 / (c->rho_l - c->rho_v);
  P.tau_v = c->tau_v;
  P.dtau = c->tau_l - c->tau_v;
  P.s_e = c->s_e;
  P.s_z = c->s_zeta;
  P.s_q = c->s_q;
  P.c_e = 1.0 - 0.5 * c->s_e;
  P.c_z = 1.0 - 0.5 * c->s_zeta;
  P.c_q = 1.0 - 0.5 * c->s_q;
  // Eq. 8 sigma terms: 12 sigma |F_m|^2 / (psi^2 (tau - 1/2)) with tau = 1/s
  P.sig_e = 12.0 * c->sigma / (1.0 / c->s_e - 0.5);
  P.sig_z = 12.0 * c->sigma / (1.0 / c->s_zeta - 0.5);
  P.g = c->g;
  P.Gw_top = c->Gw_top;
  P.cv = c->cv;
  P.k = c->k;
  P.cvk = c->cv * c->k;
  P.sigma = c->sigma;
  P.tau_l = c->tau_l;
  P.s_e_raw = c->s_e;
  P.s_z_raw = c->s_zeta;
  P.rcw = c->rho_w * c->cv_w;
  P.inv_rcw = P.rcw > 0 ? 1.0 / P.rcw : 0.0;
  P.lambda_w = c->lambda_w;
  P.T_bottom = c->T_bottom;
  P.T_top = c->T_top;
  P.q_bottom = c->q_bottom;
  P.e_k2 = (float)(2.0 * c->k);
  P.e_g1a = (float)(P.R / c->cv);
  P.e_g1b = (float)(P.a * kap * kap / Tc / c->cv);
  P.e_g2a = (float)(P.a * kap * (1.0 + kap) / std::sqrt(Tc) / c->cv);
  P.e_kk2 = (float)(kap * kap / Tc);
  P.e_kl2 = (float)(kap * (1.0 + kap) / std::sqrt(Tc));
  return P;
}

int hip_ok(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EHIP; }

// Work order of the fused FP32 step's grid (block b takes item order[b]): the collide
// items first (item c runs collide tiles 2c and 2c + 1), then the outlet block, then the
// energy tiles.  Both kinds are laid out as xcd_tile lays out a grid: the dispatcher
// sends block 8p + k to XCD k, and each XCD gets a contiguous band of collide items and
// the matching band of energy tiles, so an energy tile's halo is mostly in its XCD's L2
// and its collide neighbours finish early on the same XCD.  (Bottom-up row orders,
// measured, were 8-18% slower.)
std::vector<int> fused_order(const KParams& P) {
  const int npair = (P.nblkL + 1) / 2;
  auto band = [](int b, int n) {
    const int q = n >> 3, r = n & 7, k = b & 7;
    return k * q + (k < r ? k : r) + (b >> 3);
  };
  std::vector<int> order;
  order.reserve((size_t)npair + 1 + P.nblkE);
  for (int c = 0; c < npair; ++c) order.push_back(band(c, npair));
  order.push_back(npair);
  for (int e = 0; e < P.nblkE; ++e) order.push_back(npair + 1 + band(e, P.nblkE));
  return order;
}

}  // namespace

namespace lbmh {
int timing_begin(lbm_ctx* h, int kind) {
  if (!h->timing) return -1;
  if (h->ev_used + 2 > h->ev_pool.size()) {
    for (int i = 0; i < 2; ++i) {
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return -1;
      h->ev_pool.push_back(e);
    }
  }
  const int idx = (int)h->ev_used;
  h->ev_used += 2;
  h->ev_kind.push_back(kind);
  (void)hipEventRecord(h->ev_pool[idx], h->stream);
  return idx;
}
void timing_end(lbm_ctx* h, int idx) {
  if (idx >= 0) (void)hipEventRecord(h->ev_pool[idx + 1], h->stream);
}
}  // namespace lbmh

extern "C" {

size_t lbm_workspace_bytes(const lbm_config* cfg) {
  if (!valid_config(cfg)) return 0;
  return layout(cfg).total;
}

int lbm_init(const lbm_config* cfg, void* d_workspace, size_t ws_bytes, void* hip_stream,
             const double* rho0_host, const double* T0_host, lbm_ctx** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  if (!valid_config(cfg) || !d_workspace || !rho0_host || !T0_host) return LBM_EINVAL;
  if (reinterpret_cast<uintptr_t>(d_workspace) & 255) return LBM_EINVAL;
  Layout L = layout(cfg);
  if (ws_bytes < L.total) return LBM_ENOMEM;
  lbm_ctx* h = new (std::nothrow) lbm_ctx();
  if (!h) return LBM_ENOMEM;
  h->cfg = *cfg;
  h->cfg.n_sites = 0;  // the site table is consumed here (wall profile); do not keep host pointers
  h->cfg.site_xc = h->cfg.site_width = h->cfg.site_gmin = nullptr;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    delete h;
    return LBM_EHIP;
  }
  h->ncu = ncu;
  h->P = make_params(cfg, ncu);
  // FP32 with one energy sub-step runs each step as one fused launch when its collide
  // tile pairs fill the device's workgroup slots in one round (3 to 4 collide tiles per
  // CU): then the launch boundary and the collide tail are what the fusion saves.
  // Smaller grids would leave CUs without collide work, and larger ones keep the two
  // launches, whose collide kernel alone holds more waves per SIMD.
  const bool can_fuse = cfg->precision == LBM_F32 && !(cfg->flags & LBM_DIFF_ISOTROPIC) && cfg->n_sub == 1;
  if (cfg->flags & LBM_ONE_LAUNCH) h->fused = can_fuse;
  else if (cfg->flags & LBM_TWO_LAUNCHES) h->fused = false;
  else h->fused = can_fuse && h->P.nblkL > 3 * ncu && h->P.nblkL <= 4 * ncu;
  h->L = L;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  h->ws = reinterpret_cast<char*>(d_workspace);
  h->fcur = 0;
  h->tcur = 0;
  h->step = 0;
  h->bad = false;
  h->timing = false;
  h->ev_used = 0;
  h->hist_first = 0;
  h->hist_count = 0;
  const std::vector<double> gw = wall_profile(cfg);
  int rc = cfg->precision == LBM_F64 ? init_fields<double>(h, rho0_host, T0_host, gw.data())
                                     : init_fields<float>(h, rho0_host, T0_host, gw.data());
  if (!rc) {
    const std::vector<int> order = fused_order(h->P);
    rc = hip_ok(hipMemcpyAsync(h->at<int>(L.order), order.data(), order.size() * sizeof(int),
                               hipMemcpyHostToDevice, h->stream));
    if (!rc) rc = hip_ok(hipStreamSynchronize(h->stream));  // `order` is freed on return
  }
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return LBM_OK;
}

int lbm_step(lbm_ctx* h, int64_t nsteps) {
  if (!h || nsteps < 0) return LBM_EINVAL;
  if (h->bad) return LBM_ESTATE;
  for (int64_t s = 0; s < nsteps; ++s) {
    if (h->cfg.precision == LBM_F64) step_once<double>(h);
    else step_once<float>(h);
  }
  return hip_ok(hipGetLastError());
}

int lbm_set_stream(lbm_ctx* h, void* hip_stream) {
  if (!h) return LBM_EINVAL;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return LBM_OK;
}

// Copies the folded diagnostics of h to the host (synchronises the stream).
static int read_observation(lbm_ctx* h, lbm_obs* out) {
  const Layout& L = h->L;
  DevDiag* dd = h->at<DevDiag>(L.diag);
  DevDiag d;
  long long dstep = 0;
  // the device's step counter is authoritative: graph replays advance it without the host
  const int last = (int)((h->step + 1) & 1);
  if (hipMemcpyAsync(&d, dd, sizeof(d), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
      hipMemcpyAsync(&dstep, h->at<long long>(L.dstep[last]), sizeof(dstep), hipMemcpyDeviceToHost,
                     h->stream) != hipSuccess)
    return LBM_EHIP;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return LBM_EHIP;
  h->step = (int64_t)dstep;
  std::memset(out, 0, sizeof(*out));
  out->step = h->step;
  out->mass = d.mass;
  out->energy = d.energy;
  out->rho_ave = d.rho_ave;
  out->q_bottom = d.q_bottom;
  out->q_bottom_mean = d.q_mean;
  out->q_bottom_var = d.nred > 0 ? d.q_m2 / (double)d.nred : 0.0;
  out->q_surface = d.q_surface;
  out->Q_bottom_cum = d.Q_bottom_cum;
  out->Q_top_cum = d.Q_top_cum;
  out->Q_surface_cum = d.Q_surface_cum;
  out->dE_cum = d.dE_cum;
  out->max_speed = d.max_speed;
  out->error_flags = (int32_t)d.err;
  out->first_bad_step = d.err ? (int64_t)d.first_bad : -1;
  if (d.err) {
    h->bad = true;
    return LBM_ENONFINITE;
  }
  return LBM_OK;
}

int lbm_observe(lbm_ctx* h, lbm_obs* out) {
  if (!h || !out) return LBM_EINVAL;
  if (h->cfg.precision == LBM_F64) finish_reductions<double>(h);
  else finish_reductions<float>(h);
  return read_observation(h, out);
}

}  // extern "C"

namespace {

// The run state beyond the fields (LBM_FIELD_STATE), as a host record: a header that
// identifies the configuration, the device diagnostics and the carried mass, followed
// by the per-column exchange through the open top of the last step (ntxE doubles) and
// the last collision's per-tile partials (3 nblkL doubles: post-collision mass, largest
// |u|^2, sum of u_y on row ny - 2), from which an observation sums the current mass.
constexpr uint64_t STATE_MAGIC = 0x3154415453424c4dull;  // "MLBSTAT1"
struct StateRecord {
  uint64_t magic;
  int64_t step;
  int32_t nx, ny, nh, ntxE, nblkL;
  int32_t precision;
  lbmk::DevDiag diag;
  double mass_carried;
};

size_t state_bytes(const lbm_ctx* h) {
  return sizeof(StateRecord) + ((size_t)h->P.ntxE + 3 * (size_t)h->P.nblkL) * sizeof(double);
}

int read_state(lbm_ctx* h, void* dst) {
  if (h->hist_count > 0) {  // fold the pending diagnostics first
    if (h->cfg.precision == LBM_F64) finish_reductions<double>(h);
    else finish_reductions<float>(h);
  }
  const Layout& L = h->L;
  const int last = (int)((h->step + 1) & 1);
  StateRecord r{};
  long long dstep = 0;
  std::vector<double> pm((size_t)h->P.ntxE), pl(3 * (size_t)h->P.nblkL);
  if (hipMemcpyAsync(&r.diag, h->at<DevDiag>(L.diag), sizeof(DevDiag), hipMemcpyDeviceToHost, h->stream) ||
      hipMemcpyAsync(&r.mass_carried, h->at<double>(L.mstate[last]), sizeof(double), hipMemcpyDeviceToHost,
                     h->stream) ||
      hipMemcpyAsync(pm.data(), h->at<double>(L.pmin[last]), pm.size() * sizeof(double), hipMemcpyDeviceToHost,
                     h->stream) ||
      hipMemcpyAsync(pl.data(), h->at<double>(L.partL[last]), pl.size() * sizeof(double), hipMemcpyDeviceToHost,
                     h->stream) ||
      hipMemcpyAsync(&dstep, h->at<long long>(L.dstep[last]), sizeof(dstep), hipMemcpyDeviceToHost, h->stream) ||
      hipStreamSynchronize(h->stream))
    return LBM_EHIP;
  r.magic = STATE_MAGIC;
  r.step = dstep;
  r.nx = h->cfg.nx;
  r.ny = h->cfg.ny;
  r.nh = h->cfg.heater_rows;
  r.ntxE = h->P.ntxE;
  r.nblkL = h->P.nblkL;
  r.precision = h->cfg.precision;
  char* out = static_cast<char*>(dst);
  std::memcpy(out, &r, sizeof(r));
  std::memcpy(out + sizeof(r), pm.data(), pm.size() * sizeof(double));
  std::memcpy(out + sizeof(r) + pm.size() * sizeof(double), pl.data(), pl.size() * sizeof(double));
  return LBM_OK;
}

int write_state(lbm_ctx* h, const void* src) {
  StateRecord r;
  std::memcpy(&r, src, sizeof(r));
  if (r.magic != STATE_MAGIC || r.nx != h->cfg.nx || r.ny != h->cfg.ny || r.nh != h->cfg.heater_rows ||
      r.ntxE != h->P.ntxE || r.nblkL != h->P.nblkL || r.precision != h->cfg.precision || r.step < 0)
    return LBM_EINVAL;
  const Layout& L = h->L;
  h->step = r.step;
  const int last = (int)((h->step + 1) & 1);
  h->step_staging = (long long)r.step;
  const double* pm = reinterpret_cast<const double*>(static_cast<const char*>(src) + sizeof(r));
  const double* pl = pm + r.ntxE;
  if (hipMemcpyAsync(h->at<double>(L.partL[last]), pl, 3 * (size_t)r.nblkL * sizeof(double), hipMemcpyHostToDevice,
                     h->stream))
    return LBM_EHIP;
  if (hipMemcpyAsync(h->at<DevDiag>(L.diag), &r.diag, sizeof(DevDiag), hipMemcpyHostToDevice, h->stream) ||
      hipMemcpyAsync(h->at<double>(L.mstate[last]), &r.mass_carried, sizeof(double), hipMemcpyHostToDevice,
                     h->stream) ||
      hipMemcpyAsync(h->at<double>(L.pmin[last]), pm, (size_t)r.ntxE * sizeof(double), hipMemcpyHostToDevice,
                     h->stream) ||
      hipMemcpyAsync(h->at<long long>(L.dstep[last]), &h->step_staging, sizeof(long long), hipMemcpyHostToDevice,
                     h->stream) ||
      // the fused step's completion marks count steps: a state restored at an earlier
      // step than this context has run must not find them already reached
      hipMemsetAsync(h->at<unsigned>(L.cdone), 0, (size_t)h->P.nblkL * sizeof(unsigned), h->stream) ||
      hipStreamSynchronize(h->stream))
    return LBM_EHIP;
  h->hist_count = 0;
  h->bad = r.diag.err != 0;
  return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_field_bytes(lbm_ctx* h, int field) {
  if (!h) return 0;
  const size_t R = h->cfg.precision == LBM_F64 ? 8 : 4;
  const size_t nx = h->cfg.nx, N = nx * h->cfg.ny;
  switch (field) {
    case LBM_FIELD_F: return 9 * N * R;
    case LBM_FIELD_RHO:
    case LBM_FIELD_UX:
    case LBM_FIELD_UY: return N * R;
    case LBM_FIELD_T: return (N + nx * h->cfg.heater_rows) * R;
    case LBM_FIELD_GW: return nx * R;
    case LBM_FIELD_STATE: return state_bytes(h);
    default: return 0;
  }
}

int lbm_read_field(lbm_ctx* h, int field, void* dst, size_t bytes, int dst_is_device) {
  if (!h || !dst) return LBM_EINVAL;
  if (field == LBM_FIELD_STATE) {
    if (dst_is_device || bytes != state_bytes(h)) return LBM_EINVAL;
    return read_state(h, dst);
  }
  const Layout& L = h->L;
  const size_t R = h->cfg.precision == LBM_F64 ? 8 : 4;
  const size_t nx = h->cfg.nx, ny = h->cfg.ny, N = nx * ny;
  const hipMemcpyKind kind = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const void* src = nullptr;
  size_t need = 0;
  switch (field) {
    case LBM_FIELD_RHO: src = h->ws + L.rho; need = N * R; break;
    case LBM_FIELD_UX: src = h->ws + L.ux; need = N * R; break;
    case LBM_FIELD_UY: src = h->ws + L.uy; need = N * R; break;
    case LBM_FIELD_T: src = h->ws + L.T[h->tcur]; need = (N + nx * h->cfg.heater_rows) * R; break;
    case LBM_FIELD_GW: src = h->ws + L.gw; need = nx * R; break;
    case LBM_FIELD_F: {
      need = 9 * N * R;
      if (bytes != need) return LBM_EINVAL;
      // pull f^n into the spare population buffer, then copy it out
      void* spare = h->ws + L.f[1 - h->fcur];
      if (R == 8) gather_populations<double>(h, (double*)spare);
      else gather_populations<float>(h, (float*)spare);
      src = spare;
      break;
    }
    default: return LBM_EINVAL;
  }
  if (bytes != need) return LBM_EINVAL;
  if (hipMemcpyAsync(dst, src, need, kind, h->stream) != hipSuccess) return LBM_EHIP;
  if (!dst_is_device && hipStreamSynchronize(h->stream) != hipSuccess) return LBM_EHIP;
  return hip_ok(hipGetLastError());
}

int lbm_write_field(lbm_ctx* h, int field, const void* src, size_t bytes, int src_is_device) {
  if (!h || !src) return LBM_EINVAL;
  if (field == LBM_FIELD_STATE) {
    if (src_is_device || bytes != state_bytes(h)) return LBM_EINVAL;
    return write_state(h, src);
  }
  const Layout& L = h->L;
  const size_t R = h->cfg.precision == LBM_F64 ? 8 : 4;
  const size_t nx = h->cfg.nx, ny = h->cfg.ny, N = nx * ny;
  const hipMemcpyKind kind = src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (field == LBM_FIELD_T) {
    const size_t need = (N + nx * h->cfg.heater_rows) * R;
    if (bytes != need) return LBM_EINVAL;
    if (hipMemcpyAsync(h->ws + L.T[h->tcur], src, need, kind, h->stream) != hipSuccess) return LBM_EHIP;
    return hip_ok(hipStreamSynchronize(h->stream));
  }
  if (field == LBM_FIELD_F) {
    const size_t need = 9 * N * R;
    if (bytes != need) return LBM_EINVAL;
    void* spare = h->ws + L.f[1 - h->fcur];
    if (hipMemcpyAsync(spare, src, need, kind, h->stream) != hipSuccess) return LBM_EHIP;
    int rc = R == 8 ? scatter_state<double>(h, (const double*)spare, 0)
                    : scatter_state<float>(h, (const float*)spare, 0);
    if (rc) return rc;
    return hip_ok(hipStreamSynchronize(h->stream));
  }
  return LBM_EINVAL;
}

int lbm_set_kernel_timing(lbm_ctx* h, int enable) {
  if (!h) return LBM_EINVAL;
  h->timing = enable != 0;
  return LBM_OK;
}

int lbm_kernel_times(lbm_ctx* h, double* collide_ms, int64_t* collide_launches, double* energy_ms,
                     int64_t* energy_launches) {
  if (!h || !collide_ms || !collide_launches || !energy_ms || !energy_launches) return LBM_EINVAL;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return LBM_EHIP;
  double t[2] = {0.0, 0.0};
  int64_t n[2] = {0, 0};
  for (size_t p = 0; p < h->ev_kind.size(); ++p) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev_pool[2 * p], h->ev_pool[2 * p + 1]) != hipSuccess) return LBM_EHIP;
    t[h->ev_kind[p]] += ms;
    n[h->ev_kind[p]] += 1;
  }
  h->ev_used = 0;
  h->ev_kind.clear();
  *collide_ms = t[0];
  *collide_launches = n[0];
  *energy_ms = t[1];
  *energy_launches = n[1];
  return LBM_OK;
}

int lbm_destroy(lbm_ctx* h) {
  if (!h) return LBM_EINVAL;
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  delete h;
  return LBM_OK;
}

const char* lbm_strerror(int status) {
  switch (status) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument or configuration";
    case LBM_ENOMEM: return "workspace too small";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_ENONFINITE: return "device flagged a non-finite or unphysical state";
    case LBM_ESTATE: return "call not allowed in the current state";
    default: return "unknown status";
  }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of independent domains
// ---------------------------------------------------------------------------
namespace {

size_t batch_table_bytes(int n) { return align_up((size_t)n * sizeof(lbmk::DomainDev)); }

// the tile-to-domain maps of a batch (collide tiles, then energy tiles; the energy tile
// count bounded as in a domain's layout)
size_t batch_map_bytes(const lbm_config* cfgs, int n) {
  size_t tiles = 0;
  for (int i = 0; i < n; ++i) {
    const Grids g = grids(&cfgs[i], 0);
    tiles += (size_t)g.ntxL * g.ntyL + (size_t)g.ntxE * g.ntyE;
  }
  return align_up(tiles * sizeof(int));
}

bool batch_compatible(const lbm_config* cfgs, int n) {
  if (!cfgs || n < 1) return false;
  for (int i = 0; i < n; ++i) {
    if (!valid_config(&cfgs[i])) return false;
    if (cfgs[i].precision != cfgs[0].precision || cfgs[i].n_sub != cfgs[0].n_sub) return false;
    if ((cfgs[i].flags ^ cfgs[0].flags) & LBM_DIFF_ISOTROPIC) return false;
  }
  return true;
}

// the tile height a batch uses when the configuration leaves it open
lbm_config batch_member(const lbm_config& c) {
  lbm_config m = c;
  if (m.tile_rows == 0) m.tile_rows = m.precision == LBM_F64 ? E_HMAX : E_HMAX_F32;
  return m;
}

// Candidate energy tile heights of the autotuners.
std::vector<int> tile_candidates(const lbm_config& c) {
  const int hmax = c.precision == LBM_F64 ? E_HMAX : E_HMAX_F32;
  return {8, 12, 16, 20, 24, 32, 40, hmax};
}

// Autotuner cache key: what the timing depends on besides the tile shape.
std::string tune_key(const lbm_config* cfgs, int n) {
  std::string key = std::to_string(cfgs[0].precision) + "/" + std::to_string(cfgs[0].n_sub) + "/" +
                    std::to_string(cfgs[0].flags & LBM_DIFF_ISOTROPIC);
  for (int i = 0; i < n; ++i)
    key += "/" + std::to_string(cfgs[i].nx) + "x" + std::to_string(cfgs[i].ny) + "+" +
           std::to_string(cfgs[i].heater_rows);
  return key;
}

struct TuneEntry {
  std::vector<int> rows;
  std::vector<uint32_t> flags;
  double ms;
};
std::mutex tune_mu;
std::map<std::string, TuneEntry> tune_cache;

bool tune_cached(const std::string& key, int* rows, uint32_t* flags, double* ms, int n) {
  std::lock_guard<std::mutex> lk(tune_mu);
  auto it = tune_cache.find(key);
  if (it == tune_cache.end()) return false;
  for (int i = 0; i < n; ++i) {
    rows[i] = it->second.rows[i];
    if (flags) flags[i] = it->second.flags[i];
  }
  *ms = it->second.ms;
  return true;
}

void tune_store(const std::string& key, const int* rows, const uint32_t* flags, double ms, int n) {
  std::lock_guard<std::mutex> lk(tune_mu);
  tune_cache[key] = TuneEntry{std::vector<int>(rows, rows + n), std::vector<uint32_t>(flags, flags + n), ms};
}

// Times `steps` steps, after `steps` warm-up steps, of a batch or of one domain built in
// the caller's workspace; rc keeps the first error.
struct Timer {
  void* ws;
  size_t bytes;
  void* stream;
  const double* const* rho0;
  const double* const* T0;
  int steps;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = LBM_OK;
  Timer(void* w, size_t b, void* s, const double* const* r, const double* const* t, int n)
      : ws(w), bytes(b), stream(s), rho0(r), T0(t), steps(n) {
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = LBM_EHIP;
  }
  ~Timer() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
  template <typename Step>
  double time(Step&& step) {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    float ms = 0.f;
    int r = step();
    if (!r && (hipEventRecord(e0, st) != hipSuccess || (r = step()) != 0 || hipEventRecord(e1, st) != hipSuccess ||
               hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      r = r ? r : LBM_EHIP;
    if (r && !rc) rc = r;
    return (double)ms / steps;
  }
  double batch(const std::vector<lbm_config>& cs) {
    if (rc) return 0.0;
    lbm_batch* b = nullptr;
    const int r = lbm_batch_init(cs.data(), (int)cs.size(), ws, bytes, stream, rho0, T0, &b);
    if (r) {
      rc = r;
      return 0.0;
    }
    const double per = time([&] { return lbm_batch_step(b, steps); });
    lbm_batch_destroy(b);
    return per;
  }
  double single(const lbm_config& c) {
    if (rc) return 0.0;
    lbm_ctx* h = nullptr;
    const int r = lbm_init(&c, ws, bytes, stream, rho0[0], T0[0], &h);
    if (r) {
      rc = r;
      return 0.0;
    }
    const double per = time([&] { return lbm_step(h, steps); });
    if (!rc) {
      // a step failure surfaces only at synchronisation
      const int st = hip_ok(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
      if (st) rc = st;
    }
    lbm_destroy(h);
    return per;
  }
};

}  // namespace

extern "C" {

size_t lbm_batch_workspace_bytes(const lbm_config* cfgs, int n) {
  if (!batch_compatible(cfgs, n)) return 0;
  size_t total = batch_table_bytes(n) + batch_map_bytes(cfgs, n);
  for (int i = 0; i < n; ++i) total += align_up(lbm_workspace_bytes(&cfgs[i]));
  return total;
}

int lbm_batch_init(const lbm_config* cfgs, int n, void* d_workspace, size_t ws_bytes, void* hip_stream,
                   const double* const* rho0_host, const double* const* T0_host, lbm_batch** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  if (!batch_compatible(cfgs, n) || !d_workspace || !rho0_host || !T0_host) return LBM_EINVAL;
  if (reinterpret_cast<uintptr_t>(d_workspace) & 255) return LBM_EINVAL;
  const size_t need = lbm_batch_workspace_bytes(cfgs, n);
  if (ws_bytes < need) return LBM_ENOMEM;
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return LBM_ENOMEM;
  b->stream = reinterpret_cast<hipStream_t>(hip_stream);
  char* base = reinterpret_cast<char*>(d_workspace);
  b->table = reinterpret_cast<lbmk::DomainDev*>(base);
  b->domL = reinterpret_cast<int*>(base + batch_table_bytes(n));
  size_t off = batch_table_bytes(n) + batch_map_bytes(cfgs, n);
  std::vector<lbmk::DomainDev> tab(n);
  int tL = 0, tE = 0;
  for (int i = 0; i < n; ++i) {
    if (!rho0_host[i] || !T0_host[i]) {
      lbm_batch_destroy(b);
      return LBM_EINVAL;
    }
    const lbm_config m = batch_member(cfgs[i]);
    const size_t bytes = align_up(lbm_workspace_bytes(&m));
    lbm_ctx* h = nullptr;
    const int rc = lbm_init(&m, base + off, bytes, hip_stream, rho0_host[i], T0_host[i], &h);
    if (rc) {
      lbm_batch_destroy(b);
      return rc;
    }
    b->dom.push_back(h);
    tab[i].P = h->P;
    tab[i].L = h->L;
    tab[i].ws = h->ws;
    tab[i].tile0L = tL;
    tab[i].tile0E = tE;
    tL += h->P.nblkL;
    tE += h->P.nblkE;
    off += bytes;
  }
  b->nblkL = tL;
  b->nblkE = tE;
  b->domE = b->domL + tL;
  std::vector<int> dom((size_t)tL + tE);
  for (int i = 0; i < n; ++i) {
    std::fill(dom.begin() + tab[i].tile0L, dom.begin() + tab[i].tile0L + tab[i].P.nblkL, i);
    std::fill(dom.begin() + tL + tab[i].tile0E, dom.begin() + tL + tab[i].tile0E + tab[i].P.nblkE, i);
  }
  if (hipMemcpyAsync(b->table, tab.data(), n * sizeof(lbmk::DomainDev), hipMemcpyHostToDevice, b->stream) !=
          hipSuccess ||
      hipMemcpyAsync(b->domL, dom.data(), dom.size() * sizeof(int), hipMemcpyHostToDevice, b->stream) !=
          hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess) {
    lbm_batch_destroy(b);
    return LBM_EHIP;
  }
  *out = b;
  return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int64_t nsteps) {
  if (!b || nsteps < 0) return LBM_EINVAL;
  for (lbm_ctx* h : b->dom)
    if (h->bad) return LBM_ESTATE;
  const bool f64 = b->dom[0]->cfg.precision == LBM_F64;
  for (int64_t s = 0; s < nsteps; ++s) {
    if (f64) batch_step_once<double>(b);
    else batch_step_once<float>(b);
  }
  return hip_ok(hipGetLastError());
}

int lbm_batch_set_stream(lbm_batch* b, void* hip_stream) {
  if (!b) return LBM_EINVAL;
  b->stream = reinterpret_cast<hipStream_t>(hip_stream);
  for (lbm_ctx* h : b->dom) h->stream = b->stream;
  return LBM_OK;
}

int lbm_batch_observe(lbm_batch* b, lbm_obs* out) {
  if (!b || !out) return LBM_EINVAL;
  int status = LBM_OK;
  // every domain folds its history now (two launches for the whole batch), so the
  // shared history slot stays common
  if (b->dom[0]->cfg.precision == LBM_F64) batch_finish_reductions<double>(b);
  else batch_finish_reductions<float>(b);
  for (size_t i = 0; i < b->dom.size(); ++i) {
    const int rc = read_observation(b->dom[i], &out[i]);
    if (rc == LBM_ENONFINITE) status = LBM_ENONFINITE;
    else if (rc) return rc;
  }
  if (status) for (lbm_ctx* h : b->dom) h->bad = true;
  return status;
}

int lbm_batch_read_field(lbm_batch* b, int i, int field, void* dst, size_t bytes, int dst_is_device) {
  if (!b || i < 0 || i >= (int)b->dom.size()) return LBM_EINVAL;
  // the domains share the diagnostics history: fold it for all (lbm_batch_observe) first
  if (field == LBM_FIELD_STATE && b->dom[i]->hist_count != 0) return LBM_ESTATE;
  return lbm_read_field(b->dom[i], field, dst, bytes, dst_is_device);
}

int lbm_batch_write_field(lbm_batch* b, int i, int field, const void* src, size_t bytes, int src_is_device) {
  if (!b || i < 0 || i >= (int)b->dom.size()) return LBM_EINVAL;
  if (b->dom[i]->hist_count != 0) return LBM_ESTATE;  // call lbm_batch_observe first
  if (field == LBM_FIELD_STATE) return LBM_EINVAL;     // the domains share one step count
  return lbm_write_field(b->dom[i], field, src, bytes, src_is_device);
}

int lbm_batch_destroy(lbm_batch* b) {
  if (!b) return LBM_EINVAL;
  for (lbm_ctx* h : b->dom) lbm_destroy(h);
  delete b;
  return LBM_OK;
}

int lbm_autotune_tile_rows(const lbm_config* cfgs, int n, void* d_workspace, size_t ws_bytes, void* hip_stream,
                           const double* const* rho0_host, const double* const* T0_host, int steps,
                           int* best_rows, double* best_ms) {
  if (!best_rows || !best_ms || steps < 1 || !batch_compatible(cfgs, n)) return LBM_EINVAL;
  if (ws_bytes < lbm_batch_workspace_bytes(cfgs, n)) return LBM_ENOMEM;
  const std::string key = "rows/" + tune_key(cfgs, n);
  if (tune_cached(key, best_rows, nullptr, best_ms, 1)) return LBM_OK;
  Timer t(d_workspace, ws_bytes, hip_stream, rho0_host, T0_host, steps);
  if (t.rc) return t.rc;
  std::vector<lbm_config> cs(cfgs, cfgs + n);
  int best = 0;
  double bms = 0.0;
  for (int r : tile_candidates(cfgs[0])) {
    for (auto& c : cs) c.tile_rows = r;
    const double per = t.batch(cs);
    if (t.rc) return t.rc;
    if (best == 0 || per < bms) {
      best = r;
      bms = per;
    }
  }
  const uint32_t fl = cfgs[0].flags;
  tune_store(key, &best, &fl, bms, 1);
  *best_rows = best;
  *best_ms = bms;
  return LBM_OK;
}

int lbm_autotune(const lbm_config* cfgs, int n, void* d_workspace, size_t ws_bytes, void* hip_stream,
                 const double* const* rho0_host, const double* const* T0_host, int steps, int32_t* rows,
                 uint32_t* flags, double* best_ms) {
  if (!rows || !flags || !best_ms || steps < 1 || !batch_compatible(cfgs, n)) return LBM_EINVAL;
  if (ws_bytes < lbm_batch_workspace_bytes(cfgs, n)) return LBM_ENOMEM;
  const std::string key = "shape/" + tune_key(cfgs, n);
  int cr[1024];
  uint32_t cf[1024];
  if (n <= 1024 && tune_cached(key, cr, cf, best_ms, n)) {
    for (int i = 0; i < n; ++i) {
      rows[i] = cr[i];
      flags[i] = cf[i];
    }
    return LBM_OK;
  }
  Timer t(d_workspace, ws_bytes, hip_stream, rho0_host, T0_host, steps);
  if (t.rc) return t.rc;
  const std::vector<int> cand = tile_candidates(cfgs[0]);
  std::vector<lbm_config> cs(cfgs, cfgs + n);
  for (auto& c : cs) c.flags &= ~(LBM_ONE_LAUNCH | LBM_TWO_LAUNCHES);
  double bms = 0.0;
  if (n == 1) {
    // one domain: its own path (lbm_init / lbm_step), both launch modes where both apply
    const lbm_config& c0 = cfgs[0];
    const bool both = c0.precision == LBM_F32 && c0.n_sub == 1 && !(c0.flags & LBM_DIFF_ISOTROPIC);
    lbm_config best = cs[0];
    std::vector<int> cand1 = {0};  // the automatic height first (tiles that fill the device)
    cand1.insert(cand1.end(), cand.begin(), cand.end());
    for (uint32_t mode : {LBM_TWO_LAUNCHES, LBM_ONE_LAUNCH}) {
      if (!both && mode == LBM_ONE_LAUNCH) continue;
      for (int r : cand1) {
        lbm_config c = cs[0];
        c.tile_rows = r;
        if (both) c.flags |= mode;
        const double per = t.single(c);
        if (t.rc) return t.rc;
        if (bms == 0.0 || per < bms) {
          bms = per;
          best = c;
        }
      }
    }
    cs[0] = best;
  } else {
    // a batch: one height for all domains, then each size class on its own, the class
    // with the most nodes first, the other classes held at their best heights
    int r0 = 0;
    for (int r : cand) {
      for (auto& c : cs) c.tile_rows = r;
      const double per = t.batch(cs);
      if (t.rc) return t.rc;
      if (r0 == 0 || per < bms) {
        r0 = r;
        bms = per;
      }
    }
    for (auto& c : cs) c.tile_rows = r0;
    std::map<std::tuple<int, int, int>, long long> nodes;
    for (const auto& c : cs) nodes[{c.nx, c.ny, c.heater_rows}] += (long long)c.nx * (c.ny + c.heater_rows);
    std::vector<std::pair<long long, std::tuple<int, int, int>>> order;
    for (const auto& kv : nodes) order.push_back({kv.second, kv.first});
    std::stable_sort(order.begin(), order.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    if (order.size() > 1) {
      for (const auto& cls : order) {
        int cur = r0;
        for (const auto& c : cs)
          if (std::make_tuple(c.nx, c.ny, c.heater_rows) == cls.second) cur = c.tile_rows;
        for (int r : cand) {
          if (r == cur) continue;
          std::vector<lbm_config> trial = cs;
          for (auto& c : trial)
            if (std::make_tuple(c.nx, c.ny, c.heater_rows) == cls.second) c.tile_rows = r;
          const double per = t.batch(trial);
          if (t.rc) return t.rc;
          if (per < bms) {
            bms = per;
            cs = trial;
          }
        }
      }
    }
  }
  std::vector<int> rr(n);
  std::vector<uint32_t> ff(n);
  for (int i = 0; i < n; ++i) {
    rr[i] = rows[i] = cs[i].tile_rows;
    ff[i] = flags[i] = cs[i].flags;
  }
  if (n <= 1024) tune_store(key, rr.data(), ff.data(), bms, n);
  *best_ms = bms;
  return LBM_OK;
}

}  // extern "C"
