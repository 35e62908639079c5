// lbm_launch.hpp -- kernel launches of one precision.  Included by lbm_f32.hip and
// lbm_f64.hip, which instantiate it for float and double.
#pragma once
#include <algorithm>
#include <vector>

#include "lbm_batch.hpp"
#include "lbm_ctx.hpp"
#include "lbm_energy_f32.hpp"
#include "lbm_kernels.hpp"

namespace lbmh {

using lbmk::DevDiag;
using lbmk::KParams;
using lbmk::NT;

// Fold every step of the history into the diagnostics (deterministic step order) and
// recompute mass, rho_ave and max speed of the current state.
template <typename real>
void finish_reductions(lbm_ctx* h) {
  const Layout& L = h->L;
  const int last = (int)((h->step + 1) & 1);  // slot written by the last collide / scatter
  if (h->hist_count > 0)
    hipLaunchKernelGGL((lbmk::k_reduce_steps<real>), dim3(h->hist_count), dim3(NT), 0, h->stream, h->P,
                       h->at<double>(L.hist), h->at<double>(L.steps), h->hist_first, HIST);
  hipLaunchKernelGGL((lbmk::k_finish<real>), dim3(1), dim3(NT), 0, h->stream, h->P, h->at<double>(L.steps),
                     h->hist_first, h->hist_count, HIST, h->at<double>(L.partL[last]),
                     h->at<double>(L.pmin[last]), h->at<DevDiag>(L.diag));
  h->hist_first = (h->hist_first + h->hist_count) % HIST;
  h->hist_count = 0;
}

// One lattice step: k_collide, then k_energy once per energy sub-step (Eq. 27).
// A full history is folded at the end of the step that fills it, so any run of
// HIST steps that starts with an empty history (after init, observe, a field write or
// a multiple of HIST steps) carries its own fold and can be captured and replayed.
template <typename real>
void step_once(lbm_ctx* h) {
  const KParams& P = h->P;
  const Layout& L = h->L;
  constexpr bool f64 = sizeof(real) == 8;
  const int cur = (int)(h->step & 1), prev = 1 - cur;
  real* fs = h->at<real>(L.f[h->fcur]);
  real* fd = h->at<real>(L.f[1 - h->fcur]);
  real* topin = h->at<real>(L.topin);
  real* rho = h->at<real>(L.rho);
  real* ux = h->at<real>(L.ux);
  real* uy = h->at<real>(L.uy);
  DevDiag* diag = h->at<DevDiag>(L.diag);
  const real* gw = h->at<real>(L.gw);
  const real* Tc = h->at<real>(L.T[h->tcur]);
  const double dt = 1.0 / h->cfg.n_sub;
  const bool iso = (h->cfg.flags & LBM_DIFF_ISOTROPIC) != 0;
  double* hslot = h->at<double>(L.hist) + (size_t)((h->hist_first + h->hist_count) % HIST) * P.nblkE * 5;
  if constexpr (!f64) {
    if (h->fused) {
      // the whole step in one launch: collide tile pairs, the outlet block, energy tiles
      const int tev = timing_begin(h, 0);
      hipLaunchKernelGGL((lbmk::k_step_fused<TY_F32, NWC, E_RNW, E_BAND, E_RWPE>),
                         dim3((P.nblkL + 1) / 2 + 1 + P.nblkE),
                         dim3(E_RNW * 64), 0, h->stream, P, fs, fd, topin, Tc, h->at<real>(L.T[1 - h->tcur]), gw,
                         rho, ux, uy, h->at<double>(L.mstate[prev]), h->at<double>(L.pmin[prev]),
                         h->at<double>(L.mstate[cur]), h->at<double>(L.partL[cur]), h->at<double>(L.pmin[cur]),
                         diag, h->at<long long>(L.dstep[prev]), h->at<long long>(L.dstep[cur]), hslot,
                         h->at<unsigned>(L.cdone), h->at<int>(L.order), dt);
      timing_end(h, tev);
      h->tcur = 1 - h->tcur;
      h->hist_count += 1;
      h->fcur = 1 - h->fcur;
      h->step += 1;
      if (h->hist_count == HIST) finish_reductions<real>(h);
      return;
    }
  }
  int tev = timing_begin(h, 0);
  hipLaunchKernelGGL((lbmk::k_collide<real, f64 ? TY_F64 : TY_F32, NWC>), dim3(P.nblkL), dim3(NWC * 64), 0,
                     h->stream, P, fs, fd, topin, Tc, gw, rho, ux, uy, h->at<double>(L.mstate[prev]),
                     h->at<double>(L.pmin[prev]), h->at<double>(L.mstate[cur]),
                     h->at<double>(L.partL[cur]), diag, h->at<long long>(L.dstep[prev]),
                     h->at<long long>(L.dstep[cur]));
  timing_end(h, tev);
  for (int sub = 0; sub < h->cfg.n_sub; ++sub) {
    const real* Tin = h->at<real>(L.T[h->tcur]);
    real* Tout = h->at<real>(L.T[1 - h->tcur]);
    tev = timing_begin(h, 1);
#define LBM_E(ISO)                                                                               \
  hipLaunchKernelGGL((lbmk::k_energy<real, ISO, E_NW, E_HMAX>), dim3(P.nblkE + 1), dim3(E_NW * 64), 0, \
                     h->stream, P, Tin, Tout, rho, ux, uy, hslot, fd, topin,                       \
                     h->at<double>(L.partL[cur]), h->at<double>(L.pmin[cur]), diag, sub, dt,      \
                     h->at<long long>(L.dstep[prev]))
    if (iso) LBM_E(true);
    else if constexpr (f64) LBM_E(false);
    else
      hipLaunchKernelGGL((lbmk::k_energy_rows<E_RNW, E_BAND, E_RWPE>), dim3(P.nblkE + 1), dim3(E_RNW * 64), 0, h->stream, P,
                         Tin, Tout, rho, ux, uy, hslot, fd, topin, h->at<double>(L.partL[cur]),
                         h->at<double>(L.pmin[cur]), diag, sub, dt, h->at<long long>(L.dstep[prev]));
#undef LBM_E
    timing_end(h, tev);
    h->tcur = 1 - h->tcur;
  }
  h->hist_count += 1;
  h->fcur = 1 - h->fcur;
  h->step += 1;
  if (h->hist_count == HIST) finish_reductions<real>(h);
}

// One step of every domain of a batch: the batched collide kernel, then the batched
// energy kernel once per energy sub-step.  All domains share the parity, the buffer
// indices and the history slot; the per-domain host bookkeeping advances together.
// finish_reductions for every domain of a batch in two launches (the domains share
// the history slots, the step and the parity)
template <typename real>
void batch_finish_reductions(lbm_batch* b) {
  lbm_ctx* h0 = b->dom[0];
  const int n = (int)b->dom.size();
  const int last = (int)((h0->step + 1) & 1);
  if (h0->hist_count > 0)
    hipLaunchKernelGGL(lbmk::k_reduce_steps_batch<real>, dim3(h0->hist_count, n), dim3(NT), 0, b->stream, b->table,
                       h0->hist_first, HIST);
  hipLaunchKernelGGL(lbmk::k_finish_batch<real>, dim3(n), dim3(NT), 0, b->stream, b->table, h0->hist_first,
                     h0->hist_count, HIST, last);
  for (lbm_ctx* h : b->dom) {
    h->hist_first = (h->hist_first + h->hist_count) % HIST;
    h->hist_count = 0;
  }
}

template <typename real>
void batch_step_once(lbm_batch* b) {
  lbm_ctx* h0 = b->dom[0];
  constexpr bool f64 = sizeof(real) == 8;
  const int n = (int)b->dom.size();
  const int cur = (int)(h0->step & 1), fcur = h0->fcur;
  int tcur = h0->tcur;
  const int hslot = (h0->hist_first + h0->hist_count) % HIST;
  const bool iso = (h0->cfg.flags & LBM_DIFF_ISOTROPIC) != 0;
  hipLaunchKernelGGL((lbmk::k_collide_batch<real, f64 ? TY_F64 : TY_F32, NWC>), dim3(b->nblkL), dim3(NWC * 64), 0,
                     b->stream, b->table, b->domL, fcur, tcur, cur);
  const double dt = 1.0 / h0->cfg.n_sub;
  for (int sub = 0; sub < h0->cfg.n_sub; ++sub) {
    if (iso)
      hipLaunchKernelGGL((lbmk::k_energy_batch<real, true, E_NW, E_HMAX>), dim3(b->nblkE + n), dim3(E_NW * 64), 0,
                         b->stream, b->table, n, b->domE, 1 - fcur, tcur, cur, hslot, sub, dt);
    else if constexpr (f64)
      hipLaunchKernelGGL((lbmk::k_energy_batch<real, false, E_NW, E_HMAX>), dim3(b->nblkE + n), dim3(E_NW * 64), 0,
                         b->stream, b->table, n, b->domE, 1 - fcur, tcur, cur, hslot, sub, dt);
    else
      hipLaunchKernelGGL((lbmk::k_energy_rows_batch<E_RNW, E_BAND, E_RWPE>), dim3(b->nblkE + n), dim3(E_RNW * 64), 0,
                         b->stream, b->table, n, b->domE, 1 - fcur, tcur, cur, hslot, sub, dt);
    tcur = 1 - tcur;
  }
  for (lbm_ctx* h : b->dom) {
    h->tcur = tcur;
    h->hist_count += 1;
    h->fcur = 1 - fcur;
    h->step += 1;
  }
  if (h0->hist_count == HIST) batch_finish_reductions<real>(b);
}



// Store pre-collision populations (or the equilibrium at rest of a density field)
// as the current state; its mass partials go where the next collide kernel reads them.
template <typename real>
int scatter_state(lbm_ctx* h, const real* src, int src_is_rho) {
  const Layout& L = h->L;
  const int last = (int)((h->step + 1) & 1);
  if (hipMemsetAsync(h->at<double>(L.pmin[last]), 0, (size_t)h->P.ntxE * sizeof(double), h->stream) !=
      hipSuccess)
    return LBM_EHIP;
  // the fused step's completion marks restart with the step count (they only grow)
  if (hipMemsetAsync(h->at<unsigned>(L.cdone), 0, (size_t)h->P.nblkL * sizeof(unsigned), h->stream) != hipSuccess)
    return LBM_EHIP;
  hipLaunchKernelGGL((lbmk::k_scatter<real>), dim3(h->P.nblkL), dim3(NT), 0, h->stream, h->P, src,
                     src_is_rho, h->at<real>(L.f[h->fcur]), h->at<real>(L.topin),
                     h->at<double>(L.partL[last]));
  finish_reductions<real>(h);
  // the next collide kernel starts its mass bookkeeping from the summed mass, and its
  // step count from the host's
  if (hipMemcpyAsync(h->at<double>(L.mstate[last]), &h->at<DevDiag>(L.diag)->mass, sizeof(double),
                     hipMemcpyDeviceToDevice, h->stream) != hipSuccess)
    return LBM_EHIP;
  h->step_staging = (long long)h->step;
  if (hipMemcpyAsync(h->at<long long>(L.dstep[last]), &h->step_staging, sizeof(long long),
                     hipMemcpyHostToDevice, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return LBM_EHIP;
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EHIP;
}

template <typename real>
void gather_populations(lbm_ctx* h, real* out) {
  const Layout& L = h->L;
  const size_t N = (size_t)h->P.nx * h->P.ny;
  const int grid = (int)std::min<size_t>((N + NT - 1) / NT, 65536);
  hipLaunchKernelGGL((lbmk::k_gather<real>), dim3(grid), dim3(NT), 0, h->stream, h->P,
                     h->at<real>(L.f[h->fcur]), h->at<real>(L.topin), out);
}

template <typename real>
static int copy_converted(lbm_ctx* h, const double* host, real* dev, size_t n) {
  // host FP64 -> device real; synchronised so the staging vector outlives the copy
  std::vector<real> tmp(n);
  for (size_t i = 0; i < n; ++i) tmp[i] = (real)host[i];
  if (hipMemcpyAsync(dev, tmp.data(), n * sizeof(real), hipMemcpyHostToDevice, h->stream) != hipSuccess)
    return LBM_EHIP;
  return hipStreamSynchronize(h->stream) == hipSuccess ? LBM_OK : LBM_EHIP;
}

template <typename real>
int init_fields(lbm_ctx* h, const double* rho0, const double* T0, const double* gw) {
  const Layout& L = h->L;
  const size_t nx = h->P.nx, N = nx * h->P.ny, NTn = nx * h->P.nT;
  int rc;
  if ((rc = copy_converted<real>(h, T0, h->at<real>(L.T[0]), NTn))) return rc;
  if ((rc = copy_converted<real>(h, rho0, h->at<real>(L.rho), N))) return rc;
  if ((rc = copy_converted<real>(h, gw, h->at<real>(L.gw), nx))) return rc;
  if (hipMemsetAsync(h->at<real>(L.ux), 0, N * sizeof(real), h->stream) != hipSuccess) return LBM_EHIP;
  if (hipMemsetAsync(h->at<real>(L.uy), 0, N * sizeof(real), h->stream) != hipSuccess) return LBM_EHIP;
  if (hipMemsetAsync(h->at<real>(L.topin), 0, 3 * nx * sizeof(real), h->stream) != hipSuccess) return LBM_EHIP;
  DevDiag d{};
  d.first_bad = ~0ull;
  if (hipMemcpyAsync(h->at<DevDiag>(L.diag), &d, sizeof(d), hipMemcpyHostToDevice, h->stream) != hipSuccess)
    return LBM_EHIP;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return LBM_EHIP;
  if ((rc = scatter_state<real>(h, h->at<real>(L.rho), 1))) return rc;
  return hipStreamSynchronize(h->stream) == hipSuccess ? LBM_OK : LBM_EHIP;
}

}  // namespace lbmh

#define LBM_INSTANTIATE(T)                                                                  \
  namespace lbmh {                                                                          \
  template void step_once<T>(lbm_ctx*);                                                     \
  template int scatter_state<T>(lbm_ctx*, const T*, int);                                   \
  template void finish_reductions<T>(lbm_ctx*);                                             \
  template void gather_populations<T>(lbm_ctx*, T*);                                        \
  template int init_fields<T>(lbm_ctx*, const double*, const double*, const double*);       \
  template void batch_step_once<T>(lbm_batch*);                                             \
  template void batch_finish_reductions<T>(lbm_batch*);                                             \
  }
