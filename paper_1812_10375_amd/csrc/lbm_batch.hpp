// lbm_batch.hpp -- batched step over independent domains.  One launch covers the tiles
// of every domain of a batch: a workgroup takes global tile g (XCD-aware order), reads
// its domain from the batch's tile-to-domain map (one scalar load), and runs
// the same per-tile code as the single-domain kernels with that domain's parameters and
// buffers.  All domains share the step parity, so every argument of a launch depends
// only on the parity and the diagnostics history slot.
#pragma once
#include "lbm_energy_f32.hpp"
#include "lbm_kernels.hpp"

namespace lbmk {

template <typename real, int TY, int NW>
__global__ void __launch_bounds__(NW * 64)
    k_collide_batch(const DomainDev* __restrict__ tab, const int* __restrict__ domL, int fcur, int tcur, int cur) {
  const int g = xcd_tile(blockIdx.x, gridDim.x);
  const int d = domL[g];
  const DomainDev& D = tab[d];
  const Layout& L = D.L;
  char* ws = D.ws;
  const int prev = 1 - cur;
  collide_tile<real, TY, NW, false>(
      D.P, reinterpret_cast<const real*>(ws + L.f[fcur]), reinterpret_cast<real*>(ws + L.f[1 - fcur]),
      reinterpret_cast<const real*>(ws + L.topin), reinterpret_cast<const real*>(ws + L.T[tcur]),
      reinterpret_cast<const real*>(ws + L.gw), reinterpret_cast<real*>(ws + L.rho),
      reinterpret_cast<real*>(ws + L.ux), reinterpret_cast<real*>(ws + L.uy),
      reinterpret_cast<const double*>(ws + L.mstate[prev]), reinterpret_cast<const double*>(ws + L.pmin[prev]),
      reinterpret_cast<double*>(ws + L.mstate[cur]), reinterpret_cast<double*>(ws + L.partL[cur]),
      reinterpret_cast<DevDiag*>(ws + L.diag), reinterpret_cast<const long long*>(ws + L.dstep[prev]),
      reinterpret_cast<long long*>(ws + L.dstep[cur]), g - D.tile0L);
}

// Energy update of every domain.  Blocks [0, ndom) apply the open-top rule of domain b
// (once per LB step); the remaining blocks take the tiles.  fpost names the population
// buffer written by this step's collision (read by the open-top rule).
template <typename real, int NW>
__device__ __forceinline__ bool batch_outlet(const DomainDev* __restrict__ tab, int ndom, int fpost, int cur,
                                             int sub) {
  if ((int)blockIdx.x >= ndom) return false;
  const DomainDev& D = tab[blockIdx.x];
  const Layout& L = D.L;
  char* ws = D.ws;
  if (sub == 0)
    outlet_block<real, NW>(D.P, reinterpret_cast<const real*>(ws + L.f[fpost]), reinterpret_cast<real*>(ws + L.topin),
                           reinterpret_cast<const real*>(ws + L.ux), reinterpret_cast<const real*>(ws + L.uy),
                           reinterpret_cast<const double*>(ws + L.partL[cur]), reinterpret_cast<double*>(ws + L.pmin[cur]));
  return true;
}

// FP32 register-row kernel
template <int NW, int B, int WPE>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE)))
    k_energy_rows_batch(const DomainDev* __restrict__ tab, int ndom, const int* __restrict__ domE, int fpost,
                        int tcur, int cur, int hslot, int sub, double dtd) {
  if (batch_outlet<float, NW>(tab, ndom, fpost, cur, sub)) return;
  const int g = xcd_tile_edges_first(blockIdx.x - ndom, gridDim.x - ndom);
  const int d = domE[g];
  const DomainDev& D = tab[d];
  const Layout& L = D.L;
  char* ws = D.ws;
  energy_rows_step<NW, B>(
      D.P, reinterpret_cast<const float*>(ws + L.T[tcur]), reinterpret_cast<float*>(ws + L.T[1 - tcur]),
      reinterpret_cast<const float*>(ws + L.rho), reinterpret_cast<const float*>(ws + L.ux),
      reinterpret_cast<const float*>(ws + L.uy),
      reinterpret_cast<double*>(ws + L.hist) + (size_t)hslot * D.P.nblkE * 5, reinterpret_cast<DevDiag*>(ws + L.diag),
      sub, dtd, reinterpret_cast<const long long*>(ws + L.dstep[1 - cur]), g - D.tile0E);
}

// LDS kernel (FP64, or the isotropic scheme)
template <typename real, bool ISO, int NW, int HMAX>
__global__ void __launch_bounds__(NW * 64)
    k_energy_batch(const DomainDev* __restrict__ tab, int ndom, const int* __restrict__ domE, int fpost, int tcur,
                   int cur, int hslot, int sub, double dtd) {
  if (batch_outlet<real, NW>(tab, ndom, fpost, cur, sub)) return;
  const int g = xcd_tile_edges_first(blockIdx.x - ndom, gridDim.x - ndom);
  const int d = domE[g];
  const DomainDev& D = tab[d];
  const Layout& L = D.L;
  char* ws = D.ws;
  energy_lds_tile<real, ISO, NW, HMAX>(
      D.P, reinterpret_cast<const real*>(ws + L.T[tcur]), reinterpret_cast<real*>(ws + L.T[1 - tcur]),
      reinterpret_cast<const real*>(ws + L.rho), reinterpret_cast<const real*>(ws + L.ux),
      reinterpret_cast<const real*>(ws + L.uy),
      reinterpret_cast<double*>(ws + L.hist) + (size_t)hslot * D.P.nblkE * 5, reinterpret_cast<DevDiag*>(ws + L.diag),
      sub, dtd, reinterpret_cast<const long long*>(ws + L.dstep[1 - cur]), g - D.tile0E);
}

// The history fold for every domain of a batch at once: blockIdx.y = domain,
// blockIdx.x = history slot (all domains share the slots, the step and the parity).
template <typename real>
__global__ void __launch_bounds__(NT)
    k_reduce_steps_batch(const DomainDev* __restrict__ tab, int first, int hist_cap) {
  const DomainDev& D = tab[blockIdx.y];
  reduce_steps_block(D.P, reinterpret_cast<const double*>(D.ws + D.L.hist), reinterpret_cast<double*>(D.ws + D.L.steps),
                     first, hist_cap, blockIdx.x);
}

template <typename real>
__global__ void __launch_bounds__(NT)
    k_finish_batch(const DomainDev* __restrict__ tab, int first, int count, int hist_cap, int last) {
  const DomainDev& D = tab[blockIdx.x];
  char* ws = D.ws;
  finish_block(D.P, reinterpret_cast<const double*>(ws + D.L.steps), first, count, hist_cap,
               reinterpret_cast<const double*>(ws + D.L.partL[last]), reinterpret_cast<const double*>(ws + D.L.pmin[last]),
               reinterpret_cast<DevDiag*>(ws + D.L.diag));
}

}  // namespace lbmk
