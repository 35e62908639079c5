// lbm_ctx.hpp -- library context, shared by the host entry points (lbm_api.hip) and
// the per-precision launch code (lbm_f32.hip, lbm_f64.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "lbm_api.h"
#include "lbm_params.hpp"

namespace lbmh {

// Tiles.  k_collide: 64 columns x TY rows, NWC waves (the fused FP32 step runs two
// collide tiles per workgroup, the size of an energy workgroup).  k_energy: txE <=
// E_TXMAX columns x tyE rows (E_HMIN <= tyE <= E_HMAX), E_NW waves; the sizes are chosen
// per grid so that the tiles fill the CUs in one round when the grid allows it.
constexpr int TY_F32 = 16, TY_F64 = 8, NWC = 4;
constexpr int E_NW = 8, E_HMAX = 48, E_HMIN = 8, E_TXMAX = 56;
// FP32 register-row energy kernel: E_RNW waves of E_BAND rows each, E_RWPE waves per
// SIMD (two workgroups per CU)
constexpr int E_RNW = 8, E_BAND = 7, E_RWPE = 4;
// tallest FP32 energy tile (also within the LDS kernel's E_HMAX, used for FP32 with
// the isotropic scheme)
constexpr int E_HMAX_F32 = E_RNW * E_BAND - 8;
static_assert(E_HMAX_F32 <= E_HMAX && E_HMAX_F32 >= E_HMIN, "FP32 energy tile height");
// energy workgroups resident per CU (LDS: 57 KB per FP32 workgroup, 115 KB per FP64)
constexpr int E_PER_CU_F32 = 2, E_PER_CU_F64 = 1;
// Steps of energy partials kept before they are folded into the diagnostics.
constexpr int HIST = LBM_HISTORY_STEPS;

using lbmk::Layout;

}  // namespace lbmh

struct lbm_ctx {
  lbm_config cfg;  // site pointers cleared: the sites live on in the wall profile
  lbmk::KParams P;
  lbmh::Layout L;
  hipStream_t stream;
  char* ws;
  int fcur, tcur;  // which population / temperature buffer holds the current state
  int64_t step;
  bool bad;
  int hist_first, hist_count;  // history slots of the steps not yet folded in
  int ncu;                     // compute units of the device
  bool fused;                  // FP32 steps run as one fused launch (k_step_fused)
  long long step_staging;      // host copy source for the device step counter
  // optional per-kernel timing: events recorded in pairs (start, stop) per launch
  bool timing;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used;
  std::vector<int> ev_kind;  // 0 collide, 1 energy, one entry per recorded pair
  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
};

struct lbm_batch {
  std::vector<lbm_ctx*> dom;  // per-domain contexts; the batch keeps their bookkeeping in step
  hipStream_t stream;
  lbmk::DomainDev* table;     // device table, first in the workspace
  int* domL;                  // domain of every collide tile of the batch (device)
  int* domE;                  // domain of every energy tile of the batch (device)
  int nblkL, nblkE;           // collide and energy tiles over all domains
};

namespace lbmh {
// Event pair around one launch when timing is on: begin returns the start event's
// index (or -1), end records the stop event.
int timing_begin(lbm_ctx* h, int kind);
void timing_end(lbm_ctx* h, int idx);
// Per-precision launch code (T = float or double), defined in lbm_launch.hpp.
template <typename T> void step_once(lbm_ctx* h);
template <typename T> int scatter_state(lbm_ctx* h, const T* src, int src_is_rho);
template <typename T> void finish_reductions(lbm_ctx* h);  // fold all pending steps
template <typename T> void gather_populations(lbm_ctx* h, T* out);
template <typename T> int init_fields(lbm_ctx* h, const double* rho0, const double* T0,
                                      const double* gw);
template <typename T> void batch_step_once(lbm_batch* b);
template <typename T> void batch_finish_reductions(lbm_batch* b);  // fold every domain's pending steps
}  // namespace lbmh
