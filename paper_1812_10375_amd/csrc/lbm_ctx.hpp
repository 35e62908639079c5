// lbm_ctx.hpp -- library context, shared by the host entry points (lbm_api.hip) and
// the per-precision launch code (lbm_f32.hip, lbm_f64.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "lbm_api.h"
#include "lbm_params.hpp"

namespace lbmh {

// Tiles.  k_collide: 64 columns x TY rows.  k_energy: (W3-6) x (H3-6) interior.
constexpr int TY_F32 = 16, TY_F64 = 8;
constexpr int W3_F32 = 64, W3_F64 = 32, H3_E = 24;

// Byte offsets of the arrays carved out of the caller's workspace.
struct Layout {
  size_t f[2], T[2], rho, ux, uy, topin, gw, partL, partE, diag, total;
};

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
  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
};

namespace lbmh {
// Per-precision launch code (T = float or double), defined in lbm_launch.hpp.
template <typename T> void step_once(lbm_ctx* h);
template <typename T> int scatter_state(lbm_ctx* h, const T* src, int src_is_rho);
template <typename T> void finish_reductions(lbm_ctx* h);
template <typename T> void gather_populations(lbm_ctx* h, T* out);
template <typename T> int init_fields(lbm_ctx* h, const double* rho0, const double* T0,
                                      const double* gw);
}  // namespace lbmh
