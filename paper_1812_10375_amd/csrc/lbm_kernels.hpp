// lbm_kernels.hpp -- gfx950 kernels of the hybrid thermal pseudo-potential LB step
// (Hu & Liu, arXiv:1812.10375).  Included once, by lbm_api.hip.
//
// Data layout (all arrays live in the caller's workspace; x is the fastest index):
//   fpost[2]  9 x ny x nx   post-collision populations f*, structure of arrays.  Step
//                           n reads f*^{n-1} from one buffer by pulling (f^n_i(x) =
//                           f*^{n-1}_i(x - e_i), with bounce-back at walls) and writes
//                           f*^n into the other, aligned and coalesced.
//   topin     3 x nx        populations 4, 7, 8 entering the top row from an open top
//   T[2]      nT x nx       temperature, nT = heater_rows + ny (double-buffered)
//   rho,ux,uy ny x nx       density and Eq. 5 velocity of the last collision
//   gw        nx            wall strength of each bottom wall column (Eq. 10)
//   partL[2]  nblkL x 3     per-tile FP64 partials of the collide kernel (post-collision
//                           mass, max |u|^2, sum of u_y on row ny-2),
//                           double-buffered by step parity
//   pmin[2]   ntxE          net mass entering through an open top in the last step,
//                           per top energy tile (inflow 4, 7, 8 minus outflow 2, 5, 6)
//   mstate[2] 1             mass of the state at the start of the step
//   dstep[2]  1             index of the step being computed (for error reports); the
//                           collide kernel reads slot prev and writes slot cur, so no
//                           kernel argument depends on the absolute step
//   hist      HIST x nblkE x 5  per-step, per-tile FP64 energy partials
//   steps     HIST x 5      per-step totals of hist
//   diag      DevDiag       FP64 diagnostics
//
// Per step two kernels run: k_collide (moments, EOS, forces, MRT collision) and the
// energy update (all four RK4 stages of the temperature equation on a tile with a
// four-cell halo: k_energy_rows in FP32, k_energy in FP64 and for the isotropic scheme).
// The mass for rho_ave (Eq. 9) follows from continuity: streaming and bounce-back move
// populations and the collision conserves their sum, so only the open top changes it;
// every collide block adds the previous step's net inflow (same values, same order) to
// the stored mass.  Block 0 of the energy launch applies the outlet rule to every top
// column and records the net inflow per tile column; the energy diagnostics are reduced
// in step order later by k_reduce_steps / k_finish.  No atomics touch the diagnostics,
// so reruns are bitwise identical.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lbm_params.hpp"

namespace lbmk {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// periodic wrap of x + d, |d| <= 1
__device__ __forceinline__ int wrap1(int v, int nx) {
  v = v < 0 ? v + nx : v;
  return v >= nx ? v - nx : v;
}
// periodic wrap of any integer
__device__ __forceinline__ int wrapm(int v, int nx) {
  int r = v % nx;
  return r < 0 ? r + nx : r;
}

// 8 XCDs take blocks round-robin; give each XCD a contiguous run of tiles so that
// neighbouring tiles (which share halos) sit in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nblk) {
  int q = nblk >> 3, r = nblk & 7, k = b & 7;
  return k * q + (k < r ? k : r) + (b >> 3);
}

// Temperature-grid rows of energy tile `tile`: the first tile row holds tyE0 rows, the
// following ones tyE each, and the last one what remains of the nT rows.
__device__ __forceinline__ void energy_tile_rows(const KParams& P, int tile, int& j0, int& ty) {
  const int tr = tile / P.ntxE;
  j0 = tr == 0 ? 0 : P.tyE0 + (tr - 1) * P.tyE;
  ty = min(tr == 0 ? P.tyE0 : P.tyE, P.nT - j0);
}

// The energy grids' order: as xcd_tile, but every odd band is dispatched from its last
// tile down.  The top tile row (end of the last band) and the bottom one (start of the
// first band) then start first on their XCDs.  They run the slower boundary code, and
// the oldest waves on a CU get issue priority.
__device__ __forceinline__ int xcd_tile_edges_first(int b, int nblk) {
  const int q = nblk >> 3, r = nblk & 7, k = b & 7, pos = b >> 3;
  const int start = k * q + (k < r ? k : r), cnt = q + (k < r ? 1 : 0);
  return start + ((k & 1) ? cnt - 1 - pos : pos);
}

// 1/v: exact for FP64, the hardware reciprocal (1 ulp) for FP32
template <typename real>
__device__ __forceinline__ real fast_rcp(real v) {
  if constexpr (sizeof(real) == 8) return 1.0 / v;
  else return __builtin_amdgcn_rcpf(v);
}

// Element i of an array addressed as a uniform base pointer plus a 32-bit byte offset,
// which maps onto the scalar-base (saddr) form of the global load and store
// instructions.  One field plane stays below 4 GiB (checked when a context is made).
template <typename T>
__device__ __forceinline__ T ld32(const T* __restrict__ base, unsigned i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st32(T* __restrict__ base, unsigned i, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (unsigned)sizeof(T)) = v;
}

// Loads and stores of data that another workgroup of the same launch produces or
// consumes (COH = true): agent-scope relaxed atomic accesses, coherent across the XCDs'
// separate L2 caches without cache-wide write-back or invalidation.  With COH = false
// they are plain accesses (the data crosses a kernel boundary).
template <bool COH, typename T>
__device__ __forceinline__ T ldc(const T* p) {
  if constexpr (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return *p;
}
template <bool COH, typename T>
__device__ __forceinline__ void stc(T* p, T v) {
  if constexpr (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else *p = v;
}
// stc at element i of a uniform base (32-bit offset, as ld32 / st32)
template <bool COH, typename T>
__device__ __forceinline__ void stc32(T* __restrict__ base, unsigned i, T v) {
  stc<COH>(reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (unsigned)sizeof(T)), v);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// One DPP move of a double (both halves): the value of the lane that `CTRL` selects, 0
// where there is none or where `ROWS` leaves the row out.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, ROWS, 0xf, true);
  const unsigned hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, ROWS, 0xf, true);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum over the 64 lanes in a fixed order without LDS: running sums within each row of
// 16 lanes (shifts by 1, 2, 4, 8), then the row totals carried by row_bcast:15 into rows
// 1 and 3 and row_bcast:31 into rows 2 and 3.  Lane 63 ends with the total, which every
// lane receives.
__device__ __forceinline__ double lane63_f64(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)u, 63);
  const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), 63);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0x111, 0xf>(v);
  v += dpp_f64<0x112, 0xf>(v);
  v += dpp_f64<0x114, 0xf>(v);
  v += dpp_f64<0x118, 0xf>(v);
  v += dpp_f64<0x142, 0xa>(v);
  v += dpp_f64<0x143, 0xc>(v);
  return lane63_f64(v);
}
// The same for the maximum of values >= 0 (the lanes without a source read 0).
__device__ __forceinline__ double wave_max_dpp(double v) {
  v = fmax(v, dpp_f64<0x111, 0xf>(v));
  v = fmax(v, dpp_f64<0x112, 0xf>(v));
  v = fmax(v, dpp_f64<0x114, 0xf>(v));
  v = fmax(v, dpp_f64<0x118, 0xf>(v));
  v = fmax(v, dpp_f64<0x142, 0xa>(v));
  v = fmax(v, dpp_f64<0x143, 0xc>(v));
  return lane63_f64(v);
}

// Block-wide sums over NW waves of K doubles (K*NW <= 96 doubles of scratch).
template <int K, int NW>
__device__ __forceinline__ void block_sum_n(double (&v)[K], double* red) {
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) red[w * K + k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double a = red[k];
      for (int q = 1; q < NW; ++q) a += red[q * K + k];
      v[k] = a;
    }
  __syncthreads();
}

__device__ __forceinline__ void flag_error(DevDiag* d, unsigned bits, long long step) {
  atomicOr(&d->err, bits);
  atomicMin(&d->first_bad, (unsigned long long)step);
}

// ---------------------------------------------------------------------------
// Eq. 1 streaming in pull form with the boundary rules:
//   half-way bounce-back at the bottom wall (and a top wall): f_i(x) = f*_opp(i)(x);
//   open top: populations 4, 7, 8 of the top row come from `topin`.
// ---------------------------------------------------------------------------
template <typename real>
__device__ __forceinline__ void pull(const real* __restrict__ fs, const real* __restrict__ topin,
                                     int gx, int y, int nx, int ny, size_t N, int top_bc,
                                     real f[9]) {
  // y is uniform across the wave, so every choice below is a choice of a uniform plane
  // base and of a per-lane 32-bit offset (one load each, in the scalar-base form)
  const unsigned xm = wrap1(gx - 1, nx), xp = wrap1(gx + 1, nx), x = gx;
  const unsigned row = (unsigned)y * (unsigned)nx;
  auto pl = [&](int i) { return fs + (size_t)i * N; };
  f[0] = ld32(pl(0), row + x);
  f[1] = ld32(pl(1), row + xm);
  f[3] = ld32(pl(3), row + xp);
  // below: the row under y, or bounce-back of this node's 4, 7, 8 at the bottom wall
  const bool below = y > 0;
  const unsigned rb = row - nx;
  f[2] = ld32(pl(below ? 2 : 4), below ? rb + x : row + x);
  f[5] = ld32(pl(below ? 5 : 7), below ? rb + xm : row + x);
  f[6] = ld32(pl(below ? 6 : 8), below ? rb + xp : row + x);
  // above: the row over y, bounce-back of 2, 5, 6 under a top wall, or the open top's
  // incoming populations
  if (y < ny - 1 || top_bc == TOP_WALL) {
    const bool above = y < ny - 1;
    const unsigned ra = row + nx;
    f[4] = ld32(pl(above ? 4 : 2), above ? ra + x : row + x);
    f[7] = ld32(pl(above ? 7 : 5), above ? ra + xp : row + x);
    f[8] = ld32(pl(above ? 8 : 6), above ? ra + xm : row + x);
  } else {
    f[4] = ld32(topin, x);
    f[7] = ld32(topin, nx + x);
    f[8] = ld32(topin, 2 * nx + x);
  }
}

// Inverse of pull: store pre-collision populations v of node (gx, y) into the
// post-collision layout so that the next pull returns them.
template <typename real>
__device__ __forceinline__ void scatter(real* __restrict__ fs, real* __restrict__ topin, int gx,
                                        int y, int nx, int ny, size_t N, int top_bc,
                                        const real v[9]) {
  const unsigned xm = wrap1(gx - 1, nx), xp = wrap1(gx + 1, nx), x = gx;
  const unsigned row = (unsigned)y * (unsigned)nx;
  auto pl = [&](int i) { return fs + (size_t)i * N; };
  st32(pl(0), row + x, v[0]);
  st32(pl(1), row + xm, v[1]);
  st32(pl(3), row + xp, v[3]);
  if (y > 0) {
    const unsigned rb = row - nx;
    st32(pl(2), rb + x, v[2]);
    st32(pl(5), rb + xm, v[5]);
    st32(pl(6), rb + xp, v[6]);
  } else {
    st32(pl(4), row + x, v[2]);
    st32(pl(7), row + x, v[5]);
    st32(pl(8), row + x, v[6]);
  }
  if (y < ny - 1) {
    const unsigned ra = row + nx;
    st32(pl(4), ra + x, v[4]);
    st32(pl(7), ra + xp, v[7]);
    st32(pl(8), ra + xm, v[8]);
  } else if (top_bc == TOP_WALL) {
    st32(pl(2), row + x, v[4]);
    st32(pl(5), row + x, v[7]);
    st32(pl(6), row + x, v[8]);
  } else {
    st32(topin, x, v[4]);
    st32(topin, nx + x, v[7]);
    st32(topin, 2 * nx + x, v[8]);
  }
}

// ---------------------------------------------------------------------------
// Eq. 7 with Eq. 28, in FP64: psi = sqrt(2 (p - rho/3) / G).
// ---------------------------------------------------------------------------
// Returns the radicand 2 (p - rho/3) / G (0 when it is not positive); the caller takes
// the square root in its own precision.
// The square root and the division use the hardware FP64 estimates refined by Newton
// steps (relative error near 1e-15, far below the FP32 precision of psi).
__device__ __forceinline__ double eos_psi2(const KParams& P, double r, double TE, unsigned& err) {
  double phi;
  if (P.flags & FREEZE_EOS_T) {
    phi = P.phi_sat;
  } else {
    const double x = TE * P.inv_Tc;
    double y = __builtin_amdgcn_rsq(x);   // 1/sqrt(x), then two Newton steps
    y = y * (1.5 - (0.5 * x) * (y * y));
    y = y * (1.5 - (0.5 * x) * (y * y));
    const double s = 1.0 + P.kappa * (1.0 - x * y);
    phi = s * s;
  }
  const double br = P.b * r;
  const double d1 = 1.0 - br;
  const double d2 = 1.0 + 2.0 * br - br * br;
  // p = rho R T / d1 - a phi rho^2 / d2 over one common denominator
  const double den = d1 * d2;
  double q = __builtin_amdgcn_rcp(den);  // 1/den, then two Newton steps
  q = fma(q, fma(-den, q, 1.0), q);
  q = fma(q, fma(-den, q, 1.0), q);
  const double p = (r * P.R * TE * d2 - P.a * phi * r * r * d1) * q;
  const double rad = (p - r * P.inv3) * P.two_G;
  if (!(r > 0.0)) err |= ERR_RHO;
  if (!(d1 > 0.0)) err |= ERR_COVOLUME;
  if (!(rad > 0.0)) {
    err |= (isfinite(rad) ? ERR_RADICAND : ERR_NONFINITE);
    return 0.0;
  }
  return rad;
}

// The same in the operation order of the plain definition (used by the FP64 build,
// which is compiled without contraction so that it rounds like a plain reading of
// Eq. 7 and Eq. 28).
__device__ __forceinline__ double eos_psi_plain(const KParams& P, double rho, double T, unsigned& err) {
  double phi;
  if (P.flags & FREEZE_EOS_T) {
    phi = P.phi_sat;
  } else {
    const double s = 1.0 + P.kappa * (1.0 - sqrt(T / P.Tc));
    phi = s * s;
  }
  const double a = P.a, b = P.b;
  const double pe = rho * P.R * T / (1.0 - b * rho) -
                    a * phi * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
  const double rad = 2.0 * (pe - rho / 3.0) / P.G;
  if (!(rho > 0.0)) err |= ERR_RHO;
  if (!(1.0 - b * rho > 0.0)) err |= ERR_COVOLUME;
  if (!(rad > 0.0)) {
    err |= (isfinite(rad) ? ERR_RADICAND : ERR_NONFINITE);
    return 0.0;
  }
  return sqrt(rad);
}

// ---------------------------------------------------------------------------
// MRT collision (Eq. 2-5, Eq. 8) in increment form: f* = f + M^-1 dm, where dm is
// non-zero only for the non-conserved moments and the momentum (dm_j = F).
// ---------------------------------------------------------------------------
template <typename real>
struct CollideConst {
  real s_e, s_z, s_q, c_e, c_z, c_q, sig_e, sig_z, rho_v, inv_drho, tau_v, dtau;
};

template <typename real>
__device__ __forceinline__ void collide(real f[9], real rho, real Fx, real Fy, real qsig,
                                        const CollideConst<real>& c, real& uxo, real& uyo) {
  const real h = real(0.5);
  // momentum, summed in the order of the moment matrix rows
  const real jx = ((((f[1] - f[3]) + f[5]) - f[6]) - f[7]) + f[8];
  const real jy = ((((f[2] - f[4]) + f[5]) + f[6]) - f[7]) - f[8];
  const real irho = fast_rcp(rho);
  const real ux = (jx + h * Fx) * irho;
  const real uy = (jy + h * Fy) * irho;
  const real s14 = (f[1] + f[2]) + (f[3] + f[4]);
  const real s58 = (f[5] + f[6]) + (f[7] + f[8]);
  const real m1 = real(-4) * f[0] - s14 + real(2) * s58;
  const real m2 = real(4) * f[0] - real(2) * s14 + s58;
  const real m4 = real(-2) * (f[1] - f[3]) + ((f[5] - f[6]) - (f[7] - f[8]));
  const real m6 = real(-2) * (f[2] - f[4]) + ((f[5] + f[6]) - (f[7] + f[8]));
  const real m7 = (f[1] + f[3]) - (f[2] + f[4]);
  const real m8 = (f[5] + f[7]) - (f[6] + f[8]);
  const real usq = ux * ux + uy * uy;
  const real uF = ux * Fx + uy * Fy;
  // equilibrium moments, Eq. 4
  const real e1 = rho * (real(-2) + real(3) * usq);
  const real e2 = rho * (real(1) - real(3) * usq);
  const real e4 = -rho * ux, e6 = -rho * uy;
  const real e7 = rho * (ux * ux - uy * uy), e8 = rho * ux * uy;
  // source, Eq. 8 (sigma terms as |F_m|^2 / psi^2 times 12 sigma/(tau - 1/2))
  const real S1 = real(6) * uF + c.sig_e * qsig;
  const real S2 = real(-6) * uF - c.sig_z * qsig;
  const real S7 = real(2) * (ux * Fx - uy * Fy);
  const real S8 = ux * Fy + uy * Fx;
  // viscous rate from tau interpolated linearly in density
  real w = (rho - c.rho_v) * c.inv_drho;
  w = w < real(0) ? real(0) : (w > real(1) ? real(1) : w);
  const real snu = fast_rcp(c.tau_v + c.dtau * w);
  const real cnu = real(1) - h * snu;
  const real d1 = -c.s_e * (m1 - e1) + c.c_e * S1;
  const real d2 = -c.s_z * (m2 - e2) + c.c_z * S2;
  const real d4 = -c.s_q * (m4 - e4) - c.c_q * Fx;
  const real d6 = -c.s_q * (m6 - e6) - c.c_q * Fy;
  const real d7 = -snu * (m7 - e7) + cnu * S7;
  const real d8 = -snu * (m8 - e8) + cnu * S8;
  // f += M^-1 dm  (M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4))
  const real i9 = real(1) / real(9), i36 = real(1) / real(36), i18 = real(1) / real(18);
  const real i6 = real(1) / real(6), i12 = real(1) / real(12), i4 = real(0.25);
  const real A = -d1 * i36 - d2 * i18;
  const real B = d1 * i18 + d2 * i36;
  const real cx = (Fx - d4) * i6, cy = (Fy - d6) * i6;
  const real dx = Fx * i6 + d4 * i12, dy = Fy * i6 + d6 * i12;
  const real q7 = d7 * i4, q8 = d8 * i4;
  f[0] += (d2 - d1) * i9;
  f[1] += A + cx + q7;
  f[3] += A - cx + q7;
  f[2] += A + cy - q7;
  f[4] += A - cy - q7;
  f[5] += B + dx + dy + q8;
  f[6] += B - dx + dy - q8;
  f[7] += B - dx - dy + q8;
  f[8] += B + dx - dy - q8;
  uxo = ux;
  uyo = uy;
}

// MRT collision in the plain matrix form m* = m - L (m - m^eq) + (I - L/2) S,
// f* = M^-1 m*, summing every matrix-vector product in index order.  The FP64 build
// uses it; it is mathematically the increment form above.
struct MomentTables {
  double Mi[9][9];
  __host__ __device__ constexpr MomentTables() : Mi{} {
    constexpr int M[9][9] = {{1, 1, 1, 1, 1, 1, 1, 1, 1},     {-4, -1, -1, -1, -1, 2, 2, 2, 2},
                             {4, -2, -2, -2, -2, 1, 1, 1, 1}, {0, 1, 0, -1, 0, 1, -1, -1, 1},
                             {0, -2, 0, 2, 0, 1, -1, -1, 1},  {0, 0, 1, 0, -1, 1, 1, -1, -1},
                             {0, 0, -2, 0, 2, 1, 1, -1, -1},  {0, 1, -1, 1, -1, 0, 0, 0, 0},
                             {0, 0, 0, 0, 0, 1, -1, 1, -1}};
    for (int k = 0; k < 9; ++k) {
      double nk = 0.0;
      for (int i = 0; i < 9; ++i) nk += (double)(M[k][i] * M[k][i]);
      for (int i = 0; i < 9; ++i) Mi[i][k] = (double)M[k][i] / nk;
    }
  }
};

__device__ __forceinline__ void collide_plain(const KParams& P, double f[9], double Fx, double Fy,
                                              double Fmx, double Fmy, double psi, double& uxo,
                                              double& uyo) {
  constexpr MomentTables T;
  double m[9];
  m[0] = ((((((((f[0] + f[1]) + f[2]) + f[3]) + f[4]) + f[5]) + f[6]) + f[7]) + f[8]);
  m[1] = (((((((-4.0 * f[0] - f[1]) - f[2]) - f[3]) - f[4]) + 2.0 * f[5]) + 2.0 * f[6]) + 2.0 * f[7]) + 2.0 * f[8];
  m[2] = (((((((4.0 * f[0] + -2.0 * f[1]) + -2.0 * f[2]) + -2.0 * f[3]) + -2.0 * f[4]) + f[5]) + f[6]) + f[7]) + f[8];
  m[3] = ((((f[1] - f[3]) + f[5]) - f[6]) - f[7]) + f[8];
  m[4] = ((((-2.0 * f[1] + 2.0 * f[3]) + f[5]) - f[6]) - f[7]) + f[8];
  m[5] = ((((f[2] - f[4]) + f[5]) + f[6]) - f[7]) - f[8];
  m[6] = ((((-2.0 * f[2] + 2.0 * f[4]) + f[5]) + f[6]) - f[7]) - f[8];
  m[7] = ((f[1] - f[2]) + f[3]) - f[4];
  m[8] = ((f[5] - f[6]) + f[7]) - f[8];
  const double rho = m[0];
  const double ux = (m[3] + 0.5 * Fx) / rho;
  const double uy = (m[5] + 0.5 * Fy) / rho;
  const double usq = ux * ux + uy * uy;
  double meq[9];
  meq[0] = rho;
  meq[1] = rho * (-2.0 + 3.0 * usq);
  meq[2] = rho * (1.0 - 3.0 * usq);
  meq[3] = rho * ux;
  meq[4] = -rho * ux;
  meq[5] = rho * uy;
  meq[6] = -rho * uy;
  meq[7] = rho * (ux * ux - uy * uy);
  meq[8] = rho * ux * uy;
  double w = (rho - P.rho_v) / (P.rho_l - P.rho_v);
  if (w < 0.0) w = 0.0;
  if (w > 1.0) w = 1.0;
  const double snu = 1.0 / (P.tau_v + (P.tau_l - P.tau_v) * w);
  const double lam[9] = {1.0, P.s_e_raw, P.s_z_raw, 1.0, P.s_q, 1.0, P.s_q, snu, snu};
  const double tau_e = 1.0 / P.s_e_raw, tau_z = 1.0 / P.s_z_raw;
  const double sig = 12.0 * P.sigma;
  const double Fm2 = Fmx * Fmx + Fmy * Fmy;
  const double uF = ux * Fx + uy * Fy;
  double S[9];
  S[0] = 0.0;
  S[1] = 6.0 * uF + sig * Fm2 / (psi * psi * (tau_e - 0.5));
  S[2] = -6.0 * uF - sig * Fm2 / (psi * psi * (tau_z - 0.5));
  S[3] = Fx;
  S[4] = -Fx;
  S[5] = Fy;
  S[6] = -Fy;
  S[7] = 2.0 * (ux * Fx - uy * Fy);
  S[8] = ux * Fy + uy * Fx;
  double ms[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) ms[k] = m[k] - lam[k] * (m[k] - meq[k]) + (1.0 - 0.5 * lam[k]) * S[k];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k)
      if (T.Mi[i][k] != 0.0) acc += T.Mi[i][k] * ms[k];
    f[i] = acc;
  }
  uxo = ux;
  uyo = uy;
}

// ---------------------------------------------------------------------------
// Reductions that finish one kernel's partials inside the next kernel's block 0.
// ---------------------------------------------------------------------------

// Scratch layout of `red` (at least RED_SIZE doubles): [0, 96) block sums,
// [96, 112) per-wave maxima, [112] broadcast slot.
constexpr int RED_SIZE = 128;

// Populations 4, 7, 8 entering the top row at column x for the next step:
//   constant pressure (Sec. 3.3): equilibrium at rho_v with the velocity of the row below;
//   convective outlet (Sec. 4.2): (f^n(top) + U f^{n+1}(top-1)) / (1 + U), where the new
//   populations of the row below are pulled from the top row's post-collision values.
// Returns the net mass change of the column: inflow minus the outflow of 2, 5, 6.
template <typename real, bool COH>
__device__ __forceinline__ double outlet_column(const KParams& P, int x, real U,
                                                const real* __restrict__ fpost,
                                                real* __restrict__ topin,
                                                const real* __restrict__ uxa,
                                                const real* __restrict__ uya) {
  const int nx = P.nx, ny = P.ny;
  const size_t N = (size_t)nx * ny;
  const size_t below = (size_t)(ny - 2) * nx, top = (size_t)(ny - 1) * nx;
  real in4, in7, in8;
  if (P.top_bc == TOP_CONST_PRESSURE) {
    const real r = (real)P.rho_v, ux = ldc<COH>(uxa + below + x), uy = ldc<COH>(uya + below + x);
    const real usq = real(1.5) * (ux * ux + uy * uy);
    const real w1 = r / real(9), w2 = r / real(36);
    const real e4 = -uy, e7 = -ux - uy, e8 = ux - uy;
    in4 = w1 * (real(1) + real(3) * e4 + real(4.5) * e4 * e4 - usq);
    in7 = w2 * (real(1) + real(3) * e7 + real(4.5) * e7 * e7 - usq);
    in8 = w2 * (real(1) + real(3) * e8 + real(4.5) * e8 * e8 - usq);
  } else {
    const real inv = real(1) / (real(1) + U);
    const int xm = wrap1(x - 1, nx), xp = wrap1(x + 1, nx);
    in4 = (topin[x] + U * ldc<COH>(fpost + 4 * N + top + x)) * inv;
    in7 = (topin[nx + x] + U * ldc<COH>(fpost + 7 * N + top + xp)) * inv;
    in8 = (topin[2 * nx + x] + U * ldc<COH>(fpost + 8 * N + top + xm)) * inv;
  }
  topin[x] = in4;
  topin[nx + x] = in7;
  topin[2 * nx + x] = in8;
  // populations 2, 5, 6 of the top row leave through the opening
  const real out = (ldc<COH>(fpost + 2 * N + top + x) + ldc<COH>(fpost + 5 * N + top + x)) +
                   ldc<COH>(fpost + 6 * N + top + x);
  return (((double)in4 + (double)in7) + (double)in8) - (double)out;
}

// ---------------------------------------------------------------------------
// Collide kernel: one LB step for a 64 x TY tile.
//   phase 1  pull f^n, rho = sum f (Eq. 5), psi (Eq. 7, 28) for the tile and a
//            one-cell ring, psi into LDS;
//   phase 2  forces (Eq. 6, 9, 10), velocity (Eq. 5), MRT collision (Eq. 2, 8);
//            write f*^n, rho, u; FP64 partial of the mass that the next pull sees.
// ---------------------------------------------------------------------------
// NW waves (64 NW threads) per tile.  A workgroup of HALVES x 64 NW threads runs HALVES
// tiles side by side (one per group of NW waves, `tile` being that group's tile; a tile
// index >= nblkL is an empty tile that only takes part in the barriers).  COH: the
// tile's outputs are read by other workgroups of the same launch (the fused step), so
// they are stored coherently.
template <typename real, int TY, int NW, bool COH, int HALVES = 1>
__device__ __forceinline__ void collide_tile(
    const KParams& P, const real* __restrict__ fsrc, real* __restrict__ fdst,
    const real* __restrict__ topin, const real* __restrict__ Tcur, const real* __restrict__ gw,
    real* __restrict__ rho_out, real* __restrict__ ux_out, real* __restrict__ uy_out,
    const double* __restrict__ mstate_prev, const double* __restrict__ pmin_prev,
    double* __restrict__ mstate_cur, double* __restrict__ partL_out, DevDiag* __restrict__ diag,
    const long long* __restrict__ dstep_prev, long long* __restrict__ dstep_cur, int tile) {
  static_assert(TY % NW == 0 && NW <= 16, "rows of a collide tile per wave");
  constexpr int RPT = TY / NW;  // rows per thread
  constexpr int NTH = NW * 64;
  constexpr int LW = 66;
  __shared__ real spsi_all[HALVES][TY + 2][LW];
  __shared__ double red_all[HALVES][RED_SIZE];
  const int half = HALVES > 1 ? __builtin_amdgcn_readfirstlane((int)threadIdx.x / NTH) : 0;
  real(*spsi)[LW] = spsi_all[half];
  double* red = red_all[half];
  const bool live = tile < P.nblkL;
  if (!live) tile = 0;  // an empty tile: rows beyond the grid, no outputs

  const int t = (int)threadIdx.x - half * NTH, lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int nx = P.nx, ny = P.ny;
  const size_t N = (size_t)nx * ny;

  // Eq. 9: rho_ave = mass of the current state / fluid nodes, the mass being the stored
  // mass of the previous state plus its net inflow through the top (thread 0 sums the
  // same values in the same order in every block).
  double mnow = 0.0;
  if (t == 0) {
    mnow = mstate_prev[0];
    for (int b = 0; b < P.ntxE; ++b) mnow += pmin_prev[b];
  }

  const int x0 = (tile % P.ntxL) * 64, y0 = live ? (tile / P.ntxL) * TY : ny + 1;
  unsigned err = 0;

  real f[RPT][9];
  real rr[RPT];
  const int gxo = wrapm(x0 + lane, nx);
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int ly = wv + NW * k, y = y0 + ly;
    real ps = real(0);
    if (y < ny) {
      pull(fsrc, topin, gxo, y, nx, ny, N, P.top_bc, f[k]);
      real r = f[k][0];
#pragma unroll
      for (int i = 1; i < 9; ++i) r += f[k][i];
      rr[k] = r;
      const double TE = (P.flags & FREEZE_EOS_T) ? P.T_sat : (double)ld32(Tcur, (unsigned)(y + P.nh) * (unsigned)nx + gxo);
      if constexpr (sizeof(real) == 8) ps = eos_psi_plain(P, r, TE, err);
      else ps = sqrtf((float)eos_psi2(P, (double)r, TE, err));
    }
    spsi[ly + 1][lane + 1] = ps;
  }
  // ring of the tile: 66 + 66 + TY + TY cells
  for (int c = t; c < 2 * LW + 2 * TY; c += NTH) {
    int lx, ly;
    if (c < LW) { lx = c - 1; ly = -1; }
    else if (c < 2 * LW) { lx = c - LW - 1; ly = TY; }
    else if (c < 2 * LW + TY) { lx = -1; ly = c - 2 * LW; }
    else { lx = 64; ly = c - 2 * LW - TY; }
    const int y = y0 + ly;
    real ps = real(0);
    if (y >= 0 && y < ny) {
      const int gx = wrapm(x0 + lx, nx);
      real fr[9];
      pull(fsrc, topin, gx, y, nx, ny, N, P.top_bc, fr);
      real r = fr[0];
#pragma unroll
      for (int i = 1; i < 9; ++i) r += fr[i];
      const double TE = (P.flags & FREEZE_EOS_T) ? P.T_sat : (double)ld32(Tcur, (unsigned)(y + P.nh) * (unsigned)nx + gx);
      unsigned e2 = 0;
      if constexpr (sizeof(real) == 8) ps = eos_psi_plain(P, r, TE, e2);
      else ps = sqrtf((float)eos_psi2(P, (double)r, TE, e2));
    }
    spsi[ly + 1][lx + 1] = ps;
  }
  const long long step = dstep_prev[0];
  if (t == 0) {
    red[112] = mnow;
    if (live && tile == 0) {
      mstate_cur[0] = mnow;
      dstep_cur[0] = step + 1;
    }
  }
  __syncthreads();  // publishes spsi and the mass
  const double rho_ave_d = red[112] / ((double)nx * (double)ny);

  CollideConst<real> cc;
  cc.s_e = (real)P.s_e; cc.s_z = (real)P.s_z; cc.s_q = (real)P.s_q;
  cc.c_e = (real)P.c_e; cc.c_z = (real)P.c_z; cc.c_q = (real)P.c_q;
  cc.sig_e = (real)P.sig_e; cc.sig_z = (real)P.sig_z;
  cc.rho_v = (real)P.rho_v; cc.inv_drho = (real)P.inv_drho;
  cc.tau_v = (real)P.tau_v; cc.dtau = (real)P.dtau;
  const real w1 = real(1) / real(3), w2 = real(1) / real(12);
  const real a1 = w1 / real(3), a2 = w2 / real(3);  // Eq. 10 weights
  const real negG = (real)(-P.G), gg = (real)P.g, rho_ave = (real)rho_ave_d;
  const bool open_top = P.top_bc != TOP_WALL;
  double mass = 0.0, uyrow = 0.0;
  real umax2 = real(0);

#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int ly = wv + NW * k, y = y0 + ly;
    if (y >= ny || x0 + lane >= nx) continue;
    const int cx = lane + 1, cy = ly + 1;
    const real pc = spsi[cy][cx];
    real pE = spsi[cy][cx + 1], pW = spsi[cy][cx - 1];
    real pN, pS, pNE, pNW, pSE, pSW;
    real ax = real(0), ay = real(0);
    if (y == 0) {
      // solid neighbours below carry psi of this node (Eq. 6) and the wall strength
      // of their own column (Eq. 10)
      pS = pc; pSE = pc; pSW = pc;
      const real gC = gw[gxo], gL = gw[wrap1(gxo - 1, nx)], gR = gw[wrap1(gxo + 1, nx)];
      ay = ((-(a1 * gC)) - a2 * gL) - a2 * gR;
      ax = (-(a2 * gL)) + a2 * gR;
    } else {
      pS = spsi[cy - 1][cx]; pSE = spsi[cy - 1][cx + 1]; pSW = spsi[cy - 1][cx - 1];
    }
    if (y == ny - 1) {
      if (open_top) {  // zero-gradient ghost row above an open top
        pN = pc; pNE = pE; pNW = pW;
      } else {
        pN = pc; pNE = pc; pNW = pc;
        const real gt = (real)P.Gw_top;
        ay += (a1 * gt + a2 * gt) + a2 * gt;
      }
    } else {
      pN = spsi[cy + 1][cx]; pNE = spsi[cy + 1][cx + 1]; pNW = spsi[cy + 1][cx - 1];
    }
    // Eq. 6: F_m = -G psi(x) sum_i w_i psi(x + e_i) e_i (order e1..e8)
    const real sx = ((((w1 * pE - w1 * pW) + w2 * pNE) - w2 * pNW) - w2 * pSW) + w2 * pSE;
    const real sy = ((((w1 * pN - w1 * pS) + w2 * pNE) + w2 * pNW) - w2 * pSW) - w2 * pSE;
    const real fmx = negG * pc * sx, fmy = negG * pc * sy;
    const real r = rr[k];
    const real pc2 = pc * pc;
    const real Fx = fmx + pc2 * ax;
    const real Fy = (fmy + pc2 * ay) + (-(r - rho_ave) * gg);
    real ux, uy;
    if constexpr (sizeof(real) == 8) {
      collide_plain(P, f[k], Fx, Fy, fmx, fmy, pc, ux, uy);
    } else {
      const real qsig = (fmx * fmx + fmy * fmy) * fast_rcp(pc2);
      collide(f[k], r, Fx, Fy, qsig, cc, ux, uy);
    }
    const unsigned n = (unsigned)y * (unsigned)nx + gxo;
#pragma unroll
    for (int i = 0; i < 9; ++i) stc32<COH>(fdst + i * N, n, f[k][i]);
    stc32<COH>(rho_out, n, r);
    stc32<COH>(ux_out, n, ux);
    stc32<COH>(uy_out, n, uy);
    // post-collision mass (per node in the field precision, accumulated in FP64); the
    // open top's net exchange is added by the outlet block of the energy launch
    const real ms = ((f[k][0] + f[k][1]) + (f[k][2] + f[k][3])) + ((f[k][4] + f[k][5]) + (f[k][6] + f[k][7])) + f[k][8];
    mass += (double)ms;
    const real u2 = ux * ux + uy * uy;
    umax2 = u2 > umax2 ? u2 : umax2;
    if (y == ny - 2) uyrow += (double)uy;
    if (!isfinite(u2)) err |= ERR_NONFINITE;
  }
  if (err) flag_error(diag, err, step);
  double v[2] = {mass, uyrow};
  if constexpr (sizeof(real) == 4) {
    // FP32 path: register-only wave reductions, then the waves in order
    const double vm = wave_max_dpp((double)umax2);
    v[0] = wave_sum_dpp(v[0]);
    v[1] = wave_sum_dpp(v[1]);
    __syncthreads();
    if (lane == 0) {
      red[96 + wv] = vm;
      red[2 * wv] = v[0];
      red[2 * wv + 1] = v[1];
    }
    __syncthreads();
    if (t == 0) {
      double a = red[0], b = red[1];
      for (int q = 1; q < NW; ++q) {
        a += red[2 * q];
        b += red[2 * q + 1];
      }
      v[0] = a;
      v[1] = b;
    }
  } else {
    double vm = wave_max((double)umax2);
    __syncthreads();
    if (lane == 0) red[96 + wv] = vm;
    block_sum_n<2, NW>(v, red);
  }
  if (t == 0 && live) {
    double m = red[96];
    for (int q = 1; q < NW; ++q) m = fmax(m, red[96 + q]);
    stc<COH>(partL_out + 3 * tile, v[0]);
    stc<COH>(partL_out + 3 * tile + 1, m);
    stc<COH>(partL_out + 3 * tile + 2, v[1]);
  }
}

template <typename real, int TY, int NW>
__global__ void __launch_bounds__(NW * 64)
    k_collide(const KParams P, const real* __restrict__ fsrc, real* __restrict__ fdst,
              const real* __restrict__ topin, const real* __restrict__ Tcur,
              const real* __restrict__ gw, real* __restrict__ rho_out, real* __restrict__ ux_out,
              real* __restrict__ uy_out, const double* __restrict__ mstate_prev,
              const double* __restrict__ pmin_prev, double* __restrict__ mstate_cur,
              double* __restrict__ partL_out, DevDiag* __restrict__ diag,
              const long long* __restrict__ dstep_prev, long long* __restrict__ dstep_cur) {
  collide_tile<real, TY, NW, false>(P, fsrc, fdst, topin, Tcur, gw, rho_out, ux_out, uy_out, mstate_prev,
                                    pmin_prev, mstate_cur, partL_out, diag, dstep_prev, dstep_cur,
                                    xcd_tile(blockIdx.x, P.nblkL));
}

// ---------------------------------------------------------------------------
// Energy kernel: T^n -> T^{n+1} on a tile of the temperature grid (heater and fluid
// rows), rho^n and u^n frozen (Eq. 17-18, Eq. 22-27).
//
// The tile (txE <= 56 columns by tyE rows, both chosen per grid) plus a four-cell halo
// and the ghost rows sit in LDS as rows of 64 cells: lane = LDS column, and each wave
// owns whole LDS rows, so everything that depends on the row (ghost, heater, fluid,
// boundary, global address) is wave-uniform scalar work.  Each RK stage is evaluated
// on a region one cell smaller than the previous one, so all four stages run with one
// read of T, rho, u and one write of T.  LDS column c holds global column x0 - 4 + c
// (periodic), LDS row r holds T row j0 - 4 + r.
// ---------------------------------------------------------------------------
constexpr int EW = 64;  // LDS row length = wavefront size

template <typename real, bool ISO, int NW, int HMAX>
__device__ __forceinline__ void energy_lds_tile(
    const KParams& P, const real* __restrict__ Tin, real* __restrict__ Tout,
    const real* __restrict__ rho, const real* __restrict__ uxa, const real* __restrict__ uya,
    double* __restrict__ hist_slot, DevDiag* __restrict__ diag, int sub, double dtd,
    const long long* __restrict__ dstep_prev, int tile) {
  constexpr int H4M = HMAX + 8;
  constexpr int NR4 = (H4M + NW - 1) / NW;        // LDS rows per wave (load, faces)
  constexpr int NC = (HMAX + 6 + NW - 1) / NW;    // stage-1 rows per wave
  __shared__ real sA[H4M][EW];   // stage values (T^n first)
  __shared__ real sB[H4M][EW];   // lambda during set-up, then stage values
  __shared__ real sFx[H4M][EW];  // u_x during set-up, then x-face conductivities
  __shared__ real sFy[H4M][EW];  // u_y during set-up, then y-face conductivities
  __shared__ double red[RED_SIZE];

  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int nx = P.nx, nT = P.nT, nh = P.nh;
  // uniform tiles here (tyE0 == tyE): the LDS layout is sized for tyE rows
  const int TXr = P.txE, TY = P.tyE, H4 = TY + 8;
  const int x0 = (tile % P.ntxE) * TXr, j0 = (tile / P.ntxE) * TY;
  const int gx = wrapm(x0 - 4 + lane, nx);  // global column of this lane
  const bool top_open = P.top_bc != TOP_WALL;
  const real cv = (real)P.cv, cvk = (real)P.cvk;
  // lambda = rho c_v k (Sec. 3.1)
  auto lam_of = [&](real r) -> real {
    if constexpr (sizeof(real) == 8) return r * P.cv * P.k;
    else return r * cvk;
  };
  // Eq. 25 harmonic mean (dx = 1)
  auto face = [](real lp, real ln) -> real {
    if constexpr (sizeof(real) == 8) return 2.0 / (1.0 / lp + 1.0 / ln);
    else return real(2) * lp * ln * fast_rcp(lp + ln);
  };

  // ---- load T, lambda, u of the LDS rows this wave owns (loads first) ----
  {
    real lT[NR4], lR[NR4], lU[NR4], lV[NR4];
#pragma unroll
    for (int k = 0; k < NR4; ++k) {
      const int r = w + NW * k, j = j0 - 4 + r;
      lT[k] = real(0); lR[k] = real(-1); lU[k] = real(0); lV[k] = real(0);
      if (r < H4) {
        if (j >= 0 && j < nT) {
          lT[k] = Tin[(size_t)j * nx + gx];
          if (j >= nh) {
            const size_t n = (size_t)(j - nh) * nx + gx;
            lR[k] = rho[n];
            lU[k] = uxa[n];
            lV[k] = uya[n];
          }
        } else if (j == -1) {
          if (nh == 0) lR[k] = rho[gx];
          if (P.bottom_tbc == TBC_FLUX) lT[k] = Tin[gx];
        } else if (j == nT) {
          const size_t n = (size_t)(P.ny - 1) * nx + gx;
          lR[k] = rho[n];
          if (P.top_tbc != TBC_DIRICHLET) lT[k] = Tin[(size_t)(nT - 1) * nx + gx];
          if (top_open) { lU[k] = uxa[n]; lV[k] = uya[n]; }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NR4; ++k) {
      const int r = w + NW * k, j = j0 - 4 + r;
      if (r < H4) {
        // heater rows (and the ghost row below a heater) have lR < 0: lambda_w
        real lam = lR[k] >= real(0) ? lam_of(lR[k]) : (real)P.lambda_w;
        real T = lT[k];
        if (j == -1) T = (P.bottom_tbc == TBC_FLUX) ? T + (real)P.q_bottom / lam : (real)P.T_bottom;
        else if (j == nT && P.top_tbc == TBC_DIRICHLET) T = (real)P.T_top;
        if (j < -1 || j > nT) lam = real(1);
        sA[r][lane] = T;
        sB[r][lane] = lam;
        sFx[r][lane] = lU[k];
        sFy[r][lane] = lV[k];
      }
    }
  }
  __syncthreads();

  // ---- per-cell coefficients of the stage-1 cells (LDS rows 1 + w + NW k, lanes 1..62) ----
  real T0[NC], Cc[NC], cux[NC], cuy[NC], cla[NC], clb[NC], acc[NC];
  real lamP[ISO ? NC : 1], glx[ISO ? NC : 1], gly[ISO ? NC : 1];
  real crho[sizeof(real) == 8 ? NC : 1], cdv[sizeof(real) == 8 ? NC : 1];  // plain-order latent term
  using rc_t = typename std::conditional<sizeof(real) == 8, double, float>::type;
  rc_t rcv[NC];
  const real inv3 = real(1) / real(3), inv12 = real(1) / real(12);
  const bool lane_r3 = lane >= 1 && lane <= EW - 2;
  const bool lane_out = lane >= 4 && lane < 4 + TXr && x0 + lane - 4 < nx;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int r = 1 + w + NW * k, j = j0 - 4 + r;
    T0[k] = real(0); Cc[k] = real(0); cux[k] = real(0); cuy[k] = real(0);
    cla[k] = real(0); clb[k] = real(0); acc[k] = real(0);
    rcv[k] = 0;
    if (r <= H4 - 2) {
      T0[k] = sA[r][lane];
      if constexpr (ISO) {
        // lambda and its Eq. 19 gradient for Eq. 21 (ghost rows copy the inner lambda)
        if (lane_r3) {
          lamP[k] = sB[r][lane];
          glx[k] = (sB[r][lane + 1] - sB[r][lane - 1]) * inv3 +
                   ((sB[r + 1][lane + 1] - sB[r - 1][lane - 1]) + (sB[r - 1][lane + 1] - sB[r + 1][lane - 1])) * inv12;
          gly[k] = (sB[r + 1][lane] - sB[r - 1][lane]) * inv3 +
                   ((sB[r + 1][lane + 1] - sB[r - 1][lane - 1]) + (sB[r + 1][lane - 1] - sB[r - 1][lane + 1])) * inv12;
        }
      }
      if (j >= 0 && j < nT) {
        if (j < nh) {
          rcv[k] = (rc_t)P.rcw;
          Cc[k] = (real)P.inv_rcw;
        } else {
          real rr;
          if constexpr (sizeof(real) == 8) {
            rr = rho[(size_t)(j - nh) * nx + gx];
            crho[k] = rr;
            rcv[k] = (double)rr * P.cv;
          } else {
            rr = sB[r][lane] * (real)(1.0 / P.cvk);
            rcv[k] = rr * cv;
          }
          Cc[k] = fast_rcp(rr * cv);
          cux[k] = sFx[r][lane];
          cuy[k] = sFy[r][lane];
          if (!(P.flags & NO_LATENT) && lane_r3) {
            // div u by Eq. 19 (u = 0 on solids, zero-gradient above an open top)
            real dudx, dvdy;
            if constexpr (sizeof(real) == 8) {
              dudx = (sFx[r][lane + 1] - sFx[r][lane - 1]) / 3.0 + (sFx[r + 1][lane + 1] - sFx[r - 1][lane - 1]) / 12.0 +
                     (sFx[r - 1][lane + 1] - sFx[r + 1][lane - 1]) / 12.0;
              dvdy = (sFy[r + 1][lane] - sFy[r - 1][lane]) / 3.0 + (sFy[r + 1][lane + 1] - sFy[r - 1][lane - 1]) / 12.0 +
                     (sFy[r + 1][lane - 1] - sFy[r - 1][lane + 1]) / 12.0;
              cdv[k] = dudx + dvdy;
            } else {
              dudx = (sFx[r][lane + 1] - sFx[r][lane - 1]) * inv3 +
                     ((sFx[r + 1][lane + 1] - sFx[r - 1][lane - 1]) + (sFx[r - 1][lane + 1] - sFx[r + 1][lane - 1])) * inv12;
              dvdy = (sFy[r + 1][lane] - sFy[r - 1][lane]) * inv3 +
                     ((sFy[r + 1][lane + 1] - sFy[r - 1][lane - 1]) + (sFy[r + 1][lane - 1] - sFy[r - 1][lane + 1])) * inv12;
              // (dp/dT)_v = A(rho) - B(rho) phi'(T) (Eq. 28): A = rho R/(1 - b rho),
              // B = a rho^2/(1 + 2 b rho - b^2 rho^2); no cancellation here, FP32 suffices
              const real br = (real)P.b * rr;
              const real Ad = rr * (real)P.R * fast_rcp(real(1) - br);
              const real Bd = (real)P.a * rr * rr * fast_rcp(real(1) + real(2) * br - br * br);
              const real cd = Cc[k] * (dudx + dvdy);
              cla[k] = cd * Ad;
              clb[k] = cd * Bd * (real)P.kappa;
            }
          }
        }
      }
    }
  }
  __syncthreads();  // u and lambda have been consumed

  // ---- face conductivities (Eq. 25); a ghost face takes the inner node's lambda ----
#pragma unroll
  for (int k = 0; k < NR4; ++k) {
    const int r = w + NW * k, j = j0 - 4 + r;
    if (r < H4) {
      const real lp = sB[r][lane];
      real fx = real(0), fy = real(0);
      if (lane + 1 < EW) fx = face(lp, sB[r][lane + 1]);
      if (r + 1 < H4) {
        const real ln = sB[r + 1][lane];
        if (j == -1) fy = ln;
        else if (j == nT - 1) fy = lp;
        else fy = face(lp, ln);
      }
      sFx[r][lane] = fx;
      sFy[r][lane] = fy;
    }
  }
  __syncthreads();  // faces ready; sB is free for stage values

  const real dt = (real)dtd;
  const real kap = (real)P.kappa, onek = real(1) + (real)P.kappa, invTc = (real)P.inv_Tc;
  const real qb = (real)P.q_bottom, Tbot = (real)P.T_bottom, Ttop = (real)P.T_top;
  const bool flux_bottom = P.bottom_tbc == TBC_FLUX;
  const bool top_dirichlet = P.top_tbc == TBC_DIRICHLET;
  double Qb = 0.0, Qt = 0.0, Qs = 0.0;
  const int fl = P.flags;
  // A plain tile's halo holds fluid rows only (no heater, no ghost rows): its stages
  // need no boundary handling.
  const bool plain_tile = (j0 - 4 >= nh) && (j0 + TY + 3 <= nT - 1);

  auto run_stages = [&](auto plain_tag) {
    constexpr bool PLAIN = decltype(plain_tag)::value;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const real* inb = (s & 1) ? &sB[0][0] : &sA[0][0];
      real* outb = (s & 1) ? &sA[0][0] : &sB[0][0];
      const real* fxb = &sFx[0][0];
      const real* fyb = &sFy[0][0];
      const real wgt = (s == 0 || s == 3) ? real(1) : real(2);
      const bool lane_s = lane >= 1 + s && lane < EW - 1 - s;
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const int r = 1 + w + NW * k, j = j0 - 4 + r;
        // stage s covers LDS rows [1 + s, H4 - 1 - s) and lanes [1 + s, 63 - s)
        if (r < 1 + s || r >= H4 - 1 - s) continue;
        if (!PLAIN && (j < 0 || j >= nT)) continue;
        if (!lane_s) continue;
        const int o = r * EW + lane;
        const real Tp = inb[o];
        const real E = inb[o + 1], W = inb[o - 1], Nn = inb[o + EW], S = inb[o - EW];
        const real fe = fxb[o], fw = fxb[o - 1], fn = fyb[o], fs = fyb[o - EW];
        const bool bottom = !PLAIN && j == 0, top = !PLAIN && j == nT - 1;
        real qs;
        if (bottom && flux_bottom) qs = qb;
        else qs = fs * (S - Tp);
        const real qn = fn * (Nn - Tp);
        const real NE = inb[o + EW + 1], NW_ = inb[o + EW - 1];
        const real SE = inb[o - EW + 1], SW = inb[o - EW - 1];
        real gxd = real(0), gyd = real(0);
        if (ISO || !(fl & NO_ADVECTION)) {
          // Eq. 19 isotropic gradient
          if constexpr (sizeof(real) == 8) {
            gxd = (E - W) / 3.0 + (NE - SW) / 12.0 + (SE - NW_) / 12.0;
            gyd = (Nn - S) / 3.0 + (NE - SW) / 12.0 + (NW_ - SE) / 12.0;
          } else {
            gxd = (E - W) * inv3 + ((NE - SW) + (SE - NW_)) * inv12;
            gyd = (Nn - S) * inv3 + ((NE - SW) + (NW_ - SE)) * inv12;
          }
        }
        real D;
        if constexpr (!ISO) {
          // Eq. 22-26: heat through the four faces of the control volume (dx = 1)
          D = ((fe * (E - Tp) + fw * (W - Tp)) + qn) + qs;
        } else {
          // Eq. 21 with Eq. 20: lambda Lap T + grad lambda . grad T (comparison scheme)
          const real lap =
              (((((((((NE + NW_) + SE) + SW) + real(4) * E) + real(4) * W) + real(4) * Nn) + real(4) * S) -
                real(20) * Tp)) /
              real(6);
          D = lamP[k] * lap + (glx[k] * gxd + gly[k] * gyd);
        }
        real h;
        if constexpr (sizeof(real) == 8) h = D / rcv[k];
        else h = Cc[k] * D;
        if (PLAIN || j >= nh) {
          if (!(fl & NO_ADVECTION)) h += -(cux[k] * gxd + cuy[k] * gyd);
          if (!(fl & NO_LATENT)) {
            if constexpr (sizeof(real) == 8) {
              // -(T/(rho c_v)) (dp/dT)_v div u, Eq. 17 with Eq. 28, in plain order
              const double rr = crho[k], b = P.b;
              const double s1 = 1.0 + P.kappa * (1.0 - sqrt(Tp / P.Tc));
              const double dphi = -P.kappa * s1 / sqrt(Tp * P.Tc);
              const double dpdT = rr * P.R / (1.0 - b * rr) - P.a * dphi * rr * rr / (1.0 + 2.0 * b * rr - b * b * rr * rr);
              h += -(Tp / rcv[k]) * dpdT * cdv[k];
            } else {
              // -(T/(rho c_v)) (dp/dT)_v div u with T phi'(T) = -kappa s (1 + kappa - kappa s)
              const real sg = __builtin_amdgcn_sqrtf(Tp * invTc);
              h += -(cla[k] * Tp + clb[k] * sg * (onek - kap * sg));
            }
          }
        }
        if constexpr (!PLAIN) {
          const bool out_row = r >= 4 && r < 4 + TY;
          if (out_row && lane_out) {
            if (bottom) Qb += (double)(wgt * qs);
            if (top && top_dirichlet) Qt += (double)(wgt * qn);
            if (nh > 0 && j == nh) Qs += (double)(wgt * qs);
          }
        }
        if (s < 3) {
          const real cs = (s == 2) ? dt : real(0.5) * dt;
          const real Yn = T0[k] + cs * h;
          outb[o] = Yn;
          acc[k] = (s == 0) ? h : acc[k] + real(2) * h;
          if constexpr (!PLAIN) {
            // ghost rows follow the stage value of the row next to them
            if (bottom) outb[o - EW] = flux_bottom ? Yn + qb / fs : Tbot;
            if (top) outb[o + EW] = top_dirichlet ? Ttop : Yn;
          }
        } else {
          acc[k] = T0[k] + (dt / real(6)) * (acc[k] + h);
        }
      }
      __syncthreads();
    }
  };
  if (plain_tile) run_stages(std::true_type{});
  else run_stages(std::false_type{});

  // ---- write T^{n+1}, FP64 partials ----
  unsigned err = 0;
  double v[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int r = 1 + w + NW * k, j = j0 - 4 + r;
    if (r < 4 || r >= 4 + TY || j >= nT || !lane_out) continue;
    const real Tn = acc[k];
    if (!isfinite(Tn)) err |= ERR_NONFINITE;
    Tout[(size_t)j * nx + gx] = Tn;
    v[0] += (double)rcv[k] * ((double)Tn - (double)T0[k]);
    v[1] += (double)rcv[k] * (double)Tn;
  }
  if (err) flag_error(diag, err, dstep_prev[0]);
  const double d6 = dtd / 6.0;
  v[2] = Qb * d6;
  v[3] = Qt * d6;
  v[4] = Qs * d6;
  if (nh == 0) v[4] = v[2];
  block_sum_n<5, NW>(v, red);
  if (t == 0) {
    double* pe = hist_slot + 5 * tile;
    if (sub == 0) {
#pragma unroll
      for (int k = 0; k < 5; ++k) pe[k] = v[k];
    } else {
      pe[0] += v[0];
      pe[1] = v[1];
      pe[2] += v[2];
      pe[3] += v[3];
      pe[4] += v[4];
    }
  }
}

// Open top: the populations entering the top row at the next step, for every column, and
// the net inflow of each energy tile column (FP64, lanes summed in a fixed order).  Run
// by one whole workgroup of NW waves beside the tiles of the energy launch, once per LB
// step, so that its chain of dependent loads does not lengthen any tile.
template <typename real, int NW, bool COH = false>
__device__ __forceinline__ void outlet_block(const KParams& P, const real* __restrict__ fpost,
                                             real* __restrict__ topin, const real* __restrict__ uxa,
                                             const real* __restrict__ uya, const double* __restrict__ partL_cur,
                                             double* __restrict__ pmin_cur) {
  __shared__ double uo;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (P.top_bc == TOP_WALL) {  // closed top: no exchange
    for (int b = t; b < P.ntxE; b += NW * 64) pmin_cur[b] = 0.0;
    return;
  }
  real U = real(0);
  if (P.top_bc == TOP_CONVECTIVE) {
    if (t == 0) {
      // mean outflow velocity of the row below the top, from the collide partials
      const int ry = (P.ny - 2) / P.tyL;
      double us = 0.0;
      for (int bx = 0; bx < P.ntxL; ++bx) us += ldc<COH>(partL_cur + 3 * (ry * P.ntxL + bx) + 2);
      us /= P.nx;
      uo = us > 0.0 ? us : 0.0;
    }
    __syncthreads();
    U = (real)uo;
  }
  for (int b = w; b < P.ntxE; b += NW) {
    const int x = b * P.txE + lane;
    double d = 0.0;
    if (lane < P.txE && x < P.nx) d = outlet_column<real, COH>(P, x, U, fpost, topin, uxa, uya);
    d = wave_sum(d);
    if (lane == 0) pmin_cur[b] = d;
  }
}

template <typename real, bool ISO, int NW, int HMAX>
__global__ void __launch_bounds__(NW * 64)
    k_energy(const KParams P, const real* __restrict__ Tin, real* __restrict__ Tout,
             const real* __restrict__ rho, const real* __restrict__ uxa,
             const real* __restrict__ uya, double* __restrict__ hist_slot,
             const real* __restrict__ fpost, real* __restrict__ topin,
             const double* __restrict__ partL_cur, double* __restrict__ pmin_cur,
             DevDiag* __restrict__ diag, int sub, double dtd,
             const long long* __restrict__ dstep_prev) {
  // block 0: the open-top rule; blocks 1..nblkE: the tiles
  if (blockIdx.x == 0) {
    if (sub == 0) outlet_block<real, NW>(P, fpost, topin, uxa, uya, partL_cur, pmin_cur);
    return;
  }
  energy_lds_tile<real, ISO, NW, HMAX>(P, Tin, Tout, rho, uxa, uya, hist_slot, diag, sub, dtd, dstep_prev,
                                       xcd_tile_edges_first(blockIdx.x - 1, P.nblkE));
}

// ---------------------------------------------------------------------------
// Initialisation / field access kernels (same 64 x TY tiling as k_collide).
// ---------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(NT)
    k_scatter(const KParams P, const real* __restrict__ src, int src_is_rho, real* __restrict__ fdst,
              real* __restrict__ topin, double* __restrict__ partL_out) {
  __shared__ double red[RED_SIZE];
  const int t = threadIdx.x, lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int nx = P.nx, ny = P.ny;
  const size_t N = (size_t)nx * ny;
  const int TY = P.tyL;
  const int tile = xcd_tile(blockIdx.x, P.nblkL);
  const int x0 = (tile % P.ntxL) * 64, y0 = (tile / P.ntxL) * TY;
  double mass = 0.0;
  for (int ly = wv; ly < TY; ly += 4) {
    const int y = y0 + ly, x = x0 + lane;
    if (y >= ny || x >= nx) continue;
    const size_t n = (size_t)y * nx + x;
    real v[9];
    if (src_is_rho) {
      // equilibrium at rest: w_i rho
      const real r = src[n];
      v[0] = r * (real(4) / real(9));
      for (int i = 1; i < 5; ++i) v[i] = r / real(9);
      for (int i = 5; i < 9; ++i) v[i] = r / real(36);
    } else {
      for (int i = 0; i < 9; ++i) v[i] = src[i * N + n];
    }
    scatter(fdst, topin, x, y, nx, ny, N, P.top_bc, v);
    double ms = 0.0;
    for (int i = 0; i < 9; ++i) ms += (double)v[i];
    mass += ms;
  }
  double vv[1] = {mass};
  block_sum_n<1, NT / 64>(vv, red);
  if (t == 0) {
    partL_out[3 * tile] = vv[0];
    partL_out[3 * tile + 1] = 0.0;
    partL_out[3 * tile + 2] = 0.0;
  }
}

template <typename real>
__global__ void __launch_bounds__(NT)
    k_gather(const KParams P, const real* __restrict__ fs, const real* __restrict__ topin,
             real* __restrict__ out) {
  const int nx = P.nx, ny = P.ny;
  const size_t N = (size_t)nx * ny;
  for (size_t n = (size_t)blockIdx.x * NT + threadIdx.x; n < N; n += (size_t)gridDim.x * NT) {
    const int y = (int)(n / nx), x = (int)(n - (size_t)y * nx);
    real f[9];
    pull(fs, topin, x, y, nx, ny, N, P.top_bc, f);
    for (int i = 0; i < 9; ++i) out[i * N + n] = f[i];
  }
}

// Per-step totals of the energy partials: block b sums history slot (first + b) % hist
// over the energy tiles in tile order.  (Templated on the field type only so that each
// precision's translation unit has its own copy.)
// Per-step totals of the per-tile energy partials (one block per history slot).
__device__ __forceinline__ void reduce_steps_block(const KParams& P, const double* __restrict__ hist,
                                                   double* __restrict__ steps, int first, int hist_cap, int s) {
  __shared__ double red[RED_SIZE];
  const int slot = (first + s) % hist_cap;
  const double* h = hist + (size_t)slot * P.nblkE * 5;
  double v[5] = {0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < P.nblkE; b += NT)
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] += h[5 * b + k];
  block_sum_n<5, NT / 64>(v, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 5; ++k) steps[5 * slot + k] = v[k];
}

template <typename real>
__global__ void __launch_bounds__(NT)
    k_reduce_steps(const KParams P, const double* __restrict__ hist, double* __restrict__ steps,
                   int first, int hist_cap) {
  reduce_steps_block(P, hist, steps, first, hist_cap, blockIdx.x);
}

// Fold `count` reduced steps into the cumulative diagnostics in step order (running
// mean / variance of the bottom heat flux by Welford's update), then the mass, rho_ave
// and max speed of the current state from the last collide partials.
// Folds `count` per-step totals into the diagnostics in step order (running Welford
// statistics of the bottom flux) and recomputes mass, rho_ave and the maximum speed of
// the current state (one block).
__device__ __forceinline__ void finish_block(const KParams& P, const double* __restrict__ steps, int first,
                                             int count, int hist_cap, const double* __restrict__ partL_last,
                                             const double* __restrict__ pmin_last, DevDiag* __restrict__ diag) {
  constexpr int FOLD_CHUNK = 256;  // steps staged in LDS at a time
  __shared__ double red[RED_SIZE];
  __shared__ double sv[5 * FOLD_CHUNK];
  __shared__ double sq[2 * FOLD_CHUNK];  // each step's q_bottom and q_surface (per unit length)
  const int t = threadIdx.x;
  // thread 0 folds the steps in order; the whole block first stages each chunk of them in
  // LDS, so that the fold does not wait on one global load after another
  DevDiag& dg = *diag;
  double dE = 0, en = 0, Qb = 0, Qt = 0, Qs = 0, qb = 0, qs = 0, qm = 0, m2 = 0;
  long long nr = 0;
  if (t == 0 && count > 0) {
    dE = dg.dE_cum; en = dg.energy; Qb = dg.Q_bottom_cum; Qt = dg.Q_top_cum; Qs = dg.Q_surface_cum;
    qb = dg.q_bottom; qs = dg.q_surface; qm = dg.q_mean; m2 = dg.q_m2;
    nr = dg.nred;
  }
  for (int base = 0; base < count; base += FOLD_CHUNK) {
    const int nc = min(FOLD_CHUNK, count - base);
    for (int i = t; i < 5 * nc; i += NT) {
      const double v = steps[5 * ((first + base + i / 5) % hist_cap) + i % 5];
      sv[i] = v;
      if (i % 5 == 2) sq[2 * (i / 5)] = v / P.nx;
      if (i % 5 == 4) sq[2 * (i / 5) + 1] = v / P.nx;
    }
    __syncthreads();
    if (t == 0) {
      for (int c = 0; c < nc; ++c) {
        const double* v = sv + 5 * c;
        dE += v[0];
        en = v[1];
        Qb += v[2];
        Qt += v[3];
        Qs += v[4];
        qb = sq[2 * c];
        qs = sq[2 * c + 1];
        nr += 1;
        const double cnt = (double)nr, q = qb;
        const double dl = q - qm;
        qm += dl / cnt;
        m2 += dl * (q - qm);
      }
    }
    __syncthreads();
  }
  if (t == 0 && count > 0) {
    dg.dE_cum = dE; dg.energy = en; dg.Q_bottom_cum = Qb; dg.Q_top_cum = Qt; dg.Q_surface_cum = Qs;
    dg.q_bottom = qb; dg.q_surface = qs; dg.q_mean = qm; dg.q_m2 = m2; dg.nred = nr;
  }
  double mv[1] = {0.0};
  double vm = 0.0;
  for (int b = t; b < P.nblkL; b += NT) {
    mv[0] += partL_last[3 * b];
    vm = fmax(vm, partL_last[3 * b + 1]);
  }
  for (int b = t; b < P.ntxE; b += NT) mv[0] += pmin_last[b];
  vm = wave_max(vm);
  __syncthreads();
  if ((t & 63) == 0) red[96 + (t >> 6)] = vm;
  block_sum_n<1, NT / 64>(mv, red);
  if (t == 0) {
    diag->mass = mv[0];
    diag->rho_ave = mv[0] / ((double)P.nx * (double)P.ny);
    diag->max_speed = sqrt(fmax(fmax(red[96], red[97]), fmax(red[98], red[99])));
  }
}

template <typename real>
__global__ void __launch_bounds__(NT)
    k_finish(const KParams P, const double* __restrict__ steps, int first, int count, int hist_cap,
             const double* __restrict__ partL_last, const double* __restrict__ pmin_last,
             DevDiag* __restrict__ diag) {
  finish_block(P, steps, first, count, hist_cap, partL_last, pmin_last, diag);
}

template <typename real>
__global__ void k_convert_in(const double* __restrict__ src, real* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT)
    dst[i] = (real)src[i];
}

}  // namespace lbmk
