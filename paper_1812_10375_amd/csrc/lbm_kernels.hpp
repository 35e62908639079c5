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
//   partL     nblkL x 2     per-block FP64 partials of the collide kernel
//   partE     nblkE x 5     per-block FP64 partials of the energy kernel
//   diag      DevDiag       FP64 diagnostics, reduced in a fixed order every step
//
// Per step two kernels run: k_collide (moments, EOS, forces, MRT collision) and
// k_energy (all four RK4 stages of the temperature equation on an LDS tile with a
// four-cell halo).  Block 0 of each kernel also finishes the previous kernel's
// reductions, so no extra launch and no atomics are needed for the diagnostics.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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

template <typename real>
__device__ __forceinline__ real rcp(real v) { return real(1) / v; }

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

// Block-wide sums of K doubles in a fixed order (wave tree, then waves in order).
// Result is valid in thread 0.  red must hold 4*K (<= 32) doubles.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red) {
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
    for (int k = 0; k < K; ++k) v[k] = ((red[k] + red[K + k]) + red[2 * K + k]) + red[3 * K + k];
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
  const int xm = wrap1(gx - 1, nx), xp = wrap1(gx + 1, nx);
  const size_t row = (size_t)y * nx;
  f[0] = fs[row + gx];
  f[1] = fs[N + row + xm];
  f[3] = fs[3 * N + row + xp];
  if (y > 0) {
    const size_t rb = row - nx;
    f[2] = fs[2 * N + rb + gx];
    f[5] = fs[5 * N + rb + xm];
    f[6] = fs[6 * N + rb + xp];
  } else {
    f[2] = fs[4 * N + row + gx];
    f[5] = fs[7 * N + row + gx];
    f[6] = fs[8 * N + row + gx];
  }
  if (y < ny - 1) {
    const size_t ra = row + nx;
    f[4] = fs[4 * N + ra + gx];
    f[7] = fs[7 * N + ra + xp];
    f[8] = fs[8 * N + ra + xm];
  } else if (top_bc == TOP_WALL) {
    f[4] = fs[2 * N + row + gx];
    f[7] = fs[5 * N + row + gx];
    f[8] = fs[6 * N + row + gx];
  } else {
    f[4] = topin[gx];
    f[7] = topin[nx + gx];
    f[8] = topin[2 * nx + gx];
  }
}

// Inverse of pull: store pre-collision populations v of node (gx, y) into the
// post-collision layout so that the next pull returns them.
template <typename real>
__device__ __forceinline__ void scatter(real* __restrict__ fs, real* __restrict__ topin, int gx,
                                        int y, int nx, int ny, size_t N, int top_bc,
                                        const real v[9]) {
  const int xm = wrap1(gx - 1, nx), xp = wrap1(gx + 1, nx);
  const size_t row = (size_t)y * nx;
  fs[row + gx] = v[0];
  fs[N + row + xm] = v[1];
  fs[3 * N + row + xp] = v[3];
  if (y > 0) {
    const size_t rb = row - nx;
    fs[2 * N + rb + gx] = v[2];
    fs[5 * N + rb + xm] = v[5];
    fs[6 * N + rb + xp] = v[6];
  } else {
    fs[4 * N + row + gx] = v[2];
    fs[7 * N + row + gx] = v[5];
    fs[8 * N + row + gx] = v[6];
  }
  if (y < ny - 1) {
    const size_t ra = row + nx;
    fs[4 * N + ra + gx] = v[4];
    fs[7 * N + ra + xp] = v[7];
    fs[8 * N + ra + xm] = v[8];
  } else if (top_bc == TOP_WALL) {
    fs[2 * N + row + gx] = v[4];
    fs[5 * N + row + gx] = v[7];
    fs[6 * N + row + gx] = v[8];
  } else {
    topin[gx] = v[4];
    topin[nx + gx] = v[7];
    topin[2 * nx + gx] = v[8];
  }
}

// ---------------------------------------------------------------------------
// Eq. 7 with Eq. 28, in FP64: psi = sqrt(2 (p - rho/3) / G).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double eos_psi(const KParams& P, double r, double TE, unsigned& err) {
  double phi;
  if (P.flags & FREEZE_EOS_T) {
    phi = P.phi_sat;
  } else {
    double s = 1.0 + P.kappa * (1.0 - sqrt(TE * P.inv_Tc));
    phi = s * s;
  }
  const double br = P.b * r;
  const double d1 = 1.0 - br;
  const double d2 = 1.0 + 2.0 * br - br * br;
  // p = rho R T / d1 - a phi rho^2 / d2 over one common denominator
  const double p = (r * P.R * TE * d2 - P.a * phi * r * r * d1) / (d1 * d2);
  const double rad = 2.0 * (p - r * P.inv3) / P.G;
  if (!(r > 0.0)) err |= ERR_RHO;
  if (!(d1 > 0.0)) err |= ERR_COVOLUME;
  if (!(rad > 0.0)) {
    err |= (isfinite(rad) ? ERR_RADICAND : ERR_NONFINITE);
    return 0.0;
  }
  return sqrt(rad);
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
  const real ux = (jx + h * Fx) / rho;
  const real uy = (jy + h * Fy) / rho;
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
  const real snu = real(1) / (c.tau_v + c.dtau * w);
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

// Mass (and max speed) of the collide kernel, plus the open-top inflow of the next
// step, which is written here because it needs the whole row below the top.
template <typename real>
__device__ void finish_collide(const KParams& P, const double* __restrict__ partL,
                               const real* __restrict__ fpost, real* __restrict__ topin,
                               const real* __restrict__ uxa, const real* __restrict__ uya,
                               DevDiag* __restrict__ diag, bool apply_top, double* red) {
  const int t = threadIdx.x;
  double v[2] = {0.0, 0.0};
  for (int b = t; b < P.nblkL; b += NT) {
    v[0] += partL[2 * b];
    v[1] = fmax(v[1], partL[2 * b + 1]);
  }
  // max over the block through the same fixed tree (max is order-free anyway)
  double vm = wave_max(v[1]);
  double vs[2] = {v[0], 0.0};
  __syncthreads();
  if ((t & 63) == 0) red[8 + (t >> 6)] = vm;
  block_sum<2>(vs, red);
  double mass = vs[0];
  double vmax = fmax(fmax(red[8], red[9]), fmax(red[10], red[11]));
  __syncthreads();
  if (apply_top && P.top_bc != TOP_WALL) {
    const int nx = P.nx, ny = P.ny;
    const size_t N = (size_t)nx * ny;
    const size_t below = (size_t)(ny - 2) * nx, top = (size_t)(ny - 1) * nx;
    double U = 0.0;
    if (P.top_bc == TOP_CONVECTIVE) {
      double us[1] = {0.0};
      for (int x = t; x < nx; x += NT) us[0] += (double)uya[below + x];
      block_sum<1>(us, red);
      if (t == 0) red[12] = us[0];
      __syncthreads();
      U = red[12] / nx;
      if (U < 0.0) U = 0.0;
      __syncthreads();
    }
    double ms[1] = {0.0};
    for (int x = t; x < nx; x += NT) {
      real in4, in7, in8;
      if (P.top_bc == TOP_CONST_PRESSURE) {
        // equilibrium at rho_v with the velocity of the row below
        const real r = (real)P.rho_v, ux = uxa[below + x], uy = uya[below + x];
        const real usq = real(1.5) * (ux * ux + uy * uy);
        const real w1 = r / real(9), w2 = r / real(36);
        const real e4 = -uy, e7 = -ux - uy, e8 = ux - uy;
        in4 = w1 * (real(1) + real(3) * e4 + real(4.5) * e4 * e4 - usq);
        in7 = w2 * (real(1) + real(3) * e7 + real(4.5) * e7 * e7 - usq);
        in8 = w2 * (real(1) + real(3) * e8 + real(4.5) * e8 * e8 - usq);
      } else {
        // convective outlet: (f^n(top) + U f^{n+1}(top-1)) / (1 + U), where the new
        // populations of the row below are pulled from the top row's post-collision
        const real Ur = (real)U, inv = real(1) / (real(1) + Ur);
        const int xm = wrap1(x - 1, nx), xp = wrap1(x + 1, nx);
        in4 = (topin[x] + Ur * fpost[4 * N + top + x]) * inv;
        in7 = (topin[nx + x] + Ur * fpost[7 * N + top + xp]) * inv;
        in8 = (topin[2 * nx + x] + Ur * fpost[8 * N + top + xm]) * inv;
      }
      topin[x] = in4;
      topin[nx + x] = in7;
      topin[2 * nx + x] = in8;
      ms[0] += (double)in4 + (double)in7 + (double)in8;
    }
    block_sum<1>(ms, red);
    mass += ms[0];
  }
  if (t == 0) {
    diag->mass = mass;
    diag->rho_ave = mass / ((double)P.nx * (double)P.ny);
    diag->max_speed = sqrt(vmax);
    diag->L_pending = 0;
  }
}

// Energy, heat and Welford statistics of the energy kernel(s) of the last step.
__device__ void finish_energy(const KParams& P, const double* __restrict__ partE,
                              DevDiag* __restrict__ diag, double* red) {
  const int t = threadIdx.x;
  double v[5] = {0, 0, 0, 0, 0};
  for (int b = t; b < P.nblkE; b += NT)
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] += partE[5 * b + k];
  block_sum<5>(v, red);
  if (t == 0) {
    DevDiag& d = *diag;
    d.dE_cum += v[0];
    d.energy = v[1];
    d.Q_bottom_cum += v[2];
    d.Q_top_cum += v[3];
    d.Q_surface_cum += v[4];
    d.q_bottom = v[2] / P.nx;
    d.q_surface = v[4] / P.nx;
    d.nred += 1;
    const double cnt = (double)d.nred, q = d.q_bottom;
    const double dl = q - d.q_mean;
    d.q_mean += dl / cnt;
    d.q_m2 += dl * (q - d.q_mean);
    d.e_pending = 0;
  }
}

// ---------------------------------------------------------------------------
// Collide kernel: one LB step for a 64 x TY tile.
//   phase 1  pull f^n, rho = sum f (Eq. 5), psi (Eq. 7, 28) for the tile and a
//            one-cell ring, psi into LDS;
//   phase 2  forces (Eq. 6, 9, 10), velocity (Eq. 5), MRT collision (Eq. 2, 8);
//            write f*^n, rho, u; FP64 partial of the mass that the next pull sees.
// ---------------------------------------------------------------------------
template <typename real, int TY>
__global__ void __launch_bounds__(NT)
    k_collide(const KParams P, const real* __restrict__ fsrc, real* __restrict__ fdst,
              const real* __restrict__ topin, const real* __restrict__ Tcur,
              const real* __restrict__ gw, real* __restrict__ rho_out, real* __restrict__ ux_out,
              real* __restrict__ uy_out, double* __restrict__ partL,
              const double* __restrict__ partE, DevDiag* __restrict__ diag, long long step) {
  constexpr int RPT = TY / 4;  // rows per thread
  constexpr int LW = 66;
  __shared__ real spsi[TY + 2][LW];
  __shared__ double red[32];
  __shared__ double s_rho_ave;

  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int nx = P.nx, ny = P.ny;
  const size_t N = (size_t)nx * ny;

  __shared__ int s_pending;
  if (blockIdx.x == 0) {
    if (t == 0) s_pending = diag->e_pending;
    __syncthreads();
    if (s_pending) finish_energy(P, partE, diag, red);
  }
  if (t == 0) s_rho_ave = diag->rho_ave;

  const int tile = xcd_tile(blockIdx.x, P.nblkL);
  const int x0 = (tile % P.ntxL) * 64, y0 = (tile / P.ntxL) * TY;
  unsigned err = 0;

  real f[RPT][9];
  real rr[RPT];
  const int gxo = wrapm(x0 + lane, nx);
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int ly = wv + 4 * k, y = y0 + ly;
    real ps = real(0);
    if (y < ny) {
      pull(fsrc, topin, gxo, y, nx, ny, N, P.top_bc, f[k]);
      real r = f[k][0];
#pragma unroll
      for (int i = 1; i < 9; ++i) r += f[k][i];
      rr[k] = r;
      const double TE = (P.flags & FREEZE_EOS_T) ? P.T_sat : (double)Tcur[(size_t)(y + P.nh) * nx + gxo];
      if constexpr (sizeof(real) == 8) ps = eos_psi_plain(P, r, TE, err);
      else ps = (real)eos_psi(P, (double)r, TE, err);
    }
    spsi[ly + 1][lane + 1] = ps;
  }
  // ring of the tile: 66 + 66 + TY + TY cells
  for (int c = t; c < 2 * LW + 2 * TY; c += NT) {
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
      const double TE = (P.flags & FREEZE_EOS_T) ? P.T_sat : (double)Tcur[(size_t)(y + P.nh) * nx + gx];
      unsigned e2 = 0;
      if constexpr (sizeof(real) == 8) ps = eos_psi_plain(P, r, TE, e2);
      else ps = (real)eos_psi(P, (double)r, TE, e2);
    }
    spsi[ly + 1][lx + 1] = ps;
  }
  __syncthreads();

  CollideConst<real> cc;
  cc.s_e = (real)P.s_e; cc.s_z = (real)P.s_z; cc.s_q = (real)P.s_q;
  cc.c_e = (real)P.c_e; cc.c_z = (real)P.c_z; cc.c_q = (real)P.c_q;
  cc.sig_e = (real)P.sig_e; cc.sig_z = (real)P.sig_z;
  cc.rho_v = (real)P.rho_v; cc.inv_drho = (real)P.inv_drho;
  cc.tau_v = (real)P.tau_v; cc.dtau = (real)P.dtau;
  const real w1 = real(1) / real(3), w2 = real(1) / real(12);
  const real a1 = w1 / real(3), a2 = w2 / real(3);  // Eq. 10 weights
  const real negG = (real)(-P.G), gg = (real)P.g, rho_ave = (real)s_rho_ave;
  const bool open_top = P.top_bc != TOP_WALL;
  double mass = 0.0;
  real umax2 = real(0);

#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int ly = wv + 4 * k, y = y0 + ly;
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
      const real qsig = (fmx * fmx + fmy * fmy) / pc2;
      collide(f[k], r, Fx, Fy, qsig, cc, ux, uy);
    }
    const size_t n = (size_t)y * nx + gxo;
#pragma unroll
    for (int i = 0; i < 9; ++i) fdst[i * N + n] = f[k][i];
    rho_out[n] = r;
    ux_out[n] = ux;
    uy_out[n] = uy;
    double ms = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) ms += (double)f[k][i];
    if (y == ny - 1 && open_top) ms -= ((double)f[k][2] + (double)f[k][5]) + (double)f[k][6];
    mass += ms;
    const real u2 = ux * ux + uy * uy;
    umax2 = u2 > umax2 ? u2 : umax2;
    if (!isfinite(u2)) err |= ERR_NONFINITE;
  }
  if (err) flag_error(diag, err, step);
  double v[1] = {mass};
  double vm = wave_max((double)umax2);
  __syncthreads();
  if (lane == 0) red[8 + wv] = vm;
  block_sum<1>(v, red);
  if (t == 0) {
    partL[2 * blockIdx.x] = v[0];
    partL[2 * blockIdx.x + 1] = fmax(fmax(red[8], red[9]), fmax(red[10], red[11]));
    if (blockIdx.x == 0) diag->L_pending = 1;  // read only by the next kernel
  }
}

// ---------------------------------------------------------------------------
// Energy kernel: T^n -> T^{n+1} for a (W3-6) x (H3-6) tile of the temperature grid
// (heater and fluid rows), rho^n and u^n frozen (Eq. 17-18, Eq. 22-27).
// The tile, a four-cell halo and ghost rows sit in LDS; each of the four RK stages is
// evaluated on a region one cell smaller than the previous one, so all stages run
// with one read of T, rho, u and one write of T.  Thread t owns the cells t + 256k of
// the stage-1 region (W3 x H3) and keeps their coefficients in registers.
// ---------------------------------------------------------------------------
template <typename real, int W3, int H3, bool ISO>
__global__ void __launch_bounds__(NT)
    k_energy(const KParams P, const real* __restrict__ Tin, real* __restrict__ Tout,
             const real* __restrict__ rho, const real* __restrict__ uxa,
             const real* __restrict__ uya, double* __restrict__ partE,
             const real* __restrict__ fpost, real* __restrict__ topin,
             const double* __restrict__ partL, DevDiag* __restrict__ diag, int sub, double dtd,
             long long step) {
  constexpr int W4 = W3 + 2, H4 = H3 + 2, NC = W3 * H3 / NT;
  static_assert((W3 * H3) % NT == 0, "stage region must split evenly over the block");
  constexpr int TX = W3 - 6, TYE = H3 - 6;
  __shared__ real sA[H4][W4];
  __shared__ real sB[H4][W4];
  __shared__ real sFx[H4][W4];
  __shared__ real sFy[H4][W4];
  __shared__ real sUx[H4][W4];
  __shared__ real sUy[H4][W4];
  __shared__ double red[32];

  const int t = threadIdx.x;
  const int nx = P.nx, nT = P.nT, nh = P.nh;

  __shared__ int s_pending;
  if (blockIdx.x == 0 && sub == 0) {
    if (t == 0) s_pending = diag->L_pending;
    __syncthreads();
    if (s_pending) finish_collide(P, partL, fpost, topin, uxa, uya, diag, true, red);
  }

  const int tile = xcd_tile(blockIdx.x, P.nblkE);
  const int x0 = (tile % P.ntxE) * TX, j0 = (tile / P.ntxE) * TYE;
  const real cvk = (real)P.cvk;
  const bool top_open = P.top_bc != TOP_WALL;
  // lambda = rho c_v k (Sec. 3.1)
  auto lam_of = [&](real r) -> real {
    if constexpr (sizeof(real) == 8) return r * P.cv * P.k;
    else return r * cvk;
  };
  // Eq. 25 harmonic mean (dx = 1)
  auto face = [](real lp, real ln) -> real {
    if constexpr (sizeof(real) == 8) return 2.0 / (1.0 / lp + 1.0 / ln);
    else return real(2) * lp * ln / (lp + ln);
  };

  // ---- load T, lambda (into sB), u over the tile + 4 halo + ghost rows ----
  for (int c = t; c < W4 * H4; c += NT) {
    const int lr = c / W4, lc = c - lr * W4;
    const int j = j0 - 4 + lr;
    const int gx = wrapm(x0 - 4 + lc, nx);
    real T = real(0), lam = real(1), u = real(0), v = real(0);
    if (j >= 0 && j < nT) {
      T = Tin[(size_t)j * nx + gx];
      if (j < nh) {
        lam = (real)P.lambda_w;
      } else {
        const size_t n = (size_t)(j - nh) * nx + gx;
        lam = lam_of(rho[n]);
        u = uxa[n];
        v = uya[n];
      }
    } else if (j == -1) {
      lam = nh > 0 ? (real)P.lambda_w : lam_of(rho[gx]);
      if (P.bottom_tbc == TBC_FLUX) T = Tin[gx] + (real)P.q_bottom / lam;
      else T = (real)P.T_bottom;
    } else if (j == nT) {
      const size_t n = (size_t)(P.ny - 1) * nx + gx;
      lam = lam_of(rho[n]);
      if (P.top_tbc == TBC_DIRICHLET) T = (real)P.T_top;
      else T = Tin[(size_t)(nT - 1) * nx + gx];
      if (top_open) { u = uxa[n]; v = uya[n]; }
    }
    sA[lr][lc] = T;
    sB[lr][lc] = lam;
    sUx[lr][lc] = u;
    sUy[lr][lc] = v;
  }
  __syncthreads();

  // ---- face conductivities (Eq. 25); a ghost face takes the inner node's lambda ----
  for (int c = t; c < W4 * H4; c += NT) {
    const int lr = c / W4, lc = c - lr * W4;
    const int j = j0 - 4 + lr;
    const real lp = sB[lr][lc];
    real fx = real(0), fy = real(0);
    if (lc + 1 < W4) fx = face(lp, sB[lr][lc + 1]);
    if (lr + 1 < H4) {
      const real ln = sB[lr + 1][lc];
      if (j == -1) fy = ln;
      else if (j == nT - 1) fy = lp;
      else fy = face(lp, ln);
    }
    sFx[lr][lc] = fx;
    sFy[lr][lc] = fy;
  }

  // ---- per-cell coefficients of the cells this thread owns ----
  real T0[NC], Cc[NC], cux[NC], cuy[NC], cla[NC], clb[NC], acc[NC];
  real lamP[ISO ? NC : 1], glx[ISO ? NC : 1], gly[ISO ? NC : 1];
  real crho[sizeof(real) == 8 ? NC : 1], cdv[sizeof(real) == 8 ? NC : 1];  // plain-order latent term
  double rcv[NC];
  unsigned kind[NC];  // bit0 real node, bit1 fluid, bit2 bottom row, bit3 top row, bit4 surface row, bit5 output cell
  const real inv3 = real(1) / real(3), inv12 = real(1) / real(12);
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int cell = t + NT * k;
    const int rr = cell / W3, cc = cell - rr * W3;
    const int lr = rr + 1, lc = cc + 1;
    const int j = j0 - 3 + rr;
    const int xg = x0 - 3 + cc;
    unsigned kd = 0;
    T0[k] = sA[lr][lc];
    Cc[k] = real(0); cux[k] = real(0); cuy[k] = real(0); cla[k] = real(0); clb[k] = real(0);
    acc[k] = real(0);
    rcv[k] = 0.0;
    if constexpr (ISO) {
      // lambda and its Eq. 19 gradient for Eq. 21 (ghost rows copy the inner lambda)
      lamP[k] = sB[lr][lc];
      glx[k] = (sB[lr][lc + 1] - sB[lr][lc - 1]) * inv3 +
               ((sB[lr + 1][lc + 1] - sB[lr - 1][lc - 1]) + (sB[lr - 1][lc + 1] - sB[lr + 1][lc - 1])) * inv12;
      gly[k] = (sB[lr + 1][lc] - sB[lr - 1][lc]) * inv3 +
               ((sB[lr + 1][lc + 1] - sB[lr - 1][lc - 1]) + (sB[lr + 1][lc - 1] - sB[lr - 1][lc + 1])) * inv12;
    }
    if (j >= 0 && j < nT) {
      kd |= 1u;
      if (j == 0) kd |= 4u;
      if (j == nT - 1) kd |= 8u;
      if (nh > 0 && j == nh) kd |= 16u;
      if (rr >= 3 && rr < H3 - 3 && cc >= 3 && cc < W3 - 3 && xg < nx) kd |= 32u;
      if (j < nh) {
        rcv[k] = P.rcw;
        Cc[k] = (real)(1.0 / P.rcw);
      } else {
        kd |= 2u;
        const int gx = wrapm(xg, nx);
        const real r = rho[(size_t)(j - nh) * nx + gx];
        if constexpr (sizeof(real) == 8) crho[k] = r;
        rcv[k] = (double)r * P.cv;
        Cc[k] = real(1) / (r * (real)P.cv);
        cux[k] = sUx[lr][lc];
        cuy[k] = sUy[lr][lc];
        if (!(P.flags & NO_LATENT)) {
          // div u by Eq. 19 (u = 0 on solids, zero-gradient above an open top)
          real dudx, dvdy;
          if constexpr (sizeof(real) == 8) {
            dudx = (sUx[lr][lc + 1] - sUx[lr][lc - 1]) / 3.0 + (sUx[lr + 1][lc + 1] - sUx[lr - 1][lc - 1]) / 12.0 +
                   (sUx[lr - 1][lc + 1] - sUx[lr + 1][lc - 1]) / 12.0;
            dvdy = (sUy[lr + 1][lc] - sUy[lr - 1][lc]) / 3.0 + (sUy[lr + 1][lc + 1] - sUy[lr - 1][lc - 1]) / 12.0 +
                   (sUy[lr + 1][lc - 1] - sUy[lr - 1][lc + 1]) / 12.0;
          } else {
            dudx = (sUx[lr][lc + 1] - sUx[lr][lc - 1]) * inv3 + (sUx[lr + 1][lc + 1] - sUx[lr - 1][lc - 1]) * inv12 +
                   (sUx[lr - 1][lc + 1] - sUx[lr + 1][lc - 1]) * inv12;
            dvdy = (sUy[lr + 1][lc] - sUy[lr - 1][lc]) * inv3 + (sUy[lr + 1][lc + 1] - sUy[lr - 1][lc - 1]) * inv12 +
                   (sUy[lr + 1][lc - 1] - sUy[lr - 1][lc + 1]) * inv12;
          }
          const real divu = dudx + dvdy;
          cdv[k] = divu;
          // (dp/dT)_v = A(rho) - B(rho) phi'(T); A, B in FP64 (Eq. 28)
          const double rd = (double)r, br = P.b * rd;
          const double Ad = rd * P.R / (1.0 - br);
          const double Bd = P.a * rd * rd / (1.0 + 2.0 * br - br * br);
          const double cd = (double)Cc[k] * (double)divu;
          cla[k] = (real)(cd * Ad);
          clb[k] = (real)(cd * Bd * P.kappa);
        }
      }
    }
    kind[k] = kd;
  }
  __syncthreads();  // faces ready; sB is free for stage values

  const real dt = (real)dtd;
  const real kap = (real)P.kappa, onek = real(1) + (real)P.kappa, invTc = (real)P.inv_Tc;
  const real qb = (real)P.q_bottom;
  const bool flux_bottom = P.bottom_tbc == TBC_FLUX;
  double Qb = 0.0, Qt = 0.0, Qs = 0.0;
  const int fl = P.flags;

#pragma unroll
  for (int s = 0; s < 4; ++s) {
    real(*in)[W4] = (s & 1) ? sB : sA;
    real(*out)[W4] = (s & 1) ? sA : sB;
    const double wgt = (s == 0 || s == 3) ? 1.0 : 2.0;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int cell = t + NT * k;
      const int rr = cell / W3, cc = cell - rr * W3;
      if (!(kind[k] & 1u)) continue;
      if (rr < s || rr >= H3 - s || cc < s || cc >= W3 - s) continue;
      const int lr = rr + 1, lc = cc + 1;
      const real Tp = in[lr][lc];
      const real E = in[lr][lc + 1], W = in[lr][lc - 1], Nn = in[lr + 1][lc], S = in[lr - 1][lc];
      const real fe = sFx[lr][lc], fw = sFx[lr][lc - 1], fn = sFy[lr][lc], fs = sFy[lr - 1][lc];
      real qs;
      if ((kind[k] & 4u) && flux_bottom) qs = qb;
      else qs = fs * (S - Tp);
      const real qn = fn * (Nn - Tp);
      const real NE = in[lr + 1][lc + 1], NW = in[lr + 1][lc - 1];
      const real SE = in[lr - 1][lc + 1], SW = in[lr - 1][lc - 1];
      real gx = real(0), gy = real(0);
      if (ISO || !(fl & NO_ADVECTION)) {
        // Eq. 19 isotropic gradient
        if constexpr (sizeof(real) == 8) {
          gx = (E - W) / 3.0 + (NE - SW) / 12.0 + (SE - NW) / 12.0;
          gy = (Nn - S) / 3.0 + (NE - SW) / 12.0 + (NW - SE) / 12.0;
        } else {
          gx = (E - W) * inv3 + ((NE - SW) + (SE - NW)) * inv12;
          gy = (Nn - S) * inv3 + ((NE - SW) + (NW - SE)) * inv12;
        }
      }
      real D;
      if constexpr (!ISO) {
        // Eq. 22-26: heat through the four faces of the control volume (dx = 1)
        D = ((fe * (E - Tp) + fw * (W - Tp)) + qn) + qs;
      } else {
        // Eq. 21 with Eq. 20: lambda Lap T + grad lambda . grad T (comparison scheme)
        const real lap =
            (((((((((NE + NW) + SE) + SW) + real(4) * E) + real(4) * W) + real(4) * Nn) + real(4) * S) -
              real(20) * Tp)) /
            real(6);
        D = lamP[k] * lap + (glx[k] * gx + gly[k] * gy);
      }
      real h;
      if constexpr (sizeof(real) == 8) h = D / (real)rcv[k];
      else h = Cc[k] * D;
      if (kind[k] & 2u) {
        if (!(fl & NO_ADVECTION)) h += -(cux[k] * gx + cuy[k] * gy);
        if (!(fl & NO_LATENT)) {
          if constexpr (sizeof(real) == 8) {
            // -(T/(rho c_v)) (dp/dT)_v div u, Eq. 17 with Eq. 28, in plain order
            const double r = crho[k], b = P.b;
            const double s1 = 1.0 + P.kappa * (1.0 - sqrt(Tp / P.Tc));
            const double dphi = -P.kappa * s1 / sqrt(Tp * P.Tc);
            const double dpdT = r * P.R / (1.0 - b * r) - P.a * dphi * r * r / (1.0 + 2.0 * b * r - b * b * r * r);
            h += -(Tp / (real)rcv[k]) * dpdT * cdv[k];
          } else {
            // -(T/(rho c_v)) (dp/dT)_v div u with T phi'(T) = -kappa s (1 + kappa - kappa s)
            const real sg = sqrt(Tp * invTc);
            h += -(cla[k] * Tp + clb[k] * sg * (onek - kap * sg));
          }
        }
      }
      if (kind[k] & 32u) {
        const double w = wgt;
        if (kind[k] & 4u) Qb += w * (double)qs;
        if ((kind[k] & 8u) && P.top_tbc == TBC_DIRICHLET) Qt += w * (double)qn;
        if (kind[k] & 16u) Qs += w * (double)qs;
      }
      if (s < 3) {
        const real cs = (s == 2) ? dt : real(0.5) * dt;
        const real Yn = T0[k] + cs * h;
        out[lr][lc] = Yn;
        acc[k] = (s == 0) ? h : acc[k] + real(2) * h;
        // ghost rows follow the stage value of the row next to them
        if ((kind[k] & 4u) && flux_bottom) out[lr - 1][lc] = Yn + qb / sFy[lr - 1][lc];
        if ((kind[k] & 8u) && P.top_tbc != TBC_DIRICHLET) out[lr + 1][lc] = Yn;
        if ((kind[k] & 4u) && !flux_bottom) out[lr - 1][lc] = (real)P.T_bottom;
        if ((kind[k] & 8u) && P.top_tbc == TBC_DIRICHLET) out[lr + 1][lc] = (real)P.T_top;
      } else {
        acc[k] = T0[k] + (dt / real(6)) * (acc[k] + h);
      }
    }
    __syncthreads();
  }

  // ---- write T^{n+1}, FP64 partials ----
  unsigned err = 0;
  double v[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    if (!(kind[k] & 32u)) continue;
    const int cell = t + NT * k;
    const int rr = cell / W3, cc = cell - rr * W3;
    const int j = j0 - 3 + rr, gx = x0 - 3 + cc;
    const real Tn = acc[k];
    if (!isfinite(Tn)) err |= ERR_NONFINITE;
    Tout[(size_t)j * nx + gx] = Tn;
    v[0] += rcv[k] * ((double)Tn - (double)T0[k]);
    v[1] += rcv[k] * (double)Tn;
  }
  if (err) flag_error(diag, err, step);
  const double d6 = dtd / 6.0;
  v[2] = Qb * d6;
  v[3] = Qt * d6;
  v[4] = Qs * d6;
  if (nh == 0) v[4] = v[2];
  block_sum<5>(v, red);
  if (t == 0) {
    double* pe = partE + 5 * blockIdx.x;
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
    if (blockIdx.x == 0) diag->e_pending = 1;  // read only by the next kernel
  }
}

// ---------------------------------------------------------------------------
// Initialisation / field access kernels (same 64 x TY tiling as k_collide).
// ---------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(NT)
    k_scatter(const KParams P, const real* __restrict__ src, int src_is_rho, real* __restrict__ fdst,
              real* __restrict__ topin, double* __restrict__ partL, DevDiag* __restrict__ diag) {
  __shared__ double red[32];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
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
  block_sum<1>(vv, red);
  if (t == 0) {
    partL[2 * blockIdx.x] = vv[0];
    partL[2 * blockIdx.x + 1] = 0.0;
    if (blockIdx.x == 0) diag->L_pending = 1;
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

template <typename real>
__global__ void __launch_bounds__(NT)
    k_finish(const KParams P, const double* __restrict__ partL, const double* __restrict__ partE,
             const real* __restrict__ fpost, real* __restrict__ topin, const real* __restrict__ uxa,
             const real* __restrict__ uya, DevDiag* __restrict__ diag) {
  __shared__ double red[32];
  __shared__ int s_pl, s_pe;
  if (threadIdx.x == 0) {
    s_pl = diag->L_pending;
    s_pe = diag->e_pending;
  }
  __syncthreads();
  if (s_pl) finish_collide(P, partL, fpost, topin, uxa, uya, diag, false, red);
  __syncthreads();
  if (s_pe) finish_energy(P, partE, diag, red);
}

template <typename real>
__global__ void k_convert_in(const double* __restrict__ src, real* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT)
    dst[i] = (real)src[i];
}

}  // namespace lbmk
