// lbm_energy_f32.hpp -- FP32 temperature update with register-resident rows.
//
// Same tile, four-cell halo and fused RK4 stages as k_energy (Eq. 17-18, Eq. 19,
// Eq. 22-27), arranged for the vector ALU instead of LDS.  Each wave owns a band of B
// consecutive tile rows and keeps them in registers, lane = tile column.  West and east
// neighbours come from whole-wavefront DPP lane shifts, north and south neighbours from
// the neighbouring register row.  Only the two edge rows of each band pass through LDS,
// once per stage.  At set-up the right-hand side of Eq. 17 at a cell is folded into one
// nine-point stencil with eight coefficients, since everything but the latent term is
// linear in T with rho and u frozen:
//   h = cP T + cE E + cW W + cN N + cS S + aP (NE - SW) + aM (SE - NW) - l2 sqrt(T)
// Diffusion (Eq. 22-26) gives g_f = lambda_f / (rho c_v) per face f; advection with the
// Eq. 19 gradient gives aX = -u_x/3, aY = -u_y/3, aP = -(u_x + u_y)/12,
// aM = -(u_x - u_y)/12; the latent term -(T/(rho c_v)) (dp/dT)_v div u of Eq. 17 with
// Eq. 28, using T phi'(T) = -kappa s (1 + kappa - kappa s) and s = sqrt(T/T_c), is
// -l1 T - l2 sqrt(T) with l1 = C div(u) (A - B kappa^2/T_c) and
// l2 = C div(u) B kappa (1 + kappa)/sqrt(T_c), where C = 1/(rho c_v), A = rho R/(1 - b rho)
// and B = a rho^2/(1 + 2 b rho - b^2 rho^2).  Hence cE = g_E + aX, cW = g_W - aX,
// cN = g_N + aY, cS = g_S - aY and cP = -(g_E + g_W + g_N + g_S) - l1.
#pragma once
#include "lbm_kernels.hpp"

namespace lbmk {

// Value held by lane + 1 (east) / lane - 1 (west) of the wavefront: DPP wave_shl:1 and
// wave_shr:1.  The end lanes read 0; they are halo lanes whose results are never used.
__device__ __forceinline__ float lane_east(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_west(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}

// Tile: txE (<= 56) columns by tyE rows of the temperature grid, with tyE + 8 <= NW * B.
// Lane c holds global column x0 - 4 + c (periodic); tile row r holds T row j0 - 4 + r;
// wave w owns tile rows [w B, w B + B).  Stage s is valid on tile rows [1 + s, tyE + 7 - s)
// and lanes [1 + s, 63 - s); cells outside that cone are computed or left as they are
// and never reach a written cell.
template <int NW, int B>
struct RowsShared {
  float edge[2][NW][2][64];  // [stage parity][wave][bottom/top row][lane]
  float rcv[NW][B][64];      // rho c_v of the band rows (energy partials)
  double red[RED_SIZE];
};

// The tile work.  PLAIN: every row of the tile (halo included) is a fluid row away from
// both boundaries, so no row needs boundary handling and none is skipped, and advection
// and the latent term are both on.  COH: rho and u come from collide tiles of the same
// launch (the fused step) and are loaded coherently.
template <int NW, int B, bool PLAIN, bool COH>
__device__ __forceinline__ void energy_rows_tile(
    const KParams& P, RowsShared<NW, B>& sh, const float* __restrict__ Tin, float* __restrict__ Tout,
    const float* __restrict__ rho, const float* __restrict__ uxa, const float* __restrict__ uya,
    double* __restrict__ hist_slot, DevDiag* __restrict__ diag, int sub, double dtd,
    const long long* __restrict__ dstep_prev, int tile, int x0, int j0, int TY) {
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int nx = P.nx, nT = P.nT, nh = P.nh;
  const int TX = P.txE, H4 = TY + 8;
  const int gx = wrapm(x0 - 4 + lane, nx);
  const int r0 = w * B;          // first tile row of this wave's band
  const int jb = j0 - 4 + r0;    // its temperature row
  const bool wave_live = r0 < H4;
  const bool top_open = P.top_bc != TOP_WALL;
  const bool do_adv = !(P.flags & NO_ADVECTION), do_lat = !(P.flags & NO_LATENT);
  const bool flux_bottom = P.bottom_tbc == TBC_FLUX, top_dirichlet = P.top_tbc == TBC_DIRICHLET;
  const float cvk = (float)P.cvk, cv = (float)P.cv, lamw = (float)P.lambda_w;
  const float inv3 = 1.f / 3.f, inv12 = 1.f / 12.f;

  // ---- load temperature rows jb - 1 .. jb + B with rho and u (u = 0 on solids, and
  // zero-gradient above an open top) ----
  float lT[B + 2], lR[B + 2], lU[B + 2], lV[B + 2];
  if constexpr (PLAIN) {
    // rows outside the tile are clamped into the fluid rows; their values are unused.  A
    // wave whose band lies wholly beyond the tile loads nothing.
    if (wave_live) {
#pragma unroll
      for (int q = 0; q < B + 2; ++q) {
        const int j = min(max(jb - 1 + q, nh), nT - 1);
        lT[q] = ld32(Tin, (unsigned)j * (unsigned)nx + gx);
        const unsigned n = (unsigned)(j - nh) * (unsigned)nx + gx;
        if constexpr (COH) {
          lR[q] = ldc<true>(rho + n);
          lU[q] = ldc<true>(uxa + n);
          lV[q] = ldc<true>(uya + n);
        } else {
          lR[q] = ld32(rho, n);
          lU[q] = ld32(uxa, n);
          lV[q] = ld32(uya, n);
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < B + 2; ++q) {
        lT[q] = 0.f; lR[q] = 1.f; lU[q] = 0.f; lV[q] = 0.f;
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < B + 2; ++q) {
      const int j = jb - 1 + q;
      // rows that are not loaded keep finite values: they are computed with the others,
      // and their results reach only halo or ghost rows
      lT[q] = 0.f; lR[q] = 1.f; lU[q] = 0.f; lV[q] = 0.f;
      if (r0 - 1 + q >= H4) continue;
      if (j >= 0 && j < nT) {
        lT[q] = Tin[(size_t)j * nx + gx];
        if (j >= nh) {
          const size_t n = (size_t)(j - nh) * nx + gx;
          lR[q] = ldc<COH>(rho + n);
          lU[q] = ldc<COH>(uxa + n);
          lV[q] = ldc<COH>(uya + n);
        }
      } else if (j == nT && top_open) {
        const size_t n = (size_t)(P.ny - 1) * nx + gx;
        lU[q] = ldc<COH>(uxa + n);
        lV[q] = ldc<COH>(uya + n);
      }
    }
  }

  // ---- per-cell coefficients of the band rows ----
  float uxE[B + 2], uxW[B + 2], uyE[B + 2], uyW[B + 2];
#pragma unroll
  for (int q = 0; q < B + 2; ++q) {
    uxE[q] = lane_east(lU[q]);
    uxW[q] = lane_west(lU[q]);
    uyE[q] = lane_east(lV[q]);
    uyW[q] = lane_west(lV[q]);
  }
  float Y[B], T0[B], acc[B];
  float cP[B], cE[B], cW[B], cN[B], cS[B], aP[B], aM[B], l2[B];
  float gq = 0.f, fq0 = 0.f, fqt = 0.f, fqh = 0.f;
  // div u at band row k by Eq. 19
  auto divu = [&](int q) {
    const float dudx = (uxE[q] - uxW[q]) * inv3 + ((uxE[q + 1] - uxW[q - 1]) + (uxE[q - 1] - uxW[q + 1])) * inv12;
    const float dvdy = (lV[q + 1] - lV[q - 1]) * inv3 + ((uyE[q + 1] - uyW[q - 1]) + (uyW[q + 1] - uyE[q - 1])) * inv12;
    return dudx + dvdy;
  };
  if constexpr (PLAIN) {
    // All fluid: with lambda = rho c_v k, a face coefficient lambda_f / (rho_P c_v) of
    // Eq. 25 is 2 k rho_nb / (rho_P + rho_nb); the latent factors A/(rho c_v) and
    // B/(rho c_v) share the denominator (1 - b rho)(1 + 2 b rho - b^2 rho^2).
    const float k2 = P.e_k2, g1a = P.e_g1a, g1b = P.e_g1b, g2a = P.e_g2a;
    const float bb = (float)P.b;
    float rN[B + 1];  // 1 / (rho_q + rho_{q+1})
#pragma unroll
    for (int q = 0; q < B + 1; ++q) rN[q] = __builtin_amdgcn_rcpf(lR[q] + lR[q + 1]);
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int q = k + 1;
      const float r = lR[q];
      sh.rcv[w][k][lane] = r * cv;
      const float rE = lane_east(r), rWv = lane_west(r);
      const float iE = __builtin_amdgcn_rcpf(r + rE);
      const float ge = k2 * rE * iE, gw = k2 * rWv * lane_west(iE);
      const float gn = k2 * lR[q + 1] * rN[q], gs = k2 * lR[q - 1] * rN[q - 1];
      // advection and latent heat are both on in plain tiles
      const float ux = lU[q], uy = lV[q];
      const float ax = -ux * inv3, ay = -uy * inv3;
      aP[k] = -(ux + uy) * inv12;
      aM[k] = -(ux - uy) * inv12;
      const float br = bb * r, d1 = 1.f - br, d2 = 1.f + 2.f * br - br * br;
      const float dv = divu(q) * __builtin_amdgcn_rcpf(d1 * d2);
      const float l1 = dv * (g1a * d2 - g1b * r * d1);
      l2[k] = dv * (g2a * r * d1);
      cE[k] = ge + ax;
      cW[k] = gw - ax;
      cN[k] = gn + ay;
      cS[k] = gs - ay;
      cP[k] = -(((ge + gw) + gn) + gs) - l1;
      Y[k] = lT[q];
      T0[k] = lT[q];
      acc[k] = 0.f;
    }
  } else {
    // conductivities and faces (Eq. 25); a face to a ghost row takes the inner lambda
    float lam[B + 2];
#pragma unroll
    for (int q = 0; q < B + 2; ++q) {
      const int j = jb - 1 + q;
      lam[q] = (j >= nh && j < nT) ? lR[q] * cvk : ((j >= 0 && j < nh) ? lamw : 1.f);
    }
    float fN[B + 1];  // face between loaded rows q and q + 1
#pragma unroll
    for (int q = 0; q < B + 1; ++q) {
      const int j = jb - 1 + q;
      const float a = lam[q], b = lam[q + 1];
      const float hm = 2.f * a * b * __builtin_amdgcn_rcpf(a + b);
      fN[q] = (j == -1) ? b : ((j == nT - 1) ? a : hm);
    }
    // faces and ghost offsets that the boundary rows need (heat-flux diagnostics)
#pragma unroll
    for (int q = 0; q < B + 2; ++q) {
      const int j = jb - 1 + q;
      if (j == 0) {
        fq0 = lam[q];
        gq = (float)P.q_bottom * __builtin_amdgcn_rcpf(lam[q]);
      }
      if (j == nT - 1) fqt = lam[q];
      if (q > 0 && j == nh && nh > 0) fqh = fN[q - 1];
    }
    const float kk2 = P.e_kk2, kl2 = P.e_kl2;
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int q = k + 1, j = jb + k;
      const bool fluid = j >= nh && j < nT;
      const float r = lR[q];
      float C, rc;
      if (fluid) {
        rc = r * cv;
        C = __builtin_amdgcn_rcpf(rc);
      } else {
        rc = (float)P.rcw;
        C = (float)P.inv_rcw;
      }
      sh.rcv[w][k][lane] = rc;
      const float lE = lane_east(lam[q]);
      const float fe = 2.f * lam[q] * lE * __builtin_amdgcn_rcpf(lam[q] + lE);
      const float ge = C * fe, gw = C * lane_west(fe), gn = C * fN[q], gs = C * fN[q - 1];
      float ax = 0.f, ay = 0.f, l1 = 0.f;
      aP[k] = 0.f; aM[k] = 0.f; l2[k] = 0.f;
      if (fluid) {
        const float ux = lU[q], uy = lV[q];
        if (do_adv) {
          ax = -ux * inv3;
          ay = -uy * inv3;
          aP[k] = -(ux + uy) * inv12;
          aM[k] = -(ux - uy) * inv12;
        }
        if (do_lat) {
          const float br = (float)P.b * r;
          const float Ad = r * (float)P.R * __builtin_amdgcn_rcpf(1.f - br);
          const float Bd = (float)P.a * r * r * __builtin_amdgcn_rcpf(1.f + 2.f * br - br * br);
          const float cd = C * divu(q);
          l1 = cd * (Ad - Bd * kk2);
          l2[k] = cd * Bd * kl2;
        }
      }
      cE[k] = ge + ax;
      cW[k] = gw - ax;
      cN[k] = gn + ay;
      cS[k] = gs - ay;
      cP[k] = -(((ge + gw) + gn) + gs) - l1;
      Y[k] = lT[q];
      T0[k] = lT[q];
      acc[k] = 0.f;
    }
  }

  // ---- four RK stages (Eq. 18) ----
  const float dt = (float)dtd, Tbot = (float)P.T_bottom, Ttop = (float)P.T_top, qb = (float)P.q_bottom;
  const float dt2 = 0.5f * dt, dt6 = (float)(dtd / 6.0);
  const bool lane_out = lane >= 4 && lane < 4 + TX && x0 + lane - 4 < nx;
  float eS = lT[0], eN = lT[B + 1];  // rows below and above the band
  double Qb = 0.0, Qt = 0.0, Qs = 0.0;
  // band rows that carry a boundary-flux diagnostic (-1: none in this wave): the bottom
  // row, the top row under a Dirichlet top, the first fluid row above the heater
  auto pick = [&](int j) {
    const int k = j - jb, r = r0 + k;
    return (k >= 0 && k < B && r >= 4 && r < 4 + TY) ? k : -1;
  };
  const int kB = PLAIN ? -1 : pick(0);
  const int kT = (PLAIN || !top_dirichlet) ? -1 : pick(nT - 1);
  const int kS = (PLAIN || nh == 0) ? -1 : pick(nh);
  // band rows of the ghost rows below the bottom and above the top (-1: none)
  const int kGb = (!PLAIN && jb <= -1 && -1 < jb + B) ? -1 - jb : -1;
  const int kGt = (!PLAIN && jb <= nT && nT < jb + B) ? nT - jb : -1;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if constexpr (!PLAIN) {
      // ghost rows take their stage value from the row next to them (only the waves
      // whose band holds a ghost row)
      if (kGb >= 0 || kGt >= 0) {
#pragma unroll
        for (int k = 0; k < B; ++k) {
          if (k == kGb) Y[k] = flux_bottom ? ((k + 1 < B ? Y[k + 1] : eN) + gq) : Tbot;
          if (k == kGt) Y[k] = top_dirichlet ? Ttop : (k > 0 ? Y[k - 1] : eS);
        }
      }
      if (jb == 0) eS = flux_bottom ? Y[0] + gq : Tbot;
      if (jb + B == nT) eN = top_dirichlet ? Ttop : Y[B - 1];
    }
    const float wgt = (s == 0 || s == 3) ? 1.f : 2.f;
    float qB = 0.f, qT = 0.f, qS = 0.f;
    if (wave_live) {
      float s0 = eS, sE = lane_east(eS), sW = lane_west(eS);
      float c0 = Y[0], wE = lane_east(c0), wW = lane_west(c0);
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const float n0 = (k + 1 < B) ? Y[k + 1] : eN;
        const float nE = lane_east(n0), nW = lane_west(n0);
        {
          const float Tp = c0;
          float h = cP[k] * Tp + cE[k] * wE + cW[k] * wW + cN[k] * n0 + cS[k] * s0;
          h += aP[k] * (nE - sW) + aM[k] * (sE - nW);
          h -= l2[k] * __builtin_amdgcn_sqrtf(Tp);
          if constexpr (!PLAIN) {
            if (k == kB) qB = flux_bottom ? qb : fq0 * (s0 - Tp);
            if (k == kT) qT = fqt * (n0 - Tp);
            if (k == kS) qS = fqh * (s0 - Tp);
          }
          if (s == 0) {
            Y[k] = T0[k] + dt2 * h;
            acc[k] = h;
          } else if (s < 3) {
            Y[k] = T0[k] + ((s == 2) ? dt : dt2) * h;
            acc[k] = acc[k] + 2.f * h;
          } else {
            Y[k] = T0[k] + dt6 * (acc[k] + h);
          }
        }
        s0 = c0; sE = wE; sW = wW;
        c0 = n0; wE = nE; wW = nW;
      }
      if constexpr (!PLAIN) {
        if (kB >= 0) Qb += (double)(lane_out ? wgt * qB : 0.f);
        if (kT >= 0) Qt += (double)(lane_out ? wgt * qT : 0.f);
        if (kS >= 0) Qs += (double)(lane_out ? wgt * qS : 0.f);
      }
    }
    if (s < 3) {
      sh.edge[s & 1][w][0][lane] = Y[0];
      sh.edge[s & 1][w][1][lane] = Y[B - 1];
      __syncthreads();
      eS = w > 0 ? sh.edge[s & 1][w - 1][1][lane] : Y[0];
      eN = w < NW - 1 ? sh.edge[s & 1][w + 1][0][lane] : Y[B - 1];
    }
  }

  // ---- write T^{n+1}, FP64 partials ----
  unsigned err = 0;
  double v[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < B; ++k) {
    const int r = r0 + k, j = jb + k;
    if (r < 4 || r >= 4 + TY || j >= nT || !lane_out) continue;
    const float Tn = Y[k];
    if (!isfinite(Tn)) err |= ERR_NONFINITE;
    st32(Tout, (unsigned)j * (unsigned)nx + gx, Tn);
    const double rc = (double)sh.rcv[w][k][lane];
    v[0] += rc * ((double)Tn - (double)T0[k]);
    v[1] += rc * (double)Tn;
  }
  if (err) flag_error(diag, err, dstep_prev[0]);
  const double d6 = dtd / 6.0;
  v[2] = Qb * d6;
  v[3] = Qt * d6;
  v[4] = Qs * d6;
  if (nh == 0) v[4] = v[2];
  // interior tiles carry no boundary flux: their partials 2..4 are zero
  constexpr int KV = PLAIN ? 2 : 5;
#pragma unroll
  for (int k = 0; k < KV; ++k) v[k] = wave_sum_dpp(v[k]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < KV; ++k) sh.red[w * KV + k] = v[k];
  __syncthreads();
  // lane k of wave 0 sums partial k over the waves in order and stores it
  if (w == 0 && lane < 5) {
    double a = 0.0;
    if (lane < KV) {
      a = sh.red[lane];
      for (int q = 1; q < NW; ++q) a += sh.red[q * KV + lane];
    }
    double* pe = hist_slot + 5 * tile;
    if (sub == 0) pe[lane] = a;
    else if (lane == 1) pe[1] = a;
    else pe[lane] += a;
  }
}

template <int NW, int B, bool COH = false>
__device__ __forceinline__ void energy_rows_step(
    const KParams& P, const float* __restrict__ Tin, float* __restrict__ Tout,
    const float* __restrict__ rho, const float* __restrict__ uxa, const float* __restrict__ uya,
    double* __restrict__ hist_slot, DevDiag* __restrict__ diag, int sub, double dtd,
    const long long* __restrict__ dstep_prev, int tile) {
  __shared__ RowsShared<NW, B> sh;
  const int nT = P.nT;
  int j0, TY;
  energy_tile_rows(P, tile, j0, TY);
  const int x0 = (tile % P.ntxE) * P.txE;
  const bool plain_tile = (j0 - 4 >= P.nh) && (j0 + TY + 3 <= nT - 1) &&
                          !(P.flags & (NO_ADVECTION | NO_LATENT));
  if (plain_tile)
    energy_rows_tile<NW, B, true, COH>(P, sh, Tin, Tout, rho, uxa, uya, hist_slot, diag, sub, dtd, dstep_prev,
                                       tile, x0, j0, TY);
  else
    energy_rows_tile<NW, B, false, COH>(P, sh, Tin, Tout, rho, uxa, uya, hist_slot, diag, sub, dtd,
                                        dstep_prev, tile, x0, j0, TY);
}

template <int NW, int B, int WPE>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE)))
    k_energy_rows(const KParams P, const float* __restrict__ Tin, float* __restrict__ Tout,
                  const float* __restrict__ rho, const float* __restrict__ uxa,
                  const float* __restrict__ uya, double* __restrict__ hist_slot,
                  const float* __restrict__ fpost, float* __restrict__ topin,
                  const double* __restrict__ partL_cur, double* __restrict__ pmin_cur,
                  DevDiag* __restrict__ diag, int sub, double dtd,
                  const long long* __restrict__ dstep_prev) {
  // block 0: the open-top rule; blocks 1..nblkE: the tiles
  if (blockIdx.x == 0) {
    if (sub == 0) outlet_block<float, NW>(P, fpost, topin, uxa, uya, partL_cur, pmin_cur);
    return;
  }
  energy_rows_step<NW, B>(P, Tin, Tout, rho, uxa, uya, hist_slot, diag, sub, dtd, dstep_prev,
                          xcd_tile_edges_first(blockIdx.x - 1, P.nblkE));
}

// ---------------------------------------------------------------------------
// Fused FP32 step (one energy sub-step): one launch per LB step.  Block b takes item
// order[b] of a host-built order: first the collide items (item c runs collide tiles 2c
// and 2c + 1, one per half of the workgroup), then the open-top block (item npair),
// then the energy tiles (item npair + 1 + e), bottom-up.  A collide tile, once its
// outputs are stored, records the step it completed in cdone[tile]; the outlet block and
// each energy tile first wait until the collide tiles whose rows and columns they read
// have completed this step, so an energy tile starts as soon as its own neighbourhood is
// done, on the slot of a finished collide tile, without the launch boundary in between.
// Collide tiles wait for nothing and precede every waiting block, so with in-order
// dispatch every wait ends; a wait beyond its spin bound flags ERR_SYNC instead of
// hanging.  What is produced and consumed inside the launch (rho, u, the top row's
// populations, the collide partials) moves by agent-coherent loads and stores;
// everything else crosses a kernel boundary.
// ---------------------------------------------------------------------------
constexpr int SPIN_MAX = 1 << 20;  // polls (each with a short sleep) before ERR_SYNC

// Lane l (< 64, lane_on) of wave 0 waits until cdone of the collide tile in column
// cx and each tile row ry0..ry1 has reached `want`; then the whole block synchronises.
__device__ __forceinline__ void wait_collide_rows(const KParams& P, const unsigned* __restrict__ cdone,
                                                  unsigned want, int ry0, int ry1, int cx, bool lane_on,
                                                  DevDiag* __restrict__ diag, long long step) {
  if (threadIdx.x < 64 && lane_on) {
    for (int ry = ry0; ry <= ry1; ++ry) {
      const unsigned* f = cdone + (size_t)ry * P.ntxL + cx;
      int spins = 0;
      while ((int)(ldc<true>(f) - want) < 0) {
        if (++spins > SPIN_MAX) {
          flag_error(diag, ERR_SYNC, step);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
  }
  __syncthreads();
}

template <int TYC, int NWC, int NW, int B, int WPE>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE)))
    k_step_fused(const KParams P, const float* __restrict__ fsrc, float* __restrict__ fdst,
                 float* __restrict__ topin, const float* __restrict__ Tin, float* __restrict__ Tout,
                 const float* __restrict__ gw, float* __restrict__ rho, float* __restrict__ uxa,
                 float* __restrict__ uya, const double* __restrict__ mstate_prev,
                 const double* __restrict__ pmin_prev, double* __restrict__ mstate_cur,
                 double* __restrict__ partL_cur, double* __restrict__ pmin_cur, DevDiag* __restrict__ diag,
                 const long long* __restrict__ dstep_prev, long long* __restrict__ dstep_cur,
                 double* __restrict__ hist_slot, unsigned* __restrict__ cdone,
                 const int* __restrict__ order, double dtd) {
  constexpr int HALVES = NW / NWC;  // collide tiles per workgroup
  static_assert(HALVES * NWC == NW && (HALVES == 1 || HALVES == 2), "collide tiles per energy-sized workgroup");
  const int b = __builtin_amdgcn_readfirstlane(order[blockIdx.x]);
  const int npair = (P.nblkL + HALVES - 1) / HALVES;
  const long long step = dstep_prev[0];  // index of this step (collide tile 0 writes the other slot)
  const unsigned want = (unsigned)(step + 1);
  if (b < npair) {
    const int half = HALVES > 1 ? __builtin_amdgcn_readfirstlane((int)threadIdx.x / (NWC * 64)) : 0;
    const int tile = HALVES * b + half;  // == nblkL: an empty half
    collide_tile<float, TYC, NWC, true, HALVES>(P, fsrc, fdst, topin, Tin, gw, rho, uxa, uya, mstate_prev,
                                           pmin_prev, mstate_cur, partL_cur, diag, dstep_prev, dstep_cur, tile);
    // every wave's stores complete before a tile is marked done
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if ((threadIdx.x % (NWC * 64)) == 0 && tile < P.nblkL) stc<true>(cdone + tile, want);
    return;
  }
  const int lane = threadIdx.x & 63;
  if (b == npair) {
    // the open-top rule reads the top row's populations, u of the row below and the
    // partials of that row's tiles: all collide tiles of the last two fluid rows
    if (P.top_bc != TOP_WALL) {
      const int ry0 = max(P.ny - 2, 0) / TYC, ry1 = (P.ny - 1) / TYC;
      for (int c0 = 0; c0 < P.ntxL; c0 += 64)
        wait_collide_rows(P, cdone, want, ry0, ry1, c0 + lane, c0 + lane < P.ntxL, diag, step);
    }
    outlet_block<float, NW, true>(P, fdst, topin, uxa, uya, partL_cur, pmin_cur);
    return;
  }
  const int tile = b - npair - 1;
  int j0, TY;
  energy_tile_rows(P, tile, j0, TY);
  const int x0 = (tile % P.ntxE) * P.txE;
  // fluid rows whose rho and u the tile may read (its T rows with the four-row halo and
  // one more each way), in the tile columns of the lanes' global columns
  const int ylo = max(j0 - 5 - P.nh, 0), yhi = min(j0 + TY + 4 - P.nh, P.ny - 1);
  if (yhi >= ylo)
    wait_collide_rows(P, cdone, want, ylo / TYC, yhi / TYC, wrapm(x0 - 4 + lane, P.nx) / 64, true, diag, step);
  energy_rows_step<NW, B, true>(P, Tin, Tout, rho, uxa, uya, hist_slot, diag, 0, dtd, dstep_prev, tile);
}

}  // namespace lbmk
