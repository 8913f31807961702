// fr_kernels.hip -- gfx950 kernels of the FR residual and RK stage (FP64 operator path), and
// the C ABI of libfr.
//
// One RK stage is three kernels (section "FR Algorithm", Eq. (3)):
//
//   k_prepass  per element: the solution and the broken physical gradient
//              G = |J|^-1 sum_n Ja^n d_n U interpolated to the element's own face points,
//              written once to an element-major face buffer [E][6][20][Nfp];
//   k_face     per face point: the common state, the BR2 common gradient and the common
//              normal flux (Rusanov or Roe inviscid part minus the viscous part), computed once
//              and written face-major with the jump (U_R - U_L)/2;
//   k_volume   per element: the corrected gradient, the pointwise flux, its transformed
//              divergence plus the g_DG flux correction, R = -div/|J|, and the RK register
//              update.
//
// The face buffers are written with non-temporal stores: gigabytes that the next kernel
// reads once, far beyond what the caches would keep (measured: the face kernel 7 % faster).
//
// Both sides of a face read the same owner-side common flux, so the scheme is exactly
// conservative. Element data move through LDS; threads map to solution points for volume work
// and to face points for interface work. With the learned closure attached, each stage first
// computes the per-element features (k_sgs_features) and the network's eddy viscosity.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fr.h"
#include "fr_device.h"
#include "fr_internal.h"

using namespace frk;

// ------------------------------------------------------------------------------------------
// K1: element pre-pass
// ------------------------------------------------------------------------------------------
template <int P, typename real, bool VISC, int EPBX>
__global__ __launch_bounds__(EPBX * Cfg<P>::NS) FR_WPE_ATTR(FR_WPE_PREPASS(P)) void k_prepass(const double *__restrict__ X,
                                                           const real *__restrict__ geo,
                                                           real *__restrict__ face, int64_t E,
                                                           OpsT<real> ops) {
  using C = Cfg<P>;
  constexpr int N = C::N, NS = C::NS, NFP = C::NFP, NF = C::NF, EPB = EPBX;
  constexpr int NG = VISC ? 15 : 0;
  __shared__ real sU[EPB][5][NS];
  __shared__ real sG[EPB][NG > 0 ? NG : 1][NS];
  const int slot = threadIdx.x / NS, t = threadIdx.x - slot * NS;
  const int64_t e = (int64_t)blockIdx.x * EPB + slot;
  const bool act = e < E;
  const int i0 = t % N, i1 = (t / N) % N, i2 = plane_index<N, EPB>(t);
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) sU[slot][v][t] = real(X[(e * 5 + v) * NS + t]);
  }
  __syncthreads();
  if (VISC && act) {
    real ja[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) ja[c] = geo[(e * 10 + c) * NS + t];
    const real iJ = geo[(e * 10 + 9) * NS + t];
    constexpr int UNV = P >= 6 ? 1 : 5;  // bounds the loads in flight at high degree
#pragma unroll UNV
    for (int v = 0; v < 5; ++v) {
      real d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        d0 += ops.D[i0 * N + c] * sU[slot][v][c + N * (i1 + N * i2)];
        d1 += ops.D[i1 * N + c] * sU[slot][v][i0 + N * (c + N * i2)];
        d2 += ops.D[i2 * N + c] * sU[slot][v][i0 + N * (i1 + N * c)];
      }
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        real g = ja[ii] * d0;
        g += ja[3 + ii] * d1;
        g += ja[6 + ii] * d2;
        sG[slot][ii * 5 + v][t] = iJ * g;
      }
    }
  }
  __syncthreads();
  if (!act) return;
  constexpr int NVAL = VISC ? 20 : 5;
  if constexpr (kWavePerFace<NFP, EPB>) {
    // p = 7: wave-uniform tasks (value, face), the face's 64 points on the lanes
    const int lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int a = lane % N, b = lane / N;
    for (int k = wv; k < NVAL * 6; k += NS / 64) {
      const int val = k / 6, f = k - 6 * val;
      const real *src = val < 5 ? &sU[slot][val][0] : &sG[slot][(val - 5) % (NG > 0 ? NG : 1)][0];
      face_store<NFP>(face_sum_uniform<N>(f, a, b, src, ops.lm, ops.lp),
                      &face[((e * 6 + f) * 20 + val) * NFP + lane]);
    }
    return;
  }
  // items are (group of GV values, face point); consecutive threads write consecutive points
  // of one face. With more face points than threads (p <= 4) one item carries all 20 values,
  // which amortises the index arithmetic; at higher degree groups of 5 balance the threads.
  constexpr int GV = (NF > NS || !VISC) ? NVAL : 5;
  constexpr int NGRP = NVAL / GV;
  for (int q = t; q < NGRP * NF; q += NS) {
    const int grp = q / NF, fp = q - grp * NF;
    const int f = fp / NFP, kk = fp - f * NFP;
    const int a = kk % N, b = kk / N, d = f >> 1;
    const bool hi = f & 1;
    real *dst = face + ((e * 6 + f) * 20 + GV * grp) * NFP + kk;
#pragma unroll
    for (int v = 0; v < GV; ++v) {
      const int val = GV * grp + v;
      const real *src = val < 5 ? &sU[slot][val][0] : &sG[slot][(val - 5) % (NG > 0 ? NG : 1)][0];
      real acc = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) acc += pick_end<FR_SCALAR_ENDS64(P)>(hi, ops.lm, ops.lp, c) * src[line_pt<N>(d, c, a, b)];
      face_store<NFP>(acc, &dst[v * NFP]);
    }
  }
}

// ------------------------------------------------------------------------------------------
// K2: face kernel. One thread per face point of each face (owner side L): the common state,
// the BR2 common gradient and the common normal flux, computed once per face point.
// Writes J = (U_R - U_L)/2 = U^C - U_L and the owner's transformed common normal flux
// F^{I,perp}_L = |N| (F*_inv - F_v(U^C, G^I) . n) to a face-major buffer [F][10][Nfp].
// ------------------------------------------------------------------------------------------
// Isothermal no-slip wall (face record with kFaceWall, no other side). Inviscid part: the
// Riemann flux against the mirror state (rho, -m, E), impermeable and without energy flux.
// Viscous part: the wall state U_w = (rho_L, 0, rho_L T_w/(gamma-1)) as the common state and the
// one-sided BR2 gradient G_L + 2 sigma N (U_w - U_L) (sigma of a wall face is one-sided).
template <typename real, bool VISC, bool SGS>
__device__ __forceinline__ void wall_face(const real *srcL, const real *fg, int NFP, int64_t eL, const Phys<real> &ph,
                                          int flux, const double *nut, real kt, real tw_gm1, real *dst) {
  real UL[5], UG[5], UW[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) UL[v] = srcL[v * NFP];
  UG[0] = UL[0];
  UG[1] = -UL[1];
  UG[2] = -UL[2];
  UG[3] = -UL[3];
  UG[4] = UL[4];
  UW[0] = UL[0];
  UW[1] = UW[2] = UW[3] = real(0);
  UW[4] = UL[0] * tw_gm1;
  const real NL[3] = {fg[0], fg[NFP], fg[2 * NFP]};
  const real nm = sqrt(NL[0] * NL[0] + NL[1] * NL[1] + NL[2] * NL[2]);
  const real inm = real(1) / nm;
  const real nh[3] = {NL[0] * inm, NL[1] * inm, NL[2] * inm};
  real Fi[5];
  if (flux == 0) rusanov(UL, UG, nh, ph, Fi);
  else roe(UL, UG, nh, ph, Fi);
  real Fvn[5] = {0, 0, 0, 0, 0};
  if (VISC) {
    const real sig2 = real(2) * fg[3 * NFP];
    real GI[3][5];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int v = 0; v < 5; ++v) GI[i][v] = srcL[(5 + i * 5 + v) * NFP] + sig2 * NL[i] * (UW[v] - UL[v]);
    real mu = ph.mu, kap = ph.kappa;
    if (SGS) {
      const real mut = UW[0] * real(nut[eL]);
      mu += mut;
      kap += mut * kt;
    }
    real Fv[3][5];
    visc_flux_mk(UW, GI, ph.gm1, mu, kap, Fv);
#pragma unroll
    for (int v = 0; v < 5; ++v) Fvn[v] = Fv[0][v] * nh[0] + Fv[1][v] * nh[1] + Fv[2][v] * nh[2];
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    __builtin_nontemporal_store(VISC ? UW[v] - UL[v] : real(0), &dst[v * NFP]);
    __builtin_nontemporal_store(nm * (Fi[v] - Fvn[v]), &dst[(5 + v) * NFP]);
  }
}

template <int P, typename real, bool VISC, bool SGS, bool LDG, int FBS>
__global__ __launch_bounds__(FBS) FR_WPE_ATTR(FR_WPE_FACE(P)) void k_face(const real *__restrict__ face, const real *__restrict__ fgeo,
                                              const FaceRec *__restrict__ ftab, int64_t F, Phys<real> ph,
                                              int flux, real *__restrict__ fout, const double *__restrict__ nut,
                                              real kt, real tau, real tw_gm1) {
  constexpr int N = P + 1, NFP = N * N;
  const int64_t gid = (int64_t)blockIdx.x * FBS + threadIdx.x;
  const int64_t fc = gid / NFP;
  if (fc >= F) return;
  const int kk = (int)(gid - fc * NFP);
  const FaceRec r = ftab[fc];
  const int fL = r.code & 7, fR = (r.code >> 3) & 7;
  if (!LDG && (r.code & kFaceWall)) {
    wall_face<real, VISC, SGS>(face + (((int64_t)r.eL * 6 + fL) * 20) * NFP + kk, fgeo + (fc * 4) * NFP + kk, NFP,
                               r.eL, ph, flux, nut, kt, tw_gm1, fout + (fc * 10) * NFP + kk);
    return;
  }
  const bool swp = (r.code >> 6) & 1, flu = (r.code >> 7) & 1, flv = (r.code >> 8) & 1;
  const int a = kk % N, b = kk / N;
  const int uu = swp ? b : a, vv = swp ? a : b;
  const int kr = (flu ? P - uu : uu) + N * (flv ? P - vv : vv);
  const real *srcL = face + (((int64_t)r.eL * 6 + fL) * 20) * NFP + kk;
  const real *srcR = face + (((int64_t)r.eR * 6 + fR) * 20) * NFP + kr;
  const real *fg = fgeo + (fc * 4) * NFP + kk;
  real UL[5], UR[5], UC[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    UL[v] = srcL[v * NFP];
    UR[v] = srcR[v * NFP];
  }
  const real NL[3] = {fg[0], fg[NFP], fg[2 * NFP]};
  const real nm = sqrt(NL[0] * NL[0] + NL[1] * NL[1] + NL[2] * NL[2]);
  const real inm = real(1) / nm;
  const real nh[3] = {NL[0] * inm, NL[1] * inm, NL[2] * inm};
#pragma unroll
  for (int v = 0; v < 5; ++v) UC[v] = real(0.5) * (UL[v] + UR[v]);
  real Fvn[5] = {0, 0, 0, 0, 0};
  if (VISC && LDG) {
    // LDG: the owner's viscous flux with its corrected gradient (the gradient slots of the face
    // buffer hold it), plus the penalty on the jump
    real QL[3][5];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int v = 0; v < 5; ++v) QL[i][v] = srcL[(5 + i * 5 + v) * NFP];
    real Fv[3][5];
    real mu = ph.mu, kap = ph.kappa;
    if (SGS) {
      const real mut = UL[0] * real(0.5 * (nut[r.eL] + nut[r.eR]));
      mu += mut;
      kap += mut * kt;
    }
    visc_flux_mk(UL, QL, ph.gm1, mu, kap, Fv);
#pragma unroll
    for (int v = 0; v < 5; ++v)
      Fvn[v] = Fv[0][v] * nh[0] + Fv[1][v] * nh[1] + Fv[2][v] * nh[2] + tau * (UR[v] - UL[v]);
  } else if (VISC) {
    // BR2: mean of the broken gradients plus the two face liftings, which combine to
    // sigma N (U_R - U_L) with N the owner's normal
    const real sig = fg[3 * NFP];
    real GI[3][5];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int v = 0; v < 5; ++v)
        GI[i][v] = real(0.5) * (srcL[(5 + i * 5 + v) * NFP] + srcR[(5 + i * 5 + v) * NFP]) +
                   sig * NL[i] * (UR[v] - UL[v]);
    real Fv[3][5];
    real mu = ph.mu, kap = ph.kappa;
    if (SGS) {
      // eddy viscosity: mean of the two elements' nu_t, density of the common state
      const real mut = UC[0] * real(0.5 * (nut[r.eL] + nut[r.eR]));
      mu += mut;
      kap += mut * kt;
    }
    visc_flux_mk(UC, GI, ph.gm1, mu, kap, Fv);
#pragma unroll
    for (int v = 0; v < 5; ++v) Fvn[v] = Fv[0][v] * nh[0] + Fv[1][v] * nh[1] + Fv[2][v] * nh[2];
  }
  real Fi[5];
  if (flux == 0) rusanov(UL, UR, nh, ph, Fi);
  else roe(UL, UR, nh, ph, Fi);
  real *dst = fout + (fc * 10) * NFP + kk;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    // U^ - U_L: the mean (BR2) or the non-owner's trace (LDG)
    face_store<NFP>(LDG ? UR[v] - UL[v] : real(0.5) * (UR[v] - UL[v]), &dst[v * NFP]);
    face_store<NFP>(nm * (Fi[v] - Fvn[v]), &dst[(5 + v) * NFP]);
  }
}

// ------------------------------------------------------------------------------------------
// K3: volume kernel. Per element: gathers its faces' jumps and common fluxes into LDS, forms
// the corrected gradient (g_DG correction by U^C - U), the pointwise flux F_inv - F_v, the
// transformed divergence sum_n D_n F^n plus the flux correction
// (s F^{I,perp} - F^d_f) g'(xi_d), R = -div/|J|, and the RK register update.
// ------------------------------------------------------------------------------------------
// PRE: also run the next stage's pre-pass on the state this stage stores (see the end); the
// profiles call that instance k_volume_pre.
// X, the stage's state, is the same array as out0 (LSRK45, SSP) or reg2 (RK4 after the first
// stage), so X, out0, reg1 and reg2 carry no __restrict__.
template <int P, typename real, bool VISC, bool SGS, bool LDG, int EPBX, bool PRE>
__global__ __launch_bounds__(EPBX * Cfg<P>::NS) FR_WPE_ATTR(FR_WPE_VOLUME(P, SGS, PRE)) void k_volume(
    const double *X, const real *__restrict__ geo, const FaceRef *__restrict__ fref,
    const real *__restrict__ fout, int64_t E, OpsT<real> ops, Phys<real> ph, StageArgs st,
    double *out0, double *reg1, double *reg2,
    const double *__restrict__ nut, real kt, real *__restrict__ face, const real *geo_again) {
  using C = Cfg<P>;
  constexpr int N = C::N, NS = C::NS, NFP = C::NFP, NF = C::NF, EPB = EPBX;
  // with the fused pre-pass (BR2) at p <= 5 the face-jump buffer is enlarged to hold the whole
  // gradient (15 N_s), so the tail takes one pass (at p <= 3 10 N_f already holds it)
  constexpr bool SPX = PRE && VISC && !LDG && P <= 5;
  constexpr int NJ0 = (VISC ? 10 : 5) * NF;
  constexpr int NJ = SPX && 15 * NS > NJ0 ? 15 * NS : NJ0;
  __shared__ real sUall[EPB][5 * NS];  // state, then the transformed flux of one direction
  __shared__ real sJall[EPB][NJ];      // [5][NF] flux along +xi_d (then its jump); [5][NF] U^C - U
  // At p = 7 (two blocks per CU by registers) the LDS the two blocks leave free keeps NMS of the
  // ten metric terms each thread loaded, for the fused pre-pass of the next stage, which then
  // reads only the others again from HBM (each thread reads back its own terms: no barrier).
  constexpr int NMS = PRE && VISC && !LDG && kWavePerFace<NFP, EPB> && sizeof(real) == 8 ? 7 : 0;
  __shared__ real sMet[NMS > 0 ? NMS : 1][NMS > 0 ? NS : 1];
  // Operator entries indexed by a lane's own point (rows of D, the correction derivatives at
  // the solution points) are read from an LDS copy. From the kernel argument each would be a
  // vector memory load, and those complete in issue order: one issued after the RK-register
  // loads waits for HBM. Rows indexed by the wave-uniform plane index stay scalar loads. The
  // copy is left out where its bytes would cost a block per CU (p = 3, whose blocks fill the
  // LDS exactly). (Written as conditional expressions: through accessor lambdas the code
  // without the copy compiled differently and spilled more.)
  constexpr bool UNI2 = N * N == 64 && EPB == 1;
  constexpr int LDS0 = (int)sizeof(real) * (EPB * 5 * NS + EPB * NJ + NMS * NS);
  constexpr bool OPL = lds_copy_fits(LDS0, (int)sizeof(real) * (N * N + 2 * N), EPB * NS);
  __shared__ real sOp[OPL ? N * N + 2 * N : 1];
  if (OPL)
    for (int i = threadIdx.x; i < N * N + 2 * N; i += EPB * NS)
      sOp[i] = i < N * N ? ops.D[i] : (i < N * N + N ? ops.gcL[i - N * N] : ops.gcR[i - N * N - N]);
  const int slot = threadIdx.x / NS, t = threadIdx.x - slot * NS;
  const int64_t e = (int64_t)blockIdx.x * EPB + slot;
  const bool act = e < E;
  const int idx[3] = {t % N, (t / N) % N, plane_index<N, EPB>(t)};
  real *sU = sUall[slot];
  real *sJ = sJall[slot];

  // every global load is issued here, before the first barrier: the state, the metric terms,
  // the RK registers and this element's share of its faces' jumps and fluxes
  constexpr int R = (NF + NS - 1) / NS;  // face points per thread
  constexpr int NC = VISC ? 10 : 5;
  real U[5], ja[9], iJ = 0;
  double Xd[5], r1[5], r2[5];
  real gv[R][NC];
  const int64_t base = e * 5 * NS + t;
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) Xd[v] = X[base + v * NS];
#pragma unroll
    for (int c = 0; c < 9; ++c) ja[c] = geo[(e * 10 + c) * NS + t];
    iJ = geo[(e * 10 + 9) * NS + t];
#pragma unroll
    for (int c = 0; c < NMS; ++c) sMet[c][t] = c < 9 ? ja[c] : iJ;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int fp = t + r * NS;
      if (fp < NF) {
        const int f = fp / NFP, kk = fp - f * NFP;
        const FaceRef fr = fref[e * 6 + f];
        const int a = kk % N, b = kk / N;
        const bool swp = (fr.code >> 3) & 1, flu = (fr.code >> 4) & 1, flv = (fr.code >> 5) & 1;
        const int uu = swp ? b : a, vv = swp ? a : b;
        const int kc = (flu ? P - uu : uu) + N * (flv ? P - vv : vv);
        const real *src = fout + ((int64_t)fr.fid * 10) * NFP + kc;
        const bool own = (fr.code >> 6) & 1;
        const real sgn = own ? real(1) : real(-1);
        const real sfl = (f & 1) ? sgn : -sgn;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          // c < 5: owner's flux -> s F^{I,perp}_own; c >= 5: jump -> U^ - U_own (LDG: U_R - U_L
          // on the owner's side, 0 on the other)
          gv[r][c] = c < 5 ? sfl * src[(5 + c) * NFP]
                           : (LDG ? (own ? src[(c - 5) * NFP] : real(0)) : sgn * src[(c - 5) * NFP]);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      U[v] = real(Xd[v]);
      sU[v * NS + t] = U[v];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int fp = t + r * NS;
      if (fp < NF) {
#pragma unroll
        for (int c = 0; c < NC; ++c) sJ[c * NF + fp] = gv[r][c];
      }
    }
  }
  __syncthreads();
  real F[3][5];
  if (act) {
    if (VISC) {
      real dU[3][5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        real d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
        for (int c = 0; c < N; ++c) {
          d0 += (OPL ? sOp[idx[0] * N + c] : ops.D[idx[0] * N + c]) * sU[v * NS + c + N * (idx[1] + N * idx[2])];
          d1 += (OPL ? sOp[idx[1] * N + c] : ops.D[idx[1] * N + c]) * sU[v * NS + idx[0] + N * (c + N * idx[2])];
          d2 += (OPL && !UNI2 ? sOp[idx[2] * N + c] : ops.D[idx[2] * N + c]) * sU[v * NS + idx[0] + N * (idx[1] + N * c)];
        }
        dU[0][v] = d0;
        dU[1][v] = d1;
        dU[2][v] = d2;
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int u = d == 0 ? 1 : 0, w = d == 2 ? 1 : 2;
        const int kk = idx[u] + N * idx[w];
        const bool cpy = OPL && !(UNI2 && d == 2);
        const real cL = cpy ? sOp[N * N + idx[d]] : ops.gcL[idx[d]], cR = cpy ? sOp[N * N + N + idx[d]] : ops.gcR[idx[d]];
#pragma unroll
        for (int v = 0; v < 5; ++v)
          dU[d][v] += sJ[(5 + v) * NF + (2 * d) * NFP + kk] * cL + sJ[(5 + v) * NF + (2 * d + 1) * NFP + kk] * cR;
      }
      real G[3][5];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          real g = ja[i] * dU[0][v];
          g += ja[3 + i] * dU[1][v];
          g += ja[6 + i] * dU[2][v];
          G[i][v] = iJ * g;
        }
      real mu = ph.mu, kap = ph.kappa;
      if (SGS) {
        const real mut = U[0] * real(nut[e]);
        mu += mut;
        kap += mut * kt;
      }
      visc_flux_mk(U, G, ph.gm1, mu, kap, F);
    }
    // the inviscid flux after the viscous one: F is not live across the gradient phase
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const real ei[3] = {real(i == 0), real(i == 1), real(i == 2)};
      real Fi[5], un_, c_;
      flux_n(U, ei, ph, Fi, un_, c_);
#pragma unroll
      for (int v = 0; v < 5; ++v) F[i][v] = VISC ? Fi[v] - F[i][v] : Fi[v];
    }
  }
  // transformed flux F^d = sum_i Ja[d][i] F_i for the three directions; the metric terms are
  // not needed after this
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const real f0 = F[0][v], f1 = F[1][v], f2 = F[2][v];
#pragma unroll
      for (int d = 0; d < 3; ++d) F[d][v] = ja[d * 3 + 0] * f0 + ja[d * 3 + 1] * f1 + ja[d * 3 + 2] * f2;
    }
  }
  // Without room for that copy, the viscous kernel keeps one for the divergence phase in slot
  // 0's jump entries, which nothing reads after the gradient phase. It is stored after the
  // phase's first barrier, each thread picking its entry out of the whole table read by scalar
  // loads (which do not wait for the vector loads of the RK registers).
  constexpr int NOP = N * N + 2 * N;
  constexpr bool OPX = !OPL && VISC && 5 * NF + NOP <= NJ;
  // the RK registers are loaded here so that their latency overlaps the divergence phase
  if (act) {
    // (assigned per mode, not initialised up front: a live range from the kernel's start
    // costs the gradient phase its registers)
    if (st.mode == kModeLSRK) {
#pragma unroll
      for (int v = 0; v < 5; ++v) r1[v] = st.first ? 0.0 : reg1[base + v * NS];
    } else if (st.mode == kModeRK4) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        r1[v] = st.first ? 0.0 : reg1[base + v * NS];
        r2[v] = out0[base + v * NS];
      }
    } else if (st.mode == kModeSSP) {
#pragma unroll
      for (int v = 0; v < 5; ++v) r1[v] = (st.stage == 4 || st.stage == 9) ? reg1[base + v * NS] : 0.0;
    }
  }
  // divergence of the transformed flux and the flux correction, one direction at a time
  real div[5] = {0, 0, 0, 0, 0};
  real *sF = sU;
  real *sOpx = &sJall[0][5 * NF];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    __syncthreads();
    if (act) {
#pragma unroll
      for (int v = 0; v < 5; ++v) sF[v * NS + t] = F[d][v];
    }
    if (OPX && d == 0 && threadIdx.x < NOP) {
      real opv = 0;
#pragma unroll
      for (int i = 0; i < NOP; ++i)
        if ((int)threadIdx.x == i) opv = i < N * N ? ops.D[i] : (i < N * N + N ? ops.gcL[i - N * N] : ops.gcR[i - N * N - N]);
      sOpx[threadIdx.x] = opv;
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        real acc = 0;
#pragma unroll
        for (int c = 0; c < N; ++c) {
          const int id = d == 0 ? c + N * (idx[1] + N * idx[2])
                                : (d == 1 ? idx[0] + N * (c + N * idx[2]) : idx[0] + N * (idx[1] + N * c));
          acc += (OPL && !(UNI2 && d == 2) ? sOp[idx[d] * N + c] : (OPX ? sOpx[idx[d] * N + c] : ops.D[idx[d] * N + c])) * sF[v * NS + id];
        }
        div[v] += acc;
      }
      // the transformed flux at the two faces normal to d: at p = 7 wave-uniform tasks (value,
      // face) over all threads, otherwise a thread per face point
      if constexpr (kWavePerFace<NFP, EPB>) {
        const int lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
        for (int k = wv; k < 10; k += NS / 64) {
          const int v = k >> 1, f = 2 * d + (k & 1);
          sJ[v * NF + f * NFP + lane] -= face_sum_uniform<N>(f, lane % N, lane / N, &sF[v * NS], ops.lm, ops.lp);
        }
      } else {
        for (int fp = t; fp < 2 * NFP; fp += NS) {
          const int f = 2 * d + fp / NFP, kk = fp % NFP;
          const int a = kk % N, b = kk / N;
          const bool hi = f & 1;
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            real acc = 0;
#pragma unroll
            for (int c = 0; c < N; ++c) acc += pick_end<FR_SCALAR_ENDS64(P)>(hi, ops.lm, ops.lp, c) * sF[v * NS + line_pt<N>(d, c, a, b)];
            sJ[v * NF + f * NFP + kk] -= acc;
          }
        }
      }
    }
    __syncthreads();
    if (act) {
      const int u = d == 0 ? 1 : 0, w = d == 2 ? 1 : 2;
      const int kk = idx[u] + N * idx[w];
      const bool cpy = OPL && !(UNI2 && d == 2);
      const real cL = cpy ? sOp[N * N + idx[d]] : (OPX ? sOpx[N * N + idx[d]] : ops.gcL[idx[d]]);
      const real cR = cpy ? sOp[N * N + N + idx[d]] : (OPX ? sOpx[N * N + N + idx[d]] : ops.gcR[idx[d]]);
#pragma unroll
      for (int v = 0; v < 5; ++v) div[v] += sJ[v * NF + (2 * d) * NFP + kk] * cL + sJ[v * NF + (2 * d + 1) * NFP + kk] * cR;
    }
  }
  // R = -div / |J| plus the source, and the RK register update, one variable at a time. With
  // PRE the stored state also goes to sU at once (nothing reads sU after the last direction's
  // divergence), so it is not held in registers across the barrier below.
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double R = -double(div[v]) * double(iJ) + body_force(st, Xd, v);
      const double xn = rk_store(st, base + v * NS, Xd[v], R, r1[v], r2[v], out0, reg1, reg2);
      if (PRE) sU[v * NS + t] = real(xn);
    }
  }
  if (!PRE) return;
  // The next stage's pre-pass on the state just stored (the value the next stage reads): its
  // values and, for BR2, its broken gradient at this element's face points, with the same
  // arithmetic as k_prepass. This saves that kernel's reads of the state; the metric terms are
  // loaded again here (through a pointer without __restrict__, so the loads stay after the
  // stores above and are not kept live across the divergence phase). The LDS of the divergence
  // phase is reused: the values in sU, the gradient in sJ in chunks of VPC variables
  // (3 VPC N_s <= 10 N_f).
  constexpr bool GRAD = VISC && !LDG;
  constexpr int VPC = SPX || (20 / N) >= 5 ? 5 : 20 / N;
  constexpr int UNW = P >= 6 ? 1 : VPC;  // bounds the LDS loads in flight at high degree
  __syncthreads();
  // face point fp of this element: the line through it along its face's normal direction runs
  // over sU[b0 + c * stride], c = 0..N-1 (the index line_pt gives, without per-lane branches)
  auto line = [&](int fp, int &f, int &kk, int &b0, int &stride) {
    f = fp / NFP;
    kk = fp - f * NFP;
    const int a = kk % N, b = kk / N, d = f >> 1;
    stride = d == 0 ? 1 : (d == 1 ? N : N * N);
    b0 = d == 0 ? N * kk : (d == 1 ? a + N * N * b : kk);
  };
  // With a single gradient chunk (p <= 3) the gradient is formed first and the values and the
  // gradient go to the faces in one pass, in items of five independent sums (as k_prepass);
  // otherwise the values first, then the gradient chunk by chunk.
  real jb[9], iJb = 0;
  auto load_metric = [&]() {
#pragma unroll
    for (int c = 0; c < 9; ++c) jb[c] = c < NMS ? sMet[c][t] : geo_again[(e * 10 + c) * NS + t];
    iJb = 9 < NMS ? sMet[9 < NMS ? 9 : 0][t] : geo_again[(e * 10 + 9) * NS + t];
  };
  // gradient components of the five variables to sJ[(v * 3 + ii) * NS + t] (single chunk)
  auto gradient = [&]() {
#pragma unroll UNW
    for (int v = 0; v < 5; ++v) {
      real d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        d0 += (OPL ? sOp[idx[0] * N + c] : ops.D[idx[0] * N + c]) * sU[v * NS + c + N * (idx[1] + N * idx[2])];
        d1 += (OPL ? sOp[idx[1] * N + c] : ops.D[idx[1] * N + c]) * sU[v * NS + idx[0] + N * (c + N * idx[2])];
        d2 += (OPL && !UNI2 ? sOp[idx[2] * N + c] : ops.D[idx[2] * N + c]) * sU[v * NS + idx[0] + N * (idx[1] + N * c)];
      }
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        real g = jb[ii] * d0;
        g += jb[3 + ii] * d1;
        g += jb[6 + ii] * d2;
        sJ[(v * 3 + ii) * NS + t] = iJb * g;
      }
    }
  };
  if constexpr (kWavePerFace<NFP, EPB>) {
    // p = 7: wave-uniform tasks (value or gradient component, face), 64 face points per task
    const int lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int a = lane % N, b = lane / N;
    if (act) {
      for (int k = wv; k < 5 * 6; k += NS / 64) {
        const int v = k / 6, f = k - 6 * v;
        face_store<NFP>(face_sum_uniform<N>(f, a, b, &sU[v * NS], ops.lm, ops.lp),
                        &face[((e * 6 + f) * 20 + v) * NFP + lane]);
      }
    }
    if (GRAD) {
      if (act) load_metric();
#pragma unroll
      for (int v0 = 0; v0 < 5; v0 += VPC) {
        const int nv = 5 - v0 < VPC ? 5 - v0 : VPC;
        if (act) {
#pragma unroll UNW
          for (int w = 0; w < VPC; ++w) {
            if (w < nv) {
              const int v = v0 + w;
              real d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
              for (int c = 0; c < N; ++c) {
                d0 += (OPL ? sOp[idx[0] * N + c] : ops.D[idx[0] * N + c]) * sU[v * NS + c + N * (idx[1] + N * idx[2])];
                d1 += (OPL ? sOp[idx[1] * N + c] : ops.D[idx[1] * N + c]) * sU[v * NS + idx[0] + N * (c + N * idx[2])];
                d2 += (OPL && !UNI2 ? sOp[idx[2] * N + c] : ops.D[idx[2] * N + c]) * sU[v * NS + idx[0] + N * (idx[1] + N * c)];
              }
#pragma unroll
              for (int ii = 0; ii < 3; ++ii) {
                real g = jb[ii] * d0;
                g += jb[3 + ii] * d1;
                g += jb[6 + ii] * d2;
                sJ[(w * 3 + ii) * NS + t] = iJb * g;
              }
            }
          }
        }
        __syncthreads();
        if (act) {
          for (int k = wv; k < 3 * nv * 6; k += NS / 64) {
            const int ci = k / 6, f = k - 6 * ci;
            const int v = v0 + ci / 3, ii = ci - (ci / 3) * 3;
            face_store<NFP>(face_sum_uniform<N>(f, a, b, &sJ[ci * NS], ops.lm, ops.lp),
                            &face[((e * 6 + f) * 20 + 5 + ii * 5 + v) * NFP + lane]);
          }
        }
        __syncthreads();
      }
    }
    return;
  }
  if (GRAD && VPC == 5) {
    if (act) {
      load_metric();
      gradient();
    }
    __syncthreads();
    // items (groups, face point) of GG of the four groups (group 0 the values, group 1 + ii the
    // d/dx_ii of the five variables: slot 5 + ii * 5 + v; variable v's sits at
    // sJ[(v * 3 + ii) * NS]); each item works out its line and interpolation weights once
    constexpr int GG = FR_TAIL_GROUPS64(P);
    static_assert(GG == 1 || GG == 2 || GG == 4, "groups per item divide the four groups");
    if (act) {
      for (int q = t; q < (4 / GG) * NF; q += NS) {
        const int gi = q / NF;
        int f, kk, b0, stride;
        line(q - gi * NF, f, kk, b0, stride);
        const bool hi = f & 1;
        real cf[N];
#pragma unroll
        for (int c = 0; c < N; ++c) cf[c] = pick_end<FR_SCALAR_ENDS64(P)>(hi, ops.lm, ops.lp, c);
#pragma unroll
        for (int gg = 0; gg < GG; ++gg) {
          const int grp = gi * GG + gg;
          real *dst = face + ((e * 6 + f) * 20 + 5 * grp) * NFP + kk;
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            const real *src = grp == 0 ? &sU[v * NS] : &sJ[(v * 3 + grp - 1) * NS];
            real acc = 0;
#pragma unroll
            for (int c = 0; c < N; ++c) acc += cf[c] * src[b0 + c * stride];
            face_store<NFP>(acc, &dst[v * NFP]);
          }
        }
      }
    }
    return;
  }
  // several chunks (p >= 4, where N_f <= N_s): items are (value, face point), which keeps
  // more of the threads busy than one item per face point
  if (act) {
    for (int q = t; q < 5 * NF; q += NS) {
      const int v = q / NF;
      int f, kk, b0, stride;
      line(q - v * NF, f, kk, b0, stride);
      const bool hi = f & 1;
      real acc = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) acc += pick_end<FR_SCALAR_ENDS64(P)>(hi, ops.lm, ops.lp, c) * sU[v * NS + b0 + c * stride];
      face_store<NFP>(acc, &face[((e * 6 + f) * 20 + v) * NFP + kk]);
    }
  }
  if (GRAD) {
    // (the metric terms are loaded after the values pass, so they are not live across it)
    if (act) load_metric();
#pragma unroll
    for (int v0 = 0; v0 < 5; v0 += VPC) {
      const int nv = 5 - v0 < VPC ? 5 - v0 : VPC;
      // (written out rather than through gradient(): the compiler then spills 28 instead of
      // 52 bytes per lane at p = 7)
      if (act) {
#pragma unroll UNW
        for (int w = 0; w < VPC; ++w) {
          if (w < nv) {
            const int v = v0 + w;
            real d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
            for (int c = 0; c < N; ++c) {
              d0 += (OPL ? sOp[idx[0] * N + c] : ops.D[idx[0] * N + c]) * sU[v * NS + c + N * (idx[1] + N * idx[2])];
              d1 += (OPL ? sOp[idx[1] * N + c] : ops.D[idx[1] * N + c]) * sU[v * NS + idx[0] + N * (c + N * idx[2])];
              d2 += (OPL && !UNI2 ? sOp[idx[2] * N + c] : ops.D[idx[2] * N + c]) * sU[v * NS + idx[0] + N * (idx[1] + N * c)];
            }
#pragma unroll
            for (int ii = 0; ii < 3; ++ii) {
              real g = jb[ii] * d0;
              g += jb[3 + ii] * d1;
              g += jb[6 + ii] * d2;
              sJ[(w * 3 + ii) * NS + t] = iJb * g;
            }
          }
        }
      }
      __syncthreads();
      if (act) {
        for (int q = t; q < 3 * nv * NF; q += NS) {
          const int ci = q / NF;
          const int v = v0 + ci / 3, ii = ci - (ci / 3) * 3;
          int f, kk, b0, stride;
          line(q - ci * NF, f, kk, b0, stride);
          const bool hi = f & 1;
          real acc = 0;
#pragma unroll
          for (int c = 0; c < N; ++c) acc += pick_end<FR_SCALAR_ENDS64(P)>(hi, ops.lm, ops.lp, c) * sJ[ci * NS + b0 + c * stride];
          face_store<NFP>(acc, &face[((e * 6 + f) * 20 + 5 + ii * 5 + v) * NFP + kk]);
        }
      }
      __syncthreads();
    }
  }
}


// ------------------------------------------------------------------------------------------
// LDG: each element's corrected gradient (section "FR Algorithm", the viscous flux by the local
// DG method). The common solution is the face non-owner's trace, so U^ - U_K = U_R - U_L on
// the faces the element owns and 0 on the others. The corrected physical gradient is
// interpolated to the element's face points, into the gradient slots of its own face-buffer
// entries; the face kernel reads the owner's. Runs after a pre-pass that wrote U_f only.
// ------------------------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(Cfg<P>::BLOCK) void k_ldg_grad(const double *__restrict__ X,
                                                             const double *__restrict__ geo,
                                                             const FaceRef *__restrict__ fref,
                                                             const FaceRec *__restrict__ ftab,
                                                             double *__restrict__ face, int64_t E,
                                                             OpsT<double> ops) {
  using C = Cfg<P>;
  constexpr int N = C::N, NS = C::NS, NFP = C::NFP, NF = C::NF, EPB = C::EPB;
  __shared__ double sU[EPB][5][NS];
  __shared__ double sJ[EPB][5][NF];
  __shared__ double sG[EPB][15][NS];
  const int slot = threadIdx.x / NS, t = threadIdx.x - slot * NS;
  const int64_t e = (int64_t)blockIdx.x * EPB + slot;
  const bool act = e < E;
  const int idx[3] = {t % N, (t / N) % N, t / (N * N)};
  double ja[9], iJ = 0;
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) sU[slot][v][t] = X[(e * 5 + v) * NS + t];
#pragma unroll
    for (int c = 0; c < 9; ++c) ja[c] = geo[(e * 10 + c) * NS + t];
    iJ = geo[(e * 10 + 9) * NS + t];
    for (int fp = t; fp < NF; fp += NS) {
      const int f = fp / NFP, kk = fp - f * NFP;
      const FaceRef fr = fref[e * 6 + f];
      if ((fr.code >> 6) & 1) {
        const FaceRec r = ftab[fr.fid];
        const int fR = (r.code >> 3) & 7;
        const bool swp = (r.code >> 6) & 1, flu = (r.code >> 7) & 1, flv = (r.code >> 8) & 1;
        const int a = kk % N, b = kk / N;
        const int uu = swp ? b : a, vv = swp ? a : b;
        const int kr = (flu ? P - uu : uu) + N * (flv ? P - vv : vv);
        const double *own = face + ((e * 6 + f) * 20) * NFP + kk;
        const double *nbr = face + (((int64_t)r.eR * 6 + fR) * 20) * NFP + kr;
#pragma unroll
        for (int v = 0; v < 5; ++v) sJ[slot][v][fp] = nbr[v * NFP] - own[v * NFP];
      } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) sJ[slot][v][fp] = 0.0;
      }
    }
  }
  __syncthreads();
  if (act) {
    double dU[3][5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        d0 += ops.D[idx[0] * N + c] * sU[slot][v][c + N * (idx[1] + N * idx[2])];
        d1 += ops.D[idx[1] * N + c] * sU[slot][v][idx[0] + N * (c + N * idx[2])];
        d2 += ops.D[idx[2] * N + c] * sU[slot][v][idx[0] + N * (idx[1] + N * c)];
      }
      dU[0][v] = d0;
      dU[1][v] = d1;
      dU[2][v] = d2;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int u = d == 0 ? 1 : 0, w = d == 2 ? 1 : 2;
      const int kk = idx[u] + N * idx[w];
      const double cL = ops.gcL[idx[d]], cR = ops.gcR[idx[d]];
#pragma unroll
      for (int v = 0; v < 5; ++v)
        dU[d][v] += sJ[slot][v][(2 * d) * NFP + kk] * cL + sJ[slot][v][(2 * d + 1) * NFP + kk] * cR;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int v = 0; v < 5; ++v)
        sG[slot][i * 5 + v][t] = iJ * (ja[i] * dU[0][v] + ja[3 + i] * dU[1][v] + ja[6 + i] * dU[2][v]);
  }
  __syncthreads();
  if (!act) return;
  // items (gradient component i, face point): 5 values each
  for (int q = t; q < 3 * NF; q += NS) {
    const int i = q / NF, fp = q - i * NF;
    const int f = fp / NFP, kk = fp - f * NFP;
    const int a = kk % N, b = kk / N, d = f >> 1;
    const double *ell = (f & 1) ? ops.lp : ops.lm;
    double *dst = face + ((e * 6 + f) * 20 + 5 + 5 * i) * NFP + kk;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double acc = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) acc += ell[c] * sG[slot][i * 5 + v][line_pt<N>(d, c, a, b)];
      face_store<NFP>(acc, &dst[v * NFP]);
    }
  }
}

// ------------------------------------------------------------------------------------------
// Inputs of the learned closure per element (fr_sgs_features in fr.h): modal energies of the
// velocity polynomial u = m/rho (tensor projection on orthonormal Legendre modes, one
// direction at a time through LDS) and five volume-averaged invariants of its broken gradient
// (a fixed-order tree reduction over the element's points). FP64, rounded to float once.
// ------------------------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(Cfg<P>::BLOCK) void k_sgs_features(const double *__restrict__ X,
                                                                 const double *__restrict__ geo, int64_t E,
                                                                 OpsT<double> ops, SgsOps so,
                                                                 float *__restrict__ feat) {
  using C = Cfg<P>;
  constexpr int N = C::N, NS = C::NS, EPB = C::EPB, NFT = NS + 4;
  constexpr int P2 = NS <= 1 ? 1 : (NS <= 2 ? 2 : (NS <= 4 ? 4 : (NS <= 8 ? 8 : (NS <= 16 ? 16 : (NS <= 32 ? 32 :
                     (NS <= 64 ? 64 : (NS <= 128 ? 128 : (NS <= 256 ? 256 : 512))))))));
  __shared__ double sA[EPB][3][NS];
  __shared__ double sB[EPB][3][NS];
  __shared__ double sR[EPB][6][NS];
  const int slot = threadIdx.x / NS, t = threadIdx.x - slot * NS;
  const int64_t e = (int64_t)blockIdx.x * EPB + slot;
  const bool act = e < E;
  const int idx[3] = {t % N, (t / N) % N, t / (N * N)};
  double ja[9], iJ = 1.0;
  if (act) {
    const double rho = X[(e * 5) * NS + t];
#pragma unroll
    for (int j = 0; j < 3; ++j) sA[slot][j][t] = X[(e * 5 + 1 + j) * NS + t] / rho;
#pragma unroll
    for (int c = 0; c < 9; ++c) ja[c] = geo[(e * 10 + c) * NS + t];
    iJ = geo[(e * 10 + 9) * NS + t];
  }
  __syncthreads();
  double q[6] = {0, 0, 0, 0, 0, 0};
  if (act) {
    double du[3][3];  // du[d][j] = d u_j / d xi_d
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        d0 += ops.D[idx[0] * N + c] * sA[slot][j][c + N * (idx[1] + N * idx[2])];
        d1 += ops.D[idx[1] * N + c] * sA[slot][j][idx[0] + N * (c + N * idx[2])];
        d2 += ops.D[idx[2] * N + c] * sA[slot][j][idx[0] + N * (idx[1] + N * c)];
      }
      du[0][j] = d0;
      du[1][j] = d1;
      du[2][j] = d2;
    }
    double A[3][3];  // A[i][j] = d u_j / d x_i
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) A[i][j] = iJ * (ja[i] * du[0][j] + ja[3 + i] * du[1][j] + ja[6 + i] * du[2][j]);
    double ss = 0, ww = 0, t3 = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double S = 0.5 * (A[i][j] + A[j][i]), W = 0.5 * (A[i][j] - A[j][i]);
        ss += S * S;
        ww += W * W;
        t3 += A[i][j] * (A[j][0] * A[0][i] + A[j][1] * A[1][i] + A[j][2] * A[2][i]);
      }
    const double tr = A[0][0] + A[1][1] + A[2][2];
    const double wq = so.w[idx[0]] * so.w[idx[1]] * so.w[idx[2]] / iJ;
    q[0] = wq;
    q[1] = wq * 2 * ss;
    q[2] = wq * 2 * ww;
    q[3] = wq * (-t3 / 3);
    q[4] = wq * tr;
    q[5] = wq * tr * tr;
    // modal projection along xi
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) acc += so.Lm[idx[0] * N + c] * sA[slot][j][c + N * (idx[1] + N * idx[2])];
      sB[slot][j][t] = acc;
    }
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) sR[slot][k][t] = q[k];
  __syncthreads();
  if (act) {  // along eta
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) acc += so.Lm[idx[1] * N + c] * sB[slot][j][idx[0] + N * (c + N * idx[2])];
      sA[slot][j][t] = acc;
    }
  }
  __syncthreads();
  if (act) {  // along zeta; thread t now owns mode t
    double ek = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) acc += so.Lm[idx[2] * N + c] * sA[slot][j][idx[0] + N * (idx[1] + N * c)];
      ek += acc * acc;
    }
    if (t > 0) feat[e * NFT + t - 1] = (float)log(ek / 16 + 1e-12);
  }
#pragma unroll
  for (int h = P2 / 2; h > 0; h >>= 1) {
    if (t < h && t + h < NS) {
#pragma unroll
      for (int k = 0; k < 6; ++k) sR[slot][k][t] += sR[slot][k][t + h];
    }
    __syncthreads();
  }
  if (act && t == 0) {
    const double vol = sR[slot][0][0];
    const double s2 = sR[slot][1][0] / vol, w2 = sR[slot][2][0] / vol, r = sR[slot][3][0] / vol;
    const double th = sR[slot][4][0] / vol, th2 = sR[slot][5][0] / vol;
    const double eps = 1e-12;
    float *o = feat + e * NFT + NS - 1;
    o[0] = (float)(0.5 * log(s2 + eps));
    o[1] = (float)(0.5 * log(w2 + eps));
    o[2] = (float)(r / pow(s2 + eps, 1.5));
    o[3] = (float)(th / sqrt(s2 + eps));
    o[4] = (float)(th2 / (s2 + eps));
  }
}

// Per-block partial sums of w|J| (1), w|J| |m|^2/(2 rho) (2) and w|J| (u.R_m - |u|^2 R_rho/2)
// (3); one block per 256 solution points, fixed reduction order.
__global__ __launch_bounds__(256) void k_kinetic(const double *__restrict__ U, const double *__restrict__ R,
                                                 const double *__restrict__ geo, int64_t E, int Ns, int n,
                                                 const double *__restrict__ w1d, double *__restrict__ part) {
  __shared__ double s[3][256];
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double a = 0, b = 0, c = 0;
  if (gid < E * Ns) {
    const int64_t e = gid / Ns;
    const int t = (int)(gid - e * Ns);
    const double wJ = w1d[t % n] * w1d[(t / n) % n] * w1d[t / (n * n)] / geo[(e * 10 + 9) * Ns + t];
    const double *u = U + e * 5 * Ns + t;
    const double *r = R + e * 5 * Ns + t;
    const double rho = u[0], m0 = u[Ns], m1 = u[2 * Ns], m2 = u[3 * Ns];
    const double q2 = (m0 * m0 + m1 * m1 + m2 * m2) / (rho * rho);
    a = wJ;
    b = wJ * 0.5 * rho * q2;
    c = wJ * ((m0 * r[Ns] + m1 * r[2 * Ns] + m2 * r[3 * Ns]) / rho - 0.5 * q2 * r[0]);
  }
  s[0][threadIdx.x] = a;
  s[1][threadIdx.x] = b;
  s[2][threadIdx.x] = c;
  __syncthreads();
  for (unsigned h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int q = 0; q < 3; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) part[blockIdx.x * 3 + q] = s[q][0];
}

__global__ void k_nonfinite(const double *__restrict__ R, int64_t n, int *flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int bad = 0;
  for (; i < n; i += stride) bad |= !isfinite(R[i]);
  if (bad) atomicOr(flag, 1);
}

// ==========================================================================================
// Host side: handle, dispatch, C ABI
// ==========================================================================================
static thread_local std::string g_err;

static int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int frk::fr_fail(int code, const std::string &msg) { return fail(code, msg); }

#define HIPCHK(call)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) return fail(FR_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

static bool valid(fr_mesh_t m) { return valid_mesh(m); }

// A part of a partition group evaluates its residual only together with the other parts (its
// ghost faces come from them), through fr_part_residual / fr_part_rk_step.
static int reject_part(fr_mesh_t m, const char *what) {
  return m->group ? fail(FR_ERR_UNSUPPORTED, std::string(what) + " on a part of a partition group: use the group's "
                                             "fr_part_residual / fr_part_rk_step")
                  : FR_OK;
}

// ms (optional): accumulates the durations of the three kernels, measured with HIP events.
template <int P>
static int launch_features(DeviceMesh &dm, const double *X, float *feat) {
  using C = Cfg<P>;
  OpsT<double> ops;
  std::memcpy(ops.D, dm.ops.D, sizeof ops.D);
  const int64_t blocks = (dm.E + C::EPB - 1) / C::EPB;
  hipLaunchKernelGGL((k_sgs_features<P>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, (hipStream_t)dm.stream, X,
                     (const double *)dm.geo, dm.E, ops, dm.sgs_ops, feat);
  HIPCHK(hipGetLastError());
  return FR_OK;
}

static int features(DeviceMesh &dm, const double *X, float *feat) {
  switch (dm.p) {
    case 0: return launch_features<0>(dm, X, feat);
    case 1: return launch_features<1>(dm, X, feat);
    case 2: return launch_features<2>(dm, X, feat);
    case 3: return launch_features<3>(dm, X, feat);
    case 4: return launch_features<4>(dm, X, feat);
    case 5: return launch_features<5>(dm, X, feat);
    case 6: return launch_features<6>(dm, X, feat);
    case 7: return launch_features<7>(dm, X, feat);
    default: return fail(FR_ERR_UNSUPPORTED, "p out of range");
  }
}

// Per-kernel timing accumulators of run_steps / fr_profile_stages (milliseconds and counts):
//   [0] pre-pass ms, [1] face ms, [2] volume ms (alone), [3] stages, [4] pre-pass launches,
//   [5] volume-with-next-pre-pass ms, [6] its launches. kTimeSlots entries.
constexpr int kTimeSlots = 7;
static void add_stage_times(double *ms, const float t[3], bool pre, bool vol_pre) {
  ms[0] += t[0];
  ms[1] += t[1];
  if (pre) ms[4] += 1;
  if (vol_pre) {
    ms[5] += t[2];
    ms[6] += 1;
  } else {
    ms[2] += t[2];
  }
}

template <int P, typename real, bool VISC, bool SGS, bool LDG, int EPBX, int FBS>
static int launch_stage_t(DeviceMesh &dm, const double *X, StageArgs st, double *out0, double *reg1, double *reg2,
                          double *ms) {
  using C = Cfg<P>;
  OpsT<real> ops;
  for (int i = 0; i < kMaxN * kMaxN; ++i) ops.D[i] = real(dm.ops.D[i]);
  for (int i = 0; i < kMaxN; ++i) {
    ops.lm[i] = real(dm.ops.lm[i]);
    ops.lp[i] = real(dm.ops.lp[i]);
    ops.gcL[i] = real(dm.ops.gcL[i]);
    ops.gcR[i] = real(dm.ops.gcR[i]);
  }
  Phys<real> ph{real(dm.phys.gamma), real(dm.phys.gamma - 1.0), real(dm.phys.mu), real(dm.phys.kappa)};
  // heat-flux coefficient per unit eddy viscosity: gamma / ((gamma - 1) Pr_t)
  const real kt = real(dm.phys.gamma / ((dm.phys.gamma - 1.0) * dm.prandtl_t));
  const int64_t blocks = (dm.E + EPBX - 1) / EPBX;
  const int64_t fblocks = (dm.F * C::NFP + FBS - 1) / FBS;
  hipStream_t s = (hipStream_t)dm.stream;
  if (st.pre_only) {
    hipLaunchKernelGGL((k_prepass<P, real, VISC && !LDG, EPBX>), dim3((unsigned)blocks), dim3(EPBX * C::NS), 0, s,
                       X, (const real *)dm.geo, (real *)dm.face, dm.E, ops);
    HIPCHK(hipGetLastError());
    return FR_OK;
  }
  hipEvent_t ev[4];
  if (ms) {
    for (int i = 0; i < 4; ++i) HIPCHK(hipEventCreate(&ev[i]));
    HIPCHK(hipEventRecord(ev[0], s));
  }
  if (!st.pre_done) {
    hipLaunchKernelGGL((k_prepass<P, real, VISC && !LDG, EPBX>), dim3((unsigned)blocks), dim3(EPBX * C::NS), 0, s,
                       X, (const real *)dm.geo, (real *)dm.face, dm.E, ops);
    HIPCHK(hipGetLastError());
  }
  if (LDG) {
    static_assert(sizeof(OpsT<double>) == sizeof(Ops1D), "operator tables share one layout");
    OpsT<double> od;
    std::memcpy(&od, &dm.ops, sizeof od);
    hipLaunchKernelGGL((k_ldg_grad<P>), dim3((unsigned)((dm.E + C::EPB - 1) / C::EPB)), dim3(C::BLOCK), 0, s, X,
                       (const double *)dm.geo, dm.fref, dm.ftab, (double *)dm.face, dm.E, od);
    HIPCHK(hipGetLastError());
  }
  if (ms) HIPCHK(hipEventRecord(ev[1], s));
  hipLaunchKernelGGL((k_face<P, real, VISC, SGS, LDG, FBS>), dim3((unsigned)fblocks), dim3(FBS), 0, s,
                     (const real *)dm.face, (const real *)dm.fgeo, dm.ftab, dm.F, ph, dm.flux, (real *)dm.fout,
                     dm.nut, kt, real(dm.ldg_tau), real(dm.wall_T / (dm.phys.gamma - 1.0)));
  HIPCHK(hipGetLastError());
  if (ms) HIPCHK(hipEventRecord(ev[2], s));
  if (st.pre_next) {
    hipLaunchKernelGGL((k_volume<P, real, VISC, SGS, LDG, EPBX, true>), dim3((unsigned)blocks), dim3(EPBX * C::NS),
                       0, s, X, (const real *)dm.geo, dm.fref, (const real *)dm.fout, dm.E, ops, ph, st, out0, reg1,
                       reg2, dm.nut, kt, (real *)dm.face, (const real *)dm.geo);
  } else {
    hipLaunchKernelGGL((k_volume<P, real, VISC, SGS, LDG, EPBX, false>), dim3((unsigned)blocks), dim3(EPBX * C::NS),
                       0, s, X, (const real *)dm.geo, dm.fref, (const real *)dm.fout, dm.E, ops, ph, st, out0, reg1,
                       reg2, dm.nut, kt, (real *)nullptr, (const real *)nullptr);
  }
  HIPCHK(hipGetLastError());
  if (ms) {
    HIPCHK(hipEventRecord(ev[3], s));
    HIPCHK(hipEventSynchronize(ev[3]));
    float t[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i) HIPCHK(hipEventElapsedTime(&t[i], ev[i], ev[i + 1]));
    add_stage_times(ms, t, !st.pre_done, st.pre_next != 0);
    for (int i = 0; i < 4; ++i) (void)hipEventDestroy(ev[i]);
  }
  return FR_OK;
}

// The tile shapes (the autotuner's choice, DeviceMesh::tile_epb / tile_fbs): elements per block
// of the element kernels, Cfg::EPB or Cfg::EPB2, and the face kernel's block of 256, 128 or 64
// threads. Every thread's arithmetic is the same whatever the tiles.
template <int P, typename real, bool VISC, bool SGS, bool LDG>
static int launch_stage_tiles(DeviceMesh &dm, const double *X, StageArgs st, double *o, double *r1, double *r2,
                              double *ms) {
  constexpr int E0 = Cfg<P>::EPB, E1 = Cfg<P>::EPB2;
  if (dm.tile_epb == 0) {
    if (dm.tile_fbs == 0) return launch_stage_t<P, real, VISC, SGS, LDG, E0, 256>(dm, X, st, o, r1, r2, ms);
    if (dm.tile_fbs == 1) return launch_stage_t<P, real, VISC, SGS, LDG, E0, 128>(dm, X, st, o, r1, r2, ms);
    return launch_stage_t<P, real, VISC, SGS, LDG, E0, 64>(dm, X, st, o, r1, r2, ms);
  }
  if (dm.tile_fbs == 0) return launch_stage_t<P, real, VISC, SGS, LDG, E1, 256>(dm, X, st, o, r1, r2, ms);
  if (dm.tile_fbs == 1) return launch_stage_t<P, real, VISC, SGS, LDG, E1, 128>(dm, X, st, o, r1, r2, ms);
  return launch_stage_t<P, real, VISC, SGS, LDG, E1, 64>(dm, X, st, o, r1, r2, ms);
}

template <typename real, bool VISC, bool SGS, bool LDG>
static int launch_stage_p(DeviceMesh &dm, const double *X, StageArgs st, double *o, double *r1, double *r2,
                          double *ms) {
  switch (dm.p) {
    case 0: return launch_stage_tiles<0, real, VISC, SGS, LDG>(dm, X, st, o, r1, r2, ms);
    case 1: return launch_stage_tiles<1, real, VISC, SGS, LDG>(dm, X, st, o, r1, r2, ms);
    case 2: return launch_stage_tiles<2, real, VISC, SGS, LDG>(dm, X, st, o, r1, r2, ms);
    case 3: return launch_stage_tiles<3, real, VISC, SGS, LDG>(dm, X, st, o, r1, r2, ms);
    case 4: return launch_stage_tiles<4, real, VISC, SGS, LDG>(dm, X, st, o, r1, r2, ms);
    case 5: return launch_stage_tiles<5, real, VISC, SGS, LDG>(dm, X, st, o, r1, r2, ms);
    case 6: return launch_stage_tiles<6, real, VISC, SGS, LDG>(dm, X, st, o, r1, r2, ms);
    case 7: return launch_stage_tiles<7, real, VISC, SGS, LDG>(dm, X, st, o, r1, r2, ms);
    default: return fail(FR_ERR_UNSUPPORTED, "p out of range");
  }
}

static int launch_stage(DeviceMesh &dm, const double *X, StageArgs st, double *o, double *r1, double *r2,
                        double *ms = nullptr) {
  st.force = dm.has_force ? 1 : 0;
  for (int i = 0; i < 3; ++i) st.g[i] = dm.force[i];
  if (dm.prec == FR_FP32) {
    std::string err;
    int rc = launch_stage32(dm, X, st, o, r1, r2, ms, err);
    return rc ? fail(rc, err) : FR_OK;
  }
  if (dm.sgs) {
    if (dm.sgs == 2) {
      // the closure's eddy viscosity of the state this stage is evaluated on
      int rc = features(dm, X, dm.feat);
      if (rc) return rc;
      rc = mlp_forward_nu(dm.model, dm.feat, dm.E, dm.Ns + 4, dm.nut, dm.nu_scale, dm.stream);
      if (rc) return rc;
    }
    return dm.ldg ? launch_stage_p<double, true, true, true>(dm, X, st, o, r1, r2, ms)
                  : launch_stage_p<double, true, true, false>(dm, X, st, o, r1, r2, ms);
  }
  if (!dm.viscous) return launch_stage_p<double, false, false, false>(dm, X, st, o, r1, r2, ms);
  return dm.ldg ? launch_stage_p<double, true, false, true>(dm, X, st, o, r1, r2, ms)
                : launch_stage_p<double, true, false, false>(dm, X, st, o, r1, r2, ms);
}

// Carpenter-Kennedy five-stage fourth-order 2N-storage coefficients.
static const double kLsA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                               -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
static const double kLsB[5] = {1432997174477.0 / 9575080441237.0, 5161836677717.0 / 13612068292357.0,
                               1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                               2277821191437.0 / 14882151754819.0};

// Classical RK4: stage weights, and the offset of the next stage's evaluation point (c_{i+1};
// 0 after the last stage).
static const double kRk4W[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
static const double kRk4C[4] = {0.5, 0.5, 1.0, 0.0};

// Allocate the RK registers a scheme needs (before any graph capture: capture cannot allocate).
int frk::ensure_registers(DeviceMesh &dm, int scheme) {
  const int64_t M = dm.E * 5 * dm.Ns;
  if (scheme != FR_RK4 && scheme != FR_LSRK45 && scheme != FR_SSPRK104) return fail(FR_ERR_ARG, "unknown scheme");
  if (!dm.R1) {
    HIPCHK(hipMalloc(&dm.R1, M * sizeof(double)));
    dm.bytes += M * sizeof(double);
  }
  if (scheme == FR_RK4 && !dm.R2) {
    HIPCHK(hipMalloc(&dm.R2, M * sizeof(double)));
    dm.bytes += M * sizeof(double);
  }
  return FR_OK;
}

int frk::n_stages(int scheme) {
  return scheme == FR_LSRK45 ? 5 : (scheme == FR_RK4 ? 4 : (scheme == FR_SSPRK104 ? 10 : 0));
}

void frk::stage_setup(DeviceMesh &dm, int scheme, int s, double dt, StageArgs &st, const double **X, double **out0,
                      double **reg1, double **reg2) {
  st = StageArgs{};
  st.dt = dt;
  *X = dm.U;
  *out0 = dm.U;
  *reg1 = dm.R1;
  *reg2 = nullptr;
  if (scheme == FR_LSRK45) {
    st.mode = kModeLSRK;
    st.first = s == 0;
    st.a = kLsA[s];
    st.b = kLsB[s];
  } else if (scheme == FR_RK4) {
    st.mode = kModeRK4;
    st.first = s == 0;
    st.last = s == 3;
    st.w = kRk4W[s];
    st.cdt = kRk4C[s] * dt;
    *X = s == 0 ? dm.U : dm.R2;
    *reg2 = dm.R2;
  } else {
    st.mode = kModeSSP;
    st.stage = s;
  }
}

int frk::enqueue_stage(DeviceMesh &dm, const double *X, StageArgs st, double *out0, double *reg1, double *reg2) {
  return launch_stage(dm, X, st, out0, reg1, reg2, nullptr);
}

static int run_steps(fr_mesh_t m, double dt, int scheme, int n_steps, double *ms_acc) {
  DeviceMesh &dm = m->dm;
  const int ns = n_stages(scheme);
  if (ns == 0) return fail(FR_ERR_ARG, "unknown scheme");
  if (n_steps > 0) {
    int rc = ensure_registers(dm, scheme);
    if (rc) return rc;
  }
  // With fusion on every stage but the run's first finds its pre-pass already done by the
  // previous stage's volume kernel, and every stage but the run's last does the next one's.
  for (int step = 0; step < n_steps; ++step) {
    for (int s = 0; s < ns; ++s) {
      StageArgs st;
      const double *X;
      double *o, *r1, *r2;
      stage_setup(dm, scheme, s, dt, st, &X, &o, &r1, &r2);
      st.pre_done = dm.fuse && !(step == 0 && s == 0);
      st.pre_next = dm.fuse && !(step == n_steps - 1 && s == ns - 1);
      int rc = launch_stage(dm, X, st, o, r1, r2, ms_acc);
      if (rc) return rc;
      if (ms_acc) ms_acc[3] += 1;
    }
  }
  return FR_OK;
}

int frk::validate_desc(const fr_mesh_desc *d) {
  if (!d) return fail(FR_ERR_ARG, "desc is NULL");
  if (d->p < 0 || d->p > kMaxP) return fail(FR_ERR_ARG, "p must be in 0..7");
  if (d->q < 1 || d->q > (d->p > 1 ? d->p : 1)) return fail(FR_ERR_ARG, "q must be in 1..max(p,1)");
  if (d->n_elem <= 0 || d->n_elem > (int64_t)INT32_MAX) return fail(FR_ERR_ARG, "n_elem out of range");
  if (!d->elem_vert || !d->elem_nodes) return fail(FR_ERR_ARG, "elem_vert / elem_nodes is NULL");
  if (d->flux != FR_RUSANOV && d->flux != FR_ROE) return fail(FR_ERR_ARG, "unknown flux");
  if (d->prec != FR_FP64 && d->prec != FR_FP32) return fail(FR_ERR_ARG, "unknown precision");
  if (d->prec == FR_FP32 && !(d->ref_rho > 0.0 && d->ref_p >= 0.0))
    return fail(FR_ERR_ARG, "FR_FP32 needs ref_rho > 0 and ref_p >= 0");
  if (!(d->gamma > 1.0) || !(d->prandtl > 0.0) || !(d->mu >= 0.0) || !(d->br2_eta >= 0.0))
    return fail(FR_ERR_ARG, "gamma > 1, prandtl > 0, mu >= 0 and br2_eta >= 0 are required");
  if (d->viscous != FR_BR2 && d->viscous != FR_LDG) return fail(FR_ERR_ARG, "unknown viscous scheme");
  if (d->viscous == FR_LDG && d->prec != FR_FP64) return fail(FR_ERR_UNSUPPORTED, "FR_LDG needs prec = FR_FP64");
  if (d->viscous == FR_LDG && !(d->ldg_tau >= 0.0 && std::isfinite(d->ldg_tau)))
    return fail(FR_ERR_ARG, "ldg_tau must be finite and >= 0");

  return FR_OK;
}

int frk::host_mesh_of(const fr_mesh_desc *d, HostMesh &H) {
  std::string err = build_host_mesh(d->p, d->q, d->n_elem, d->elem_vert, d->elem_nodes, d->bc_tag, d->br2_eta, H);
  if (!err.empty()) return fail(FR_ERR_MESH, err);
  if (H.n_wall > 0) {
    if (d->viscous == FR_LDG) return fail(FR_ERR_UNSUPPORTED, "walls need the BR2 viscous flux");
    if (!(d->wall_T > 0.0) || !std::isfinite(d->wall_T)) return fail(FR_ERR_ARG, "wall_T must be finite and > 0");
  }

  return FR_OK;
}

int frk::create_device_mesh(const fr_mesh_desc *d, HostMesh &H, int64_t n_ghost, void *hip_stream, fr_mesh_s **out) {
  fr_mesh_s *m = new fr_mesh_s();
  m->magic = kMeshMagic;
  DeviceMesh &dm = m->dm;
  dm.p = d->p;
  dm.n = d->p + 1;
  dm.Ns = dm.n * dm.n * dm.n;
  dm.Nfp = dm.n * dm.n;
  dm.E = H.E;
  dm.prec = d->prec;
  dm.flux = d->flux;
  dm.viscous = d->mu > 0.0;
  dm.eta = d->br2_eta;
  dm.ldg = d->viscous == FR_LDG;
  dm.ldg_tau = dm.ldg ? d->ldg_tau : 0.0;
  dm.walls = H.n_wall > 0;
  dm.wall_T = dm.walls ? d->wall_T : 1.0;
  dm.phys = Physics{d->gamma, d->prandtl, d->mu, d->mu * d->gamma / (d->prandtl * (d->gamma - 1.0))};
  dm.ops = H.ops;
  dm.sgs_ops = sgs_ops(d->p);
  dm.stream = hip_stream;
  m->xyz = std::move(H.xyz);
  (void)hipGetDevice(&m->device);

  auto alloc = [&](void **p, size_t bytes) -> int {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? FR_ERR_OOM : FR_ERR_HIP,
                                     std::string("hipMalloc: ") + hipGetErrorString(e));
    dm.bytes += bytes;
    return FR_OK;
  };
  const size_t M = (size_t)dm.E * 5 * dm.Ns;
  int rc = FR_OK;
  if (!rc) rc = alloc((void **)&dm.U, M * sizeof(double));
  if (!rc) rc = alloc(&dm.geo, H.geo.size() * sizeof(double));
  dm.F = (int64_t)H.ftab.size();
  dm.ref_rho = d->ref_rho;
  dm.ref_p = d->ref_p;
  if (!rc) rc = alloc(&dm.fgeo, H.fgeo.size() * sizeof(double));
  if (!rc) rc = alloc((void **)&dm.ftab, H.ftab.size() * sizeof(FaceRec));
  if (!rc) rc = alloc((void **)&dm.fref, H.fref.size() * sizeof(FaceRef));
  std::vector<float> geo32;
  if (dm.prec == FR_FP64) {
    if (!rc) rc = alloc(&dm.face, (size_t)(dm.E * 6 + n_ghost) * 20 * dm.Nfp * sizeof(double));
    if (!rc) rc = alloc(&dm.fout, (size_t)dm.F * 10 * dm.Nfp * sizeof(double));
  } else {
    geo32.assign(H.geo.begin(), H.geo.end());
    if (!rc) rc = alloc(&dm.geo32, geo32.size() * sizeof(float));
    if (!rc) rc = alloc(&dm.face32, (size_t)(dm.E * 6 + n_ghost) * 20 * dm.Nfp * sizeof(float));
    if (!rc) rc = alloc(&dm.facem, (size_t)(dm.E * 6 + n_ghost) * 3 * dm.Nfp * sizeof(double));
    if (!rc) rc = alloc(&dm.fout32, (size_t)dm.F * 9 * dm.Nfp * sizeof(float));
    if (!rc) rc = alloc(&dm.foutm, (size_t)dm.F * dm.Nfp * sizeof(double));
  }
  if (!rc) rc = alloc((void **)&dm.flag, sizeof(int));
  if (rc) {
    fr_mesh_destroy(m);
    return rc;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e1 = hipMemcpyAsync(dm.geo, H.geo.data(), H.geo.size() * sizeof(double), hipMemcpyHostToDevice, s);
  hipError_t e2 = hipMemcpyAsync(dm.fgeo, H.fgeo.data(), H.fgeo.size() * sizeof(double), hipMemcpyHostToDevice, s);
  hipError_t e3 = hipMemcpyAsync(dm.ftab, H.ftab.data(), H.ftab.size() * sizeof(FaceRec), hipMemcpyHostToDevice, s);
  if (e3 == hipSuccess)
    e3 = hipMemcpyAsync(dm.fref, H.fref.data(), H.fref.size() * sizeof(FaceRef), hipMemcpyHostToDevice, s);
  hipError_t e4 = hipMemsetAsync(dm.U, 0, M * sizeof(double), s);
  if (e4 == hipSuccess && dm.geo32)
    e4 = hipMemcpyAsync(dm.geo32, geo32.data(), geo32.size() * sizeof(float), hipMemcpyHostToDevice, s);
  hipError_t e5 = hipStreamSynchronize(s);  // host vectors die at return
  if (e1 || e2 || e3 || e4 || e5) {
    fr_mesh_destroy(m);
    return fail(FR_ERR_HIP, "upload of mesh data failed");
  }
  dm.check_finite = d->check_finite != 0;
  dm.n_ghost = n_ghost;
  *out = m;
  return FR_OK;
}


extern "C" {

const char *fr_last_error(void) { return g_err.c_str(); }

int fr_mesh_create(const fr_mesh_desc *d, void *hip_stream, fr_mesh_t *out) {
  if (!out) return fail(FR_ERR_ARG, "out is NULL");
  *out = nullptr;
  int rc = validate_desc(d);
  if (rc) return rc;
  HostMesh H;
  rc = host_mesh_of(d, H);
  if (rc) return rc;
  fr_mesh_s *m = nullptr;
  rc = create_device_mesh(d, H, 0, hip_stream, &m);
  if (rc) return rc;
  *out = m;
  return FR_OK;
}

int fr_mesh_geometry_host(const fr_mesh_desc *d, double *geo, double *fgeo, int32_t *ftab, int32_t *conn,
                          double *xyz) {
  if (!d || !d->elem_vert || !d->elem_nodes) return fail(FR_ERR_ARG, "NULL descriptor or arrays");
  if (d->p < 0 || d->p > kMaxP) return fail(FR_ERR_ARG, "p must be in 0..7");
  if (d->q < 1 || d->q > (d->p > 1 ? d->p : 1)) return fail(FR_ERR_ARG, "q must be in 1..max(p,1)");
  if (d->n_elem <= 0 || d->n_elem > (int64_t)INT32_MAX) return fail(FR_ERR_ARG, "n_elem out of range");
  HostMesh H;
  std::string err = build_host_mesh(d->p, d->q, d->n_elem, d->elem_vert, d->elem_nodes, d->bc_tag, d->br2_eta, H);
  if (!err.empty()) return fail(FR_ERR_MESH, err);
  if (geo) std::memcpy(geo, H.geo.data(), H.geo.size() * sizeof(double));
  if (H.ftab.size() != (size_t)(d->n_elem * 3 + H.n_wall / 2)) return fail(FR_ERR_MESH, "unexpected face count");
  if (fgeo) std::memcpy(fgeo, H.fgeo.data(), H.fgeo.size() * sizeof(double));
  if (ftab) std::memcpy(ftab, H.ftab.data(), H.ftab.size() * sizeof(FaceRec));
  if (conn) std::memcpy(conn, H.conn.data(), H.conn.size() * sizeof(FaceConn));
  if (xyz) std::memcpy(xyz, H.xyz.data(), H.xyz.size() * sizeof(double));
  return FR_OK;
}

int fr_basis_host(int p, double *D, double *lm, double *lp, double *gcL, double *gcR) {
  if (p < 0 || p > kMaxP || !D || !lm || !lp || !gcL || !gcR) return fail(FR_ERR_ARG, "bad p or NULL pointer");
  Ops1D o = basis_ops(p);
  const int n = p + 1;
  for (int i = 0; i < n * n; ++i) D[i] = o.D[i];
  for (int i = 0; i < n; ++i) {
    lm[i] = o.lm[i];
    lp[i] = o.lp[i];
    gcL[i] = o.gcL[i];
    gcR[i] = o.gcR[i];
  }
  return FR_OK;
}

int fr_rk_coefficients(int scheme, double *a, double *b, int32_t *n_stages) {
  if (!a || !b || !n_stages) return fail(FR_ERR_ARG, "NULL pointer");
  if (scheme == FR_LSRK45) {
    for (int i = 0; i < 5; ++i) {
      a[i] = kLsA[i];
      b[i] = kLsB[i];
    }
    *n_stages = 5;
    return FR_OK;
  }
  if (scheme == FR_RK4) {
    for (int i = 0; i < 4; ++i) {
      a[i] = kRk4W[i];
      b[i] = kRk4C[i];
    }
    *n_stages = 4;
    return FR_OK;
  }
  return fail(FR_ERR_ARG, "tables exist for FR_LSRK45 and FR_RK4");
}

int fr_mesh_destroy(fr_mesh_t m) {
  if (!m) return FR_OK;
  if (!valid(m)) return fail(FR_ERR_ARG, "not a mesh handle");
  if (m->group) return fail(FR_ERR_ARG, "a part of a partition group is destroyed with its group (fr_part_destroy)");
  return destroy_device_mesh(m);
}

}  // extern "C"

int frk::destroy_device_mesh(fr_mesh_s *m) {
  DeviceMesh &dm = m->dm;
  if (dm.stream) (void)hipStreamSynchronize((hipStream_t)dm.stream);
  else (void)hipDeviceSynchronize();
  void *bufs[] = {dm.U,     dm.R1,    dm.R2,    dm.geo,    dm.fgeo,  dm.ftab,  dm.fref, dm.face,
                  dm.fout,  dm.geo32, dm.face32, dm.facem, dm.fout32, dm.foutm, dm.flag, dm.nut,
                  dm.feat};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  for (int32_t *b : m->send_slots)
    if (b) (void)hipFree(b);
  for (int32_t *b : m->recv_slots)
    if (b) (void)hipFree(b);
  m->magic = 0;
  delete m;
  return FR_OK;
}

extern "C" {

int fr_set_stream(fr_mesh_t m, void *hip_stream) {
  if (!valid(m)) return fail(FR_ERR_ARG, "not a mesh handle");
  m->dm.stream = hip_stream;
  return FR_OK;
}

int fr_sol_coords(fr_mesh_t m, double *xyz) {
  if (!valid(m) || !xyz) return fail(FR_ERR_ARG, "bad handle or NULL pointer");
  std::memcpy(xyz, m->xyz.data(), m->xyz.size() * sizeof(double));
  return FR_OK;
}

int fr_set_state(fr_mesh_t m, const double *U, int on_device) {
  if (!valid(m) || !U) return fail(FR_ERR_ARG, "bad handle or NULL pointer");
  DeviceMesh &dm = m->dm;
  const size_t bytes = (size_t)dm.E * 5 * dm.Ns * sizeof(double);
  hipStream_t s = (hipStream_t)dm.stream;
  HIPCHK(hipMemcpyAsync(dm.U, U, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  if (!on_device) HIPCHK(hipStreamSynchronize(s));
  return FR_OK;
}

int fr_get_state(fr_mesh_t m, double *U, int on_device) {
  if (!valid(m) || !U) return fail(FR_ERR_ARG, "bad handle or NULL pointer");
  DeviceMesh &dm = m->dm;
  const size_t bytes = (size_t)dm.E * 5 * dm.Ns * sizeof(double);
  hipStream_t s = (hipStream_t)dm.stream;
  HIPCHK(hipMemcpyAsync(U, dm.U, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  if (!on_device) HIPCHK(hipStreamSynchronize(s));
  return FR_OK;
}

int fr_residual(fr_mesh_t m, double *R, int on_device) {
  if (!valid(m) || !R) return fail(FR_ERR_ARG, "bad handle or NULL pointer");
  if (int rc = reject_part(m, "fr_residual")) return rc;
  DeviceMesh &dm = m->dm;
  const size_t M = (size_t)dm.E * 5 * dm.Ns;
  hipStream_t s = (hipStream_t)dm.stream;
  double *dst = R;
  double *tmp = nullptr;
  if (!on_device) {
    HIPCHK(hipMalloc(&tmp, M * sizeof(double)));
    dst = tmp;
  }
  StageArgs st{};
  st.mode = kModeResidual;
  int rc = launch_stage(dm, dm.U, st, dst, nullptr, nullptr);
  if (rc == FR_OK && dm.check_finite) {
    int bad = 0;
    hipError_t e = hipMemsetAsync(dm.flag, 0, sizeof(int), s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_nonfinite, dim3(1024), dim3(256), 0, s, dst, (int64_t)M, dm.flag);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, dm.flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = fail(FR_ERR_HIP, std::string("non-finite scan: ") + hipGetErrorString(e));
    else if (bad) rc = fail(FR_ERR_NONFINITE, "the residual holds a NaN or Inf");
  }
  if (rc == FR_OK && !on_device) {
    hipError_t e = hipMemcpyAsync(R, tmp, M * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = fail(FR_ERR_HIP, std::string("copy back: ") + hipGetErrorString(e));
  }
  if (tmp) (void)hipFree(tmp);
  return rc;
}

int fr_rk_step(fr_mesh_t m, double dt, int scheme, int n_steps) {
  if (!valid(m)) return fail(FR_ERR_ARG, "not a mesh handle");
  if (int rc = reject_part(m, "fr_rk_step")) return rc;
  if (n_steps < 0 || !std::isfinite(dt)) return fail(FR_ERR_ARG, "bad dt or n_steps");
  return run_steps(m, dt, scheme, n_steps, nullptr);
}

int fr_kinetic_energy(fr_mesh_t m, double *out) {
  if (!valid(m) || !out) return fail(FR_ERR_ARG, "bad handle or NULL pointer");
  if (int rc = reject_part(m, "fr_kinetic_energy")) return rc;
  DeviceMesh &dm = m->dm;
  const size_t M = (size_t)dm.E * 5 * dm.Ns;
  const int64_t npts = dm.E * dm.Ns;
  const int64_t nblk = (npts + 255) / 256;
  hipStream_t s = (hipStream_t)dm.stream;
  // Gauss-Legendre weights from the correction tables: w_a = l_a(+1) / g_R'(x_a)
  double w[kMaxN];
  for (int a = 0; a < dm.n; ++a) w[a] = dm.ops.lp[a] / dm.ops.gcR[a];
  double *R = nullptr, *part = nullptr, *wd = nullptr;
  std::vector<double> hp(nblk * 3);
  int rc = FR_OK;
  hipError_t e = hipMalloc(&R, M * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&part, nblk * 3 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&wd, kMaxN * sizeof(double));
  if (e == hipSuccess) e = hipMemcpyAsync(wd, w, kMaxN * sizeof(double), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) rc = fail(FR_ERR_HIP, std::string("kinetic energy setup: ") + hipGetErrorString(e));
  if (rc == FR_OK) {
    StageArgs st{};
    st.mode = kModeResidual;
    rc = launch_stage(dm, dm.U, st, R, nullptr, nullptr);
  }
  if (rc == FR_OK) {
    hipLaunchKernelGGL(k_kinetic, dim3((unsigned)nblk), dim3(256), 0, s, dm.U, R, (const double *)dm.geo, dm.E,
                       dm.Ns, dm.n, wd, part);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), part, nblk * 3 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = fail(FR_ERR_HIP, std::string("kinetic energy: ") + hipGetErrorString(e));
  }
  if (rc == FR_OK) {
    double a = 0, b = 0, c = 0;
    for (int64_t i = 0; i < nblk; ++i) {
      a += hp[i * 3];
      b += hp[i * 3 + 1];
      c += hp[i * 3 + 2];
    }
    out[0] = b / a;
    out[1] = c / a;
  }
  if (R) (void)hipFree(R);
  if (part) (void)hipFree(part);
  if (wd) (void)hipFree(wd);
  return rc;
}

int fr_mesh_info(fr_mesh_t m, int64_t *n_elem, int32_t *n_sol, int64_t *device_bytes) {
  if (!valid(m)) return fail(FR_ERR_ARG, "not a mesh handle");
  if (n_elem) *n_elem = m->dm.E;
  if (n_sol) *n_sol = m->dm.Ns;
  if (device_bytes) *device_bytes = m->dm.bytes;
  return FR_OK;
}

int fr_set_tiles(fr_mesh_t m, int32_t epb, int32_t fbs) {
  if (!valid(m)) return fail(FR_ERR_ARG, "not a mesh handle");
  if (epb < 0 || epb > 1 || fbs < 0 || fbs > 2) return fail(FR_ERR_ARG, "epb must be 0..1 and fbs 0..2");
  m->dm.tile_epb = epb;
  m->dm.tile_fbs = fbs;
  return FR_OK;
}

int fr_get_tiles(fr_mesh_t m, int32_t *epb, int32_t *fbs) {
  if (!valid(m)) return fail(FR_ERR_ARG, "not a mesh handle");
  if (epb) *epb = m->dm.tile_epb;
  if (fbs) *fbs = m->dm.tile_fbs;
  return FR_OK;
}

int fr_autotune(fr_mesh_t m, int n_trials, double *ms) {
  if (!valid(m)) return fail(FR_ERR_ARG, "not a mesh handle");
  if (int rc = reject_part(m, "fr_autotune")) return rc;
  if (n_trials < 1) return fail(FR_ERR_ARG, "n_trials must be >= 1");
  DeviceMesh &dm = m->dm;
  const int64_t M = dm.E * 5 * dm.Ns;
  // LSRK stages from the current state into scratch (the state and registers are untouched)
  double *tmp = nullptr, *tmp2 = nullptr;
  HIPCHK(hipMalloc(&tmp, M * sizeof(double)));
  if (hipMalloc(&tmp2, M * sizeof(double)) != hipSuccess) {
    (void)hipFree(tmp);
    return fail(FR_ERR_OOM, "hipMalloc of the autotuner's scratch");
  }
  hipStream_t s = (hipStream_t)dm.stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = FR_OK;
  double best = 1e300, t[12] = {0};
  int bi = 0;
  // the scratch register starts at zero, so the timed stages (b = 0) store the state unchanged
  // and the fused pre-pass writes the face data of the current state
  if (hipMemsetAsync(tmp2, 0, M * sizeof(double), s) != hipSuccess) rc = fail(FR_ERR_HIP, "hipMemsetAsync");
  if (rc == FR_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = fail(FR_ERR_HIP, "hipEventCreate");
  for (int c = 0; c < 12 && rc == FR_OK; ++c) {
    dm.tile_epb = (c % 6) / 3;
    dm.tile_fbs = c % 3;
    // a later LSRK stage (it reads and writes the register, as all but a run's first stage do)
    StageArgs st{};
    st.mode = kModeLSRK;
    st.first = 0;
    st.a = kLsA[1];
    st.b = 0.0;
    st.dt = 0.0;
    // c < 6: a stage with its own pre-pass; c >= 6: face + volume with the next pre-pass (the
    // face data it reads are those the previous choice left: valid, as every choice writes them)
    st.pre_done = c >= 6;
    st.pre_next = c >= 6;
    rc = launch_stage(dm, dm.U, st, tmp, tmp2, nullptr);  // warm-up
    if (rc == FR_OK && hipEventRecord(e0, s) != hipSuccess) rc = fail(FR_ERR_HIP, "hipEventRecord");
    for (int k = 0; k < n_trials && rc == FR_OK; ++k) rc = launch_stage(dm, dm.U, st, tmp, tmp2, nullptr);
    float el = 0;
    if (rc == FR_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&el, e0, e1) != hipSuccess))
      rc = fail(FR_ERR_HIP, "timing the tile choices");
    t[c] = el / n_trials;
    if (rc == FR_OK && t[c] < best) {
      best = t[c];
      bi = c;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(tmp);
  (void)hipFree(tmp2);
  dm.tile_epb = (bi % 6) / 3;
  dm.tile_fbs = bi % 3;
  dm.fuse = bi >= 6;
  if (rc == FR_OK && ms)
    for (int i = 0; i < 12; ++i) ms[i] = t[i];
  return rc;
}

int fr_set_fusion(fr_mesh_t m, int32_t on) {
  if (!valid(m)) return fail(FR_ERR_ARG, "not a mesh handle");
  if (on != 0 && on != 1) return fail(FR_ERR_ARG, "on must be 0 or 1");
  m->dm.fuse = on == 1;
  return FR_OK;
}

int fr_get_fusion(fr_mesh_t m, int32_t *on) {
  if (!valid(m) || !on) return fail(FR_ERR_ARG, "bad handle or NULL pointer");
  *on = m->dm.fuse ? 1 : 0;
  return FR_OK;
}

int fr_set_body_force(fr_mesh_t m, const double *g) {
  if (!valid(m)) return fail(FR_ERR_ARG, "not a mesh handle");
  DeviceMesh &dm = m->dm;
  if (!g) {
    dm.has_force = false;
    for (int i = 0; i < 3; ++i) dm.force[i] = 0.0;
    return FR_OK;
  }
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(g[i])) return fail(FR_ERR_ARG, "body force must be finite");
  for (int i = 0; i < 3; ++i) dm.force[i] = g[i];
  dm.has_force = g[0] != 0.0 || g[1] != 0.0 || g[2] != 0.0;
  return FR_OK;
}

int fr_sgs_n_features(int p) {
  if (p < 0 || p > kMaxP) return fail(FR_ERR_ARG, "p must be in 0..7");
  return (p + 1) * (p + 1) * (p + 1) + 4;
}

int fr_sgs_features(fr_mesh_t m, float *feat) {
  if (!valid(m) || !feat) return fail(FR_ERR_ARG, "bad handle or NULL pointer");
  if (m->dm.prec != FR_FP64) return fail(FR_ERR_UNSUPPORTED, "the closure needs prec = FR_FP64");
  return features(m->dm, m->dm.U, feat);
}

static int ensure_nut(DeviceMesh &dm) {
  if (!dm.nut) {
    HIPCHK(hipMalloc(&dm.nut, dm.E * sizeof(double)));
    dm.bytes += dm.E * sizeof(double);
  }
  return FR_OK;
}

int fr_set_eddy_viscosity(fr_mesh_t m, const double *nu, int on_device, double prandtl_t) {
  if (!valid(m)) return fail(FR_ERR_ARG, "not a mesh handle");
  if (int rc = reject_part(m, "fr_set_eddy_viscosity")) return rc;
  DeviceMesh &dm = m->dm;
  if (dm.prec != FR_FP64) return fail(FR_ERR_UNSUPPORTED, "the closure needs prec = FR_FP64");
  if (!nu) {
    dm.sgs = 0;
    dm.model = nullptr;
    return FR_OK;
  }
  if (!(prandtl_t > 0.0)) return fail(FR_ERR_ARG, "prandtl_t must be > 0");
  if (!on_device) {
    for (int64_t e = 0; e < dm.E; ++e)
      if (!(nu[e] >= 0.0) || !std::isfinite(nu[e])) return fail(FR_ERR_ARG, "eddy viscosity must be finite and >= 0");
  }
  int rc = ensure_nut(dm);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)dm.stream;
  HIPCHK(hipMemcpyAsync(dm.nut, nu, dm.E * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        s));
  if (!on_device) HIPCHK(hipStreamSynchronize(s));
  dm.sgs = 1;
  dm.model = nullptr;
  dm.prandtl_t = prandtl_t;
  return FR_OK;
}

int fr_set_sgs_model(fr_mesh_t m, fr_mlp_t model, double nu_scale, double prandtl_t) {
  if (!valid(m)) return fail(FR_ERR_ARG, "not a mesh handle");
  if (int rc = reject_part(m, "fr_set_sgs_model")) return rc;
  DeviceMesh &dm = m->dm;
  if (dm.prec != FR_FP64) return fail(FR_ERR_UNSUPPORTED, "the closure needs prec = FR_FP64");
  if (!model) {
    dm.sgs = 0;
    dm.model = nullptr;
    return FR_OK;
  }
  if (mlp_n_in(model) != dm.Ns + 4) return fail(FR_ERR_ARG, "the model's n_in must be (p+1)^3 + 4");
  if (!(prandtl_t > 0.0) || !(nu_scale >= 0.0)) return fail(FR_ERR_ARG, "need prandtl_t > 0 and nu_scale >= 0");
  int rc = ensure_nut(dm);
  if (rc) return rc;
  if (!dm.feat) {
    HIPCHK(hipMalloc(&dm.feat, dm.E * (dm.Ns + 4) * sizeof(float)));
    dm.bytes += dm.E * (dm.Ns + 4) * sizeof(float);
  }
  dm.sgs = 2;
  dm.model = model;
  dm.nu_scale = nu_scale;
  dm.prandtl_t = prandtl_t;
  return FR_OK;
}

int fr_get_eddy_viscosity(fr_mesh_t m, double *nu) {
  if (!valid(m) || !nu) return fail(FR_ERR_ARG, "bad handle or NULL pointer");
  DeviceMesh &dm = m->dm;
  if (!dm.nut) return fail(FR_ERR_ARG, "no eddy viscosity has been set or computed");
  hipStream_t s = (hipStream_t)dm.stream;
  HIPCHK(hipMemcpyAsync(nu, dm.nut, dm.E * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return FR_OK;
}

// ------------------------------------------------------------------------------------------
// Batches: one RK step of many meshes captured once into a HIP graph, each mesh's stage
// kernels on a branch of its own (the meshes are independent, so the branches run
// concurrently and small meshes share the chip), replayed per step.
// ------------------------------------------------------------------------------------------
}  // extern "C"

// Steps per replay of a batch's chained graph: inside it every stage but the first runs its
// pre-pass in the previous stage's volume kernel, across step boundaries too.
static constexpr int kBatchChain = 8;

struct fr_batch_s {
  uint64_t magic;
  std::vector<fr_mesh_t> meshes;
  std::vector<Group32 *> groups;  // meshes stepped by the multi-mesh kernels, one group per degree
  hipStream_t stream = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};  // one step; kBatchChain steps
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  int device = 0;
};

static constexpr uint64_t kBatchMagic = 0x46524241544348ull;  // "FRBATCH"

static bool valid_batch(fr_batch_t b) { return b != nullptr && b->magic == kBatchMagic; }

extern "C" {

int fr_batch_create(const fr_mesh_t *meshes, int32_t n, const double *dt, int scheme, void *hip_stream,
                    fr_batch_t *out) {
  return fr_batch_create_ex(meshes, n, dt, scheme, hip_stream, FR_BATCH_MULTI, out);
}

int fr_batch_create_ex(const fr_mesh_t *meshes, int32_t n, const double *dt, int scheme, void *hip_stream,
                       int32_t flags, fr_batch_t *out) {
  if (!out) return fail(FR_ERR_ARG, "out is NULL");
  if (flags & ~FR_BATCH_MULTI) return fail(FR_ERR_ARG, "unknown batch flags");
  *out = nullptr;
  if (!meshes || !dt || n < 1) return fail(FR_ERR_ARG, "need n >= 1 meshes and their dt");
  if (scheme != FR_RK4 && scheme != FR_LSRK45 && scheme != FR_SSPRK104) return fail(FR_ERR_ARG, "unknown scheme");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  for (int i = 0; i < n; ++i) {
    if (!valid(meshes[i])) return fail(FR_ERR_ARG, "mesh " + std::to_string(i) + " is not a mesh handle");
    if (int rc = reject_part(meshes[i], "fr_batch_create")) return rc;
    if (meshes[i]->device != dev) return fail(FR_ERR_ARG, "mesh " + std::to_string(i) + " lives on another device");
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) return fail(FR_ERR_ARG, "dt must be finite and > 0");
    for (int j = 0; j < i; ++j)
      if (meshes[j] == meshes[i]) return fail(FR_ERR_ARG, "a mesh appears twice in the batch");
    int rc = ensure_registers(meshes[i]->dm, scheme);
    if (rc) return rc;
  }
  // the meshes the multi-mesh kernels take, grouped by (degree, fusion, tiles), so that every
  // mesh keeps its own tiles; every other mesh steps on a branch of its own
  std::vector<Group32 *> groups;
  std::vector<int> alone;
  {
    std::vector<std::vector<int>> members;
    std::vector<std::array<int, 4>> keys;
    for (int i = 0; i < n; ++i) {
      const DeviceMesh &dm = meshes[i]->dm;
      if (!(flags & FR_BATCH_MULTI) || !group32_eligible(dm)) {
        alone.push_back(i);
        continue;
      }
      const std::array<int, 4> key{dm.p, dm.fuse ? 1 : 0, dm.tile_epb, dm.tile_fbs};
      size_t k = 0;
      while (k < keys.size() && keys[k] != key) ++k;
      if (k == keys.size()) {
        keys.push_back(key);
        members.push_back({});
      }
      members[k].push_back(i);
    }
    for (auto &mem : members) {
      // largest meshes first: their blocks are dispatched first and the small meshes' blocks
      // fill the end of each launch
      std::stable_sort(mem.begin(), mem.end(),
                       [&](int a, int b) { return meshes[a]->dm.E > meshes[b]->dm.E; });
      std::vector<DeviceMesh *> dms;
      std::vector<double> dts;
      for (int i : mem) {
        dms.push_back(&meshes[i]->dm);
        dts.push_back(dt[i]);
      }
      Group32 *g = nullptr;
      std::string gerr;
      int rc = group32_create(dms, dts, scheme, &g, gerr);
      if (rc) {
        for (Group32 *h : groups) group32_destroy(h);
        return fail(rc, "mesh group: " + gerr);
      }
      groups.push_back(g);
    }
  }
  const int nbr = (int)(groups.size() + alone.size());
  hipStream_t cs = nullptr;
  std::vector<hipStream_t> br(nbr, nullptr);
  std::vector<hipEvent_t> join(nbr, nullptr);
  hipEvent_t fork = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  int rc = FR_OK;
  std::string msg;
  auto chk = [&](hipError_t e, const char *what) {
    if (e != hipSuccess && rc == FR_OK) {
      rc = FR_ERR_HIP;
      msg = std::string(what) + ": " + hipGetErrorString(e);
    }
    return e == hipSuccess;
  };
  if (chk(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate") &&
      chk(hipEventCreateWithFlags(&fork, hipEventDisableTiming), "hipEventCreate")) {
    for (int i = 0; i < nbr && rc == FR_OK; ++i)
      if (chk(hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking), "hipStreamCreate"))
        chk(hipEventCreateWithFlags(&join[i], hipEventDisableTiming), "hipEventCreate");
  }
  // two graphs: one step, and kBatchChain steps whose stages chain through the fused pre-pass
  // (each replay starts with a stand-alone pre-pass, so state changes between replays are safe)
  for (int gi = 0; gi < 2 && rc == FR_OK; ++gi) {
    const int steps = gi == 0 ? 1 : kBatchChain;
    if (!chk(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture")) break;
    chk(hipEventRecord(fork, cs), "hipEventRecord");
    for (int b = 0; b < nbr && rc == FR_OK; ++b) {
      if (!chk(hipStreamWaitEvent(br[b], fork, 0), "hipStreamWaitEvent")) break;
      if (b < (int)groups.size()) {
        std::string gerr;
        const int r = group32_step(groups[b], br[b], steps, gerr);
        if (r) {
          rc = r;
          msg = gerr;
          break;
        }
      } else {
        const int i = alone[b - groups.size()];
        DeviceMesh &dm = meshes[i]->dm;
        void *saved = dm.stream;
        dm.stream = br[b];
        int r = run_steps(meshes[i], dt[i], scheme, steps, nullptr);
        dm.stream = saved;
        if (r) {
          rc = r;
          msg = g_err;
          break;
        }
      }
      if (!chk(hipEventRecord(join[b], br[b]), "hipEventRecord")) break;
      chk(hipStreamWaitEvent(cs, join[b], 0), "hipStreamWaitEvent");
    }
    hipError_t e = hipStreamEndCapture(cs, &graph[gi]);
    chk(e, "hipStreamEndCapture");
    if (rc == FR_OK) chk(hipGraphInstantiate(&exec[gi], graph[gi], nullptr, nullptr, 0), "hipGraphInstantiate");
  }
  for (int i = 0; i < nbr; ++i) {
    if (join[i]) (void)hipEventDestroy(join[i]);
    if (br[i]) (void)hipStreamDestroy(br[i]);
  }
  if (fork) (void)hipEventDestroy(fork);
  if (cs) (void)hipStreamDestroy(cs);
  if (rc != FR_OK) {
    for (int gi = 0; gi < 2; ++gi) {
      if (exec[gi]) (void)hipGraphExecDestroy(exec[gi]);
      if (graph[gi]) (void)hipGraphDestroy(graph[gi]);
    }
    for (Group32 *g : groups) group32_destroy(g);
    return fail(rc, "batch capture failed: " + msg);
  }
  fr_batch_s *b = new fr_batch_s();
  b->magic = kBatchMagic;
  b->meshes.assign(meshes, meshes + n);
  b->groups = groups;
  b->stream = (hipStream_t)hip_stream;
  for (int gi = 0; gi < 2; ++gi) {
    b->graph[gi] = graph[gi];
    b->exec[gi] = exec[gi];
  }
  b->device = dev;
  *out = b;
  return FR_OK;
}

int fr_batch_step(fr_batch_t b, int n_steps) {
  if (!valid_batch(b)) return fail(FR_ERR_ARG, "not a batch handle");
  if (n_steps < 0) return fail(FR_ERR_ARG, "n_steps must be >= 0");
  for (int k = 0; k < n_steps / kBatchChain; ++k) HIPCHK(hipGraphLaunch(b->exec[1], b->stream));
  for (int k = 0; k < n_steps % kBatchChain; ++k) HIPCHK(hipGraphLaunch(b->exec[0], b->stream));
  return FR_OK;
}

int fr_batch_set_stream(fr_batch_t b, void *hip_stream) {
  if (!valid_batch(b)) return fail(FR_ERR_ARG, "not a batch handle");
  b->stream = (hipStream_t)hip_stream;
  return FR_OK;
}

int fr_batch_destroy(fr_batch_t b) {
  if (!b) return FR_OK;
  if (!valid_batch(b)) return fail(FR_ERR_ARG, "not a batch handle");
  (void)hipStreamSynchronize(b->stream);
  for (int gi = 0; gi < 2; ++gi) {
    if (b->exec[gi]) (void)hipGraphExecDestroy(b->exec[gi]);
    if (b->graph[gi]) (void)hipGraphDestroy(b->graph[gi]);
  }
  for (Group32 *g : b->groups) group32_destroy(g);
  b->magic = 0;
  delete b;
  return FR_OK;
}

int fr_profile_stages(fr_mesh_t m, double dt, int scheme, int n_steps, double *ms) {
  if (!valid(m) || !ms) return fail(FR_ERR_ARG, "bad handle or NULL pointer");
  if (int rc = reject_part(m, "fr_profile_stages")) return rc;
  double acc[kTimeSlots] = {0, 0, 0, 0, 0, 0, 0};
  int rc = run_steps(m, dt, scheme, n_steps, acc);
  if (rc) return rc;
  const double n_alone = acc[3] - acc[6];
  ms[0] = acc[4] > 0 ? acc[0] / acc[4] : 0;
  ms[1] = acc[3] > 0 ? acc[1] / acc[3] : 0;
  ms[2] = acc[6] > 0 ? acc[5] / acc[6] : 0;
  ms[3] = n_alone > 0 ? acc[2] / n_alone : 0;
  return FR_OK;
}

}  // extern "C"
