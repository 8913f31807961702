// fr_kernels32.hip -- the FP32 form of the FR stage (enum FR_FP32): operators and fluxes in
// FP32 with FP64 state, RK registers and mass equation.
//
// At low Mach number the conserved fluxes are dominated by constants: the pressure p0 in the
// momentum flux and the enthalpy H ~ c^2/(gamma-1) in the energy flux are 10^3-10^4 times their
// divergence, and demoting them costs 0.4-2 % of the residual. This form therefore works on
// U' = U - U_ref (formed in FP64; U_ref = (rho_r, 0, 0, 0, E_r) at rest) and splits fluxes:
//
//   mass     F_rho = m                                  FP64 throughout (volume and face)
//   momentum F_m   = m u + p' I,  p' = p - p_r          FP32 (the constant p_r I has zero
//                                                       FR divergence and is dropped)
//   energy   F_E   = H_r m + h' m,  h' = H - H_r        FP32 for h' m; the H_r m part is
//                                                       H_r times the mass flux, so
//                                                       R_E = R''_E + H_r R_rho in FP64
//
// Each identity is exact in exact arithmetic (the FR operator is linear in the flux and a
// constant flux has zero residual), so this computes the same residual as the FP64 form up to
// FP32 round-off in the reduced parts. Common fluxes: the Rusanov / Roe dissipation of the
// reduced energy E'' = E - H_r rho uses the same wave decomposition as the FP64 solvers.
#include <hip/hip_runtime.h>

#include <cstring>

#include <cmath>
#include <cstdint>
#include <string>

#include "fr.h"
#include "fr_device.h"
#include "fr_internal.h"

namespace {

struct Ref32 {
  float rho, E, H;    // reference density, energy, enthalpy (FP32 copies)
  double rho_d, E_d, H_d;
  float p;            // reference pressure
};

// Reduced inviscid flux along unit n of U' (rho', m, E'), and the speeds u.n, c.
//   Fr[0] = m.n (mass, used for the dissipation bookkeeping only)
//   Fr[1..3] = m u.n + p' n;  Fr[4] = h' m.n
__device__ __forceinline__ void reduced_flux_n(const float Up[5], const float n[3], const Phys<float> &ph,
                                               const Ref32 &r, float Fr[5], float &un, float &c, float &pp,
                                               float &hp) {
  const float rho = r.rho + Up[0];
  const float ir = 1.0f / rho;
  const float u = Up[1] * ir, v = Up[2] * ir, w = Up[3] * ir;
  pp = ph.gm1 * (Up[4] - 0.5f * rho * (u * u + v * v + w * w));  // p - p_r (u_ref = 0)
  hp = (Up[4] - r.H * Up[0] + pp) * ir;                            // H - H_r
  un = u * n[0] + v * n[1] + w * n[2];
  const float mn = Up[1] * n[0] + Up[2] * n[1] + Up[3] * n[2];
  Fr[0] = mn;
  Fr[1] = Up[1] * un + pp * n[0];
  Fr[2] = Up[2] * un + pp * n[1];
  Fr[3] = Up[3] * un + pp * n[2];
  Fr[4] = hp * mn;
  c = sqrtf(ph.gamma * (r.p + pp) * ir);
}

// Common reduced flux: Fr[0] carries only the dissipative part of the mass flux (its central
// part is formed in FP64 by the caller); Fr[1..3] momentum; Fr[4] energy minus H_r times mass.
__device__ __forceinline__ void riemann32(const float UL[5], const float UR[5], const float n[3],
                                          const Phys<float> &ph, const Ref32 &r, int flux, float Fr[5]) {
  float FL[5], FR[5], unL, unR, cL, cR, pL, pR, hL, hR;
  reduced_flux_n(UL, n, ph, r, FL, unL, cL, pL, hL);
  reduced_flux_n(UR, n, ph, r, FR, unR, cR, pR, hR);
  float dis[5];
  if (flux == 0) {
    const float lam = fmaxf(fabsf(unL) + cL, fabsf(unR) + cR);
    dis[0] = lam * (UR[0] - UL[0]);
    dis[1] = lam * (UR[1] - UL[1]);
    dis[2] = lam * (UR[2] - UL[2]);
    dis[3] = lam * (UR[3] - UL[3]);
    dis[4] = lam * ((UR[4] - UL[4]) - r.H * (UR[0] - UL[0]));
  } else {
    const float rL = r.rho + UL[0], rR = r.rho + UR[0];
    const float iL = 1.0f / rL, iR = 1.0f / rR;
    const float uL[3] = {UL[1] * iL, UL[2] * iL, UL[3] * iL};
    const float uR[3] = {UR[1] * iR, UR[2] * iR, UR[3] * iR};
    const float sL = sqrtf(rL), sR = sqrtf(rR);
    const float is = 1.0f / (sL + sR);
    const float rt = sL * sR;
    float ut[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) ut[i] = (sL * uL[i] + sR * uR[i]) * is;
    const float ht = (sL * hL + sR * hR) * is;  // Roe-averaged H - H_r
    const float q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
    const float c2 = ph.gm1 * ((r.H + ht) - 0.5f * q2);
    const float ct = sqrtf(c2);
    const float ic2 = 1.0f / c2;
    const float unt = ut[0] * n[0] + ut[1] * n[1] + ut[2] * n[2];
    const float dr = UR[0] - UL[0], dp = pR - pL;
    const float du[3] = {uR[0] - uL[0], uR[1] - uL[1], uR[2] - uL[2]};
    const float dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
    const float a1 = 0.5f * (dp - rt * ct * dun) * ic2;
    const float a5 = 0.5f * (dp + rt * ct * dun) * ic2;
    const float a2 = dr - dp * ic2;
    const float l1 = fabsf(unt - ct), l2 = fabsf(unt), l5 = fabsf(unt + ct);
    const float w1 = l1 * a1, w5 = l5 * a5, w2 = l2 * a2;
    dis[0] = w1 + w5 + w2;
    float udu = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float sh = du[i] - dun * n[i];
      dis[1 + i] = w1 * (ut[i] - ct * n[i]) + w5 * (ut[i] + ct * n[i]) + w2 * ut[i] + l2 * rt * sh;
      udu += ut[i] * sh;
    }
    // energy eigenvector entries minus H_r times the mass entries
    dis[4] = w1 * (ht - unt * ct) + w5 * (ht + unt * ct) + w2 * (0.5f * q2 - r.H) + l2 * rt * udu;
  }
  Fr[0] = -0.5f * dis[0];
#pragma unroll
  for (int v = 1; v < 5; ++v) Fr[v] = 0.5f * (FL[v] + FR[v]) - 0.5f * dis[v];
}

// full float state from U' (for the viscous flux)
__device__ __forceinline__ void full_state(const float Up[5], const Ref32 &r, float U[5]) {
  U[0] = r.rho + Up[0];
  U[1] = Up[1];
  U[2] = Up[2];
  U[3] = Up[3];
  U[4] = r.E + Up[4];
}

// ------------------------------------------------------------------------------------------
// K1 (FP32 form): U' and its broken gradient to the faces in FP32, momentum to the faces in FP64
// ------------------------------------------------------------------------------------------
template <int P, bool VISC, int EPBX>
__device__ __forceinline__ void prepass32_body(unsigned blk, const double *__restrict__ X,
                                                                 const float *__restrict__ geo32,
                                                                 float *__restrict__ face32,
                                                                 double *__restrict__ facem, int64_t E,
                                                                 OpsT<float> ops, OpsT<double> opsd, Ref32 ref) {
  using C = Cfg<P>;
  constexpr int N = C::N, NS = C::NS, NFP = C::NFP, NF = C::NF, EPB = EPBX;
  constexpr int NG = VISC ? 15 : 1;
  // (16-byte aligned: the p = 7 face sums read whole lines with 16-byte loads)
  __shared__ alignas(16) float sU[EPB][5][NS];
  __shared__ alignas(16) double sM[EPB][3][NS];
  __shared__ alignas(16) float sG[EPB][NG][NS];
  constexpr bool WPF = kWavePerFace<NFP, EPB>;
  __shared__ float sRot[WPF ? 4 * N : 1];  // the rotated face sums' weights, FP32 and FP64
  __shared__ double sRotd[WPF ? 4 * N : 1];
  if (WPF)
    for (int i = threadIdx.x; i < 4 * N; i += EPB * NS) {
      sRot[i] = rot_entry<N>(ops.lm, ops.lp, i);
      sRotd[i] = rot_entry<N>(opsd.lm, opsd.lp, i);
    }
  const int slot = threadIdx.x / NS, t = threadIdx.x - slot * NS;
  const int64_t e = (int64_t)blk * EPB + slot;
  const bool act = e < E;
  const int i0 = t % N, i1 = (t / N) % N, i2 = plane_index<N, EPB>(t);
  if (act) {
    const double x0 = X[(e * 5 + 0) * NS + t], x4 = X[(e * 5 + 4) * NS + t];
    sU[slot][0][t] = float(x0 - ref.rho_d);
    sU[slot][4][t] = float(x4 - ref.E_d);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double m = X[(e * 5 + 1 + i) * NS + t];
      sU[slot][1 + i][t] = float(m);
      sM[slot][i][t] = m;
    }
  }
  __syncthreads();
  if (VISC && act) {
    float ja[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) ja[c] = geo32[(e * 10 + c) * NS + t];
    const float iJ = geo32[(e * 10 + 9) * NS + t];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      float d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        d0 += ops.D[i0 * N + c] * sU[slot][v][c + N * (i1 + N * i2)];
        d1 += ops.D[i1 * N + c] * sU[slot][v][i0 + N * (c + N * i2)];
        d2 += ops.D[i2 * N + c] * sU[slot][v][i0 + N * (i1 + N * c)];
      }
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) sG[slot][(ii * 5 + v) % NG][t] = iJ * (ja[ii] * d0 + ja[3 + ii] * d1 + ja[6 + ii] * d2);
    }
  }
  __syncthreads();
  if (!act) return;
  if constexpr (kWavePerFace<NFP, EPB>) {
    // p = 7: wave-uniform tasks (value, face), the face's 64 points on the lanes: U' (5), the
    // gradient (15), then the FP64 momentum (3)
    const int lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int a = lane % N, b = lane / N;
    constexpr int NV = VISC ? 20 : 5;
    for (int k = wv; k < (NV + 3) * 6; k += NS / 64) {
      const int val = k / 6, f = k - 6 * val;
      if (val < NV) {
        const float *src = val < 5 ? &sU[slot][val][0] : &sG[slot][(val - 5) % NG][0];
        face_store<NFP>(face_sum_uniform<N, true>(f, a, b, src, ops.lm, ops.lp, sRot),
                        &face32[((e * 6 + f) * 20 + val) * NFP + lane]);
      } else {
        const int i = val - NV;
        face_store<NFP>(face_sum_uniform<N, true>(f, a, b, &sM[slot][i][0], opsd.lm, opsd.lp, sRotd),
                        &facem[((e * 6 + f) * 3 + i) * NFP + lane]);
      }
    }
    return;
  }
  for (int fp = t; fp < NF; fp += NS) {
    const int f = fp / NFP, kk = fp - f * NFP;
    const int a = kk % N, b = kk / N, d = f >> 1;
    const bool hi = f & 1;
    float ell[N];
    double elld[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      ell[c] = pick_end<FR_SCALAR_ENDS32(P)>(hi, ops.lm, ops.lp, c);
      elld[c] = pick_end<FR_SCALAR_ENDS32(P)>(hi, opsd.lm, opsd.lp, c);
    }
    float *dst = face32 + ((e * 6 + f) * 20) * NFP + kk;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      float acc = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) acc += ell[c] * sU[slot][v][line_pt<N>(d, c, a, b)];
      face_store<NFP>(acc, &dst[v * NFP]);
    }
    if (VISC) {
#pragma unroll 5
      for (int g = 0; g < 15; ++g) {
        float acc = 0;
#pragma unroll
        for (int c = 0; c < N; ++c) acc += ell[c] * sG[slot][g % NG][line_pt<N>(d, c, a, b)];
        face_store<NFP>(acc, &dst[(5 + g) * NFP]);
      }
    }
    double *dm = facem + ((e * 6 + f) * 3) * NFP + kk;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double acc = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) acc += elld[c] * sM[slot][i][line_pt<N>(d, c, a, b)];
      face_store<NFP>(acc, &dm[i * NFP]);
    }
  }
}

template <int P, bool VISC, int EPBX>
__global__ __launch_bounds__(EPBX * Cfg<P>::NS) void k_prepass32(const double *__restrict__ X,
                                                                 const float *__restrict__ geo32,
                                                                 float *__restrict__ face32,
                                                                 double *__restrict__ facem, int64_t E,
                                                                 OpsT<float> ops, OpsT<double> opsd, Ref32 ref) {
  prepass32_body<P, VISC, EPBX>(blockIdx.x, X, geo32, face32, facem, E, ops, opsd, ref);
}

// ------------------------------------------------------------------------------------------
// K2 (FP32 form): common jump and flux per face point. Outputs
//   fout32 [F][9][Nfp]: J' = (U'_R - U'_L)/2 (5), owner's momentum flux (3), reduced energy (1)
//   foutm  [F][Nfp]   : owner's mass flux (FP64)
// ------------------------------------------------------------------------------------------
// Isothermal no-slip wall (face record with kFaceWall, owner side only) in the reduced
// variables. Inviscid part: the Riemann flux against the mirror state (rho', -m, E'), whose mass
// and reduced energy fluxes vanish (the central mass flux (m - m)/2 . N is exactly zero).
// Viscous part: the wall state U_w = (rho_L, 0, rho_L T_w/(gamma-1)) as the common state with the
// one-sided BR2 gradient G_L + 2 sigma N (U_w - U_L). The energy jump is formed as
// E'_w - E'_L = c_w + rho'_L T_w/(gamma-1) - E'_L, with c_w = rho_r T_w/(gamma-1) - E_r taken in
// FP64 on the host, so no FP32 difference of two reference-sized energies is taken.
template <bool VISC>
__device__ __forceinline__ void wall_face32(const float *srcL, const double *fg, int NFP, const Phys<float> &ph,
                                            const Ref32 &ref, int flux, float tw_gm1, float cw, float *dst,
                                            double *dmass) {
  float UL[5], UG[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) UL[v] = srcL[v * NFP];
  UG[0] = UL[0];
  UG[1] = -UL[1];
  UG[2] = -UL[2];
  UG[3] = -UL[3];
  UG[4] = UL[4];
  const float NL[3] = {float(fg[0]), float(fg[NFP]), float(fg[2 * NFP])};
  const float nm = sqrtf(NL[0] * NL[0] + NL[1] * NL[1] + NL[2] * NL[2]);
  const float inm = 1.0f / nm;
  const float nh[3] = {NL[0] * inm, NL[1] * inm, NL[2] * inm};
  float Fr[5];
  riemann32(UL, UG, nh, ph, ref, flux, Fr);
  float Jw[5] = {0, 0, 0, 0, 0};
  if (VISC) {
    Jw[1] = -UL[1];
    Jw[2] = -UL[2];
    Jw[3] = -UL[3];
    Jw[4] = cw + UL[0] * tw_gm1 - UL[4];
    const float sig2 = 2.0f * float(fg[3 * NFP]);
    float GI[3][5];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int v = 0; v < 5; ++v) GI[i][v] = srcL[(5 + i * 5 + v) * NFP] + sig2 * NL[i] * Jw[v];
    float UW[5];
    UW[0] = ref.rho + UL[0];
    UW[1] = UW[2] = UW[3] = 0.0f;
    UW[4] = UW[0] * tw_gm1;
    float Fv[3][5];
    visc_flux(UW, GI, ph, Fv);
#pragma unroll
    for (int v = 1; v < 5; ++v) Fr[v] -= Fv[0][v] * nh[0] + Fv[1][v] * nh[1] + Fv[2][v] * nh[2];
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) __builtin_nontemporal_store(Jw[v], &dst[v * NFP]);
#pragma unroll
  for (int v = 1; v < 5; ++v) __builtin_nontemporal_store(nm * Fr[v], &dst[(4 + v) * NFP]);
  __builtin_nontemporal_store(double(nm * Fr[0]), dmass);
}

template <int P, bool VISC, int FBS>
__device__ __forceinline__ void face32_body(unsigned blk, const float *__restrict__ face32, const double *__restrict__ facem,
                                                const double *__restrict__ fgeo, const FaceRec *__restrict__ ftab,
                                                int64_t F, Phys<float> ph, Ref32 ref, int flux, float tw_gm1,
                                                float cw, float *__restrict__ fout32, double *__restrict__ foutm) {
  constexpr int N = P + 1, NFP = N * N;
  const int64_t gid = (int64_t)blk * FBS + threadIdx.x;
  const int64_t fc = gid / NFP;
  if (fc >= F) return;
  const int kk = (int)(gid - fc * NFP);
  const FaceRec r = ftab[fc];
  const int fL = r.code & 7, fR = (r.code >> 3) & 7;
  if (r.code & kFaceWall) {
    wall_face32<VISC>(face32 + (((int64_t)r.eL * 6 + fL) * 20) * NFP + kk, fgeo + (fc * 4) * NFP + kk, NFP, ph, ref,
                      flux, tw_gm1, cw, fout32 + (fc * 9) * NFP + kk, foutm + fc * NFP + kk);
    return;
  }
  const bool swp = (r.code >> 6) & 1, flu = (r.code >> 7) & 1, flv = (r.code >> 8) & 1;
  const int a = kk % N, b = kk / N;
  const int uu = swp ? b : a, vv = swp ? a : b;
  const int kr = (flu ? P - uu : uu) + N * (flv ? P - vv : vv);
  const float *srcL = face32 + (((int64_t)r.eL * 6 + fL) * 20) * NFP + kk;
  const float *srcR = face32 + (((int64_t)r.eR * 6 + fR) * 20) * NFP + kr;
  const double *mL = facem + (((int64_t)r.eL * 6 + fL) * 3) * NFP + kk;
  const double *mR = facem + (((int64_t)r.eR * 6 + fR) * 3) * NFP + kr;
  const double *fg = fgeo + (fc * 4) * NFP + kk;
  float UL[5], UR[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    UL[v] = srcL[v * NFP];
    UR[v] = srcR[v * NFP];
  }
  const double Nd[3] = {fg[0], fg[NFP], fg[2 * NFP]};
  // central mass flux in FP64: (m_L + m_R)/2 . N
  const double fc_rho = 0.5 * ((mL[0] + mR[0]) * Nd[0] + (mL[NFP] + mR[NFP]) * Nd[1] + (mL[2 * NFP] + mR[2 * NFP]) * Nd[2]);
  const float NL[3] = {float(Nd[0]), float(Nd[1]), float(Nd[2])};
  const float nm = sqrtf(NL[0] * NL[0] + NL[1] * NL[1] + NL[2] * NL[2]);
  const float inm = 1.0f / nm;
  const float nh[3] = {NL[0] * inm, NL[1] * inm, NL[2] * inm};
  float Fr[5];
  riemann32(UL, UR, nh, ph, ref, flux, Fr);
  if (VISC) {
    const float sig = float(fg[3 * NFP]);
    float GI[3][5];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int v = 0; v < 5; ++v)
        GI[i][v] = 0.5f * (srcL[(5 + i * 5 + v) * NFP] + srcR[(5 + i * 5 + v) * NFP]) + sig * NL[i] * (UR[v] - UL[v]);
    float UCp[5], UC[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) UCp[v] = 0.5f * (UL[v] + UR[v]);
    full_state(UCp, ref, UC);
    float Fv[3][5];
    visc_flux(UC, GI, ph, Fv);
#pragma unroll
    for (int v = 1; v < 5; ++v) Fr[v] -= Fv[0][v] * nh[0] + Fv[1][v] * nh[1] + Fv[2][v] * nh[2];
  }
  float *dst = fout32 + (fc * 9) * NFP + kk;
#pragma unroll
  for (int v = 0; v < 5; ++v) face_store<NFP>(0.5f * (UR[v] - UL[v]), &dst[v * NFP]);
#pragma unroll
  for (int v = 1; v < 5; ++v) face_store<NFP>(nm * Fr[v], &dst[(4 + v) * NFP]);
  __builtin_nontemporal_store(fc_rho + double(nm * Fr[0]), &foutm[fc * NFP + kk]);
}

template <int P, bool VISC, int FBS>
__global__ __launch_bounds__(FBS) void k_face32(const float *__restrict__ face32, const double *__restrict__ facem,
                                                const double *__restrict__ fgeo, const FaceRec *__restrict__ ftab,
                                                int64_t F, Phys<float> ph, Ref32 ref, int flux, float tw_gm1,
                                                float cw, float *__restrict__ fout32, double *__restrict__ foutm) {
  face32_body<P, VISC, FBS>(blockIdx.x, face32, facem, fgeo, ftab, F, ph, ref, flux, tw_gm1, cw, fout32, foutm);
}

// ------------------------------------------------------------------------------------------
// K3 (FP32 form): corrected gradient, reduced fluxes, divergence + correction in FP32 for
// momentum and reduced energy, in FP64 for mass; R_E = R''_E + H_r R_rho; RK update in FP64.
// ------------------------------------------------------------------------------------------
// PRE: also run the next stage's pre-pass (k_prepass32's outputs) on the state this stage
// stores (see the end); the profiles call that instance k_volume32_pre.
// X, the stage's state, is the same array as out0 (LSRK45, SSP) or reg2 (RK4 after the first
// stage), so X, out0, reg1 and reg2 carry no __restrict__.
template <int P, bool VISC, int EPBX, bool PRE>
__device__ __forceinline__ void volume32_body(unsigned blk,
    const double *X, const double *__restrict__ geo, const FaceRef *__restrict__ fref,
    const float *__restrict__ fout32, const double *__restrict__ foutm, int64_t E, OpsT<float> ops,
    OpsT<double> opsd, Phys<float> ph, Ref32 ref, StageArgs st, double *out0,
    double *reg1, double *reg2, float *__restrict__ face32,
    double *__restrict__ facem, const float *geo32_again) {
  using C = Cfg<P>;
  constexpr int N = C::N, NS = C::NS, NFP = C::NFP, NF = C::NF, EPB = EPBX;
  constexpr int R = (NF + NS - 1) / NS;
  // with the fused pre-pass at p <= 6 (SP) the tail takes one pass: sJ and sM are enlarged to
  // hold the whole gradient (15 N_s) and the three momentum components (measured: faster than
  // the rounds below by 27% at p = 4 and 6% at p = 6; at p = 7 the larger LDS costs 3%)
  constexpr bool SP = PRE && P <= 6;
  constexpr int NJ0 = (VISC ? 9 : 4) * NF;  // [4][NF] flux (mom 3, reduced energy), [5][NF] jumps
  constexpr int NJ = SP && VISC && 15 * NS > NJ0 ? 15 * NS : NJ0;
  constexpr int NMS = SP ? 3 * NS : NS;
  // (16-byte aligned: the p = 7 face sums read whole lines with 16-byte loads)
  __shared__ alignas(16) float sUall[EPB][5 * NS];  // U', later 4 components of the transformed flux
  __shared__ alignas(16) double sMall[EPB][NMS];    // transformed mass flux of one direction
  __shared__ alignas(16) float sJall[EPB][NJ];
  __shared__ double sJmall[EPB][NF];       // mass flux along +xi_d, then its jump
  // With the fused pre-pass at p = 3 and p = 7 the LDS left free at these kernels' occupancy
  // (four blocks of four waves, two of eight) keeps the FP32 metric terms each thread converts
  // from the FP64 ones it loaded (the same roundings as the FP32 geometry copy), so the tail does
  // not read that copy from HBM again; each thread reads back its own terms (no barrier).
  constexpr bool MST = PRE && VISC && (P == 3 || P == 7);
  __shared__ float sMetall[EPB][MST ? 10 * NS : 1];
  // Operator entries indexed by a lane's own point (rows of D, the correction derivatives at
  // the solution points) come from LDS copies, as in the FP64 volume kernel: from the kernel
  // argument each would be a vector memory load, which completes in issue order, after the
  // RK-register loads. Rows indexed by the wave-uniform plane index stay scalar loads; the copies
  // are left out where their bytes would cost a block per CU. (Conditional expressions rather
  // than accessor lambdas, which changed the code generated without the copies.)
  constexpr bool UNI2 = N * N == 64 && EPB == 1;
  constexpr int NOP = N * N + 2 * N;
  constexpr int LDS0 = EPB * (4 * 5 * NS + 8 * NMS + 4 * NJ + 8 * NF + (MST ? 4 * 10 * NS : 0));
  constexpr bool OPL = lds_copy_fits(LDS0, 12 * NOP, EPB * NS);
  __shared__ float sOpf[OPL ? NOP : 1];
  __shared__ double sOpd[OPL ? NOP : 1];
  if (OPL)
    for (int i = threadIdx.x; i < NOP; i += EPB * NS) {
      sOpf[i] = i < N * N ? ops.D[i] : (i < N * N + N ? ops.gcL[i - N * N] : ops.gcR[i - N * N - N]);
      sOpd[i] = i < N * N ? opsd.D[i] : (i < N * N + N ? opsd.gcL[i - N * N] : opsd.gcR[i - N * N - N]);
    }
  constexpr bool WPF = kWavePerFace<NFP, EPB>;
  __shared__ float sRot[WPF ? 4 * N : 1];  // the rotated face sums' weights, FP32 and FP64
  __shared__ double sRotd[WPF ? 4 * N : 1];
  if (WPF)
    for (int i = threadIdx.x; i < 4 * N; i += EPB * NS) {
      sRot[i] = rot_entry<N>(ops.lm, ops.lp, i);
      sRotd[i] = rot_entry<N>(opsd.lm, opsd.lp, i);
    }
  const int slot = threadIdx.x / NS, t = threadIdx.x - slot * NS;
  const int64_t e = (int64_t)blk * EPB + slot;
  const bool act = e < E;
  const int idx[3] = {t % N, (t / N) % N, plane_index<N, EPB>(t)};
  float *sU = sUall[slot];
  double *sM = sMall[slot];
  float *sJ = sJall[slot];
  double *sJm = sJmall[slot];
  const int64_t base = e * 5 * NS + t;
  double Xd[5], jad[9], iJd = 0, r1[5], r2[5];
  if (act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) Xd[v] = X[base + v * NS];
#pragma unroll
    for (int c = 0; c < 9; ++c) jad[c] = geo[(e * 10 + c) * NS + t];
    iJd = geo[(e * 10 + 9) * NS + t];
    if (MST) {
#pragma unroll
      for (int c = 0; c < 9; ++c) sMetall[slot][c * NS + t] = float(jad[c]);
      sMetall[slot][9 * NS + t] = float(iJd);
    }
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
        const float *src = fout32 + ((int64_t)fr.fid * 9) * NFP + kc;
        const bool owner = (fr.code >> 6) & 1;
        const float sgn = owner ? 1.0f : -1.0f;
        const float sfl = (f & 1) ? sgn : -sgn;
#pragma unroll
        for (int c = 0; c < 4; ++c) sJ[c * NF + fp] = sfl * src[(5 + c) * NFP];
        if (VISC) {
#pragma unroll
          for (int c = 0; c < 5; ++c) sJ[(4 + c) * NF + fp] = sgn * src[c * NFP];
        }
        sJm[fp] = double(sfl) * foutm[(int64_t)fr.fid * NFP + kc];
      }
    }
    sU[0 * NS + t] = float(Xd[0] - ref.rho_d);
    sU[1 * NS + t] = float(Xd[1]);
    sU[2 * NS + t] = float(Xd[2]);
    sU[3 * NS + t] = float(Xd[3]);
    sU[4 * NS + t] = float(Xd[4] - ref.E_d);
  }
  __syncthreads();
  float F[3][5];  // [direction][component]: 0 unused, 1-3 momentum, 4 reduced energy
  double Fm[3];   // transformed mass flux per direction (FP64)
  if (act) {
    float Up[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) Up[v] = sU[v * NS + t];
    if (VISC) {
      float ja[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) ja[c] = float(jad[c]);
      const float iJ = float(iJd);
      float dU[3][5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        float d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
        for (int c = 0; c < N; ++c) {
          d0 += (OPL ? sOpf[idx[0] * N + c] : ops.D[idx[0] * N + c]) * sU[v * NS + c + N * (idx[1] + N * idx[2])];
          d1 += (OPL ? sOpf[idx[1] * N + c] : ops.D[idx[1] * N + c]) * sU[v * NS + idx[0] + N * (c + N * idx[2])];
          d2 += (OPL && !UNI2 ? sOpf[idx[2] * N + c] : ops.D[idx[2] * N + c]) * sU[v * NS + idx[0] + N * (idx[1] + N * c)];
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
        const float cL = cpy ? sOpf[N * N + idx[d]] : ops.gcL[idx[d]], cR = cpy ? sOpf[N * N + N + idx[d]] : ops.gcR[idx[d]];
#pragma unroll
        for (int v = 0; v < 5; ++v)
          dU[d][v] += sJ[(4 + v) * NF + (2 * d) * NFP + kk] * cL + sJ[(4 + v) * NF + (2 * d + 1) * NFP + kk] * cR;
      }
      float G[3][5];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int v = 0; v < 5; ++v) G[i][v] = iJ * (ja[i] * dU[0][v] + ja[3 + i] * dU[1][v] + ja[6 + i] * dU[2][v]);
      float Uf[5];
      full_state(Up, ref, Uf);
      visc_flux(Uf, G, ph, F);
    }
    // the inviscid flux after the viscous one: F is not live across the gradient phase
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float ei[3] = {float(i == 0), float(i == 1), float(i == 2)};
      float Fi[5], un_, c_, pp_, hp_;
      reduced_flux_n(Up, ei, ph, ref, Fi, un_, c_, pp_, hp_);
#pragma unroll
      for (int v = 1; v < 5; ++v) F[i][v] = VISC ? Fi[v] - F[i][v] : Fi[v];
    }
    // transformed fluxes per direction
#pragma unroll
    for (int v = 1; v < 5; ++v) {
      const float f0 = F[0][v], f1 = F[1][v], f2 = F[2][v];
#pragma unroll
      for (int d = 0; d < 3; ++d)
        F[d][v] = float(jad[d * 3 + 0]) * f0 + float(jad[d * 3 + 1]) * f1 + float(jad[d * 3 + 2]) * f2;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) Fm[d] = jad[d * 3 + 0] * Xd[1] + jad[d * 3 + 1] * Xd[2] + jad[d * 3 + 2] * Xd[3];
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
  float div[5] = {0, 0, 0, 0, 0};
  double divm = 0;
  float *sF = sU;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    __syncthreads();
    if (act) {
#pragma unroll
      for (int v = 1; v < 5; ++v) sF[(v - 1) * NS + t] = F[d][v];
      sM[t] = Fm[d];
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float acc = 0;
#pragma unroll
        for (int c = 0; c < N; ++c) {
          const int id = d == 0 ? c + N * (idx[1] + N * idx[2])
                                : (d == 1 ? idx[0] + N * (c + N * idx[2]) : idx[0] + N * (idx[1] + N * c));
          acc += (OPL && !(UNI2 && d == 2) ? sOpf[idx[d] * N + c] : ops.D[idx[d] * N + c]) * sF[v * NS + id];
        }
        div[1 + v] += acc;
      }
      {
        double acc = 0;
#pragma unroll
        for (int c = 0; c < N; ++c) {
          const int id = d == 0 ? c + N * (idx[1] + N * idx[2])
                                : (d == 1 ? idx[0] + N * (c + N * idx[2]) : idx[0] + N * (idx[1] + N * c));
          acc += (OPL && !(UNI2 && d == 2) ? sOpd[idx[d] * N + c] : opsd.D[idx[d] * N + c]) * sM[id];
        }
        divm += acc;
      }
      if constexpr (kWavePerFace<NFP, EPB>) {
        // p = 7: wave-uniform tasks (component, face of direction d), component 4 the FP64 mass
        const int lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
        for (int k = wv; k < 10; k += NS / 64) {
          const int v = k >> 1, f = 2 * d + (k & 1);
          if (v < 4)
            sJ[v * NF + f * NFP + lane] -= face_sum_uniform<N>(f, lane % N, lane / N, &sF[v * NS], ops.lm, ops.lp);
          else
            sJm[f * NFP + lane] -= face_sum_uniform<N>(f, lane % N, lane / N, sM, opsd.lm, opsd.lp);
        }
      } else
      for (int fp = t; fp < 2 * NFP; fp += NS) {
        const int f = 2 * d + fp / NFP, kk = fp % NFP;
        const int a = kk % N, b = kk / N;
        const bool hi = f & 1;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float acc = 0;
#pragma unroll
          for (int c = 0; c < N; ++c) acc += pick_end<FR_SCALAR_ENDS32(P)>(hi, ops.lm, ops.lp, c) * sF[v * NS + line_pt<N>(d, c, a, b)];
          sJ[v * NF + f * NFP + kk] -= acc;
        }
        double acc = 0;
#pragma unroll
        for (int c = 0; c < N; ++c) acc += pick_end<FR_SCALAR_ENDS32(P)>(hi, opsd.lm, opsd.lp, c) * sM[line_pt<N>(d, c, a, b)];
        sJm[f * NFP + kk] -= acc;
      }
    }
    __syncthreads();
    if (act) {
      const int u = d == 0 ? 1 : 0, w = d == 2 ? 1 : 2;
      const int kk = idx[u] + N * idx[w];
      const bool cpy = OPL && !(UNI2 && d == 2);
      const float cL = cpy ? sOpf[N * N + idx[d]] : ops.gcL[idx[d]], cR = cpy ? sOpf[N * N + N + idx[d]] : ops.gcR[idx[d]];
#pragma unroll
      for (int v = 0; v < 4; ++v) div[1 + v] += sJ[v * NF + (2 * d) * NFP + kk] * cL + sJ[v * NF + (2 * d + 1) * NFP + kk] * cR;
      divm += sJm[(2 * d) * NFP + kk] * (cpy ? sOpd[N * N + idx[d]] : opsd.gcL[idx[d]]) + sJm[(2 * d + 1) * NFP + kk] * (cpy ? sOpd[N * N + N + idx[d]] : opsd.gcR[idx[d]]);
    }
  }
  // the RK update; with PRE the stored state also goes to LDS at once as U' (nothing reads sU
  // after the last direction's divergence), and its momentum is kept for the FP64 face values
  double xm[3] = {0, 0, 0};
  if (act) {
    double Rv[5];
    Rv[0] = -divm * iJd;
    Rv[1] = -double(div[1]) * iJd;
    Rv[2] = -double(div[2]) * iJd;
    Rv[3] = -double(div[3]) * iJd;
    Rv[4] = -double(div[4]) * iJd + ref.H_d * Rv[0];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double xn =
          rk_store(st, base + v * NS, Xd[v], Rv[v] + body_force(st, Xd, v), r1[v], r2[v], out0, reg1, reg2);
      if (PRE) {
        sU[v * NS + t] = v == 0 ? float(xn - ref.rho_d) : (v == 4 ? float(xn - ref.E_d) : float(xn));
        if (v >= 1 && v <= 3) xm[v - 1] = xn;
      }
    }
  }
  if (!PRE) return;
  // The next stage's pre-pass on the state just stored, with the same sums as k_prepass32: U'
  // and (viscous) its broken gradient to face32, the momentum in FP64 to facem. The LDS of the
  // divergence phase is reused: U' in sU; at p <= 6 (SP) the momentum and gradient whole in the
  // enlarged sM and sJ, above that one momentum component at a time in sM and the gradient in
  // sJ in chunks of VPC variables (3 VPC N_s <= 9 N_f), round r interpolating momentum
  // component r (r < 3) and gradient chunk r.
  constexpr int VPC = (18 / N) < 5 ? (18 / N) : 5;
  constexpr int NCH = VISC ? (5 + VPC - 1) / VPC : 0;
  constexpr int NR = NCH > 3 ? NCH : 3;
  constexpr int UNW = P >= 6 ? 1 : VPC;  // bounds the LDS loads in flight at high degree
  // face point fp: its line along the face normal runs over [b0 + c * stride], c = 0..N-1
  auto line = [&](int fp, int &f, int &kk, int &b0, int &stride) {
    f = fp / NFP;
    kk = fp - f * NFP;
    const int a = kk % N, b = kk / N, d = f >> 1;
    stride = d == 0 ? 1 : (d == 1 ? N : N * N);
    b0 = d == 0 ? N * kk : (d == 1 ? a + N * N * b : kk);
  };
  __syncthreads();
  if (SP) {
    // one pass: the momentum and the whole gradient to LDS, then items (group, face point) of
    // independent sums: group 0 U', groups 1-3 d/dx_ii of the five variables (face slot
    // 5 + ii * 5 + v, LDS sJ[(v * 3 + ii) * N_s]), the last group the FP64 momentum
    constexpr int NGRP = VISC ? 5 : 2;
    if (act) {
#pragma unroll
      for (int i = 0; i < 3; ++i) sM[i * NS + t] = xm[i];
      if (VISC) {
        float jb[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) jb[c] = MST ? sMetall[slot][c * NS + t] : geo32_again[(e * 10 + c) * NS + t];
        const float iJb = MST ? sMetall[slot][9 * NS + t] : geo32_again[(e * 10 + 9) * NS + t];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          float d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
          for (int c = 0; c < N; ++c) {
            d0 += (OPL ? sOpf[idx[0] * N + c] : ops.D[idx[0] * N + c]) * sU[v * NS + c + N * (idx[1] + N * idx[2])];
            d1 += (OPL ? sOpf[idx[1] * N + c] : ops.D[idx[1] * N + c]) * sU[v * NS + idx[0] + N * (c + N * idx[2])];
            d2 += (OPL && !UNI2 ? sOpf[idx[2] * N + c] : ops.D[idx[2] * N + c]) * sU[v * NS + idx[0] + N * (idx[1] + N * c)];
          }
#pragma unroll
          for (int ii = 0; ii < 3; ++ii) sJ[(v * 3 + ii) * NS + t] = iJb * (jb[ii] * d0 + jb[3 + ii] * d1 + jb[6 + ii] * d2);
        }
      }
    }
    __syncthreads();
    if constexpr (FR_TAIL_PER_POINT32(P)) {
      // whole face points per thread: each point's line and interpolation weights once, then
      // every group; the same sums as the items below
      for (int fp = t; act && fp < NF; fp += NS) {
        int f, kk, b0, stride;
        line(fp, f, kk, b0, stride);
        const bool hi = f & 1;
        float cf[N];
        double cd[N];
#pragma unroll
        for (int c = 0; c < N; ++c) {
          cf[c] = pick_end<FR_SCALAR_ENDS32(P)>(hi, ops.lm, ops.lp, c);
          cd[c] = pick_end<FR_SCALAR_ENDS32(P)>(hi, opsd.lm, opsd.lp, c);
        }
#pragma unroll
        for (int grp = 0; grp < NGRP - 1; ++grp) {
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            const float *src = grp == 0 ? &sU[v * NS] : &sJ[(v * 3 + grp - 1) * NS];
            float acc = 0;
#pragma unroll
            for (int c = 0; c < N; ++c) acc += cf[c] * src[b0 + c * stride];
            face_store<NFP>(acc, &face32[((e * 6 + f) * 20 + 5 * grp + v) * NFP + kk]);
          }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          double acc = 0;
#pragma unroll
          for (int c = 0; c < N; ++c) acc += cd[c] * sM[i * NS + b0 + c * stride];
          face_store<NFP>(acc, &facem[((e * 6 + f) * 3 + i) * NFP + kk]);
        }
      }
      return;
    }
    if (act) {
      for (int q = t; q < NGRP * NF; q += NS) {
        const int grp = q / NF;
        int f, kk, b0, stride;
        line(q - grp * NF, f, kk, b0, stride);
        const bool hi = f & 1;
        if (grp == NGRP - 1) {
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            double acc = 0;
#pragma unroll
            for (int c = 0; c < N; ++c) acc += pick_end<FR_SCALAR_ENDS32(P)>(hi, opsd.lm, opsd.lp, c) * sM[i * NS + b0 + c * stride];
            face_store<NFP>(acc, &facem[((e * 6 + f) * 3 + i) * NFP + kk]);
          }
        } else {
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            const float *src = grp == 0 ? &sU[v * NS] : &sJ[(v * 3 + grp - 1) * NS];
            float acc = 0;
#pragma unroll
            for (int c = 0; c < N; ++c) acc += pick_end<FR_SCALAR_ENDS32(P)>(hi, ops.lm, ops.lp, c) * src[b0 + c * stride];
            face_store<NFP>(acc, &face32[((e * 6 + f) * 20 + 5 * grp + v) * NFP + kk]);
          }
        }
      }
    }
    return;
  }
  // p = 7: the face loops as wave-uniform tasks (value, face), 64 face points per task
  const int lane = t & 63, wv = WPF ? __builtin_amdgcn_readfirstlane(t >> 6) : 0;
  const int la = lane % N, lb = lane / N;
  if (act) {
    if constexpr (WPF) {
      for (int k = wv; k < 5 * 6; k += NS / 64) {
        const int v = k / 6, f = k - 6 * v;
        face_store<NFP>(face_sum_uniform<N, true>(f, la, lb, &sU[v * NS], ops.lm, ops.lp, sRot),
                        &face32[((e * 6 + f) * 20 + v) * NFP + lane]);
      }
    } else
    for (int q = t; q < 5 * NF; q += NS) {
      const int v = q / NF;
      int f, kk, b0, stride;
      line(q - v * NF, f, kk, b0, stride);
      const bool hi = f & 1;
      float acc = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) acc += pick_end<FR_SCALAR_ENDS32(P)>(hi, ops.lm, ops.lp, c) * sU[v * NS + b0 + c * stride];
      face_store<NFP>(acc, &face32[((e * 6 + f) * 20 + v) * NFP + kk]);
    }
  }
  float jb[9], iJb = 0;
  if (VISC && act) {
#pragma unroll
    for (int c = 0; c < 9; ++c) jb[c] = MST ? sMetall[slot][c * NS + t] : geo32_again[(e * 10 + c) * NS + t];
    iJb = MST ? sMetall[slot][9 * NS + t] : geo32_again[(e * 10 + 9) * NS + t];
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int v0 = r * VPC;
    const int nv = r < NCH ? (5 - v0 < VPC ? 5 - v0 : VPC) : 0;
    if (act) {
      if (r < 3) sM[t] = xm[r];
      if (VISC) {
#pragma unroll UNW
        for (int w = 0; w < VPC; ++w) {
          if (w < nv) {
            const int v = v0 + w;
            float d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
            for (int c = 0; c < N; ++c) {
              d0 += (OPL ? sOpf[idx[0] * N + c] : ops.D[idx[0] * N + c]) * sU[v * NS + c + N * (idx[1] + N * idx[2])];
              d1 += (OPL ? sOpf[idx[1] * N + c] : ops.D[idx[1] * N + c]) * sU[v * NS + idx[0] + N * (c + N * idx[2])];
              d2 += (OPL && !UNI2 ? sOpf[idx[2] * N + c] : ops.D[idx[2] * N + c]) * sU[v * NS + idx[0] + N * (idx[1] + N * c)];
            }
#pragma unroll
            for (int ii = 0; ii < 3; ++ii) sJ[(w * 3 + ii) * NS + t] = iJb * (jb[ii] * d0 + jb[3 + ii] * d1 + jb[6 + ii] * d2);
          }
        }
      }
    }
    __syncthreads();
    if (act && WPF) {
      for (int k = wv; k < (r < 3 ? 6 : 0) + 3 * nv * 6; k += NS / 64) {
        if (r < 3 && k < 6) {
          face_store<NFP>(face_sum_uniform<N, true>(k, la, lb, sM, opsd.lm, opsd.lp, sRotd),
                          &facem[((e * 6 + k) * 3 + r) * NFP + lane]);
          continue;
        }
        const int kg = r < 3 ? k - 6 : k;
        const int ci = kg / 6, f = kg - 6 * ci;
        const int v = v0 + ci / 3, ii = ci - (ci / 3) * 3;
        face_store<NFP>(face_sum_uniform<N, true>(f, la, lb, &sJ[ci * NS], ops.lm, ops.lp, sRot),
                        &face32[((e * 6 + f) * 20 + 5 + ii * 5 + v) * NFP + lane]);
      }
    }
    if (act && !WPF) {
      if (r < 3) {
        for (int fp = t; fp < NF; fp += NS) {
          int f, kk, b0, stride;
          line(fp, f, kk, b0, stride);
          const bool hi = f & 1;
          double acc = 0;
#pragma unroll
          for (int c = 0; c < N; ++c) acc += pick_end<FR_SCALAR_ENDS32(P)>(hi, opsd.lm, opsd.lp, c) * sM[b0 + c * stride];
          face_store<NFP>(acc, &facem[((e * 6 + f) * 3 + r) * NFP + kk]);
        }
      }
      for (int q = t; q < 3 * nv * NF; q += NS) {
        const int ci = q / NF;
        const int v = v0 + ci / 3, ii = ci - (ci / 3) * 3;
        int f, kk, b0, stride;
        line(q - ci * NF, f, kk, b0, stride);
        const bool hi = f & 1;
        float acc = 0;
#pragma unroll
        for (int c = 0; c < N; ++c) acc += pick_end<FR_SCALAR_ENDS32(P)>(hi, ops.lm, ops.lp, c) * sJ[ci * NS + b0 + c * stride];
        face_store<NFP>(acc, &face32[((e * 6 + f) * 20 + 5 + ii * 5 + v) * NFP + kk]);
      }
    }
    __syncthreads();
  }
}

template <int P, bool VISC, int EPBX, bool PRE>
__global__ __launch_bounds__(EPBX * Cfg<P>::NS) FR_WPE_ATTR(FR_WPE_VOLUME32(P)) void k_volume32(
    const double *X, const double *__restrict__ geo, const FaceRef *__restrict__ fref,
    const float *__restrict__ fout32, const double *__restrict__ foutm, int64_t E, OpsT<float> ops,
    OpsT<double> opsd, Phys<float> ph, Ref32 ref, StageArgs st, double *out0,
    double *reg1, double *reg2, float *__restrict__ face32,
    double *__restrict__ facem, const float *geo32_again) {
  volume32_body<P, VISC, EPBX, PRE>(blockIdx.x, X, geo, fref, fout32, foutm, E, ops, opsd, ph, ref, st, out0, reg1, reg2, face32, facem, geo32_again);
}

#define HIPCHK32(call)                                           \
  do {                                                           \
    hipError_t e_ = (call);                                      \
    if (e_ != hipSuccess) {                                      \
      err = std::string(#call) + ": " + hipGetErrorString(e_);   \
      return -3;                                                 \
    }                                                            \
  } while (0)

// The kernels' arguments of one mesh: its operator tables in both precisions, the physics in
// FP32 and the reference state of the split.
void ops_of(const DeviceMesh &dm, OpsT<float> &ops, OpsT<double> &opsd) {
  for (int i = 0; i < kMaxN * kMaxN; ++i) {
    ops.D[i] = float(dm.ops.D[i]);
    opsd.D[i] = dm.ops.D[i];
  }
  for (int i = 0; i < kMaxN; ++i) {
    ops.lm[i] = float(dm.ops.lm[i]);
    ops.lp[i] = float(dm.ops.lp[i]);
    ops.gcL[i] = float(dm.ops.gcL[i]);
    ops.gcR[i] = float(dm.ops.gcR[i]);
    opsd.lm[i] = dm.ops.lm[i];
    opsd.lp[i] = dm.ops.lp[i];
    opsd.gcL[i] = dm.ops.gcL[i];
    opsd.gcR[i] = dm.ops.gcR[i];
  }
}

Phys<float> phys32_of(const DeviceMesh &dm) {
  return Phys<float>{float(dm.phys.gamma), float(dm.phys.gamma - 1.0), float(dm.phys.mu), float(dm.phys.kappa)};
}

Ref32 ref32_of(const DeviceMesh &dm) {
  Ref32 ref;
  ref.rho_d = dm.ref_rho;
  ref.E_d = dm.ref_p / (dm.phys.gamma - 1.0);
  ref.H_d = (ref.E_d + dm.ref_p) / dm.ref_rho;
  ref.rho = float(ref.rho_d);
  ref.E = float(ref.E_d);
  ref.H = float(ref.H_d);
  ref.p = float(dm.ref_p);
  return ref;
}

// ------------------------------------------------------------------------------------------
// Many meshes in one launch (batches). A group holds meshes of one degree; each kernel launch
// covers every mesh of the group with one block per work item: an element block (pre-pass,
// volume) or a face block (face kernel) of some mesh. Block b finds its mesh m in the table's
// prefix sums of item counts, first[m] <= b < first[m + 1], and runs the single-mesh kernel's
// body for block b - first[m] with that mesh's arguments from a device table, so every mesh's
// results equal what the single-mesh kernels give it. The hardware's block dispatcher balances
// the items over the CUs; a block does exactly one item, as in the single-mesh kernels, so the
// bodies compile to the same register budget.
// ------------------------------------------------------------------------------------------
struct Slice32 {
  const double *X[10];  // the state stage s is evaluated on
  StageArgs st[10];     // stage s's register update (dt of this mesh)
  double *out0, *reg1, *reg2;
  const double *geo;
  const float *geo32;
  const FaceRef *fref;
  float *face32;
  double *facem;
  const double *fgeo;
  const FaceRec *ftab;
  float *fout32;
  double *foutm;
  int64_t E, F;
  Phys<float> ph;
  Ref32 ref;
  int flux;
  float tw_gm1, cw;
};

// The mesh of work item `item`: the largest m with first[m] <= item (first[0] = 0), by bisection
// (uniform over the block: the table is read by scalar loads).
__device__ __forceinline__ int slice_of(const int64_t *first, int nm, int64_t item) {
  int lo = 0, hi = nm - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= item)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <int P, bool VISC, int EPBX>
__global__ __launch_bounds__(EPBX * Cfg<P>::NS) void k_prepass32_multi(const Slice32 *__restrict__ tab,
                                                                       const int64_t *__restrict__ first, int nm,
                                                                       int s, OpsT<float> ops, OpsT<double> opsd) {
  const int m = slice_of(first, nm, blockIdx.x);
  const Slice32 &sl = tab[m];
  prepass32_body<P, VISC, EPBX>(blockIdx.x - (unsigned)first[m], sl.X[s], sl.geo32, sl.face32, sl.facem, sl.E, ops,
                                opsd, sl.ref);
}

template <int P, bool VISC, int FBS>
__global__ __launch_bounds__(FBS) void k_face32_multi(const Slice32 *__restrict__ tab,
                                                      const int64_t *__restrict__ first, int nm) {
  const int m = slice_of(first, nm, blockIdx.x);
  const Slice32 &sl = tab[m];
  face32_body<P, VISC, FBS>(blockIdx.x - (unsigned)first[m], sl.face32, sl.facem, sl.fgeo, sl.ftab, sl.F, sl.ph,
                            sl.ref, sl.flux, sl.tw_gm1, sl.cw, sl.fout32, sl.foutm);
}

template <int P, bool VISC, int EPBX, bool PRE>
__global__ __launch_bounds__(EPBX * Cfg<P>::NS) FR_WPE_ATTR(FR_WPE_VOLUME32(P)) void k_volume32_multi(
    const Slice32 *__restrict__ tab, const int64_t *__restrict__ first, int nm, int s, OpsT<float> ops,
    OpsT<double> opsd) {
  const int m = slice_of(first, nm, blockIdx.x);
  const Slice32 &sl = tab[m];
  volume32_body<P, VISC, EPBX, PRE>(blockIdx.x - (unsigned)first[m], sl.X[s], sl.geo, sl.fref, sl.fout32, sl.foutm,
                                    sl.E, ops, opsd, sl.ph, sl.ref, sl.st[s], sl.out0, sl.reg1, sl.reg2,
                                    PRE ? sl.face32 : nullptr, PRE ? sl.facem : nullptr, PRE ? sl.geo32 : nullptr);
}

template <int P, bool VISC, int EPBX, int FBS>
int launch32_t(DeviceMesh &dm, const double *X, StageArgs st, double *out0, double *reg1, double *reg2,
               double *ms, std::string &err) {
  using C = Cfg<P>;
  OpsT<float> ops;
  OpsT<double> opsd;
  ops_of(dm, ops, opsd);
  const Phys<float> ph = phys32_of(dm);
  const Ref32 ref = ref32_of(dm);
  const double tw_gm1 = dm.wall_T / (dm.phys.gamma - 1.0);
  const float cw = float(ref.rho_d * tw_gm1 - ref.E_d);
  const int64_t blocks = (dm.E + EPBX - 1) / EPBX;
  const int64_t fblocks = (dm.F * C::NFP + FBS - 1) / FBS;
  hipStream_t s = (hipStream_t)dm.stream;
  if (st.pre_only) {
    hipLaunchKernelGGL((k_prepass32<P, VISC, EPBX>), dim3((unsigned)blocks), dim3(EPBX * C::NS), 0, s, X,
                       (const float *)dm.geo32, (float *)dm.face32, (double *)dm.facem, dm.E, ops, opsd, ref);
    HIPCHK32(hipGetLastError());
    return FR_OK;
  }
  hipEvent_t ev[4];
  if (ms) {
    for (int i = 0; i < 4; ++i) HIPCHK32(hipEventCreate(&ev[i]));
    HIPCHK32(hipEventRecord(ev[0], s));
  }
  if (!st.pre_done) {
    hipLaunchKernelGGL((k_prepass32<P, VISC, EPBX>), dim3((unsigned)blocks), dim3(EPBX * C::NS), 0, s, X,
                       (const float *)dm.geo32, (float *)dm.face32, (double *)dm.facem, dm.E, ops, opsd, ref);
    HIPCHK32(hipGetLastError());
  }
  if (ms) HIPCHK32(hipEventRecord(ev[1], s));
  hipLaunchKernelGGL((k_face32<P, VISC, FBS>), dim3((unsigned)fblocks), dim3(FBS), 0, s, (const float *)dm.face32,
                     (const double *)dm.facem, (const double *)dm.fgeo, dm.ftab, dm.F, ph, ref, dm.flux,
                     float(tw_gm1), cw, (float *)dm.fout32, (double *)dm.foutm);
  HIPCHK32(hipGetLastError());
  if (ms) HIPCHK32(hipEventRecord(ev[2], s));
  if (st.pre_next) {
    hipLaunchKernelGGL((k_volume32<P, VISC, EPBX, true>), dim3((unsigned)blocks), dim3(EPBX * C::NS), 0, s, X,
                       (const double *)dm.geo, dm.fref, (const float *)dm.fout32, (const double *)dm.foutm, dm.E, ops,
                       opsd, ph, ref, st, out0, reg1, reg2, (float *)dm.face32, (double *)dm.facem,
                       (const float *)dm.geo32);
  } else {
    hipLaunchKernelGGL((k_volume32<P, VISC, EPBX, false>), dim3((unsigned)blocks), dim3(EPBX * C::NS), 0, s, X,
                       (const double *)dm.geo, dm.fref, (const float *)dm.fout32, (const double *)dm.foutm, dm.E, ops,
                       opsd, ph, ref, st, out0, reg1, reg2, (float *)nullptr, (double *)nullptr,
                       (const float *)nullptr);
  }
  HIPCHK32(hipGetLastError());
  if (ms) {
    HIPCHK32(hipEventRecord(ev[3], s));
    HIPCHK32(hipEventSynchronize(ev[3]));
    float tms[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i) HIPCHK32(hipEventElapsedTime(&tms[i], ev[i], ev[i + 1]));
    // run_steps' timing slots: [0] pre-pass, [1] face, [2] volume alone, [4] pre-pass launches,
    // [5] / [6] volume with the next pre-pass (ms, launches)
    ms[0] += tms[0];
    ms[1] += tms[1];
    if (!st.pre_done) ms[4] += 1;
    if (st.pre_next) {
      ms[5] += tms[2];
      ms[6] += 1;
    } else {
      ms[2] += tms[2];
    }
    for (int i = 0; i < 4; ++i) (void)hipEventDestroy(ev[i]);
  }
  return 0;
}

// The tile shapes, as for the FP64 kernels: elements per block Cfg::EPB or Cfg::EPB2
// (DeviceMesh::tile_epb 0 / 1) and a face block of 256, 128 or 64 threads (tile_fbs 0 / 1 / 2).
template <int P, bool VISC>
int launch32_tiles(DeviceMesh &dm, const double *X, StageArgs st, double *o, double *r1, double *r2, double *ms,
                   std::string &err) {
  constexpr int E0 = Cfg<P>::EPB, E1 = Cfg<P>::EPB2;
  if (dm.tile_epb == 0) {
    if (dm.tile_fbs == 0) return launch32_t<P, VISC, E0, 256>(dm, X, st, o, r1, r2, ms, err);
    if (dm.tile_fbs == 1) return launch32_t<P, VISC, E0, 128>(dm, X, st, o, r1, r2, ms, err);
    return launch32_t<P, VISC, E0, 64>(dm, X, st, o, r1, r2, ms, err);
  }
  if (dm.tile_fbs == 0) return launch32_t<P, VISC, E1, 256>(dm, X, st, o, r1, r2, ms, err);
  if (dm.tile_fbs == 1) return launch32_t<P, VISC, E1, 128>(dm, X, st, o, r1, r2, ms, err);
  return launch32_t<P, VISC, E1, 64>(dm, X, st, o, r1, r2, ms, err);
}

template <bool VISC>
int launch32_p(DeviceMesh &dm, const double *X, StageArgs st, double *o, double *r1, double *r2, double *ms,
               std::string &err) {
  switch (dm.p) {
    case 0: return launch32_tiles<0, VISC>(dm, X, st, o, r1, r2, ms, err);
    case 1: return launch32_tiles<1, VISC>(dm, X, st, o, r1, r2, ms, err);
    case 2: return launch32_tiles<2, VISC>(dm, X, st, o, r1, r2, ms, err);
    case 3: return launch32_tiles<3, VISC>(dm, X, st, o, r1, r2, ms, err);
    case 4: return launch32_tiles<4, VISC>(dm, X, st, o, r1, r2, ms, err);
    case 5: return launch32_tiles<5, VISC>(dm, X, st, o, r1, r2, ms, err);
    case 6: return launch32_tiles<6, VISC>(dm, X, st, o, r1, r2, ms, err);
    case 7: return launch32_tiles<7, VISC>(dm, X, st, o, r1, r2, ms, err);
    default: err = "p out of range"; return -5;
  }
}

// A group's device tables and item counts (see Slice32).
struct Group32Impl {
  int p = 0, ns = 0, epb = 0, fbs = 0, nm = 0;
  bool fuse = true;
  Slice32 *tab = nullptr;
  int64_t *first_e = nullptr, *first_f = nullptr;
  OpsT<float> ops;
  OpsT<double> opsd;
  int64_t items_e = 0, items_f = 0;
};

// setup: check that the item counts fit a launch; otherwise enqueue `steps` RK steps of every mesh
// of the group. With fusion every stage but the first finds its pre-pass done by the previous
// stage's volume kernel, across step boundaries too, as fr_rk_step's run of steps does.
template <int P, int EPB, int FBS>
int group32_t(Group32Impl &g, hipStream_t s, bool setup, int steps, std::string &err) {
  constexpr int TB = EPB * Cfg<P>::NS;
  if (setup) {
    if (g.items_e * TB > (int64_t)UINT32_MAX || g.items_f * FBS > (int64_t)UINT32_MAX) {
      err = "a mesh group's launch exceeds 2^32 threads";
      return -1;
    }
    return 0;
  }
  const dim3 ge((unsigned)g.items_e), gf((unsigned)g.items_f);
  for (int step = 0; step < steps; ++step) {
    for (int st = 0; st < g.ns; ++st) {
      const bool first = step == 0 && st == 0, last = step == steps - 1 && st == g.ns - 1;
      if (first || !g.fuse) {
        hipLaunchKernelGGL((k_prepass32_multi<P, true, EPB>), ge, dim3(TB), 0, s, g.tab, g.first_e, g.nm, st,
                           g.ops, g.opsd);
        HIPCHK32(hipGetLastError());
      }
      hipLaunchKernelGGL((k_face32_multi<P, true, FBS>), gf, dim3(FBS), 0, s, g.tab, g.first_f, g.nm);
      HIPCHK32(hipGetLastError());
      if (g.fuse && !last)
        hipLaunchKernelGGL((k_volume32_multi<P, true, EPB, true>), ge, dim3(TB), 0, s, g.tab, g.first_e, g.nm, st,
                           g.ops, g.opsd);
      else
        hipLaunchKernelGGL((k_volume32_multi<P, true, EPB, false>), ge, dim3(TB), 0, s, g.tab, g.first_e, g.nm, st,
                           g.ops, g.opsd);
      HIPCHK32(hipGetLastError());
    }
  }
  return 0;
}

template <int P>
int group32_tiles(Group32Impl &g, hipStream_t s, bool setup, int steps, std::string &err) {
  constexpr int E0 = Cfg<P>::EPB, E1 = Cfg<P>::EPB2;
  if (g.epb == 0) {
    if (g.fbs == 0) return group32_t<P, E0, 256>(g, s, setup, steps, err);
    if (g.fbs == 1) return group32_t<P, E0, 128>(g, s, setup, steps, err);
    return group32_t<P, E0, 64>(g, s, setup, steps, err);
  }
  if (g.fbs == 0) return group32_t<P, E1, 256>(g, s, setup, steps, err);
  if (g.fbs == 1) return group32_t<P, E1, 128>(g, s, setup, steps, err);
  return group32_t<P, E1, 64>(g, s, setup, steps, err);
}

int group32_dispatch(Group32Impl &g, hipStream_t s, bool setup, int steps, std::string &err) {
  switch (g.p) {
    case 1: return group32_tiles<1>(g, s, setup, steps, err);
    case 2: return group32_tiles<2>(g, s, setup, steps, err);
    case 3: return group32_tiles<3>(g, s, setup, steps, err);
    case 4: return group32_tiles<4>(g, s, setup, steps, err);
    case 5: return group32_tiles<5>(g, s, setup, steps, err);
    case 6: return group32_tiles<6>(g, s, setup, steps, err);
    case 7: return group32_tiles<7>(g, s, setup, steps, err);
    default: err = "multi-mesh groups take p = 1..7"; return -5;
  }
}

void free_group32(Group32Impl *g) {
  for (void *b : {(void *)g->tab, (void *)g->first_e, (void *)g->first_f})
    if (b) (void)hipFree(b);
  delete g;
}

}  // namespace

namespace frk {
// Enqueue one stage of the FP32 form; returns 0 or a negative FR_ERR_* code with `err` set.
// StageArgs::pre_done skips the stand-alone pre-pass and StageArgs::pre_next makes the volume
// kernel run the next stage's, as in the FP64 path; ms, when given, accumulates run_steps'
// timing slots.
int launch_stage32(DeviceMesh &dm, const double *X, StageArgs st, double *o, double *r1, double *r2, double *ms,
                   std::string &err) {
  return dm.viscous ? launch32_p<true>(dm, X, st, o, r1, r2, ms, err) : launch32_p<false>(dm, X, st, o, r1, r2, ms, err);
}

bool group32_eligible(const DeviceMesh &dm) {
  return dm.prec == 1 && dm.viscous && !dm.ldg && dm.sgs == 0 && dm.p >= 1 && dm.p <= kMaxP;
}

int group32_create(const std::vector<DeviceMesh *> &meshes, const std::vector<double> &dt, int scheme, Group32 **out,
                   std::string &err) {
  *out = nullptr;
  const int nm = (int)meshes.size();
  if (nm < 1) {
    err = "empty group";
    return -1;
  }
  Group32Impl *g = new Group32Impl();
  g->p = meshes[0]->p;
  g->nm = nm;
  g->ns = n_stages(scheme);
  g->fuse = meshes[0]->fuse;
  ops_of(*meshes[0], g->ops, g->opsd);
  // the tiles of the group's meshes (one setting per group)
  g->epb = meshes[0]->tile_epb;
  g->fbs = meshes[0]->tile_fbs;
  const int NFP = meshes[0]->Nfp;
  const int epb = tile_elements(meshes[0]->Ns, g->epb);
  const int fbs = g->fbs == 0 ? 256 : (g->fbs == 1 ? 128 : 64);
  std::vector<Slice32> tab(nm);
  std::vector<int64_t> fe(nm + 1, 0), ff(nm + 1, 0);
  for (int i = 0; i < nm; ++i) {
    DeviceMesh &dm = *meshes[i];
    if (dm.p != g->p || !group32_eligible(dm) || dm.fuse != g->fuse || dm.tile_epb != g->epb || dm.tile_fbs != g->fbs) {
      free_group32(g);
      err = "meshes of a group need one degree, the viscous FP32 form without closure or LDG, one fusion setting "
            "and one tile setting";
      return -1;
    }
    Slice32 &sl = tab[i];
    std::memset(&sl, 0, sizeof sl);
    for (int st = 0; st < g->ns; ++st) {
      const double *X;
      double *o, *r1, *r2;
      stage_setup(dm, scheme, st, dt[i], sl.st[st], &X, &o, &r1, &r2);
      sl.st[st].force = dm.has_force ? 1 : 0;
      for (int k = 0; k < 3; ++k) sl.st[st].g[k] = dm.force[k];
      sl.X[st] = X;
      sl.out0 = o;
      sl.reg1 = r1;
      sl.reg2 = r2;
    }
    sl.geo = (const double *)dm.geo;
    sl.geo32 = (const float *)dm.geo32;
    sl.fref = dm.fref;
    sl.face32 = (float *)dm.face32;
    sl.facem = (double *)dm.facem;
    sl.fgeo = (const double *)dm.fgeo;
    sl.ftab = dm.ftab;
    sl.fout32 = (float *)dm.fout32;
    sl.foutm = (double *)dm.foutm;
    sl.E = dm.E;
    sl.F = dm.F;
    sl.ph = phys32_of(dm);
    sl.ref = ref32_of(dm);
    sl.flux = dm.flux;
    const double tw_gm1 = dm.wall_T / (dm.phys.gamma - 1.0);
    sl.tw_gm1 = float(tw_gm1);
    sl.cw = float(sl.ref.rho_d * tw_gm1 - sl.ref.E_d);
    fe[i + 1] = fe[i] + (dm.E + epb - 1) / epb;
    ff[i + 1] = ff[i] + (dm.F * NFP + fbs - 1) / fbs;
  }
  g->items_e = fe[nm];
  g->items_f = ff[nm];
  if (hipMalloc(&g->tab, nm * sizeof(Slice32)) != hipSuccess ||
      hipMalloc(&g->first_e, (nm + 1) * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&g->first_f, (nm + 1) * sizeof(int64_t)) != hipSuccess ||
      hipMemcpy(g->tab, tab.data(), nm * sizeof(Slice32), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(g->first_e, fe.data(), (nm + 1) * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(g->first_f, ff.data(), (nm + 1) * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess) {
    free_group32(g);
    err = "device tables of a mesh group";
    return -4;
  }
  int rc = group32_dispatch(*g, nullptr, true, 0, err);
  if (rc) {
    free_group32(g);
    return rc;
  }
  *out = reinterpret_cast<Group32 *>(g);
  return 0;
}

int group32_step(Group32 *g, void *stream, int steps, std::string &err) {
  return group32_dispatch(*reinterpret_cast<Group32Impl *>(g), (hipStream_t)stream, false, steps, err);
}

void group32_destroy(Group32 *g) {
  if (g) free_group32(reinterpret_cast<Group32Impl *>(g));
}

int group32_items(const Group32 *g, int64_t *elem_items, int64_t *face_items) {
  const Group32Impl *gi = reinterpret_cast<const Group32Impl *>(g);
  *elem_items = gi->items_e;
  *face_items = gi->items_f;
  return 0;
}
}  // namespace frk
