// fr_device.h -- device-side building blocks shared by the FP64 and FP32 kernels of libfr:
// the physical and numerical fluxes of the compressible Navier-Stokes equations (the paper's
// section "FR Algorithm", Eq. (1) and the interface Riemann solver), the launch configuration
// per polynomial degree and the 1-D operator tables passed to the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "fr_internal.h"

using namespace frk;

// ------------------------------------------------------------------------------------------
// Device physics (Eq. (1)): inviscid flux, viscous flux with constant mu, Riemann solvers.
// ------------------------------------------------------------------------------------------
template <typename real>
struct Phys {
  real gamma, gm1, mu, kappa;
};

template <typename real>
__device__ __forceinline__ real pressure(const real U[5], real gm1) {
  const real ir = real(1) / U[0];
  return gm1 * (U[4] - real(0.5) * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) * ir);
}

// Inviscid flux along a unit or scaled direction n: F(U).n, plus u.n and c.
template <typename real>
__device__ __forceinline__ void flux_n(const real U[5], const real n[3], const Phys<real> &ph, real F[5],
                                       real &un, real &c) {
  const real ir = real(1) / U[0];
  const real u = U[1] * ir, v = U[2] * ir, w = U[3] * ir;
  const real p = ph.gm1 * (U[4] - real(0.5) * U[0] * (u * u + v * v + w * w));
  un = u * n[0] + v * n[1] + w * n[2];
  F[0] = U[0] * un;
  F[1] = U[1] * un + p * n[0];
  F[2] = U[2] * un + p * n[1];
  F[3] = U[3] * un + p * n[2];
  F[4] = (U[4] + p) * un;
  c = sqrt(ph.gamma * p * ir);
}

template <typename real>
__device__ __forceinline__ void rusanov(const real UL[5], const real UR[5], const real n[3], const Phys<real> &ph,
                                        real F[5]) {
  real FL[5], FR[5], unL, unR, cL, cR;
  flux_n(UL, n, ph, FL, unL, cL);
  flux_n(UR, n, ph, FR, unR, cR);
  const real lam = fmax(fabs(unL) + cL, fabs(unR) + cR);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] = real(0.5) * (FL[v] + FR[v]) - real(0.5) * lam * (UR[v] - UL[v]);
}

// Roe: mean flux minus half of sum |lambda_k| alpha_k r_k; sqrt(rho) averages; no entropy fix.
template <typename real>
__device__ __forceinline__ void roe(const real UL[5], const real UR[5], const real n[3], const Phys<real> &ph,
                                    real F[5]) {
  real FL[5], FR[5], t0, t1;
  flux_n(UL, n, ph, FL, t0, t1);
  flux_n(UR, n, ph, FR, t0, t1);
  const real rL = UL[0], rR = UR[0];
  const real iL = real(1) / rL, iR = real(1) / rR;
  const real uL[3] = {UL[1] * iL, UL[2] * iL, UL[3] * iL};
  const real uR[3] = {UR[1] * iR, UR[2] * iR, UR[3] * iR};
  const real pL = ph.gm1 * (UL[4] - real(0.5) * rL * (uL[0] * uL[0] + uL[1] * uL[1] + uL[2] * uL[2]));
  const real pR = ph.gm1 * (UR[4] - real(0.5) * rR * (uR[0] * uR[0] + uR[1] * uR[1] + uR[2] * uR[2]));
  const real HL = (UL[4] + pL) * iL, HR = (UR[4] + pR) * iR;
  const real sL = sqrt(rL), sR = sqrt(rR);
  const real is = real(1) / (sL + sR);
  const real rt = sL * sR;
  real ut[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) ut[i] = (sL * uL[i] + sR * uR[i]) * is;
  const real Ht = (sL * HL + sR * HR) * is;
  const real q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
  const real c2 = ph.gm1 * (Ht - real(0.5) * q2);
  const real ct = sqrt(c2);
  const real ic2 = real(1) / c2;
  const real unt = ut[0] * n[0] + ut[1] * n[1] + ut[2] * n[2];
  const real dr = rR - rL, dp = pR - pL;
  const real du[3] = {uR[0] - uL[0], uR[1] - uL[1], uR[2] - uL[2]};
  const real dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
  const real a1 = real(0.5) * (dp - rt * ct * dun) * ic2;
  const real a5 = real(0.5) * (dp + rt * ct * dun) * ic2;
  const real a2 = dr - dp * ic2;
  const real l1 = fabs(unt - ct), l2 = fabs(unt), l5 = fabs(unt + ct);
  const real w1 = l1 * a1, w5 = l5 * a5, w2 = l2 * a2;
  real dis[5];
  dis[0] = w1 + w5 + w2;
  real udu = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const real sh = du[i] - dun * n[i];
    dis[1 + i] = w1 * (ut[i] - ct * n[i]) + w5 * (ut[i] + ct * n[i]) + w2 * ut[i] + l2 * rt * sh;
    udu += ut[i] * sh;
  }
  dis[4] = w1 * (Ht - unt * ct) + w5 * (Ht + unt * ct) + w2 * real(0.5) * q2 + l2 * rt * udu;
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] = real(0.5) * (FL[v] + FR[v]) - real(0.5) * dis[v];
}

// Viscous flux Fv[i][v] from U and the gradient of the conserved variables G[i][v], with
// dynamic viscosity mu and heat-flux coefficient kappa (on d(p/rho)).
template <typename real>
__device__ __forceinline__ void visc_flux_mk(const real U[5], const real G[3][5], real gm1, real mu, real kappa,
                                             real Fv[3][5]) {
  const real ir = real(1) / U[0];
  const real u[3] = {U[1] * ir, U[2] * ir, U[3] * ir};
  const real e = U[4] * ir;
  real du[3][3], dT[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) du[i][j] = (G[i][1 + j] - u[j] * G[i][0]) * ir;
    const real de = (G[i][4] - e * G[i][0]) * ir;
    dT[i] = gm1 * (de - (u[0] * du[i][0] + u[1] * du[i][1] + u[2] * du[i][2]));
  }
  const real lam = real(-2.0 / 3.0) * mu * (du[0][0] + du[1][1] + du[2][2]);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    real tau[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) tau[j] = mu * (du[j][i] + du[i][j]) + (i == j ? lam : real(0));
    Fv[i][0] = 0;
    Fv[i][1] = tau[0];
    Fv[i][2] = tau[1];
    Fv[i][3] = tau[2];
    Fv[i][4] = tau[0] * u[0] + tau[1] * u[1] + tau[2] * u[2] + kappa * dT[i];
  }
}

template <typename real>
__device__ __forceinline__ void visc_flux(const real U[5], const real G[3][5], const Phys<real> &ph, real Fv[3][5]) {
  visc_flux_mk(U, G, ph.gm1, ph.mu, ph.kappa, Fv);
}

// ------------------------------------------------------------------------------------------
// Fused epilogue of the volume kernels: the source term and the RK register update of one
// point, in double precision.
// ------------------------------------------------------------------------------------------

// Body force g per unit mass (the source term S of Eq. (3)): component v of
// (0, rho g, m . g) from the point's state X.
__device__ __forceinline__ double body_force(const StageArgs &st, const double X[5], int v) {
  if (!st.force || v == 0) return 0.0;
  if (v < 4) return X[0] * st.g[v - 1];
  return X[1] * st.g[0] + X[2] * st.g[1] + X[3] * st.g[2];
}

// x: the state the stage was evaluated on; R: its residual; r1, r2: the registers' old values.
//   LSRK45:   dU <- a dU + dt R; U <- x + b dU                       (out0 = U, reg1 = dU)
//   RK4:      acc <- acc + w R; S <- Q + c dt R, or at the last stage Q <- Q + dt acc
//                                                (out0 = Q, reg1 = acc, reg2 = S)
//   SSP(10,4) (out0 = q1 = U, reg1 = q2): stages 0-3 and 5-8 take a forward-Euler step
//             q1 <- q1 + dt/6 R (stage 0 also sets q2 <- q1); stage 4 then combines
//             q2 <- q2/25 + 9/25 q1, q1 <- 15 q2 - 5 q1; stage 9 sets q1 <- q2 + 3/5 q1 + dt/10 R.
// Returns the value of the state the next stage is evaluated on (RK4: S, or Q after the last
// stage; the others: U), which the volume kernel's fused pre-pass of the next stage uses.
__device__ __forceinline__ double rk_store(const StageArgs &st, int64_t o, double x, double R, double r1,
                                           double r2, double *out0, double *reg1, double *reg2) {
  if (st.mode == kModeResidual) {
    out0[o] = R;
    return 0.0;
  }
  if (st.mode == kModeLSRK) {
    const double du = st.a * r1 + st.dt * R;
    const double u = x + st.b * du;
    reg1[o] = du;
    out0[o] = u;
    return u;
  }
  if (st.mode == kModeRK4) {
    const double acc = r1 + st.w * R;
    if (!st.last) {
      const double sn = r2 + st.cdt * R;
      reg1[o] = acc;
      reg2[o] = sn;
      return sn;
    }
    const double q = r2 + st.dt * acc;
    out0[o] = q;
    return q;
  }
  if (st.stage == 9) {
    const double q = r1 + 0.6 * x + st.dt / 10 * R;
    out0[o] = q;
    return q;
  }
  const double q1 = x + st.dt / 6 * R;
  if (st.stage == 4) {
    const double q2 = r1 / 25 + 9.0 / 25 * q1;
    const double q = 15 * q2 - 5 * q1;
    reg1[o] = q2;
    out0[o] = q;
    return q;
  }
  if (st.stage == 0) reg1[o] = x;
  out0[o] = q1;
  return q1;
}

// ------------------------------------------------------------------------------------------
// Kernel configuration
// ------------------------------------------------------------------------------------------
template <int P>
struct Cfg {
  static constexpr int N = P + 1;
  static constexpr int NS = N * N * N;
  static constexpr int NFP = N * N;
  static constexpr int NF = 6 * NFP;
  static constexpr int EPB = (256 / NS) > 64 ? 64 : ((256 / NS) > 0 ? (256 / NS) : 1);  // elements per block
  static constexpr int BLOCK = EPB * NS;
  // the second tile choice: half of EPB; where EPB is one element whose points do not fill
  // whole waves (p = 5: 216 points in 4 waves, p = 6: 343 in 6), two elements per block, which
  // fill 7 and 11 waves
  static constexpr int EPB2 = EPB > 1 ? EPB / 2 : (NS % 64 != 0 && 2 * NS <= 1024 ? 2 : 1);
};

// Occupancy targets (waves per SIMD) per kernel and degree; 0 lets the compiler decide.
// The volume kernel without the closure asks for 4 at p = 3 and p = 7. At p = 3 the compiler's
// own choice is 130 VGPRs (3 waves) and 128 fit without spilling (the kernel 7.5% faster at
// 64^3); with the fused pre-pass (PRE) both degrees spill a few bytes per lane at 4 waves and
// are still faster than at the compiler's 2-3 waves (measured at 64^3 p=3 and 32^3 p=7).
// Elsewhere forcing more waves than the compiler picks spilled more and ran slower.
#ifndef FR_WPE_PREPASS
#define FR_WPE_PREPASS(P) 0
#endif
#ifndef FR_WPE_FACE
#define FR_WPE_FACE(P) 0
#endif
#ifndef FR_WPE_VOLUME
#define FR_WPE_VOLUME(P, SGS, PRE) (((P) == 3 || (P) == 7) && !(SGS) ? 4 : 0)
#endif
// The FP32 form's volume kernel asks for 4 at p = 5 and p = 7. At p = 7 the compiler's choice
// is 130 VGPRs and 128 fit without spill; at p = 5 it is 132 (3 waves), and at 128 the fused
// instance spills 4 bytes per lane and runs 10% faster (43^3 p=5: 2.23 -> 1.99 ms, same box).
// At p = 2 and 4 the compiler already picks 4; the FP64 kernels at p = 4 and 5 lost 1-5% at 4.
#ifndef FR_WPE_VOLUME32
#define FR_WPE_VOLUME32(P) ((P) == 5 || (P) == 7 ? 4 : 0)
#endif
// How a single-pass fused tail spreads the face values over its threads. FP32 form: whole face
// points per thread (each point's line and interpolation weights worked out once for all its
// values) at the degrees listed, else (group, face point) items of five sums. FP64: items of
// FR_TAIL_GROUPS64 of the four groups (4: whole face points). Measured per degree (A/B in one
// call): whole points are faster at p = 2 (FP32 +13%, FP64 +5%; taken for p = 0, 1 too, where
// the points also divide evenly over the threads), p = 4 (+1%, +2%) and at p = 5, 6 in the FP32
// form (+3%, +1%), slower at p = 3 in FP64 (-10%; items of two groups were no faster than one,
// 5.78-5.85e9 against 5.80-5.82e9, nor whole points after the operator reads moved to LDS and
// scalar loads, 5.87e9 against 5.92e9) and at p = 5 in FP64 (-1%). In the FP32 form at p = 3
// whole points were 2% slower at first and 6% faster after those changes (7.89e9 -> 8.36e9).
#ifndef FR_TAIL_GROUPS64
#define FR_TAIL_GROUPS64(P) ((P) <= 2 || (P) == 4 ? 4 : 1)
#endif
#ifndef FR_TAIL_PER_POINT32
#define FR_TAIL_PER_POINT32(P) ((P) <= 6)
#endif
// Degrees at which the kernels make that choice from scalar loads (pick_end); elsewhere the
// compiler's vector load of a selected address stays. Measured per degree (A/B in one call):
// FP64 64^3 p=3 +1-2%, 52^3 p=4 +2.5%, 43^3 p=5 +4%, while at 80^3 p=2 the fused volume kernel
// went from 1.99 to 2.09 ms and at 37^3 p=6 it took 130 VGPRs (a wave per SIMD less); FP32 form
// 64^3 p=3 +3%, 52^3 p=4 +12%, 43^3 p=5 +11%, 37^3 p=6 +8%, 80^3 p=2 -3%. At p = 7 the choice
// is made per wave (no difference).
#ifndef FR_SCALAR_ENDS64
#define FR_SCALAR_ENDS64(P) ((P) == 3 || (P) == 4 || (P) == 5)
#endif
#ifndef FR_SCALAR_ENDS32
#define FR_SCALAR_ENDS32(P) ((P) >= 3)
#endif
#define FR_WPE_ATTR(w) __attribute__((amdgpu_waves_per_eu((w) > 0 ? (w) : 1, (w) > 0 ? 8 : 8)))

// Whether `extra` more bytes of LDS per block leave the blocks a CU can hold unchanged: a block
// of `threads` threads using `bytes` of the CU's 160 KB (and at most 32 waves per CU).
constexpr int lds_blocks(int bytes, int threads) {
  const int by_lds = (160 * 1024) / bytes, by_waves = 32 / ((threads + 63) / 64);
  return by_lds < by_waves ? by_lds : by_waves;
}
constexpr bool lds_copy_fits(int bytes, int extra, int threads) {
  return lds_blocks(bytes + extra, threads) == lds_blocks(bytes, threads);
}

// An operator entry at a uniform index, chosen per lane between two tables (the interpolation
// to the face at -1 or at +1). As a select of the two values the compiler makes it one vector
// load from a selected address, and a vector load completes only after every vector memory
// access the wave issued before it (the RK-register loads, the stores of earlier face points).
// Passing both through readfirstlane keeps them scalar loads and the choice a register select.
template <typename T>
__device__ __forceinline__ T uniform_value(T x) {
  if constexpr (sizeof(T) == 8) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = __builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
  }
}
template <bool SCALAR, typename T>
__device__ __forceinline__ T pick_end(bool hi, const T *lm, const T *lp, int c) {
  if constexpr (SCALAR) return hi ? uniform_value(lp[c]) : uniform_value(lm[c]);
  else return hi ? lp[c] : lm[c];
}

template <typename real>
struct OpsT {
  real D[kMaxN * kMaxN];
  real lm[kMaxN];
  real lp[kMaxN];
  real gcL[kMaxN];
  real gcR[kMaxN];
};

// Stores to the per-face-point buffers, which are written once and read once by the next
// kernel, as runs of NFP entries per value. They are non-temporal (+2.8% per stage at 64^3
// p=3) except where a run is shorter than a 128-byte line and does not divide it (doubles at
// p = 2, floats at p = 2 and 4): there consecutive runs share lines, and plain stores let L2
// merge the pieces (the p = 2 pre-pass 3.56 -> 1.52 ms at 80^3).
template <int NFP, typename T>
__device__ __forceinline__ void face_store(T v, T *p) {
  constexpr int run = NFP * (int)sizeof(T);
  if constexpr (run >= 128 || 128 % run == 0) {
    __builtin_nontemporal_store(v, p);
  } else {
    *p = v;
  }
}

// A thread's point index along xi_2 within its element. With one element per block and N*N = 64
// points per xi_2-plane (p = 7), each wavefront covers exactly one plane, so the index is the same
// on every lane; saying so lets the compiler keep the operator row D[i2][.] in scalar registers.
template <int N, int EPB>
__device__ __forceinline__ int plane_index(int t) {
  if constexpr (N * N == 64 && EPB == 1) return __builtin_amdgcn_readfirstlane(t / (N * N));
  else return t / (N * N);
}

// Face interpolation of a point-ordered element array src: the sum over the line normal to
// face f (direction d = f/2) through its face point (a, b) of ell[c] src[line_pt(d, c, a, b)],
// with ell = l(-1) or l(+1) by the face's side. f must be the same on every lane of the
// wavefront (the p = 7 kernels give each wavefront one face of 64 points): the direction then
// picks one of three loops whose LDS strides are constants.
// * In ascending c (ROT false, and faces normal to xi_2 always) ell is read through scalar
//   loads. On faces normal to xi_0 and xi_1 the lines' common stride (8 or 64 entries) then puts
//   8 lanes of a wavefront on one LDS bank at every step (16 for doubles): an 8-way conflict.
// * With ROT, a lane of a face normal to xi_0 reads its whole line (contiguous) with 16-byte
//   loads, two for floats and four for doubles, and sums it in ascending c; src must then be
//   16-byte aligned. On faces normal to xi_1 lane (a, b) starts at c = b and wraps around
//   (mod 8): every step then reads 64 different banks for floats, and 32 different 8-byte bank
//   pairs per half-wavefront for doubles. The weights of the rotated order come from rot, an
//   LDS table [l(-1), l(-1), l(+1), l(+1)] (rot_entry) where they are contiguous.
// A form's kernels all take the same ROT, so fused and separate stages keep the same sums. The
// FP32 form's p = 7 kernels take it (32^3: the pre-pass, at 6.5 conflict cycles per LDS
// instruction, went from 0.66 to 0.56 ms); the FP64 ones do not: there the rotated sums cost
// the fused volume kernel more than they saved (1.74 -> 1.80 ms), and their table would cost
// the pre-pass, whose two blocks fill the LDS exactly, one of them.
template <int N, typename C>
__device__ __forceinline__ C rot_entry(const C *lm, const C *lp, int i) {
  return i < 2 * N ? lm[i % N] : lp[i % N];
}
template <int N, bool ROT = false, typename T, typename C>
__device__ __forceinline__ T face_sum_uniform(int f, int a, int b, const T *src, const C *lm, const C *lp,
                                              const C *rot = nullptr) {
  constexpr bool R = ROT && N == 8;  // the rotation is worked out for lines of eight points
  const C *ell = (f & 1) ? lp : lm;
  const int d = f >> 1;
  T acc = 0;
  if (R && d == 0) {
    constexpr int K = 16 / (int)sizeof(T);
    using V = T __attribute__((ext_vector_type(K)));
    const V *q = reinterpret_cast<const V *>(src + N * (a + N * b));
#pragma unroll
    for (int j = 0; j < N / K; ++j) {
      const V x = q[j];
#pragma unroll
      for (int k = 0; k < K; ++k) acc += ell[j * K + k] * x[k];
    }
  } else if (R && d == 1) {
    const int r = b & (N - 1);
    const C *w = rot + ((f & 1) ? 2 * N : 0) + r;
    const T *q = src + a + N * N * b;
#pragma unroll
    for (int s = 0; s < N; ++s) acc += w[s] * q[((s + r) & (N - 1)) * N];
  } else if (d == 0) {
    const T *q = src + N * (a + N * b);
#pragma unroll
    for (int c = 0; c < N; ++c) acc += ell[c] * q[c];
  } else if (d == 1) {
    const T *q = src + a + N * N * b;
#pragma unroll
    for (int c = 0; c < N; ++c) acc += ell[c] * q[c * N];
  } else {
    const T *q = src + a + N * b;
#pragma unroll
    for (int c = 0; c < N; ++c) acc += ell[c] * q[c * N * N];
  }
  return acc;
}

// One wavefront per face of the element (64 face points, one per lane): p = 7 with one element
// per block, where the kernels take their face loops as wave-uniform (value, face) tasks.
template <int NFP, int EPB>
constexpr bool kWavePerFace = NFP == 64 && EPB == 1;

// index of solution point with coordinate c along direction d and (a, b) along the face's
// tangential directions (increasing axis order)
template <int N>
__device__ __forceinline__ int line_pt(int d, int c, int a, int b) {
  return d == 0 ? c + N * (a + N * b) : (d == 1 ? a + N * (c + N * b) : a + N * (b + N * c));
}

