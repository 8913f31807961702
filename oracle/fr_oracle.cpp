// fr_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow CPU reference for the flux-reconstruction (FR) residual of the 3-D
// compressible Navier-Stokes equations on hexahedral meshes and for the Runge-Kutta update,
// written directly from the paper's statement of the method (section "FR Algorithm",
// Eqs. (1)-(3)) and the readings listed with each function below. It shares no code with the
// HIP library: it has its own basis, face matching, metrics, fluxes and time stepping. Only
// the tests, the smoke check and the bench's CPU-baseline leg may load it.
//
// Everything is templated on the scalar type so that a `long double` build measures the
// rounding floor of the `double` result. Loops are plain: tensor-product operators are
// applied one reference direction at a time, which is the definition of a tensor-product
// interpolant, and there is no other blocking, fusion or reordering.
//
// Parity status: every function here is pinned by tests under tests/ (see the pin list in
// the test files); nothing is "parity unpinned".

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <memory>
#include <string>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using std::vector;

// ---------------------------------------------------------------------------------------------
// 1-D polynomial basis (section "FR Algorithm", Eq. (2): nodal Lagrange representation).
// ---------------------------------------------------------------------------------------------

// Legendre polynomial P_n(x) and its derivative by the three-term recurrence.
template <class T>
void legendre(int n, T x, T &P, T &dP) {
  T p0 = 1, p1 = x;
  if (n == 0) { P = 1; dP = 0; return; }
  for (int k = 2; k <= n; ++k) {
    T p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  // (1 - x^2) P_n' = n (P_{n-1} - x P_n); at x = +-1 use P_n'(+-1) = (+-1)^{n+1} n(n+1)/2.
  if (x == T(1) || x == T(-1)) {
    T s = (x > 0 || (n % 2 == 1)) ? T(1) : T(-1);
    dP = s * T(n) * T(n + 1) / 2;
  } else {
    dP = T(n) * (p0 - x * p1) / (1 - x * x);
  }
}

template <class T>
T pi_t() { return T(3.14159265358979323846264338327950288L); }

// Gauss-Legendre points (roots of P_n) and weights, ascending. Newton from a cosine guess.
template <class T>
void gauss_legendre(int n, vector<T> &x, vector<T> &w) {
  x.assign(n, 0);
  w.assign(n, 0);
  for (int k = 0; k < n; ++k) {
    T r = -std::cos(pi_t<T>() * (T(k) + T(0.75)) / (T(n) + T(0.5)));
    for (int it = 0; it < 100; ++it) {
      T P, dP;
      legendre<T>(n, r, P, dP);
      T dr = P / dP;
      r -= dr;
      if (std::fabs(dr) < T(1e-3) * std::numeric_limits<T>::epsilon()) break;
    }
    T P, dP;
    legendre<T>(n, r, P, dP);
    x[k] = r;
    w[k] = T(2) / ((1 - r * r) * dP * dP);
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return x[a] < x[b]; });
  vector<T> xs(n), ws(n);
  for (int i = 0; i < n; ++i) { xs[i] = x[idx[i]]; ws[i] = w[idx[i]]; }
  x = xs;
  w = ws;
}

// Gauss-Lobatto-Legendre points of degree N (N+1 points: +-1 and the roots of P_N'), weights.
template <class T>
void gauss_lobatto(int N, vector<T> &x, vector<T> &w) {
  x.assign(N + 1, 0);
  w.assign(N + 1, 0);
  x[0] = -1;
  x[N] = 1;
  for (int k = 1; k < N; ++k) {
    T r = -std::cos(pi_t<T>() * T(k) / T(N));
    for (int it = 0; it < 100; ++it) {
      T P, dP;
      legendre<T>(N, r, P, dP);
      // Legendre ODE: (1-x^2) P'' = 2x P' - N(N+1) P
      T d2P = (2 * r * dP - T(N) * T(N + 1) * P) / (1 - r * r);
      T dr = dP / d2P;
      r -= dr;
      if (std::fabs(dr) < T(1e-3) * std::numeric_limits<T>::epsilon()) break;
    }
    x[k] = r;
  }
  std::sort(x.begin(), x.end());
  for (int k = 0; k <= N; ++k) {
    T P, dP;
    legendre<T>(N, x[k], P, dP);
    w[k] = T(2) / (T(N) * T(N + 1) * P * P);
  }
}

// Lagrange basis polynomial l_b on `nodes`, evaluated at x (product form).
template <class T>
T lagrange(const vector<T> &nodes, int b, T x) {
  T v = 1;
  for (size_t m = 0; m < nodes.size(); ++m)
    if ((int)m != b) v *= (x - nodes[m]) / (nodes[b] - nodes[m]);
  return v;
}

// Derivative of l_b at x (sum over the dropped factor).
template <class T>
T lagrange_deriv(const vector<T> &nodes, int b, T x) {
  T s = 0;
  for (size_t m = 0; m < nodes.size(); ++m) {
    if ((int)m == b) continue;
    T t = T(1) / (nodes[b] - nodes[m]);
    for (size_t k = 0; k < nodes.size(); ++k)
      if ((int)k != b && k != m) t *= (x - nodes[k]) / (nodes[b] - nodes[k]);
    s += t;
  }
  return s;
}

// Derivative of the right correction function g_R = (P_p + P_{p+1})/2 at x. With g_L(x) =
// g_R(-x) this is Huynh's g_DG (Radau) choice, which makes FR identical to a nodal
// collocated DG method (section "FR Algorithm", the choice of g).
template <class T>
T gR_deriv(int p, T x) {
  T P1, dP1, P2, dP2;
  legendre<T>(p, x, P1, dP1);
  legendre<T>(p + 1, x, P2, dP2);
  return (dP1 + dP2) / 2;
}

template <class T>
struct Basis {
  int p = 0, n = 1;  // degree and points per direction
  vector<T> xs, ws;  // Gauss-Legendre solution points / weights
  vector<T> D;       // D[a*n + b] = l_b'(xs_a)
  vector<T> lm, lp;  // l_b(-1), l_b(+1)
  vector<T> gcR;     // g_R'(+xs_a): correction from the face at xi = +1
  vector<T> gcL;     // g_R'(-xs_a): correction from the face at xi = -1 (sign s applied later)
  int pg = 1;        // degree of the geometry interpolant used for metrics (max(p,1))
  vector<T> xg, wg;  // GLL points of degree pg

  void build(int p_) {
    p = p_;
    n = p + 1;
    gauss_legendre<T>(n, xs, ws);
    D.assign(n * n, 0);
    lm.assign(n, 0);
    lp.assign(n, 0);
    gcR.assign(n, 0);
    gcL.assign(n, 0);
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) D[a * n + b] = n == 1 ? T(0) : lagrange_deriv<T>(xs, b, xs[a]);
    for (int b = 0; b < n; ++b) {
      lm[b] = lagrange<T>(xs, b, T(-1));
      lp[b] = lagrange<T>(xs, b, T(1));
      gcR[b] = gR_deriv<T>(p, xs[b]);
      gcL[b] = gR_deriv<T>(p, -xs[b]);
    }
    pg = std::max(p, 1);
    gauss_lobatto<T>(pg, xg, wg);
  }
};

// ---------------------------------------------------------------------------------------------
// Tensor-product application: out[tx + Nx*(ty + Ny*tz)] = sum_{i,j,k} Mz[tz][k] My[ty][j]
// Mx[tx][i] in[i + n*(j + n*k)], done one direction at a time.
// ---------------------------------------------------------------------------------------------
template <class T>
struct Mat {
  int rows = 0, cols = 0;
  vector<T> a;
  T operator()(int r, int c) const { return a[r * cols + c]; }
};

template <class T>
void apply_tensor(const Mat<T> &Mx, const Mat<T> &My, const Mat<T> &Mz, const T *in, T *out) {
  const int n = Mx.cols;  // same source size in each direction
  const int Nx = Mx.rows, Ny = My.rows, Nz = Mz.rows;
  vector<T> t1(Nx * n * n, 0), t2(Nx * Ny * n, 0);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int tx = 0; tx < Nx; ++tx) {
        T s = 0;
        for (int i = 0; i < n; ++i) s += Mx(tx, i) * in[i + n * (j + n * k)];
        t1[tx + Nx * (j + n * k)] = s;
      }
  for (int k = 0; k < n; ++k)
    for (int ty = 0; ty < Ny; ++ty)
      for (int tx = 0; tx < Nx; ++tx) {
        T s = 0;
        for (int j = 0; j < n; ++j) s += My(ty, j) * t1[tx + Nx * (j + n * k)];
        t2[tx + Nx * (ty + Ny * k)] = s;
      }
  for (int tz = 0; tz < Nz; ++tz)
    for (int ty = 0; ty < Ny; ++ty)
      for (int tx = 0; tx < Nx; ++tx) {
        T s = 0;
        for (int k = 0; k < n; ++k) s += Mz(tz, k) * t2[tx + Nx * (ty + Ny * k)];
        out[tx + Nx * (ty + Ny * tz)] = s;
      }
}

// Interpolation (deriv=false) or derivative (deriv=true) matrix from `nodes` to `targets`.
template <class T>
Mat<T> lag_matrix(const vector<T> &nodes, const vector<T> &targets, bool deriv) {
  Mat<T> M;
  M.rows = (int)targets.size();
  M.cols = (int)nodes.size();
  M.a.assign(M.rows * M.cols, 0);
  for (int r = 0; r < M.rows; ++r)
    for (int c = 0; c < M.cols; ++c)
      M.a[r * M.cols + c] = deriv ? (M.cols == 1 ? T(0) : lagrange_deriv<T>(nodes, c, targets[r]))
                                  : lagrange<T>(nodes, c, targets[r]);
  return M;
}

// ---------------------------------------------------------------------------------------------
// Physics (Eq. (1); the readings: conserved gradients + chain rule, constant viscosity,
// Stokes hypothesis, Fourier heat flux with kappa' = mu gamma / (Pr (gamma-1)) acting on p/rho).
// ---------------------------------------------------------------------------------------------
template <class T>
struct Gas {
  T gamma, prandtl, mu;
};

// Inviscid flux projected on a direction n (not necessarily unit): F_i(U) n_i.
template <class T>
void inviscid_flux_n(const T U[5], const T n[3], T gamma, T F[5], T *un_out, T *c_out) {
  T rho = U[0];
  T u = U[1] / rho, v = U[2] / rho, w = U[3] / rho;
  T p = (gamma - 1) * (U[4] - T(0.5) * rho * (u * u + v * v + w * w));
  T un = u * n[0] + v * n[1] + w * n[2];
  F[0] = rho * un;
  F[1] = U[1] * un + p * n[0];
  F[2] = U[2] * un + p * n[1];
  F[3] = U[3] * un + p * n[2];
  F[4] = (U[4] + p) * un;
  if (un_out) *un_out = un;
  if (c_out) *c_out = std::sqrt(gamma * p / rho);
}

// Rusanov (local Lax-Friedrichs): mean normal flux minus half the largest wave speed times
// the jump. Reading: the speed is max over both sides of |u.n| + c.
template <class T>
void rusanov(const T UL[5], const T UR[5], const T n[3], T gamma, T F[5]) {
  T FL[5], FR[5], unL, unR, cL, cR;
  inviscid_flux_n<T>(UL, n, gamma, FL, &unL, &cL);
  inviscid_flux_n<T>(UR, n, gamma, FR, &unR, &cR);
  T lam = std::max(std::fabs(unL) + cL, std::fabs(unR) + cR);
  for (int v = 0; v < 5; ++v) F[v] = T(0.5) * (FL[v] + FR[v]) - T(0.5) * lam * (UR[v] - UL[v]);
}

// Roe's approximate Riemann solver (textbook wave decomposition, sqrt(rho)-weighted averages,
// no entropy fix): F = mean normal flux - 1/2 sum_k |lambda_k| alpha_k r_k.
template <class T>
void roe(const T UL[5], const T UR[5], const T n[3], T gamma, T F[5]) {
  T FL[5], FR[5];
  inviscid_flux_n<T>(UL, n, gamma, FL, nullptr, nullptr);
  inviscid_flux_n<T>(UR, n, gamma, FR, nullptr, nullptr);
  T rL = UL[0], rR = UR[0];
  T uL[3] = {UL[1] / rL, UL[2] / rL, UL[3] / rL};
  T uR[3] = {UR[1] / rR, UR[2] / rR, UR[3] / rR};
  T pL = (gamma - 1) * (UL[4] - T(0.5) * rL * (uL[0] * uL[0] + uL[1] * uL[1] + uL[2] * uL[2]));
  T pR = (gamma - 1) * (UR[4] - T(0.5) * rR * (uR[0] * uR[0] + uR[1] * uR[1] + uR[2] * uR[2]));
  T HL = (UL[4] + pL) / rL, HR = (UR[4] + pR) / rR;
  T sL = std::sqrt(rL), sR = std::sqrt(rR);
  T rt = sL * sR;  // Roe-average density
  T ut[3];
  for (int i = 0; i < 3; ++i) ut[i] = (sL * uL[i] + sR * uR[i]) / (sL + sR);
  T Ht = (sL * HL + sR * HR) / (sL + sR);
  T q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
  T c2 = (gamma - 1) * (Ht - T(0.5) * q2);
  T ct = std::sqrt(c2);
  T unt = ut[0] * n[0] + ut[1] * n[1] + ut[2] * n[2];
  T dr = rR - rL, dp = pR - pL;
  T du[3] = {uR[0] - uL[0], uR[1] - uL[1], uR[2] - uL[2]};
  T dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
  // wave strengths
  T a1 = (dp - rt * ct * dun) / (2 * c2);  // u_n - c
  T a5 = (dp + rt * ct * dun) / (2 * c2);  // u_n + c
  T a2 = dr - dp / c2;                     // entropy wave, u_n
  T l1 = std::fabs(unt - ct), l2 = std::fabs(unt), l5 = std::fabs(unt + ct);
  T dis[5];
  // acoustic waves
  dis[0] = l1 * a1 + l5 * a5;
  for (int i = 0; i < 3; ++i) dis[1 + i] = l1 * a1 * (ut[i] - ct * n[i]) + l5 * a5 * (ut[i] + ct * n[i]);
  dis[4] = l1 * a1 * (Ht - unt * ct) + l5 * a5 * (Ht + unt * ct);
  // entropy wave
  dis[0] += l2 * a2;
  for (int i = 0; i < 3; ++i) dis[1 + i] += l2 * a2 * ut[i];
  dis[4] += l2 * a2 * T(0.5) * q2;
  // shear waves: rho~ (du - dun n)
  T udu = 0;
  for (int i = 0; i < 3; ++i) {
    T sh = du[i] - dun * n[i];
    dis[1 + i] += l2 * rt * sh;
    udu += ut[i] * sh;
  }
  dis[4] += l2 * rt * udu;
  for (int v = 0; v < 5; ++v) F[v] = T(0.5) * (FL[v] + FR[v]) - T(0.5) * dis[v];
}

// Viscous flux Fv[i][v] from the state U and the gradient of the conserved variables,
// G[i][v] = d U_v / d x_i.
//
// Eddy viscosity (learned sub-grid closure): mut = rho * nu_t is added to mu in the stress and
// mut / Pr_t to mu / Pr in the heat flux (an eddy-viscosity reading of the "LES sub-grid scale
// models" the solver supports; the paper gives no model). mut = 0 reproduces the plain flux
// bit for bit.
template <class T>
void viscous_flux(const T U[5], const T G[3][5], const Gas<T> &gas, T Fv[3][5], T mut = T(0),
                  T prandtl_t = T(1)) {
  const T gamma = gas.gamma, mu = gas.mu + mut;
  const T kappa = gas.mu * gamma / (gas.prandtl * (gamma - 1)) +
                  (mut != T(0) ? mut * gamma / (prandtl_t * (gamma - 1)) : T(0));
  T rho = U[0];
  T u[3] = {U[1] / rho, U[2] / rho, U[3] / rho};
  T e = U[4] / rho;
  T du[3][3];  // du[i][j] = d u_j / d x_i
  T dT[3];     // d (p/rho) / d x_i
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) du[i][j] = (G[i][1 + j] - u[j] * G[i][0]) / rho;
    T de = (G[i][4] - e * G[i][0]) / rho;  // d(E/rho)/dx_i
    T udu = u[0] * du[i][0] + u[1] * du[i][1] + u[2] * du[i][2];
    dT[i] = (gamma - 1) * (de - udu);
  }
  T divu = du[0][0] + du[1][1] + du[2][2];
  for (int i = 0; i < 3; ++i) {
    T tau[3];
    for (int j = 0; j < 3; ++j) tau[j] = mu * (du[j][i] + du[i][j]) - (i == j ? T(2) / 3 * mu * divu : T(0));
    Fv[i][0] = 0;
    Fv[i][1] = tau[0];
    Fv[i][2] = tau[1];
    Fv[i][3] = tau[2];
    Fv[i][4] = tau[0] * u[0] + tau[1] * u[1] + tau[2] * u[2] + kappa * dT[i];
  }
}

// ---------------------------------------------------------------------------------------------
// Reference hexahedron: VTK corner order, faces 0:xi=-1 1:xi=+1 2:eta=-1 3:eta=+1 4:zeta=-1
// 5:zeta=+1. A face's points are indexed a + n*b over its two tangential directions in
// increasing order.
// ---------------------------------------------------------------------------------------------
const int kCorner[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                           {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};

int corner_of(int bx, int by, int bz) {
  for (int c = 0; c < 8; ++c)
    if (kCorner[c][0] == bx && kCorner[c][1] == by && kCorner[c][2] == bz) return c;
  return -1;
}

void face_tangents(int d, int &t1, int &t2) {
  t1 = d == 0 ? 1 : 0;
  t2 = d == 2 ? 1 : 2;
}

struct FaceLink {
  int64_t nbr = -1;   // neighbour element (-1: a wall)
  int nface = -1;     // neighbour's local face
  bool owner = false; // this side supplies the face normal ("left" side)
  bool wall = false;  // isothermal no-slip wall (no neighbour)
  vector<int> perm;   // face point k of this side == point perm[k] of the neighbour's face
};

// ---------------------------------------------------------------------------------------------
// The oracle proper.
// ---------------------------------------------------------------------------------------------
// ---------------------------------------------------------------------------------------------
// Explicit Runge-Kutta drivers for dU/dt = R(U).
//   scheme 0: classical four-stage RK4 (nodes 0, 1/2, 1/2, 1; weights 1/6, 1/3, 1/3, 1/6).
//   scheme 1: Carpenter-Kennedy five-stage fourth-order 2N-storage scheme:
//             dU <- A_i dU + dt R(U);  U <- U + B_i dU.
// ---------------------------------------------------------------------------------------------
// The 2N-storage coefficients (A_i, B_i) of the Carpenter-Kennedy scheme, i = 0..4, as the
// published ratios of integers.
template <class T>
void lsrk45_tables(T A[5], T B[5]) {
  A[0] = T(0);
  A[1] = -T(567301805773.0) / T(1357537059087.0);
  A[2] = -T(2404267990393.0) / T(2016746695238.0);
  A[3] = -T(3550918686646.0) / T(2091501179385.0);
  A[4] = -T(1275806237668.0) / T(842570457699.0);
  B[0] = T(1432997174477.0) / T(9575080441237.0);
  B[1] = T(5161836677717.0) / T(13612068292357.0);
  B[2] = T(1720146321549.0) / T(2090206949498.0);
  B[3] = T(3134564353537.0) / T(4481467310338.0);
  B[4] = T(2277821191437.0) / T(14882151754819.0);
}

template <class T>
int rk_advance(vector<T> &U, T dt, int scheme, int nsteps,
               const std::function<void(const vector<T> &, vector<T> &)> &resid) {
  const size_t M = U.size();
  vector<T> R(M);
  for (int step = 0; step < nsteps; ++step) {
    if (scheme == 0) {
      const T c[4] = {T(0), T(1) / 2, T(1) / 2, T(1)};
      const T w[4] = {T(1) / 6, T(1) / 3, T(1) / 3, T(1) / 6};
      vector<T> U0 = U, acc(M, T(0)), Us(M);
      for (int st = 0; st < 4; ++st) {
        for (size_t i = 0; i < M; ++i) Us[i] = st == 0 ? U0[i] : U0[i] + c[st] * dt * R[i];
        resid(Us, R);
        for (size_t i = 0; i < M; ++i) acc[i] += w[st] * R[i];
      }
      for (size_t i = 0; i < M; ++i) U[i] = U0[i] + dt * acc[i];
    } else if (scheme == 1) {
      T A[5], Bc[5];
      lsrk45_tables<T>(A, Bc);
      vector<T> dU(M, T(0));
      for (int st = 0; st < 5; ++st) {
        resid(U, R);
        for (size_t i = 0; i < M; ++i) {
          dU[i] = A[st] * dU[i] + dt * R[i];
          U[i] = U[i] + Bc[st] * dU[i];
        }
      }
    } else if (scheme == 2) {
      // Ketcheson's ten-stage, fourth-order strong-stability-preserving method (SSP
      // coefficient 6) in its two-register form: five forward-Euler stages of dt/6, a
      // combination of the two registers, four more stages, and a final combined stage
      vector<T> q1 = U, q2 = U;
      auto euler_stage = [&]() {
        resid(q1, R);
        for (size_t i = 0; i < M; ++i) q1[i] = q1[i] + dt / 6 * R[i];
      };
      for (int st = 0; st < 5; ++st) euler_stage();
      for (size_t i = 0; i < M; ++i) {
        q2[i] = q2[i] / 25 + T(9) / 25 * q1[i];
        q1[i] = 15 * q2[i] - 5 * q1[i];
      }
      for (int st = 0; st < 4; ++st) euler_stage();
      resid(q1, R);
      for (size_t i = 0; i < M; ++i) U[i] = q2[i] + T(3) / 5 * q1[i] + dt / 10 * R[i];
    } else {
      return -1;
    }
  }
  return 0;
}

struct Iface {
  virtual ~Iface() {}
  virtual int residual(const double *U, double *R) = 0;
  virtual int rk_step(double *U, double dt, int scheme, int nsteps) = 0;
  virtual int sol_coords(double *xyz) = 0;
  virtual int geometry(double *Ja, double *detJ, double *Nf, double *Jf) = 0;
  virtual int connectivity(int64_t *nbr, int32_t *nface, int32_t *owner, int32_t *perm) = 0;
  virtual int sgs_features(const double *U, double *feat) = 0;
  virtual int n_features() const = 0;
  virtual int set_eddy_viscosity(const double *nu, double prandtl_t) = 0;
  virtual std::string last_err() const = 0;
  virtual void set_body_force(const double *g) = 0;
  virtual int set_viscous_scheme(int scheme, double tau) = 0;
};

template <class T>
struct Oracle : Iface {
  int p, n, Ns, Nfp;
  int64_t E;
  Basis<T> B;
  Gas<T> gas;
  T eta;
  int flux;         // 0 Rusanov, 1 Roe
  int metric_form;  // 0 curl form (freestream preserving); 1 cross-product (negative control)
  uint64_t jitter;  // non-zero: move each rounded metric term by -1, 0 or +1 unit in the last
                    // place (seeded); measures the residual's sensitivity to independently
                    // rounded metric terms (a test knob, never part of the method)
  vector<int64_t> active;  // elements whose residual is returned
  vector<char> need;       // elements whose face data is needed (active + neighbours)
  vector<int64_t> slot;    // element -> geometry slot, -1 if not stored
  vector<FaceLink> links;  // [E*6]
  // geometry per stored element
  vector<T> Ja;    // [slot][Ns][3][3]  Ja[n][i] = |J| d xi_n / d x_i
  vector<T> detJ;  // [slot][Ns]
  vector<T> Nf;    // [slot][6][Nfp][3] outward scaled normal from this element's metrics
  vector<T> Jf;    // [slot][6][Nfp]    |J| interpolated to face points
  vector<T> Xs;    // [slot][3][Ns]     solution point coordinates
  int nthreads;
  T force[3] = {0, 0, 0};  // body force per unit mass (the source term S of Eq. (3))
  const int32_t *bc_tag = nullptr;  // [E][6] during setup: 1 = isothermal no-slip wall
  T wall_T = T(1);         // wall temperature p/rho
  int visc_scheme = 0;     // 0 BR2, 1 LDG
  T ldg_tau = T(0.1);      // LDG penalty on the jump of every conserved variable
  vector<T> nut;          // [E] eddy kinematic viscosity per element; empty = none
  T prandtl_t = T(0.9);   // turbulent Prandtl number

  // per-stage scratch over stored elements
  vector<T> Uf, Gf, UCf, FIf;  // [slot][6][Nfp][5], [slot][6][Nfp][3][5], ..

  int pt(int d, int c, int a, int b) const {  // solution point on the line normal to face d
    int t1, t2;
    face_tangents(d, t1, t2);
    int idx[3];
    idx[d] = c;
    idx[t1] = a;
    idx[t2] = b;
    return idx[0] + n * (idx[1] + n * idx[2]);
  }

  std::string err;
  std::string last_err() const override { return err; }
  int set_viscous_scheme(int scheme, double tau) override {
    if (scheme != 0 && scheme != 1) { err = "unknown viscous scheme"; return -1; }
    if (scheme == 1 && (int64_t)active.size() != E) { err = "LDG needs the full mesh"; return -1; }
    if (scheme == 1 && has_walls) { err = "LDG with walls is not supported"; return -1; }
    visc_scheme = scheme;
    ldg_tau = T(tau);
    return 0;
  }
  void set_body_force(const double *g) override {
    for (int i = 0; i < 3; ++i) force[i] = T(g[i]);
  }

  // rounding of a long-double metric term to T, optionally moved by one unit in the last place
  T round_geo(long double v, uint64_t key) const {
    T r = T(v);
    if (!jitter) return r;
    uint64_t h = (key + jitter) * 0x9e3779b97f4a7c15ull;
    h ^= h >> 31;
    h *= 0xbf58476d1ce4e5b9ull;
    h ^= h >> 29;
    const int k = int(h % 3);
    if (k == 1) r = std::nextafter(r, std::numeric_limits<T>::infinity());
    if (k == 2) r = std::nextafter(r, -std::numeric_limits<T>::infinity());
    return r;
  }

  bool has_walls = false;

  int setup(int p_, int64_t E_, const int64_t *ev, int q, const double *nodes, const Gas<T> &g,
            T eta_, int flux_, int mform, int64_t nact, const int64_t *act, int nth) {
    p = p_;
    n = p + 1;
    Ns = n * n * n;
    Nfp = n * n;
    E = E_;
    gas = g;
    eta = eta_;
    flux = flux_;
    metric_form = mform;
    nthreads = nth;
    B.build(p);
    if (q < 1 || q > B.pg) { err = "geometry degree q must be in 1..max(p,1)"; return -1; }
    if (act) active.assign(act, act + nact);
    else { active.resize(E); for (int64_t e = 0; e < E; ++e) active[e] = e; }
    for (int64_t e : active)
      if (e < 0 || e >= E) { err = "active element out of range"; return -1; }

    // --- face matching: sort each face's corner ids, pair equal keys (paper, pre-processor) ---
    links.assign(E * 6, FaceLink());
    std::map<std::array<int64_t, 4>, vector<std::pair<int64_t, int>>> faces;
    for (int64_t e = 0; e < E; ++e)
      for (int f = 0; f < 6; ++f) {
        std::array<int64_t, 4> key;
        int m = 0;
        int d = f / 2, s = f % 2;
        for (int c = 0; c < 8; ++c)
          if (kCorner[c][d] == s) key[m++] = ev[e * 8 + c];
        std::sort(key.begin(), key.end());
        for (int i = 0; i < 3; ++i)
          if (key[i] == key[i + 1]) { err = "face with repeated vertex id in element " + std::to_string(e); return -1; }
        faces[key].push_back({e, f});
      }
    for (auto &kv : faces) {
      if (kv.second.size() == 1 && bc_tag && bc_tag[kv.second[0].first * 6 + kv.second[0].second] == 1) {
        // an isothermal no-slip wall: this element owns the face; there is no neighbour
        FaceLink &lw = links[kv.second[0].first * 6 + kv.second[0].second];
        lw.nbr = -1; lw.nface = -1; lw.owner = true; lw.wall = true; lw.perm.assign(Nfp, 0);
        has_walls = true;
        for (int k = 0; k < Nfp; ++k) lw.perm[k] = k;
        continue;
      }
      if (kv.second.size() != 2) { err = "unpaired face without a wall tag"; return -1; }
      auto A = kv.second[0], Bf = kv.second[1];  // A < B lexicographically (insertion order)
      if (Bf < A) std::swap(A, Bf);
      // corner correspondence: face-local corner (alpha, beta) of A -> vertex id
      auto local_corner_ids = [&](int64_t e, int f, int64_t ids[2][2]) {
        int d = f / 2, s = f % 2, t1, t2;
        face_tangents(d, t1, t2);
        for (int al = 0; al < 2; ++al)
          for (int be = 0; be < 2; ++be) {
            int b3[3];
            b3[d] = s;
            b3[t1] = al;
            b3[t2] = be;
            ids[al][be] = ev[e * 8 + corner_of(b3[0], b3[1], b3[2])];
          }
      };
      int64_t ia[2][2], ib[2][2];
      local_corner_ids(A.first, A.second, ia);
      local_corner_ids(Bf.first, Bf.second, ib);
      auto find_b = [&](int64_t id, int &x, int &y) {
        for (x = 0; x < 2; ++x)
          for (y = 0; y < 2; ++y)
            if (ib[x][y] == id) return true;
        return false;
      };
      int o[2], e1[2], e2[2], c11[2];
      if (!find_b(ia[0][0], o[0], o[1]) || !find_b(ia[1][0], e1[0], e1[1]) ||
          !find_b(ia[0][1], e2[0], e2[1]) || !find_b(ia[1][1], c11[0], c11[1])) {
        err = "inconsistent face corners";
        return -1;
      }
      int d1[2] = {e1[0] - o[0], e1[1] - o[1]}, d2[2] = {e2[0] - o[0], e2[1] - o[1]};
      if (c11[0] != o[0] + d1[0] + d2[0] || c11[1] != o[1] + d1[1] + d2[1]) {
        err = "inconsistent face corners";
        return -1;
      }
      // point (a, b) of A -> point (o*p + a*d1 + b*d2) of B, and the inverse
      FaceLink &la = links[A.first * 6 + A.second];
      FaceLink &lb = links[Bf.first * 6 + Bf.second];
      la.nbr = Bf.first; la.nface = Bf.second; la.owner = true; la.perm.assign(Nfp, 0);
      lb.nbr = A.first; lb.nface = A.second; lb.owner = false; lb.perm.assign(Nfp, 0);
      for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
          int x = o[0] * p + a * d1[0] + b * d2[0];
          int y = o[1] * p + a * d1[1] + b * d2[1];
          la.perm[a + n * b] = x + n * y;
          lb.perm[x + n * y] = a + n * b;
        }
    }

    need.assign(E, 0);
    for (int64_t e : active) {
      need[e] = 1;
      for (int f = 0; f < 6; ++f)
        if (!links[e * 6 + f].wall) need[links[e * 6 + f].nbr] = 1;
    }
    slot.assign(E, -1);
    int64_t ns = 0;
    for (int64_t e = 0; e < E; ++e)
      if (need[e]) slot[e] = ns++;

    // --- geometry (section "FR Algorithm", Eq. (1): J_ij = dx_i/dxi_j, Q^ = |J| Q) ---
    Ja.assign(ns * Ns * 9, 0);
    detJ.assign(ns * Ns, 0);
    Nf.assign(ns * 6 * Nfp * 3, 0);
    Jf.assign(ns * 6 * Nfp, 0);
    Xs.assign(ns * 3 * Ns, 0);
    const int nq = q + 1, ng = B.pg + 1;
    // The metric terms are computed in long double whatever T is, then rounded to T: the
    // residual multiplies them by fluxes that are large against their divergence (the
    // pressure p0 in the momentum flux), so their round-off must sit below T's.
    using G = long double;
    Basis<G> BG;
    BG.build(p);
    vector<G> xq, wq;
    gauss_lobatto<G>(q, xq, wq);
    Mat<G> Iqg = lag_matrix<G>(xq, BG.xg, false);  // degree q nodes -> degree pg GLL nodes
    Mat<G> Igs = lag_matrix<G>(BG.xg, BG.xs, false), Dgs = lag_matrix<G>(BG.xg, BG.xs, true);
    Mat<G> Igg = lag_matrix<G>(BG.xg, BG.xg, false), Dgg = lag_matrix<G>(BG.xg, BG.xg, true);
    vector<G> mone(1, G(-1)), pone(1, G(1));
    Mat<G> Ige[2] = {lag_matrix<G>(BG.xg, mone, false), lag_matrix<G>(BG.xg, pone, false)};
    Mat<G> Dge[2] = {lag_matrix<G>(BG.xg, mone, true), lag_matrix<G>(BG.xg, pone, true)};
    int bad = 0;
    int64_t bad_e = -1;

#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t e = 0; e < E; ++e) {
      if (!need[e]) continue;
      const int64_t sl = slot[e];
      // nodal coordinates at degree-pg GLL points
      vector<G> Xg(3 * ng * ng * ng), in(nq * nq * nq);
      for (int c = 0; c < 3; ++c) {
        for (int m = 0; m < nq * nq * nq; ++m) in[m] = G(nodes[(e * nq * nq * nq + m) * 3 + c]);
        apply_tensor<G>(Iqg, Iqg, Iqg, in.data(), &Xg[c * ng * ng * ng]);
      }
      const int NG = ng * ng * ng;
      // element-local coordinates: every metric quantity below is a derivative of X, so the
      // shift by the first node changes nothing but the round-off (which otherwise grows with |X|)
      G xorig[3];
      for (int c = 0; c < 3; ++c) {
        xorig[c] = Xg[c * NG];
        for (int g2 = 0; g2 < NG; ++g2) Xg[c * NG + g2] -= xorig[c];
      }
      // dX[c][k] at GLL nodes
      vector<G> dXg(9 * NG);
      for (int c = 0; c < 3; ++c)
        for (int k = 0; k < 3; ++k)
          apply_tensor<G>(k == 0 ? Dgg : Igg, k == 1 ? Dgg : Igg, k == 2 ? Dgg : Igg, &Xg[c * NG],
                          &dXg[(c * 3 + k) * NG]);
      // solution-point coordinates and Jacobian matrix J[c][k] = dX_c/dxi_k
      vector<G> Jm(9 * Ns), xs_g(Ns), detG(Ns);
      for (int c = 0; c < 3; ++c) {
        apply_tensor<G>(Igs, Igs, Igs, &Xg[c * NG], xs_g.data());
        for (int s = 0; s < Ns; ++s) Xs[(sl * 3 + c) * Ns + s] = T(xs_g[s] + xorig[c]);
        for (int k = 0; k < 3; ++k)
          apply_tensor<G>(k == 0 ? Dgs : Igs, k == 1 ? Dgs : Igs, k == 2 ? Dgs : Igs, &Xg[c * NG],
                          &Jm[(c * 3 + k) * Ns]);
      }
      for (int s = 0; s < Ns; ++s) {
        G J[3][3];
        for (int c = 0; c < 3; ++c)
          for (int k = 0; k < 3; ++k) J[c][k] = Jm[(c * 3 + k) * Ns + s];
        G det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        detG[s] = det;
        detJ[sl * Ns + s] = round_geo(det, (uint64_t)(e * Ns + s) * 16 + 9);
        if (!(det > 0)) {
#pragma omp critical
          { bad = 1; bad_e = e; }
        }
      }
      // metric terms Ja[n][i] = |J| dxi_n/dx_i evaluated at a target tensor set given by the
      // interpolation matrices (Mi) and derivative matrices (Md) per direction.
      auto metrics_at = [&](const Mat<G> *Mi[3], const Mat<G> *Md[3], int NT, G *out /*[NT][3][3]*/) {
        if (metric_form == 0) {
          // conservative curl form: Ja^n_i = -[curl_xi I(X_l grad_xi X_m)]_n, (i,m,l) cyclic
          // (X is element-local here; the curl of a constant times a gradient vanishes)
          vector<G> V(3 * NG);
          for (int i = 0; i < 3; ++i) {
            int m = (i + 1) % 3, l = (i + 2) % 3;
            for (int k = 0; k < 3; ++k)
              for (int g2 = 0; g2 < NG; ++g2) V[k * NG + g2] = Xg[l * NG + g2] * dXg[(m * 3 + k) * NG + g2];
            for (int nn = 0; nn < 3; ++nn) {
              int a1 = (nn + 1) % 3, a2 = (nn + 2) % 3;
              // d_{a1} V_{a2} - d_{a2} V_{a1}
              vector<G> t1(NT), t2(NT);
              const Mat<G> *M1[3] = {Mi[0], Mi[1], Mi[2]};
              M1[a1] = Md[a1];
              apply_tensor<G>(*M1[0], *M1[1], *M1[2], &V[a2 * NG], t1.data());
              const Mat<G> *M2[3] = {Mi[0], Mi[1], Mi[2]};
              M2[a2] = Md[a2];
              apply_tensor<G>(*M2[0], *M2[1], *M2[2], &V[a1 * NG], t2.data());
              for (int t = 0; t < NT; ++t) out[t * 9 + nn * 3 + i] = -(t1[t] - t2[t]);
            }
          }
        } else {
          // cross-product form (negative control): Ja^n = d_{n+1} X x d_{n+2} X
          vector<G> dX(9 * NT);
          for (int c = 0; c < 3; ++c)
            for (int k = 0; k < 3; ++k) {
              const Mat<G> *M1[3] = {Mi[0], Mi[1], Mi[2]};
              M1[k] = Md[k];
              apply_tensor<G>(*M1[0], *M1[1], *M1[2], &Xg[c * NG], &dX[(c * 3 + k) * NT]);
            }
          for (int t = 0; t < NT; ++t)
            for (int nn = 0; nn < 3; ++nn) {
              int a1 = (nn + 1) % 3, a2 = (nn + 2) % 3;
              G A[3], Bv[3];
              for (int c = 0; c < 3; ++c) { A[c] = dX[(c * 3 + a1) * NT + t]; Bv[c] = dX[(c * 3 + a2) * NT + t]; }
              out[t * 9 + nn * 3 + 0] = A[1] * Bv[2] - A[2] * Bv[1];
              out[t * 9 + nn * 3 + 1] = A[2] * Bv[0] - A[0] * Bv[2];
              out[t * 9 + nn * 3 + 2] = A[0] * Bv[1] - A[1] * Bv[0];
            }
        }
      };
      {
        const Mat<G> *Mi[3] = {&Igs, &Igs, &Igs}, *Md[3] = {&Dgs, &Dgs, &Dgs};
        vector<G> Jas(Ns * 9);
        metrics_at(Mi, Md, Ns, Jas.data());
        for (int t = 0; t < Ns * 9; ++t) Ja[sl * Ns * 9 + t] = round_geo(Jas[t], (uint64_t)(e * Ns * 9 + t) * 16 + 1);
      }
      for (int f = 0; f < 6; ++f) {
        int d = f / 2, s = f % 2;
        const Mat<G> *Mi[3] = {&Igs, &Igs, &Igs}, *Md[3] = {&Dgs, &Dgs, &Dgs};
        Mi[d] = &Ige[s];
        Md[d] = &Dge[s];
        vector<G> Jaf(Nfp * 9);
        metrics_at(Mi, Md, Nfp, Jaf.data());
        G sg = s ? G(1) : G(-1);
        for (int k = 0; k < Nfp; ++k)
          for (int i = 0; i < 3; ++i)
            Nf[((sl * 6 + f) * Nfp + k) * 3 + i] =
                round_geo(sg * Jaf[k * 9 + d * 3 + i], (uint64_t)(((e * 6 + f) * Nfp + k) * 3 + i) * 16 + 2);
        // |J| at face points: interpolation of the solution-point |J| along the normal line
        const vector<G> &ell = s ? BG.lp : BG.lm;
        for (int b = 0; b < n; ++b)
          for (int a = 0; a < n; ++a) {
            G v = 0;
            for (int c = 0; c < n; ++c) v += ell[c] * detG[pt(d, c, a, b)];
            Jf[(sl * 6 + f) * Nfp + a + n * b] = round_geo(v, (uint64_t)((e * 6 + f) * Nfp + a + n * b) * 16 + 3);
          }
      }
    }
    if (bad) { err = "non-positive Jacobian in element " + std::to_string(bad_e); return -2; }
    Uf.assign(ns * 6 * Nfp * 5, 0);
    Gf.assign(ns * 6 * Nfp * 15, 0);
    UCf.assign(ns * 6 * Nfp * 5, 0);
    FIf.assign(ns * 6 * Nfp * 5, 0);
    return 0;
  }

  // reference-space derivative along direction d of field X (Ns values)
  void ref_deriv(int d, const T *X, T *out) const {
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          int idx[3] = {i, j, k};
          int a = idx[d];
          T s = 0;
          for (int c = 0; c < n; ++c) {
            int id2[3] = {i, j, k};
            id2[d] = c;
            s += B.D[a * n + c] * X[id2[0] + n * (id2[1] + n * id2[2])];
          }
          out[i + n * (j + n * k)] = s;
        }
  }

  // ---- the residual: dU/dt of Eq. (3) with S = 0 ----
  int residual_impl(const vector<T> &Ufull /*[E][5][Ns]*/, T *R /*[n_active][5][Ns]*/) {
    const bool viscous = gas.mu != T(0) || !nut.empty();
    // pass 1: per element, interpolate U and the broken physical gradient to the faces
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t e = 0; e < E; ++e) {
      if (!need[e]) continue;
      const int64_t sl = slot[e];
      const T *U = &Ufull[e * 5 * Ns];
      vector<T> dU(3 * 5 * Ns), Gbr(3 * 5 * Ns, 0);
      for (int d = 0; d < 3; ++d)
        for (int v = 0; v < 5; ++v) ref_deriv(d, U + v * Ns, &dU[(d * 5 + v) * Ns]);
      for (int s = 0; s < Ns; ++s) {
        const T *ja = &Ja[(sl * Ns + s) * 9];
        T iJ = T(1) / detJ[sl * Ns + s];
        for (int i = 0; i < 3; ++i)
          for (int v = 0; v < 5; ++v) {
            T g = 0;
            for (int d = 0; d < 3; ++d) g += ja[d * 3 + i] * dU[(d * 5 + v) * Ns + s];
            Gbr[(i * 5 + v) * Ns + s] = iJ * g;
          }
      }
      for (int f = 0; f < 6; ++f) {
        int d = f / 2, sd = f % 2;
        const vector<T> &ell = sd ? B.lp : B.lm;
        for (int b = 0; b < n; ++b)
          for (int a = 0; a < n; ++a) {
            int k = a + n * b;
            for (int v = 0; v < 5; ++v) {
              T su = 0;
              for (int c = 0; c < n; ++c) su += ell[c] * U[v * Ns + pt(d, c, a, b)];
              Uf[((sl * 6 + f) * Nfp + k) * 5 + v] = su;
              for (int i = 0; i < 3; ++i) {
                T sg = 0;
                for (int c = 0; c < n; ++c) sg += ell[c] * Gbr[(i * 5 + v) * Ns + pt(d, c, a, b)];
                Gf[(((sl * 6 + f) * Nfp + k) * 3 + i) * 5 + v] = sg;
              }
            }
          }
      }
    }
    // pass 1b (LDG, section "FR Algorithm": the viscous flux by the local DG method): the
    // common solution is one-sided, U^ = U_R (beta = +n_owner / 2), so each element's
    // corrected gradient uses U^ - U_K = U_R - U_L on the faces it owns and 0 on the others;
    // the corrected physical gradient is interpolated to the element's face points (it takes
    // the place of the broken gradient in Gf)
    const bool ldg = viscous && visc_scheme == 1;
    if (ldg) {
      vector<T> Gc(Gf.size());
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
      for (int64_t e = 0; e < E; ++e) {
        const int64_t sl = slot[e];
        const T *U = &Ufull[e * 5 * Ns];
        vector<T> dU(3 * 5 * Ns);
        for (int d = 0; d < 3; ++d)
          for (int v = 0; v < 5; ++v) ref_deriv(d, U + v * Ns, &dU[(d * 5 + v) * Ns]);
        for (int f = 0; f < 6; ++f) {
          const FaceLink &lk = links[e * 6 + f];
          if (!lk.owner) continue;  // U^ - U_K = 0 on faces this element does not own
          int d = f / 2, sd = f % 2;
          T sg = sd ? T(1) : T(-1);
          const vector<T> &gc = sd ? B.gcR : B.gcL;
          const int64_t sR = slot[lk.nbr];
          for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
              int k = a + n * b;
              for (int v = 0; v < 5; ++v) {
                T jump = Uf[((sR * 6 + lk.nface) * Nfp + lk.perm[k]) * 5 + v] - Uf[((sl * 6 + f) * Nfp + k) * 5 + v];
                for (int c = 0; c < n; ++c) dU[(d * 5 + v) * Ns + pt(d, c, a, b)] += sg * jump * gc[c];
              }
            }
        }
        vector<T> G(3 * 5 * Ns);
        for (int s = 0; s < Ns; ++s) {
          const T *ja = &Ja[(sl * Ns + s) * 9];
          T iJ = T(1) / detJ[sl * Ns + s];
          for (int i = 0; i < 3; ++i)
            for (int v = 0; v < 5; ++v) {
              T g = 0;
              for (int d = 0; d < 3; ++d) g += ja[d * 3 + i] * dU[(d * 5 + v) * Ns + s];
              G[(i * 5 + v) * Ns + s] = iJ * g;
            }
        }
        for (int f = 0; f < 6; ++f) {
          int d = f / 2, sd = f % 2;
          const vector<T> &ell = sd ? B.lp : B.lm;
          for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
              int k = a + n * b;
              for (int i = 0; i < 3; ++i)
                for (int v = 0; v < 5; ++v) {
                  T sgv = 0;
                  for (int c = 0; c < n; ++c) sgv += ell[c] * G[(i * 5 + v) * Ns + pt(d, c, a, b)];
                  Gc[(((sl * 6 + f) * Nfp + k) * 3 + i) * 5 + v] = sgv;
                }
            }
        }
      }
      Gf.swap(Gc);
    }
    // pass 2: per face (owner side L), common state and transformed common normal flux
    const T cl = T(n) * T(n) / 2;  // g_R'(1) = (p+1)^2/2
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t e = 0; e < E; ++e) {
      if (!need[e]) continue;
      for (int f = 0; f < 6; ++f) {
        const FaceLink &lk = links[e * 6 + f];
        if (!lk.owner) continue;
        if (lk.wall) {
          // isothermal no-slip wall. Inviscid part: the Riemann flux against the mirror state
          // (rho, -m, E), which is impermeable and carries no energy; viscous part: the wall
          // state U_w = (rho_L, 0, rho_L T_w / (gamma-1)) as the common state and the one-sided
          // BR2 gradient G_L + eta r_L with r_L the lifting of U_w - U_L
          const int64_t sL = slot[e];
          for (int k = 0; k < Nfp; ++k) {
            const T *UL = &Uf[((sL * 6 + f) * Nfp + k) * 5];
            const T *N = &Nf[((sL * 6 + f) * Nfp + k) * 3];
            T nm = std::sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
            T nh[3] = {N[0] / nm, N[1] / nm, N[2] / nm};
            T UG[5] = {UL[0], -UL[1], -UL[2], -UL[3], UL[4]};
            T UW[5] = {UL[0], T(0), T(0), T(0), UL[0] * wall_T / (gas.gamma - 1)};
            T Fi[5];
            if (flux == 0) rusanov<T>(UL, UG, nh, gas.gamma, Fi);
            else roe<T>(UL, UG, nh, gas.gamma, Fi);
            T Fvn[5] = {0, 0, 0, 0, 0};
            if (viscous) {
              const T JL = Jf[(sL * 6 + f) * Nfp + k];
              T GI[3][5];
              for (int i = 0; i < 3; ++i)
                for (int v = 0; v < 5; ++v)
                  GI[i][v] = Gf[(((sL * 6 + f) * Nfp + k) * 3 + i) * 5 + v] + eta * cl * N[i] / JL * (UW[v] - UL[v]);
              T Fv[3][5];
              const T mut = nut.empty() ? T(0) : UW[0] * nut[e];
              viscous_flux<T>(UW, GI, gas, Fv, mut, prandtl_t);
              for (int v = 0; v < 5; ++v) Fvn[v] = Fv[0][v] * nh[0] + Fv[1][v] * nh[1] + Fv[2][v] * nh[2];
            }
            for (int v = 0; v < 5; ++v) {
              UCf[((sL * 6 + f) * Nfp + k) * 5 + v] = viscous ? UW[v] : UL[v];
              FIf[((sL * 6 + f) * Nfp + k) * 5 + v] = nm * (Fi[v] - Fvn[v]);
            }
          }
          continue;
        }
        const int64_t eR = lk.nbr;
        const int fR = lk.nface;
        // the face is needed if either side is active; stored data exists if both are needed
        if (!need[eR]) continue;
        const int64_t sL = slot[e], sR = slot[eR];
        for (int k = 0; k < Nfp; ++k) {
          const int kR = lk.perm[k];
          const T *UL = &Uf[((sL * 6 + f) * Nfp + k) * 5];
          const T *UR = &Uf[((sR * 6 + fR) * Nfp + kR) * 5];
          const T *N = &Nf[((sL * 6 + f) * Nfp + k) * 3];
          T nm = std::sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
          T nh[3] = {N[0] / nm, N[1] / nm, N[2] / nm};
          T UC[5];
          for (int v = 0; v < 5; ++v) UC[v] = ldg ? UR[v] : T(0.5) * (UL[v] + UR[v]);
          T Fi[5];
          if (flux == 0) rusanov<T>(UL, UR, nh, gas.gamma, Fi);
          else roe<T>(UL, UR, nh, gas.gamma, Fi);
          T Fvn[5] = {0, 0, 0, 0, 0};
          if (ldg) {
            // LDG: the owner's viscous flux with its corrected gradient, plus the penalty
            T QL[3][5];
            for (int i = 0; i < 3; ++i)
              for (int v = 0; v < 5; ++v) QL[i][v] = Gf[(((sL * 6 + f) * Nfp + k) * 3 + i) * 5 + v];
            T Fv[3][5];
            const T mut = nut.empty() ? T(0) : UL[0] * (nut[e] + nut[eR]) / 2;
            viscous_flux<T>(UL, QL, gas, Fv, mut, prandtl_t);
            for (int v = 0; v < 5; ++v)
              Fvn[v] = Fv[0][v] * nh[0] + Fv[1][v] * nh[1] + Fv[2][v] * nh[2] + ldg_tau * (UR[v] - UL[v]);
          } else if (viscous) {
            const T JL = Jf[(sL * 6 + f) * Nfp + k], JR = Jf[(sR * 6 + fR) * Nfp + kR];
            T GI[3][5];
            for (int i = 0; i < 3; ++i)
              for (int v = 0; v < 5; ++v) {
                T rL = cl * N[i] / JL * (UC[v] - UL[v]);
                T rR = cl * (-N[i]) / JR * (UC[v] - UR[v]);
                T gL = Gf[(((sL * 6 + f) * Nfp + k) * 3 + i) * 5 + v];
                T gR = Gf[(((sR * 6 + fR) * Nfp + kR) * 3 + i) * 5 + v];
                GI[i][v] = T(0.5) * ((gL + eta * rL) + (gR + eta * rR));
              }
            T Fv[3][5];
            // common eddy viscosity: mean of the two elements' values, density of the common state
            const T mut = nut.empty() ? T(0) : UC[0] * (nut[e] + nut[eR]) / 2;
            viscous_flux<T>(UC, GI, gas, Fv, mut, prandtl_t);
            for (int v = 0; v < 5; ++v) Fvn[v] = Fv[0][v] * nh[0] + Fv[1][v] * nh[1] + Fv[2][v] * nh[2];
          }
          for (int v = 0; v < 5; ++v) {
            T FI = nm * (Fi[v] - Fvn[v]);
            UCf[((sL * 6 + f) * Nfp + k) * 5 + v] = UC[v];
            UCf[((sR * 6 + fR) * Nfp + kR) * 5 + v] = UC[v];
            FIf[((sL * 6 + f) * Nfp + k) * 5 + v] = FI;
            FIf[((sR * 6 + fR) * Nfp + kR) * 5 + v] = -FI;
          }
        }
      }
    }
    // pass 3: per active element, corrected gradient, flux, divergence and correction
    const int64_t NA = (int64_t)active.size();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t ia = 0; ia < NA; ++ia) {
      const int64_t e = active[ia];
      const int64_t sl = slot[e];
      const T *U = &Ufull[e * 5 * Ns];
      vector<T> dU(3 * 5 * Ns), Fh(3 * 5 * Ns), div(5 * Ns, 0);
      for (int d = 0; d < 3; ++d)
        for (int v = 0; v < 5; ++v) ref_deriv(d, U + v * Ns, &dU[(d * 5 + v) * Ns]);
      if (viscous) {
        // corrected gradient: each face (d, s) adds s (U^C - U_K) g_R'(s xi_d) to d_d U
        for (int f = 0; f < 6; ++f) {
          int d = f / 2, sd = f % 2;
          T sg = sd ? T(1) : T(-1);
          const vector<T> &gc = sd ? B.gcR : B.gcL;
          for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
              int k = a + n * b;
              for (int v = 0; v < 5; ++v) {
                T jump = UCf[((sl * 6 + f) * Nfp + k) * 5 + v] - Uf[((sl * 6 + f) * Nfp + k) * 5 + v];
                for (int c = 0; c < n; ++c) dU[(d * 5 + v) * Ns + pt(d, c, a, b)] += sg * jump * gc[c];
              }
            }
        }
      }
      for (int s = 0; s < Ns; ++s) {
        const T *ja = &Ja[(sl * Ns + s) * 9];
        T Us[5];
        for (int v = 0; v < 5; ++v) Us[v] = U[v * Ns + s];
        T F[3][5];
        for (int i = 0; i < 3; ++i) {
          T ei[3] = {T(i == 0), T(i == 1), T(i == 2)};
          inviscid_flux_n<T>(Us, ei, gas.gamma, F[i], nullptr, nullptr);
        }
        if (viscous) {
          T iJ = T(1) / detJ[sl * Ns + s];
          T G[3][5];
          for (int i = 0; i < 3; ++i)
            for (int v = 0; v < 5; ++v) {
              T g = 0;
              for (int d = 0; d < 3; ++d) g += ja[d * 3 + i] * dU[(d * 5 + v) * Ns + s];
              G[i][v] = iJ * g;
            }
          T Fv[3][5];
          const T mut = nut.empty() ? T(0) : Us[0] * nut[e];
          viscous_flux<T>(Us, G, gas, Fv, mut, prandtl_t);
          for (int i = 0; i < 3; ++i)
            for (int v = 0; v < 5; ++v) F[i][v] -= Fv[i][v];
        }
        for (int d = 0; d < 3; ++d)
          for (int v = 0; v < 5; ++v)
            Fh[(d * 5 + v) * Ns + s] = ja[d * 3 + 0] * F[0][v] + ja[d * 3 + 1] * F[1][v] + ja[d * 3 + 2] * F[2][v];
      }
      vector<T> tmp(Ns);
      for (int d = 0; d < 3; ++d)
        for (int v = 0; v < 5; ++v) {
          ref_deriv(d, &Fh[(d * 5 + v) * Ns], tmp.data());
          for (int s = 0; s < Ns; ++s) div[v * Ns + s] += tmp[s];
        }
      // flux correction: (F^{I,perp} - s * interp(F^d)) g_R'(s xi_d) along each normal line
      for (int f = 0; f < 6; ++f) {
        int d = f / 2, sd = f % 2;
        T sg = sd ? T(1) : T(-1);
        const vector<T> &ell = sd ? B.lp : B.lm;
        const vector<T> &gc = sd ? B.gcR : B.gcL;
        for (int b = 0; b < n; ++b)
          for (int a = 0; a < n; ++a) {
            int k = a + n * b;
            for (int v = 0; v < 5; ++v) {
              T fp = 0;
              for (int c = 0; c < n; ++c) fp += ell[c] * Fh[(d * 5 + v) * Ns + pt(d, c, a, b)];
              T jump = FIf[((sl * 6 + f) * Nfp + k) * 5 + v] - sg * fp;
              for (int c = 0; c < n; ++c) div[v * Ns + pt(d, c, a, b)] += jump * gc[c];
            }
          }
      }
      for (int v = 0; v < 5; ++v)
        for (int s = 0; s < Ns; ++s) R[(ia * 5 + v) * Ns + s] = -div[v * Ns + s] / detJ[sl * Ns + s];
      // source term S of Eq. (3): a body force g per unit mass adds rho g to the momentum and
      // the work m . g to the energy
      if (force[0] != T(0) || force[1] != T(0) || force[2] != T(0)) {
        for (int s = 0; s < Ns; ++s) {
          T work = 0;
          for (int i = 0; i < 3; ++i) {
            R[(ia * 5 + 1 + i) * Ns + s] += U[s] * force[i];
            work += U[(1 + i) * Ns + s] * force[i];
          }
          R[(ia * 5 + 4) * Ns + s] += work;
        }
      }
    }
    return 0;
  }

  // ---- per-element inputs of the learned eddy-viscosity closure ----
  // From the element's own velocity polynomial u_j (nodal values m_j / rho at the solution
  // points):
  //  * modal energies e_k = (1/8) * 1/2 * sum_j uhat_{j,k}^2 over the orthonormal tensor
  //    Legendre modes k = (a, b, c) of the reference element (uhat by Gauss quadrature, exact for
  //    a degree-p polynomial), so that sum_k e_k is the reference-element mean of |u|^2 / 2;
  //    the constant mode is dropped (Galilean invariance), leaving (p+1)^3 - 1 values;
  //  * five volume averages over the element of the broken velocity gradient
  //    A_ij = d u_j / d x_i: s2 = <2 S:S>, w2 = <2 W:W> (S, W its symmetric and antisymmetric
  //    parts), r = <-tr(A^3) / 3>, th = <tr A>, th2 = <(tr A)^2>.
  // Features: ln(e_k + eps) for each kept mode, then ln(s2 + eps) / 2, ln(w2 + eps) / 2,
  // r / (s2 + eps)^(3/2), th / (s2 + eps)^(1/2), th2 / (s2 + eps), with eps = 1e-12.
  int n_features() const override { return Ns - 1 + 5; }

  int sgs_features(const double *Uin, double *feat) override {
    const int NF = n_features();
    const T eps = T(1e-12);
    vector<T> L(n * n);  // L[a*n + i] = orthonormal Legendre a at xs_i, times w_i
    for (int a = 0; a < n; ++a)
      for (int i = 0; i < n; ++i) {
        T P, dP;
        legendre<T>(a, B.xs[i], P, dP);
        L[a * n + i] = std::sqrt(T(2 * a + 1) / 2) * P * B.ws[i];
      }
    const int64_t NA = (int64_t)active.size();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t ia = 0; ia < NA; ++ia) {
      const int64_t e = active[ia];
      const int64_t sl = slot[e];
      vector<T> u(3 * Ns), du(3 * 3 * Ns);
      for (int s = 0; s < Ns; ++s) {
        T rho = T(Uin[(e * 5 + 0) * Ns + s]);
        for (int j = 0; j < 3; ++j) u[j * Ns + s] = T(Uin[(e * 5 + 1 + j) * Ns + s]) / rho;
      }
      for (int d = 0; d < 3; ++d)
        for (int j = 0; j < 3; ++j) ref_deriv(d, &u[j * Ns], &du[(d * 3 + j) * Ns]);
      double *out = feat + ia * NF;
      int col = 0;
      for (int c = 0; c < n; ++c)
        for (int b = 0; b < n; ++b)
          for (int a = 0; a < n; ++a) {
            if (a == 0 && b == 0 && c == 0) continue;
            T ek = 0;
            for (int j = 0; j < 3; ++j) {
              T uh = 0;
              for (int kk = 0; kk < n; ++kk)
                for (int jj = 0; jj < n; ++jj)
                  for (int ii = 0; ii < n; ++ii)
                    uh += L[a * n + ii] * L[b * n + jj] * L[c * n + kk] * u[j * Ns + ii + n * (jj + n * kk)];
              ek += uh * uh;
            }
            ek = ek / 16;
            out[col++] = double(std::log(ek + eps));
          }
      T vol = 0, s2 = 0, w2 = 0, r = 0, th = 0, th2 = 0;
      for (int kk = 0; kk < n; ++kk)
        for (int jj = 0; jj < n; ++jj)
          for (int ii = 0; ii < n; ++ii) {
            const int s = ii + n * (jj + n * kk);
            const T *ja = &Ja[(sl * Ns + s) * 9];
            const T dJ = detJ[sl * Ns + s];
            T A[3][3];
            for (int i = 0; i < 3; ++i)
              for (int j = 0; j < 3; ++j) {
                T g = 0;
                for (int d = 0; d < 3; ++d) g += ja[d * 3 + i] * du[(d * 3 + j) * Ns + s];
                A[i][j] = g / dJ;
              }
            T ss = 0, ww = 0, t3 = 0;
            for (int i = 0; i < 3; ++i)
              for (int j = 0; j < 3; ++j) {
                T S = (A[i][j] + A[j][i]) / 2, W = (A[i][j] - A[j][i]) / 2;
                ss += S * S;
                ww += W * W;
                for (int k = 0; k < 3; ++k) t3 += A[i][j] * A[j][k] * A[k][i];
              }
            T tr = A[0][0] + A[1][1] + A[2][2];
            T wq = B.ws[ii] * B.ws[jj] * B.ws[kk] * dJ;
            vol += wq;
            s2 += wq * 2 * ss;
            w2 += wq * 2 * ww;
            r += wq * (-t3 / 3);
            th += wq * tr;
            th2 += wq * tr * tr;
          }
      s2 /= vol; w2 /= vol; r /= vol; th /= vol; th2 /= vol;
      out[col++] = double(std::log(s2 + eps) / 2);
      out[col++] = double(std::log(w2 + eps) / 2);
      out[col++] = double(r / std::pow(s2 + eps, T(1.5)));
      out[col++] = double(th / std::sqrt(s2 + eps));
      out[col++] = double(th2 / (s2 + eps));
    }
    return 0;
  }

  int set_eddy_viscosity(const double *nu, double prt) override {
    if (!nu) { nut.clear(); return 0; }
    nut.assign(nu, nu + E);
    for (auto &x : nut) if (!(x >= 0)) { err = "eddy viscosity must be >= 0"; nut.clear(); return -1; }
    prandtl_t = T(prt);
    return 0;
  }

  int residual(const double *U, double *R) override {
    vector<T> Ut(E * 5 * Ns);
    for (int64_t i = 0; i < E * 5 * Ns; ++i) Ut[i] = T(U[i]);
    vector<T> Rt(active.size() * 5 * Ns);
    int rc = residual_impl(Ut, Rt.data());
    for (size_t i = 0; i < Rt.size(); ++i) R[i] = double(Rt[i]);
    return rc;
  }

  // ---- time integration (section "FR Algorithm": an explicit Runge-Kutta ODE solver) ----
  int rk_step(double *Uio, double dt_, int scheme, int nsteps) override {
    if ((int64_t)active.size() != E) { err = "rk_step needs the full mesh"; return -1; }
    const int64_t M = E * 5 * Ns;
    vector<T> U(M);
    for (int64_t i = 0; i < M; ++i) U[i] = T(Uio[i]);
    int rc = rk_advance<T>(U, T(dt_), scheme, nsteps,
                           [&](const vector<T> &X, vector<T> &R) { residual_impl(X, R.data()); });
    if (rc) { err = "unknown scheme"; return -1; }
    for (int64_t i = 0; i < M; ++i) Uio[i] = double(U[i]);
    return 0;
  }

  int sol_coords(double *xyz) override {
    for (size_t ia = 0; ia < active.size(); ++ia) {
      int64_t sl = slot[active[ia]];
      for (int i = 0; i < 3 * Ns; ++i) xyz[ia * 3 * Ns + i] = double(Xs[sl * 3 * Ns + i]);
    }
    return 0;
  }

  int geometry(double *ja, double *dj, double *nf, double *jf) override {
    for (size_t ia = 0; ia < active.size(); ++ia) {
      int64_t sl = slot[active[ia]];
      if (ja) for (int i = 0; i < Ns * 9; ++i) ja[ia * Ns * 9 + i] = double(Ja[sl * Ns * 9 + i]);
      if (dj) for (int i = 0; i < Ns; ++i) dj[ia * Ns + i] = double(detJ[sl * Ns + i]);
      if (nf) for (int i = 0; i < 6 * Nfp * 3; ++i) nf[ia * 6 * Nfp * 3 + i] = double(Nf[sl * 6 * Nfp * 3 + i]);
      if (jf) for (int i = 0; i < 6 * Nfp; ++i) jf[ia * 6 * Nfp + i] = double(Jf[sl * 6 * Nfp + i]);
    }
    return 0;
  }

  int connectivity(int64_t *nbr, int32_t *nface, int32_t *owner, int32_t *perm) override {
    for (int64_t e = 0; e < E; ++e)
      for (int f = 0; f < 6; ++f) {
        const FaceLink &lk = links[e * 6 + f];
        nbr[e * 6 + f] = lk.nbr;
        nface[e * 6 + f] = lk.nface;
        owner[e * 6 + f] = lk.owner;
        for (int k = 0; k < Nfp; ++k) perm[(e * 6 + f) * Nfp + k] = lk.perm[k];
      }
    return 0;
  }
};

thread_local std::string g_err;

}  // namespace

// =============================================================================================
// C API (consumed through ctypes by the tests; never by the product library).
// prec: 0 = double, 1 = long double, 2 = float.
// =============================================================================================
extern "C" {

const char *ora_last_error() { return g_err.c_str(); }

// bc_tag: [n_elem][6] or NULL; 1 marks an isothermal no-slip wall at temperature wall_T (p/rho)
void *ora_create(int prec, int p, int64_t n_elem, const int64_t *elem_vert, int q, const double *elem_nodes,
                 double gamma, double prandtl, double mu, double eta, int flux, int metric_form,
                 int64_t n_active, const int64_t *active, int nthreads, uint64_t metric_jitter,
                 const int32_t *bc_tag, double wall_T) {
  if (p < 0 || p > 15) { g_err = "p out of range"; return nullptr; }
  if (nthreads <= 0) {
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
  }
  Iface *h = nullptr;
  int rc = 0;
  std::string e;
  auto go = [&](auto *o, auto tag) {
    using T = decltype(tag);
    Gas<T> g{T(gamma), T(prandtl), T(mu)};
    o->jitter = metric_jitter;
    o->bc_tag = bc_tag;
    o->wall_T = T(wall_T);
    rc = o->setup(p, n_elem, elem_vert, q, elem_nodes, g, T(eta), flux, metric_form, n_active, active, nthreads);
    o->bc_tag = nullptr;  // borrowed for the setup only
    e = o->err;
    h = o;
  };
  if (prec == 0) go(new Oracle<double>(), double());
  else if (prec == 1) go(new Oracle<long double>(), (long double)0);
  else if (prec == 2) go(new Oracle<float>(), float());
  else { g_err = "bad precision"; return nullptr; }
  if (rc != 0) { g_err = e; delete h; return nullptr; }
  return h;
}

void ora_destroy(void *h) { delete static_cast<Iface *>(h); }

int ora_n_features(void *h) { return static_cast<Iface *>(h)->n_features(); }

// viscous scheme: 0 BR2 (default), 1 LDG with penalty tau
int ora_set_viscous_scheme(void *h, int scheme, double tau) {
  Iface *o = static_cast<Iface *>(h);
  int rc = o->set_viscous_scheme(scheme, tau);
  if (rc) g_err = o->last_err();
  return rc;
}

// body force per unit mass g[3] (the source term of Eq. (3)); zero switches it off
int ora_set_body_force(void *h, const double *g) {
  static_cast<Iface *>(h)->set_body_force(g);
  return 0;
}

// feat: [n_active][n_features] doubles
int ora_sgs_features(void *h, const double *U, double *feat) { return static_cast<Iface *>(h)->sgs_features(U, feat); }

// nu: [E] per-element eddy kinematic viscosity (>= 0), or NULL to switch the closure off
int ora_set_eddy_viscosity(void *h, const double *nu, double prandtl_t) {
  Iface *o = static_cast<Iface *>(h);
  int rc = o->set_eddy_viscosity(nu, prandtl_t);
  if (rc) g_err = o->last_err();
  return rc;
}

int ora_residual(void *h, const double *U, double *R) { return static_cast<Iface *>(h)->residual(U, R); }

int ora_rk_step(void *h, double *U, double dt, int scheme, int nsteps) {
  return static_cast<Iface *>(h)->rk_step(U, dt, scheme, nsteps);
}

int ora_sol_coords(void *h, double *xyz) { return static_cast<Iface *>(h)->sol_coords(xyz); }

int ora_geometry(void *h, double *Ja, double *detJ, double *Nf, double *Jf) {
  return static_cast<Iface *>(h)->geometry(Ja, detJ, Nf, Jf);
}

int ora_connectivity(void *h, int64_t *nbr, int32_t *nface, int32_t *owner, int32_t *perm) {
  return static_cast<Iface *>(h)->connectivity(nbr, nface, owner, perm);
}

// 1-D tables for degree p: xs, ws [n]; D [n*n]; lm, lp [n]; gcR, gcL [n]; xg, wg [max(p,1)+1]
int ora_basis(int prec, int p, double *xs, double *ws, double *D, double *lm, double *lp, double *gcR,
              double *gcL, double *xg, double *wg) {
  auto fill = [&](auto tag) {
    using T = decltype(tag);
    Basis<T> B;
    B.build(p);
    int n = p + 1;
    for (int i = 0; i < n; ++i) {
      xs[i] = double(B.xs[i]); ws[i] = double(B.ws[i]);
      lm[i] = double(B.lm[i]); lp[i] = double(B.lp[i]);
      gcR[i] = double(B.gcR[i]); gcL[i] = double(B.gcL[i]);
    }
    for (int i = 0; i < n * n; ++i) D[i] = double(B.D[i]);
    for (int i = 0; i <= B.pg; ++i) { xg[i] = double(B.xg[i]); wg[i] = double(B.wg[i]); }
  };
  if (prec == 1) fill((long double)0);
  else if (prec == 2) fill(float());
  else fill(double());
  return 0;
}

// Interface flux for one state pair: flux 0 Rusanov, 1 Roe; n must be a unit vector.
int ora_riemann(int flux, double gamma, const double *UL, const double *UR, const double *n, double *F) {
  if (flux == 0) rusanov<double>(UL, UR, n, gamma, F);
  else roe<double>(UL, UR, n, gamma, F);
  return 0;
}

// Physical inviscid flux F_i(U) n_i.
int ora_inviscid_flux(double gamma, const double *U, const double *n, double *F) {
  inviscid_flux_n<double>(U, n, gamma, F, nullptr, nullptr);
  return 0;
}

// Viscous flux Fv[i][v] from U and conserved-variable gradient G[i][v].
int ora_viscous_flux(double gamma, double prandtl, double mu, const double *U, const double *G, double *Fv) {
  Gas<double> g{gamma, prandtl, mu};
  double Gm[3][5], F[3][5];
  for (int i = 0; i < 3; ++i)
    for (int v = 0; v < 5; ++v) Gm[i][v] = G[i * 5 + v];
  viscous_flux<double>(U, Gm, g, F);
  for (int i = 0; i < 3; ++i)
    for (int v = 0; v < 5; ++v) Fv[i * 5 + v] = F[i][v];
  return 0;
}

// The same RK drivers applied to a scalar ODE (ode 0: y' = lam*y; ode 1: y' = -y^2), so the
// time integrators can be pinned by their convergence order. out[nsteps+1] holds y_0..y_n.
// The Runge-Kutta driver on first-order upwind advection u_j' = u_{j-1} - u_j on a periodic
// grid of n cells (unit spacing; forward Euler keeps it monotone for dt <= 1): u [n] is
// advanced in place by nsteps steps of size dt.
int ora_rk_upwind(int scheme, int n, double dt, int nsteps, double *u) {
  vector<double> y(u, u + n);
  int rc = rk_advance<double>(y, dt, scheme, nsteps, [&](const vector<double> &Y, vector<double> &R) {
    for (int j = 0; j < n; ++j) R[j] = Y[(j + n - 1) % n] - Y[j];
  });
  for (int j = 0; j < n; ++j) u[j] = y[j];
  return rc;
}

// The LSRK45 driver's 2N tables in double precision: A[5], B[5].
int ora_lsrk45_tables(double *A, double *B) {
  lsrk45_tables<double>(A, B);
  return 0;
}

int ora_rk_scalar(int scheme, int ode, double lam, double y0, double dt, int nsteps, double *out) {
  vector<double> y(1, y0);
  out[0] = y0;
  for (int s = 0; s < nsteps; ++s) {
    int rc = rk_advance<double>(y, dt, scheme, 1, [&](const vector<double> &Y, vector<double> &R) {
      R[0] = ode == 0 ? lam * Y[0] : -Y[0] * Y[0];
    });
    if (rc) return rc;
    out[s + 1] = y[0];
  }
  return 0;
}

}  // extern "C"
