// fr_host.cpp -- host-side setup of a mesh: 1-D operators, face pairing and orientation, metric
// terms and face normals. Everything here runs once in fr_mesh_create, in long double, and the
// results are rounded to the device working precision.
//
// Method references (the paper's section "FR Algorithm"):
//   * Eq. (2): nodal Lagrange basis on N_s solution points -> tensor Gauss-Legendre points.
//   * the correction function g chosen so FR equals nodal collocated DG (Huynh's g_DG). At
//     Gauss-Legendre points its derivative is the DG lifting l_a(+-1)/w_a, which is how it is
//     built here.
//   * Eq. (1): J_ij = dx_i/dxi_j and the transformed fluxes |J| J^-1 F. The rows |J| dxi_n/dx
//     are evaluated in the conservative curl form -curl_xi I(X_l grad_xi X_m), (i,m,l) cyclic,
//     of the degree-max(p,1) Gauss-Lobatto interpolant of the geometry, so that sum_n d_n of
//     them vanishes exactly for the discrete operators (a uniform flow stays uniform).
//   * pre-processing: faces are paired by sorting each face's corner vertex ids and matching
//     equal keys (the paper's local face matching).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fr_internal.h"

namespace frh {

using LD = long double;

// ------------------------------------------------------------------------------------------
// 1-D nodes and operators
// ------------------------------------------------------------------------------------------

// (P_n(x), P_n'(x)) by Bonnet's recursion, derivative from the recursion of (1-x^2) P_n'.
static void legendre_pair(int n, LD x, LD *P, LD *dP) {
  LD a = 1, b = x, da = 0, db = 1;
  if (n == 0) { *P = 1; *dP = 0; return; }
  for (int k = 1; k < n; ++k) {
    LD c = ((2 * k + 1) * x * b - k * a) / (k + 1);
    LD dc = da + (2 * k + 1) * b;  // P'_{k+1} = P'_{k-1} + (2k+1) P_k
    a = b; b = c; da = db; db = dc;
  }
  *P = b;
  *dP = db;
}

// Roots of P_n (Gauss-Legendre) or of (1-x^2) P_n' (Gauss-Lobatto with n+1 nodes), ascending.
static std::vector<LD> legendre_roots(int n, bool lobatto) {
  const LD pi = 3.141592653589793238462643383279502884L;
  std::vector<LD> x;
  if (!lobatto) {
    for (int k = n; k >= 1; --k) {
      LD r = std::cos(pi * (k - 0.25L) / (n + 0.5L));
      for (int it = 0; it < 60; ++it) {
        LD P, dP;
        legendre_pair(n, r, &P, &dP);
        LD step = P / dP;
        r -= step;
        if (std::fabs(step) < 1e-21L) break;
      }
      x.push_back(r);
    }
  } else {
    x.push_back(-1);
    for (int k = n - 1; k >= 1; --k) {
      LD r = std::cos(pi * k / n);
      for (int it = 0; it < 60; ++it) {
        LD P, dP;
        legendre_pair(n, r, &P, &dP);
        // root of P_n': Newton on f = P_n' with f' = (2x P_n' - n(n+1) P_n)/(1-x^2)
        LD d2P = (2 * r * dP - n * (n + 1) * P) / (1 - r * r);
        LD step = dP / d2P;
        r -= step;
        if (std::fabs(step) < 1e-21L) break;
      }
      x.push_back(r);
    }
    x.push_back(1);
  }
  std::sort(x.begin(), x.end());
  return x;
}

// Barycentric weights of a node set.
static std::vector<LD> bary_weights(const std::vector<LD> &x) {
  std::vector<LD> w(x.size(), 1);
  for (size_t j = 0; j < x.size(); ++j)
    for (size_t k = 0; k < x.size(); ++k)
      if (k != j) w[j] /= (x[j] - x[k]);
  return w;
}

// Row of Lagrange values l_b(t) (barycentric form; exact node hits handled).
static std::vector<LD> lagrange_row(const std::vector<LD> &x, const std::vector<LD> &bw, LD t) {
  std::vector<LD> r(x.size(), 0);
  for (size_t b = 0; b < x.size(); ++b)
    if (t == x[b]) { r[b] = 1; return r; }
  LD s = 0;
  for (size_t b = 0; b < x.size(); ++b) s += bw[b] / (t - x[b]);
  for (size_t b = 0; b < x.size(); ++b) r[b] = (bw[b] / (t - x[b])) / s;
  return r;
}

// Row of Lagrange derivatives l_b'(t) for arbitrary t (direct product rule on l_b).
static std::vector<LD> lagrange_deriv_row(const std::vector<LD> &x, LD t) {
  const size_t n = x.size();
  std::vector<LD> r(n, 0);
  if (n == 1) return r;
  for (size_t b = 0; b < n; ++b) {
    LD denom = 1;
    for (size_t k = 0; k < n; ++k)
      if (k != b) denom *= (x[b] - x[k]);
    LD num = 0;
    for (size_t m = 0; m < n; ++m) {
      if (m == b) continue;
      LD prod = 1;
      for (size_t k = 0; k < n; ++k)
        if (k != b && k != m) prod *= (t - x[k]);
      num += prod;
    }
    r[b] = num / denom;
  }
  return r;
}

// Dense 1-D matrix rows x cols, row-major.
struct M1 {
  int r = 0, c = 0;
  std::vector<LD> a;
  LD at(int i, int j) const { return a[i * c + j]; }
};

static M1 interp_matrix(const std::vector<LD> &src, const std::vector<LD> &dst) {
  M1 m;
  m.r = (int)dst.size();
  m.c = (int)src.size();
  std::vector<LD> bw = bary_weights(src);
  for (LD t : dst) {
    std::vector<LD> row = lagrange_row(src, bw, t);
    m.a.insert(m.a.end(), row.begin(), row.end());
  }
  return m;
}

static M1 deriv_matrix(const std::vector<LD> &src, const std::vector<LD> &dst) {
  M1 m;
  m.r = (int)dst.size();
  m.c = (int)src.size();
  for (LD t : dst) {
    std::vector<LD> row = lagrange_deriv_row(src, t);
    m.a.insert(m.a.end(), row.begin(), row.end());
  }
  return m;
}

struct Basis {
  int p = 0, n = 1, pg = 1;
  std::vector<LD> xs, ws;  // Gauss-Legendre points, weights
  std::vector<LD> xg;      // Gauss-Lobatto points of degree pg
  std::vector<LD> D, lm, lp, gcL, gcR;
};

static Basis make_basis(int p) {
  Basis B;
  B.p = p;
  B.n = p + 1;
  B.pg = std::max(p, 1);
  B.xs = legendre_roots(B.n, false);
  B.ws.resize(B.n);
  for (int a = 0; a < B.n; ++a) {
    LD P, dP;
    legendre_pair(B.n, B.xs[a], &P, &dP);
    B.ws[a] = 2 / ((1 - B.xs[a] * B.xs[a]) * dP * dP);
  }
  B.xg = legendre_roots(B.pg, true);
  // D via barycentric weights: D_ab = (bw_b / bw_a) / (x_a - x_b), D_aa = -sum of the row
  std::vector<LD> bw = bary_weights(B.xs);
  B.D.assign(B.n * B.n, 0);
  for (int a = 0; a < B.n; ++a) {
    LD diag = 0;
    for (int b = 0; b < B.n; ++b) {
      if (a == b) continue;
      LD v = (bw[b] / bw[a]) / (B.xs[a] - B.xs[b]);
      B.D[a * B.n + b] = v;
      diag -= v;
    }
    B.D[a * B.n + a] = diag;
  }
  B.lm = lagrange_row(B.xs, bw, -1);
  B.lp = lagrange_row(B.xs, bw, 1);
  // g_DG corrections: g_R'(x_a) = l_a(+1) / w_a and g_L'(x_a) = -l_a(-1) / w_a
  B.gcR.resize(B.n);
  B.gcL.resize(B.n);
  for (int a = 0; a < B.n; ++a) {
    B.gcR[a] = B.lp[a] / B.ws[a];
    B.gcL[a] = -B.lm[a] / B.ws[a];
  }
  return B;
}

// ------------------------------------------------------------------------------------------
// Tensor contraction on an element: out(t0,t1,t2) = sum A0(t0,i) A1(t1,j) A2(t2,k) in(i,j,k)
// ------------------------------------------------------------------------------------------
static void contract3(const M1 &A0, const M1 &A1, const M1 &A2, const LD *in, LD *out) {
  const int s = A0.c;
  std::vector<LD> w1((size_t)A2.r * s * s), w2((size_t)A2.r * A1.r * s);
  // z first
  for (int t2 = 0; t2 < A2.r; ++t2)
    for (int j = 0; j < s; ++j)
      for (int i = 0; i < s; ++i) {
        LD acc = 0;
        for (int k = 0; k < s; ++k) acc += A2.at(t2, k) * in[i + s * (j + s * k)];
        w1[i + s * (j + s * t2)] = acc;
      }
  for (int t2 = 0; t2 < A2.r; ++t2)
    for (int t1 = 0; t1 < A1.r; ++t1)
      for (int i = 0; i < s; ++i) {
        LD acc = 0;
        for (int j = 0; j < s; ++j) acc += A1.at(t1, j) * w1[i + s * (j + s * t2)];
        w2[i + s * (t1 + A1.r * t2)] = acc;
      }
  for (int t2 = 0; t2 < A2.r; ++t2)
    for (int t1 = 0; t1 < A1.r; ++t1)
      for (int t0 = 0; t0 < A0.r; ++t0) {
        LD acc = 0;
        for (int i = 0; i < s; ++i) acc += A0.at(t0, i) * w2[i + s * (t1 + A1.r * t2)];
        out[t0 + A0.r * (t1 + A1.r * t2)] = acc;
      }
}

// ------------------------------------------------------------------------------------------
// Face topology
// ------------------------------------------------------------------------------------------
// VTK corner c <-> reference corner bits (bx, by, bz)
static const int kVtk[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                               {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};

static int vtk_index(int bx, int by, int bz) {
  for (int c = 0; c < 8; ++c)
    if (kVtk[c][0] == bx && kVtk[c][1] == by && kVtk[c][2] == bz) return c;
  return -1;
}

// tangential axes of a face normal to direction d, increasing
static inline void tangents(int d, int *u, int *v) {
  *u = (d == 0) ? 1 : 0;
  *v = (d == 2) ? 1 : 2;
}

// corner ids of face f at face-local corner (cu, cv)
static int64_t face_corner(const int64_t *ev, int64_t e, int f, int cu, int cv) {
  int d = f >> 1, s = f & 1, u, v;
  tangents(d, &u, &v);
  int b[3];
  b[d] = s;
  b[u] = cu;
  b[v] = cv;
  return ev[e * 8 + vtk_index(b[0], b[1], b[2])];
}

struct Key4 {
  int64_t v[4];
  bool operator==(const Key4 &o) const { return std::memcmp(v, o.v, sizeof v) == 0; }
};
struct Key4Hash {
  size_t operator()(const Key4 &k) const {
    uint64_t h = 1469598103934665603ull;
    for (int i = 0; i < 4; ++i) {
      h ^= (uint64_t)k.v[i] + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    }
    return (size_t)h;
  }
};

struct Topology {
  std::vector<frk::FaceConn> conn;  // [E*6]
  std::vector<int32_t> perm;        // [E*6*Nfp] neighbour point index of each own point
};

// Returns "" on success or an error message.
static std::string pair_faces(int64_t E, const int64_t *ev, const int32_t *bc_tag, int p, Topology &T) {
  const int n = p + 1, Nfp = n * n;
  T.conn.assign(E * 6, frk::FaceConn{-1, 0});
  T.perm.assign(E * 6 * Nfp, -1);
  std::unordered_map<Key4, int64_t, Key4Hash> open;  // key -> e*6+f of the first side seen
  open.reserve((size_t)E * 4);
  for (int64_t e = 0; e < E; ++e) {
    for (int f = 0; f < 6; ++f) {
      Key4 k;
      k.v[0] = face_corner(ev, e, f, 0, 0);
      k.v[1] = face_corner(ev, e, f, 1, 0);
      k.v[2] = face_corner(ev, e, f, 0, 1);
      k.v[3] = face_corner(ev, e, f, 1, 1);
      std::sort(k.v, k.v + 4);
      if (k.v[0] == k.v[1] || k.v[1] == k.v[2] || k.v[2] == k.v[3])
        return "element " + std::to_string(e) + " face " + std::to_string(f) + " repeats a vertex id";
      auto it = open.find(k);
      if (it == open.end()) {
        open.emplace(k, e * 6 + f);
        continue;
      }
      const int64_t a = it->second;  // first side seen (smaller element, then face): owner
      open.erase(it);
      const int64_t ea = a / 6;
      const int fa = (int)(a % 6);
      // corner correspondence: B's corner holding A's corner (cu, cv)
      int mapu[2][2], mapv[2][2];
      for (int cu = 0; cu < 2; ++cu)
        for (int cv = 0; cv < 2; ++cv) {
          int64_t id = face_corner(ev, ea, fa, cu, cv);
          bool found = false;
          for (int bu = 0; bu < 2 && !found; ++bu)
            for (int bv = 0; bv < 2 && !found; ++bv)
              if (face_corner(ev, e, f, bu, bv) == id) { mapu[cu][cv] = bu; mapv[cu][cv] = bv; found = true; }
          if (!found) return "faces of elements " + std::to_string(ea) + " and " + std::to_string(e) + " do not share corners";
        }
      // A's local axes expressed in B's: u-axis of A maps along B's axis au, etc.
      auto build = [&](int64_t e1, int f1, int64_t e2, int f2, bool owner,
                       const int mu[2][2], const int mv[2][2]) -> std::string {
        // e1 point (a, b) -> e2 point; corners: (cu,cv) of e1 -> (mu[cu][cv], mv[cu][cv]) of e2
        bool swap = mu[1][0] == mu[0][0];  // moving along e1's u leaves e2's u unchanged
        int flip_u, flip_v;
        if (!swap) {
          flip_u = mu[0][0];
          flip_v = mv[0][0];
          if (mu[1][0] == mu[0][0] || mv[0][1] == mv[0][0]) return "degenerate face orientation";
        } else {
          // e1's u runs along e2's v and e1's v along e2's u
          flip_u = mu[0][0];  // e2 u-coordinate at e1's origin
          flip_v = mv[0][0];
          if (mv[1][0] == mv[0][0] || mu[0][1] == mu[0][0]) return "degenerate face orientation";
        }
        // consistency on the far corner
        int eu = swap ? (flip_u ? 0 : 1) : (flip_u ? 0 : 1);
        int evv = swap ? (flip_v ? 0 : 1) : (flip_v ? 0 : 1);
        if (mu[1][1] != eu || mv[1][1] != evv) return "inconsistent face corners";
        frk::FaceConn &c = T.conn[e1 * 6 + f1];
        c.nbr = (int32_t)e2;
        c.code = f2 | (swap ? 8 : 0) | (flip_u ? 16 : 0) | (flip_v ? 32 : 0) | (owner ? 64 : 0);
        for (int b = 0; b < n; ++b)
          for (int a2 = 0; a2 < n; ++a2) {
            int uu = swap ? b : a2, vv = swap ? a2 : b;
            int up = flip_u ? p - uu : uu, vp = flip_v ? p - vv : vv;
            T.perm[(e1 * 6 + f1) * Nfp + a2 + n * b] = up + n * vp;
          }
        return "";
      };
      std::string err = build(ea, fa, e, f, true, mapu, mapv);
      if (!err.empty()) return err;
      // inverse map for B -> A
      int iu[2][2], iv[2][2];
      for (int cu = 0; cu < 2; ++cu)
        for (int cv = 0; cv < 2; ++cv) {
          iu[mapu[cu][cv]][mapv[cu][cv]] = cu;
          iv[mapu[cu][cv]][mapv[cu][cv]] = cv;
        }
      err = build(e, f, ea, fa, false, iu, iv);
      if (!err.empty()) return err;
    }
  }
  // unpaired faces: isothermal no-slip walls where tagged (owned by their element, no
  // neighbour, identity point map), an error otherwise
  for (const auto &kv : open) {
    const int64_t a = kv.second;
    if (!bc_tag || bc_tag[a] != 1)
      return "unpaired face: element " + std::to_string(a / 6) + " face " + std::to_string(a % 6) +
             " (every face must pair or be tagged as a wall)";
    T.conn[a] = frk::FaceConn{-1, (int32_t)(64 | 128)};
    for (int k = 0; k < Nfp; ++k) T.perm[a * Nfp + k] = k;
  }
  return "";
}

// ------------------------------------------------------------------------------------------
// Geometry
// ------------------------------------------------------------------------------------------
struct Geometry {
  // per element, long double
  std::vector<double> xyz;     // [E][3][Ns] solution-point coordinates
  std::vector<LD> ja;          // [E][Ns][9] Ja[n][i]
  std::vector<LD> detj;        // [E][Ns]
  std::vector<LD> nface;       // [E][6][Nfp][3] own outward N = s Ja^d at face points
  std::vector<LD> jface;       // [E][6][Nfp] |J| interpolated to face points
  int64_t bad_elem = -1;
};

// 1-D matrices reused by every element of a mesh.
struct GeoOps {
  M1 up, Dg, Ig, Is, Ds, Ie[2], De[2];
};

static GeoOps make_geo_ops(const Basis &B, int q) {
  GeoOps O;
  std::vector<LD> xq = legendre_roots(q, true);
  O.up = interp_matrix(xq, B.xg);
  O.Dg = deriv_matrix(B.xg, B.xg);
  O.Ig = interp_matrix(B.xg, B.xg);
  O.Is = interp_matrix(B.xg, B.xs);
  O.Ds = deriv_matrix(B.xg, B.xs);
  std::vector<LD> m1{-1.0L}, p1{1.0L};
  O.Ie[0] = interp_matrix(B.xg, m1);
  O.Ie[1] = interp_matrix(B.xg, p1);
  O.De[0] = deriv_matrix(B.xg, m1);
  O.De[1] = deriv_matrix(B.xg, p1);
  return O;
}

static void element_geometry(const Basis &B, const GeoOps &O, int q, const double *nodes, int64_t e, Geometry &G) {
  const int n = B.n, Ns = n * n * n, Nfp = n * n, ng = B.pg + 1, NG = ng * ng * ng, nq = q + 1;
  const M1 &up = O.up, &Dg = O.Dg, &Ig = O.Ig, &Is = O.Is, &Ds = O.Ds;
  const M1 *Ie = O.Ie, *De = O.De;

  // geometry nodes at degree-pg GLL points
  std::vector<LD> X(3 * NG), src(nq * nq * nq);
  for (int c = 0; c < 3; ++c) {
    for (int m = 0; m < nq * nq * nq; ++m) src[m] = (LD)nodes[((size_t)e * nq * nq * nq + m) * 3 + c];
    contract3(up, up, up, src.data(), &X[c * NG]);
  }
  // element-local coordinates (shifted by the first node): only derivatives of X enter the
  // metric terms, and without the shift their round-off would grow with |X| / h
  LD xorig[3];
  for (int c = 0; c < 3; ++c) {
    xorig[c] = X[c * NG];
    for (int g = 0; g < NG; ++g) X[c * NG + g] -= xorig[c];
  }
  // grad X at the GLL nodes: dX[(c*3+k)*NG]
  std::vector<LD> dX(9 * NG);
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < 3; ++k)
      contract3(k == 0 ? Dg : Ig, k == 1 ? Dg : Ig, k == 2 ? Dg : Ig, &X[c * NG], &dX[(c * 3 + k) * NG]);
  // W[i][k] = X_l d_k X_m at the nodes, (i, m, l) cyclic (local X: the curl of a constant
  // times a gradient is zero, so the shift leaves the metric unchanged)
  std::vector<LD> W(9 * NG);
  for (int i = 0; i < 3; ++i) {
    int m = (i + 1) % 3, l = (i + 2) % 3;
    for (int k = 0; k < 3; ++k)
      for (int g = 0; g < NG; ++g) W[(i * 3 + k) * NG + g] = X[l * NG + g] * dX[(m * 3 + k) * NG + g];
  }
  // evaluate Ja at a tensor target set described by interpolation rows (T[3]) and derivative
  // rows (Td[3]) per direction; out[t][n*3+i]
  auto curl_at = [&](const M1 *T[3], const M1 *Td[3], int NT, LD *out) {
    std::vector<LD> t1(NT), t2(NT);
    for (int i = 0; i < 3; ++i)
      for (int nn = 0; nn < 3; ++nn) {
        int a1 = (nn + 1) % 3, a2 = (nn + 2) % 3;
        const M1 *P1[3] = {T[0], T[1], T[2]};
        P1[a1] = Td[a1];
        contract3(*P1[0], *P1[1], *P1[2], &W[(i * 3 + a2) * NG], t1.data());
        const M1 *P2[3] = {T[0], T[1], T[2]};
        P2[a2] = Td[a2];
        contract3(*P2[0], *P2[1], *P2[2], &W[(i * 3 + a1) * NG], t2.data());
        for (int t = 0; t < NT; ++t) out[t * 9 + nn * 3 + i] = t2[t] - t1[t];
      }
  };
  {
    const M1 *T[3] = {&Is, &Is, &Is}, *Td[3] = {&Ds, &Ds, &Ds};
    curl_at(T, Td, Ns, &G.ja[(size_t)e * Ns * 9]);
  }
  // coordinates and |J| at the solution points
  std::vector<LD> xs(Ns), J(9 * Ns);
  for (int c = 0; c < 3; ++c) {
    contract3(Is, Is, Is, &X[c * NG], xs.data());
    for (int s = 0; s < Ns; ++s) G.xyz[((size_t)e * 3 + c) * Ns + s] = (double)(xs[s] + xorig[c]);
    for (int k = 0; k < 3; ++k)
      contract3(k == 0 ? Ds : Is, k == 1 ? Ds : Is, k == 2 ? Ds : Is, &X[c * NG], &J[(c * 3 + k) * Ns]);
  }
  for (int s = 0; s < Ns; ++s) {
    auto j = [&](int c, int k) { return J[(c * 3 + k) * Ns + s]; };
    LD det = j(0, 0) * (j(1, 1) * j(2, 2) - j(2, 1) * j(1, 2)) - j(1, 0) * (j(0, 1) * j(2, 2) - j(2, 1) * j(0, 2)) +
             j(2, 0) * (j(0, 1) * j(1, 2) - j(1, 1) * j(0, 2));
    G.detj[(size_t)e * Ns + s] = det;
    if (!(det > 0)) G.bad_elem = e;
  }
  // faces
  std::vector<LD> jaf(Nfp * 9);
  for (int f = 0; f < 6; ++f) {
    int d = f >> 1, sd = f & 1;
    const M1 *T[3] = {&Is, &Is, &Is}, *Td[3] = {&Ds, &Ds, &Ds};
    T[d] = &Ie[sd];
    Td[d] = &De[sd];
    curl_at(T, Td, Nfp, jaf.data());
    LD sg = sd ? 1 : -1;
    for (int k = 0; k < Nfp; ++k)
      for (int i = 0; i < 3; ++i) G.nface[(((size_t)e * 6 + f) * Nfp + k) * 3 + i] = sg * jaf[k * 9 + d * 3 + i];
    // |J| at the face points by interpolating the solution-point values along the normal line
    const std::vector<LD> &ell = sd ? B.lp : B.lm;
    int u, v;
    tangents(d, &u, &v);
    for (int b = 0; b < n; ++b)
      for (int a = 0; a < n; ++a) {
        LD acc = 0;
        for (int c = 0; c < n; ++c) {
          int idx[3];
          idx[d] = c;
          idx[u] = a;
          idx[v] = b;
          acc += ell[c] * G.detj[(size_t)e * Ns + idx[0] + n * (idx[1] + n * idx[2])];
        }
        G.jface[((size_t)e * 6 + f) * Nfp + a + n * b] = acc;
      }
  }
}

}  // namespace frh

// ==========================================================================================
// Entry used by the C ABI: builds every host-side array of a mesh.
// ==========================================================================================
namespace frk {

Ops1D basis_ops(int p) {
  frh::Basis B = frh::make_basis(p);
  Ops1D o;
  std::memset(&o, 0, sizeof o);
  const int n = p + 1;
  for (int i = 0; i < n * n; ++i) o.D[i] = (double)B.D[i];
  for (int i = 0; i < n; ++i) {
    o.lm[i] = (double)B.lm[i];
    o.lp[i] = (double)B.lp[i];
    o.gcL[i] = (double)B.gcL[i];
    o.gcR[i] = (double)B.gcR[i];
  }
  return o;
}

SgsOps sgs_ops(int p) {
  frh::Basis B = frh::make_basis(p);
  SgsOps o;
  std::memset(&o, 0, sizeof o);
  const int n = p + 1;
  for (int a = 0; a < n; ++a)
    for (int i = 0; i < n; ++i) {
      frh::LD P, dP;
      frh::legendre_pair(a, B.xs[i], &P, &dP);
      o.Lm[a * n + i] = (double)(std::sqrt((frh::LD)(2 * a + 1) / 2) * P * B.ws[i]);
    }
  for (int i = 0; i < n; ++i) o.w[i] = (double)B.ws[i];
  return o;
}

std::string build_host_mesh(int p, int q, int64_t E, const int64_t *ev, const double *nodes, const int32_t *bc_tag,
                            double eta, HostMesh &H) {
  using frh::LD;
  H.p = p;
  H.q = q;
  H.E = E;
  const int n = p + 1, Ns = n * n * n, Nfp = n * n;
  frh::Basis B = frh::make_basis(p);
  H.ops = basis_ops(p);
  frh::Topology T;
  std::string err = frh::pair_faces(E, ev, bc_tag, p, T);
  if (!err.empty()) return err;

  frh::Geometry G;
  G.xyz.assign((size_t)E * 3 * Ns, 0);
  G.ja.assign((size_t)E * Ns * 9, 0);
  G.detj.assign((size_t)E * Ns, 0);
  G.nface.assign((size_t)E * 6 * Nfp * 3, 0);
  G.jface.assign((size_t)E * 6 * Nfp, 0);
  const frh::GeoOps O = frh::make_geo_ops(B, q);
  unsigned nth = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < nth; ++t)
    pool.emplace_back([&, t]() {
      for (int64_t e = t; e < E; e += nth) frh::element_geometry(B, O, q, nodes, e, G);
    });
  for (auto &th : pool) th.join();
  for (int64_t e = 0; e < E; ++e)
    for (int s = 0; s < Ns; ++s)
      if (!(G.detj[(size_t)e * Ns + s] > 0)) return "non-positive Jacobian in element " + std::to_string(e);

  H.xyz = std::move(G.xyz);
  H.geo.assign((size_t)E * 10 * Ns, 0);
  for (int64_t e = 0; e < E; ++e)
    for (int s = 0; s < Ns; ++s) {
      for (int t = 0; t < 9; ++t) H.geo[((size_t)e * 10 + t) * Ns + s] = (double)G.ja[((size_t)e * Ns + s) * 9 + t];
      // 1/|J| from the rounded |J|, as a double division
      H.geo[((size_t)e * 10 + 9) * Ns + s] = 1.0 / (double)G.detj[(size_t)e * Ns + s];
    }
  // faces in owner order: the owner's outward normal and the BR2 factor
  // sigma = eta (p+1)^2/2 (1/|J|_L + 1/|J|_R) / 4 per face point
  H.conn = T.conn;
  H.ftab.clear();
  H.fref.assign((size_t)E * 6, FaceRef{-1, 0});
  const LD cl = (LD)(n * n) / 2;
  for (int64_t e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      const FaceConn c = T.conn[e * 6 + f];
      if (!((c.code >> 6) & 1)) continue;
      const int32_t fid = (int32_t)H.ftab.size();
      if (c.nbr < 0) {  // a wall: no other side
        H.ftab.push_back(FaceRec{(int32_t)e, -1, f | kFaceWall, 0});
        H.fref[e * 6 + f] = FaceRef{fid, 64};
        ++H.n_wall;
        continue;
      }
      const int fn = c.code & 7;
      FaceRec r;
      r.eL = (int32_t)e;
      r.eR = c.nbr;
      r.code = f | (fn << 3) | (((c.code >> 3) & 7) << 6);
      r.pad = 0;
      H.ftab.push_back(r);
      H.fref[e * 6 + f] = FaceRef{fid, 64};
      // the other side maps its points to the owner's with its own FaceConn bits
      const FaceConn co = T.conn[(size_t)c.nbr * 6 + fn];
      H.fref[(size_t)c.nbr * 6 + fn] = FaceRef{fid, co.code & (8 | 16 | 32)};
    }
  const int64_t F = (int64_t)H.ftab.size();
  H.fgeo.assign((size_t)F * 4 * Nfp, 0);
  for (int64_t fid = 0; fid < F; ++fid) {
    const FaceRec &r = H.ftab[fid];
    const int fL = r.code & 7, fR = (r.code >> 3) & 7;
    double *dst = &H.fgeo[(size_t)fid * 4 * Nfp];
    for (int k = 0; k < Nfp; ++k) {
      for (int i = 0; i < 3; ++i) dst[i * Nfp + k] = (double)G.nface[(((size_t)r.eL * 6 + fL) * Nfp + k) * 3 + i];
      const double jl = (double)G.jface[((size_t)r.eL * 6 + fL) * Nfp + k];
      if (r.eR < 0) {
        // wall: the one-sided lifting, as if the other side's |J| equalled this side's
        dst[3 * Nfp + k] = (double)((LD)eta * cl * (2.0L / (LD)jl) / 4);
        continue;
      }
      const int kr = T.perm[((size_t)r.eL * 6 + fL) * Nfp + k];
      const double jr = (double)G.jface[((size_t)r.eR * 6 + fR) * Nfp + kr];
      dst[3 * Nfp + k] = (double)((LD)eta * cl * (1.0L / (LD)jl + 1.0L / (LD)jr) / 4);
    }
  }
  return "";
}

std::string build_partition(const HostMesh &G, const int32_t *part, int n_part, int which, HostPart &P) {
  const int64_t E = G.E;
  const int n = G.p + 1, Ns = n * n * n, Nfp = n * n;
  std::vector<int64_t> loc((size_t)E, -1);
  P.elems.clear();
  for (int64_t e = 0; e < E; ++e) {
    if (part[e] < 0 || part[e] >= n_part) return "element " + std::to_string(e) + " has a part outside 0..n_part-1";
    if (part[e] == which) {
      loc[e] = (int64_t)P.elems.size();
      P.elems.push_back(e);
    }
  }
  const int64_t El = (int64_t)P.elems.size();
  if (El == 0) return "part " + std::to_string(which) + " has no elements";
  HostMesh &H = P.H;
  H.p = G.p;
  H.q = G.q;
  H.E = El;
  H.n_wall = 0;
  H.ops = G.ops;
  H.geo.resize((size_t)El * 10 * Ns);
  H.xyz.resize((size_t)El * 3 * Ns);
  H.conn.assign((size_t)El * 6, FaceConn{-1, 0});
  for (int64_t l = 0; l < El; ++l) {
    const int64_t e = P.elems[l];
    std::copy(&G.geo[(size_t)e * 10 * Ns], &G.geo[(size_t)(e + 1) * 10 * Ns], &H.geo[(size_t)l * 10 * Ns]);
    std::copy(&G.xyz[(size_t)e * 3 * Ns], &G.xyz[(size_t)(e + 1) * 3 * Ns], &H.xyz[(size_t)l * 3 * Ns]);
  }
  H.ftab.clear();
  H.fgeo.clear();
  H.fref.assign((size_t)El * 6, FaceRef{-1, 0});
  P.send.assign(n_part, {});
  P.recv.assign(n_part, {});
  P.n_ghost = 0;
  // every face with a side in this part, in the whole mesh's face order
  for (size_t fid = 0; fid < G.ftab.size(); ++fid) {
    const FaceRec r = G.ftab[fid];
    const int fL = r.code & 7, fR = (r.code >> 3) & 7;
    const bool wall = (r.code & kFaceWall) != 0;
    const bool inL = loc[r.eL] >= 0;
    const bool inR = !wall && loc[r.eR] >= 0;
    if (!inL && !inR) continue;
    FaceRec lr = r;
    const int32_t lid = (int32_t)H.ftab.size();
    if (inL) {
      lr.eL = (int32_t)loc[r.eL];
      H.fref[(size_t)lr.eL * 6 + fL] = FaceRef{lid, G.fref[(size_t)r.eL * 6 + fL].code};
    } else {  // the owner side is another part's: a ghost slot
      const int64_t g = P.n_ghost++;
      lr.eL = (int32_t)(El + g / 6);
      lr.code = (lr.code & ~7) | (int32_t)(g % 6);
      P.recv[part[r.eL]].push_back((int32_t)g);
      P.send[part[r.eL]].push_back((int32_t)(loc[r.eR] * 6 + fR));
    }
    if (wall) {
      ++H.n_wall;
    } else if (inR) {
      lr.eR = (int32_t)loc[r.eR];
      H.fref[(size_t)lr.eR * 6 + fR] = FaceRef{lid, G.fref[(size_t)r.eR * 6 + fR].code};
    } else {
      const int64_t g = P.n_ghost++;
      lr.eR = (int32_t)(El + g / 6);
      lr.code = (lr.code & ~(7 << 3)) | (int32_t)((g % 6) << 3);
      P.recv[part[r.eR]].push_back((int32_t)g);
      P.send[part[r.eR]].push_back((int32_t)(loc[r.eL] * 6 + fL));
    }
    H.ftab.push_back(lr);
    H.fgeo.insert(H.fgeo.end(), &G.fgeo[fid * 4 * Nfp], &G.fgeo[(fid + 1) * 4 * Nfp]);
  }
  if (El * 6 + P.n_ghost > (int64_t)INT32_MAX) return "too many face slots in part " + std::to_string(which);
  return "";
}

}  // namespace frk
