// fr_internal.h -- library-private declarations shared by the host setup (fr_host.cpp), the HIP
// kernels and entry points (fr_kernels.hip, fr_kernels32.hip, fr_mlp.hip) and the partition
// groups (fr_partition.hip). Not part of the C ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "fr.h"

struct fr_mlp_s;

namespace frk {

constexpr int kMaxP = 7;
constexpr int kMaxN = kMaxP + 1;

// 1-D operator tables of degree p on the Gauss-Legendre solution points, passed to kernels
// by value (they live in the kernel-argument segment).
struct Ops1D {
  double D[kMaxN * kMaxN];  // D[a*n + b] = l_b'(x_a)
  double lm[kMaxN];         // l_b(-1)
  double lp[kMaxN];         // l_b(+1)
  double gcL[kMaxN];        // correction from the face at xi = -1, multiplied by its sign -1:
                            // the derivative of g_L at x_a
  double gcR[kMaxN];        // derivative of g_R at x_a (face at xi = +1)
};

// Tables of the closure's features: Lm[a*n + i] = orthonormal Legendre a at x_i times the
// Gauss weight w_i (the modal projection), and the weights w.
struct SgsOps {
  double Lm[kMaxN * kMaxN];
  double w[kMaxN];
};

struct Ops1Df {
  float D[kMaxN * kMaxN];
  float lm[kMaxN];
  float lp[kMaxN];
  float gcL[kMaxN];
  float gcR[kMaxN];
};

// Per element face: packed neighbour information.
//   nbr   : neighbour element index
//   code  : bits 0-2 neighbour's local face, bit 3 swap, bit 4 flip u, bit 5 flip v,
//           bit 6 this side owns the face (its normal is the face's normal)
// Point (a, b) of this face is point (u', v') of the neighbour's face with
//   (u, v) = swap ? (b, a) : (a, b); u' = flip_u ? p - u : u; v' = flip_v ? p - v : v.
struct FaceConn {
  int32_t nbr;
  int32_t code;
};

// Per element face, for the volume kernel: the face record index and the map from this
// side's face point to the owner's (the same bits as FaceConn.code; identity for the owner).
struct FaceRef {
  int32_t fid;
  int32_t code;
};

struct Physics {
  double gamma;
  double prandtl;
  double mu;
  double kappa;  // mu * gamma / (prandtl * (gamma - 1)): heat-flux coefficient on d(p/rho)
};

// One face (owner side "L", other side "R"), the unit of the face kernel.
//   eL, eR : elements; code: bits 0-2 L's local face, 3-5 R's local face, 6 swap, 7 flip u,
//   8 flip v -- the map from L's face point (a, b) to R's point, as in FaceConn; bit 9
//   (kFaceWall) an isothermal no-slip wall, with eR = -1.
constexpr int32_t kFaceWall = 1 << 9;
struct FaceRec {
  int32_t eL;
  int32_t eR;
  int32_t code;
  int32_t pad;
};

// RK stage parameters for the volume kernel.
enum StageMode : int32_t {
  kModeResidual = 0,  // write R
  kModeLSRK = 1,      // dU <- a dU + dt R; U <- U + b dU   (a == 0: dU is not read)
  kModeRK4 = 2,       // acc <- (first ? 0 : acc) + w R; S <- Q + cdt R, or Q <- Q + dt acc
  kModeSSP = 3        // ten-stage SSP method, two registers q1 = U and q2 (see rk_store)
};

struct StageArgs {
  int32_t mode;
  int32_t first;  // RK4: first stage (acc not read); LSRK: a == 0
  int32_t last;   // RK4: last stage (Q updated instead of S)
  int32_t stage;  // SSP: stage index 0..9
  double a, b, dt;  // LSRK coefficients and step
  double w, cdt;    // RK4 weight and next-stage offset c_{i+1} * dt
  double g[3];      // body force per unit mass (source term), applied when force != 0
  int32_t force;
  int32_t pre_done;  // host: the face buffer already holds this stage's pre-pass
  int32_t pre_next;  // the volume kernel also writes the next stage's pre-pass
  int32_t pre_only;  // host: launch the stage's pre-pass and nothing else (partition groups
                     // exchange the face data between the pre-pass and the face kernel)
};

// Device buffers of one mesh (FP64 or FP32 operator path; the state is always FP64).
struct DeviceMesh {
  int p, n, Ns, Nfp;
  int64_t E;
  int prec;
  int flux;
  bool viscous;
  double eta;
  Physics phys;
  Ops1D ops;
  Ops1Df opsf;
  // state registers [E][5][Ns] doubles
  double *U = nullptr;   // solution (LSRK: U; RK4: Q)
  double *R1 = nullptr;  // LSRK: dU; RK4: accumulator
  double *R2 = nullptr;  // RK4: stage state S
  // geometry
  void *geo = nullptr;    // [E][10][Ns]: Ja[n][i] (9, n-major) then 1/|J|  (double or float)
  int64_t F = 0;          // number of faces
  void *fgeo = nullptr;   // [F][4][Nfp]: owner's outward scaled normal N (3), BR2 factor sigma
  FaceRec *ftab = nullptr;   // [F]
  FaceRef *fref = nullptr;   // [E][6]
  void *face = nullptr;   // [E][6][20][Nfp]: U_f (5) then broken gradient G[i][v] (15, i-major)
  void *fout = nullptr;   // [F][10][Nfp]: J = (U_R - U_L)/2 (5), owner's F^{I,perp} (5)
  // FP32 form (prec == 1): FP32 copies of the volume geometry and of the face data; the
  // momentum at face points and the mass fluxes stay FP64
  void *geo32 = nullptr;    // [E][10][Ns] float
  void *face32 = nullptr;   // [E][6][20][Nfp] float: U - U_ref (5), broken gradient (15)
  void *facem = nullptr;    // [E][6][3][Nfp] double: momentum at the face points
  void *fout32 = nullptr;   // [F][9][Nfp] float: J (5), owner's momentum flux (3), reduced energy flux
  void *foutm = nullptr;    // [F][Nfp] double: owner's mass flux
  double ref_rho = 1.0, ref_p = 0.0;
  int tile_epb = 0;             // element kernels: 0 = 256/Ns elements per block, 1 = half
  int tile_fbs = 0;             // face kernel block: 0 = 256, 1 = 128, 2 = 64 threads
  bool fuse = true;             // each stage's volume kernel runs the next stage's pre-pass
  bool walls = false;           // isothermal no-slip wall faces present
  double wall_T = 1.0;          // their temperature p/rho
  bool ldg = false;             // LDG common viscous flux (else BR2)
  double ldg_tau = 0.0;
  double force[3] = {0, 0, 0};  // body force per unit mass (source term S)
  bool has_force = false;
  // learned eddy-viscosity closure (FP64 path only)
  int sgs = 0;                 // 0 off, 1 fixed per-element nu_t, 2 nu_t from the model per stage
  double *nut = nullptr;       // [E] eddy kinematic viscosity
  float *feat = nullptr;       // [E][Ns + 4] model inputs
  fr_mlp_s *model = nullptr;
  double nu_scale = 0.0, prandtl_t = 0.9;
  SgsOps sgs_ops;
  int64_t n_ghost = 0;    // face slots after the 6E local ones in face / face32 / facem: the
                          // other parts' faces of a partition group, filled by the halo unpack
  int *flag = nullptr;    // non-finite flag
  bool check_finite = false;
  void *stream = nullptr;
  int64_t bytes = 0;
};

// Host-side arrays of a mesh, built once by build_host_mesh (fr_host.cpp); for a part of a
// partition group, by build_partition from the whole mesh's.
struct HostMesh {
  int p = 0, q = 1;
  int64_t E = 0;
  int64_t n_wall = 0;          // wall faces
  Ops1D ops;
  std::vector<double> geo;     // [E][10][Ns]
  std::vector<double> fgeo;    // [F][4][Nfp]
  std::vector<FaceConn> conn;  // [E][6]
  std::vector<FaceRec> ftab;   // [F]
  std::vector<FaceRef> fref;   // [E][6]
  std::vector<double> xyz;     // [E][3][Ns]
};

// Enqueue one RK stage (or a residual) of the FP32 form (fr_kernels32.hip); 0 or a negative
// FR_ERR_* code with `err` set. ms (optional) accumulates the three kernel durations.
int launch_stage32(DeviceMesh &dm, const double *X, StageArgs st, double *o, double *r1, double *r2, double *ms,
                   std::string &err);

// Batches of FP32-form meshes advanced by multi-mesh kernels (fr_kernels32.hip): a group holds
// meshes of one degree (viscous, no closure or LDG, one fusion setting, one tile setting);
// group32_step enqueues `steps` RK steps of every mesh with one launch per kernel and stage
// covering all of them. 0 or a negative FR_ERR_* code with `err` set.
struct Group32;
bool group32_eligible(const DeviceMesh &dm);
int group32_create(const std::vector<DeviceMesh *> &meshes, const std::vector<double> &dt, int scheme, Group32 **out,
                   std::string &err);
int group32_step(Group32 *g, void *stream, int steps, std::string &err);
void group32_destroy(Group32 *g);
int group32_items(const Group32 *g, int64_t *elem_items, int64_t *face_items);

// 1-D operator tables of degree p (computed in long double, rounded to double).
Ops1D basis_ops(int p);
SgsOps sgs_ops(int p);

// Records msg as the thread's last error and returns code (fr_last_error).
int fr_fail(int code, const std::string &msg);

// The closure network (fr_mlp.hip): its input count, and nu[s] = nu_scale * model(X[s]) for
// s < n, enqueued on `stream`.
int mlp_n_in(fr_mlp_s *m);
int mlp_forward_nu(fr_mlp_s *m, const float *X, int64_t n, int64_t ldx, double *nu, double nu_scale,
                   void *stream);

// Returns "" on success or a message naming the offending element / face.
std::string build_host_mesh(int p, int q, int64_t E, const int64_t *elem_vert, const double *elem_nodes,
                            const int32_t *bc_tag, double br2_eta, HostMesh &H);

// One part of a mesh split into parts by an element -> part map (the paper's pre-processor splits
// the mesh across processes; section "Pre-processor Parallelization"). Its elements are the
// part's, in increasing global order. Its face list is every face of the whole mesh (in the whole
// mesh's owner order) with at least one side in the part, with the whole mesh's normals, BR2
// factors and orientation codes; a side in another part is a ghost face slot 6 E_loc + g of the
// face buffer, written as element E_loc + g / 6 and local face g % 6 of the face record. send[q]
// lists the face-buffer slots (6 e + f) of the part's own faces whose other side is in part q,
// recv[q] the ghost slots g those faces of part q fill; both in the whole mesh's face order, so
// part a's send[b] and part b's recv[a] name the same faces in the same order.
struct HostPart {
  std::vector<int64_t> elems;  // local -> global element index
  HostMesh H;                  // the part's arrays (E = elems.size())
  int64_t n_ghost = 0;
  std::vector<std::vector<int32_t>> send, recv;  // [n_part]
};

std::string build_partition(const HostMesh &G, const int32_t *part, int n_part, int which, HostPart &P);

// Stage plumbing shared by the single-mesh entry points (fr_kernels.hip) and the partition
// groups (fr_partition.hip).
int n_stages(int scheme);  // 4, 5 or 10; 0 for an unknown scheme

// Elements per block of the element kernels for tile choice `epb` (0 or 1) at Ns solution
// points, as the kernels' Cfg<P>::EPB and Cfg<P>::EPB2 give it: 256/Ns (at least one, at most
// 64), then half of it, or two where one element leaves lanes of its last wave idle.
inline int tile_elements(int Ns, int epb) {
  const int e0 = (256 / Ns) > 64 ? 64 : ((256 / Ns) > 0 ? (256 / Ns) : 1);
  if (epb == 0) return e0;
  return e0 > 1 ? e0 / 2 : (Ns % 64 != 0 && 2 * Ns <= 1024 ? 2 : 1);
}
// The register update of stage s of `scheme` with step dt (st.mode, coefficients) and the state,
// output and register arrays that stage reads and writes on the handle's buffers.
void stage_setup(DeviceMesh &dm, int scheme, int s, double dt, StageArgs &st, const double **X, double **out0,
                 double **reg1, double **reg2);
int ensure_registers(DeviceMesh &dm, int scheme);
// Enqueue one stage (or its pre-pass alone, st.pre_only) with the handle's source term; 0 or an
// FR_ERR_* code with the message set.
int enqueue_stage(DeviceMesh &dm, const double *X, StageArgs st, double *out0, double *reg1, double *reg2);

}  // namespace frk

// The opaque mesh handle of the C ABI.
struct fr_part_s;
struct fr_mesh_s {
  uint64_t magic;
  frk::DeviceMesh dm;
  std::vector<double> xyz;
  int device;
  // a part of a partition group (fr_part_create): the group owns it; the device lists of face
  // slots exchanged with each other part (send: own faces packed for part q; recv: ghost slots
  // unpacked from part q) and their lengths in faces
  fr_part_s *group = nullptr;
  std::vector<int32_t *> send_slots, recv_slots;
  std::vector<int64_t> n_send, n_recv;
};

namespace frk {
constexpr uint64_t kMeshMagic = 0x46524d4553484d31ull;  // "FRMESHM1"
inline bool valid_mesh(const fr_mesh_s *m) { return m != nullptr && m->magic == kMeshMagic; }
// The argument checks of fr_mesh_create, and the host setup with its wall checks; 0 or an
// FR_ERR_* code with the message set.
int validate_desc(const fr_mesh_desc *d);
int host_mesh_of(const fr_mesh_desc *d, HostMesh &H);
// Device buffers of a mesh from its host arrays (n_ghost extra face slots); *out on success.
int create_device_mesh(const fr_mesh_desc *d, HostMesh &H, int64_t n_ghost, void *stream, fr_mesh_s **out);
// Free a handle's device memory and the handle (waits for its stream).
int destroy_device_mesh(fr_mesh_s *m);
}  // namespace frk
