/* fr.h -- C ABI of libfr: the flux-reconstruction (FR) residual and Runge-Kutta stage update
 * of the 3-D compressible Navier-Stokes equations on hexahedral meshes, on one AMD MI355X
 * (gfx950) GPU.
 *
 * The discretisation is the paper's (section "FR Algorithm"):
 *   Eq. (1)  the conservation law mapped to each element's reference cube, with the
 *            transformed solution |J| Q and transformed fluxes |J| J^-1 F;
 *   Eq. (2)  nodal Lagrange representation on N_s = (p+1)^3 solution points
 *            (tensor Gauss-Legendre points, index i + (p+1)*(j + (p+1)*k), xi fastest);
 *   Eq. (3)  the semi-discrete update dQ/dt = -|J|^-1 [div_xi F^ + sum over faces and flux
 *            points of div_xi g (F^{I,perp} - F^{perp})], with the correction function g
 *            that makes FR equal to nodal collocated DG (Radau g_DG), an approximate Riemann
 *            solver for the common inviscid flux, and BR2 liftings for the viscous flux.
 * Time integration is an explicit Runge-Kutta method.
 *
 * Conventions shared by every call:
 *   - All functions return int: FR_OK (0) or a negative FR_ERR_* code. None aborts or throws.
 *     fr_last_error() returns a thread-local message describing the last failure.
 *   - State layout (the external layout of every state/residual array):
 *     [n_elem][5][N_s] doubles, variables (rho, rho u, rho v, rho w, E), points innermost.
 *   - "on_device" = 1: the pointer is device memory on the handle's GPU; the call is enqueued
 *     on the handle's stream and returns without waiting. "on_device" = 0: host memory; the
 *     call waits for the stream before returning.
 *   - Arrays passed in are borrowed for the duration of the call only (deep-copied where
 *     kept). The handle owns all device memory it allocates and frees it in fr_mesh_destroy.
 */
#ifndef FR_H
#define FR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fr_mesh_s *fr_mesh_t; /* opaque handle */

enum fr_status {
  FR_OK = 0,
  FR_ERR_ARG = -1,         /* bad argument (null pointer, range, unknown enum, foreign handle) */
  FR_ERR_MESH = -2,        /* invalid mesh: unpaired face, inconsistent corners, |J| <= 0 */
  FR_ERR_HIP = -3,         /* a HIP runtime call failed */
  FR_ERR_OOM = -4,         /* device allocation failed */
  FR_ERR_UNSUPPORTED = -5, /* a valid request this build does not implement */
  FR_ERR_NONFINITE = -6    /* the residual holds a NaN or Inf (only with check_finite) */
};

enum fr_flux { FR_RUSANOV = 0, FR_ROE = 1 };     /* interface Riemann solver */
enum fr_prec { FR_FP64 = 0, FR_FP32 = 1 };       /* FP32: operators and fluxes in FP32 with a
                                                    reference-state split; state, RK registers
                                                    and the mass equation in FP64 */
enum fr_scheme { FR_RK4 = 0, FR_LSRK45 = 1 };    /* classical RK4; Carpenter-Kennedy 5-stage 2N */

/* Mesh and physics description, read by fr_mesh_create (section "FR Algorithm", Eq. (1)).
 *   p          polynomial degree of the solution, 0..7.
 *   q          degree of the geometry, 1..max(p,1); the mesh is isoparametric when q == p.
 *   n_elem     number of hexahedra.
 *   elem_vert  [n_elem][8] corner vertex ids in VTK hexahedron order. Faces are paired by
 *              their sorted corner ids, so periodic images must share one id; every face must
 *              pair (no physical boundaries in this build), which needs >= 3 elements across
 *              a periodic direction.
 *   elem_nodes [n_elem][(q+1)^3][3] node coordinates at the tensor Gauss-Lobatto-Legendre
 *              points of degree q, reference index i + (q+1)*(j + (q+1)*k).
 *   gamma, prandtl   ratio of specific heats and Prandtl number.
 *   mu         dynamic viscosity (constant); mu == 0 gives the Euler equations.
 *   br2_eta    BR2 penalty factor (the number of faces, 6, is the usual choice).
 *   flux       enum fr_flux.   prec: enum fr_prec.
 *   check_finite  non-zero: fr_residual scans its result and reports FR_ERR_NONFINITE.
 *   ref_rho, ref_p  reference state at rest used by FR_FP32 (ignored by FR_FP64): the FP32
 *              operators work on U - U_ref, formed in double precision, with the reference
 *              pressure and enthalpy split out of the momentum and energy fluxes. Choose the
 *              flow's mean density and pressure (for the Taylor-Green vortex at Mach 0.1:
 *              1 and 1/(gamma 0.01)). ref_rho must be > 0 for FR_FP32. */
typedef struct {
  int32_t p;
  int32_t q;
  int64_t n_elem;
  const int64_t *elem_vert;
  const double *elem_nodes;
  double gamma;
  double prandtl;
  double mu;
  double br2_eta;
  int32_t flux;
  int32_t prec;
  int32_t check_finite;
  int32_t reserved; /* must be 0 */
  double ref_rho;
  double ref_p;
} fr_mesh_desc;

/* Build a mesh on the current HIP device: pair faces (sort-and-match on corner ids, as the
 * paper's pre-processor does), compute the metric terms |J| dxi/dx in conservative curl form
 * and the face normals on the host in extended precision, and upload everything. The state
 * starts at zero. hip_stream: a hipStream_t (NULL = the default stream) on which every later
 * call of this handle is enqueued. Errors: FR_ERR_ARG, FR_ERR_MESH (message names the element
 * or face), FR_ERR_OOM, FR_ERR_HIP. On error *out is set to NULL. */
int fr_mesh_create(const fr_mesh_desc *desc, void *hip_stream, fr_mesh_t *out);

/* Release the handle and all device memory it owns. NULL is accepted. */
int fr_mesh_destroy(fr_mesh_t m);

/* Replace the stream later calls are enqueued on. */
int fr_set_stream(fr_mesh_t m, void *hip_stream);

/* Physical coordinates of the solution points, host array [n_elem][3][N_s]. */
int fr_sol_coords(fr_mesh_t m, double *xyz);

/* Copy a state [n_elem][5][N_s] into / out of the handle (see on_device above). */
int fr_set_state(fr_mesh_t m, const double *U, int on_device);
int fr_get_state(fr_mesh_t m, double *U, int on_device);

/* R = dQ/dt of Eq. (3) (source term 0) for the handle's current state, always in double
 * precision, layout [n_elem][5][N_s]. Errors: FR_ERR_ARG, FR_ERR_HIP, FR_ERR_NONFINITE. */
int fr_residual(fr_mesh_t m, double *R, int on_device);

/* Advance the state by n_steps explicit Runge-Kutta steps of size dt (enum fr_scheme). Every
 * stage is three kernels: the element pre-pass (solution and broken gradient to the faces),
 * the face kernel (common state, BR2 common gradient and common normal flux, once per face
 * point) and the volume kernel (corrected gradient, flux divergence and correction, and the
 * RK register update). Enqueued on the stream; returns without waiting. */
int fr_rk_step(fr_mesh_t m, double dt, int scheme, int n_steps);

/* Kinetic-energy diagnostics of the current state (a quadrature over the mesh with the
 * solution-point weights w and |J|): out[0] = E_k = sum w|J| |m|^2/(2 rho) / sum w|J|,
 * out[1] = dE_k/dt = sum w|J| (u . R_m - |u|^2 R_rho / 2) / sum w|J| evaluated from the
 * residual R of the handle's precision (one residual is computed). The dissipation rate is
 * -out[1]. The reduction is deterministic (fixed order). Waits for the stream. */
int fr_kinetic_energy(fr_mesh_t m, double *out);

/* Sizes of the handle: n_elem, points per element, bytes of device memory held. */
int fr_mesh_info(fr_mesh_t m, int64_t *n_elem, int32_t *n_sol, int64_t *device_bytes);

/* Measurement helper: run n_steps RK steps with each kernel launch bracketed by HIP events on
 * the handle's stream, and return the mean duration in milliseconds per stage of the element
 * pre-pass (ms[0]), the face kernel (ms[1]) and the volume kernel with the RK update (ms[2]).
 * Waits for the stream. */
int fr_profile_stages(fr_mesh_t m, double dt, int scheme, int n_steps, double *ms);

/* Host-only: run the mesh setup of fr_mesh_create without a GPU and return its arrays, for
 * inspection. Faces are numbered in owner order (the owner of a face is the side with the
 * smaller element index, then the smaller local face); a fully paired mesh has 3 n_elem.
 *   geo  [n_elem][10][N_s]: rows |J| dxi_n/dx_i (n-major, 9) then 1/|J|;
 *   fgeo [3 n_elem][4][N_fp]: the owner's outward scaled normal (3) and the BR2 factor
 *        sigma = eta (p+1)^2/8 (1/|J|_L + 1/|J|_R) at each owner face point;
 *   ftab [3 n_elem][4]: owner element, other element, code (bits 0-2 owner's face, 3-5 other
 *        face, 6 swap, 7 flip u, 8 flip v: the owner point -> other point map), 0;
 *   conn [n_elem][6][2]: neighbour element and packed code (bits 0-2 neighbour face, 3 swap,
 *        4 flip u, 5 flip v, 6 this side owns the face);
 *   xyz  [n_elem][3][N_s] solution-point coordinates.
 * Point (a, b) maps to (u', v') with (u, v) = swap ? (b, a) : (a, b), u' = flip_u ? p-u : u,
 * v' = flip_v ? p-v : v. Any output pointer may be NULL. Errors: FR_ERR_ARG, FR_ERR_MESH. */
int fr_mesh_geometry_host(const fr_mesh_desc *desc, double *geo, double *fgeo, int32_t *ftab, int32_t *conn,
                          double *xyz);

/* Host-only: the 1-D operator tables of degree p (0..7) the kernels use, each of n = p+1
 * doubles except D (n*n, row-major D[a*n+b] = l_b'(x_a)): lm = l_b(-1), lp = l_b(+1),
 * gcL = g_L'(x_a) and gcR = g_R'(x_a) of the DG-equivalent correction functions. */
int fr_basis_host(int p, double *D, double *lm, double *lp, double *gcL, double *gcR);

/* Thread-local description of the last error (empty string if none). */
const char *fr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FR_H */
