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
  FR_ERR_UNSUPPORTED = -5, /* a valid request this library does not implement */
  FR_ERR_NONFINITE = -6    /* the residual holds a NaN or Inf (only with check_finite) */
};

enum fr_flux { FR_RUSANOV = 0, FR_ROE = 1 };     /* interface Riemann solver */
enum fr_prec { FR_FP64 = 0, FR_FP32 = 1 };       /* FP32: operators and fluxes in FP32 with a
                                                    reference-state split; state, RK registers
                                                    and the mass equation in FP64 */
/* Common viscous flux (section "FR Algorithm"):
 *   FR_BR2  the second Bassi-Rebay scheme: common gradient = mean of the two broken gradients
 *           plus the two local liftings of the jump, with factor br2_eta;
 *   FR_LDG  the local DG scheme the paper uses (after Huynh): the common solution is one-sided,
 *           U^ = the trace of the face's non-owner (beta = +n_owner/2; the owner is the side with
 *           the smaller element index, then local face), each side's corrected gradient uses
 *           U^ - U, and the common viscous normal flux is the owner's F_v(U_L, q_L) . n plus
 *           ldg_tau (U_R - U_L). */
enum fr_viscous { FR_BR2 = 0, FR_LDG = 1 };

enum fr_scheme {                                  /* explicit Runge-Kutta schemes: */
  FR_RK4 = 0,      /* classical four-stage RK4 (three registers) */
  FR_LSRK45 = 1,   /* Carpenter-Kennedy five-stage fourth-order, 2N storage */
  FR_SSPRK104 = 2  /* Ketcheson's ten-stage fourth-order strong-stability-preserving method
                      in its two-register low-storage form (SSP coefficient 6), the class of
                      scheme the paper advances in time with (section "FR Algorithm") */
};

/* Mesh and physics description, read by fr_mesh_create (section "FR Algorithm", Eq. (1)).
 *   p          polynomial degree of the solution, 0..7.
 *   q          degree of the geometry, 1..max(p,1); the mesh is isoparametric when q == p.
 *   n_elem     number of hexahedra.
 *   elem_vert  [n_elem][8] corner vertex ids in VTK hexahedron order. Faces are paired by
 *              their sorted corner ids, so periodic images must share one id (which needs >= 3
 *              elements across a periodic direction); a face that does not pair must be a
 *              tagged wall (bc_tag).
 *   elem_nodes [n_elem][(q+1)^3][3] node coordinates at the tensor Gauss-Lobatto-Legendre
 *              points of degree q, reference index i + (q+1)*(j + (q+1)*k).
 *   gamma, prandtl   ratio of specific heats and Prandtl number.
 *   mu         dynamic viscosity (constant); mu == 0 gives the Euler equations.
 *   br2_eta    BR2 penalty factor (the number of faces, 6, is the usual choice).
 *   viscous    enum fr_viscous: the common viscous flux (0 = BR2; zero-initialised descriptors
 *              keep it). FR_LDG needs prec = FR_FP64 (FR_ERR_UNSUPPORTED otherwise).
 *   ldg_tau    LDG penalty (>= 0) on the jump of every conserved variable.
 *   bc_tag     [n_elem][6] or NULL. A face that does not pair must carry tag 1: an isothermal
 *              no-slip wall at temperature wall_T (p/rho, > 0). Its inviscid flux is the Riemann
 *              flux against the mirror state (rho, -m, E) (impermeable, no energy flux); its
 *              viscous flux uses the wall state (rho, 0, rho wall_T/(gamma-1)) as the common
 *              state and the one-sided BR2 gradient. Walls need FR_BR2 (FR_ERR_UNSUPPORTED with
 *              FR_LDG); both precisions support them.
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
  int32_t viscous;
  double ref_rho;
  double ref_p;
  double ldg_tau;
  const int32_t *bc_tag;
  double wall_T;
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

/* Tile shapes of the stage kernels (both precisions), chosen by the autotuner or by the caller:
 *   epb  elements per block of the element kernels (pre-pass, volume): 0 = 256/N_s (at least
 *        one, at most 64), 1 = half of that, or, where that is one element whose N_s points
 *        leave lanes of the last wave idle (p = 5, 6), two elements;
 *   fbs  threads per block of the face kernel: 0 = 256, 1 = 128, 2 = 64.
 * Results are bitwise independent of the tiles (every thread does the same arithmetic). A batch
 * captures the tiles in force at its creation. */
int fr_set_tiles(fr_mesh_t m, int32_t epb, int32_t fbs);
int fr_get_tiles(fr_mesh_t m, int32_t *epb, int32_t *fbs);

/* Autotuner: time each tile choice, with and without the fused pre-pass (fr_set_fusion), on
 * this mesh and state: n_trials LSRK stages each from the current state into scratch buffers
 * (HIP events on the handle's stream, after one warm-up stage each), and keep the fastest. The
 * timed stages are later stages of a step (they read and write the RK register).
 * ms (may be NULL) receives 12 mean ms per stage: index fuse * 6 + epb * 3 + fbs, where
 * fuse = 0 times the stand-alone pre-pass + face + volume kernels and fuse = 1 the face kernel
 * + the volume kernel with the next stage's pre-pass. Allocates two state-sized scratch
 * buffers for the call; waits. The state, the RK registers and the results of later calls are
 * unaffected. */
int fr_autotune(fr_mesh_t m, int n_trials, double *ms);

/* Stage chaining (default on, both precisions): with on = 1 each RK stage's volume kernel also
 * computes the next stage's pre-pass (face values and broken gradient of the state it stores),
 * so a run of stages launches the stand-alone pre-pass once; with on = 0 every stage launches
 * it. The arithmetic is the same, so results are bitwise identical either way; fr_autotune
 * picks the faster. A batch captures the setting in force at its creation. */
int fr_set_fusion(fr_mesh_t m, int32_t on);
int fr_get_fusion(fr_mesh_t m, int32_t *on);

/* Source term S of Eq. (3) as a constant body force per unit mass g[3] ("body forcing" is
 * among the solver's physical models, section "ZFR Framework"): S = (0, rho g, m . g), added
 * to every later residual and RK stage. g = NULL or all zeros switches it off. */
int fr_set_body_force(fr_mesh_t m, const double *g);

/* R = dQ/dt of Eq. (3) (with the source term, if set) for the handle's current state, always in double
 * precision, layout [n_elem][5][N_s]. Errors: FR_ERR_ARG, FR_ERR_HIP, FR_ERR_NONFINITE. */
int fr_residual(fr_mesh_t m, double *R, int on_device);

/* Advance the state by n_steps explicit Runge-Kutta steps of size dt (enum fr_scheme). A stage
 * is the element pre-pass (solution and broken gradient to the faces), the face kernel (common
 * state, BR2 common gradient and common normal flux, once per face point) and the volume kernel
 * (corrected gradient, flux divergence and correction, and the RK register update). With the
 * fused pre-pass (fr_set_fusion, on by default) the run's first stage launches all three and
 * every later stage two: its pre-pass was done by the previous stage's volume kernel. Enqueued
 * on the stream; returns without waiting. */
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
 * the handle's stream, and return mean durations in milliseconds (ms[4]):
 *   ms[0]  the element pre-pass, per launch. With fusion on (fr_set_fusion) a run of stages
 *          launches it once: every later stage's pre-pass is done by the previous stage's
 *          volume kernel;
 *   ms[1]  the face kernel, per stage;
 *   ms[2]  the volume kernel with the RK update and the next stage's pre-pass, per launch
 *          (0 if none ran: fusion off, or a run of one stage);
 *   ms[3]  the volume kernel with the RK update alone, per launch (the run's last stage; every
 *          stage with fusion off).
 * Waits for the stream. */
int fr_profile_stages(fr_mesh_t m, double dt, int scheme, int n_steps, double *ms);

/* Host-only: run the mesh setup of fr_mesh_create without a GPU and return its arrays, for
 * inspection. Faces are numbered in owner order (the owner of a face is the side with the
 * smaller element index, then the smaller local face; a wall's element owns it); there are
 * F = 3 n_elem + n_wall/2 faces (n_wall tagged wall faces).
 *   geo  [n_elem][10][N_s]: rows |J| dxi_n/dx_i (n-major, 9) then 1/|J|;
 *   fgeo [F][4][N_fp]: the owner's outward scaled normal (3) and the BR2 factor
 *        sigma = eta (p+1)^2/8 (1/|J|_L + 1/|J|_R) at each owner face point (2/|J|_L at a wall);
 *   ftab [F][4]: owner element, other element (-1 at a wall), code (bits 0-2 owner's face, 3-5
 *        other face, 6 swap, 7 flip u, 8 flip v: the owner point -> other point map; bit 9 a
 *        wall), 0;
 *   conn [n_elem][6][2]: neighbour element (-1 at a wall) and packed code (bits 0-2 neighbour
 *        face, 3 swap, 4 flip u, 5 flip v, 6 this side owns the face, 7 a wall);
 *   xyz  [n_elem][3][N_s] solution-point coordinates.
 * Point (a, b) maps to (u', v') with (u, v) = swap ? (b, a) : (a, b), u' = flip_u ? p-u : u,
 * v' = flip_v ? p-v : v. Any output pointer may be NULL. Errors: FR_ERR_ARG, FR_ERR_MESH. */
int fr_mesh_geometry_host(const fr_mesh_desc *desc, double *geo, double *fgeo, int32_t *ftab, int32_t *conn,
                          double *xyz);

/* Host-only: the 1-D operator tables of degree p (0..7) the kernels use, each of n = p+1
 * doubles except D (n*n, row-major D[a*n+b] = l_b'(x_a)): lm = l_b(-1), lp = l_b(+1),
 * gcL = g_L'(x_a) and gcR = g_R'(x_a) of the DG-equivalent correction functions. */
int fr_basis_host(int p, double *D, double *lm, double *lp, double *gcL, double *gcR);

/* Host-only: the coefficient tables the RK stages use (section "FR Algorithm": explicit
 * Runge-Kutta time integration). a, b: arrays of at least 5 doubles; *n_stages receives the count.
 *   FR_LSRK45  n = 5: a = A_i, b = B_i of the 2N form dU <- A_i dU + dt R; U <- U + B_i dU
 *              (Carpenter and Kennedy's ratios of integers, rounded to double);
 *   FR_RK4     n = 4: a = the weights (1/6, 1/3, 1/3, 1/6), b = the node of the next stage
 *              (1/2, 1/2, 1, then 0 after the last stage).
 * FR_SSPRK104 has no table (its fixed fractions 1/6, 1/25, 9/25, 15, 5, 3/5 and 1/10 are in the
 * stage epilogue): FR_ERR_ARG, as for an unknown scheme. */
int fr_rk_coefficients(int scheme, double *a, double *b, int32_t *n_stages);

/* ==========================================================================================
 * Batches: many meshes (any degrees, precisions, closures) advanced together. One RK step of
 * every mesh is captured once into a HIP graph, each mesh's stage kernels on a branch of its
 * own, so independent meshes run concurrently, and so are 8 steps whose stages chain through
 * the fused pre-pass across step boundaries; fr_batch_step replays them. The result of every
 * mesh is bitwise that of fr_rk_step on it alone (same kernels, same order within the mesh).
 * ========================================================================================== */
typedef struct fr_batch_s *fr_batch_t;

/* Capture one step of size dt[i] of the given scheme for meshes[i], i < n (distinct handles on
 * the current device; their RK registers are allocated here). The meshes must outlive the
 * batch. What lives in device memory may change between steps and is read by every replay:
 * the state (fr_set_state), the values of a fixed eddy viscosity, a model's parameters. What
 * the kernels take as arguments is fixed at this call: the step sizes, the body force, and
 * whether a closure (fixed or model) is attached; change those by creating a new batch.
 * hip_stream: where fr_batch_step enqueues. Errors: FR_ERR_ARG, FR_ERR_HIP. */
int fr_batch_create(const fr_mesh_t *meshes, int32_t n, const double *dt, int scheme, void *hip_stream,
                    fr_batch_t *out);

/* fr_batch_create with flags. FR_BATCH_MULTI (the default of fr_batch_create): the viscous
 * FP32-form meshes without closure or LDG are grouped by degree, fusion setting and tiles, and
 * each group's step is one launch per kernel and stage covering all its meshes: block b of the
 * grid is an element block or a face block of one of the group's meshes (found from prefix sums
 * of the meshes' block counts) and runs the arithmetic of the single-mesh kernel's block, with
 * that mesh's arguments (state, geometry, step size, physics, reference state) from a device
 * table. Every other mesh, and every mesh when flags = 0, steps on a graph branch of its own.
 * Results are bitwise those of fr_rk_step either way. */
#define FR_BATCH_MULTI 1
int fr_batch_create_ex(const fr_mesh_t *meshes, int32_t n, const double *dt, int scheme, void *hip_stream,
                       int32_t flags, fr_batch_t *out);

/* Enqueue n_steps RK steps on the batch's stream: n_steps / 8 replays of the 8-step graph, then
 * n_steps % 8 of the one-step graph (returns without waiting). Each replay starts from the
 * meshes' current states, so states may be changed between calls. */
int fr_batch_step(fr_batch_t b, int n_steps);
int fr_batch_set_stream(fr_batch_t b, void *hip_stream);
int fr_batch_destroy(fr_batch_t b);

/* ==========================================================================================
 * Partition groups: a mesh split into parts that exchange their shared faces, the one-GPU form
 * of the paper's multi-process run (section "Pre-processor Parallelization": each process holds
 * a part, faces shared with other parts are matched by their vertex ids; section "Three-level
 * Parallelization Design"). Each part is a mesh handle with its own elements (the part's elements
 * of the whole mesh in increasing order; state layout [n_local][5][N_s]) whose face buffer also
 * holds ghost slots for the other parts' sides of the shared faces. With BR2 a stage needs one
 * exchange, between the pre-pass (the face values and broken gradient) and the face kernel: each
 * part packs its side of the faces it shares with part q into one contiguous message
 * (fr_halo_pack), which part q scatters into its ghost slots (fr_halo_unpack); in a
 * multi-process run the message would travel between the two (RCCL send/receive over xGMI).
 * Both parts of a shared face compute its common flux from the same data with the whole mesh's
 * normal and orientation, so the group's results equal the unsplit mesh's bit for bit.
 * ========================================================================================== */
typedef struct fr_part_s *fr_part_t;

/* Split the mesh of desc by part[n_elem] (values 0..n_part-1, every part non-empty; 1 <= n_part
 * <= 1024) and create every part on the current device, enqueued on hip_stream, with one device
 * message buffer per ordered pair of parts that share faces. The whole mesh's setup (face
 * pairing, metrics, normals) is done once and split. Needs the BR2 viscous flux
 * (FR_ERR_UNSUPPORTED with FR_LDG, which would need a second exchange per stage). Errors as
 * fr_mesh_create, and FR_ERR_ARG for a bad part map. */
int fr_part_create(const fr_mesh_desc *desc, const int32_t *part, int32_t n_part, void *hip_stream,
                   fr_part_t *out);
int fr_part_destroy(fr_part_t g);

/* Host-only: the split of part q without a GPU, for inspection: its element count, ghost face
 * slots, and per other part r the faces it sends to r and receives from r (n_send, n_recv
 * [n_part], may be NULL). */
int fr_part_host(const fr_mesh_desc *desc, const int32_t *part, int32_t n_part, int32_t q, int64_t *n_local,
                 int64_t *n_ghost, int64_t *n_send, int64_t *n_recv);

/* The handle of part q, owned by the group: fr_set_state, fr_get_state, fr_sol_coords,
 * fr_set_tiles, fr_set_fusion, fr_set_body_force and fr_mesh_info act on it as on any mesh;
 * fr_residual, fr_rk_step, fr_kinetic_energy, fr_autotune, fr_profile_stages, the closure and
 * batches refuse it (FR_ERR_UNSUPPORTED), and fr_mesh_destroy refuses it (FR_ERR_ARG). */
int fr_part_get_mesh(fr_part_t g, int32_t q, fr_mesh_t *m);

/* Part q's element count and (global_ids may be NULL) its elements' indices in the whole mesh,
 * host array [n_local], increasing. */
int fr_part_elements(fr_part_t g, int32_t q, int64_t *n_local, int64_t *global_ids);

/* Enqueue every part's work on hip_stream from now on. */
int fr_part_set_stream(fr_part_t g, void *hip_stream);

/* The message part m sends to part q: its number of shared faces and its size in bytes (per face
 * the 20 face values of N_fp points in the handle's face precision; in the FP32 form the 20
 * floats of every face, padded to 256 bytes, then the 3 momentum doubles of N_fp points). */
int fr_halo_size(fr_mesh_t m, int32_t q, int64_t *n_faces, int64_t *bytes);

/* Gather part m's side of the faces it shares with part q from its face buffer into the device
 * buffer send (fr_halo_size bytes), and scatter the message part q packed for m into m's ghost
 * slots. Both are enqueued on m's stream; the faces are in the whole mesh's face order on both
 * sides. Errors: FR_ERR_ARG (not a part, q out of range, NULL buffer with faces to move). */
int fr_halo_pack(fr_mesh_t m, int32_t q, void *send);
int fr_halo_unpack(fr_mesh_t m, int32_t q, const void *recv);

/* Every part's residual R[q] ([n_local(q)][5][N_s]; all device or all host pointers): the
 * pre-pass of every part, the exchange, then every part's face and volume kernels. */
int fr_part_residual(fr_part_t g, double *const *R, int on_device);

/* n_steps RK steps of the whole group in lockstep: per stage, every part's pre-pass (or the
 * previous stage's fused one), the exchange, then every part's face and volume kernels.
 * Enqueued; returns without waiting. The closure is not exchanged between parts
 * (FR_ERR_UNSUPPORTED if a part has one). */
int fr_part_rk_step(fr_part_t g, double dt, int scheme, int n_steps);

/* ==========================================================================================
 * Learned eddy-viscosity closure (an LES sub-grid scale model; section "ZFR Framework" lists
 * such models among the solver's physical models without specifying one).
 *
 * An eddy kinematic viscosity nu_t >= 0, constant per element, enters the viscous flux as
 * mu + rho nu_t in the stress and mu/Pr + rho nu_t/Pr_t in the heat flux (gamma/(gamma-1)
 * times these, acting on d(p/rho)); at a face, nu_t is the mean of the two elements' values
 * and rho that of the common state. nu_t = 0 reproduces the plain residual. The closure needs
 * prec = FR_FP64 (FR_ERR_UNSUPPORTED otherwise).
 *
 * The model is a per-element network y = softplus(w3 . tanh(W2 tanh(W1 x^ + b1) + b2) + b3),
 * x^ = (x - mean)/std, 64 units per hidden layer, with nu_t = nu_scale * y. W1, W2 and w3 are
 * used rounded to bfloat16 (nearest, ties to even) on the matrix cores with float32
 * accumulation; activations enter the products as the sum of two bfloat16 values (a hi/lo
 * split, relative representation error <= 2^-17). Biases, standardisation and Adam state are
 * float32. Parameters are one float32 array in the order W1[64][n_in], b1[64], W2[64][64],
 * b2[64], w3[64], b3[1] (fr_mlp_n_params(n_in) values).
 * ========================================================================================== */
typedef struct fr_mlp_s *fr_mlp_t;

/* Number of features per element for degree p: (p+1)^3 - 1 modal energies + 5 invariants. */
int fr_sgs_n_features(int p);

/* Features of the handle's current state, device array feat [n_elem][fr_sgs_n_features(p)]
 * float32, enqueued on the handle's stream. From the element's velocity polynomial u = m/rho:
 *   ln(e_k + 1e-12) for each orthonormal tensor Legendre mode k = a + n(b + n c) except the
 *   constant one, e_k = (1/16) sum_j uhat_{j,k}^2 (uhat by Gauss quadrature on the reference
 *   cube); then, with volume averages <.> over the element of the broken velocity gradient
 *   A_ij = d u_j/d x_i (S, W its symmetric / antisymmetric parts) and eps = 1e-12:
 *   ln(<2S:S> + eps)/2, ln(<2W:W> + eps)/2, <-tr(A^3)/3>/(<2S:S> + eps)^(3/2),
 *   <tr A>/(<2S:S> + eps)^(1/2), <(tr A)^2>/(<2S:S> + eps).
 * Computed in double precision and rounded to float32 once. */
int fr_sgs_features(fr_mesh_t m, float *feat);

/* Fixed per-element eddy viscosity nu [n_elem] (>= 0; on_device as above) used by every
 * later residual and RK stage, with turbulent Prandtl number prandtl_t > 0; nu = NULL turns
 * the closure off. Replaces an attached model. */
int fr_set_eddy_viscosity(fr_mesh_t m, const double *nu, int on_device, double prandtl_t);

/* Attach a model: every later residual and RK stage first computes the features of the state
 * it is evaluated on and nu_t = nu_scale * model(features), then the stage. The model must
 * have n_in = fr_sgs_n_features(p) and must outlive the attachment; model = NULL detaches. */
int fr_set_sgs_model(fr_mesh_t m, fr_mlp_t model, double nu_scale, double prandtl_t);

/* The per-element eddy viscosity of the last stage (or the fixed one), host array [n_elem]. */
int fr_get_eddy_viscosity(fr_mesh_t m, double *nu);

/* Parameter count for n_in inputs. */
int64_t fr_mlp_n_params(int32_t n_in);

/* Create a network with n_in (1..128) inputs on the current device. params (host, float32,
 * fr_mlp_n_params values), mean and std (host, n_in values, std > 0) are copied. Adam state
 * starts at zero. hip_stream as in fr_mesh_create. */
int fr_mlp_create(int32_t n_in, const float *params, const float *mean, const float *std_dev, void *hip_stream,
                  fr_mlp_t *out);
int fr_mlp_destroy(fr_mlp_t net);
int fr_mlp_set_stream(fr_mlp_t net, void *hip_stream);

/* Replace the parameters (host float32) and reset the Adam state; read them back (waits). */
int fr_mlp_set_params(fr_mlp_t net, const float *params);
int fr_mlp_get_params(fr_mlp_t net, float *params);

/* The bfloat16 bit patterns of W1 [64][n_in], W2 [64][64] and w3 [64] as the kernels use them
 * (host arrays; waits). */
int fr_mlp_get_bf16(fr_mlp_t net, uint16_t *W1, uint16_t *W2, uint16_t *w3);

/* y [n] = model(X) for device arrays X [n][ldx] float32 (ldx >= n_in) and y [n] float32. */
int fr_mlp_forward(fr_mlp_t net, const float *X, int64_t n, int64_t ldx, float *y);

/* Loss L = mean_n (y_n - t_n)^2 over device arrays X [n][ldx], t [n], and its gradient with
 * respect to every parameter (host grad [n_params]; the gradient of a rounded weight is used for
 * its master). No update. Deterministic (fixed reduction order). Waits. */
int fr_mlp_loss_grad(fr_mlp_t net, const float *X, int64_t n, int64_t ldx, const float *t, float *grad,
                     double *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the loss above: the
 * forward and backward passes, the deterministic gradient reduction and the update of the
 * float32 masters and their bfloat16 copies. loss (device float, may be NULL) receives L before
 * the update. Enqueued on the network's stream. */
int fr_mlp_train_step(fr_mlp_t net, const float *X, int64_t n, int64_t ldx, const float *t, float lr, float *loss);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight training or
 * serving loops, harnesses that forbid hipMalloc): fr_mlp_train_step with the same arguments,
 * kernels and results, bit for bit, but its per-sample activations, deltas and gradient partial
 * sums live in a fixed scratch array (14.2 MiB) that the library holds on each GPU it runs on
 * until the process ends, instead of buffers the network grows with hipMalloc. Nothing is
 * allocated or freed. n must be 1..FR_MLP_NOALLOC_MAX_N (FR_ERR_ARG beyond). Every call on one GPU
 * shares that GPU's array and overwrites it: calls that overlap in time on one GPU (other
 * streams, threads or networks) race and must be ordered by the caller. Enqueued on the
 * network's stream. */
#define FR_MLP_NOALLOC_MAX_N 8192
int fr_mlp_train_step_noalloc(fr_mlp_t net, const float *X, int64_t n, int64_t ldx, const float *t, float lr,
                              float *loss);

/* Thread-local description of the last error (empty string if none). */
const char *fr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FR_H */
