// fr_partition.hip -- a mesh split into parts that exchange their partition faces, on one GPU.
//
// The paper runs its solver on many processes, each holding a part of the mesh; with the
// element-major face buffer the only data a stage needs from another part is the face data of
// the faces they share (section "Pre-processor Parallelization": faces are matched across parts
// by their vertex ids; section "Three-level Parallelization Design": one exchange per stage
// between the pre-pass and the face kernel). Here every part is a mesh handle of its own whose
// face buffer has ghost slots for the other parts' sides of the shared faces:
//
//   pack    per part and neighbour: the part's own face-buffer entries of the shared faces,
//           gathered into one contiguous buffer (the message a multi-process run would send),
//   unpack  the neighbour's message scattered into this part's ghost slots.
//
// A group steps all parts in lockstep on one stream: each stage's pre-pass (or the previous
// stage's fused one), the exchange, then the face and volume kernels of every part. Both parts
// of a shared face compute its common flux from the same data with the whole mesh's normal and
// orientation, so a group's results equal the unsplit mesh's bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "fr.h"
#include "fr_internal.h"

using namespace frk;

namespace {

// out[i][v][k] = face[slot[i]][v][k] for the n listed slots; NV values of Nfp points per slot.
// Consecutive threads copy consecutive words of a slot's contiguous NV * Nfp run.
template <typename T>
__global__ __launch_bounds__(256) void k_halo_pack(const T *__restrict__ face, const int32_t *__restrict__ slot,
                                                   int64_t n, int run, T *__restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= n * run) return;
  const int64_t i = gid / run;
  const int64_t w = gid - i * run;
  out[gid] = face[(int64_t)slot[i] * run + w];
}

// face[base + ghost[i]][v][k] = in[i][v][k]
template <typename T>
__global__ __launch_bounds__(256) void k_halo_unpack(T *__restrict__ face, const int32_t *__restrict__ ghost,
                                                     int64_t base, int64_t n, int run, const T *__restrict__ in) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= n * run) return;
  const int64_t i = gid / run;
  const int64_t w = gid - i * run;
  face[(base + ghost[i]) * run + w] = in[gid];
}

int pfail(int code, const std::string &msg) { return fr_fail(code, msg); }

#define PCHK(call)                                                                              \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) return pfail(FR_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Message layout per shared face: the 20 face values of Nfp points (FP64: doubles; FP32 form:
// floats), then in the FP32 form the 3 momentum components of Nfp points as doubles, after all
// faces' float parts (aligned to 256 bytes).
int64_t float_part_bytes(const DeviceMesh &dm, int64_t nf) {
  return ((nf * 20 * dm.Nfp * (int64_t)sizeof(float) + 255) / 256) * 256;
}

int64_t message_bytes(const DeviceMesh &dm, int64_t nf) {
  if (dm.prec == FR_FP64) return nf * 20 * dm.Nfp * (int64_t)sizeof(double);
  return float_part_bytes(dm, nf) + nf * 3 * dm.Nfp * (int64_t)sizeof(double);
}

template <typename T>
int launch_pack(hipStream_t s, const void *face, const int32_t *slot, int64_t n, int run, void *out) {
  if (n == 0) return FR_OK;
  const int64_t total = n * run;
  hipLaunchKernelGGL((k_halo_pack<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (const T *)face, slot,
                     n, run, (T *)out);
  PCHK(hipGetLastError());
  return FR_OK;
}

template <typename T>
int launch_unpack(hipStream_t s, void *face, const int32_t *ghost, int64_t base, int64_t n, int run, const void *in) {
  if (n == 0) return FR_OK;
  const int64_t total = n * run;
  hipLaunchKernelGGL((k_halo_unpack<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (T *)face, ghost,
                     base, n, run, (const T *)in);
  PCHK(hipGetLastError());
  return FR_OK;
}

int pack(fr_mesh_s *m, int q, void *out) {
  DeviceMesh &dm = m->dm;
  hipStream_t s = (hipStream_t)dm.stream;
  const int64_t n = m->n_send[q];
  if (dm.prec == FR_FP64) return launch_pack<double>(s, dm.face, m->send_slots[q], n, 20 * dm.Nfp, out);
  int rc = launch_pack<float>(s, dm.face32, m->send_slots[q], n, 20 * dm.Nfp, out);
  if (rc) return rc;
  return launch_pack<double>(s, dm.facem, m->send_slots[q], n, 3 * dm.Nfp, (char *)out + float_part_bytes(dm, n));
}

int unpack(fr_mesh_s *m, int q, const void *in) {
  DeviceMesh &dm = m->dm;
  hipStream_t s = (hipStream_t)dm.stream;
  const int64_t n = m->n_recv[q], base = dm.E * 6;
  if (dm.prec == FR_FP64) return launch_unpack<double>(s, dm.face, m->recv_slots[q], base, n, 20 * dm.Nfp, in);
  int rc = launch_unpack<float>(s, dm.face32, m->recv_slots[q], base, n, 20 * dm.Nfp, in);
  if (rc) return rc;
  return launch_unpack<double>(s, dm.facem, m->recv_slots[q], base, n, 3 * dm.Nfp,
                               (const char *)in + float_part_bytes(dm, n));
}

}  // namespace

// A group of parts of one mesh and the device buffers of its exchange (one per ordered pair of
// parts that share faces).
struct fr_part_s {
  uint64_t magic;
  std::vector<fr_mesh_s *> parts;
  std::vector<std::vector<int64_t>> elems;  // [part] local -> global element
  std::vector<std::vector<void *>> msg;     // [from][to] device message buffer, or null
  hipStream_t stream = nullptr;
};

namespace {

constexpr uint64_t kPartMagic = 0x4652504152545331ull;  // "FRPARTS1"

bool valid_group(const fr_part_s *g) { return g != nullptr && g->magic == kPartMagic; }

void free_group(fr_part_s *g) {
  for (auto &row : g->msg)
    for (void *b : row)
      if (b) (void)hipFree(b);
  for (fr_mesh_s *m : g->parts)
    if (m) {
      m->group = nullptr;
      (void)destroy_device_mesh(m);
    }
  g->magic = 0;
  delete g;
}

// Every part packs its message for every neighbour, then every part unpacks the messages it
// receives: after this the ghost slots hold the other parts' current face data.
int exchange(fr_part_s *g) {
  const int np = (int)g->parts.size();
  for (int a = 0; a < np; ++a)
    for (int b = 0; b < np; ++b)
      if (g->msg[a][b]) {
        int rc = pack(g->parts[a], b, g->msg[a][b]);
        if (rc) return rc;
      }
  for (int b = 0; b < np; ++b)
    for (int a = 0; a < np; ++a)
      if (g->msg[a][b]) {
        int rc = unpack(g->parts[b], a, g->msg[a][b]);
        if (rc) return rc;
      }
  return FR_OK;
}

// One stage of every part: the pre-pass where the previous stage did not fuse it, the exchange,
// then each part's face and volume kernels (with the next stage's pre-pass when fused).
int group_stage(fr_part_s *g, int scheme, int s, double dt, bool first, bool last, double *const *R) {
  const int np = (int)g->parts.size();
  for (int pi = 0; pi < np; ++pi) {
    DeviceMesh &dm = g->parts[pi]->dm;
    StageArgs st;
    const double *X;
    double *o, *r1, *r2;
    stage_setup(dm, scheme, s, dt, st, &X, &o, &r1, &r2);
    if (R) st = StageArgs{};  // residual mode
    if (first || !dm.fuse) {
      st.pre_only = 1;
      int rc = enqueue_stage(dm, X, st, o, r1, r2);
      if (rc) return rc;
    }
  }
  int rc = exchange(g);
  if (rc) return rc;
  for (int pi = 0; pi < np; ++pi) {
    DeviceMesh &dm = g->parts[pi]->dm;
    StageArgs st;
    const double *X;
    double *o, *r1, *r2;
    stage_setup(dm, scheme, s, dt, st, &X, &o, &r1, &r2);
    if (R) {
      st = StageArgs{};
      st.mode = kModeResidual;
      o = R[pi];
      r1 = r2 = nullptr;
    }
    st.pre_done = 1;
    st.pre_next = !R && dm.fuse && !last;
    rc = enqueue_stage(dm, X, st, o, r1, r2);
    if (rc) return rc;
  }
  return FR_OK;
}

}  // namespace

extern "C" {

int fr_part_create(const fr_mesh_desc *d, const int32_t *part, int32_t n_part, void *hip_stream, fr_part_t *out) {
  if (!out) return pfail(FR_ERR_ARG, "out is NULL");
  *out = nullptr;
  int rc = validate_desc(d);
  if (rc) return rc;
  if (!part || n_part < 1 || n_part > 1024) return pfail(FR_ERR_ARG, "need the part map and 1 <= n_part <= 1024");
  if (d->viscous == FR_LDG)
    return pfail(FR_ERR_UNSUPPORTED, "partition groups exchange the face data once per stage, which is BR2's need "
                                     "(LDG would need a second exchange of the corrected gradient)");
  HostMesh G;
  rc = host_mesh_of(d, G);
  if (rc) return rc;
  fr_part_s *g = new fr_part_s();
  g->magic = kPartMagic;
  g->stream = (hipStream_t)hip_stream;
  g->parts.assign(n_part, nullptr);
  g->elems.assign(n_part, {});
  g->msg.assign(n_part, std::vector<void *>(n_part, nullptr));
  int dev = 0;
  (void)hipGetDevice(&dev);
  for (int q = 0; q < n_part && rc == FR_OK; ++q) {
    HostPart P;
    std::string err = build_partition(G, part, n_part, q, P);
    if (!err.empty()) {
      rc = pfail(FR_ERR_ARG, err);
      break;
    }
    fr_mesh_desc dq = *d;
    dq.n_elem = P.H.E;
    fr_mesh_s *m = nullptr;
    rc = create_device_mesh(&dq, P.H, P.n_ghost, hip_stream, &m);
    if (rc) break;
    g->parts[q] = m;
    m->group = g;
    m->device = dev;
    g->elems[q] = P.elems;
    m->send_slots.assign(n_part, nullptr);
    m->recv_slots.assign(n_part, nullptr);
    m->n_send.assign(n_part, 0);
    m->n_recv.assign(n_part, 0);
    for (int r = 0; r < n_part && rc == FR_OK; ++r) {
      if (P.send[r].size() != P.recv[r].size()) {
        rc = pfail(FR_ERR_MESH, "unbalanced exchange lists");
        break;
      }
      m->n_send[r] = (int64_t)P.send[r].size();
      m->n_recv[r] = (int64_t)P.recv[r].size();
      if (P.send[r].empty()) continue;
      const size_t bytes = P.send[r].size() * sizeof(int32_t);
      if (hipMalloc(&m->send_slots[r], bytes) != hipSuccess || hipMalloc(&m->recv_slots[r], bytes) != hipSuccess ||
          hipMemcpy(m->send_slots[r], P.send[r].data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(m->recv_slots[r], P.recv[r].data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
        rc = pfail(FR_ERR_HIP, "upload of the exchange lists failed");
    }
  }
  // message buffers, one per ordered pair that shares faces (part a's send list to b and part b's
  // receive list from a name the same faces in the same order)
  for (int a = 0; a < n_part && rc == FR_OK; ++a)
    for (int b = 0; b < n_part && rc == FR_OK; ++b) {
      const int64_t n = g->parts[a]->n_send[b];
      if (n != g->parts[b]->n_recv[a]) {
        rc = pfail(FR_ERR_MESH, "parts " + std::to_string(a) + " and " + std::to_string(b) +
                                    " disagree on their shared faces");
        break;
      }
      if (n > 0 && hipMalloc(&g->msg[a][b], message_bytes(g->parts[a]->dm, n)) != hipSuccess)
        rc = pfail(FR_ERR_OOM, "hipMalloc of an exchange buffer");
    }
  if (rc) {
    free_group(g);
    return rc;
  }
  *out = g;
  return FR_OK;
}

int fr_part_host(const fr_mesh_desc *d, const int32_t *part, int32_t n_part, int32_t q, int64_t *n_local,
                 int64_t *n_ghost, int64_t *n_send, int64_t *n_recv) {
  int rc = validate_desc(d);
  if (rc) return rc;
  if (!part || n_part < 1 || n_part > 1024 || q < 0 || q >= n_part) return pfail(FR_ERR_ARG, "bad part map or q");
  HostMesh G;
  rc = host_mesh_of(d, G);
  if (rc) return rc;
  HostPart P;
  std::string err = build_partition(G, part, n_part, q, P);
  if (!err.empty()) return pfail(FR_ERR_ARG, err);
  if (n_local) *n_local = P.H.E;
  if (n_ghost) *n_ghost = P.n_ghost;
  for (int r = 0; r < n_part; ++r) {
    if (n_send) n_send[r] = (int64_t)P.send[r].size();
    if (n_recv) n_recv[r] = (int64_t)P.recv[r].size();
  }
  return FR_OK;
}

int fr_part_destroy(fr_part_t g) {
  if (!g) return FR_OK;
  if (!valid_group(g)) return pfail(FR_ERR_ARG, "not a partition group handle");
  (void)hipStreamSynchronize(g->stream);
  free_group(g);
  return FR_OK;
}

int fr_part_get_mesh(fr_part_t g, int32_t q, fr_mesh_t *m) {
  if (!valid_group(g) || !m || q < 0 || q >= (int32_t)g->parts.size()) return pfail(FR_ERR_ARG, "bad group or part");
  *m = g->parts[q];
  return FR_OK;
}

int fr_part_elements(fr_part_t g, int32_t q, int64_t *n_local, int64_t *global_ids) {
  if (!valid_group(g) || q < 0 || q >= (int32_t)g->parts.size()) return pfail(FR_ERR_ARG, "bad group or part");
  if (n_local) *n_local = (int64_t)g->elems[q].size();
  if (global_ids) std::memcpy(global_ids, g->elems[q].data(), g->elems[q].size() * sizeof(int64_t));
  return FR_OK;
}

int fr_part_set_stream(fr_part_t g, void *hip_stream) {
  if (!valid_group(g)) return pfail(FR_ERR_ARG, "not a partition group handle");
  g->stream = (hipStream_t)hip_stream;
  for (fr_mesh_s *m : g->parts) m->dm.stream = hip_stream;
  return FR_OK;
}

int fr_halo_size(fr_mesh_t m, int32_t q, int64_t *n_faces, int64_t *bytes) {
  if (!valid_mesh(m) || !m->group || q < 0 || q >= (int32_t)m->n_send.size())
    return pfail(FR_ERR_ARG, "not a part of a partition group, or q out of range");
  if (n_faces) *n_faces = m->n_send[q];
  if (bytes) *bytes = message_bytes(m->dm, m->n_send[q]);
  return FR_OK;
}

int fr_halo_pack(fr_mesh_t m, int32_t q, void *send) {
  if (!valid_mesh(m) || !m->group || q < 0 || q >= (int32_t)m->n_send.size())
    return pfail(FR_ERR_ARG, "not a part of a partition group, or q out of range");
  if (m->n_send[q] > 0 && !send) return pfail(FR_ERR_ARG, "send is NULL");
  return pack(m, q, send);
}

int fr_halo_unpack(fr_mesh_t m, int32_t q, const void *recv) {
  if (!valid_mesh(m) || !m->group || q < 0 || q >= (int32_t)m->n_recv.size())
    return pfail(FR_ERR_ARG, "not a part of a partition group, or q out of range");
  if (m->n_recv[q] > 0 && !recv) return pfail(FR_ERR_ARG, "recv is NULL");
  return unpack(m, q, recv);
}

int fr_part_residual(fr_part_t g, double *const *R, int on_device) {
  if (!valid_group(g) || !R) return pfail(FR_ERR_ARG, "bad group or NULL pointer");
  for (fr_mesh_s *m : g->parts)
    if (m->dm.sgs) return pfail(FR_ERR_UNSUPPORTED, "the eddy-viscosity closure is not exchanged between parts");
  const int np = (int)g->parts.size();
  std::vector<double *> dst(np, nullptr);
  int rc = FR_OK;
  for (int q = 0; q < np && rc == FR_OK; ++q) {
    if (!R[q]) rc = pfail(FR_ERR_ARG, "R[" + std::to_string(q) + "] is NULL");
    else if (on_device) dst[q] = R[q];
    else if (hipMalloc(&dst[q], (size_t)g->parts[q]->dm.E * 5 * g->parts[q]->dm.Ns * sizeof(double)) != hipSuccess)
      rc = pfail(FR_ERR_OOM, "hipMalloc of a residual staging buffer");
  }
  if (rc == FR_OK) rc = group_stage(g, FR_LSRK45, 0, 0.0, true, true, dst.data());
  for (int q = 0; q < np && rc == FR_OK && !on_device; ++q) {
    const DeviceMesh &dm = g->parts[q]->dm;
    if (hipMemcpyAsync(R[q], dst[q], (size_t)dm.E * 5 * dm.Ns * sizeof(double), hipMemcpyDeviceToHost,
                       (hipStream_t)dm.stream) != hipSuccess ||
        hipStreamSynchronize((hipStream_t)dm.stream) != hipSuccess)
      rc = pfail(FR_ERR_HIP, "copy of a part's residual");
  }
  if (!on_device)
    for (double *p : dst)
      if (p) (void)hipFree(p);
  return rc;
}

int fr_part_rk_step(fr_part_t g, double dt, int scheme, int n_steps) {
  if (!valid_group(g)) return pfail(FR_ERR_ARG, "not a partition group handle");
  const int ns = n_stages(scheme);
  if (ns == 0) return pfail(FR_ERR_ARG, "unknown scheme");
  if (n_steps < 0 || !std::isfinite(dt)) return pfail(FR_ERR_ARG, "bad dt or n_steps");
  if (n_steps == 0) return FR_OK;
  for (fr_mesh_s *m : g->parts) {
    if (m->dm.sgs) return pfail(FR_ERR_UNSUPPORTED, "the eddy-viscosity closure is not exchanged between parts");
    int rc = ensure_registers(m->dm, scheme);
    if (rc) return rc;
  }
  for (int step = 0; step < n_steps; ++step)
    for (int s = 0; s < ns; ++s) {
      int rc = group_stage(g, scheme, s, dt, step == 0 && s == 0, step == n_steps - 1 && s == ns - 1, nullptr);
      if (rc) return rc;
    }
  return FR_OK;
}

}  // extern "C"
