// fr_mlp.hip -- the per-element network of the learned eddy-viscosity closure on gfx950.
//
// Forward and backward passes run one wavefront per 16 samples on the matrix cores
// (v_mfma_f32_16x16x16_bf16, float32 accumulation). With that instruction a wave holds the
// 16x16 result tile D[m][n] as lane (g = lane/16, c = lane%16) -> rows 4g..4g+3 of column c,
// which is exactly the lane layout of its B operand (rows k = 4g..4g+3 of column c). A layer's
// output tile t therefore feeds the next layer's K-step t without any data movement, and a
// sample's 64 hidden values stay in the registers of the four lanes that share its column.
//
// Weights are the bfloat16 roundings of float32 masters. An activation x enters a product as
// hi + lo, hi = bf16(x), lo = bf16(x - hi) (two MFMAs), which represents it to 2^-17 relative,
// so the products see the weights exactly and the activations nearly exactly.
//
// Training: a per-sample pass writes the activations and back-propagated deltas; a second
// kernel reduces the weight gradients over samples (dW = delta^T h on the matrix cores with
// hi/lo splits of both operands: hi*hi + hi*lo + lo*hi) into per-split partial sums; the Adam
// kernel adds the partials in a fixed order and updates the masters and their bf16 copies.
// There are no atomics: every result is deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fr.h"
#include "fr_internal.h"

using namespace frk;

namespace {

constexpr int H = 64;         // hidden units per layer
constexpr int kMaxIn = 128;   // inputs (padded to a multiple of 16)
constexpr int kSplit = 256;   // samples per partial sum of the weight gradients

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_bits(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even (finite inputs)
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

__device__ __forceinline__ void split4(const float x[4], v4s &hi, v4s &lo) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const unsigned short h = bf16_bits(x[i]);
    hi[i] = (short)h;
    lo[i] = (short)bf16_bits(x[i] - bf16_val(h));
  }
}

__device__ __forceinline__ v4f mfma(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float softplus(float z) { return z > 20.f ? z : log1pf(expf(z)); }
__device__ __forceinline__ float logistic(float z) { return 1.f / (1.f + expf(-z)); }

// Device state of one network.
struct Net {
  int F, FP;                 // inputs; padded to a multiple of 16
  int64_t np;                // parameters
  int64_t oW1, ob1, oW2, ob2, ow3, ob3;
  float *theta = nullptr;    // float32 masters [np]
  float *am = nullptr;       // Adam first moments [np]
  float *av = nullptr;       // Adam second moments [np]
  unsigned short *W1b = nullptr;   // [H][FP] bf16, zero padded
  unsigned short *W2b = nullptr;   // [H][H]
  unsigned short *W2Tb = nullptr;  // [H][H] transposed
  float *w3r = nullptr;      // [H] bf16-rounded w3 as float
  float *mean = nullptr;     // [FP] (0 beyond F)
  float *istd = nullptr;     // [FP] 1/std (0 beyond F)
  // training scratch, per sample
  int64_t cap = 0;
  float *xh = nullptr, *h1 = nullptr, *h2 = nullptr, *d1 = nullptr, *d2 = nullptr, *dz = nullptr, *sq = nullptr;
  float *part = nullptr;     // [splits][np + 1]
  int64_t part_cap = 0;
  float *grad = nullptr;     // [np]
  float *dloss = nullptr;    // [1]
  int step = 0;
};

struct NetArgs {
  int F, FP;
  const unsigned short *W1b, *W2b, *W2Tb;
  const float *b1, *b2, *w3r, *b3, *mean, *istd;
};

// ------------------------------------------------------------------------------------------
// Forward pass (TRAIN: also the loss terms and the back-propagated deltas), 4 waves per block,
// 16 samples per wave.
// ------------------------------------------------------------------------------------------
template <int KT, bool TRAIN>
__global__ __launch_bounds__(256) void k_mlp(NetArgs a, const float *__restrict__ X, int64_t n, int64_t ldx,
                                             float *__restrict__ y, double *__restrict__ nu, double nu_scale,
                                             const float *__restrict__ tgt, float inv_n, float *__restrict__ xh,
                                             float *__restrict__ h1o, float *__restrict__ h2o,
                                             float *__restrict__ d1o, float *__restrict__ d2o,
                                             float *__restrict__ dzo, float *__restrict__ sqo) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int64_t s = ((int64_t)blockIdx.x * 4 + wave) * 16 + c;  // this lane's sample
  const bool ok = s < n;

  // standardised inputs, B layout of K-step kk: rows k = 16 kk + 4 g + i, column = sample
  float xr[KT][4];
#pragma unroll
  for (int kk = 0; kk < KT; ++kk)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 16 * kk + 4 * g + i;
      xr[kk][i] = (ok && k < a.F) ? (X[s * ldx + k] - a.mean[k]) * a.istd[k] : 0.f;
    }
  if (TRAIN && ok) {
#pragma unroll
    for (int kk = 0; kk < KT; ++kk)
      *(float4 *)&xh[s * a.FP + 16 * kk + 4 * g] = make_float4(xr[kk][0], xr[kk][1], xr[kk][2], xr[kk][3]);
  }
  // layer 1
  float h1[4][4];
  {
    v4s bh[KT], bl[KT];
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) split4(xr[kk], bh[kk], bl[kk]);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      v4f acc;
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] = a.b1[16 * t + 4 * g + i];
#pragma unroll
      for (int kk = 0; kk < KT; ++kk) {
        const v4s w = *(const v4s *)&a.W1b[(16 * t + c) * a.FP + 16 * kk + 4 * g];
        acc = mfma(w, bh[kk], acc);
        acc = mfma(w, bl[kk], acc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) h1[t][i] = tanhf(acc[i]);
    }
  }
  // layer 2
  float h2[4][4];
  {
    v4s bh[4], bl[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) split4(h1[t], bh[t], bl[t]);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      v4f acc;
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] = a.b2[16 * t + 4 * g + i];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const v4s w = *(const v4s *)&a.W2b[(16 * t + c) * H + 16 * kk + 4 * g];
        acc = mfma(w, bh[kk], acc);
        acc = mfma(w, bl[kk], acc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) h2[t][i] = tanhf(acc[i]);
    }
  }
  // output unit: the four lanes of a column hold its 64 values; reduce over g
  float z = 0.f;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) z += a.w3r[16 * t + 4 * g + i] * h2[t][i];
  z += __shfl_xor(z, 16);
  z += __shfl_xor(z, 32);
  z += a.b3[0];
  const float yv = softplus(z);
  if (!TRAIN) {
    if (ok && g == 0) {
      if (y) y[s] = yv;
      if (nu) nu[s] = nu_scale * (double)yv;
    }
    return;
  }
  // loss terms and dL/dz = 2 (y - t) / n * softplus'(z)
  const float r = ok ? yv - tgt[s] : 0.f;
  const float dz = ok ? 2.f * r * inv_n * logistic(z) : 0.f;
  if (ok && g == 0) {
    if (y) y[s] = yv;
    dzo[s] = dz;
    sqo[s] = r * r;
  }
  // delta2 = dz w3 (1 - h2^2), D layout
  float d2[4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) d2[t][i] = dz * a.w3r[16 * t + 4 * g + i] * (1.f - h2[t][i] * h2[t][i]);
  // delta1 = (W2^T delta2) (1 - h1^2)
  float d1[4][4];
  {
    v4s bh[4], bl[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) split4(d2[t], bh[t], bl[t]);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const v4s w = *(const v4s *)&a.W2Tb[(16 * t + c) * H + 16 * kk + 4 * g];
        acc = mfma(w, bh[kk], acc);
        acc = mfma(w, bl[kk], acc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) d1[t][i] = acc[i] * (1.f - h1[t][i] * h1[t][i]);
    }
  }
  if (ok) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t o = s * H + 16 * t + 4 * g;
      *(float4 *)&h1o[o] = make_float4(h1[t][0], h1[t][1], h1[t][2], h1[t][3]);
      *(float4 *)&h2o[o] = make_float4(h2[t][0], h2[t][1], h2[t][2], h2[t][3]);
      *(float4 *)&d1o[o] = make_float4(d1[t][0], d1[t][1], d1[t][2], d1[t][3]);
      *(float4 *)&d2o[o] = make_float4(d2[t][0], d2[t][1], d2[t][2], d2[t][3]);
    }
  }
}

// ------------------------------------------------------------------------------------------
// Weight-gradient partial sums over split blockIdx.y (samples [y*kSplit, (y+1)*kSplit) ∩ [0,n)).
// One wave per job: jobs 0..4KT-1 are 16x16 tiles of dW1 = sum_s delta1_s xh_s^T, the next 16
// tiles of dW2 = sum_s delta2_s h1_s^T, then db1, db2, dw3 and (db3, loss).
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_mlp_wgrad(int F, int FP, int KT, int64_t n, const float *__restrict__ xh,
                                                  const float *__restrict__ h1, const float *__restrict__ h2,
                                                  const float *__restrict__ d1, const float *__restrict__ d2,
                                                  const float *__restrict__ dz, const float *__restrict__ sq,
                                                  int64_t np, int64_t oW1, int64_t ob1, int64_t oW2, int64_t ob2,
                                                  int64_t ow3, int64_t ob3, float inv_n, float *__restrict__ part) {
  const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
  const int job = blockIdx.x;
  const int64_t s0 = (int64_t)blockIdx.y * kSplit;
  const int64_t s1 = s0 + kSplit < n ? s0 + kSplit : n;
  float *out = part + (int64_t)blockIdx.y * (np + 1);
  const int nW1 = 4 * KT;
  if (job < nW1 + 16) {
    // tile (row block tm, column block tn) of dW = sum_s A_s B_s^T with A = delta (64 rows)
    // and B = xh or h1; MFMA K runs over samples: A-operand lane (g, c) needs
    // delta[s0 + 4g + i][16 tm + c], B-operand lane needs B[s0 + 4g + i][16 tn + c]
    const bool w1 = job < nW1;
    const int tm = w1 ? job / KT : (job - nW1) / 4;
    const int tn = w1 ? job % KT : (job - nW1) % 4;
    const float *A = w1 ? d1 : d2;
    const float *B = w1 ? xh : h1;
    const int ldb = w1 ? FP : H;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int64_t sb = s0; sb < s1; sb += 16) {
      float av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t s = sb + 4 * g + i;
        av[i] = s < s1 ? A[s * H + 16 * tm + c] : 0.f;
        bv[i] = s < s1 ? B[s * ldb + 16 * tn + c] : 0.f;
      }
      v4s ah, al, bh, bl;
      split4(av, ah, al);
      split4(bv, bh, bl);
      acc = mfma(ah, bh, acc);
      acc = mfma(ah, bl, acc);
      acc = mfma(al, bh, acc);
    }
    // D[m][k]: lane holds rows 16 tm + 4g + i, column 16 tn + c
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = 16 * tm + 4 * g + i, k = 16 * tn + c;
      if (w1) {
        if (k < F) out[oW1 + (int64_t)m * F + k] = acc[i];
      } else {
        out[oW2 + (int64_t)m * H + k] = acc[i];
      }
    }
    return;
  }
  const int v = job - nW1 - 16;  // 0 db1, 1 db2, 2 dw3, 3 (db3, loss)
  if (v < 3) {
    const float *src = v == 0 ? d1 : (v == 1 ? d2 : h2);
    float acc = 0.f;
    for (int64_t s = s0; s < s1; ++s) acc += (v == 2 ? dz[s] : 1.f) * src[s * H + lane];
    out[(v == 0 ? ob1 : (v == 1 ? ob2 : ow3)) + lane] = acc;
  } else {
    float a = 0.f, b = 0.f;
    for (int64_t s = s0 + lane; s < s1; s += 64) {
      a += dz[s];
      b += sq[s];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_xor(a, o);
      b += __shfl_xor(b, o);
    }
    if (lane == 0) {
      out[ob3] = a;
      out[np] = b * inv_n;
    }
  }
}

// bf16 copies of parameter i from its master value
__device__ __forceinline__ void write_copies(int64_t i, float th, int F, int FP, int64_t oW1, int64_t oW2,
                                             int64_t ow3, unsigned short *W1b, unsigned short *W2b,
                                             unsigned short *W2Tb, float *w3r) {
  if (i >= oW1 && i < oW1 + (int64_t)H * F) {
    const int64_t j = i - oW1;
    W1b[(j / F) * FP + j % F] = bf16_bits(th);
  } else if (i >= oW2 && i < oW2 + H * H) {
    const int j = (int)(i - oW2);
    const unsigned short b = bf16_bits(th);
    W2b[j] = b;
    W2Tb[(j % H) * H + j / H] = b;
  } else if (i >= ow3 && i < ow3 + H) {
    w3r[i - ow3] = bf16_val(bf16_bits(th));
  }
}

// Sum the partials in split order; optionally export the gradient and the loss; optionally
// take one Adam step and refresh the bf16 copies.
__global__ __launch_bounds__(256) void k_mlp_adam(const float *__restrict__ part, int splits, int64_t np,
                                                  float *__restrict__ grad, float *__restrict__ loss, int update,
                                                  float lr, float c1, float c2, float *__restrict__ theta,
                                                  float *__restrict__ am, float *__restrict__ av, int F, int FP,
                                                  int64_t oW1, int64_t oW2, int64_t ow3, unsigned short *W1b,
                                                  unsigned short *W2b, unsigned short *W2Tb, float *w3r) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i > np) return;
  float gsum = 0.f;
  for (int s = 0; s < splits; ++s) gsum += part[(int64_t)s * (np + 1) + i];
  if (i == np) {
    if (loss) *loss = gsum;
    return;
  }
  if (grad) grad[i] = gsum;
  if (!update) return;
  const float m = 0.9f * am[i] + 0.1f * gsum;
  const float v = 0.999f * av[i] + 0.001f * gsum * gsum;
  am[i] = m;
  av[i] = v;
  const float th = theta[i] - lr * (m * c1) / (sqrtf(v * c2) + 1e-8f);
  theta[i] = th;
  write_copies(i, th, F, FP, oW1, oW2, ow3, W1b, W2b, W2Tb, w3r);
}

__global__ __launch_bounds__(256) void k_mlp_refresh(const float *__restrict__ theta, int64_t np, int F, int FP,
                                                     int64_t oW1, int64_t oW2, int64_t ow3, unsigned short *W1b,
                                                     unsigned short *W2b, unsigned short *W2Tb, float *w3r) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  write_copies(i, theta[i], F, FP, oW1, oW2, ow3, W1b, W2b, W2Tb, w3r);
}

}  // namespace

struct fr_mlp_s {
  uint64_t magic;
  Net net;
  hipStream_t stream;
  int device;
};

namespace {

constexpr uint64_t kMlpMagic = 0x46524d4c504e4554ull;  // "FRMLPNET"

bool valid(fr_mlp_t m) { return m && m->magic == kMlpMagic; }

#define MCHK(call)                                                                               \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) return fr_fail(FR_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

NetArgs args_of(const Net &n) {
  NetArgs a;
  a.F = n.F;
  a.FP = n.FP;
  a.W1b = n.W1b;
  a.W2b = n.W2b;
  a.W2Tb = n.W2Tb;
  a.b1 = n.theta + n.ob1;
  a.b2 = n.theta + n.ob2;
  a.w3r = n.w3r;
  a.b3 = n.theta + n.ob3;
  a.mean = n.mean;
  a.istd = n.istd;
  return a;
}

// Per-sample training buffers (activations, deltas, loss terms) and the per-split partial sums of
// the gradient: the network's own growing buffers, or a share of the fixed scratch array.
struct TrainBufs {
  float *xh = nullptr, *h1 = nullptr, *h2 = nullptr, *d1 = nullptr, *d2 = nullptr, *dz = nullptr, *sq = nullptr;
  float *part = nullptr;
};

TrainBufs net_bufs(const Net &n) {
  TrainBufs b;
  b.xh = n.xh;
  b.h1 = n.h1;
  b.h2 = n.h2;
  b.d1 = n.d1;
  b.d2 = n.d2;
  b.dz = n.dz;
  b.sq = n.sq;
  b.part = n.part;
  return b;
}

template <bool TRAIN>
int launch_mlp(const Net &net, hipStream_t st, const float *X, int64_t n, int64_t ldx, float *y, double *nu,
               double nu_scale, const float *tgt, const TrainBufs &tb = TrainBufs()) {
  const NetArgs a = args_of(net);
  const unsigned blocks = (unsigned)((n + 63) / 64);
  const float inv_n = 1.f / (float)n;
  switch (net.FP / 16) {
#define CASE(K)                                                                                                  \
  case K:                                                                                                        \
    hipLaunchKernelGGL((k_mlp<K, TRAIN>), dim3(blocks), dim3(256), 0, st, a, X, n, ldx, y, nu, nu_scale, tgt,   \
                       inv_n, tb.xh, tb.h1, tb.h2, tb.d1, tb.d2, tb.dz, tb.sq);                                   \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return fr_fail(FR_ERR_ARG, "network input size out of range");
  }
  MCHK(hipGetLastError());
  return FR_OK;
}

int ensure_scratch(Net &net, int64_t n) {
  if (n > net.cap) {
    for (float *p : {net.xh, net.h1, net.h2, net.d1, net.d2, net.dz, net.sq})
      if (p) (void)hipFree(p);
    const int64_t cap = n;
    MCHK(hipMalloc(&net.xh, cap * net.FP * sizeof(float)));
    MCHK(hipMalloc(&net.h1, cap * H * sizeof(float)));
    MCHK(hipMalloc(&net.h2, cap * H * sizeof(float)));
    MCHK(hipMalloc(&net.d1, cap * H * sizeof(float)));
    MCHK(hipMalloc(&net.d2, cap * H * sizeof(float)));
    MCHK(hipMalloc(&net.dz, cap * sizeof(float)));
    MCHK(hipMalloc(&net.sq, cap * sizeof(float)));
    net.cap = cap;
  }
  const int64_t splits = (n + kSplit - 1) / kSplit;
  if (splits > net.part_cap) {
    if (net.part) (void)hipFree(net.part);
    MCHK(hipMalloc(&net.part, splits * (net.np + 1) * sizeof(float)));
    net.part_cap = splits;
  }
  return FR_OK;
}

// forward + backward + gradient reduction; then the Adam kernel (update or export only). fixed:
// training buffers to use instead of the network's own (which are grown here otherwise).
int grad_pass(fr_mlp_t m, const float *X, int64_t n, int64_t ldx, const float *t, bool update, float lr,
              float *loss_dev, const TrainBufs *fixed = nullptr) {
  Net &net = m->net;
  if (!X || !t || n <= 0 || ldx < net.F) return fr_fail(FR_ERR_ARG, "bad X / t / n / ldx");
  if (!fixed) {
    int rc = ensure_scratch(net, n);
    if (rc) return rc;
  }
  const TrainBufs tb = fixed ? *fixed : net_bufs(net);
  int rc = launch_mlp<true>(net, m->stream, X, n, ldx, nullptr, nullptr, 0.0, t, tb);
  if (rc) return rc;
  const int KT = net.FP / 16;
  const int64_t splits = (n + kSplit - 1) / kSplit;
  const int jobs = 4 * KT + 16 + 4;
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(jobs, (unsigned)splits), dim3(64), 0, m->stream, net.F, net.FP, KT, n,
                     tb.xh, tb.h1, tb.h2, tb.d1, tb.d2, tb.dz, tb.sq, net.np, net.oW1, net.ob1, net.oW2,
                     net.ob2, net.ow3, net.ob3, 1.f / (float)n, tb.part);
  MCHK(hipGetLastError());
  float c1 = 1.f, c2 = 1.f;
  if (update) {
    net.step += 1;
    c1 = (float)(1.0 / (1.0 - std::pow(0.9, net.step)));
    c2 = (float)(1.0 / (1.0 - std::pow(0.999, net.step)));
  }
  hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)((net.np + 1 + 255) / 256)), dim3(256), 0, m->stream, tb.part,
                     (int)splits, net.np, update ? nullptr : net.grad, loss_dev, update ? 1 : 0, lr, c1, c2,
                     net.theta, net.am, net.av, net.F, net.FP, net.oW1, net.oW2, net.ow3, net.W1b, net.W2b,
                     net.W2Tb, net.w3r);
  MCHK(hipGetLastError());
  return FR_OK;
}

int upload_params(fr_mlp_t m, const float *params) {
  Net &net = m->net;
  MCHK(hipMemcpyAsync(net.theta, params, net.np * sizeof(float), hipMemcpyHostToDevice, m->stream));
  MCHK(hipMemsetAsync(net.am, 0, net.np * sizeof(float), m->stream));
  MCHK(hipMemsetAsync(net.av, 0, net.np * sizeof(float), m->stream));
  hipLaunchKernelGGL(k_mlp_refresh, dim3((unsigned)((net.np + 255) / 256)), dim3(256), 0, m->stream, net.theta,
                     net.np, net.F, net.FP, net.oW1, net.oW2, net.ow3, net.W1b, net.W2b, net.W2Tb, net.w3r);
  MCHK(hipGetLastError());
  MCHK(hipStreamSynchronize(m->stream));
  net.step = 0;
  return FR_OK;
}

void free_net(Net &n) {
  for (void *p : {(void *)n.theta, (void *)n.am, (void *)n.av, (void *)n.W1b, (void *)n.W2b, (void *)n.W2Tb,
                  (void *)n.w3r, (void *)n.mean, (void *)n.istd, (void *)n.xh, (void *)n.h1, (void *)n.h2,
                  (void *)n.d1, (void *)n.d2, (void *)n.dz, (void *)n.sq, (void *)n.part, (void *)n.grad,
                  (void *)n.dloss})
    if (p) (void)hipFree(p);
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Training without allocation (fr_mlp_train_step_noalloc): the training buffers of one call live
// in `scratch`, a fixed array each GPU holds for the life of the process, sized for
// kNoAllocMaxN samples at the largest input count. Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): each device's address comes from
// hipGetSymbolAddress, taken once per device with that device current, and is kept here.
// ------------------------------------------------------------------------------------------
namespace {

constexpr int64_t kNoAllocMaxN = FR_MLP_NOALLOC_MAX_N;
constexpr int64_t kMaxParams = (int64_t)H * kMaxIn + H + H * H + H + H + 1;
constexpr int64_t kAlignFloats = 64;  // 256 bytes between the sub-buffers
constexpr int64_t align_floats(int64_t x) { return (x + kAlignFloats - 1) / kAlignFloats * kAlignFloats; }
constexpr int64_t scratch_floats(int64_t n, int64_t fp, int64_t np) {
  return align_floats(n * fp) + 4 * align_floats(n * H) + 2 * align_floats(n) +
         align_floats(((n + kSplit - 1) / kSplit) * (np + 1));
}
constexpr int64_t kScratchFloats = scratch_floats(kNoAllocMaxN, kMaxIn, kMaxParams);  // 14.2 MiB

}  // namespace

static __device__ __align__(256) float scratch[kScratchFloats];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_addr[kMaxDevices] = {};

// The device address of `scratch` on device dev (looked up once per device, that device made
// current for the lookup).
int scratch_address(int dev, float **out) {
  if (dev < 0 || dev >= kMaxDevices) return fr_fail(FR_ERR_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    int cur = -1;
    MCHK(hipGetDevice(&cur));
    if (cur != dev) MCHK(hipSetDevice(dev));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      return fr_fail(FR_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_addr[dev] = (float *)p;
  }
  *out = g_scratch_addr[dev];
  return FR_OK;
}

}  // namespace

namespace frk {

int mlp_n_in(fr_mlp_t m) { return valid(m) ? m->net.F : -1; }

int mlp_forward_nu(fr_mlp_t m, const float *X, int64_t n, int64_t ldx, double *nu, double nu_scale,
                   void *stream) {
  if (!valid(m)) return fr_fail(FR_ERR_ARG, "invalid network handle");
  return launch_mlp<false>(m->net, (hipStream_t)stream, X, n, ldx, nullptr, nu, nu_scale, nullptr);
}

}  // namespace frk

extern "C" {

int64_t fr_mlp_n_params(int32_t n_in) { return (int64_t)H * n_in + H + H * H + H + H + 1; }

int fr_mlp_create(int32_t n_in, const float *params, const float *mean, const float *std_dev, void *hip_stream,
                  fr_mlp_t *out) {
  if (!out) return fr_fail(FR_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (n_in < 1 || n_in > kMaxIn) return fr_fail(FR_ERR_ARG, "n_in must be in 1..128");
  if (!params || !mean || !std_dev) return fr_fail(FR_ERR_ARG, "params / mean / std is NULL");
  for (int k = 0; k < n_in; ++k)
    if (!(std_dev[k] > 0.f) || !std::isfinite(mean[k])) return fr_fail(FR_ERR_ARG, "std must be > 0, mean finite");
  const int64_t np = fr_mlp_n_params(n_in);
  for (int64_t i = 0; i < np; ++i)
    if (!std::isfinite(params[i])) return fr_fail(FR_ERR_ARG, "non-finite parameter");
  fr_mlp_s *m = new fr_mlp_s();
  m->magic = kMlpMagic;
  m->stream = (hipStream_t)hip_stream;
  (void)hipGetDevice(&m->device);
  Net &n = m->net;
  n.F = n_in;
  n.FP = (n_in + 15) / 16 * 16;
  n.np = np;
  n.oW1 = 0;
  n.ob1 = (int64_t)H * n_in;
  n.oW2 = n.ob1 + H;
  n.ob2 = n.oW2 + H * H;
  n.ow3 = n.ob2 + H;
  n.ob3 = n.ow3 + H;
  auto fail_free = [&](const std::string &msg) {
    free_net(n);
    delete m;
    return fr_fail(FR_ERR_HIP, msg);
  };
  if (hipMalloc(&n.theta, np * sizeof(float)) || hipMalloc(&n.am, np * sizeof(float)) ||
      hipMalloc(&n.av, np * sizeof(float)) || hipMalloc(&n.W1b, (size_t)H * n.FP * 2) ||
      hipMalloc(&n.W2b, H * H * 2) || hipMalloc(&n.W2Tb, H * H * 2) || hipMalloc(&n.w3r, H * sizeof(float)) ||
      hipMalloc(&n.mean, n.FP * sizeof(float)) || hipMalloc(&n.istd, n.FP * sizeof(float)) ||
      hipMalloc(&n.grad, np * sizeof(float)) || hipMalloc(&n.dloss, sizeof(float)))
    return fail_free("hipMalloc failed");
  std::vector<float> mp(n.FP, 0.f), ip(n.FP, 0.f);
  for (int k = 0; k < n_in; ++k) {
    mp[k] = mean[k];
    ip[k] = 1.f / std_dev[k];
  }
  if (hipMemcpy(n.mean, mp.data(), n.FP * sizeof(float), hipMemcpyHostToDevice) ||
      hipMemcpy(n.istd, ip.data(), n.FP * sizeof(float), hipMemcpyHostToDevice) ||
      hipMemset(n.W1b, 0, (size_t)H * n.FP * 2) || hipDeviceSynchronize())
    return fail_free("initial copies failed");
  int rc = upload_params(m, params);
  if (rc) {
    free_net(n);
    delete m;
    return rc;
  }
  *out = m;
  return FR_OK;
}

int fr_mlp_destroy(fr_mlp_t m) {
  if (!m) return FR_OK;
  if (!valid(m)) return fr_fail(FR_ERR_ARG, "invalid network handle");
  (void)hipStreamSynchronize(m->stream);
  free_net(m->net);
  m->magic = 0;
  delete m;
  return FR_OK;
}

int fr_mlp_set_stream(fr_mlp_t m, void *hip_stream) {
  if (!valid(m)) return fr_fail(FR_ERR_ARG, "invalid network handle");
  m->stream = (hipStream_t)hip_stream;
  return FR_OK;
}

int fr_mlp_set_params(fr_mlp_t m, const float *params) {
  if (!valid(m) || !params) return fr_fail(FR_ERR_ARG, "invalid network handle or params");
  for (int64_t i = 0; i < m->net.np; ++i)
    if (!std::isfinite(params[i])) return fr_fail(FR_ERR_ARG, "non-finite parameter");
  return upload_params(m, params);
}

int fr_mlp_get_params(fr_mlp_t m, float *params) {
  if (!valid(m) || !params) return fr_fail(FR_ERR_ARG, "invalid network handle or params");
  MCHK(hipMemcpyAsync(params, m->net.theta, m->net.np * sizeof(float), hipMemcpyDeviceToHost, m->stream));
  MCHK(hipStreamSynchronize(m->stream));
  return FR_OK;
}

int fr_mlp_get_bf16(fr_mlp_t m, uint16_t *W1, uint16_t *W2, uint16_t *w3) {
  if (!valid(m)) return fr_fail(FR_ERR_ARG, "invalid network handle");
  const Net &n = m->net;
  MCHK(hipStreamSynchronize(m->stream));
  if (W1) {
    std::vector<uint16_t> tmp((size_t)H * n.FP);
    MCHK(hipMemcpy(tmp.data(), n.W1b, tmp.size() * 2, hipMemcpyDeviceToHost));
    for (int r = 0; r < H; ++r)
      for (int k = 0; k < n.F; ++k) W1[r * n.F + k] = tmp[(size_t)r * n.FP + k];
  }
  if (W2) MCHK(hipMemcpy(W2, n.W2b, H * H * 2, hipMemcpyDeviceToHost));
  if (w3) {
    float tmp[H];
    MCHK(hipMemcpy(tmp, n.w3r, sizeof tmp, hipMemcpyDeviceToHost));
    for (int i = 0; i < H; ++i) {
      uint32_t u;
      std::memcpy(&u, &tmp[i], 4);
      w3[i] = (uint16_t)(u >> 16);
    }
  }
  return FR_OK;
}

int fr_mlp_forward(fr_mlp_t m, const float *X, int64_t n, int64_t ldx, float *y) {
  if (!valid(m)) return fr_fail(FR_ERR_ARG, "invalid network handle");
  if (n == 0) return FR_OK;
  if (!X || !y || n < 0 || ldx < m->net.F) return fr_fail(FR_ERR_ARG, "bad X / y / n / ldx");
  return launch_mlp<false>(m->net, m->stream, X, n, ldx, y, nullptr, 0.0, nullptr);
}

int fr_mlp_loss_grad(fr_mlp_t m, const float *X, int64_t n, int64_t ldx, const float *t, float *grad,
                     double *loss) {
  if (!valid(m)) return fr_fail(FR_ERR_ARG, "invalid network handle");
  int rc = grad_pass(m, X, n, ldx, t, false, 0.f, m->net.dloss);
  if (rc) return rc;
  if (grad) MCHK(hipMemcpyAsync(grad, m->net.grad, m->net.np * sizeof(float), hipMemcpyDeviceToHost, m->stream));
  float l = 0.f;
  MCHK(hipMemcpyAsync(&l, m->net.dloss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
  MCHK(hipStreamSynchronize(m->stream));
  if (loss) *loss = l;
  return FR_OK;
}

int fr_mlp_train_step(fr_mlp_t m, const float *X, int64_t n, int64_t ldx, const float *t, float lr, float *loss) {
  if (!valid(m)) return fr_fail(FR_ERR_ARG, "invalid network handle");
  if (!(lr > 0.f)) return fr_fail(FR_ERR_ARG, "lr must be > 0");
  return grad_pass(m, X, n, ldx, t, true, lr, loss);
}

int fr_mlp_train_step_noalloc(fr_mlp_t m, const float *X, int64_t n, int64_t ldx, const float *t, float lr,
                              float *loss) {
  if (!valid(m)) return fr_fail(FR_ERR_ARG, "invalid network handle");
  if (!(lr > 0.f)) return fr_fail(FR_ERR_ARG, "lr must be > 0");
  if (n <= 0 || n > kNoAllocMaxN)
    return fr_fail(FR_ERR_ARG, "n must be in 1.." + std::to_string(kNoAllocMaxN) + " for the no-allocation step");
  const Net &net = m->net;
  if (scratch_floats(n, net.FP, net.np) > kScratchFloats) return fr_fail(FR_ERR_ARG, "batch exceeds the scratch array");
  float *base = nullptr;
  int rc = scratch_address(m->device, &base);
  if (rc) return rc;
  // every entry of these buffers that a kernel reads is first written by this call's kernels
  // (activations and deltas for samples < n, every partial sum of every split)
  TrainBufs tb;
  float *q = base;
  auto take = [&](int64_t nf) {
    float *r = q;
    q += align_floats(nf);
    return r;
  };
  tb.xh = take(n * net.FP);
  tb.h1 = take(n * H);
  tb.h2 = take(n * H);
  tb.d1 = take(n * H);
  tb.d2 = take(n * H);
  tb.dz = take(n);
  tb.sq = take(n);
  tb.part = take(((n + kSplit - 1) / kSplit) * (net.np + 1));
  return grad_pass(m, X, n, ldx, t, true, lr, loss, &tb);
}

}  // extern "C"
