// Training of the extraction-threshold model (an addition to the paper's
// method: a small MLP that picks how many minima a parDijkstra round pulls).
//
//  k_trace_labels  label of a traced round = log2 of the longest prefix of
//                  B_0 (in key order) whose keys are already final distances
//                  (pulling that many minima wastes no relaxation)
//  k_feat_stats    per-feature mean and standard deviation of the dataset
//  k_mlp_grad      one mini-batch: forward 8 -> 64 -> 64 -> 1 (GELU, weights
//                  rounded to bfloat16, FP32 accumulation), mean squared error,
//                  backward to the FP32 master weights (the rounding is taken
//                  as identity)
//  k_adam          Adam step on the master weights
//
// Layout of the parameter blob: see sssp_opts.k_model in include/pbh.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "../../include/pbh.h"
#include "pbh_core.h"

namespace bkt {

constexpr int H = MLP_H;
constexpr int F = NFEAT;
constexpr int OW1 = 0, OB1 = F * H, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H;
constexpr int OMU = MLP_PARAMS, OSD = OMU + F, OSC = OSD + F;

__device__ __forceinline__ float gelu_d(float x) {
  // d/dx [x Phi(x)] = Phi(x) + x phi(x)
  const float phi = 0.3989422804014327f * expf(-0.5f * x * x);
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * phi;
}

// Every record names a query < nq, and every traced id (padding keys KINF
// aside) is a vertex of that query's graph; *bad != 0 otherwise.
__global__ void k_trace_check(const u64* tk, const u32* tv, const u32* tq, u32 count, const u32* dist_n, u32 nq,
                              u32* bad) {
  for (u32 r = blockIdx.x * blockDim.x + threadIdx.x; r < count; r += gridDim.x * blockDim.x) {
    const u32 q = tq[r];
    bool b = q >= nq;
    if (!b) {
      const u32 n = dist_n[q];
      for (int k = 0; k < TRACE_K; ++k)
        b = b || (tk[(u64)r * TRACE_K + k] != KINF && tv[(u64)r * TRACE_K + k] >= n);
    }
    if (b) atomicOr(bad, 1u);
  }
}

__global__ void k_trace_labels(const u64* tk, const u32* tv, const u32* tq, u32 count, const u64* const* dists,
                               float* labels) {
  for (u32 r = blockIdx.x * blockDim.x + threadIdx.x; r < count; r += gridDim.x * blockDim.x) {
    const u64* dist = dists[tq[r]];
    u32 k = 0;
    while (k < (u32)TRACE_K) {
      u64 key = tk[(u64)r * TRACE_K + k];
      if (key == KINF || dist[tv[(u64)r * TRACE_K + k]] != key) break;
      ++k;
    }
    labels[r] = log2f((float)(k < 1 ? 1 : k));
  }
}

// mu[f], sd[f] over n samples (one workgroup per feature).
__global__ void k_feat_stats(const float* X, u32 n, float* blob) {
  __shared__ double s1[256], s2[256];
  const int f = blockIdx.x;
  double a = 0, b = 0;
  for (u32 i = threadIdx.x; i < n; i += blockDim.x) {
    double x = X[(u64)i * F + f];
    a += x;
    b += x * x;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s1[threadIdx.x] += s1[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double m = s1[0] / (n ? n : 1), v = s2[0] / (n ? n : 1) - m * m;
    blob[OMU + f] = (float)m;
    blob[OSD + f] = (float)sqrt(v > 1e-12 ? v : 1e-12);
  }
}

// One mini-batch of B samples X[idx0 .. idx0+B) (one workgroup of 256
// threads).  grad[MLP_PARAMS] receives the gradient of the mean squared error,
// loss[0] the loss.  Scratch: 4 * B * H floats.
__global__ __launch_bounds__(256) void k_mlp_grad(const float* blob, const float* X, const float* Y, u32 idx0, u32 B,
                                                  float* grad, float* loss, float* scr) {
  __shared__ float w[MLP_PARAMS];
  __shared__ float red[256];
  float* H1 = scr;               // gelu(z1)   [B][H]
  float* Z1 = scr + B * H;       // z1         [B][H], later dL/dz1
  float* Z2 = scr + 2 * B * H;   // z2         [B][H], later dL/dz2
  float* DY = scr + 3 * B * H;   // dL/dy      [B]
  const float* mu = blob + OMU;
  const float* sd = blob + OSD;
  for (int i = threadIdx.x; i < MLP_PARAMS; i += 256) w[i] = bf16r(blob[i]);
  __syncthreads();
  // forward, one sample per thread
  float lsum = 0.f;
  for (u32 s = threadIdx.x; s < B; s += 256) {
    const float* xs = X + (u64)(idx0 + s) * F;
    float x[F];
#pragma unroll
    for (int f = 0; f < F; ++f) x[f] = (xs[f] - mu[f]) / sd[f];
    float h1[H];
    for (int j = 0; j < H; ++j) {
      float a = w[OB1 + j];
#pragma unroll
      for (int f = 0; f < F; ++f) a += w[OW1 + f * H + j] * x[f];
      Z1[s * H + j] = a;
      h1[j] = gelu(a);
      H1[s * H + j] = h1[j];
    }
    float y = w[OB3];
    for (int j = 0; j < H; ++j) {
      float a = w[OB2 + j];
      for (int i = 0; i < H; ++i) a += w[OW2 + i * H + j] * h1[i];
      Z2[s * H + j] = a;
      y += w[OW3 + j] * gelu(a);
    }
    const float e = y - Y[idx0 + s];
    lsum += e * e;
    DY[s] = 2.f * e / (float)B;
  }
  __syncthreads();
  // dL/dz2 and dL/dz1, one sample per thread (in place over Z2, Z1)
  for (u32 s = threadIdx.x; s < B; s += 256) {
    const float dy = DY[s];
    float dz2[H];
    for (int j = 0; j < H; ++j) {
      dz2[j] = dy * w[OW3 + j] * gelu_d(Z2[s * H + j]);
    }
    for (int i = 0; i < H; ++i) {
      float a = 0.f;
      for (int j = 0; j < H; ++j) a += w[OW2 + i * H + j] * dz2[j];
      Z1[s * H + i] = a * gelu_d(Z1[s * H + i]);
    }
    for (int j = 0; j < H; ++j) Z2[s * H + j] = dz2[j];
  }
  __syncthreads();
  // parameter gradients, one parameter per thread (sums over the batch)
  for (int p = threadIdx.x; p < MLP_PARAMS; p += 256) {
    float g = 0.f;
    if (p < OB1) {  // W1[f][j]
      const int f = p / H, j = p % H;
      for (u32 s = 0; s < B; ++s) g += (X[(u64)(idx0 + s) * F + f] - mu[f]) / sd[f] * Z1[s * H + j];
    } else if (p < OW2) {  // b1
      const int j = p - OB1;
      for (u32 s = 0; s < B; ++s) g += Z1[s * H + j];
    } else if (p < OB2) {  // W2[i][j]
      const int i = (p - OW2) / H, j = (p - OW2) % H;
      for (u32 s = 0; s < B; ++s) g += H1[s * H + i] * Z2[s * H + j];
    } else if (p < OW3) {  // b2
      const int j = p - OB2;
      for (u32 s = 0; s < B; ++s) g += Z2[s * H + j];
    } else if (p < OB3) {  // w3[j]: dL/dy * h2[j]; h2 = dz2 / (dy w3 gelu'(z2)) is not
                           // recoverable, so recompute h2 from h1
      const int j = p - OW3;
      for (u32 s = 0; s < B; ++s) {
        float a = w[OB2 + j];
        for (int i = 0; i < H; ++i) a += w[OW2 + i * H + j] * H1[s * H + i];
        g += DY[s] * gelu(a);
      }
    } else {  // b3
      for (u32 s = 0; s < B; ++s) g += DY[s];
    }
    grad[p] = g;
  }
  red[threadIdx.x] = lsum;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] / (float)B;
}

// Adam (Kingma & Ba 2015) on the master weights; t = step number from 1.
__global__ void k_adam(float* blob, const float* grad, float* m, float* v, float lr, float b1, float b2, float eps,
                       int t) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < MLP_PARAMS; p += gridDim.x * blockDim.x) {
    float g = grad[p];
    m[p] = b1 * m[p] + (1.f - b1) * g;
    v[p] = b2 * v[p] + (1.f - b2) * g * g;
    blob[p] -= lr * (m[p] / c1) / (sqrtf(v[p] / c2) + eps);
  }
}

// Final rounding of the trained weights to bfloat16 values.
__global__ void k_round_bf16(float* blob) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < MLP_PARAMS; p += gridDim.x * blockDim.x)
    blob[p] = bf16r(blob[p]);
}

}  // namespace bkt

using namespace bkt;

namespace {
thread_local char g_lerr[256] = "";
std::mutex g_learn_mu;
}

#define LCHK(expr)                                                                   \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      snprintf(g_lerr, sizeof g_lerr, "%s: %s", #expr, hipGetErrorString(e_));       \
      return e_ == hipErrorOutOfMemory ? PBH_ENOMEM : PBH_EDEVICE;                   \
    }                                                                                \
  } while (0)

extern "C" {

int mlp_trace_labels(const uint64_t* trace_keys, const uint32_t* trace_ids, const uint32_t* trace_query,
                     uint32_t count, const uint64_t* const* dists, const uint32_t* dist_n, uint32_t nq,
                     float* labels) {
  if (count == 0) return PBH_OK;
  if (!trace_keys || !trace_ids || !trace_query || !dists || !dist_n || nq == 0 || !labels) return PBH_EINVAL;
  u32 grid = (count + 255) / 256;
  grid = grid > 4096 ? 4096 : grid;
  std::lock_guard<std::mutex> lock(g_learn_mu);
  u32* bad = nullptr;
  LCHK(hipMalloc(&bad, sizeof(u32)));
  u32 hbad = 0;
  hipError_t e = hipMemset(bad, 0, sizeof(u32));
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_trace_check, dim3(grid), dim3(256), 0, 0, (const u64*)trace_keys, trace_ids, trace_query,
                       count, dist_n, nq, bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(&hbad, bad, sizeof(u32), hipMemcpyDeviceToHost);
  (void)hipFree(bad);
  LCHK(e);
  if (hbad) {
    snprintf(g_lerr, sizeof g_lerr, "mlp_trace_labels: a record names a query >= nq or an id >= its n");
    return PBH_EINVAL;
  }
  hipLaunchKernelGGL(k_trace_labels, dim3(grid), dim3(256), 0, 0, (const u64*)trace_keys, trace_ids, trace_query,
                     count, (const u64* const*)dists, labels);
  LCHK(hipGetLastError());
  LCHK(hipDeviceSynchronize());
  return PBH_OK;
}

int mlp_feature_stats(const float* X, uint32_t n, float* blob) {
  if (!X || !blob || n == 0) return PBH_EINVAL;
  hipLaunchKernelGGL(k_feat_stats, dim3(F), dim3(256), 0, 0, X, n, blob);
  LCHK(hipGetLastError());
  LCHK(hipDeviceSynchronize());
  return PBH_OK;
}

int mlp_grad(const float* X, const float* Y, uint32_t n, const float* blob, float* grad, float* loss) {
  if (!X || !Y || !blob || !grad || !loss || n == 0 || n > (1u << 16)) return PBH_EINVAL;
  std::lock_guard<std::mutex> lock(g_learn_mu);
  float* scr = nullptr;
  LCHK(hipMalloc(&scr, (size_t)4 * n * H * sizeof(float)));
  hipLaunchKernelGGL(k_mlp_grad, dim3(1), dim3(256), 0, 0, blob, X, Y, 0u, n, grad, loss, scr);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  (void)hipFree(scr);
  LCHK(e);
  return PBH_OK;
}

int mlp_train(const float* X, const float* Y, uint32_t n, float* blob, uint32_t batch, uint32_t steps, float lr,
              float* loss_trace) {
  if (!X || !Y || !blob || n == 0 || batch == 0 || batch > 4096) return PBH_EINVAL;
  std::lock_guard<std::mutex> lock(g_learn_mu);
  if (batch > n) batch = n;
  float *scr = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr, *loss = nullptr;
  hipError_t e = hipMalloc(&scr, (size_t)4 * batch * H * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&grad, MLP_PARAMS * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m, MLP_PARAMS * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&v, MLP_PARAMS * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&loss, (size_t)(steps ? steps : 1) * sizeof(float));
  if (e == hipSuccess) e = hipMemset(m, 0, MLP_PARAMS * sizeof(float));
  if (e == hipSuccess) e = hipMemset(v, 0, MLP_PARAMS * sizeof(float));
  const u32 nb = n / batch;
  for (u32 t = 0; e == hipSuccess && t < steps; ++t) {
    u32 idx0 = (t % nb) * batch;
    hipLaunchKernelGGL(k_mlp_grad, dim3(1), dim3(256), 0, 0, blob, X, Y, idx0, batch, grad, loss + t, scr);
    hipLaunchKernelGGL(k_adam, dim3((MLP_PARAMS + 255) / 256), dim3(256), 0, 0, blob, grad, m, v, lr, 0.9f, 0.999f,
                       1e-8f, (int)t + 1);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_round_bf16, dim3((MLP_PARAMS + 255) / 256), dim3(256), 0, 0, blob);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess && loss_trace && steps)
    e = hipMemcpy(loss_trace, loss, steps * sizeof(float), hipMemcpyDeviceToHost);
  for (float* p : {scr, grad, m, v, loss})
    if (p) (void)hipFree(p);
  LCHK(e);
  return PBH_OK;
}

}  // extern "C"
