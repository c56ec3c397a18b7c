// Cost-model MLP: forward, backward and Adam kernels (FP32); the host
// forward for the planner is in sv_mlp_host.cpp.  Sizes are tiny (5k
// parameters, batches of a few thousand rows): one thread per output
// element, reductions over the batch in a fixed order so every run gives
// the same bits.
#include <cmath>
#include <vector>

#include "sv_internal.h"
#include "sv_mlp.h"
#include "sv_mlp_layout.h"

namespace sv {
namespace {

constexpr int kT = 256;

using Off = MlpOffsets;
inline Off offsets(int nin, int hid) { return mlp_offsets(nin, hid); }

// z[r][u] = sum_i in[r][i] W[i][u] + b[u]; relu_in: apply relu to `in` on read
__global__ __launch_bounds__(kT) void k_dense(const float *__restrict__ in, int nin, bool relu_in,
                                              const float *__restrict__ W, const float *__restrict__ b, int hid,
                                              int batch, float *__restrict__ z) {
  const int64_t idx = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (idx >= int64_t(batch) * hid) return;
  const int r = int(idx / hid), u = int(idx % hid);
  float acc = b[u];
  for (int i = 0; i < nin; ++i) {
    float x = in[int64_t(r) * nin + i];
    if (relu_in) x = x > 0.f ? x : 0.f;
    acc = fmaf(x, W[i * hid + u], acc);
  }
  z[idx] = acc;
}

__global__ __launch_bounds__(kT) void k_out(const float *__restrict__ z2, int hid, const float *__restrict__ w3,
                                            const float *__restrict__ b3, int batch, float *__restrict__ y) {
  const int r = blockIdx.x * kT + threadIdx.x;
  if (r >= batch) return;
  float acc = b3[0];
  for (int u = 0; u < hid; ++u) {
    const float h = z2[int64_t(r) * hid + u];
    acc = fmaf(h > 0.f ? h : 0.f, w3[u], acc);
  }
  y[r] = acc;
}

// loss = 0.5 mean (y - t)^2, one workgroup, fixed tree
__global__ __launch_bounds__(kT) void k_loss(const float *__restrict__ y, const float *__restrict__ t, int batch,
                                             float *__restrict__ loss) {
  __shared__ float red[kT];
  float s = 0.f;
  for (int r = threadIdx.x; r < batch; r += kT) {
    const float d = y[r] - t[r];
    s = fmaf(d, d, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = 0.5f * red[0] / float(batch);
}

// dz2[r][u] = (y - t)/B * w3[u] * [z2 > 0]
__global__ __launch_bounds__(kT) void k_dz2(const float *__restrict__ y, const float *__restrict__ t,
                                            const float *__restrict__ z2, const float *__restrict__ w3, int hid,
                                            int batch, float *__restrict__ dz2) {
  const int64_t idx = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (idx >= int64_t(batch) * hid) return;
  const int r = int(idx / hid), u = int(idx % hid);
  const float dy = (y[r] - t[r]) / float(batch);
  dz2[idx] = z2[idx] > 0.f ? dy * w3[u] : 0.f;
}

// dz1[r][a] = sum_u dz2[r][u] W2[a][u] * [z1 > 0]
__global__ __launch_bounds__(kT) void k_dz1(const float *__restrict__ dz2, const float *__restrict__ W2,
                                            const float *__restrict__ z1, int hid, int batch,
                                            float *__restrict__ dz1) {
  const int64_t idx = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (idx >= int64_t(batch) * hid) return;
  const int r = int(idx / hid), a = int(idx % hid);
  float acc = 0.f;
  for (int u = 0; u < hid; ++u) acc = fmaf(dz2[int64_t(r) * hid + u], W2[a * hid + u], acc);
  dz1[idx] = z1[idx] > 0.f ? acc : 0.f;
}

// gW[i][u] = sum_r act(in[r][i]) d[r][u]; gb[u] = sum_r d[r][u]   (rows i = nin are the bias)
__global__ __launch_bounds__(kT) void k_wgrad(const float *__restrict__ in, int nin, bool relu_in,
                                              const float *__restrict__ d, int hid, int batch,
                                              float *__restrict__ gW, float *__restrict__ gb) {
  const int idx = blockIdx.x * kT + threadIdx.x;
  if (idx >= (nin + 1) * hid) return;
  const int i = idx / hid, u = idx % hid;
  float acc = 0.f;
  if (i < nin) {
    for (int r = 0; r < batch; ++r) {
      float x = in[int64_t(r) * nin + i];
      if (relu_in) x = x > 0.f ? x : 0.f;
      acc = fmaf(x, d[int64_t(r) * hid + u], acc);
    }
    gW[i * hid + u] = acc;
  } else {
    for (int r = 0; r < batch; ++r) acc += d[int64_t(r) * hid + u];
    gb[u] = acc;
  }
}

// output layer: gW3[u] = sum_r relu(z2[r][u]) dy[r]; gb3 = sum_r dy[r]
__global__ __launch_bounds__(kT) void k_out_grad(const float *__restrict__ z2, const float *__restrict__ y,
                                                 const float *__restrict__ t, int hid, int batch,
                                                 float *__restrict__ gw3, float *__restrict__ gb3) {
  const int u = blockIdx.x * kT + threadIdx.x;
  if (u > hid) return;
  float acc = 0.f;
  for (int r = 0; r < batch; ++r) {
    const float dy = (y[r] - t[r]) / float(batch);
    if (u < hid) {
      const float h = z2[int64_t(r) * hid + u];
      acc = fmaf(h > 0.f ? h : 0.f, dy, acc);
    } else {
      acc += dy;
    }
  }
  if (u < hid)
    gw3[u] = acc;
  else
    gb3[0] = acc;
}

__global__ __launch_bounds__(kT) void k_adam(float *__restrict__ p, const float *__restrict__ g,
                                             float *__restrict__ m, float *__restrict__ v, int count, float lr,
                                             float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mhat = mi / c1, vhat = vi / c2;
  p[i] -= lr * mhat / (sqrtf(vhat) + eps);
}

unsigned blocks(int64_t n) { return unsigned((n + kT - 1) / kT); }

}  // namespace
}  // namespace sv

using namespace sv;

extern "C" {

int sv_mlp_forward(const float *params, int nin, int hid, const float *X, int batch, float *y, float *cache,
                   void *stream) {
  return guard([&]() -> int {
    if (!params || !X || !y || nin < 1 || hid < 1 || batch < 1 || !cache) {
      set_error("bad mlp forward argument (cache is required)");
      return SV_ERR_ARG;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Off o = offsets(nin, hid);
    float *z1 = cache, *z2 = cache + int64_t(hid) * batch;
    hipLaunchKernelGGL(k_dense, dim3(blocks(int64_t(batch) * hid)), dim3(kT), 0, st, X, nin, false, params + o.w1,
                       params + o.b1, hid, batch, z1);
    hipLaunchKernelGGL(k_dense, dim3(blocks(int64_t(batch) * hid)), dim3(kT), 0, st, z1, hid, true, params + o.w2,
                       params + o.b2, hid, batch, z2);
    hipLaunchKernelGGL(k_out, dim3(blocks(batch)), dim3(kT), 0, st, z2, hid, params + o.w3, params + o.b3, batch, y);
    SV_HIP_CHECK(hipGetLastError());
    return SV_OK;
  });
}

int sv_mlp_backward(const float *params, int nin, int hid, const float *X, const float *target, int batch,
                    const float *y, const float *cache, float *grads, float *loss, void *stream) {
  return guard([&]() -> int {
    if (!params || !X || !target || !y || !cache || !grads || !loss || nin < 1 || hid < 1 || batch < 1) {
      set_error("bad mlp backward argument");
      return SV_ERR_ARG;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Off o = offsets(nin, hid);
    const float *z1 = cache, *z2 = cache + int64_t(hid) * batch;
    float *dz2 = const_cast<float *>(cache) + 2 * int64_t(hid) * batch;
    float *dz1 = const_cast<float *>(cache) + 3 * int64_t(hid) * batch;
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(kT), 0, st, y, target, batch, loss);
    hipLaunchKernelGGL(k_out_grad, dim3(blocks(hid + 1)), dim3(kT), 0, st, z2, y, target, hid, batch, grads + o.w3,
                       grads + o.b3);
    hipLaunchKernelGGL(k_dz2, dim3(blocks(int64_t(batch) * hid)), dim3(kT), 0, st, y, target, z2, params + o.w3, hid,
                       batch, dz2);
    hipLaunchKernelGGL(k_wgrad, dim3(blocks((hid + 1) * hid)), dim3(kT), 0, st, z1, hid, true, dz2, hid, batch,
                       grads + o.w2, grads + o.b2);
    hipLaunchKernelGGL(k_dz1, dim3(blocks(int64_t(batch) * hid)), dim3(kT), 0, st, dz2, params + o.w2, z1, hid, batch,
                       dz1);
    hipLaunchKernelGGL(k_wgrad, dim3(blocks((nin + 1) * hid)), dim3(kT), 0, st, X, nin, false, dz1, hid, batch,
                       grads + o.w1, grads + o.b1);
    SV_HIP_CHECK(hipGetLastError());
    return SV_OK;
  });
}

int sv_mlp_adam(float *params, const float *grads, float *m, float *v, int count, int t, float lr, float beta1,
                float beta2, float eps, void *stream) {
  return guard([&]() -> int {
    if (!params || !grads || !m || !v || count < 1 || t < 1) {
      set_error("bad adam argument");
      return SV_ERR_ARG;
    }
    const float c1 = 1.f - std::pow(beta1, float(t)), c2 = 1.f - std::pow(beta2, float(t));
    hipLaunchKernelGGL(k_adam, dim3(blocks(count)), dim3(kT), 0, static_cast<hipStream_t>(stream), params, grads, m,
                       v, count, lr, beta1, beta2, eps, c1, c2);
    SV_HIP_CHECK(hipGetLastError());
    return SV_OK;
  });
}

}  // extern "C"
