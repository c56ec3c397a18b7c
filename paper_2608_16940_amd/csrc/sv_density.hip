// Density matrices over the fused-operator interface (Section IV-B, the
// vectorised density matrix): a handle is a 2N-qubit state holding vec(rho)
// column-major, channels become 2k-target superoperators applied by
// sv_apply_fused, and the measurement distribution is the diagonal of rho.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "sv_density.h"
#include "sv_internal.h"

namespace sv {
namespace {

// Physical vector index of the diagonal entry rho_xx: logical row bit q and
// column bit q (vector qubits q and q + N) both equal bit q of x, so
// y(x) = sum over set bits q of x of m[q], m[q] = 2^L(q) | 2^L(q + N).
struct DmMasks {
  int64_t m[SV_DM_MAX_QUBITS];
};

__device__ __forceinline__ int64_t dm_diag_index(int64_t x, int n, const DmMasks &mk) {
  int64_t y = 0;
  for (int q = 0; q < n; ++q)
    if ((x >> q) & 1) y |= mk.m[q];
  return y;
}

__global__ __launch_bounds__(256) void k_dm_diag(const float2 *__restrict__ psi, int n, DmMasks mk,
                                                 double *__restrict__ out) {
  const int64_t x = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (x < (int64_t(1) << n)) {
    // a density matrix has a non-negative diagonal; FP32 rounding can leave -eps,
    // which the sampler's fixed-point conversion must not see (NaN passes through)
    const double v = double(psi[dm_diag_index(x, n, mk)].x);
    out[x] = v < 0.0 ? 0.0 : v;
  }
}

// One workgroup: 2^N <= 2^17 diagonal entries, fixed summation order.
constexpr int kTraceThreads = 1024;
__global__ __launch_bounds__(kTraceThreads) void k_dm_trace(const float2 *__restrict__ psi, int n, DmMasks mk,
                                                            double *__restrict__ result) {
  __shared__ double red[kTraceThreads];
  double s = 0.0;
  for (int64_t x = threadIdx.x; x < (int64_t(1) << n); x += kTraceThreads) s += double(psi[dm_diag_index(x, n, mk)].x);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kTraceThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *result = red[0];
}

bool valid_dm_n(int n) { return n >= SV_DM_MIN_QUBITS && n <= SV_DM_MAX_QUBITS; }

DmMasks diag_masks(const sv_state *s) {
  DmMasks mk;
  std::memset(&mk, 0, sizeof(mk));
  for (int q = 0; q < s->dm_n; ++q) mk.m[q] = (int64_t(1) << s->L[q]) | (int64_t(1) << s->L[q + s->dm_n]);
  return mk;
}

int require_dm(const sv_state *s) {
  if (!s) {
    set_error("null handle");
    return SV_ERR_ARG;
  }
  if (s->dm_n <= 0) {
    set_error("not a density-matrix handle");
    return SV_ERR_ARG;
  }
  return SV_OK;
}

hipError_t launch_dm_diag(const sv_state *s, double *out) {
  const int n = s->dm_n;
  const unsigned blocks = unsigned(((int64_t(1) << n) + 255) / 256);
  hipLaunchKernelGGL(k_dm_diag, dim3(blocks), dim3(256), 0, s->st, s->amps, n, diag_masks(s), out);
  return hipGetLastError();
}

}  // namespace
}  // namespace sv

using namespace sv;

extern "C" {

size_t sv_dm_state_bytes(int n_qubits) { return valid_dm_n(n_qubits) ? (size_t(8) << (2 * n_qubits)) : 0; }

size_t sv_dm_workspace_bytes(int n_qubits) { return valid_dm_n(n_qubits) ? sv_workspace_bytes(2 * n_qubits) : 0; }

int sv_dm_alloc(sv_state **out, int n_qubits, void *amps_dev, size_t amps_bytes, void *ws_dev, size_t ws_bytes,
                void *stream) {
  return guard([&]() -> int {
    if (!out) {
      set_error("null pointer");
      return SV_ERR_ARG;
    }
    *out = nullptr;
    if (!valid_dm_n(n_qubits)) {
      set_error("density-matrix qubit count out of range [2, 17]");
      return SV_ERR_ARG;
    }
    const int rc = sv_alloc(out, 2 * n_qubits, amps_dev, amps_bytes, ws_dev, ws_bytes, stream);
    if (rc != SV_OK) return rc;
    (*out)->dm_n = n_qubits;
    return SV_OK;
  });
}

int sv_dm_qubits(const sv_state *s) {
  return guard([&]() -> int {
    if (!s) {
      set_error("null handle");
      return SV_ERR_ARG;
    }
    return s->dm_n;
  });
}

int sv_dm_superop(const double *kraus, int n_kraus, int k, double *out) {
  return guard([&]() -> int {
    if (!kraus || !out || n_kraus < 1 || k < 1 || k > SV_DM_MAX_K) {
      set_error("superoperator: bad argument (1 <= k <= 4, n_kraus >= 1, non-null)");
      return SV_ERR_ARG;
    }
    const int d = 1 << k, dd = d * d;
    std::memset(out, 0, sizeof(double) * 2 * size_t(dd) * size_t(dd));
    for (int i = 0; i < n_kraus; ++i) {
      const double *e = kraus + size_t(i) * 2 * d * d;
      for (int rr = 0; rr < d; ++rr)      // row of E (row copy)
        for (int rc = 0; rc < d; ++rc)    // row of conj(E) (column copy)
          for (int cr = 0; cr < d; ++cr)
            for (int cc = 0; cc < d; ++cc) {
              const double ar = e[2 * (rr * d + cr)], ai = e[2 * (rr * d + cr) + 1];
              const double br = e[2 * (rc * d + cc)], bi = -e[2 * (rc * d + cc) + 1];
              const size_t r = size_t(rr + d * rc), c = size_t(cr + d * cc);
              out[2 * (r * dd + c)] += ar * br - ai * bi;
              out[2 * (r * dd + c) + 1] += ar * bi + ai * br;
            }
    }
    return SV_OK;
  });
}

int sv_dm_apply_channel(sv_state *s, const double *kraus, int n_kraus, const int32_t *targets, int k) {
  return guard([&]() -> int {
    int rc = require_dm(s);
    if (rc != SV_OK) return rc;
    if (!targets || k < 1 || k > SV_DM_MAX_K) {
      set_error("channel width out of range [1, 4]");
      return SV_ERR_ARG;
    }
    const int n = s->dm_n;
    int32_t t2[2 * SV_DM_MAX_K];
    for (int j = 0; j < k; ++j) {
      if (targets[j] < 0 || targets[j] >= n) {
        set_error("channel target out of range");
        return SV_ERR_ARG;
      }
      for (int i = 0; i < j; ++i)
        if (targets[i] == targets[j]) {
          set_error("duplicate channel target");
          return SV_ERR_ARG;
        }
      t2[j] = targets[j];
      t2[k + j] = targets[j] + n;
    }
    const size_t dd = size_t(1) << (2 * k);
    std::vector<double> S(2 * dd * dd);
    rc = sv_dm_superop(kraus, n_kraus, k, S.data());
    if (rc != SV_OK) return rc;
    return sv_apply_fused(s, S.data(), t2, 2 * k);
  });
}

int sv_dm_probs(sv_state *s, double *out_dev) {
  return guard([&]() -> int {
    const int rc = require_dm(s);
    if (rc != SV_OK) return rc;
    if (!out_dev) {
      set_error("null pointer");
      return SV_ERR_ARG;
    }
    SV_HIP_CHECK(launch_dm_diag(s, out_dev));
    return SV_OK;
  });
}

int sv_dm_trace(sv_state *s, double *out_host) {
  return guard([&]() -> int {
    const int rc = require_dm(s);
    if (rc != SV_OK) return rc;
    if (!out_host) {
      set_error("null pointer");
      return SV_ERR_ARG;
    }
    double *res = reinterpret_cast<double *>(s->ws.scalars);
    hipLaunchKernelGGL(k_dm_trace, dim3(1), dim3(kTraceThreads), 0, s->st, s->amps, s->dm_n, diag_masks(s), res);
    SV_HIP_CHECK(hipGetLastError());
    SV_HIP_CHECK(hipMemcpyAsync(out_host, res, sizeof(double), hipMemcpyDeviceToHost, s->st));
    SV_HIP_CHECK(hipStreamSynchronize(s->st));
    return SV_OK;
  });
}

int sv_dm_sample(sv_state *s, uint64_t seed, int64_t shots, uint64_t *out_host, double *probs_dev) {
  return guard([&]() -> int {
    const int rc = require_dm(s);
    if (rc != SV_OK) return rc;
    if (!probs_dev || (!out_host && shots > 0) || shots < 0) {
      set_error("bad argument");
      return SV_ERR_ARG;
    }
    if (shots == 0) return SV_OK;
    SV_HIP_CHECK(launch_dm_diag(s, probs_dev));
    // the 2N-qubit workspace holds the N-qubit sampler's (the layout grows with n)
    return sv_sample_probs(probs_dev, s->dm_n, seed, shots, out_host, s->ws_base, s->ws_bytes, s->st);
  });
}

}  // extern "C"
