// Batched persistent kernel: thousands of small independent circuits in one
// launch.  Each workgroup (512 threads) takes packs from an atomic queue; a
// pack is P circuits with the same qubit count and gate structure, run in
// lockstep by 512/P threads each.  States of up to 2^14 amplitudes per slice
// live in LDS from |0...0> to the final write-back.  Larger states run as
// passes: a pass names the 14 qubits a 2^14-amplitude LDS slice holds and the
// gates that act only on them; every slice of the state is gathered into LDS,
// gets all of the pass's gates, and is written back (one read and one write
// of the state per pass instead of one per gate).
#include <algorithm>
#include <atomic>
#include <climits>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "sv_batch.h"
#include "sv_batch_host.h"
#include "sv_internal.h"

namespace sv {
namespace {

using namespace batch;


// x with a zero bit inserted at position p (LDS indices: states and slices of
// at most 2^14 amplitudes)
__device__ __forceinline__ int ins0(int x, int p) { return ((x >> p) << (p + 1)) | (x & ((1 << p) - 1)); }

__device__ __forceinline__ float2 cmad(float ar, float ai, float2 x, float2 acc) {
  acc.x = fmaf(ar, x.x, acc.x);
  acc.x = fmaf(-ai, x.y, acc.x);
  acc.y = fmaf(ar, x.y, acc.y);
  acc.y = fmaf(ai, x.x, acc.y);
  return acc;
}


// LDS bank spreading.  When a gate's lowest qubit is low, the groups of
// neighbouring lanes start 2^q amplitudes apart and a wave's accesses pile
// onto a few banks (up to 32 lanes per 8-byte slot for qubits 0..3).  Each
// lane therefore walks its group in an XOR-rotated order: element t of the
// lane's registers holds amplitude t ^ r, with r taken from the group index
// bits just above the lowest qubit, which puts neighbouring lanes on
// different slots.  The rotation is exact: where r has bit j set, the pair
// of qubit j arrives swapped, and the lane applies the 2x2 factor with rows
// and columns swapped.  A CNOT's swap is symmetric and only its access order
// changes.
__device__ __forceinline__ int rot_shift(int lowest_qubit) { return lowest_qubit < 6 ? lowest_qubit : 6; }

// One CNOT on a state of `dim` amplitudes at st (LDS or global), threads lt of Tc.
__device__ __forceinline__ void apply_cnot(const BGate &G, float2 *st, int dim, int lt, int Tc) {
  const int cq = G.q0, tq = G.q1;
  const int lo = cq < tq ? cq : tq, hi = cq < tq ? tq : cq;
  const int s = rot_shift(lo);
  for (int p = lt; p < dim / 4; p += Tc) {
    const int x = ins0(ins0(p, lo), hi) | (1 << cq);
    const int x0 = x | (((p >> s) & 1) << tq), x1 = x0 ^ (1 << tq);
    const float2 a = st[x0], b = st[x1];
    st[x0] = b;
    st[x1] = a;
  }
}

// A group record (kind SV_BATCH_GATE_GROUP, q0 = c in 2..5) is followed by c
// single-qubit records on distinct qubits.  They commute, so one sweep
// applies all of them: each thread holds the 2^c amplitudes of a group in
// registers and applies every 2x2 factor there (one LDS read and write per
// amplitude instead of c).
// The 2x2 factors of a group on the 2^C amplitudes a lane holds (element t
// holds amplitude t ^ r of its group).
template <int C>
__device__ __forceinline__ void group_factors(const BGate *M, int r, float2 *a) {
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const float *m = M[j].m;
    const bool sw = (r >> j) & 1;  // this lane holds qubit j's pairs swapped
    const float m0 = sw ? m[6] : m[0], m1 = sw ? m[7] : m[1], m2 = sw ? m[4] : m[2], m3 = sw ? m[5] : m[3];
    const float m4 = sw ? m[2] : m[4], m5 = sw ? m[3] : m[5], m6 = sw ? m[0] : m[6], m7 = sw ? m[1] : m[7];
#pragma unroll
    for (int t = 0; t < (1 << C); ++t) {
      if ((t >> j) & 1) continue;
      const float2 x = a[t], y = a[t | (1 << j)];
      float2 o0 = make_float2(0.f, 0.f), o1 = make_float2(0.f, 0.f);
      o0 = cmad(m0, m1, x, o0);
      o0 = cmad(m2, m3, y, o0);
      o1 = cmad(m4, m5, x, o1);
      o1 = cmad(m6, m7, y, o1);
      a[t] = o0;
      a[t | (1 << j)] = o1;
    }
  }
}

// Qubits of a group's members, ascending, and their bits.
template <int C>
__device__ __forceinline__ void group_qubits(const BGate *M, int *qs, int *srt, int *qbit) {
#pragma unroll
  for (int j = 0; j < C; ++j) {
    qs[j] = srt[j] = M[j].q0;
    qbit[j] = 1 << qs[j];
  }
#pragma unroll
  for (int i = 1; i < C; ++i)
#pragma unroll
    for (int j = C - 1; j >= i; --j)
      if (srt[j - 1] > srt[j]) {
        const int t = srt[j];
        srt[j] = srt[j - 1];
        srt[j - 1] = t;
      }
}

template <int C>
__device__ __forceinline__ void apply_group_c(const BGate *M, float2 *st, int dim, int lt, int Tc) {
  int qs[C], srt[C], qbit[C];
  group_qubits<C>(M, qs, srt, qbit);
  const int s = rot_shift(srt[0]);
  for (int p = lt; p < (dim >> C); p += Tc) {
    int base = p;
#pragma unroll
    for (int j = 0; j < C; ++j) base = ins0(base, srt[j]);
    const int r = int(p >> s) & ((1 << C) - 1);  // element t holds amplitude t ^ r
    int orot = 0;
#pragma unroll
    for (int j = 0; j < C; ++j)
      if ((r >> j) & 1) orot |= qbit[j];
    float2 a[1 << C];
#pragma unroll
    for (int t = 0; t < (1 << C); ++t) {
      int o = 0;
#pragma unroll
      for (int j = 0; j < C; ++j)
        if ((t >> j) & 1) o |= qbit[j];
      a[t] = st[base + (o ^ orot)];
    }
    group_factors<C>(M, r, a);
#pragma unroll
    for (int t = 0; t < (1 << C); ++t) {
      int o = 0;
#pragma unroll
      for (int j = 0; j < C; ++j)
        if ((t >> j) & 1) o |= qbit[j];
      st[base + (o ^ orot)] = a[t];
    }
  }
}

// A linear record (kind SV_BATCH_GATE_LINEAR, only inside passes, where one
// workgroup runs one circuit) replaces a run of CNOTs on slice bits: the run
// maps the amplitude at y to the one at f(y), f linear over GF(2), so the new
// slice is new[y] = old[f(y)] with f(y) the XOR of mask[b] over the set bits
// b of y.  The 14 masks ride in the float slots of the record and of the one
// after it.  Every thread gathers its 32 amplitudes, the workgroup meets a
// barrier, then every thread writes them back: one LDS sweep for the run.
__device__ __forceinline__ void apply_linear(const BGate *R, float2 *lds, int tid) {
  constexpr int PER = kLdsAmps / kBT;  // 32 amplitudes per thread: y = tid + kBT * i
  int32_t mk[kSliceBits];
#pragma unroll
  for (int b = 0; b < 8; ++b) mk[b] = __float_as_int(R[0].m[b]);
#pragma unroll
  for (int b = 8; b < kSliceBits; ++b) mk[b] = __float_as_int(R[1].m[b - 8]);
  int32_t ft = 0;  // f(tid): tid covers the low 9 bits of y
#pragma unroll
  for (int b = 0; b < 9; ++b)
    if ((tid >> b) & 1) ft ^= mk[b];
  float2 v[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    int32_t fi = ft;  // i covers the high 5 bits
#pragma unroll
    for (int b = 0; b < 5; ++b)
      if ((i >> b) & 1) fi ^= mk[9 + b];
    v[i] = lds[fi];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) lds[tid + kBT * i] = v[i];
}
static_assert(kLdsAmps == kBT << 5 && kSliceBits == 14, "linear records assume 2^14 slices over 512 threads");

// A linear record followed by a five-gate group (the CNOT ladder of one
// layer, then the next layer's rotations), inside a pass: the group's lane
// gathers its 32 amplitudes of the mapped slice, old[f(y)], straight from
// the slice as it was before the linear map, the workgroup meets a barrier,
// and the lane applies the five factors and writes new[y] in place.  One
// LDS sweep and one barrier fewer than the two units.  f is linear, and a
// group position y = base ^ o (o a combination of the group's qubit bits)
// maps to f(base) ^ f(o), so f(o) is the XOR of the masks of o's bits.
// Passes hold kLdsAmps = 2^14 amplitudes over kBT = 512 threads: 2^14 / 2^5
// groups, one per thread, so every thread meets the barrier once.
__device__ __forceinline__ void apply_linear_group5(const BGate *RL, const BGate *M, float2 *lds, int tid) {
  constexpr int C = 5;
  static_assert((kLdsAmps >> C) == kBT, "one five-qubit group per thread of a pass");
  int32_t mk[kSliceBits];
#pragma unroll
  for (int b = 0; b < 8; ++b) mk[b] = __float_as_int(RL[0].m[b]);
#pragma unroll
  for (int b = 8; b < kSliceBits; ++b) mk[b] = __float_as_int(RL[1].m[b - 8]);
  auto fmap = [&](int y) {
    int32_t v = 0;
#pragma unroll
    for (int b = 0; b < kSliceBits; ++b)
      if ((y >> b) & 1) v ^= mk[b];
    return v;
  };
  int qs[C], srt[C], qbit[C];
  group_qubits<C>(M, qs, srt, qbit);
  const int s = rot_shift(srt[0]);
  const int p = tid;
  int base = p;
#pragma unroll
  for (int j = 0; j < C; ++j) base = ins0(base, srt[j]);
  const int r = (p >> s) & ((1 << C) - 1);  // element t holds amplitude t ^ r
  int orot = 0, forot = 0;
  int32_t fq[C];
#pragma unroll
  for (int j = 0; j < C; ++j) {
    fq[j] = mk[qs[j]];  // f of qubit j's bit
    if ((r >> j) & 1) {
      orot |= qbit[j];
      forot ^= fq[j];
    }
  }
  const int32_t fb = fmap(base) ^ forot;
  float2 a[1 << C];
#pragma unroll
  for (int t = 0; t < (1 << C); ++t) {
    int32_t fo = fb;
#pragma unroll
    for (int j = 0; j < C; ++j)
      if ((t >> j) & 1) fo ^= fq[j];
    a[t] = lds[fo];
  }
  __syncthreads();  // every lane has gathered before any position is overwritten
  group_factors<C>(M, r, a);
#pragma unroll
  for (int t = 0; t < (1 << C); ++t) {
    int o = 0;
#pragma unroll
    for (int j = 0; j < C; ++j)
      if ((t >> j) & 1) o |= qbit[j];
    lds[base + (o ^ orot)] = a[t];
  }
}

// One unit at record r (a gate, a group header and its members, or a linear
// record and its mask record) on an LDS state or slice of dim <= 2^14
// amplitudes; returns the number of records it spans.  MAXC: the widest
// group the caller's records hold (the host groups at most kMaxGroupLds
// gates for states in LDS and kMaxGroupPass inside passes).
template <int MAXC>
__device__ __forceinline__ int apply_unit(const BGate *R, float2 *st, int dim, int lt, int Tc) {
  if (R[0].kind == SV_BATCH_GATE_LINEAR) {
    apply_linear(R, st, lt);  // only in passes: dim = kLdsAmps, Tc = kBT
    return 2;
  }
  if (R[0].kind == SV_BATCH_GATE_GROUP) {
    const int c = R[0].q0;
    if (c == 2) apply_group_c<2>(R + 1, st, dim, lt, Tc);
    else if (c == 3) apply_group_c<3>(R + 1, st, dim, lt, Tc);
    else if (MAXC == 4 || c == 4) apply_group_c<4>(R + 1, st, dim, lt, Tc);
    else apply_group_c<(MAXC > 4 ? 5 : 4)>(R + 1, st, dim, lt, Tc);
    return 1 + c;
  }
  if (R[0].kind == SV_BATCH_GATE_1Q)
    apply_group_c<1>(R, st, dim, lt, Tc);
  else if (R[0].kind == SV_BATCH_GATE_CNOT)
    apply_cnot(R[0], st, dim, lt, Tc);
  return 1;
}
static_assert(kMaxGroupLds == 4 && kMaxGroupPass == 5, "the kernel instantiates groups of 2..5");

__global__ void k_batch_reset(unsigned *counter) {
  if (threadIdx.x == 0) *counter = 0u;
}

__global__ __launch_bounds__(kBT) void k_batch(const BItem *__restrict__ items, int nitems,
                                               const BGate *__restrict__ gates, float2 *__restrict__ states,
                                               double *__restrict__ z0, unsigned *__restrict__ counter) {
  __shared__ float2 lds[kLdsAmps];
  __shared__ double red[kBT];
  __shared__ int32_t offlo[128], offhi[128];  // slice index -> state offset, low and high 7 bits
  __shared__ int item_s;
  const int tid = threadIdx.x;
  while (true) {
    if (tid == 0) item_s = int(atomicAdd(counter, 1u));
    __syncthreads();
    const int it = item_s;
    __syncthreads();  // every thread has read item_s before it is overwritten
    if (it >= nitems) break;  // uniform: all waves leave together
    const BItem &I = items[it];
    const int n = I.n, P = I.P, ngates = I.ngates;
    const int Tc = kBT / P;
    const int c = tid / Tc, lt = tid % Tc;
    const int64_t dim = int64_t(1) << n;
    const bool in_lds = int64_t(P) * dim <= kLdsAmps;
    // the LDS state is addressed through the shared array itself, so that its
    // accesses compile to LDS instructions (a pointer that may also point to
    // global memory makes every access a flat one)
    float2 *const sl = lds + (in_lds ? int64_t(c) * dim : 0);
    float2 *const sg = states + I.state_off[c];
    const BGate *gl = gates + I.gate_off[c];
    const int my_ng = I.ngc[c];

    if (in_lds) {
      for (int64_t x = lt; x < dim; x += Tc) sl[x] = make_float2(x == 0 ? 1.f : 0.f, 0.f);
    } else {
      for (int64_t x = lt; x < dim; x += Tc) sg[x] = make_float2(x == 0 ? 1.f : 0.f, 0.f);
    }
    __syncthreads();
    if (in_lds) {
      // lockstep over the pack, one unit (gate or group) per step: a circuit
      // past its last unit only meets the barriers
      int r = 0;  // this circuit's next record
      for (int g = 0; g < ngates; ++g) {
        if (g < my_ng) r += apply_unit<kMaxGroupLds>(gl + r, sl, int(dim), lt, Tc);
        __syncthreads();
      }
    } else {
      float2 *const st = sg;
      // P = 1: every thread runs the same circuit, so its records are read
      // through a wave-uniform pointer (scalar loads, matrices in SGPRs)
      const uint64_t gp = reinterpret_cast<uint64_t>(gl);
      const BGate *const glu = reinterpret_cast<const BGate *>(
          (uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(int(gp >> 32)))) << 32) |
          uint32_t(__builtin_amdgcn_readfirstlane(int(gp & 0xffffffffu))));
      // P = 1: the whole workgroup runs the passes of one circuit
      for (int g = 0; g < my_ng;) {
        const BGate M = glu[g];  // pass record
        const uint32_t mask = uint32_t(M.q0);
        const int cnt = M.q1;
        if (tid < 256) {
          // slice bit j (j = 0..13) is the j-th lowest qubit of the mask
          const int half = tid >> 7, v = tid & 127;
          int32_t off = 0;
          int j = 0;
          for (int q = 0; q < n; ++q) {
            if (!((mask >> q) & 1u)) continue;
            const int jj = j - 7 * half;
            if (jj >= 0 && jj < 7 && ((v >> jj) & 1)) off |= int32_t(1) << q;
            ++j;
          }
          (half ? offhi : offlo)[v] = off;
        }
        __syncthreads();
        const int nsl = 1 << (n - kSliceBits);
        auto slice_base = [&](int si) {
          int64_t b = 0;
          int r = 0;
          for (int q = 0; q < n; ++q) {
            if ((mask >> q) & 1u) continue;
            if ((si >> r) & 1) b |= int64_t(1) << q;
            ++r;
          }
          return b;
        };
        int64_t base = slice_base(0);
        for (int x = tid; x < kLdsAmps; x += kBT) lds[x] = st[base + offlo[x & 127] + offhi[x >> 7]];
        __syncthreads();
        for (int si = 0; si < nsl; ++si) {
          for (int j = 1; j <= cnt;) {
            const BGate *R = glu + g + j;
            if (R[0].kind == SV_BATCH_GATE_LINEAR && j + 2 <= cnt && R[2].kind == SV_BATCH_GATE_GROUP &&
                R[2].q0 == 5) {
              apply_linear_group5(R, R + 3, lds, tid);  // its members follow the header inside the pass
              j += 2 + 1 + 5;
            } else {
              j += apply_unit<kMaxGroupPass>(R, lds, kLdsAmps, tid, kBT);
            }
            __syncthreads();
          }
          // write this slice back and gather the next one in the same sweep:
          // each thread moves only its own LDS entries, so no barrier is
          // needed between the two, and the stores overlap the loads
          if (si + 1 < nsl) {
            constexpr int PER = kLdsAmps / kBT;
            const int64_t nbase = slice_base(si + 1);
            float2 w[PER];  // the next slice's entries of this thread, all loads in flight
#pragma unroll
            for (int i = 0; i < PER; ++i) {
              const int x = tid + i * kBT;
              w[i] = st[nbase + offlo[x & 127] + offhi[x >> 7]];
            }
#pragma unroll
            for (int i = 0; i < PER; ++i) {
              const int x = tid + i * kBT;
              st[base + offlo[x & 127] + offhi[x >> 7]] = lds[x];
              lds[x] = w[i];
            }
            base = nbase;
          } else {
            for (int x = tid; x < kLdsAmps; x += kBT) st[base + offlo[x & 127] + offhi[x >> 7]] = lds[x];
          }
          __syncthreads();
        }
        g += 1 + cnt;
      }
    }
    // <Z_0> in FP64 over this circuit's state
    double s = 0.0;
    for (int64_t x = lt; x < dim; x += Tc) {
      const float2 a = in_lds ? sl[x] : sg[x];
      const double pr = double(a.x) * double(a.x) + double(a.y) * double(a.y);
      s += (x & 1) ? -pr : pr;
    }
    red[tid] = s;
    __syncthreads();
    for (int w = Tc / 2; w > 0; w >>= 1) {
      if (lt < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (lt == 0) z0[I.circ[c]] = red[tid];
    if (in_lds)
      for (int64_t x = lt; x < dim; x += Tc) sg[x] = sl[x];
    __syncthreads();
  }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Device side of a packed batch: where its records sit in the workspace.
struct DevBatch {
  unsigned *counter = nullptr;
  double *z0 = nullptr;
  BItem *items = nullptr;
  BGate *gates = nullptr;
  int nitems = 0, ncirc = 0;
};

// Copy a packed batch's records into the workspace (asynchronous on st).
int upload_packed(const Packed &pk, void *ws_dev, size_t ws_bytes, hipStream_t st, DevBatch *d) {
  const size_t o_cnt = 0;
  const size_t o_z0 = 256;
  const size_t o_items = o_z0 + align256(sizeof(double) * size_t(std::max(1, pk.ncirc)));
  const size_t o_gates = o_items + align256(sizeof(BItem) * std::max<size_t>(1, pk.items.size()));
  const size_t need = o_gates + align256(sizeof(BGate) * std::max<size_t>(1, pk.gates.size()));
  if (!ws_dev || ws_bytes < need) {
    set_error("batch workspace too small");
    return SV_ERR_ARG;
  }
  char *ws = static_cast<char *>(ws_dev);
  d->counter = reinterpret_cast<unsigned *>(ws + o_cnt);
  d->z0 = reinterpret_cast<double *>(ws + o_z0);
  d->items = reinterpret_cast<BItem *>(ws + o_items);
  d->gates = reinterpret_cast<BGate *>(ws + o_gates);
  d->nitems = int(pk.items.size());
  d->ncirc = pk.ncirc;
  if (!pk.items.empty())
    SV_HIP_CHECK(hipMemcpyAsync(d->items, pk.items.data(), sizeof(BItem) * pk.items.size(), hipMemcpyHostToDevice, st));
  if (!pk.gates.empty())
    SV_HIP_CHECK(hipMemcpyAsync(d->gates, pk.gates.data(), sizeof(BGate) * pk.gates.size(), hipMemcpyHostToDevice, st));
  return SV_OK;
}

// One persistent launch over an uploaded batch; z0_host (optional) receives
// <Z_0> per circuit and makes the call synchronous; ms_out (optional) times the kernel.
int launch_packed(const DevBatch &d, void *states_dev, double *z0_host, hipStream_t st, float *ms_out) {
  int dev = 0, cus = 256;
  SV_HIP_CHECK(hipGetDevice(&dev));
  SV_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms_out) {
    SV_HIP_CHECK(hipEventCreate(&e0));
    SV_HIP_CHECK(hipEventCreate(&e1));
  }
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, d.counter);
  SV_HIP_CHECK(hipGetLastError());
  if (ms_out) SV_HIP_CHECK(hipEventRecord(e0, st));
  const int grid = std::max(1, std::min<int>(cus, d.nitems));
  hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kBT), 0, st, d.items, d.nitems, d.gates,
                     static_cast<float2 *>(states_dev), d.z0, d.counter);
  SV_HIP_CHECK(hipGetLastError());
  if (ms_out) SV_HIP_CHECK(hipEventRecord(e1, st));
  if (z0_host && d.ncirc > 0)
    SV_HIP_CHECK(hipMemcpyAsync(z0_host, d.z0, sizeof(double) * size_t(d.ncirc), hipMemcpyDeviceToHost, st));
  if (z0_host || ms_out) SV_HIP_CHECK(hipStreamSynchronize(st));
  if (ms_out) {
    SV_HIP_CHECK(hipEventElapsedTime(ms_out, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  return SV_OK;
}

int run_packed(const Packed &pk, void *states_dev, double *z0_host, void *ws_dev, size_t ws_bytes, hipStream_t st,
               float *ms_out) {
  DevBatch d;
  const int rc = upload_packed(pk, ws_dev, ws_bytes, st, &d);
  if (rc) return rc;
  return launch_packed(d, states_dev, z0_host, st, ms_out);
}

}  // namespace
}  // namespace sv

using namespace sv;
using namespace sv::batch;

extern "C" {


int sv_batch_run(int count, const sv_batch_circuit *circs, void *states_dev, size_t states_bytes,
                 const int64_t *state_offsets, double *z0_host, const int32_t *config, void *ws_dev, size_t ws_bytes,
                 void *stream) {
  return guard([&]() -> int {
    if (count < 0 || (count > 0 && (!circs || !states_dev || !state_offsets || !z0_host)) || !ws_dev) {
      set_error("bad batch argument");
      return SV_ERR_ARG;
    }
    int32_t cfg[SV_BATCH_CONFIG_LEN];
    if (config) {
      std::memcpy(cfg, config, sizeof(cfg));
      if (!valid_config(cfg)) {
        set_error("bad batch config");
        return SV_ERR_ARG;
      }
    } else {
      default_config(cfg);
    }
    Packed pk;
    int rc = pack_batch(count, circs, states_bytes, state_offsets, cfg, &pk);
    if (rc) return rc;
    return run_packed(pk, states_dev, z0_host, ws_dev, ws_bytes, static_cast<hipStream_t>(stream), nullptr);
  });
}

int sv_batch_autotune(int count, const sv_batch_circuit *circs, void *states_dev, size_t states_bytes,
                      const int64_t *state_offsets, int sample_per_size, int32_t *config_out, double *times_out,
                      void *ws_dev, size_t ws_bytes, void *stream) {
  return guard([&]() -> int {
    if (count < 0 || (count > 0 && (!circs || !states_dev || !state_offsets)) || !config_out || !ws_dev ||
        sample_per_size < 1) {
      set_error("bad autotune argument");
      return SV_ERR_ARG;
    }
    // tuning subset: up to sample_per_size circuits of every size, run together
    // so that the measured time is the throughput of a full launch
    std::vector<sv_batch_circuit> sample;
    std::vector<int64_t> offs;
    int per_size[SV_BATCH_CONFIG_LEN] = {0};
    for (int i = 0; i < count; ++i) {
      const int n = circs[i].n_qubits;
      if (n < 1 || n > SV_BATCH_MAX_QUBITS || per_size[n] >= sample_per_size) continue;
      ++per_size[n];
      sample.push_back(circs[i]);
      offs.push_back(state_offsets[i]);
    }
    int32_t cfg[SV_BATCH_CONFIG_LEN];
    default_config(cfg);
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<double> z(std::max<size_t>(1, sample.size()));
    auto measure = [&](const int32_t *c, double *t_out) -> int {
      Packed pk;
      int rc = pack_batch(int(sample.size()), sample.data(), states_bytes, offs.data(), c, &pk);
      if (rc) return rc;
      float ms = 0.f;
      rc = run_packed(pk, states_dev, z.data(), ws_dev, ws_bytes, st, &ms);  // warm-up
      if (rc) return rc;
      rc = run_packed(pk, states_dev, z.data(), ws_dev, ws_bytes, st, &ms);
      if (rc) return rc;
      *t_out = double(ms) * 1e-3;
      return SV_OK;
    };
    double best_t = 0;
    int rc = measure(cfg, &best_t);
    if (rc) return rc;
    if (times_out)
      for (int n = 0; n < SV_BATCH_CONFIG_LEN; ++n) times_out[n] = 0.0;
    // coordinate descent over the pack size of every size present
    for (int n = 1; n <= SV_BATCH_MAX_QUBITS; ++n) {
      if (per_size[n] == 0) continue;
      for (int P = 1; P <= kMaxPack; P *= 2) {
        if (P == cfg[n] || (P > 1 && (int64_t(P) << n) > kLdsAmps)) continue;
        int32_t trial[SV_BATCH_CONFIG_LEN];
        std::memcpy(trial, cfg, sizeof(trial));
        trial[n] = P;
        double t = 0;
        rc = measure(trial, &t);
        if (rc) return rc;
        if (t < best_t) {
          best_t = t;
          cfg[n] = P;
        }
      }
      if (times_out) times_out[n] = best_t;
    }
    std::memcpy(config_out, cfg, sizeof(cfg));
    return SV_OK;
  });
}

}  // extern "C"

struct sv_batch_prepared {
  DevBatch d;
};

extern "C" int sv_batch_prepare(int count, const sv_batch_circuit *circs, size_t states_bytes,
                                const int64_t *state_offsets, const int32_t *config, void *ws_dev, size_t ws_bytes,
                                void *stream, sv_batch_prepared **out) {
  return guard([&]() -> int {
    if (!out || count < 0 || (count > 0 && (!circs || !state_offsets)) || !ws_dev) {
      set_error("bad batch argument");
      return SV_ERR_ARG;
    }
    int32_t cfg[SV_BATCH_CONFIG_LEN];
    if (config) {
      std::memcpy(cfg, config, sizeof(cfg));
      if (!valid_config(cfg)) {
        set_error("bad batch config");
        return SV_ERR_ARG;
      }
    } else {
      default_config(cfg);
    }
    Packed pk;
    int rc = pack_batch(count, circs, states_bytes, state_offsets, cfg, &pk);
    if (rc) return rc;
    sv_batch_prepared *p = new sv_batch_prepared();
    hipStream_t st = static_cast<hipStream_t>(stream);
    rc = upload_packed(pk, ws_dev, ws_bytes, st, &p->d);
    if (rc == SV_OK && hipStreamSynchronize(st) != hipSuccess) {
      set_error("batch upload failed");
      rc = SV_ERR_DEVICE;
    }
    if (rc) {
      delete p;
      return rc;
    }
    *out = p;
    return SV_OK;
  });
}

extern "C" int sv_batch_launch(sv_batch_prepared *p, void *states_dev, double *z0_host, void *stream) {
  return guard([&]() -> int {
    if (!p || !states_dev) {
      set_error("bad batch argument");
      return SV_ERR_ARG;
    }
    return launch_packed(p->d, states_dev, z0_host, static_cast<hipStream_t>(stream), nullptr);
  });
}

extern "C" int sv_batch_prepared_free(sv_batch_prepared *p) {
  return guard([&]() -> int {
    delete p;
    return SV_OK;
  });
}
