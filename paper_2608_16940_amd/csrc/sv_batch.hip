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
#include "sv_internal.h"

namespace sv {
namespace {

constexpr int kBT = 512;             // threads per workgroup
constexpr int kLdsAmps = 1 << 14;    // 128 KiB of complex64 state slices
constexpr int kMaxPack = 16;

struct BGate {
  int32_t kind, q0, q1, pad;
  float m[8];  // 2x2 complex64 row-major interleaved
};

struct BItem {
  int32_t n, P, ngates, pad;  // ngates: longest circuit of the pack
  int32_t circ[kMaxPack];
  int32_t ngc[kMaxPack];      // gate count of each circuit
  int64_t gate_off[kMaxPack];
  int64_t state_off[kMaxPack];  // in amplitudes
};


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

constexpr int kSliceBits = 14;
constexpr int kGatePass = SV_BATCH_PASS;  // record: q0 = slice qubit mask, q1 = gates in the pass

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

// A group record (kind SV_BATCH_GATE_GROUP, q0 = c in 2..4) is followed by c
// single-qubit records on distinct qubits.  They commute, so one sweep
// applies all of them: each thread holds the 2^c amplitudes of a group in
// registers and applies every 2x2 factor there (one LDS read and write per
// amplitude instead of c).
template <int C>
__device__ __forceinline__ void apply_group_c(const BGate *M, float2 *st, int dim, int lt, int Tc) {
  int qs[C], srt[C];
  int qbit[C];
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

// One unit at record r (a gate, a group header and its members, or a linear
// record and its mask record) on an LDS state or slice of dim <= 2^14
// amplitudes; returns the number of records it spans.
__device__ __forceinline__ int apply_unit(const BGate *R, float2 *st, int dim, int lt, int Tc) {
  if (R[0].kind == SV_BATCH_GATE_LINEAR) {
    apply_linear(R, st, lt);  // only in passes: dim = kLdsAmps, Tc = kBT
    return 2;
  }
  if (R[0].kind == SV_BATCH_GATE_GROUP) {
    const int c = R[0].q0;
    if (c == 2) apply_group_c<2>(R + 1, st, dim, lt, Tc);
    else if (c == 3) apply_group_c<3>(R + 1, st, dim, lt, Tc);
    else apply_group_c<4>(R + 1, st, dim, lt, Tc);
    return 1 + c;
  }
  if (R[0].kind == SV_BATCH_GATE_1Q)
    apply_group_c<1>(R, st, dim, lt, Tc);
  else if (R[0].kind == SV_BATCH_GATE_CNOT)
    apply_cnot(R[0], st, dim, lt, Tc);
  return 1;
}

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
    float2 *st = in_lds ? lds + int64_t(c) * dim : states + I.state_off[c];
    const BGate *gl = gates + I.gate_off[c];
    const int my_ng = I.ngc[c];

    for (int64_t x = lt; x < dim; x += Tc) st[x] = make_float2(x == 0 ? 1.f : 0.f, 0.f);
    __syncthreads();
    if (in_lds) {
      // lockstep over the pack, one unit (gate or group) per step: a circuit
      // past its last unit only meets the barriers
      int r = 0;  // this circuit's next record
      for (int g = 0; g < ngates; ++g) {
        if (g < my_ng) r += apply_unit(gl + r, st, int(dim), lt, Tc);
        __syncthreads();
      }
    } else {
      // P = 1: the whole workgroup runs the passes of one circuit
      for (int g = 0; g < my_ng;) {
        const BGate M = gl[g];  // pass record
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
        for (int sl = 0; sl < nsl; ++sl) {
          int64_t base = 0;
          int r = 0;
          for (int q = 0; q < n; ++q) {
            if ((mask >> q) & 1u) continue;
            if ((sl >> r) & 1) base |= int64_t(1) << q;
            ++r;
          }
          for (int x = tid; x < kLdsAmps; x += kBT) lds[x] = st[base + offlo[x & 127] + offhi[x >> 7]];
          __syncthreads();
          for (int j = 1; j <= cnt;) {
            j += apply_unit(gl + g + j, lds, kLdsAmps, tid, kBT);
            __syncthreads();
          }
          for (int x = tid; x < kLdsAmps; x += kBT) st[base + offlo[x & 127] + offhi[x >> 7]] = lds[x];
          __syncthreads();
        }
        g += 1 + cnt;
      }
    }
    // <Z_0> in FP64 over this circuit's slice
    double s = 0.0;
    for (int64_t x = lt; x < dim; x += Tc) {
      const float2 a = st[x];
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
    if (in_lds) {
      float2 *out = states + I.state_off[c];
      for (int64_t x = lt; x < dim; x += Tc) out[x] = st[x];
    }
    __syncthreads();
  }
}

struct Packed {
  std::vector<BGate> gates;
  std::vector<BItem> items;
  int ncirc = 0;
};

// Rewrite the gate list of a circuit with more than 2^14 amplitudes as
// passes (a pass record, then its gates with qubits renumbered to slice bit
// positions).  A gate joins the current pass when it is ready (every earlier
// gate on its qubits applied) and all its qubits are in the pass's slice;
// ready gates of one moment act on disjoint qubits, so any order among them
// is exact.  When none is left, the next slice keeps qubits 0..2 (runs of 8
// contiguous amplitudes), the qubits of the earliest ready gate, then the
// qubits whose next gate comes soonest: the farthest next use stays out
// (Corollary 1), ties to the lower qubit.
std::vector<BGate> make_passes(const std::vector<BGate> &g, int n) {
  std::vector<std::vector<int>> per_q(static_cast<size_t>(n));
  for (int i = 0; i < int(g.size()); ++i) {
    per_q[size_t(g[size_t(i)].q0)].push_back(i);
    if (g[size_t(i)].kind == SV_BATCH_GATE_CNOT) per_q[size_t(g[size_t(i)].q1)].push_back(i);
  }
  std::vector<size_t> head(static_cast<size_t>(n), 0);
  auto head_gate = [&](int q) {
    return head[size_t(q)] < per_q[size_t(q)].size() ? per_q[size_t(q)][head[size_t(q)]] : INT_MAX;
  };
  auto qubits_of = [&](const BGate &b) {
    uint32_t m = 1u << b.q0;
    if (b.kind == SV_BATCH_GATE_CNOT) m |= 1u << b.q1;
    return m;
  };
  auto ready = [&](int i) {
    const BGate &b = g[size_t(i)];
    return head_gate(b.q0) == i && (b.kind != SV_BATCH_GATE_CNOT || head_gate(b.q1) == i);
  };
  uint32_t mask = (1u << kSliceBits) - 1;
  std::vector<BGate> out;
  size_t left = g.size();
  while (left > 0) {
    std::vector<BGate> pass;
    for (bool progress = true; progress;) {
      progress = false;
      for (int q = 0; q < n; ++q) {
        const int i = head_gate(q);
        if (i == INT_MAX || !ready(i)) continue;
        const BGate &b = g[size_t(i)];
        if (qubits_of(b) & ~mask) continue;
        BGate l = b;
        l.q0 = __builtin_popcount(mask & ((1u << b.q0) - 1));
        if (b.kind == SV_BATCH_GATE_CNOT) l.q1 = __builtin_popcount(mask & ((1u << b.q1) - 1));
        pass.push_back(l);
        ++head[size_t(b.q0)];
        if (b.kind == SV_BATCH_GATE_CNOT) ++head[size_t(b.q1)];
        --left;
        progress = true;
      }
    }
    if (!pass.empty()) {
      BGate rec;
      std::memset(&rec, 0, sizeof(rec));
      rec.kind = kGatePass;
      rec.q0 = int32_t(mask);
      rec.q1 = int32_t(pass.size());
      out.push_back(rec);
      out.insert(out.end(), pass.begin(), pass.end());
    }
    if (left == 0) break;
    int first = INT_MAX;
    for (int q = 0; q < n; ++q) {
      const int i = head_gate(q);
      if (i != INT_MAX && ready(i)) first = std::min(first, i);
    }
    uint32_t m = 0x7u | qubits_of(g[size_t(first)]);
    std::vector<int> rest;
    for (int q = 0; q < n; ++q)
      if (!((m >> q) & 1u)) rest.push_back(q);
    std::stable_sort(rest.begin(), rest.end(), [&](int a, int b) { return head_gate(a) < head_gate(b); });
    for (int q : rest) {
      if (__builtin_popcount(m) >= kSliceBits) break;
      m |= 1u << q;
    }
    mask = m;
  }
  return out;
}

// Runs of up to four consecutive single-qubit records on distinct qubits
// become one group (a header, then the members).  Within a pass list (after
// make_passes) only the gates inside each pass are grouped and the pass
// header's record count follows.
std::vector<BGate> group_run(const std::vector<BGate> &g, size_t a, size_t b) {
  std::vector<BGate> out;
  size_t i = a;
  while (i < b) {
    size_t j = i;
    uint32_t used = 0;
    while (j < b && j - i < 4 && g[j].kind == SV_BATCH_GATE_1Q && !((used >> g[j].q0) & 1u)) {
      used |= 1u << g[j].q0;
      ++j;
    }
    if (j - i >= 2) {
      BGate h;
      std::memset(&h, 0, sizeof(h));
      h.kind = SV_BATCH_GATE_GROUP;
      h.q0 = int32_t(j - i);
      out.push_back(h);
      out.insert(out.end(), g.begin() + long(i), g.begin() + long(j));
      i = j;
    } else {
      out.push_back(g[i]);
      ++i;
    }
  }
  return out;
}

// Runs of three or more consecutive CNOT records inside a pass (slice bit
// positions) become one linear record and its mask record.  A CNOT maps the
// amplitude at y to the one at g(y) = y ^ (bit c of y) << t; the run
// g_1 .. g_m (g_1 applied first) gives new[y] = old[g_1(g_2(... g_m(y)))],
// whose value on each basis vector e_b is mask[b].
std::vector<BGate> merge_cnots(const std::vector<BGate> &g, size_t a, size_t b) {
  std::vector<BGate> out;
  size_t i = a;
  while (i < b) {
    size_t j = i;
    while (j < b && g[j].kind == SV_BATCH_GATE_CNOT) ++j;
    if (j - i >= 3) {
      int32_t mk[kSliceBits];
      for (int bit = 0; bit < kSliceBits; ++bit) {
        int32_t y = int32_t(1) << bit;
        for (size_t r = j; r-- > i;) y ^= ((y >> g[r].q0) & 1) << g[r].q1;
        mk[bit] = y;
      }
      BGate h, d;
      std::memset(&h, 0, sizeof(h));
      std::memset(&d, 0, sizeof(d));
      h.kind = SV_BATCH_GATE_LINEAR;
      h.q0 = int32_t(j - i);  // CNOTs replaced (informational)
      d.kind = SV_BATCH_GATE_LINEAR;
      d.q0 = -1;  // the mask record
      for (int bit = 0; bit < 8; ++bit) std::memcpy(&h.m[bit], &mk[bit], 4);
      for (int bit = 8; bit < kSliceBits; ++bit) std::memcpy(&d.m[bit - 8], &mk[bit], 4);
      out.push_back(h);
      out.push_back(d);
      i = j;
    } else {
      for (; i < j; ++i) out.push_back(g[i]);
      if (i < b && g[i].kind != SV_BATCH_GATE_CNOT) out.push_back(g[i++]);
    }
  }
  return out;
}

std::vector<BGate> group_single_qubit(const std::vector<BGate> &g, bool passes) {
  if (!passes) return group_run(g, 0, g.size());
  std::vector<BGate> out;
  size_t i = 0;
  while (i < g.size()) {
    const size_t cnt = size_t(g[i].q1);
    std::vector<BGate> merged = merge_cnots(g, i + 1, i + 1 + cnt);
    std::vector<BGate> body = group_run(merged, 0, merged.size());
    BGate h = g[i];
    h.q1 = int32_t(body.size());
    out.push_back(h);
    out.insert(out.end(), body.begin(), body.end());
    i += 1 + cnt;
  }
  return out;
}

// Units (a gate, or a group with its members) in a record list without passes.
int count_units(const std::vector<BGate> &g) {
  int u = 0;
  for (size_t i = 0; i < g.size(); i += (g[i].kind == SV_BATCH_GATE_GROUP) ? 1 + size_t(g[i].q0) : 1) ++u;
  return u;
}

bool valid_config(const int32_t *cfg) {
  for (int n = 1; n <= SV_BATCH_MAX_QUBITS; ++n) {
    const int P = cfg[n];
    if (P < 1 || P > kMaxPack || (P & (P - 1))) return false;
    if (P > 1 && (int64_t(P) << n) > kLdsAmps) return false;
  }
  return true;
}

void default_config(int32_t *cfg) {
  cfg[0] = 1;
  for (int n = 1; n <= SV_BATCH_MAX_QUBITS; ++n) {
    int P = 1;
    while (P < kMaxPack && (int64_t(P * 2) << n) <= kLdsAmps) P *= 2;
    cfg[n] = (n <= 14) ? P : 1;
  }
}

// Per-circuit outcome of the host pass (worker threads report here; the
// calling thread turns the first failure into the error message).
enum CircStatus { CIRC_OK = 0, CIRC_BAD, CIRC_BAD_1Q, CIRC_BAD_CNOT, CIRC_BAD_KIND, CIRC_NOMEM };

// Validate circuit i, fuse adjacent single-qubit gates on the same qubit
// (FP64, later gate on the left), cut it into passes if its state exceeds a
// slice, group single-qubit runs.  Touches only circuit i's inputs and g.
int prepare_circuit(const sv_batch_circuit &C, int64_t state_offset, size_t states_bytes, std::vector<BGate> &g) {
  if (C.n_qubits < 1 || C.n_qubits > SV_BATCH_MAX_QUBITS || C.n_gates < 0 ||
      (C.n_gates > 0 && (!C.kinds || !C.qubits)) || state_offset < 0 || (state_offset & 7) ||
      uint64_t(state_offset) + (uint64_t(8) << C.n_qubits) > uint64_t(states_bytes))
    return CIRC_BAD;
  double cur[8];
  int cur_q = -1;
  auto flush = [&]() {
    if (cur_q < 0) return;
    BGate b;
    b.kind = SV_BATCH_GATE_1Q;
    b.q0 = cur_q;
    b.q1 = -1;
    b.pad = 0;
    for (int e = 0; e < 8; ++e) b.m[e] = float(cur[e]);
    g.push_back(b);
    cur_q = -1;
  };
  for (int j = 0; j < C.n_gates; ++j) {
    const int kind = C.kinds[j];
    const int q0 = C.qubits[2 * j], q1 = C.qubits[2 * j + 1];
    if (kind == SV_BATCH_GATE_1Q) {
      if (q0 < 0 || q0 >= C.n_qubits || !C.mats) return CIRC_BAD_1Q;
      const double *m = C.mats + 8 * size_t(j);
      if (cur_q == q0) {
        // cur <- m * cur
        double r[8];
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) {
            double re = 0, im = 0;
            for (int k = 0; k < 2; ++k) {
              const double xr = m[2 * (2 * a + k)], xi = m[2 * (2 * a + k) + 1];
              const double yr = cur[2 * (2 * k + b)], yi = cur[2 * (2 * k + b) + 1];
              re += xr * yr - xi * yi;
              im += xr * yi + xi * yr;
            }
            r[2 * (2 * a + b)] = re;
            r[2 * (2 * a + b) + 1] = im;
          }
        std::memcpy(cur, r, sizeof(r));
      } else {
        flush();
        std::memcpy(cur, m, sizeof(cur));
        cur_q = q0;
      }
    } else if (kind == SV_BATCH_GATE_CNOT) {
      if (q0 < 0 || q1 < 0 || q0 >= C.n_qubits || q1 >= C.n_qubits || q0 == q1) return CIRC_BAD_CNOT;
      flush();
      BGate b;
      std::memset(&b, 0, sizeof(b));
      b.kind = SV_BATCH_GATE_CNOT;
      b.q0 = q0;
      b.q1 = q1;
      g.push_back(b);
    } else {
      return CIRC_BAD_KIND;
    }
  }
  flush();
  if (C.n_qubits > kSliceBits) g = make_passes(g, C.n_qubits);
  g = group_single_qubit(g, C.n_qubits > kSliceBits);
  return CIRC_OK;
}

// Prepare every circuit (on up to 16 host threads taking circuits from a
// shared counter: circuits are independent, and a thread that cannot be
// started only costs parallelism), group by qubit count, sort each group by
// gate count so that packs hold circuits of similar length, cut packs, order
// by cost.
int pack_batch(int count, const sv_batch_circuit *circs, size_t states_bytes, const int64_t *state_offsets,
               const int32_t *cfg, Packed *out) {
  std::vector<std::vector<BGate>> fused(static_cast<size_t>(count));
  std::vector<int> status(static_cast<size_t>(count), CIRC_OK);
  std::atomic<int> next{0};
  auto work = [&]() {
    for (int i; (i = next.fetch_add(1)) < count;) {
      try {
        status[size_t(i)] = prepare_circuit(circs[i], state_offsets[i], states_bytes, fused[size_t(i)]);
      } catch (const std::bad_alloc &) {
        status[size_t(i)] = CIRC_NOMEM;
      }
    }
  };
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int nth = int(std::min<unsigned>({hw, 16u, unsigned(count / 64 + 1)}));
  std::vector<std::thread> pool;
  for (int t = 1; t < nth; ++t) {
    try {
      pool.emplace_back(work);
    } catch (const std::system_error &) {
      break;
    }
  }
  work();
  for (auto &th : pool) th.join();
  static const char *const what[] = {"", "bad batch circuit ", "bad single-qubit gate in batch circuit ",
                                     "bad CNOT in batch circuit ", "unknown gate kind in batch circuit ",
                                     "host allocation failed for batch circuit "};
  std::map<int, std::vector<int>> groups;
  for (int i = 0; i < count; ++i) {
    if (status[size_t(i)] != CIRC_OK) {
      set_error(what[status[size_t(i)]] + std::to_string(i));
      return SV_ERR_ARG;
    }
    groups[circs[i].n_qubits].push_back(i);
  }
  out->ncirc = count;
  std::vector<int64_t> gate_off(static_cast<size_t>(count));
  for (int i = 0; i < count; ++i) {
    gate_off[size_t(i)] = int64_t(out->gates.size());
    out->gates.insert(out->gates.end(), fused[size_t(i)].begin(), fused[size_t(i)].end());
  }
  std::vector<std::pair<double, BItem>> items;
  for (auto &kv : groups) {
    std::vector<int> ids = kv.second;
    const int n = kv.first;
    std::stable_sort(ids.begin(), ids.end(),
                     [&](int a, int b) { return fused[size_t(a)].size() > fused[size_t(b)].size(); });
    size_t pos = 0;
    while (pos < ids.size()) {
      int P = cfg[n];
      while (size_t(P) > ids.size() - pos) P /= 2;
      BItem it;
      std::memset(&it, 0, sizeof(it));
      it.n = n;
      it.P = P;
      int ng = 0;
      for (int c = 0; c < P; ++c) {
        const int id = ids[pos + size_t(c)];
        it.circ[c] = id;
        // records for a circuit run in passes, units for one held in LDS
        it.ngc[c] = (n > kSliceBits) ? int(fused[size_t(id)].size()) : count_units(fused[size_t(id)]);
        ng = std::max(ng, it.ngc[c]);
        it.gate_off[c] = gate_off[size_t(id)];
        it.state_off[c] = state_offsets[id] / 8;
      }
      it.ngates = ng;
      pos += size_t(P);
      const double cost = double(ng + 1) * double(int64_t(1) << n) * double(P);
      items.push_back({cost, it});
    }
  }
  std::stable_sort(items.begin(), items.end(),
                   [](const std::pair<double, BItem> &a, const std::pair<double, BItem> &b) { return a.first > b.first; });
  for (auto &pr : items) out->items.push_back(pr.second);
  return SV_OK;
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

extern "C" {

size_t sv_batch_workspace_bytes(int count, const sv_batch_circuit *circs) {
  if (count < 0 || (count > 0 && !circs)) return 0;
  size_t ng = 0;  // at most one pass record and half a group record per gate on top of the gates
  for (int i = 0; i < count; ++i) ng += 3 * size_t(std::max(0, circs[i].n_gates));
  return 256 + align256(sizeof(double) * size_t(std::max(1, count))) +
         align256(sizeof(BItem) * size_t(std::max(1, count))) + align256(sizeof(BGate) * std::max<size_t>(1, ng));
}

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

extern "C" int sv_batch_records(const sv_batch_circuit *c, int cap, int32_t *records, float *mats, int *n_out) {
  return guard([&]() -> int {
    if (!c || !records || !mats || !n_out || cap < 0) {
      set_error("null pointer");
      return SV_ERR_ARG;
    }
    if (c->n_qubits < 1 || c->n_qubits > SV_BATCH_MAX_QUBITS) {
      set_error("bad batch circuit");
      return SV_ERR_ARG;
    }
    int32_t cfg[SV_BATCH_CONFIG_LEN];
    default_config(cfg);
    const int64_t off = 0;
    Packed pk;
    const int rc = pack_batch(1, c, size_t(8) << c->n_qubits, &off, cfg, &pk);
    if (rc) return rc;
    if (pk.gates.size() > size_t(cap)) {
      set_error("record capacity too small");
      return SV_ERR_ARG;
    }
    for (size_t i = 0; i < pk.gates.size(); ++i) {
      const BGate &g = pk.gates[i];
      records[4 * i + 0] = g.kind;
      records[4 * i + 1] = g.q0;
      records[4 * i + 2] = g.q1;
      records[4 * i + 3] = 0;
      for (int e = 0; e < 8; ++e) mats[8 * i + size_t(e)] = g.m[e];
    }
    *n_out = int(pk.gates.size());
    return SV_OK;
  });
}
