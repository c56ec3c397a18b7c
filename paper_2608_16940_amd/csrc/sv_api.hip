// C-ABI of libsv: handle management, layout map, kernel selection, operand
// staging, probabilities, norm and sampling.  Host code only; kernels live in
// sv_kernels.hip and sv_tile.hip.
#include <algorithm>
#include <cmath>
#include <climits>
#include <utility>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sv_diagcover.h"
#include "sv_permute_host.h"
#include "sv_internal.h"
#include "sv_plan.h"

namespace sv {

namespace {
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

size_t workspace_layout(int n, char *base, Workspace *ws) {
  const int64_t nb = n > kCdfBlockBits ? (int64_t(1) << (n - kCdfBlockBits)) : 1;
  const int64_t nc = (nb + 1023) / 1024;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t o_ring = take(size_t(kRingSlots) * kRingSlotBytes);
  const size_t o_bs = take(size_t(nb) * 8);
  const size_t o_cs = take(size_t(nc) * 8);
  const size_t o_sh = take(size_t(kShotChunk) * 8);
  const size_t o_pa = take(size_t(kNormPartials) * 8);
  const size_t o_sc = take(64 * 8);
  if (base && ws) {
    ws->ring = base + o_ring;
    ws->blocksum = reinterpret_cast<uint64_t *>(base + o_bs);
    ws->chunksum = reinterpret_cast<uint64_t *>(base + o_cs);
    ws->shots = reinterpret_cast<uint64_t *>(base + o_sh);
    ws->partials = reinterpret_cast<double *>(base + o_pa);
    ws->scalars = reinterpret_cast<uint64_t *>(base + o_sc);
  }
  return off;
}

LayoutArg identity_layout(int n) {
  LayoutArg L;
  std::memset(&L, 0, sizeof(L));
  for (int q = 0; q < n; ++q) L.pos[q] = int8_t(q);
  return L;
}

// The sampler behind the sampling entry points:
// CDF build, then shots in chunks of `chunk` through ws.shots.  bad_code is
// the status for inputs the CDF build flags (entries outside [0, 4) or not a
// number, or a total of 2^64 or more in fixed point).
int sample_impl(const float2 *psi, const double *probs, int n, const Workspace &ws, int64_t chunk, uint64_t seed,
                int64_t shots, uint64_t *out_host, const LayoutArg &L, hipStream_t st, int bad_code) {
  SV_HIP_CHECK(launch_cdf_build(psi, probs, n, ws, st));
  const int64_t nb = n > kCdfBlockBits ? (int64_t(1) << (n - kCdfBlockBits)) : 1;
  uint64_t total = 0;
  unsigned bad = 0;
  SV_HIP_CHECK(hipMemcpyAsync(&total, ws.blocksum + (nb - 1), 8, hipMemcpyDeviceToHost, st));
  SV_HIP_CHECK(hipMemcpyAsync(&bad, cdf_flag(ws), sizeof(unsigned), hipMemcpyDeviceToHost, st));
  SV_HIP_CHECK(hipStreamSynchronize(st));
  if (bad) {
    set_error(psi ? "state probabilities not finite, or total probability of 4 or more"
                  : "probabilities must be finite, in [0, 4) and sum to less than 4");
    return bad_code;
  }
  if (total == 0) {
    set_error("zero total probability");
    return SV_ERR_STATE;
  }
  for (int64_t s0 = 0; s0 < shots; s0 += chunk) {
    const int64_t cnt = std::min<int64_t>(chunk, shots - s0);
    SV_HIP_CHECK(launch_shots(psi, probs, n, ws, seed, s0, cnt, L, st));
    SV_HIP_CHECK(hipMemcpyAsync(out_host + s0, ws.shots, size_t(cnt) * 8, hipMemcpyDeviceToHost, st));
    SV_HIP_CHECK(hipStreamSynchronize(st));
  }
  return SV_OK;
}

}  // namespace sv

namespace sv {

}  // namespace sv

using namespace sv;



namespace {

bool valid_n(int n) { return n >= SV_MIN_QUBITS && n <= SV_MAX_QUBITS; }

void reset_layout(sv_state *s) {
  for (int q = 0; q < s->n; ++q) {
    s->L[q] = s->Linv[q] = q;
    s->last_use[q] = 0;
    s->next_use[q] = INT64_MAX;
  }
  s->clock = 0;
  s->have_hints = false;
}

LayoutArg layout_arg(const sv_state *s) {
  LayoutArg a;
  std::memset(&a, 0, sizeof(a));
  for (int q = 0; q < s->n; ++q) a.pos[q] = int8_t(s->L[q]);
  return a;
}

// Stage `bytes` of host data into the next ring slot; returns the device pointer.
int stage(sv_state *s, const void *host, size_t bytes, void **dev, int *slot_out) {
  if (bytes > kRingSlotBytes) {
    set_error("operand too large for a staging slot");
    return SV_ERR_UNSUPPORTED;
  }
  const int slot = s->ring_next;
  s->ring_next = (s->ring_next + 1) % kRingSlots;
  if (s->ev_live[slot]) SV_HIP_CHECK(hipEventSynchronize(s->ev[slot]));
  char *ph = s->pinned + size_t(slot) * kRingSlotBytes;
  std::memcpy(ph, host, bytes);
  char *dv = s->ws.ring + size_t(slot) * kRingSlotBytes;
  SV_HIP_CHECK(hipMemcpyAsync(dv, ph, bytes, hipMemcpyHostToDevice, s->st));
  *dev = dv;
  *slot_out = slot;
  return SV_OK;
}

int release_slot(sv_state *s, int slot) {
  SV_HIP_CHECK(hipEventRecord(s->ev[slot], s->st));
  s->ev_live[slot] = true;
  return SV_OK;
}

void swap_physical(sv_state *s, int p, int q) {
  const int a = s->Linv[p], b = s->Linv[q];
  s->L[a] = q;
  s->L[b] = p;
  s->Linv[p] = b;
  s->Linv[q] = a;
}

// Victim choice among candidate physical positions (Corollary 1: farthest next
// use; without hints, least recently used; FIRST_FREE: lowest position).
// Ties go to the lowest physical position.
int pick_victim(int policy, const std::vector<int> &cand, const int32_t *Linv, bool have_hints,
                const int64_t *next_use, const int64_t *last_use) {
  int best = -1;
  for (int p : cand) {
    if (best < 0) {
      best = p;
      continue;
    }
    const int q = Linv[p], qb = Linv[best];
    bool better = false;
    if (policy == SV_POLICY_FIRST_FREE) {
      better = p < best;
    } else if (policy == SV_POLICY_BELADY && have_hints) {
      better = next_use[q] > next_use[qb] || (next_use[q] == next_use[qb] && p < best);
    } else {
      better = last_use[q] < last_use[qb] || (last_use[q] == last_use[qb] && p < best);
    }
    if (better) best = p;
  }
  return best;
}

// Lazy relabel plan for an MFMA sweep: targets at physical bits >= low_bits
// are exchanged with victim low non-target bits inside the tile.  Victims are
// drawn only from the tile's own non-target bits (the M lowest non-target
// bits), leaving its three lowest ones alone, so the relabelling sweep keeps
// exactly the access pattern of a plain sweep.  Returns the exchanged pairs.
std::vector<std::pair<int, int>> plan_relabel(const sv_state *s, const int32_t *A, int k, int M) {
  std::vector<std::pair<int, int>> pairs;
  uint64_t tmask = 0;
  for (int j = 0; j < k; ++j) tmask |= uint64_t(1) << A[j];
  std::vector<int> cand;
  int seen = 0;
  for (int p = 0; p < s->n && seen < M; ++p) {
    if ((tmask >> p) & 1) continue;
    ++seen;
    if (seen > 3 && p < s->low_bits) cand.push_back(p);
  }
  const int budget = M - 3;
  for (int j = 0; j < k && int(pairs.size()) < budget; ++j) {
    if (A[j] < s->low_bits || cand.empty()) continue;
    const int v = pick_victim(s->policy, cand, s->Linv, s->have_hints, s->next_use, s->last_use);
    cand.erase(std::find(cand.begin(), cand.end(), v));
    pairs.push_back({A[j], v});
  }
  return pairs;
}

// A gate resolved to one kernel launch: the chosen lowering, its physical
// targets, operands passed by value, and the host bytes of an operand that
// has to sit in device memory (MFMA operand, generic matrix, wide diagonal).
struct Lowered {
  int variant = SV_VARIANT_AUTO;
  int k = 0;
  int32_t A[8] = {0};
  DiagCover cover;             // diagonal: the subcubes its sweeps visit
  float2 m[256];               // by value: VALU matrix, shuffle 2x2, diagonal table with k <= 4
  bool by_value = false;
  std::vector<char> op;        // device operand bytes (empty when by value)
  TilePlan tp;                 // MFMA tile geometry
  int prec = SV_PREC_FP32, opsrc = SV_MFMA_OPERAND_AUTO;
  std::vector<std::pair<int, int>> relabel;  // MFMA store-side bit exchanges
};

// Choose the kernel for a gate on physical targets A and prepare its
// operands (the selector of the lowering step; Section IV-E).
int lower(const sv_state *s, const double *matrix, const int32_t *A, int k, bool allow_relabel, Lowered *L) {
  const int n = s->n;
  int v = s->variant;
  const bool shuffle_ok = (k == 1 && A[0] <= 6);
  const bool mfma_ok = (k >= 4 && k <= 7 && n >= k + mfma_tile_M(k));
  const bool valu_ok = (k <= 4);
  const int D = 1 << k;
  bool diag = true;  // every off-diagonal entry exactly zero
  for (int r = 0; r < D && diag; ++r)
    for (int c = 0; c < D; ++c)
      if (r != c && (matrix[2 * (r * D + c)] != 0.0 || matrix[2 * (r * D + c) + 1] != 0.0)) {
        diag = false;
        break;
      }
  if (v == SV_VARIANT_AUTO) {
    if (diag)
      v = SV_VARIANT_DIAG;
    else if (shuffle_ok)
      v = SV_VARIANT_SHUFFLE;
    else if (mfma_ok && k >= s->mfma_min_k)
      v = SV_VARIANT_MFMA;
    else if (valu_ok)
      v = SV_VARIANT_VALU;
    else
      v = SV_VARIANT_GENERIC;
  }
  L->variant = v;
  L->k = k;
  for (int j = 0; j < k; ++j) L->A[j] = A[j];
  L->prec = s->prec;
  L->opsrc = s->opsrc;
  switch (v) {
    case SV_VARIANT_DIAG: {
      if (!diag) {
        set_error("diagonal lowering needs a diagonal matrix");
        return SV_ERR_UNSUPPORTED;
      }
      std::vector<float2> d(static_cast<size_t>(D));
      for (int r = 0; r < D; ++r)
        d[r] = make_float2(float(matrix[2 * (r * D + r)]), float(matrix[2 * (r * D + r) + 1]));
      std::vector<double> dd(2 * size_t(D));
      for (int r = 0; r < D; ++r) {
        dd[2 * size_t(r)] = matrix[2 * (r * D + r)];
        dd[2 * size_t(r) + 1] = matrix[2 * (r * D + r) + 1];
      }
      L->cover = diag_cover(k, dd.data(), A);
      if (k <= 4) {  // small tables ride in the kernel arguments
        L->by_value = true;
        for (int r = 0; r < D; ++r) L->m[r] = d[r];
      } else {
        L->op.resize(d.size() * sizeof(float2));
        std::memcpy(L->op.data(), d.data(), L->op.size());
      }
      return SV_OK;
    }
    case SV_VARIANT_SHUFFLE:
    case SV_VARIANT_VALU:
      if ((v == SV_VARIANT_SHUFFLE && !shuffle_ok) || (v == SV_VARIANT_VALU && !valu_ok)) {
        set_error("forced variant does not apply to this gate");
        return SV_ERR_UNSUPPORTED;
      }
      L->by_value = true;
      for (int i = 0; i < D * D; ++i) L->m[i] = make_float2(float(matrix[2 * i]), float(matrix[2 * i + 1]));
      return SV_OK;
    case SV_VARIANT_MFMA: {
      if (!mfma_ok) {
        set_error("MFMA lowering needs 4 <= k <= 7 and a state of at least k + tile bits");
        return SV_ERR_UNSUPPORTED;
      }
      if (s->lazy && allow_relabel) L->relabel = plan_relabel(s, A, k, mfma_tile_M(k));
      uint64_t extra = 0;
      for (auto &pr : L->relabel) extra |= uint64_t(1) << pr.second;
      if (!make_gate_tile(n, k, A, extra, &L->tp)) {
        set_error("tile geometry failed");
        return SV_ERR_UNSUPPORTED;
      }
      L->tp.order = s->tile_order;
      // store side: output tile-order bit of position a reads the local bit that
      // held position v on load, and vice versa (a physical bit exchange)
      for (auto &pr : L->relabel) {
        int ba = -1, bv = -1;
        for (int b = 0; b < L->tp.s; ++b) {
          if (L->tp.sbit[b] == pr.first) ba = b;
          if (L->tp.sbit[b] == pr.second) bv = b;
        }
        const int t = L->tp.loc_out[ba];
        L->tp.loc_out[ba] = L->tp.loc_out[bv];
        L->tp.loc_out[bv] = t;
      }
      L->op.resize(mfma_operand_bytes(k, s->prec));
      pack_mfma_operand(k, s->prec, matrix, L->op.data());
      return SV_OK;
    }
    case SV_VARIANT_GENERIC: {
      if (k > 8) {
        set_error("generic lowering supports k <= 8");
        return SV_ERR_UNSUPPORTED;
      }
      std::vector<float2> m(size_t(D) * D);
      for (size_t i = 0; i < m.size(); ++i) m[i] = make_float2(float(matrix[2 * i]), float(matrix[2 * i + 1]));
      L->op.resize(m.size() * sizeof(float2));
      std::memcpy(L->op.data(), m.data(), L->op.size());
      return SV_OK;
    }
    default:
      set_error("unknown variant");
      return SV_ERR_ARG;
  }
}

// Launch a lowered gate; op_dev holds L.op in device memory when it is not by value.
// 16-byte chunks a diagonal block's sweeps read and write (a full sweep is 2^(N-1)).
int64_t diag_chunks(const Lowered &L, int n) {
  int64_t c = 0;
  for (int i = 0; i < L.cover.nsub; ++i) c += (int64_t(1) << (n - 1)) >> __builtin_popcount(L.cover.mask[i]);
  return c;
}

int launch_lowered(sv_state *s, const Lowered &L, const void *op_dev) {
  const int n = s->n;
  hipError_t e = hipSuccess;
  switch (L.variant) {
    case SV_VARIANT_DIAG:
      for (int i = 0; i < L.cover.nsub && e == hipSuccess; ++i) {
        int32_t fp[8];
        int nf = 0, fv = 0;
        for (int j = 0; j < L.k; ++j)
          if ((L.cover.mask[i] >> j) & 1) {
            fp[nf] = L.A[j];
            fv |= ((L.cover.val[i] >> j) & 1) << nf;
            ++nf;
          }
        e = L.by_value ? launch_diag(s->amps, n, L.k, L.A, nullptr, L.m, nf, fp, fv, s->st)
                       : launch_diag(s->amps, n, L.k, L.A, static_cast<const float2 *>(op_dev), nullptr, nf, fp, fv,
                                     s->st);
      }
      break;
    case SV_VARIANT_SHUFFLE: e = launch_1q_shuffle(s->amps, n, L.A[0], L.m, s->st); break;
    case SV_VARIANT_VALU: e = launch_dense_valu(s->amps, n, L.k, L.A, L.m, s->st); break;
    case SV_VARIANT_MFMA: e = launch_tile_mfma(L.tp, L.prec, L.opsrc, s->amps, op_dev, s->st); break;
    case SV_VARIANT_GENERIC:
      e = launch_dense_generic(s->amps, n, L.k, L.A, static_cast<const float2 *>(op_dev), s->st);
      break;
    default: e = hipErrorInvalidValue;
  }
  if (e != hipSuccess) {
    set_error(std::string("kernel launch failed: ") + hipGetErrorString(e));
    return SV_ERR_DEVICE;
  }
  s->stats.gate_sweeps += 1;
  s->stats.launches += (L.variant == SV_VARIANT_DIAG) ? L.cover.nsub : 1;
  if (L.variant >= 0 && L.variant < 6) s->stats.by_variant[L.variant] += 1;
  if (L.variant == SV_VARIANT_DIAG) s->stats.diag_chunks += diag_chunks(L, n);
  return SV_OK;
}

int apply_physical(sv_state *s, const double *matrix, const int32_t *A, int k) {
  Lowered L;
  int rc = lower(s, matrix, A, k, true, &L);
  if (rc) return rc;
  if (L.op.empty()) return launch_lowered(s, L, nullptr);
  void *dev = nullptr;
  int slot = 0;
  rc = stage(s, L.op.data(), L.op.size(), &dev, &slot);
  if (rc) return rc;
  rc = launch_lowered(s, L, dev);
  if (rc) return rc;
  rc = release_slot(s, slot);
  if (rc) return rc;
  for (auto &pr : L.relabel) swap_physical(s, pr.first, pr.second);
  s->stats.relabels += int64_t(L.relabel.size());
  return SV_OK;
}

}  // namespace

extern "C" {

size_t sv_workspace_bytes(int n_qubits) {
  if (!valid_n(n_qubits)) return 0;
  return workspace_layout(n_qubits, nullptr, nullptr);
}

int sv_alloc(sv_state **out, int n, void *amps_dev, size_t amps_bytes, void *ws_dev, size_t ws_bytes,
             void *stream) {
  return guard([&]() -> int {
    clear_error();
    if (!out || !amps_dev || !ws_dev) {
      set_error("null pointer");
      return SV_ERR_ARG;
    }
    *out = nullptr;
    if (!valid_n(n)) {
      set_error("n_qubits out of range [1, 35]");
      return SV_ERR_ARG;
    }
    if (amps_bytes < (size_t(8) << n)) {
      set_error("state buffer smaller than 8 * 2^N bytes");
      return SV_ERR_ARG;
    }
    if (ws_bytes < sv_workspace_bytes(n)) {
      set_error("workspace smaller than sv_workspace_bytes(N)");
      return SV_ERR_ARG;
    }
    if ((reinterpret_cast<uintptr_t>(amps_dev) & 255) || (reinterpret_cast<uintptr_t>(ws_dev) & 255)) {
      set_error("device buffers must be 256-byte aligned");
      return SV_ERR_ARG;
    }
    sv_state *s = new sv_state();
    s->n = n;
    s->amps = static_cast<float2 *>(amps_dev);
    s->ws_base = static_cast<char *>(ws_dev);
    s->ws_bytes = ws_bytes;
    workspace_layout(n, s->ws_base, &s->ws);
    s->st = static_cast<hipStream_t>(stream);
    std::memset(&s->stats, 0, sizeof(s->stats));
    for (int i = 0; i < kRingSlots; ++i) s->ev_live[i] = false;
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&s->pinned), size_t(kRingSlots) * kRingSlotBytes,
                                 hipHostMallocDefault);
    if (e != hipSuccess) {
      set_error(std::string("hipHostMalloc failed: ") + hipGetErrorString(e));
      delete s;
      return SV_ERR_DEVICE;
    }
    for (int i = 0; i < kRingSlots; ++i) {
      e = hipEventCreateWithFlags(&s->ev[i], hipEventDisableTiming);
      if (e != hipSuccess) {
        set_error(std::string("hipEventCreate failed: ") + hipGetErrorString(e));
        for (int j = 0; j < i; ++j) (void)hipEventDestroy(s->ev[j]);
        (void)hipHostFree(s->pinned);
        delete s;
        return SV_ERR_DEVICE;
      }
    }
    reset_layout(s);
    e = launch_init_zero(s->amps, n, s->st);
    if (e != hipSuccess) {
      set_error(std::string("init launch failed: ") + hipGetErrorString(e));
      for (int j = 0; j < kRingSlots; ++j) (void)hipEventDestroy(s->ev[j]);
      (void)hipHostFree(s->pinned);
      delete s;
      return SV_ERR_DEVICE;
    }
    *out = s;
    return SV_OK;
  });
}

int sv_free(sv_state *s) {
  return guard([&]() -> int {
    if (!s) return SV_OK;
    (void)hipStreamSynchronize(s->st);
    for (int i = 0; i < kRingSlots; ++i) (void)hipEventDestroy(s->ev[i]);
    if (s->pinned) (void)hipHostFree(s->pinned);
    delete s;
    return SV_OK;
  });
}

int sv_reset(sv_state *s) {
  return guard([&]() -> int {
    if (!s) {
      set_error("null handle");
      return SV_ERR_ARG;
    }
    reset_layout(s);
    std::memset(&s->stats, 0, sizeof(s->stats));
    SV_HIP_CHECK(launch_init_zero(s->amps, s->n, s->st));
    return SV_OK;
  });
}

int sv_apply_fused(sv_state *s, const double *matrix, const int32_t *targets, int k) {
  return guard([&]() -> int {
    if (!s || !matrix || !targets) {
      set_error("null pointer");
      return SV_ERR_ARG;
    }
    if (k < 1 || k > s->n || k > SV_MAX_K) {
      set_error("k out of range [1, min(N, SV_MAX_K)]");
      return SV_ERR_ARG;
    }
    int32_t A[SV_MAX_K];
    for (int j = 0; j < k; ++j) {
      if (targets[j] < 0 || targets[j] >= s->n) {
        set_error("target qubit out of range");
        return SV_ERR_ARG;
      }
      for (int i = 0; i < j; ++i)
        if (targets[i] == targets[j]) {
          set_error("duplicate target qubit");
          return SV_ERR_ARG;
        }
      A[j] = s->L[targets[j]];
    }
    // A block that only permutes its qubits (a SWAP network) moves no data: the
    // value of logical qubit targets[j] now sits under targets[perm[j]], which
    // the layout map records (Lemma 2 per exchanged pair): L'(targets[perm[j]])
    // = L(targets[j]).  Forced variants still sweep.
    int perm[SV_MAX_K];
    if (s->variant == SV_VARIANT_AUTO && qubit_permutation(matrix, k, perm)) {
      int32_t old[SV_MAX_K];
      for (int j = 0; j < k; ++j) old[j] = s->L[targets[j]];
      for (int j = 0; j < k; ++j) {
        s->L[targets[perm[j]]] = old[j];
        s->Linv[old[j]] = targets[perm[j]];
      }
      s->stats.layout_only += 1;
      ++s->clock;
      for (int j = 0; j < k; ++j) s->last_use[targets[j]] = s->clock;
      return SV_OK;
    }
    const int rc = apply_physical(s, matrix, A, k);
    if (rc == SV_OK) {
      ++s->clock;
      for (int j = 0; j < k; ++j) s->last_use[targets[j]] = s->clock;
    }
    return rc;
  });
}

int sv_permute_layout(sv_state *s, const int32_t *new_layout) {
  return guard([&]() -> int {
    if (!s || !new_layout) {
      set_error("null pointer");
      return SV_ERR_ARG;
    }
    const int n = s->n;
    bool seen[64] = {false};
    for (int q = 0; q < n; ++q) {
      const int p = new_layout[q];
      if (p < 0 || p >= n || seen[p]) {
        set_error("new layout is not a bijection");
        return SV_ERR_ARG;
      }
      seen[p] = true;
    }
    // Selection order (permutation_swaps): fill physical positions 0..n-1
    // with their final qubits, one bit transposition at a time.  Consecutive
    // disjoint transpositions commute, so several of them run as one
    // in-place tile pass (permutation_pass_end) when the state has at least
    // kPermTileBits qubits; smaller states use single transposition passes.
    const std::vector<std::pair<int, int>> swaps = permutation_swaps(s->L, new_layout, n);
    size_t i = 0;
    while (i < swaps.size()) {
      if (n < kPermTileBits) {
        SV_HIP_CHECK(launch_swap_bits(s->amps, n, swaps[i].first, swaps[i].second, s->st));
        swap_physical(s, swaps[i].first, swaps[i].second);
        s->stats.swap_half_sweeps += 1;
        s->stats.launches += 1;
        ++i;
        continue;
      }
      const size_t j = permutation_pass_end(swaps, i);
      uint64_t used = 0;
      for (size_t t = i; t < j; ++t) used |= (uint64_t(1) << swaps[t].first) | (uint64_t(1) << swaps[t].second);
      // tile: the exchanged bits plus the lowest other bits, kPermTileBits in all
      uint64_t smask = used;
      for (int p = 0; p < n && __builtin_popcountll(smask) < kPermTileBits; ++p) smask |= uint64_t(1) << p;
      TilePlan tp;
      tp.n = n;
      tp.s = kPermTileBits;
      tp.order = s->tile_order;
      int b = 0;
      for (int p = 0; p < n; ++p)
        if ((smask >> p) & 1) {
          tp.sbit[b] = p;
          tp.loc_in[b] = b;
          tp.loc_out[b] = b;
          ++b;
        }
      for (size_t t = i; t < j; ++t) {
        int ba = -1, bb = -1;
        for (int c = 0; c < tp.s; ++c) {
          if (tp.sbit[c] == swaps[t].first) ba = c;
          if (tp.sbit[c] == swaps[t].second) bb = c;
        }
        tp.loc_out[ba] = bb;
        tp.loc_out[bb] = ba;
      }
      SV_HIP_CHECK(launch_tile_permute(tp, s->amps, s->st));
      for (size_t t = i; t < j; ++t) swap_physical(s, swaps[t].first, swaps[t].second);
      s->stats.permute_sweeps += 1;
      s->stats.launches += 1;
      i = j;
    }
    return SV_OK;
  });
}

int sv_hint_next_use(sv_state *s, const int64_t *next_use) {
  return guard([&]() -> int {
    if (!s || !next_use) {
      set_error("null pointer");
      return SV_ERR_ARG;
    }
    for (int q = 0; q < s->n; ++q) s->next_use[q] = next_use[q];
    s->have_hints = true;
    return SV_OK;
  });
}

int sv_policy_simulate(int n, int frames, int policy, int n_tuples, const int32_t *ks, const int32_t *targets,
                       int64_t *out) {
  return guard([&]() -> int {
    if (!out || n < 1 || n > 64 || frames < 1 || frames > n || n_tuples < 0 || (n_tuples > 0 && (!ks || !targets)) ||
        policy < SV_POLICY_BELADY || policy > SV_POLICY_LRU) {
      set_error("bad argument");
      return SV_ERR_ARG;
    }
    std::vector<std::vector<int>> tup(static_cast<size_t>(n_tuples));
    size_t off = 0;
    for (int i = 0; i < n_tuples; ++i) {
      if (ks[i] < 1 || ks[i] > frames) {
        set_error("tuple wider than the frame count");
        return SV_ERR_ARG;
      }
      for (int j = 0; j < ks[i]; ++j) {
        const int q = targets[off + j];
        if (q < 0 || q >= n) {
          set_error("target out of range");
          return SV_ERR_ARG;
        }
        tup[size_t(i)].push_back(q);
      }
      off += size_t(ks[i]);
    }
    // positions 0..frames-1 are frames; position of qubit q is L[q]
    int32_t L[64], Linv[64];
    int64_t last_use[64] = {0}, next_use[64];
    for (int q = 0; q < n; ++q) L[q] = Linv[q] = q;
    int64_t promotions = 0;
    for (int i = 0; i < n_tuples; ++i) {
      for (int q = 0; q < n; ++q) {
        next_use[q] = INT64_MAX;
        for (int t = i + 1; t < n_tuples; ++t)
          if (std::find(tup[size_t(t)].begin(), tup[size_t(t)].end(), q) != tup[size_t(t)].end()) {
            next_use[q] = t;
            break;
          }
      }
      for (int q : tup[size_t(i)]) {
        if (L[q] < frames) continue;
        std::vector<int> cand;
        for (int p = 0; p < frames; ++p)
          if (std::find(tup[size_t(i)].begin(), tup[size_t(i)].end(), Linv[p]) == tup[size_t(i)].end())
            cand.push_back(p);
        const int v = pick_victim(policy, cand, Linv, true, next_use, last_use);
        const int a = q, b = Linv[v], pa = L[q];
        L[a] = v;
        L[b] = pa;
        Linv[v] = a;
        Linv[pa] = b;
        ++promotions;
      }
      for (int q : tup[size_t(i)]) last_use[q] = i + 1;
    }
    *out = promotions;
    return SV_OK;
  });
}

int sv_get_layout(const sv_state *s, int32_t *out) {
  return guard([&]() -> int {
    if (!s || !out) {
      set_error("null pointer");
      return SV_ERR_ARG;
    }
    for (int q = 0; q < s->n; ++q) out[q] = s->L[q];
    return SV_OK;
  });
}

int sv_probs(sv_state *s, double *out_dev, int logical_order) {
  return guard([&]() -> int {
    if (!s || !out_dev) {
      set_error("null pointer");
      return SV_ERR_ARG;
    }
    SV_HIP_CHECK(launch_probs(s->amps, s->n, out_dev, logical_order ? 1 : 0, layout_arg(s), s->st));
    return SV_OK;
  });
}

int sv_norm(sv_state *s, double *out_host) {
  return guard([&]() -> int {
    if (!s || !out_host) {
      set_error("null pointer");
      return SV_ERR_ARG;
    }
    double *res = reinterpret_cast<double *>(s->ws.scalars);
    SV_HIP_CHECK(launch_norm(s->amps, s->n, s->ws.partials, res, s->st));
    SV_HIP_CHECK(hipMemcpyAsync(out_host, res, sizeof(double), hipMemcpyDeviceToHost, s->st));
    SV_HIP_CHECK(hipStreamSynchronize(s->st));
    return SV_OK;
  });
}

int sv_sample(sv_state *s, uint64_t seed, int64_t shots, uint64_t *out_host) {
  return guard([&]() -> int {
    if (!s || (!out_host && shots > 0) || shots < 0) {
      set_error("bad argument");
      return SV_ERR_ARG;
    }
    if (shots == 0) return SV_OK;
    return sample_impl(s->amps, nullptr, s->n, s->ws, kShotChunk, seed, shots, out_host, layout_arg(s), s->st,
                       SV_ERR_STATE);
  });
}

int sv_sample_probs(const double *probs_dev, int n, uint64_t seed, int64_t shots, uint64_t *out_host,
                    void *ws_dev, size_t ws_bytes, void *stream) {
  return guard([&]() -> int {
    if (!probs_dev || !ws_dev || (!out_host && shots > 0) || shots < 0 || !valid_n(n)) {
      set_error("bad argument");
      return SV_ERR_ARG;
    }
    if (ws_bytes < sv_workspace_bytes(n)) {
      set_error("workspace smaller than sv_workspace_bytes(n)");
      return SV_ERR_ARG;
    }
    if (shots == 0) return SV_OK;
    Workspace ws;
    workspace_layout(n, static_cast<char *>(ws_dev), &ws);
    return sample_impl(nullptr, probs_dev, n, ws, kShotChunk, seed, shots, out_host, identity_layout(n),
                       static_cast<hipStream_t>(stream), SV_ERR_ARG);
  });
}

int sv_copy_out(sv_state *s, void *out_host, int logical_order) {
  return guard([&]() -> int {
    if (!s || !out_host) {
      set_error("null pointer");
      return SV_ERR_ARG;
    }
    const int n = s->n;
    const uint64_t dim = uint64_t(1) << n;
    SV_HIP_CHECK(hipStreamSynchronize(s->st));
    if (!logical_order) {
      SV_HIP_CHECK(hipMemcpy(out_host, s->amps, dim * sizeof(float2), hipMemcpyDeviceToHost));
      return SV_OK;
    }
    // Stream the state through a bounded staging buffer in physical order and
    // scatter each amplitude to its logical index: bit q of x is bit L(q) of y,
    // assembled from one table lookup per byte of y.
    constexpr uint64_t kStage = uint64_t(1) << 22;  // 32 MiB of complex64
    const int nbytes = (n + 7) / 8;
    std::vector<uint64_t> tab(size_t(nbytes) * 256, 0);
    std::vector<float2> buf(size_t(std::min(dim, kStage)));
    for (int q = 0; q < n; ++q) {
      const int p = s->L[q];
      for (int v = 0; v < 256; ++v)
        if ((v >> (p & 7)) & 1) tab[size_t(p >> 3) * 256 + size_t(v)] |= uint64_t(1) << q;
    }
    float2 *out = static_cast<float2 *>(out_host);
    for (uint64_t a = 0; a < dim; a += buf.size()) {
      const uint64_t cnt = std::min<uint64_t>(buf.size(), dim - a);
      SV_HIP_CHECK(hipMemcpy(buf.data(), s->amps + a, cnt * sizeof(float2), hipMemcpyDeviceToHost));
      for (uint64_t i = 0; i < cnt; ++i) {
        const uint64_t y = a + i;
        uint64_t x = 0;
        for (int byte = 0; byte < nbytes; ++byte) x |= tab[size_t(byte) * 256 + ((y >> (8 * byte)) & 255)];
        out[x] = buf[size_t(i)];
      }
    }
    return SV_OK;
  });
}

int sv_sync(sv_state *s) {
  return guard([&]() -> int {
    if (!s) {
      set_error("null handle");
      return SV_ERR_ARG;
    }
    SV_HIP_CHECK(hipStreamSynchronize(s->st));
    return SV_OK;
  });
}

int sv_set_option(sv_state *s, int key, int value) {
  return guard([&]() -> int {
    if (!s) {
      set_error("null handle");
      return SV_ERR_ARG;
    }
    switch (key) {
      case SV_OPT_VARIANT:
        if (value < SV_VARIANT_AUTO || value > SV_VARIANT_DIAG) break;
        s->variant = value;
        return SV_OK;
      case SV_OPT_PRECISION:
        if (value != SV_PREC_FP32 && value != SV_PREC_BF16X3) break;
        s->prec = value;
        return SV_OK;
      case SV_OPT_MFMA_MIN_K:
        if (value < 4 || value > 8) break;
        s->mfma_min_k = value;
        return SV_OK;
      case SV_OPT_LAZY_RELABEL:
        s->lazy = value ? 1 : 0;
        return SV_OK;
      case SV_OPT_LOW_BITS:
        if (value < 1 || value > 35) break;
        s->low_bits = value;
        return SV_OK;
      case SV_OPT_POLICY:
        if (value < SV_POLICY_BELADY || value > SV_POLICY_LRU) break;
        s->policy = value;
        return SV_OK;
      case SV_OPT_MFMA_OPERAND:
        if (value < SV_MFMA_OPERAND_REGS || value > SV_MFMA_OPERAND_AUTO) break;
        s->opsrc = value;
        return SV_OK;
      case SV_OPT_TILE_ORDER:
        if (value < -1 || value > 30) break;
        s->tile_order = value;
        return SV_OK;
      default:
        break;
    }
    set_error("bad option key or value");
    return SV_ERR_ARG;
  });
}

int sv_get_option(const sv_state *s, int key, int *value) {
  return guard([&]() -> int {
    if (!s || !value) {
      set_error("null pointer");
      return SV_ERR_ARG;
    }
    switch (key) {
      case SV_OPT_VARIANT: *value = s->variant; return SV_OK;
      case SV_OPT_PRECISION: *value = s->prec; return SV_OK;
      case SV_OPT_MFMA_MIN_K: *value = s->mfma_min_k; return SV_OK;
      case SV_OPT_LAZY_RELABEL: *value = s->lazy; return SV_OK;
      case SV_OPT_LOW_BITS: *value = s->low_bits; return SV_OK;
      case SV_OPT_MFMA_OPERAND: *value = s->opsrc; return SV_OK;
      case SV_OPT_TILE_ORDER: *value = s->tile_order; return SV_OK;
      case SV_OPT_POLICY: *value = s->policy; return SV_OK;
      default: break;
    }
    set_error("bad option key");
    return SV_ERR_ARG;
  });
}

int sv_get_stats(const sv_state *s, sv_stats *out) {
  return guard([&]() -> int {
    if (!s || !out) {
      set_error("null pointer");
      return SV_ERR_ARG;
    }
    *out = s->stats;
    return SV_OK;
  });
}

}  // extern "C"

// ------------------------------------------------------------------ bound plans
struct sv_bound {
  sv_state *s = nullptr;
  std::vector<Lowered> ops;  // variant -1: a qubit permutation, absorbed by the layout map
  std::vector<size_t> off;   // operand offset in op_dev (SIZE_MAX: by value)
  char *op_dev = nullptr;
  int32_t L[64];             // layout a run starts from
  int32_t Lend[64];          // layout a run leaves (after the absorbed permutations)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;  // private stream the graph is captured on
  sv_stats per_run;               // statistics one run adds
};

namespace {

int lower_plan(sv_state *s, const sv_plan *p, std::vector<Lowered> *ops, std::vector<size_t> *off, size_t *bytes,
               int32_t *Lend) {
  if (s->lazy) {
    set_error("bound plans need lazy relabel off");
    return SV_ERR_ARG;
  }
  int nb = 0;
  int rc = sv_plan_num_blocks(p, &nb);
  if (rc) return rc;
  ops->assign(static_cast<size_t>(nb), Lowered());
  off->assign(static_cast<size_t>(nb), SIZE_MAX);
  size_t total = 0;
  int32_t L[64];  // the layout as the run will see it block by block
  std::memcpy(L, s->L, sizeof(L));
  for (int i = 0; i < nb; ++i) {
    int sw = 0;
    rc = sv_plan_block_swap(p, i, &sw, nullptr);
    if (rc) return rc;
    if (sw) {
      set_error("a plan with layout-swap blocks runs through sv_run_plan, not as a bound plan");
      return SV_ERR_UNSUPPORTED;
    }
    int k = 0, ng = 0, dg = 0;
    int32_t t[8];
    rc = sv_plan_block_info(p, i, &k, t, &ng, &dg);
    if (rc) return rc;
    std::vector<double> m(size_t(2) << (2 * k));
    rc = sv_plan_block_matrix(p, i, m.data());
    if (rc) return rc;
    int32_t A[8];
    for (int j = 0; j < k; ++j) {
      if (t[j] < 0 || t[j] >= s->n) {
        set_error("plan target outside the state");
        return SV_ERR_ARG;
      }
      A[j] = L[t[j]];
    }
    int perm[SV_MAX_K];
    if (s->variant == SV_VARIANT_AUTO && qubit_permutation(m.data(), k, perm)) {  // as sv_apply_fused
      int32_t old[SV_MAX_K];
      for (int j = 0; j < k; ++j) old[j] = L[t[j]];
      for (int j = 0; j < k; ++j) L[t[perm[j]]] = old[j];
      (*ops)[size_t(i)].variant = -1;
      continue;
    }
    rc = lower(s, m.data(), A, k, false, &(*ops)[size_t(i)]);
    if (rc) return rc;
    if (!(*ops)[size_t(i)].op.empty()) {
      (*off)[size_t(i)] = total;
      total += align256((*ops)[size_t(i)].op.size());
    }
  }
  *bytes = total;
  if (Lend) std::memcpy(Lend, L, sizeof(L));
  return SV_OK;
}

int bound_check(const sv_bound *b) {
  if (!b || !b->s) {
    set_error("null bound plan");
    return SV_ERR_ARG;
  }
  if (std::memcmp(b->L, b->s->L, sizeof(int32_t) * size_t(b->s->n)) != 0) {
    set_error("layout changed since the plan was bound");
    return SV_ERR_ARG;
  }
  return SV_OK;
}

int bound_launch_all(sv_bound *b) {
  for (size_t i = 0; i < b->ops.size(); ++i) {
    if (b->ops[i].variant < 0) continue;
    const void *dev = b->off[i] == SIZE_MAX ? nullptr : b->op_dev + b->off[i];
    const int rc = launch_lowered(b->s, b->ops[i], dev);
    if (rc) return rc;
  }
  return SV_OK;
}

void add_stats(sv_stats *a, const sv_stats &d) {
  a->gate_sweeps += d.gate_sweeps;
  a->launches += d.launches;
  a->layout_only += d.layout_only;
  for (int v = 0; v < 6; ++v) a->by_variant[v] += d.by_variant[v];
  a->diag_chunks += d.diag_chunks;
}

// After a run: the handle's layout is the one the absorbed permutations leave.
void bound_finish(sv_bound *b) {
  sv_state *s = b->s;
  for (int q = 0; q < s->n; ++q) {
    s->L[q] = b->Lend[q];
    s->Linv[b->Lend[q]] = q;
  }
}

}  // namespace

extern "C" {

int sv_bound_bytes(sv_state *s, const sv_plan *p, size_t *out) {
  return guard([&]() -> int {
    if (!s || !p || !out) {
      set_error("null pointer");
      return SV_ERR_ARG;
    }
    std::vector<Lowered> ops;
    std::vector<size_t> off;
    return lower_plan(s, p, &ops, &off, out, nullptr);
  });
}

int sv_plan_bind(sv_state *s, const sv_plan *p, void *op_dev, size_t op_bytes, sv_bound **out) {
  return guard([&]() -> int {
    if (!s || !p || !out) {
      set_error("null pointer");
      return SV_ERR_ARG;
    }
    sv_bound *b = new sv_bound();
    b->s = s;
    size_t need = 0;
    int rc = lower_plan(s, p, &b->ops, &b->off, &need, b->Lend);
    if (rc) {
      delete b;
      return rc;
    }
    if (need > 0 && (!op_dev || op_bytes < need || (reinterpret_cast<uintptr_t>(op_dev) & 255))) {
      delete b;
      set_error("operand buffer missing, too small or not 256-byte aligned");
      return SV_ERR_ARG;
    }
    b->op_dev = static_cast<char *>(op_dev);
    std::vector<char> host(need);
    for (size_t i = 0; i < b->ops.size(); ++i) {
      if (b->off[i] == SIZE_MAX) continue;
      std::memcpy(host.data() + b->off[i], b->ops[i].op.data(), b->ops[i].op.size());
      b->ops[i].op.clear();
      b->ops[i].op.shrink_to_fit();
    }
    if (need > 0) {
      hipError_t e = hipMemcpyAsync(op_dev, host.data(), need, hipMemcpyHostToDevice, s->st);
      if (e == hipSuccess) e = hipStreamSynchronize(s->st);
      if (e != hipSuccess) {
        delete b;
        set_error(std::string("operand upload failed: ") + hipGetErrorString(e));
        return SV_ERR_DEVICE;
      }
    }
    std::memcpy(b->L, s->L, sizeof(b->L));
    std::memset(&b->per_run, 0, sizeof(b->per_run));
    for (const Lowered &L : b->ops) {
      if (L.variant < 0) {
        b->per_run.layout_only += 1;
        continue;
      }
      b->per_run.gate_sweeps += 1;
      b->per_run.launches += (L.variant == SV_VARIANT_DIAG) ? L.cover.nsub : 1;
      if (L.variant < 6) b->per_run.by_variant[L.variant] += 1;
      if (L.variant == SV_VARIANT_DIAG) b->per_run.diag_chunks += diag_chunks(L, s->n);
    }
    *out = b;
    return SV_OK;
  });
}

int sv_bound_run(sv_bound *b) {
  return guard([&]() -> int {
    int rc = bound_check(b);
    if (rc) return rc;
    const int64_t before = b->s->stats.layout_only;
    rc = bound_launch_all(b);
    if (rc) return rc;
    b->s->stats.layout_only = before + b->per_run.layout_only;
    bound_finish(b);
    return SV_OK;
  });
}

int sv_bound_graph_run(sv_bound *b) {
  return guard([&]() -> int {
    int rc = bound_check(b);
    if (rc) return rc;
    sv_state *s = b->s;
    if (!b->exec) {
      // The handle's stream may be the legacy default stream, which cannot be
      // captured: capture on a private stream (default priority), launch the
      // graph on the handle's stream.
      hipError_t e = hipSuccess;
      if (!b->capture) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed);
      if (e != hipSuccess) {
        set_error(std::string("graph capture failed to start: ") + hipGetErrorString(e));
        return SV_ERR_DEVICE;
      }
      const sv_stats saved = s->stats;
      hipStream_t user = s->st;
      s->st = b->capture;
      rc = bound_launch_all(b);
      s->st = user;
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(b->capture, &g);
      s->stats = saved;  // nothing ran while capturing
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess || !g) {
        set_error(std::string("graph capture failed: ") + hipGetErrorString(e));
        return SV_ERR_DEVICE;
      }
      e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        b->exec = nullptr;
        set_error(std::string("graph instantiation failed: ") + hipGetErrorString(e));
        return SV_ERR_DEVICE;
      }
      b->graph = g;
    }
    const hipError_t e = hipGraphLaunch(b->exec, s->st);
    if (e != hipSuccess) {
      set_error(std::string("graph launch failed: ") + hipGetErrorString(e));
      return SV_ERR_DEVICE;
    }
    add_stats(&s->stats, b->per_run);
    bound_finish(b);
    return SV_OK;
  });
}

int sv_bound_free(sv_bound *b) {
  return guard([&]() -> int {
    if (!b) return SV_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    delete b;
    return SV_OK;
  });
}

}  // extern "C"
