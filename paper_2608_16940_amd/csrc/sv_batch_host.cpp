// Batched path, host pass: per-circuit records for the persistent kernel
// (see sv_batch_host.h).  Plain C++, no HIP: also built on its own for the
// host sanitizer checks.
#include "sv_batch_host.h"

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

#include "sv_guard.h"

namespace sv {
namespace batch {

namespace {
size_t align256_(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

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

// Runs of up to maxc consecutive single-qubit records on distinct qubits
// become one group (a header, then the members).  Within a pass list (after
// make_passes) only the gates inside each pass are grouped and the pass
// header's record count follows.
std::vector<BGate> group_run(const std::vector<BGate> &g, size_t a, size_t b, int maxc) {
  std::vector<BGate> out;
  size_t i = a;
  while (i < b) {
    size_t j = i;
    uint32_t used = 0;
    while (j < b && j - i < size_t(maxc) && g[j].kind == SV_BATCH_GATE_1Q && !((used >> g[j].q0) & 1u)) {
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
  if (!passes) return group_run(g, 0, g.size(), kMaxGroupLds);
  std::vector<BGate> out;
  size_t i = 0;
  while (i < g.size()) {
    const size_t cnt = size_t(g[i].q1);
    std::vector<BGate> merged = merge_cnots(g, i + 1, i + 1 + cnt);
    std::vector<BGate> body = group_run(merged, 0, merged.size(), kMaxGroupPass);
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

// Worker threads report each circuit's CircStatus; the calling thread
// turns the first failure into the error message.

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

}  // namespace batch
}  // namespace sv

using namespace sv;
using namespace sv::batch;

extern "C" {

size_t sv_batch_workspace_bytes(int count, const sv_batch_circuit *circs) {
  if (count < 0 || (count > 0 && !circs)) return 0;
  size_t ng = 0;  // at most one pass record and half a group record per gate on top of the gates
  for (int i = 0; i < count; ++i) ng += 3 * size_t(std::max(0, circs[i].n_gates));
  return 256 + align256_(sizeof(double) * size_t(std::max(1, count))) +
         align256_(sizeof(BItem) * size_t(std::max(1, count))) + align256_(sizeof(BGate) * std::max<size_t>(1, ng));
}

}  // extern "C"

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
