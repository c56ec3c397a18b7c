// Fusion planning on the host: greedy block formation and FP64 block products.
#include "sv_plan.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "sv_diagcover.h"
#include "sv_permute_host.h"
#include "sv_guard.h"
#include "sv_mlp.h"

namespace sv {
bool qubit_permutation(const double *G, int k, int *perm);
}

struct SvBlock {
  int k = 0;
  int ngates = 0;
  bool diag = true;
  std::vector<int32_t> tuple;    // ordered logical targets (ascending)
  std::vector<double> matrix;    // complex128 interleaved, 2^k x 2^k
  bool swap = false;             // a layout-swap block: no matrix, tuple[j] goes to physical bit dest[j]
  std::vector<int32_t> dest;
};

struct sv_plan {
  int n = 0;
  std::vector<SvBlock> blocks;
};

namespace {

struct GateView {
  int k;
  const int32_t *t;
  const double *m;
  bool diag;       // eligible for the streaming diagonal lowering: matrix exactly diagonal
  int weight = 1;  // input gates this view stands for (a block of an earlier round)
  const double *dtab = nullptr;  // a diagonal view of a later round: its 2^k diagonal entries (m is null)
};

// Diagonal entry r of a diagonal view, complex128.
inline void diag_entry(const GateView &g, int r, double *re, double *im) {
  if (g.m) {
    const int d = 1 << g.k;
    *re = g.m[2 * (size_t(r) * d + r)];
    *im = g.m[2 * (size_t(r) * d + r) + 1];
  } else {
    *re = g.dtab[2 * r];
    *im = g.dtab[2 * r + 1];
  }
}

// The diagonal of a run of diagonal gates, built one gate at a time: bit j
// of the table index is qubit q[j] (first-seen order); a gate's entries
// multiply the table (diagonal operators commute, so the order of the gates
// does not matter beyond rounding).
struct SpanDiag {
  int k = 0;
  int32_t q[8];
  double tab[2 * 256];
  void reset() {
    k = 0;
    tab[0] = 1.0;
    tab[1] = 0.0;
  }
  // false when the span would exceed 8 qubits (the table is then unchanged)
  bool add(const GateView &g) {
    int loc[8], fresh = 0;
    for (int j = 0; j < g.k; ++j) {
      loc[j] = -1;
      for (int b = 0; b < k; ++b)
        if (q[b] == g.t[j]) loc[j] = b;
      if (loc[j] < 0) ++fresh;
    }
    if (k + fresh > 8) return false;
    for (int j = 0; j < g.k; ++j) {
      if (loc[j] >= 0) continue;
      const int D = 1 << k;
      for (int x = 0; x < D; ++x) {  // the new qubit doubles the table
        tab[2 * (x + D)] = tab[2 * x];
        tab[2 * (x + D) + 1] = tab[2 * x + 1];
      }
      q[k] = g.t[j];
      loc[j] = k++;
    }
    const int D = 1 << k;
    for (int x = 0; x < D; ++x) {
      int r = 0;
      for (int j = 0; j < g.k; ++j) r |= ((x >> loc[j]) & 1) << j;
      double gr, gi;
      diag_entry(g, r, &gr, &gi);
      const double ar = tab[2 * x], ai = tab[2 * x + 1];
      tab[2 * x] = ar * gr - ai * gi;
      tab[2 * x + 1] = ar * gi + ai * gr;
    }
    return true;
  }
};

// What the streaming lowering sweeps for a diagonal block on physical
// positions A (table index bit j <-> A[j]): the fraction of the state its
// exact subcube cover visits and the number of launches (0 for an identity).
struct DiagCost {
  double fraction = 1.0;
  int launches = 1;
};

inline DiagCost diag_sweep_cost(int k, const double *tab, const int32_t *A) {
  const sv::DiagCover cv = sv::diag_cover(k, tab, A);
  DiagCost c;
  c.launches = cv.nsub;
  c.fraction = 0.0;
  for (int i = 0; i < cv.nsub; ++i) c.fraction += std::ldexp(1.0, -__builtin_popcount(cv.mask[i]));
  return c;
}

bool is_diagonal(const double *m, int k) {
  const int d = 1 << k;
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c)
      if (r != c && (m[2 * (r * d + c)] != 0.0 || m[2 * (r * d + c) + 1] != 0.0)) return false;
  return true;
}

// M <- E(g) M, where E(g) is gate g embedded into the block's k-qubit space:
// each column of M is a k-qubit vector and g acts on the local positions of
// its targets inside the block tuple.
void left_multiply(std::vector<double> &M, int k, const GateView &g, const std::vector<int32_t> &tuple) {
  const int D = 1 << k;
  const int d = 1 << g.k;
  int loc[8];
  for (int j = 0; j < g.k; ++j)
    for (int b = 0; b < k; ++b)
      if (tuple[b] == g.t[j]) loc[j] = b;
  int gmask = 0;
  for (int j = 0; j < g.k; ++j) gmask |= 1 << loc[j];
  std::vector<double> in(2 * d), out(2 * d);
  for (int col = 0; col < D; ++col) {
    for (int rest = 0; rest < D; ++rest) {
      if (rest & gmask) continue;  // enumerate the non-target local bits once
      for (int c = 0; c < d; ++c) {
        int idx = rest;
        for (int j = 0; j < g.k; ++j)
          if ((c >> j) & 1) idx |= 1 << loc[j];
        in[2 * c] = M[2 * (size_t(idx) * D + col)];
        in[2 * c + 1] = M[2 * (size_t(idx) * D + col) + 1];
      }
      for (int r = 0; r < d; ++r) {
        double re = 0, im = 0;
        for (int c = 0; c < d; ++c) {
          const double gr = g.m[2 * (r * d + c)], gi = g.m[2 * (r * d + c) + 1];
          re += gr * in[2 * c] - gi * in[2 * c + 1];
          im += gr * in[2 * c + 1] + gi * in[2 * c];
        }
        out[2 * r] = re;
        out[2 * r + 1] = im;
      }
      for (int r = 0; r < d; ++r) {
        int idx = rest;
        for (int j = 0; j < g.k; ++j)
          if ((r >> j) & 1) idx |= 1 << loc[j];
        M[2 * (size_t(idx) * D + col)] = out[2 * r];
        M[2 * (size_t(idx) * D + col) + 1] = out[2 * r + 1];
      }
    }
  }
}

SvBlock make_block(const std::vector<GateView> &gates) {
  SvBlock b;
  for (const auto &g : gates)
    for (int j = 0; j < g.k; ++j)
      if (std::find(b.tuple.begin(), b.tuple.end(), g.t[j]) == b.tuple.end()) b.tuple.push_back(g.t[j]);
  std::sort(b.tuple.begin(), b.tuple.end());
  b.k = int(b.tuple.size());
  b.ngates = 0;
  for (const auto &g : gates) b.ngates += g.weight;
  const int D = 1 << b.k;
  b.matrix.assign(size_t(2) * D * D, 0.0);
  for (int i = 0; i < D; ++i) b.matrix[2 * (size_t(i) * D + i)] = 1.0;
  for (const auto &g : gates) {
    b.diag = b.diag && g.diag;
    left_multiply(b.matrix, b.k, g, b.tuple);
  }
  return b;
}

bool parse_gates(int n, int ngates, const int32_t *ks, const int32_t *targets, const double *mats,
                 const int8_t *diag, std::vector<GateView> *out) {
  size_t toff = 0, moff = 0;
  for (int i = 0; i < ngates; ++i) {
    const int k = ks[i];
    if (k < 1 || k > 8 || k > n) return false;
    const int32_t *t = targets + toff;
    for (int j = 0; j < k; ++j) {
      if (t[j] < 0 || t[j] >= n) return false;
      for (int a = 0; a < j; ++a)
        if (t[a] == t[j]) return false;
    }
    // the marker is conservative: a gate is diagonal when its matrix is; a
    // caller flag that claims a non-diagonal matrix is an error
    const bool d = is_diagonal(mats + moff, k);
    if (diag && diag[i] != 0 && !d) return false;
    out->push_back(GateView{k, t, mats + moff, d, 1});
    toff += size_t(k);
    moff += size_t(2) << (2 * k);
  }
  return true;
}

}  // namespace

extern "C" {

int sv_plan_greedy(int n, int ngates, const int32_t *ks, const int32_t *targets, const double *mats,
                   const int8_t *diag, int k_max, sv_plan **out) {
  return sv::guard([&]() -> int {
    if (!out || (ngates > 0 && (!ks || !targets || !mats)) || ngates < 0 || k_max < 1 || k_max > 8 ||
        n < SV_MIN_QUBITS || n > SV_MAX_QUBITS) {
      sv::set_error("bad planner argument");
      return SV_ERR_ARG;
    }
    std::vector<GateView> gates;
    if (!parse_gates(n, ngates, ks, targets, mats, diag, &gates)) {
      sv::set_error("bad gate in list");
      return SV_ERR_ARG;
    }
    sv_plan *p = new sv_plan();
    p->n = n;
    std::vector<GateView> cur;
    std::vector<int32_t> cur_set;
    auto flush = [&]() {
      if (!cur.empty()) p->blocks.push_back(make_block(cur));
      cur.clear();
      cur_set.clear();
    };
    for (const auto &g : gates) {
      if (g.k > k_max) {
        flush();
        cur.push_back(g);
        flush();
        continue;
      }
      std::vector<int32_t> u = cur_set;
      for (int j = 0; j < g.k; ++j)
        if (std::find(u.begin(), u.end(), g.t[j]) == u.end()) u.push_back(g.t[j]);
      if (int(u.size()) > k_max) {
        flush();
        u.assign(g.t, g.t + g.k);
      }
      cur.push_back(g);
      cur_set = u;
    }
    flush();
    *out = p;
    return SV_OK;
  });
}

int sv_plan_num_blocks(const sv_plan *p, int *out) {
  return sv::guard([&]() -> int {
    if (!p || !out) {
      sv::set_error("null pointer");
      return SV_ERR_ARG;
    }
    *out = int(p->blocks.size());
    return SV_OK;
  });
}

int sv_plan_block_info(const sv_plan *p, int i, int *k, int32_t *targets, int *ngates, int *diag) {
  return sv::guard([&]() -> int {
    if (!p || i < 0 || i >= int(p->blocks.size())) {
      sv::set_error("bad block index");
      return SV_ERR_ARG;
    }
    const SvBlock &b = p->blocks[size_t(i)];
    if (k) *k = b.k;
    if (targets)
      for (int j = 0; j < b.k; ++j) targets[j] = b.tuple[size_t(j)];
    if (ngates) *ngates = b.ngates;
    if (diag) *diag = b.diag ? 1 : 0;
    return SV_OK;
  });
}

int sv_plan_block_matrix(const sv_plan *p, int i, double *out) {
  return sv::guard([&]() -> int {
    if (!p || !out || i < 0 || i >= int(p->blocks.size())) {
      sv::set_error("bad block index");
      return SV_ERR_ARG;
    }
    const SvBlock &b = p->blocks[size_t(i)];
    if (b.swap) {
      sv::set_error("a layout-swap block has no matrix");
      return SV_ERR_ARG;
    }
    std::memcpy(out, b.matrix.data(), b.matrix.size() * sizeof(double));
    return SV_OK;
  });
}

int sv_plan_block_swap(const sv_plan *p, int i, int *is_swap, int32_t *dest) {
  return sv::guard([&]() -> int {
    if (!p || !is_swap || i < 0 || i >= int(p->blocks.size())) {
      sv::set_error("bad block index");
      return SV_ERR_ARG;
    }
    const SvBlock &b = p->blocks[size_t(i)];
    *is_swap = b.swap ? 1 : 0;
    if (b.swap && dest)
      for (int j = 0; j < b.k; ++j) dest[j] = b.dest[size_t(j)];
    return SV_OK;
  });
}

int sv_run_plan(sv_state *s, const sv_plan *p) {
  return sv::guard([&]() -> int {
    if (!s || !p) {
      sv::set_error("null pointer");
      return SV_ERR_ARG;
    }
    // next use of every logical qubit after each block: the relabel policy's
    // view of the future (Corollary 1)
    const size_t nb = p->blocks.size();
    std::vector<int64_t> next(size_t(p->n), INT64_MAX);
    std::vector<std::vector<int64_t>> hints(nb);
    for (size_t i = nb; i-- > 0;) {
      hints[i] = next;
      if (!p->blocks[i].swap)
        for (int32_t q : p->blocks[i].tuple) next[size_t(q)] = int64_t(i);
    }
    for (size_t i = 0; i < nb; ++i) {
      const SvBlock &b = p->blocks[i];
      int rc;
      if (b.swap) {
        // each listed qubit to its physical bit, the occupant to its old place
        std::vector<int32_t> L(static_cast<size_t>(p->n)), Linv(static_cast<size_t>(p->n));
        rc = sv_get_layout(s, L.data());
        if (rc) return rc;
        for (int q = 0; q < p->n; ++q) Linv[size_t(L[size_t(q)])] = q;
        for (int j = 0; j < b.k; ++j) {
          const int32_t q = b.tuple[size_t(j)], to = b.dest[size_t(j)], from = L[size_t(q)];
          if (from == to) continue;
          const int32_t r = Linv[size_t(to)];
          L[size_t(q)] = to;
          L[size_t(r)] = from;
          Linv[size_t(to)] = q;
          Linv[size_t(from)] = r;
        }
        rc = sv_permute_layout(s, L.data());
        if (rc) return rc;
        continue;
      }
      rc = sv_hint_next_use(s, hints[i].data());
      if (rc) return rc;
      rc = sv_apply_fused(s, b.matrix.data(), b.tuple.data(), b.k);
      if (rc) return rc;
    }
    return SV_OK;
  });
}

int sv_plan_free(sv_plan *p) {
  return sv::guard([&]() -> int {
    delete p;
    return SV_OK;
  });
}

int sv_cost_features(int n, int k, const int32_t *A, int diagonal, double swept_fraction, int launches,
                     float *out) {
  return sv::guard([&]() -> int {
    if (!A || !out || k < 1 || k > 7 || n < 1 || n > SV_MAX_QUBITS || !(swept_fraction >= 0.0) ||
        swept_fraction > 1.0 || launches < 0 || launches > 64) {
      sv::set_error("bad feature argument");
      return SV_ERR_ARG;
    }
    int s[7];
    for (int j = 0; j < k; ++j) s[j] = A[j];
    std::sort(s, s + k);
    out[0] = float(n) / 35.f;
    out[1] = float(k) / 8.f;
    for (int j = 0; j < 7; ++j) out[2 + j] = (j < k) ? float(s[j]) / 35.f : -0.25f;
    out[9] = diagonal ? 1.f : 0.f;
    out[10] = diagonal ? float(swept_fraction) : 1.f;
    out[11] = diagonal ? float(launches) / 16.f : 1.f / 16.f;
    return SV_OK;
  });
}

int sv_diag_sweep_cost(int k, const double *diag, const int32_t *A, double *fraction, int *launches) {
  return sv::guard([&]() -> int {
    if (!diag || !A || !fraction || !launches || k < 1 || k > 8) {
      sv::set_error("bad diagonal-cost argument");
      return SV_ERR_ARG;
    }
    for (int j = 0; j < k; ++j) {
      if (A[j] < 0 || A[j] >= 64) {
        sv::set_error("target position out of range");
        return SV_ERR_ARG;
      }
      for (int i = 0; i < j; ++i)
        if (A[i] == A[j]) {
          sv::set_error("duplicate target position");
          return SV_ERR_ARG;
        }
    }
    const DiagCost c = diag_sweep_cost(k, diag, A);
    *fraction = c.fraction;
    *launches = c.launches;
    return SV_OK;
  });
}

}  // extern "C"

namespace {

// Block cost Gamma for the DP.  dc: what a diagonal block's sweeps visit
// (null: one full sweep).
struct Scorer {
  int score;
  int n;
  const float *params;
  int nin, hid;
  std::map<std::vector<int32_t>, double> cache;  // (sorted targets..., diag, cover) -> Gamma

  double operator()(const std::vector<int32_t> &tuple_sorted, bool all_diag, const DiagCost *dc = nullptr) {
    const int k = int(tuple_sorted.size());
    if (score == SV_SCORE_PAPER) return all_diag ? 1.0 : std::ldexp(1.0, 2 * k);
    DiagCost full;
    const DiagCost &c = (all_diag && dc) ? *dc : full;
    if (all_diag && c.launches == 0) return 0.0;  // the product is the identity: nothing runs
    if (score == SV_SCORE_ROOFLINE) return roofline_ms(k, all_diag, c);
    if (k > 7) return 1e30;
    std::vector<int32_t> key(tuple_sorted);
    key.push_back(all_diag ? 1 : 0);
    if (all_diag) {
      key.push_back(int32_t(std::lround(c.fraction * 65536.0)));
      key.push_back(c.launches);
    }
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    float f[SV_MLP_FEATURES];
    sv_cost_features(n, k, tuple_sorted.data(), all_diag ? 1 : 0, c.fraction, c.launches, f);
    double y = 0;
    sv_mlp_forward_host(params, nin, hid, f, 1, &y);
    // the model predicts log(ms) at N = 30 scale; a sweep's time grows as 2^N
    const double g = std::exp(y + (n - 30) * std::log(2.0));
    cache.emplace(std::move(key), g);
    return g;
  }

  // The analytic score: a sweep's time at MI355X's peaks, the larger of its
  // HBM time (16 B per amplitude visited, 8 TB/s) and its arithmetic time
  // (complex multiply-adds of the kernel that runs it: 8 * 2^k flops per
  // amplitude on the vector ALU at 78.6 TFLOP/s without packed FP32 for
  // k <= 3, on FP32 MFMA at 157.3 TFLOP/s for k = 4, the three-product
  // complex form 6 * 2^k for 5 <= k <= 7); a diagonal block costs the
  // fraction of the state its cover visits plus kDiagLaunchCost of a sweep
  // per launch.  In ms.
  double roofline_ms(int k, bool all_diag, const DiagCost &c) const {
    const double amps = std::ldexp(1.0, n);
    const double sweep = 16.0 * amps / 8e12 * 1e3;
    if (all_diag) return sweep * (c.fraction + double(c.launches) * sv::kDiagLaunchCost);
    double flops, peak;
    if (k <= 3) {
      flops = 8.0 * std::ldexp(1.0, k);
      peak = 78.6e12;
    } else if (k == 4) {
      flops = 8.0 * 16.0;
      peak = 157.3e12;
    } else if (k <= 7) {
      flops = 6.0 * std::ldexp(1.0, k);
      peak = 157.3e12;
    } else {
      flops = 8.0 * std::ldexp(1.0, k);
      peak = 78.6e12;
    }
    return std::max(sweep, flops * amps / peak * 1e3);
  }
};

// Cost of gates [a, b) as one block: its sorted tuple, diagonal flag and, for
// a diagonal block, what its cover sweeps (identity layout: physical
// position = logical qubit at planning time).
double span_cost(const std::vector<GateView> &gates, size_t a, size_t b, Scorer &gamma) {
  std::vector<int32_t> tuple;
  bool diag = true;
  for (size_t g = a; g < b; ++g) {
    for (int j = 0; j < gates[g].k; ++j)
      if (std::find(tuple.begin(), tuple.end(), gates[g].t[j]) == tuple.end()) tuple.push_back(gates[g].t[j]);
    diag = diag && gates[g].diag;
  }
  std::sort(tuple.begin(), tuple.end());
  if (!diag || gamma.score == SV_SCORE_PAPER || tuple.size() > 8) return gamma(tuple, diag);
  SpanDiag sd;
  sd.reset();
  for (size_t g = a; g < b; ++g) sd.add(gates[g]);
  const DiagCost dc = diag_sweep_cost(sd.k, sd.tab, sd.q);
  return gamma(tuple, true, &dc);
}

struct Span {
  size_t a, b;  // gates [a, b)
};

void span_info(const std::vector<GateView> &gates, size_t a, size_t b, std::vector<int32_t> *tuple, bool *diag) {
  tuple->clear();
  *diag = true;
  for (size_t g = a; g < b; ++g) {
    for (int j = 0; j < gates[g].k; ++j)
      if (std::find(tuple->begin(), tuple->end(), gates[g].t[j]) == tuple->end()) tuple->push_back(gates[g].t[j]);
    *diag = *diag && gates[g].diag;
  }
  std::sort(tuple->begin(), tuple->end());
}

// Commute-aware reorder (Section IV-C: a gate moves only across neighbours it
// commutes with; here, gates on disjoint qubits).  Any order that keeps each
// qubit's gate sequence is equivalent.  Clusters are grown from the dependency
// front: start with the earliest ready gate, then repeatedly take the ready
// gate whose qubits enlarge the cluster's set least (earliest on ties) while
// the set stays within `cap`; emit the cluster's gates consecutively.
std::vector<size_t> commute_order(const std::vector<GateView> &gates, int n, int cap) {
  const size_t G = gates.size();
  std::vector<std::vector<size_t>> per_q(static_cast<size_t>(n));
  for (size_t g = 0; g < G; ++g)
    for (int j = 0; j < gates[g].k; ++j) per_q[size_t(gates[g].t[j])].push_back(g);
  std::vector<size_t> head(size_t(n), 0);
  std::vector<bool> done(G, false);
  auto ready = [&](size_t g) {
    for (int j = 0; j < gates[g].k; ++j) {
      const size_t q = size_t(gates[g].t[j]);
      if (head[q] >= per_q[q].size() || per_q[q][head[q]] != g) return false;
    }
    return true;
  };
  auto take = [&](size_t g, std::vector<size_t> &out) {
    done[g] = true;
    out.push_back(g);
    for (int j = 0; j < gates[g].k; ++j) ++head[size_t(gates[g].t[j])];
  };
  std::vector<size_t> order;
  order.reserve(G);
  size_t first = 0;
  while (order.size() < G) {
    while (done[first]) ++first;
    // the earliest unscheduled gate is always ready: its predecessors are earlier
    std::vector<int32_t> set(gates[first].t, gates[first].t + gates[first].k);
    take(first, order);
    while (true) {
      size_t best = G;
      int best_w = 1 << 30;
      // candidates: the head gate of every qubit (ready gates are heads of all their qubits)
      for (int q = 0; q < n; ++q) {
        if (head[size_t(q)] >= per_q[size_t(q)].size()) continue;
        const size_t g = per_q[size_t(q)][head[size_t(q)]];
        if (done[g] || !ready(g)) continue;
        int w = int(set.size());
        for (int j = 0; j < gates[g].k; ++j)
          if (std::find(set.begin(), set.end(), gates[g].t[j]) == set.end()) ++w;
        if (w > cap && gates[g].k <= cap) continue;
        if (w > cap) continue;
        if (w < best_w || (w == best_w && g < best)) {
          best_w = w;
          best = g;
        }
      }
      if (best == G) break;
      for (int j = 0; j < gates[best].k; ++j)
        if (std::find(set.begin(), set.end(), gates[best].t[j]) == set.end()) set.push_back(gates[best].t[j]);
      take(best, order);
    }
  }
  return order;
}

}  // namespace

namespace {

// One reorder-and-fuse pass over `views`: the optional commute-aware reorder,
// the windowed DP (Eq. dp-recurrence) and the cross-window greedy merge.
// Returns the partition as lists of view indices in application order and
// the total score.  Views of later rounds carry no matrix: only k, targets,
// the diagonal marker and the weight are read here.
std::vector<std::vector<size_t>> dp_pass(int n, const std::vector<GateView> &views, int k_max, int diag_max,
                                         int window, int flags, Scorer &gamma, double *predicted) {
  std::vector<size_t> order(views.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  if (flags & SV_PLAN_REORDER) order = commute_order(views, n, std::max(k_max, diag_max));
  std::vector<GateView> gates;
  gates.reserve(order.size());
  for (size_t g : order) gates.push_back(views[g]);
  const int cap_any = std::max(k_max, diag_max);
  std::vector<Span> spans;
  for (size_t w0 = 0; w0 < gates.size(); w0 += size_t(window)) {
    const size_t h = std::min(size_t(window), gates.size() - w0);
    std::vector<double> D(h + 1, 0.0);
    std::vector<size_t> arg(h + 1, 0);
    for (size_t i = 1; i <= h; ++i) {
      double best = 1e300;
      size_t bj = i - 1;
      std::vector<int32_t> set;
      bool all_diag = true;
      const bool need_cover = gamma.score != SV_SCORE_PAPER;
      bool have_tab = need_cover;
      SpanDiag sd;
      sd.reset();
      for (size_t j = i; j-- > 0;) {
        const GateView &g = gates[w0 + j];
        for (int q = 0; q < g.k; ++q)
          if (std::find(set.begin(), set.end(), g.t[q]) == set.end()) set.push_back(g.t[q]);
        all_diag = all_diag && g.diag;
        if (have_tab && (!all_diag || !sd.add(g))) have_tab = false;
        const int width = int(set.size());
        const int cap = all_diag ? diag_max : k_max;
        if (width <= cap || j == i - 1) {
          std::vector<int32_t> srt(set);
          std::sort(srt.begin(), srt.end());
          DiagCost dc;
          if (all_diag && have_tab) dc = diag_sweep_cost(sd.k, sd.tab, sd.q);
          const double c = D[j] + gamma(srt, all_diag, all_diag && have_tab ? &dc : nullptr);
          if (c < best) {
            best = c;
            bj = j;
          }
        }
        if (width > cap_any) break;
      }
      D[i] = best;
      arg[i] = bj;
    }
    std::vector<Span> win;
    for (size_t i = h; i > 0; i = arg[i]) win.push_back(Span{w0 + arg[i], w0 + i});
    std::reverse(win.begin(), win.end());
    spans.insert(spans.end(), win.begin(), win.end());
  }
  // cross-window greedy merge of adjacent blocks
  std::vector<Span> merged;
  for (const Span &sp : spans) {
    if (!merged.empty()) {
      Span &last = merged.back();
      std::vector<int32_t> tm;
      bool dm;
      span_info(gates, last.a, sp.b, &tm, &dm);
      const int cap = dm ? diag_max : k_max;
      if (int(tm.size()) <= cap &&
          span_cost(gates, last.a, sp.b, gamma) < span_cost(gates, last.a, last.b, gamma) + span_cost(gates, sp.a, sp.b, gamma)) {
        last.b = sp.b;
        continue;
      }
    }
    merged.push_back(sp);
  }
  std::vector<std::vector<size_t>> out;
  out.reserve(merged.size());
  double total = 0;
  for (const Span &sp : merged) {
    total += span_cost(gates, sp.a, sp.b, gamma);
    std::vector<size_t> m;
    for (size_t i = sp.a; i < sp.b; ++i) m.push_back(order[i]);
    out.push_back(std::move(m));
  }
  *predicted = total;
  return out;
}

// A partition of the input gates: each block lists input indices in application order.
struct Partition {
  std::vector<std::vector<size_t>> blocks;
  double predicted = 0;
};

// The pipeline, and with SV_PLAN_REPEAT up to three more rounds whose views
// are the previous round's blocks (Section IV-C: at most four rounds,
// stopping when the block count no longer decreases).  Every round's DP may
// keep each block of the previous round as a singleton, so the score never
// rises from round to round.
Partition dp_rounds(int n, const std::vector<GateView> &gates, int k_max, int diag_max, int window, int flags,
                    Scorer &gamma) {
  std::vector<GateView> views(gates);
  std::vector<std::vector<size_t>> members(gates.size());
  for (size_t i = 0; i < gates.size(); ++i) members[i] = {i};
  std::vector<std::vector<int32_t>> tuples;  // target storage of the current round's views
  std::vector<std::vector<double>> dtabs;    // diagonal tables of the current round's diagonal views
  Partition best;
  const int rounds = (flags & SV_PLAN_REPEAT) ? 4 : 1;
  for (int r = 0; r < rounds; ++r) {
    double t = 0;
    const std::vector<std::vector<size_t>> part = dp_pass(n, views, k_max, diag_max, window, flags, gamma, &t);
    if (r > 0 && part.size() >= views.size()) break;
    std::vector<std::vector<size_t>> next_members;
    next_members.reserve(part.size());
    for (const auto &blk : part) {
      std::vector<size_t> m;
      for (size_t v : blk) m.insert(m.end(), members[v].begin(), members[v].end());
      next_members.push_back(std::move(m));
    }
    best.blocks = next_members;
    best.predicted = t;
    if (r + 1 == rounds) break;
    std::vector<std::vector<int32_t>> next_tuples(part.size());
    std::vector<std::vector<double>> next_dtabs(part.size());
    std::vector<GateView> next_views;
    next_views.reserve(part.size());
    for (size_t b = 0; b < part.size(); ++b) {
      bool dg = true;
      int w = 0;
      for (size_t v : part[b]) {
        for (int j = 0; j < views[v].k; ++j)
          if (std::find(next_tuples[b].begin(), next_tuples[b].end(), views[v].t[j]) == next_tuples[b].end())
            next_tuples[b].push_back(views[v].t[j]);
        dg = dg && views[v].diag;
        w += views[v].weight;
      }
      std::sort(next_tuples[b].begin(), next_tuples[b].end());
      const double *dt = nullptr;
      if (dg && next_tuples[b].size() <= 8) {
        // the block's diagonal over its sorted tuple, for the next round's cover costs
        SpanDiag sd;
        sd.reset();
        for (int32_t q : next_tuples[b]) {  // fix the table's bit order to the sorted tuple
          const double one[4] = {1.0, 0.0, 1.0, 0.0};
          sd.add(GateView{1, &q, nullptr, true, 0, one});
        }
        for (size_t v : part[b]) sd.add(views[v]);
        next_dtabs[b].assign(sd.tab, sd.tab + 2 * (size_t(1) << sd.k));
        dt = next_dtabs[b].data();
      }
      next_views.push_back(GateView{int(next_tuples[b].size()), next_tuples[b].data(), nullptr, dg, w, dt});
    }
    tuples = std::move(next_tuples);  // the inner buffers (and the views' pointers) stay where they are
    dtabs = std::move(next_dtabs);
    views = std::move(next_views);
    members = std::move(next_members);
  }
  return best;
}

sv_plan *build_plan(int n, const std::vector<GateView> &gates, const Partition &part) {
  sv_plan *p = new sv_plan();
  p->n = n;
  p->blocks.reserve(part.blocks.size());
  for (const auto &blk : part.blocks) {
    std::vector<GateView> seg;
    seg.reserve(blk.size());
    for (size_t g : blk) seg.push_back(gates[g]);
    p->blocks.push_back(make_block(seg));
  }
  return p;
}
}  // namespace

extern "C" int sv_plan_dp(int n, int ngates, const int32_t *ks, const int32_t *targets, const double *mats,
                          const int8_t *diag, int k_max, int diag_max, int window, int score,
                          const float *mlp_params, int mlp_nin, int mlp_hid, int flags, sv_plan **out) {
  return sv::guard([&]() -> int {
    if (!out || ngates < 0 || (ngates > 0 && (!ks || !targets || !mats)) || k_max < 1 || k_max > 8 ||
        diag_max < 1 || diag_max > 8 || window < 1 || n < SV_MIN_QUBITS || n > SV_MAX_QUBITS ||
        (score != SV_SCORE_PAPER && score != SV_SCORE_LEARNED && score != SV_SCORE_ROOFLINE) ||
        (score == SV_SCORE_LEARNED && (!mlp_params || mlp_nin != SV_MLP_FEATURES || mlp_hid < 1))) {
      sv::set_error("bad dp planner argument");
      return SV_ERR_ARG;
    }
    std::vector<GateView> gates;
    if (!parse_gates(n, ngates, ks, targets, mats, diag, &gates)) {
      sv::set_error("bad gate in list");
      return SV_ERR_ARG;
    }
    Scorer gamma{score, n, mlp_params, mlp_nin, mlp_hid, {}};  // one cache for every pass
    if ((flags & SV_PLAN_SEARCH_CAP) && score != SV_SCORE_PAPER) {
      // The cost model also picks the caps: plan with every dense cap c up to
      // k_max, with the diagonal cap at min(c, diag_max) and at diag_max
      // (diagonal blocks stream at one sweep's cost whatever their width, but
      // the reorder grows clusters up to the larger cap, which changes the
      // order), and keep the partition of least predicted time.  Products are
      // formed for the chosen partition only.
      Partition best;
      best.predicted = 1e300;
      for (int cap = std::min(4, k_max); cap <= k_max; ++cap) {
        const int lo = std::min(cap, diag_max);
        for (int dcap : {lo, diag_max}) {
          Partition part = dp_rounds(n, gates, cap, dcap, window, flags, gamma);
          if (part.predicted < best.predicted) best = std::move(part);
          if (diag_max == lo) break;
        }
      }
      *out = build_plan(n, gates, best);
      return SV_OK;
    }
    *out = build_plan(n, gates, dp_rounds(n, gates, k_max, diag_max, window, flags, gamma));
    return SV_OK;
  });
}

// ------------------------------------------------------------------ layout swaps chosen by the cost model
namespace {

// Apply a block that only permutes qubits to a layout, as sv_apply_fused
// does: L'(t[perm[j]]) = L(t[j]).
bool absorb_permutation(const SvBlock &b, std::vector<int32_t> *L) {
  if (b.swap || b.k > SV_MAX_K) return false;
  int perm[SV_MAX_K];
  if (!sv::qubit_permutation(b.matrix.data(), b.k, perm)) return false;
  int32_t old[SV_MAX_K];
  for (int j = 0; j < b.k; ++j) old[j] = (*L)[size_t(b.tuple[size_t(j)])];
  for (int j = 0; j < b.k; ++j) (*L)[size_t(b.tuple[size_t(perm[j])])] = old[j];
  return true;
}

// The layout after moving the logical qubits `tuple` onto physical bits
// s0 .. s0+k-1: targets already there stay; each other target, in order of
// its current position, exchanges places with the qubit on the lowest free
// window bit.  *moves = the exchanges made.
std::vector<int32_t> move_onto(const std::vector<int32_t> &L, const std::vector<int32_t> &tuple, int s0,
                               int *moves) {
  const int n = int(L.size()), k = int(tuple.size());
  std::vector<int32_t> L2(L), Linv(static_cast<size_t>(n));
  for (int q = 0; q < n; ++q) Linv[size_t(L2[size_t(q)])] = q;
  std::vector<char> is_target(static_cast<size_t>(n), 0);
  for (int32_t q : tuple) is_target[size_t(q)] = 1;
  std::vector<int32_t> movers, free_bits;
  for (int32_t q : tuple)
    if (L2[size_t(q)] < s0 || L2[size_t(q)] >= s0 + k) movers.push_back(q);
  std::sort(movers.begin(), movers.end(), [&](int32_t a, int32_t b) { return L2[size_t(a)] < L2[size_t(b)]; });
  for (int p = s0; p < s0 + k; ++p)
    if (!is_target[size_t(Linv[size_t(p)])]) free_bits.push_back(p);
  for (size_t j = 0; j < movers.size(); ++j) {
    const int32_t q = movers[j], to = free_bits[j], from = L2[size_t(q)], r = Linv[size_t(to)];
    L2[size_t(q)] = to;
    L2[size_t(r)] = from;
    Linv[size_t(to)] = q;
    Linv[size_t(from)] = r;
  }
  *moves = int(movers.size());
  return L2;
}

}  // namespace

extern "C" int sv_plan_swaps(sv_plan *p, const float *mlp_params, int mlp_nin, int mlp_hid, int horizon,
                             double margin, int *inserted) {
  return sv::guard([&]() -> int {
    if (!p || !mlp_params || mlp_nin != SV_MLP_FEATURES || mlp_hid < 1 || horizon < 1 || margin < 0) {
      sv::set_error("bad swap-pass argument");
      return SV_ERR_ARG;
    }
    if (inserted) *inserted = 0;
    const int n = p->n;
    if (n < SV_PLAN_SWAP_MIN_QUBITS) return SV_OK;
    Scorer gamma{SV_SCORE_LEARNED, n, mlp_params, mlp_nin, mlp_hid, {}};
    auto cost = [&](const SvBlock &b, const std::vector<int32_t> &L) {
      std::vector<int32_t> ph;
      for (int32_t q : b.tuple) ph.push_back(L[size_t(q)]);
      std::sort(ph.begin(), ph.end());
      return gamma(ph, b.diag);
    };
    const double stream = gamma(std::vector<int32_t>{0}, true);  // one streaming sweep
    std::vector<int32_t> L(static_cast<size_t>(n));
    for (int q = 0; q < n; ++q) L[size_t(q)] = q;
    std::vector<SvBlock> out;
    const size_t nb = p->blocks.size();
    int added = 0;
    for (size_t i = 0; i < nb; ++i) {
      const SvBlock &b = p->blocks[i];
      std::vector<int32_t> Lperm(L);
      const bool permutes = absorb_permutation(b, &Lperm);
      if (!b.swap && !b.diag && !permutes && b.k <= 7) {
        double best = 0.0;
        std::vector<int32_t> bestL;
        for (int s0 = 0; s0 + b.k <= n; ++s0) {
          int moves = 0;
          std::vector<int32_t> L2 = move_onto(L, b.tuple, s0, &moves);
          if (moves == 0) continue;
          // the next `horizon` blocks at their positions under both layouts
          std::vector<int32_t> La(L), Lb(L2);
          double gain = 0.0;
          for (size_t j = i; j < nb && j < i + size_t(horizon); ++j) {
            const SvBlock &c = p->blocks[j];
            if (c.swap) break;
            if (absorb_permutation(c, &La)) {
              absorb_permutation(c, &Lb);
              continue;
            }
            if (!c.diag) gain += cost(c, La) - cost(c, Lb);
          }
          // the tile passes sv_permute_layout will run for this move
          const double price =
              double(sv::permutation_passes(L.data(), L2.data(), n)) * stream * SV_PLAN_SWAP_SWEEP_FACTOR;
          if (gain > price * (1.0 + margin) && gain - price > best) {
            best = gain - price;
            bestL = std::move(L2);
          }
        }
        if (!bestL.empty()) {
          SvBlock sw;
          sw.swap = true;
          sw.ngates = 0;
          sw.diag = false;
          for (int q = 0; q < n; ++q)
            if (bestL[size_t(q)] != L[size_t(q)]) {
              sw.tuple.push_back(q);
              sw.dest.push_back(bestL[size_t(q)]);
            }
          sw.k = int(sw.tuple.size());
          out.push_back(std::move(sw));
          L = bestL;
          Lperm = L;
          absorb_permutation(b, &Lperm);
          ++added;
        }
      }
      out.push_back(b);
      L = Lperm;
    }
    p->blocks = std::move(out);
    if (inserted) *inserted = added;
    return SV_OK;
  });
}
