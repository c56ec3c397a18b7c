// Host code of libsv under the compiler's sanitizers (no GPU): the fusion
// planners (greedy, windowed DP on every score, cap search, repeated rounds,
// layout-swap pass), the diagonal cover, the batched path's host pass (the
// threaded packing included) and the host MLP forward, on seeded random
// inputs and on bad arguments.  Built with g++ from the library's plain C++
// sources (-fsanitize=address,undefined, or thread); the device entry points
// the planner's sv_run_plan would call are stubbed.  Exits 0 when every
// check holds; a sanitizer report aborts the run.
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <new>
#include <vector>

#include "sv.h"
#include "sv_batch.h"
#include "sv_batch_host.h"
#include "sv_diagcover.h"
#include "sv_mlp.h"
#include "sv_plan.h"
#include "sv_permute_host.h"

// ------------------------------------------------------------------ stubs
extern "C" int sv_apply_fused(sv_state *, const double *, const int32_t *, int) { return SV_ERR_UNSUPPORTED; }
extern "C" int sv_permute_layout(sv_state *, const int32_t *) { return SV_ERR_UNSUPPORTED; }
extern "C" int sv_get_layout(const sv_state *, int32_t *) { return SV_ERR_UNSUPPORTED; }
extern "C" int sv_hint_next_use(sv_state *, const int64_t *) { return SV_ERR_UNSUPPORTED; }

// ------------------------------------------------------------------ allocation counter
static std::atomic<long> g_allocs{0};
void *operator new(size_t n) {
  g_allocs.fetch_add(1, std::memory_order_relaxed);
  if (void *p = std::malloc(n ? n : 1)) return p;
  throw std::bad_alloc();
}
void *operator new[](size_t n) { return operator new(n); }
void *operator new(size_t n, const std::nothrow_t &) noexcept {
  g_allocs.fetch_add(1, std::memory_order_relaxed);
  return std::malloc(n ? n : 1);
}
void *operator new[](size_t n, const std::nothrow_t &) noexcept { return operator new(n, std::nothrow); }
void operator delete(void *p, const std::nothrow_t &) noexcept { std::free(p); }
void operator delete[](void *p, const std::nothrow_t &) noexcept { std::free(p); }
void operator delete(void *p) noexcept { std::free(p); }
void operator delete[](void *p) noexcept { std::free(p); }
void operator delete(void *p, size_t) noexcept { std::free(p); }
void operator delete[](void *p, size_t) noexcept { std::free(p); }

// ------------------------------------------------------------------ helpers
static int g_fail = 0;
#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      ++g_fail;                                                     \
    }                                                               \
  } while (0)

struct Rng {  // SplitMix64
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  int below(int m) { return int(next() % uint64_t(m)); }
  double unit() { return double(next() >> 11) * (1.0 / 9007199254740992.0); }
};

struct Circuit {
  std::vector<int32_t> ks, targets;
  std::vector<double> mats;
  std::vector<int8_t> diag;
};

// k-qubit gates on distinct random qubits: dense, diagonal phases, controlled phases
static Circuit random_circuit(Rng &r, int n, int ngates, int kmax) {
  Circuit c;
  for (int i = 0; i < ngates; ++i) {
    const int k = 1 + r.below(std::min(kmax, n));
    std::vector<int32_t> t;
    while (int(t.size()) < k) {
      const int q = r.below(n);
      bool dup = false;
      for (int x : t) dup = dup || x == q;
      if (!dup) t.push_back(q);
    }
    const int kind = r.below(3);
    const int D = 1 << k;
    for (int row = 0; row < D; ++row)
      for (int col = 0; col < D; ++col) {
        double re = 0, im = 0;
        if (kind == 0) {
          re = r.unit() - 0.5;
          im = r.unit() - 0.5;
        } else if (row == col) {
          const bool ctl = kind == 2 && row != D - 1;
          const double ph = 6.283185307179586 * r.unit();
          re = ctl ? 1.0 : std::cos(ph);
          im = ctl ? 0.0 : std::sin(ph);
        }
        c.mats.push_back(re);
        c.mats.push_back(im);
      }
    c.ks.push_back(k);
    c.targets.insert(c.targets.end(), t.begin(), t.end());
    c.diag.push_back(kind != 0 ? 1 : 0);
  }
  return c;
}

static void check_plan(sv_plan *p, int ngates) {
  int nb = -1;
  CHECK(sv_plan_num_blocks(p, &nb) == SV_OK && nb >= 0);
  int total = 0;
  for (int i = 0; i < nb; ++i) {
    int k = 0, ng = 0, dg = 0, sw = 0;
    CHECK(sv_plan_block_info(p, i, &k, nullptr, &ng, &dg) == SV_OK);
    std::vector<int32_t> t(static_cast<size_t>(std::max(k, 1)));
    CHECK(sv_plan_block_info(p, i, &k, t.data(), &ng, &dg) == SV_OK);
    CHECK(sv_plan_block_swap(p, i, &sw, nullptr) == SV_OK);
    if (!sw) {
      std::vector<double> m(size_t(2) << (2 * k));
      CHECK(sv_plan_block_matrix(p, i, m.data()) == SV_OK);
      total += ng;
    } else {
      std::vector<int32_t> dest(static_cast<size_t>(k));
      CHECK(sv_plan_block_swap(p, i, &sw, dest.data()) == SV_OK);
      CHECK(sv_plan_block_matrix(p, i, nullptr) == SV_ERR_ARG);
    }
  }
  CHECK(total == ngates);
  int k = 0;
  CHECK(sv_plan_block_info(p, nb, &k, nullptr, nullptr, nullptr) == SV_ERR_ARG);
}

static std::vector<float> random_params(Rng &r, int nin, int hid) {
  std::vector<float> p(size_t(sv_mlp_param_count(nin, hid)));
  for (auto &x : p) x = float(r.unit() - 0.5) * 0.3f;
  return p;
}

// ------------------------------------------------------------------ checks
static void planners(Rng &r) {
  const int nin = SV_MLP_FEATURES, hid = 16;
  for (int trial = 0; trial < 24; ++trial) {
    const int n = 2 + r.below(30);
    const int ng = r.below(90);
    Circuit c = random_circuit(r, n, ng, 4);
    const int32_t *ks = c.ks.data(), *tg = c.targets.data();
    const double *mt = c.mats.data();
    const int8_t *dg = c.diag.data();
    sv_plan *p = nullptr;
    CHECK(sv_plan_greedy(n, ng, ks, tg, mt, dg, 1 + r.below(7), &p) == SV_OK);
    check_plan(p, ng);
    CHECK(sv_plan_free(p) == SV_OK);
    std::vector<float> prm = random_params(r, nin, hid);
    for (int score = SV_SCORE_PAPER; score <= SV_SCORE_ROOFLINE; ++score)
      for (int flags = 0; flags < 8; ++flags) {
        const int kmax = 1 + r.below(7), dmax = 1 + r.below(8), window = 1 + r.below(70);
        p = nullptr;
        const int rc = sv_plan_dp(n, ng, ks, tg, mt, dg, kmax, dmax, window, score,
                                  score == SV_SCORE_LEARNED ? prm.data() : nullptr, nin, hid, flags, &p);
        CHECK(rc == SV_OK);
        if (rc != SV_OK) continue;
        check_plan(p, ng);
        if (score == SV_SCORE_LEARNED && n >= SV_PLAN_SWAP_MIN_QUBITS) {
          int ins = -1;
          CHECK(sv_plan_swaps(p, prm.data(), nin, hid, 1 + r.below(40), 0.1 * r.below(5), &ins) == SV_OK);
          check_plan(p, ng);
        }
        CHECK(sv_plan_free(p) == SV_OK);
      }
  }
  // bad arguments
  sv_plan *p = nullptr;
  int32_t k1 = 1, t_bad = 40;
  double m1[8] = {1, 0, 0, 0, 0, 0, 1, 0};
  CHECK(sv_plan_greedy(10, 1, &k1, &t_bad, m1, nullptr, 4, &p) == SV_ERR_ARG);
  CHECK(sv_plan_dp(10, 0, nullptr, nullptr, nullptr, nullptr, 4, 4, 0, SV_SCORE_PAPER, nullptr, 0, 0, 0, &p) ==
        SV_ERR_ARG);
  CHECK(sv_plan_dp(10, 0, nullptr, nullptr, nullptr, nullptr, 4, 4, 8, SV_SCORE_LEARNED, nullptr, 12, 16, 0, &p) ==
        SV_ERR_ARG);
  CHECK(sv_plan_dp(10, 0, nullptr, nullptr, nullptr, nullptr, 4, 4, 8, 7, nullptr, 0, 0, 0, &p) == SV_ERR_ARG);
}

static void diagonal_cover(Rng &r) {
  for (int trial = 0; trial < 4000; ++trial) {
    const int k = 1 + r.below(8);
    const int D = 1 << k;
    std::vector<int32_t> A;
    while (int(A.size()) < k) {
      const int q = r.below(40);
      bool dup = false;
      for (int x : A) dup = dup || x == q;
      if (!dup) A.push_back(q);
    }
    std::vector<double> d(2 * size_t(D));
    const int ones = r.below(4);  // how often an entry is exactly 1
    for (int i = 0; i < D; ++i) {
      const bool one = ones > 0 && r.below(4) < ones;
      d[2 * i] = one ? 1.0 : std::cos(r.unit() * 6.28);
      d[2 * i + 1] = one ? 0.0 : std::sin(r.unit() * 6.28);
    }
    double fr = -1;
    int ln = -1;
    CHECK(sv_diag_sweep_cost(k, d.data(), A.data(), &fr, &ln) == SV_OK);
    CHECK(fr >= 0.0 && fr <= 1.0 && ln >= 0 && ln <= sv::kDiagMaxSweeps);
    // every entry other than 1 lies in exactly one swept subcube; the fraction adds up
    const sv::DiagCover cv = sv::diag_cover(k, d.data(), A.data());
    double sum = 0;
    for (int s = 0; s < cv.nsub; ++s) sum += std::ldexp(1.0, -__builtin_popcount(cv.mask[s]));
    CHECK(std::fabs(sum - fr) < 1e-12 && cv.nsub == ln);
    for (int i = 0; i < D; ++i) {
      int hits = 0;
      for (int s = 0; s < cv.nsub; ++s) hits += ((i & cv.mask[s]) == cv.val[s]) ? 1 : 0;
      const bool one = d[2 * i] == 1.0 && d[2 * i + 1] == 0.0;
      CHECK(hits <= 1);
      CHECK(one || hits == 1);
    }
  }
  double fr;
  int ln;
  int32_t A2[2] = {3, 3};
  double d2[8] = {1, 0, 1, 0, 1, 0, -1, 0};
  CHECK(sv_diag_sweep_cost(2, d2, A2, &fr, &ln) == SV_ERR_ARG);
  // after a thread's first call the cover allocates nothing
  int32_t A[6] = {4, 9, 17, 23, 30, 33};
  std::vector<double> d(128);
  for (int i = 0; i < 64; ++i) {
    d[2 * i] = (i % 5 == 0) ? -1.0 : 1.0;
    d[2 * i + 1] = 0.0;
  }
  (void)sv::diag_cover(6, d.data(), A);
  const long before = g_allocs.load();
  for (int i = 0; i < 2000; ++i) (void)sv::diag_cover(6, d.data(), A);
  CHECK(g_allocs.load() == before);
}

static void batch_host(Rng &r) {
  // records of single circuits
  for (int trial = 0; trial < 60; ++trial) {
    const int n = 1 + r.below(SV_BATCH_MAX_QUBITS);
    const int ng = r.below(120);
    std::vector<int32_t> kinds, qubits;
    std::vector<double> mats;
    for (int i = 0; i < ng; ++i) {
      const bool cnot = n > 1 && r.below(3) == 0;
      kinds.push_back(cnot ? SV_BATCH_GATE_CNOT : SV_BATCH_GATE_1Q);
      const int a = r.below(n);
      int b = r.below(n);
      if (cnot && b == a) b = (a + 1) % n;
      qubits.push_back(a);
      qubits.push_back(cnot ? b : -1);
      for (int e = 0; e < 8; ++e) mats.push_back(r.unit() - 0.5);
    }
    sv_batch_circuit c{n, ng, kinds.data(), qubits.data(), mats.data()};
    const int cap = 3 * ng + 2;
    std::vector<int32_t> rec(4 * size_t(cap));
    std::vector<float> rm(8 * size_t(cap));
    int nout = -1;
    CHECK(sv_batch_records(&c, cap, rec.data(), rm.data(), &nout) == SV_OK);
    CHECK(nout >= 0 && nout <= cap);
    if (nout > 0) CHECK(sv_batch_records(&c, nout - 1, rec.data(), rm.data(), &nout) == SV_ERR_ARG);
  }
  // the threaded packing of a whole batch (up to 16 host threads)
  const int count = 700;
  std::vector<std::vector<int32_t>> K(count), Q(count);
  std::vector<std::vector<double>> M(count);
  std::vector<sv_batch_circuit> circs(count);
  std::vector<int64_t> offs(count);
  int64_t off = 0;
  for (int i = 0; i < count; ++i) {
    const int n = 1 + r.below(16);
    const int ng = r.below(60);
    for (int g = 0; g < ng; ++g) {
      const bool cnot = n > 1 && r.below(3) == 0;
      K[i].push_back(cnot ? SV_BATCH_GATE_CNOT : SV_BATCH_GATE_1Q);
      const int a = r.below(n);
      int b = r.below(n);
      if (cnot && b == a) b = (a + 1) % n;
      Q[i].push_back(a);
      Q[i].push_back(cnot ? b : 0);
      for (int e = 0; e < 8; ++e) M[i].push_back(r.unit());
    }
    circs[i] = sv_batch_circuit{n, ng, K[i].data(), Q[i].data(), M[i].data()};
    offs[i] = off;
    off += int64_t(8) << n;
  }
  int32_t cfg[SV_BATCH_CONFIG_LEN];
  sv::batch::default_config(cfg);
  CHECK(sv::batch::valid_config(cfg));
  sv::batch::Packed pk;
  CHECK(sv::batch::pack_batch(count, circs.data(), size_t(off), offs.data(), cfg, &pk) == SV_OK);
  CHECK(pk.ncirc == count);
  int covered = 0;
  for (const auto &it : pk.items) covered += it.P;
  CHECK(covered == count);
  // a bad circuit in the middle is reported, whichever thread meets it
  Q[350][0] = 99;
  sv::batch::Packed bad;
  CHECK(sv::batch::pack_batch(count, circs.data(), size_t(off), offs.data(), cfg, &bad) == SV_ERR_ARG);
  CHECK(sv_batch_workspace_bytes(count, circs.data()) > 0);
}

static void mlp_host(Rng &r) {
  const int nin = SV_MLP_FEATURES, hid = 64;
  std::vector<float> p = random_params(r, nin, hid);
  std::vector<float> x(size_t(nin) * 33);
  for (auto &v : x) v = float(r.unit());
  std::vector<double> y(33);
  CHECK(sv_mlp_forward_host(p.data(), nin, hid, x.data(), 33, y.data()) == SV_OK);
  for (double v : y) CHECK(std::isfinite(v));
  CHECK(sv_mlp_forward_host(nullptr, nin, hid, x.data(), 1, y.data()) == SV_ERR_ARG);
  float f[SV_MLP_FEATURES];
  int32_t t[3] = {29, 3, 0};
  CHECK(sv_cost_features(30, 3, t, 0, 1.0, 1, f) == SV_OK);
  CHECK(sv_cost_features(30, 3, t, 1, 1.5, 1, f) == SV_ERR_ARG);
  CHECK(sv_cost_features(30, 9, t, 0, 1.0, 1, f) == SV_ERR_ARG);
}

// ------------------------------------------------------------------ permutation-tile swizzle
// For tile permutations made of up to five disjoint bit exchanges and for
// arbitrary ones: the chosen map is a bijection of the 2^12 local indices,
// linear over GF(2), keeps a chunk's two amplitudes (l, l ^ 1) adjacent, and
// puts the 64 lanes of every wave instruction two to an 8-byte LDS slot in
// both phases.
static void perm_swizzle(Rng &r) {
  for (int trial = 0; trial < 2000; ++trial) {
    int lo[12];
    for (int b = 0; b < 12; ++b) lo[b] = b;
    if (trial % 2) {
      for (int b = 11; b > 0; --b) {
        const int j = r.below(b + 1);
        const int t = lo[b];
        lo[b] = lo[j];
        lo[j] = t;
      }
    } else {
      const int np = 1 + r.below(5);
      for (int e = 0; e < np; ++e) {
        const int a = r.below(12), b = r.below(12);
        const int t = lo[a];
        lo[a] = lo[b];
        lo[b] = t;
      }
    }
    int32_t px[7];
    sv::choose_perm_swizzle(lo, px);
    for (int j = 0; j < 7; ++j) CHECK(px[j] >= 0 && px[j] < 32);
    if (trial < 50) {
      std::vector<char> hit(4096, 0);
      for (int l = 0; l < 4096; ++l) {
        const int a = sv::lin_swz_host(l, px);
        CHECK(a >= 0 && a < 4096 && !hit[a] && sv::lin_swz_host(l ^ 1, px) == (a ^ 1));
        if (a >= 0 && a < 4096) hit[a] = 1;
      }
    }
    for (int t = 0; t < 16; ++t) {
      const int a = r.below(4096), b = r.below(4096);
      CHECK(sv::lin_swz_host(a ^ b, px) == (sv::lin_swz_host(a, px) ^ sv::lin_swz_host(b, px)));
    }
    // lanes: tile-order bits 1..6; store side through lo[], with a uniform rest
    const int rest_w = r.below(64) << 7, rest_r = r.below(2);
    int cw[32] = {0}, cr[32] = {0};
    for (int lane = 0; lane < 64; ++lane) {
      int lw = rest_w | (lane << 1), lr = 0;
      for (int b = 0; b < 6; ++b)
        if ((lane >> b) & 1) lr |= 1 << lo[b + 1];
      if (rest_r) lr |= 1 << lo[7];
      ++cw[sv::lin_swz_host(lw, px) & 31];
      ++cr[sv::lin_swz_host(lr, px) & 31];
    }
    for (int s = 0; s < 32; ++s) CHECK(cw[s] <= 2 && cr[s] <= 2);
  }
}

// ------------------------------------------------------------------ permutation passes
// Random layouts of 12..30 qubits: the exchanges take L to the target, each
// pass holds disjoint exchanges, at most five, and a tile of 12 bits that
// keeps physical bits 0..3; the pass count matches.
static void perm_passes(Rng &r) {
  for (int trial = 0; trial < 500; ++trial) {
    const int n = 12 + r.below(19);
    int32_t L[64], T[64];
    for (int q = 0; q < n; ++q) L[q] = T[q] = q;
    for (int q = n - 1; q > 0; --q) {
      int j = r.below(q + 1), t = L[q];
      L[q] = L[j];
      L[j] = t;
      j = r.below(q + 1);
      t = T[q];
      T[q] = T[j];
      T[j] = t;
    }
    const std::vector<std::pair<int, int>> sw = sv::permutation_swaps(L, T, n);
    int32_t cur[64], inv[64];
    for (int q = 0; q < n; ++q) {
      cur[q] = L[q];
      inv[L[q]] = q;
    }
    int passes = 0;
    for (size_t i = 0; i < sw.size();) {
      const size_t j = sv::permutation_pass_end(sw, i);
      CHECK(j > i && j - i <= size_t(sv::kPermMaxPairs));
      uint64_t used = 0;
      for (size_t t = i; t < j; ++t) {
        const uint64_t m = (uint64_t(1) << sw[t].first) | (uint64_t(1) << sw[t].second);
        CHECK(!(used & m));
        used |= m;
        const int a = inv[sw[t].first], b = inv[sw[t].second];
        cur[a] = sw[t].second;
        cur[b] = sw[t].first;
        inv[sw[t].first] = b;
        inv[sw[t].second] = a;
      }
      CHECK(j - i == 1 || __builtin_popcountll(used | sv::kPermLowRun) <= sv::kPermTileBits);
      ++passes;
      i = j;
    }
    for (int q = 0; q < n; ++q) CHECK(cur[q] == T[q]);
    CHECK(passes == sv::permutation_passes(L, T, n));
  }
}

int main() {
  Rng r{20261203};
  planners(r);
  diagonal_cover(r);
  batch_host(r);
  mlp_host(r);
  perm_swizzle(r);
  perm_passes(r);
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
