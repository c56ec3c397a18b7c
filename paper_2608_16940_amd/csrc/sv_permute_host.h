// Layout permutations, host side: the bit exchanges that take one layout
// to another, their grouping into in-place tile passes, and the LDS swizzle
// of a pass (k_tile_permute).  Plain C++, no HIP types.
#pragma once

#include <cstdint>
#include <cstring>
#include <utility>
#include <vector>

namespace sv {

constexpr int kPermTileBits = 12;   // bits of a permutation tile (2^12 amplitudes, 32 KiB of LDS)
constexpr int kPermMaxPairs = 5;    // exchanges per pass (the tile keeps physical bit 0)
constexpr uint64_t kPermLowRun = 0xF;  // physical bits 0..3 stay in every tile: runs of >= 16 amplitudes

// Exchanges of physical bits that take layout L (logical qubit -> physical
// bit) to `target`, in selection order: physical positions 0..n-1 are filled
// with their final qubits one transposition at a time (Lemma 2: each
// exchange updates L = tau o L).
inline std::vector<std::pair<int, int>> permutation_swaps(const int32_t *L_in, const int32_t *target, int n) {
  int32_t L[64], Linv[64];
  for (int q = 0; q < n; ++q) {
    L[q] = L_in[q];
    Linv[L_in[q]] = q;
  }
  std::vector<std::pair<int, int>> swaps;
  for (int p = 0; p < n; ++p) {
    int want = -1;
    for (int q = 0; q < n; ++q)
      if (target[q] == p) want = q;
    const int cur = L[want];
    if (cur == p) continue;
    swaps.push_back({p, cur});
    const int a = Linv[p], b = Linv[cur];
    L[a] = cur;
    L[b] = p;
    Linv[p] = b;
    Linv[cur] = a;
  }
  return swaps;
}

// End (exclusive) of the tile pass that starts at swaps[i]: consecutive
// exchanges on disjoint bits commute, so up to kPermMaxPairs of them run as
// one in-place pass, as long as the tile -- the exchanged bits plus the
// lowest other bits, kPermTileBits in all -- still holds physical bits 0..3.
// Measured at N=30: five exchanges that left only bits 0..1 in the tile (runs
// of 4 amplitudes) took 18 ms, four that kept bits 0..3 3.0-3.4 ms.
inline size_t permutation_pass_end(const std::vector<std::pair<int, int>> &swaps, size_t i) {
  uint64_t used = 0;
  size_t j = i;
  while (j < swaps.size() && j - i < size_t(kPermMaxPairs)) {
    const uint64_t m = (uint64_t(1) << swaps[j].first) | (uint64_t(1) << swaps[j].second);
    if (used & m) break;
    if (j > i && __builtin_popcountll(used | m | kPermLowRun) > kPermTileBits) break;
    used |= m;
    ++j;
  }
  return j;
}

// Tile passes a permutation from L to target takes (states of at least
// kPermTileBits qubits).
inline int permutation_passes(const int32_t *L, const int32_t *target, int n) {
  const std::vector<std::pair<int, int>> sw = permutation_swaps(L, target, n);
  int passes = 0;
  for (size_t i = 0; i < sw.size(); i = permutation_pass_end(sw, i)) ++passes;
  return passes;
}

// GF(2) rank of m vectors of five bits.
inline int rank5(const int *v, int m) {
  int basis[5] = {0, 0, 0, 0, 0}, r = 0;
  for (int i = 0; i < m; ++i) {
    int x = v[i] & 31;
    for (int b = 4; b >= 0 && x; --b) {
      if (!((x >> b) & 1)) continue;
      if (!basis[b]) {
        basis[b] = x;
        ++r;
        x = 0;
      } else {
        x ^= basis[b];
      }
    }
  }
  return r;
}

// l ^ X(l >> 5) for a 12-bit local index l: bit 5 + j of l contributes px[j]
// (five bits) to the low five bits.  A bijection, linear over GF(2).
inline int lin_swz_host(int l, const int32_t *px) {
  int x = 0;
  for (int j = 0; j < 7; ++j)
    if ((l >> (5 + j)) & 1) x ^= px[j];
  return l ^ x;
}

// The 64 lanes of a wave instruction vary in six local bits (tile-order bits
// 1..6: local bits 1..6 on load, their loc_out images on store) and the rest
// of the address is uniform, so the lanes' 8-byte LDS slots (address mod 32)
// form an affine image of those six bits: each slot is hit 2^(6 - rank)
// times.  Rank 5 (two lanes per slot, the minimum for 64 lanes) in both
// phases is the goal; candidates are the identity, a fold, a shift and a
// fixed pseudo-random sequence, and the first that reaches rank 5 twice is
// taken (else the best sum).  X reads bits 5..11 only, so f(l ^ 1) =
// f(l) ^ 1: a chunk's two amplitudes stay adjacent.
inline void choose_perm_swizzle(const int *loc_out, int32_t px[7]) {
  auto score = [&](const int32_t *c) {
    int w[6], r[6];
    for (int b = 0; b < 6; ++b) {
      w[b] = lin_swz_host(1 << (b + 1), c);
      r[b] = lin_swz_host(1 << loc_out[b + 1], c);
    }
    return rank5(w, 6) + rank5(r, 6);
  };
  int32_t best[7] = {0, 0, 0, 0, 0, 0, 0};
  int best_s = score(best);
  uint32_t lcg = 12345u;
  for (int cand = 0; cand < 512 && best_s < 10; ++cand) {
    int32_t c[7];
    for (int j = 0; j < 7; ++j) {
      if (cand == 0) {
        c[j] = 1 << (j % 5);  // fold of bits 5..9 and 10..11 onto 0..4
      } else if (cand == 1) {
        c[j] = j < 5 ? 1 << j : 0;
      } else {
        lcg = lcg * 1664525u + 1013904223u;
        c[j] = int32_t((lcg >> 27) & 31);
      }
    }
    const int s = score(c);
    if (s > best_s) {
      best_s = s;
      std::memcpy(best, c, sizeof(best));
    }
  }
  std::memcpy(px, best, sizeof(best));
}

}  // namespace sv
