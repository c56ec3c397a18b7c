// Cover of a diagonal operator's entries other than 1 by subcubes of the
// state: the lowering launches one partial sweep per subcube.  Host code
// only, no HIP types.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <functional>

namespace sv {

// Partial diagonal sweeps.  Amplitudes whose diagonal entry is exactly 1
// stay as they are, so a diagonal block may sweep only subcubes of the state
// (target bits held fixed) that together hold every entry that is not 1.
// Fixed bits sit at physical position 4 or above, so a skipped run is at
// least 2^4 amplitudes (128 bytes, whole cache lines).  The cover minimises
// the swept fraction of the state plus kDiagLaunchCost per sweep, over at
// most kDiagSplitBits candidate bits (the highest targets).
constexpr int kDiagFixMinBit = 4;
constexpr int kDiagMaxSweeps = 16;
constexpr int kDiagSplitBits = 6;
constexpr double kDiagLaunchCost = 1.0 / 256;  // about 10 us against a 2.5 ms sweep at N=30

struct DiagCover {
  int nsub = 0;                  // sweeps (0: the table is all ones, nothing to do)
  uint8_t mask[kDiagMaxSweeps];  // block bits held fixed by each sweep
  uint8_t val[kDiagMaxSweeps];   // and their values
};

// Exact minimum over recursive splits: a subcube with no entry other than 1
// costs nothing, otherwise either one sweep of it or the best split on a
// free candidate bit.  Subcubes are keyed by the candidate bits they fix
// (at most 3^6 reachable, 4^6 keys); the memo lives in thread-local arrays
// stamped per call, so a call allocates nothing (this runs on every
// diagonal apply).
inline DiagCover diag_cover(int k, const double *diag, const int32_t *A) {
  const int D = 1 << k;
  DiagCover out;
  bool one[256];
  int nones = 0;
  for (int r = 0; r < D; ++r) {
    one[r] = diag[2 * r] == 1.0 && diag[2 * r + 1] == 0.0;
    nones += one[r];
  }
  if (nones == D) return out;  // identity: nothing to sweep
  out.nsub = 1;                // default: one full sweep
  out.mask[0] = out.val[0] = 0;
  int cand[8], nc = 0;  // block bits of the highest targets from kDiagFixMinBit up
  for (int j = 0; j < k; ++j)
    if (A[j] >= kDiagFixMinBit) cand[nc++] = j;
  std::sort(cand, cand + nc, [&](int x, int y) { return A[x] > A[y]; });
  nc = std::min(nc, kDiagSplitBits);
  if (nones == 0 || nc == 0) return out;  // every subcube holds entries other than 1
  // entries as 256-bit sets: those other than 1, and per candidate bit and
  // value the entries with that bit at that value; a subcube's entries are
  // the intersection over its fixed bits
  uint64_t nonone[4] = {0, 0, 0, 0}, sel[kDiagSplitBits][2][4] = {};
  for (int r = 0; r < D; ++r) {
    if (!one[r]) nonone[r >> 6] |= uint64_t(1) << (r & 63);
    for (int c = 0; c < nc; ++c) sel[c][(r >> cand[c]) & 1][r >> 6] |= uint64_t(1) << (r & 63);
  }
  constexpr int kKeys = 1 << (2 * kDiagSplitBits);
  thread_local double cost[kKeys];
  thread_local int8_t choice[kKeys];  // -2 nothing to do, -1 one sweep, c: split on candidate c
  thread_local uint32_t stamp[kKeys];
  thread_local uint32_t gen = 0;
  if (++gen == 0) {  // stamps wrapped: clear them
    std::fill(stamp, stamp + kKeys, 0u);
    gen = 1;
  }
  std::function<double(uint32_t, uint32_t)> best = [&](uint32_t mask, uint32_t val) -> double {
    const uint32_t key = (mask << kDiagSplitBits) | val;
    if (stamp[key] == gen) return cost[key];
    uint64_t w[4] = {nonone[0], nonone[1], nonone[2], nonone[3]};
    for (int q = 0; q < nc; ++q)
      if ((mask >> q) & 1)
        for (int i = 0; i < 4; ++i) w[i] &= sel[q][(val >> q) & 1][i];
    const bool any = (w[0] | w[1] | w[2] | w[3]) != 0;
    double c = 0;
    int8_t ch = -2;
    if (any) {
      c = std::ldexp(1.0, -__builtin_popcount(mask)) + kDiagLaunchCost;
      ch = -1;
      for (int q = 0; q < nc; ++q) {
        const uint32_t b = 1u << q;
        if (mask & b) continue;
        const double sp = best(mask | b, val) + best(mask | b, val | b);
        if (sp < c - 1e-12) {
          c = sp;
          ch = int8_t(q);
        }
      }
    }
    stamp[key] = gen;
    cost[key] = c;
    choice[key] = ch;
    return c;
  };
  best(0, 0);
  DiagCover cv;
  std::function<bool(uint32_t, uint32_t)> emit = [&](uint32_t mask, uint32_t val) -> bool {
    const int8_t ch = choice[(mask << kDiagSplitBits) | val];
    if (ch == -2) return true;
    if (ch == -1) {
      if (cv.nsub == kDiagMaxSweeps) return false;
      uint8_t bm = 0, bv = 0;  // back to block bits
      for (int q = 0; q < nc; ++q) {
        if ((mask >> q) & 1) bm |= uint8_t(1u << cand[q]);
        if ((val >> q) & 1) bv |= uint8_t(1u << cand[q]);
      }
      cv.mask[cv.nsub] = bm;
      cv.val[cv.nsub] = bv;
      ++cv.nsub;
      return true;
    }
    const uint32_t b = 1u << ch;
    return emit(mask | b, val) && emit(mask | b, val | b);
  };
  if (emit(0, 0)) return cv;
  return out;  // more sweeps than allowed: one full sweep
}

}  // namespace sv
