// Cover of a diagonal operator's entries other than 1 by subcubes of the
// state: the lowering launches one partial sweep per subcube.  Host code
// only, no HIP types.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>

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

namespace detail {

// Working state of one cover computation: the entries other than 1 and, per
// candidate bit and value, the entries with that bit at that value, as
// 256-bit sets (a subcube's entries are the intersection over its fixed
// bits); the memo of subcube costs and choices, keyed by the candidate bits
// a subcube fixes and their values.
struct CoverWork {
  static constexpr int kKeys = 1 << (2 * kDiagSplitBits);
  int nc = 0;
  int cand[kDiagSplitBits];
  uint64_t nonone[4];
  uint64_t sel[kDiagSplitBits][2][4];
  double cost[kKeys];
  int8_t choice[kKeys];  // -2 nothing to do, -1 one sweep, c: split on candidate c
  uint32_t stamp[kKeys];
  uint32_t gen = 0;
};

inline double cover_best(CoverWork &w, uint32_t mask, uint32_t val) {
  const uint32_t key = (mask << kDiagSplitBits) | val;
  if (w.stamp[key] == w.gen) return w.cost[key];
  uint64_t s[4] = {w.nonone[0], w.nonone[1], w.nonone[2], w.nonone[3]};
  for (int q = 0; q < w.nc; ++q)
    if ((mask >> q) & 1)
      for (int i = 0; i < 4; ++i) s[i] &= w.sel[q][(val >> q) & 1][i];
  const bool any = (s[0] | s[1] | s[2] | s[3]) != 0;
  double c = 0;
  int8_t ch = -2;
  if (any) {
    c = std::ldexp(1.0, -__builtin_popcount(mask)) + kDiagLaunchCost;
    ch = -1;
    for (int q = 0; q < w.nc; ++q) {
      const uint32_t b = 1u << q;
      if (mask & b) continue;
      const double sp = cover_best(w, mask | b, val) + cover_best(w, mask | b, val | b);
      if (sp < c - 1e-12) {
        c = sp;
        ch = int8_t(q);
      }
    }
  }
  w.stamp[key] = w.gen;
  w.cost[key] = c;
  w.choice[key] = ch;
  return c;
}

inline bool cover_emit(const CoverWork &w, uint32_t mask, uint32_t val, DiagCover &cv) {
  const int8_t ch = w.choice[(mask << kDiagSplitBits) | val];
  if (ch == -2) return true;
  if (ch == -1) {
    if (cv.nsub == kDiagMaxSweeps) return false;
    uint8_t bm = 0, bv = 0;  // back to block bits
    for (int q = 0; q < w.nc; ++q) {
      if ((mask >> q) & 1) bm |= uint8_t(1u << w.cand[q]);
      if ((val >> q) & 1) bv |= uint8_t(1u << w.cand[q]);
    }
    cv.mask[cv.nsub] = bm;
    cv.val[cv.nsub] = bv;
    ++cv.nsub;
    return true;
  }
  const uint32_t b = 1u << ch;
  return cover_emit(w, mask | b, val, cv) && cover_emit(w, mask | b, val | b, cv);
}

}  // namespace detail

// Exact minimum over recursive splits: a subcube with no entry other than 1
// costs nothing, otherwise either one sweep of it or the best split on a
// free candidate bit.  Subcubes are keyed by the candidate bits they fix
// (at most 3^6 reachable, 4^6 keys).  The working state is one thread-local
// object (53 KB) whose memo is invalidated per call by a generation stamp,
// and the recursion passes it by reference, so after a thread's first call
// (whose thread-local storage the runtime may set up) a call allocates
// nothing; this runs on every diagonal apply.
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
  thread_local detail::CoverWork w;
  if (++w.gen == 0) {  // stamps wrapped: clear them
    std::fill(w.stamp, w.stamp + detail::CoverWork::kKeys, 0u);
    w.gen = 1;
  }
  w.nc = nc;
  for (int c = 0; c < nc; ++c) w.cand[c] = cand[c];
  for (int i = 0; i < 4; ++i) w.nonone[i] = 0;
  for (int c = 0; c < nc; ++c)
    for (int v = 0; v < 2; ++v)
      for (int i = 0; i < 4; ++i) w.sel[c][v][i] = 0;
  for (int r = 0; r < D; ++r) {
    if (!one[r]) w.nonone[r >> 6] |= uint64_t(1) << (r & 63);
    for (int c = 0; c < nc; ++c) w.sel[c][(r >> cand[c]) & 1][r >> 6] |= uint64_t(1) << (r & 63);
  }
  detail::cover_best(w, 0, 0);
  DiagCover cv;
  if (detail::cover_emit(w, 0, 0, cv)) return cv;
  return out;  // more sweeps than allowed: one full sweep
}

}  // namespace sv
