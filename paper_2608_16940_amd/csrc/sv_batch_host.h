// Batched path, host side: the gate records the persistent kernel runs and
// the host pass that builds them (validation, FP64 fusion of single-qubit
// runs, LDS slice passes, groups, linear CNOT runs, packing).  Plain C++ (no
// HIP types), shared by the kernel's translation unit and the host pass.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "sv_batch.h"

namespace sv {
namespace batch {

constexpr int kBT = 512;           // threads per workgroup of the batched kernel
constexpr int kLdsAmps = 1 << 14;  // 128 KiB of complex64 state slices
constexpr int kMaxPack = 16;
// Single-qubit gates applied in one LDS sweep: up to five inside slice
// passes (2^5 amplitudes per thread, gate records read through a
// wave-uniform pointer), up to four for states held in LDS, whose
// per-lane records would not fit the register budget with five.
constexpr int kMaxGroupPass = 5;
constexpr int kMaxGroupLds = 4;
constexpr int kSliceBits = 14;
constexpr int kGatePass = SV_BATCH_PASS;  // record: q0 = slice qubit mask, q1 = gates in the pass

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

struct Packed {
  std::vector<BGate> gates;
  std::vector<BItem> items;
  int ncirc = 0;
};

// Pass rewriting, grouping and CNOT merging of one circuit's records.
std::vector<BGate> make_passes(const std::vector<BGate> &g, int n);
std::vector<BGate> group_run(const std::vector<BGate> &g, size_t a, size_t b, int maxc);
std::vector<BGate> merge_cnots(const std::vector<BGate> &g, size_t a, size_t b);
std::vector<BGate> group_single_qubit(const std::vector<BGate> &g, bool passes);
int count_units(const std::vector<BGate> &g);

// Pack sizes per qubit count (SV_BATCH_CONFIG_LEN entries).
bool valid_config(const int32_t *cfg);
void default_config(int32_t *cfg);

// Per-circuit outcome of the host pass.
enum CircStatus { CIRC_OK = 0, CIRC_BAD, CIRC_BAD_1Q, CIRC_BAD_CNOT, CIRC_BAD_KIND, CIRC_NOMEM };
int prepare_circuit(const sv_batch_circuit &C, int64_t state_offset, size_t states_bytes, std::vector<BGate> &g);

// Prepare every circuit (on up to 16 host threads), group by qubit count,
// cut packs, order by cost.  SV_OK or SV_ERR_ARG (the first bad circuit by
// index is the one reported).
int pack_batch(int count, const sv_batch_circuit *circs, size_t states_bytes, const int64_t *state_offsets,
               const int32_t *cfg, Packed *out);

}  // namespace batch
}  // namespace sv
