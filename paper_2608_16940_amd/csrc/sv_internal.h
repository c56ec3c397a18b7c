// Internal declarations shared by the libsv translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "sv.h"
#include "sv_guard.h"

namespace sv {

// ------------------------------------------------------------------ workspace
// Matrix ring: per-apply operands travel host -> pinned staging slot ->
// device slot with one async copy; a slot is reused only after the event
// recorded after its copy has completed.
constexpr int kRingSlots = 16;
constexpr size_t kRingSlotBytes = 512 * 1024;  // k <= 8 complex64 matrix, or k <= 7 packed MFMA operand
constexpr int64_t kShotChunk = int64_t(1) << 20;
constexpr int kNormPartials = 2048;
constexpr int kCdfBlockBits = 10;  // hierarchical-CDF block of 2^10 entries (Section IV-E)

struct Workspace {
  char *ring = nullptr;          // kRingSlots * kRingSlotBytes
  uint64_t *blocksum = nullptr;  // nb entries: inclusive prefix of block totals after the scan
  uint64_t *chunksum = nullptr;  // ceil(nb / 1024) chunk totals
  uint64_t *shots = nullptr;     // kShotChunk decoded outcomes
  double *partials = nullptr;    // kNormPartials FP64 partial sums
  uint64_t *scalars = nullptr;   // 64 small results: [0] the FP64 norm, [1] the sampler's bad-input flag
};

// Set by the CDF build when an entry is outside [0, 4) or not a number, or
// when the fixed-point total wraps past 2^64 (cleared at the start of each build).
inline unsigned *cdf_flag(const Workspace &ws) { return reinterpret_cast<unsigned *>(ws.scalars + 1); }

// Bytes needed for an n-qubit workspace; if base != nullptr also fills *ws.
size_t workspace_layout(int n, char *base, Workspace *ws);

// ------------------------------------------------------------------ layout argument
struct LayoutArg {
  int8_t pos[64];  // pos[q] = physical bit of logical qubit q
};
LayoutArg identity_layout(int n);

// The sampler (CDF build, then shots in chunks of `chunk` through ws.shots;
// psi != nullptr: probabilities of the state, decoded through L; else the
// caller's array).  Synchronises st.  bad_code: status for flagged inputs.
int sample_impl(const float2 *psi, const double *probs, int n, const Workspace &ws, int64_t chunk, uint64_t seed,
                int64_t shots, uint64_t *out_host, const LayoutArg &L, hipStream_t st, int bad_code);

// ------------------------------------------------------------------ error reporting
void set_error(const std::string &msg);

#define SV_HIP_CHECK(expr)                                                              \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      ::sv::set_error(std::string(#expr) + " failed: " + hipGetErrorString(e_));        \
      return SV_ERR_DEVICE;                                                             \
    }                                                                                   \
  } while (0)

// ------------------------------------------------------------------ kernels: launchers
// All launchers enqueue on `st` and return the launch status.

// |0...0>
hipError_t launch_init_zero(float2 *psi, int n, hipStream_t st);

// k <= 4, per-thread group gather/FMA/scatter.  m: complex64 row-major 2^k x 2^k (host).
hipError_t launch_dense_valu(float2 *psi, int n, int k, const int32_t *phys_targets, const float2 *m,
                             hipStream_t st);

// k = 1 on physical bit b <= 6 with wavefront shuffles.  m: 2x2 complex64 (host).
hipError_t launch_1q_shuffle(float2 *psi, int n, int b, const float2 *m, hipStream_t st);

// Diagonal operator: the 2^k diagonal entries (complex64) in device memory
// (d_dev), or for k <= 4 from the host by value (d_dev null, d_host set).
// Partial sweep: fix_phys[0..nfix) are distinct physical positions >= 1 held
// at the values of bits 0.. of fix_val; only that subcube of the state is
// read and written (nfix = 0: a full sweep).
hipError_t launch_diag(float2 *psi, int n, int k, const int32_t *phys_targets, const float2 *d_dev,
                       const float2 *d_host, int nfix, const int32_t *fix_phys, int fix_val, hipStream_t st);
// any k <= 8; m_dev: device complex64 row-major matrix.
hipError_t launch_dense_generic(float2 *psi, int n, int k, const int32_t *phys_targets, const float2 *m_dev,
                                hipStream_t st);

// Exchange physical bits p and q (a bit transposition; half the amplitudes move).
hipError_t launch_swap_bits(float2 *psi, int n, int p, int q, hipStream_t st);

hipError_t launch_probs(const float2 *psi, int n, double *out, int logical, const LayoutArg &L, hipStream_t st);
hipError_t launch_norm(const float2 *psi, int n, double *partials, double *result, hipStream_t st);

// Sampler.  src_state != nullptr: probabilities from the state; else from probs.
hipError_t launch_cdf_build(const float2 *src_state, const double *src_probs, int n, const Workspace &ws,
                            hipStream_t st);
hipError_t launch_shots(const float2 *src_state, const double *src_probs, int n, const Workspace &ws,
                        uint64_t seed, int64_t shot0, int64_t count, const LayoutArg &L, hipStream_t st);

// ------------------------------------------------------------------ LDS-tiled kernels
// A tile is the set of 2^s amplitudes that share every physical bit outside
// the tile mask S.  Bits of the tile-order index v (s bits, ascending physical
// position) are scattered into the local (LDS) index: on load bit b of v goes
// to local bit loc_in[b]; on store local bit loc_out[b] supplies bit b of the
// output tile-order index (loc_out == loc_in means no relabel).
struct TilePlan {
  int n = 0, s = 0, K = 0, M = 0;
  int order = -1;  // workgroup-to-tile order: -1 the default, 0 plain, x > 0 see tile_order_shift
  uint64_t smask = 0;
  int sbit[32] = {0};
  int loc_in[32] = {0};
  int loc_out[32] = {0};
};

// Real-embedded, lane-major MFMA operand for gate matrix G (FP64 host, 2^K x 2^K).
// prec = SV_PREC_FP32: float; SV_PREC_BF16X3: uint16 (k = 4: embedding hi then lo;
// k >= 5: Gr hi, Gr lo, Gi hi, Gi lo planes).
size_t mfma_operand_bytes(int K, int prec);
void pack_mfma_operand(int K, int prec, const double *G, void *out);

// Tile geometry for a dense gate on physical targets A (gate order).  The
// non-target tile bits are the bits of `extra` (which must not contain targets)
// followed by the lowest other non-target bits, M in total, except that up to
// three non-target bits from bit 7 up are left to the tile index.  Returns false if
// the state is too small for the MFMA tiling.
bool make_gate_tile(int n, int K, const int32_t *A, uint64_t extra, TilePlan *tp);
int mfma_tile_M(int K);

// True when the 2^k x 2^k complex128 matrix G (row-major interleaved) maps
// every basis state |c> to |pi(c)>, pi moving bit j of c to bit perm[j]: a
// permutation of the block's qubits, which the layout map absorbs.
bool qubit_permutation(const double *G, int k, int *perm);

// opsrc: SV_MFMA_OPERAND_* (where k <= 5 waves keep the embedded operand).
hipError_t launch_tile_mfma(const TilePlan &tp, int prec, int opsrc, float2 *psi, const void *operand_dev,
                            hipStream_t st);

// Pure bit permutation within a tile: tp.loc_out describes where each tile bit goes.
hipError_t launch_tile_permute(const TilePlan &tp, float2 *psi, hipStream_t st);

}  // namespace sv

// The state handle behind the C-ABI's opaque sv_state (one per state vector).
struct sv_state {
  int n = 0;
  int dm_n = 0;  // density-matrix handle: N of the 2N-qubit vectorised state, else 0
  float2 *amps = nullptr;
  char *ws_base = nullptr;
  size_t ws_bytes = 0;
  sv::Workspace ws;
  hipStream_t st = nullptr;
  int32_t L[64];
  int32_t Linv[64];
  // options
  int variant = SV_VARIANT_AUTO;
  int prec = SV_PREC_FP32;
  int mfma_min_k = 4;
  int lazy = 0;
  int low_bits = 12;
  int policy = SV_POLICY_BELADY;
  int opsrc = SV_MFMA_OPERAND_AUTO;
  int tile_order = -1;
  // relabel policy state: planner hints and recency per logical qubit
  bool have_hints = false;
  int64_t next_use[64];
  int64_t last_use[64];
  int64_t clock = 0;
  // operand staging ring
  char *pinned = nullptr;
  hipEvent_t ev[sv::kRingSlots];
  bool ev_live[sv::kRingSlots];
  int ring_next = 0;
  sv_stats stats;
};
