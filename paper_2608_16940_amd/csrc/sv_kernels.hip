// Streaming kernels of the state-vector path for gfx950 (wave64):
//   - |0...0> initialisation,
//   - per-thread dense gate apply for k <= 4 (vector ALU),
//   - single-qubit apply with cross-lane exchange for low physical bits,
//   - a generic one-group-per-workgroup apply for any k <= 8,
//   - the streaming diagonal apply (any k <= 8),
//   - physical bit transposition (the on-demand layout swap),
//   - FP64 probabilities and norm,
//   - the two-level integer CDF sampler.
// Every index is 64-bit: the state reaches 2^35 amplitudes.
#include <algorithm>
#include <cstring>
#include <utility>

#include "sv_internal.h"

namespace sv {
namespace {

constexpr int kThreads = 256;
constexpr int64_t kFullGrid = int64_t(1) << 23;
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t insert_zero_bit(int64_t x, int p) {
  const int64_t low = x & ((int64_t(1) << p) - 1);
  return ((x >> p) << (p + 1)) | low;
}

// Streaming order.  Work item `lin` (one 16-byte chunk per thread) is moved
// to chunk stream_chunk(lin): within each aligned block of 2^14 chunks the
// six low workgroup bits go to chunk bits 6..11 and the two wave bits to
// bits 12..13, so 64 consecutive workgroups interleave at 1 KiB granularity
// and a workgroup's waves sit 64 KiB apart.  A bijection that keeps the lane
// bits; measured on MI355X at N=30 it raises an in-place streaming pass from
// 6.1 to 6.8 TB/s (sequential order leaves HBM channels unevenly loaded).
// It is an HBM effect: work sets below 2^24 items (states that stay in the
// caches) keep the plain order.  Used by every kernel whose work items are
// independent chunks, amplitudes or groups.
__device__ __forceinline__ int64_t stream_chunk(int64_t lin, int64_t nchunks) {
  if (nchunks < (int64_t(1) << 24)) return lin;
  const int64_t lane = lin & 63, wave = (lin >> 6) & 3, blk = (lin >> 8) & 63;
  return (lin & ~int64_t(16383)) | (wave << 12) | (blk << 6) | lane;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 acc) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
  return acc;
}

// Workgroups for `items` per-thread work units; streaming kernels here run
// fastest with one unit per thread over a full grid.  kFullGrid = 2^23
// workgroups of 256 (2^31 work-items) stays inside the 2^32 - 1 dispatch
// limit and covers every chunk of a 2^32-amplitude state once; larger states
// grid-stride.
inline unsigned grid_for(int64_t items, int per_block, int64_t cap = 1 << 20) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return unsigned(g);
}

// ------------------------------------------------------------------ init
__global__ __launch_bounds__(kThreads) void k_init_zero(float4 *psi4, int64_t n4, float2 *psi) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n4; i += stride)
    psi4[stream_chunk(i, n4)] = make_float4(0.f, 0.f, 0.f, 0.f);
  // chunk 0 was zeroed by this same thread (item 0 maps to chunk 0)
  if (blockIdx.x == 0 && threadIdx.x == 0) psi[0] = make_float2(1.f, 0.f);
}

__global__ void k_init_small(float2 *psi, int64_t dim) {
  for (int64_t i = threadIdx.x; i < dim; i += blockDim.x) psi[i] = make_float2(i == 0 ? 1.f : 0.f, 0.f);
}

// ------------------------------------------------------------------ dense, vector ALU
template <int K>
struct ValuArgs {
  float2 m[1 << (2 * K)];   // row-major complex64
  int64_t off[1 << K];      // in-group offset of amplitude c: sum_j bit_j(c) << A_j
  int sorted[K];            // target positions ascending
};

// One thread owns one group of 2^K amplitudes.  Consecutive threads take
// consecutive values of the non-target bits, lowest first, so a wave's loads
// are contiguous whenever the low physical bits are not targets.
template <int K>
__global__ __launch_bounds__(kThreads) void k_dense_valu(float2 *__restrict__ psi, int64_t ngroups,
                                                         ValuArgs<K> a) {
  constexpr int D = 1 << K;
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x; g < ngroups; g += stride) {
    int64_t base = stream_chunk(g, ngroups);
#pragma unroll
    for (int j = 0; j < K; ++j) base = insert_zero_bit(base, a.sorted[j]);
    float2 in[D];
#pragma unroll
    for (int c = 0; c < D; ++c) in[c] = psi[base + a.off[c]];
#pragma unroll
    for (int r = 0; r < D; ++r) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int c = 0; c < D; ++c) acc = cfma(a.m[r * D + c], in[c], acc);
      psi[base + a.off[r]] = acc;
    }
  }
}

// ------------------------------------------------------------------ single qubit, wave exchange
// Each lane holds two consecutive amplitudes (one 16-byte load).  For target
// bit 0 the pair is inside the lane; for bit b in 1..6 the partner pair sits
// in lane (lane ^ 2^(b-1)) of the same wave and arrives by a cross-lane
// shuffle, so every load and store of the wave is one contiguous 1 KiB run.
// The grid is capped (a dispatch holds at most 2^32 - 1 work-items), so each
// workgroup strides over chunk blocks; the stride is uniform per workgroup, so
// whole waves stay together for the exchange.
__global__ __launch_bounds__(kThreads) void k_1q_shuffle(float4 *__restrict__ psi4, int64_t nchunks, int b,
                                                         float2 m00, float2 m01, float2 m10, float2 m11) {
  for (int64_t blk = int64_t(blockIdx.x) * kThreads; blk < nchunks; blk += int64_t(gridDim.x) * kThreads) {
    const int64_t t = blk + threadIdx.x;
    const bool active = t < nchunks;
    // the streaming order keeps lane bits: partners (bits 1..6) stay in the wave
    const int64_t c = active ? stream_chunk(t, nchunks) : 0;
    float4 v = active ? psi4[c] : make_float4(0.f, 0.f, 0.f, 0.f);
    float2 a0 = make_float2(v.x, v.y), a1 = make_float2(v.z, v.w);
    float2 o0, o1;
    if (b == 0) {
      o0 = cfma(m01, a1, cmul(m00, a0));
      o1 = cfma(m11, a1, cmul(m10, a0));
    } else {
      const int mask = 1 << (b - 1);
      float4 p;
      p.x = __shfl_xor(v.x, mask);
      p.y = __shfl_xor(v.y, mask);
      p.z = __shfl_xor(v.z, mask);
      p.w = __shfl_xor(v.w, mask);
      const float2 p0 = make_float2(p.x, p.y), p1 = make_float2(p.z, p.w);
      if ((t >> (b - 1)) & 1) {  // this lane's amplitudes have bit b = 1; partners have bit b = 0
        o0 = cfma(m11, a0, cmul(m10, p0));
        o1 = cfma(m11, a1, cmul(m10, p1));
      } else {
        o0 = cfma(m01, p0, cmul(m00, a0));
        o1 = cfma(m01, p1, cmul(m00, a1));
      }
    }
    if (active) psi4[c] = make_float4(o0.x, o0.y, o1.x, o1.y);
  }
}

// ------------------------------------------------------------------ diagonal, any k <= 8
// A diagonal fused operator multiplies amplitude y by d[r(y)], where bit j of
// r(y) is physical bit A_j of y, and leaves the layout unchanged (the diag
// branch of the lazy-TTGT lowering, Eq. cost-diag-formal: one streaming pass
// whatever the target positions).  Each thread takes UNR 16-byte chunks (two
// amplitudes that differ in physical bit 0), in the streaming order of
// stream_chunk; the 2^k table sits in LDS.  One chunk per thread over a full
// grid (four per thread on a capped, grid-strided launch was 10% slower).
//
// Partial sweeps.  Amplitudes whose table entry is exactly 1 stay as they
// are, so a sweep may visit only a subcube of the state: some target bits
// held at fixed values (a controlled phase fixes its control bits to 1).
// Work item w becomes a chunk index by inserting each fixed bit's value at
// its chunk-bit position (lowest first); with f fixed bits the pass reads and
// writes 2^-f of the state.  The host covers the entries that are not 1 with
// a few such subcubes, one launch each.
//
// Fixed bits low in the address (physical 4..13) narrow the set of HBM
// channels that the workgroups in flight at one time reach: at N=30, 32 and
// 34 a sixteenth of the state with physical bits 6..9 fixed streamed at
// 3.8-4.3 TB/s against 6.2-6.4 with bits 20..23 fixed.  Such sweeps exchange
// work index bits 14..18 (the 2^14-chunk block index, above what
// stream_chunk permutes) with the five work bits that land at physical bits
// 25..29, so consecutive blocks sit 32 MiB apart.  Over the sets of three to
// five fixed bits in 4..13 measured at those sizes the rate went from
// 3.6-5.6 to 4.6-6.3 TB/s, and no set lost more than 3%.  With one or two
// fixed bits, or fixed bits higher up, the plain order was as fast or faster
// (the exchange with bits 21..24 fixed: 3.5-4.2 TB/s), so the host asks for
// it only for the low sets.
constexpr int kDiagByValue = 16;  // tables up to k = 4 travel in the kernel arguments
constexpr int kDiagXchgLo = 14;   // lowest work bit of the exchanged block-index field
constexpr int kDiagXchgBits = 5;
struct DiagArgs {
  int k;
  int tgt[8];  // physical position of block bit j
  int bit0;    // r-bit set by physical bit 0 (0 if bit 0 is not a target)
  int nfix;    // bits held fixed by this partial sweep
  int fix[8];  // their chunk-bit positions (physical position - 1), ascending
  int fixval;  // bit i: the value of fix[i]
  int xhi;     // work bit where the field exchanged with bits 14..18 starts (0: no exchange)
  float2 small[kDiagByValue];  // the table when dtab is null
};

__device__ __forceinline__ int64_t insert_bit(int64_t x, int p, int64_t v) {
  const int64_t low = x & ((int64_t(1) << p) - 1);
  return ((x >> p) << (p + 1)) | (v << p) | low;
}

// Exchange of the disjoint bit fields [kDiagXchgLo, +5) and [hi, +5) of x.
__device__ __forceinline__ int64_t xchg_fields(int64_t x, int hi) {
  const int64_t m = (int64_t(1) << kDiagXchgBits) - 1;
  const int64_t lo = (x >> kDiagXchgLo) & m, up = (x >> hi) & m;
  return (x & ~((m << kDiagXchgLo) | (m << hi))) | (up << kDiagXchgLo) | (lo << hi);
}

// nwork = chunks visited: 2^(N-1) >> nfix.  The first chunk's load goes out
// before the table is staged in LDS, so the two round trips overlap (partial
// sweeps of the N=30 headline 2-4% faster, full sweeps unchanged).  The
// fixed-bit and target loops stay dynamic: unrolled to eight predicated
// steps they cost about 150 vector instructions per 16-byte chunk and made
// the sweep ALU-bound (diagonal sweeps of the headline 313 -> 379 ms).
template <bool XCHG>
__global__ __launch_bounds__(kThreads) void k_diag(float4 *__restrict__ psi4, int64_t nwork,
                                                   const float2 *__restrict__ dtab, DiagArgs a) {
  __shared__ float2 tab[256];
  const int64_t step = int64_t(gridDim.x) * kThreads;
  auto chunk_of = [&](int64_t lin) {
    int64_t c = stream_chunk(XCHG ? xchg_fields(lin, a.xhi) : lin, nwork);
    for (int i = 0; i < a.nfix; ++i) c = insert_bit(c, a.fix[i], (a.fixval >> i) & 1);
    return c;
  };
  int64_t lin = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  int64_t c = 0;
  floatx4 v = {0.f, 0.f, 0.f, 0.f};
  if (lin < nwork) {
    c = chunk_of(lin);
    v = __builtin_nontemporal_load(reinterpret_cast<const floatx4 *>(psi4 + c));
  }
  for (int i = threadIdx.x; i < (1 << a.k); i += kThreads) tab[i] = dtab ? dtab[i] : a.small[i];
  __syncthreads();
  while (lin < nwork) {
    const int64_t y = c << 1;  // first amplitude of the chunk; physical bit 0 is clear
    int r = 0;
    for (int j = 0; j < a.k; ++j) r |= int((y >> a.tgt[j]) & 1) << j;
    const float2 d0 = tab[r], d1 = tab[r | a.bit0];
    const float2 o0 = cmul(d0, make_float2(v.x, v.y));
    const float2 o1 = cmul(d1, make_float2(v.z, v.w));
    const floatx4 o = {o0.x, o0.y, o1.x, o1.y};
    __builtin_nontemporal_store(o, reinterpret_cast<floatx4 *>(psi4 + c));
    lin += step;
    if (lin < nwork) {
      c = chunk_of(lin);
      v = __builtin_nontemporal_load(reinterpret_cast<const floatx4 *>(psi4 + c));
    }
  }
}

// ------------------------------------------------------------------ generic, any k <= 8
struct GenericArgs {
  int k;
  int sorted[8];
  int tgt[8];
};

__global__ __launch_bounds__(kThreads) void k_dense_generic(float2 *__restrict__ psi, int64_t ngroups,
                                                            const float2 *__restrict__ m, GenericArgs a) {
  __shared__ float2 buf[256];
  const int D = 1 << a.k;
  for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
    int64_t base = g;
    for (int j = 0; j < a.k; ++j) base = insert_zero_bit(base, a.sorted[j]);
    for (int c = threadIdx.x; c < D; c += kThreads) {
      int64_t off = 0;
      for (int j = 0; j < a.k; ++j) off |= int64_t((c >> j) & 1) << a.tgt[j];
      buf[c] = psi[base + off];
    }
    __syncthreads();
    for (int r = threadIdx.x; r < D; r += kThreads) {
      float2 acc = make_float2(0.f, 0.f);
      for (int c = 0; c < D; ++c) acc = cfma(m[int64_t(r) * D + c], buf[c], acc);
      int64_t off = 0;
      for (int j = 0; j < a.k; ++j) off |= int64_t((r >> j) & 1) << a.tgt[j];
      psi[base + off] = acc;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ physical bit transposition
// For every index with bit p = 0 and bit q = 0 (p < q), exchange the
// amplitudes at x | 2^q and x | 2^p.  Consecutive threads take consecutive
// values of the remaining bits.
__global__ __launch_bounds__(kThreads) void k_swap_bits(float2 *__restrict__ psi, int64_t m, int p, int q) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t t = int64_t(blockIdx.x) * kThreads + threadIdx.x; t < m; t += stride) {
    const int64_t x = insert_zero_bit(insert_zero_bit(t, p), q);
    const int64_t ia = x | (int64_t(1) << q);
    const int64_t ib = x | (int64_t(1) << p);
    const float2 va = psi[ia];
    const float2 vb = psi[ib];
    psi[ia] = vb;
    psi[ib] = va;
  }
}

// ------------------------------------------------------------------ probabilities and norm
__device__ __forceinline__ double prob_of(float2 a) {
  // Both products are exact in FP64 (24-bit significands), so the one rounding
  // of the sum is the only one, with or without contraction into an FMA.
  return double(a.x) * double(a.x) + double(a.y) * double(a.y);
}

__device__ __forceinline__ int64_t logical_to_physical(int64_t x, int n, const LayoutArg &L) {
  int64_t y = 0;
  for (int q = 0; q < n; ++q) y |= ((x >> q) & 1) << L.pos[q];
  return y;
}

__device__ __forceinline__ uint64_t physical_to_logical(uint64_t y, int n, const LayoutArg &L) {
  uint64_t x = 0;
  for (int q = 0; q < n; ++q) x |= ((y >> L.pos[q]) & 1ull) << q;
  return x;
}

__global__ __launch_bounds__(kThreads) void k_probs(const float2 *__restrict__ psi, int64_t dim, int n,
                                                    double *__restrict__ out, int logical, LayoutArg L) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < dim; i += stride) {
    const int64_t x = stream_chunk(i, dim);
    const int64_t y = logical ? logical_to_physical(x, n, L) : x;
    out[x] = prob_of(psi[y]);
  }
}

// Deterministic two-pass FP64 norm: fixed per-thread ranges, fixed tree.
__global__ __launch_bounds__(kThreads) void k_norm_partial(const float2 *__restrict__ psi, int64_t dim,
                                                           double *__restrict__ partials) {
  __shared__ double red[kThreads];
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  double s = 0.0;
  for (int64_t x = int64_t(blockIdx.x) * kThreads + threadIdx.x; x < dim; x += stride) s += prob_of(psi[x]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kThreads) void k_norm_final(const double *__restrict__ partials, int np,
                                                         double *__restrict__ result) {
  __shared__ double red[kThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += kThreads) s += partials[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *result = red[0];
}

// ------------------------------------------------------------------ sampler
// Fixed-point probability: q = floor(p * 2^62), exact (power-of-two scaling,
// truncating conversion).  Integer sums are exact and order-independent, so
// the block totals do not depend on the reduction tree.  The scaling needs
// 0 <= p < 4 (so that q fits in 64 bits); an entry outside that range (NaN
// included) counts as 0 and raises the caller's bad-input flag, as does any
// sum that wraps past 2^64 on the way to the total T.
__device__ __forceinline__ bool q_ok(double p) { return p >= 0.0 && p < 4.0; }
__device__ __forceinline__ uint64_t fixed_q(double p) { return (uint64_t)(p * 4611686018427387904.0); }

__device__ __forceinline__ uint64_t q_checked(double p, bool &bad) {
  if (!q_ok(p)) {
    bad = true;
    return 0;
  }
  return fixed_q(p);
}

__device__ __forceinline__ uint64_t q_at(const float2 *psi, const double *probs, int64_t i) {
  const double p = psi ? prob_of(psi[i]) : probs[i];
  return q_ok(p) ? fixed_q(p) : 0ull;
}

// a + b, noting a carry out of 64 bits
__device__ __forceinline__ uint64_t add_c(uint64_t a, uint64_t b, bool &wrap) {
  const uint64_t r = a + b;
  wrap |= r < a;
  return r;
}

// Exact total of each 2^10-entry block; workgroups stride over blocks (the
// grid is capped below the 2^32 work-item limit of one dispatch).  Thread t
// takes entries 4t..4t+3 of the block with two 16-byte loads, the wave sums
// by shuffles and four wave totals meet in LDS.  Integer sums do not depend
// on the order, so the totals equal any other summation of the same q_x.
// vec = 0 (a caller's probability array not 16-byte aligned) reads entry by entry.
static_assert((1 << kCdfBlockBits) == 4 * kThreads, "one block = four entries per thread");

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v, bool &wrap) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    const unsigned lo = __shfl_xor(unsigned(v), m), hi = __shfl_xor(unsigned(v >> 32), m);
    v = add_c(v, (uint64_t(hi) << 32) | lo, wrap);
  }
  return v;
}

__global__ void k_clear_flag(unsigned *flag) { *flag = 0u; }

__global__ __launch_bounds__(kThreads) void k_block_totals(const float2 *__restrict__ psi,
                                                           const double *__restrict__ probs, int64_t dim, int64_t nb,
                                                           int vec, uint64_t *__restrict__ blocksum,
                                                           unsigned *__restrict__ bad_flag) {
  __shared__ uint64_t red[kThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  bool bad = false;
  for (int64_t blk = blockIdx.x; blk < nb; blk += gridDim.x) {
    const int64_t x0 = (blk << kCdfBlockBits) + 4 * int64_t(threadIdx.x);
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    if (vec && x0 + 3 < dim) {
      if (psi) {
        const float4 a = reinterpret_cast<const float4 *>(psi)[x0 / 2];
        const float4 b = reinterpret_cast<const float4 *>(psi)[x0 / 2 + 1];
        p[0] = prob_of(make_float2(a.x, a.y));
        p[1] = prob_of(make_float2(a.z, a.w));
        p[2] = prob_of(make_float2(b.x, b.y));
        p[3] = prob_of(make_float2(b.z, b.w));
      } else {
        const double2 a = reinterpret_cast<const double2 *>(probs)[x0 / 2];
        const double2 b = reinterpret_cast<const double2 *>(probs)[x0 / 2 + 1];
        p[0] = a.x;
        p[1] = a.y;
        p[2] = b.x;
        p[3] = b.y;
      }
    } else {
      for (int j = 0; j < 4; ++j)
        if (x0 + j < dim) p[j] = psi ? prob_of(psi[x0 + j]) : probs[x0 + j];
    }
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) s = add_c(s, q_checked(p[j], bad), bad);
    s = wave_sum_u64(s, bad);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t t = 0;
#pragma unroll
      for (int w = 0; w < kThreads / 64; ++w) t = add_c(t, red[w], bad);
      blocksum[blk] = t;
    }
    __syncthreads();
  }
  if (bad) *bad_flag = 1u;
}

// Inclusive scan of 1024-element chunks in place (256 threads x 4), chunk total out.
__global__ __launch_bounds__(kThreads) void k_scan_chunks(uint64_t *__restrict__ v, int64_t nb,
                                                          uint64_t *__restrict__ chunk_total,
                                                          unsigned *__restrict__ bad_flag) {
  __shared__ uint64_t sh[kThreads];
  const int64_t c0 = int64_t(blockIdx.x) * 1024;
  bool wrap = false;
  uint64_t loc[4];
  uint64_t run = 0;
  for (int i = 0; i < 4; ++i) {
    const int64_t idx = c0 + threadIdx.x * 4 + i;
    run = add_c(run, (idx < nb) ? v[idx] : 0ull, wrap);
    loc[i] = run;
  }
  sh[threadIdx.x] = run;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread totals
  for (int off = 1; off < kThreads; off <<= 1) {
    uint64_t add = (threadIdx.x >= off) ? sh[threadIdx.x - off] : 0ull;
    __syncthreads();
    sh[threadIdx.x] = add_c(sh[threadIdx.x], add, wrap);
    __syncthreads();
  }
  const uint64_t excl = (threadIdx.x > 0) ? sh[threadIdx.x - 1] : 0ull;
  for (int i = 0; i < 4; ++i) {
    const int64_t idx = c0 + threadIdx.x * 4 + i;
    if (idx < nb) v[idx] = add_c(loc[i], excl, wrap);
  }
  if (threadIdx.x == kThreads - 1) chunk_total[blockIdx.x] = sh[kThreads - 1];
  if (wrap) *bad_flag = 1u;
}

// One workgroup: exclusive scan of the chunk totals in place (sequential per thread slice).
__global__ __launch_bounds__(kThreads) void k_scan_totals(uint64_t *__restrict__ t, int64_t nc,
                                                          unsigned *__restrict__ bad_flag) {
  __shared__ uint64_t sh[kThreads];
  bool wrap = false;
  const int64_t per = (nc + kThreads - 1) / kThreads;
  const int64_t lo = threadIdx.x * per;
  const int64_t hi = lo + per < nc ? lo + per : nc;
  uint64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s = add_c(s, t[i], wrap);
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    uint64_t add = (threadIdx.x >= off) ? sh[threadIdx.x - off] : 0ull;
    __syncthreads();
    sh[threadIdx.x] = add_c(sh[threadIdx.x], add, wrap);
    __syncthreads();
  }
  uint64_t run = (threadIdx.x > 0) ? sh[threadIdx.x - 1] : 0ull;
  for (int64_t i = lo; i < hi; ++i) {
    const uint64_t v = t[i];
    t[i] = run;
    run = add_c(run, v, wrap);
  }
  if (wrap) *bad_flag = 1u;
}

__global__ __launch_bounds__(kThreads) void k_scan_add(uint64_t *__restrict__ v, int64_t nb,
                                                       const uint64_t *__restrict__ chunk_excl,
                                                       unsigned *__restrict__ bad_flag) {
  const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i < nb) {
    bool wrap = false;
    v[i] = add_c(v[i], chunk_excl[i >> 10], wrap);
    if (wrap) *bad_flag = 1u;
  }
}

// Philox4x32-10 (Salmon et al., SC'11): per round two 32x32 -> 64-bit
// products of counter words 0 and 2 with the multipliers; the high halves are
// mixed into words 1 and 3 with the round key, which grows by the Weyl
// increments after each round.
__device__ __forceinline__ uint64_t philox_draw(uint64_t seed, uint64_t ctr) {
  uint32_t x0 = uint32_t(ctr), x1 = uint32_t(ctr >> 32), x2 = 0u, x3 = 0u;
  uint32_t k0 = uint32_t(seed), k1 = uint32_t(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo_a = 0xD2511F53u * x0, hi_a = __umulhi(0xD2511F53u, x0);
    const uint32_t lo_b = 0xCD9E8D57u * x2, hi_b = __umulhi(0xCD9E8D57u, x2);
    const uint32_t y0 = hi_b ^ x1 ^ k0;
    const uint32_t y2 = hi_a ^ x3 ^ k1;
    x0 = y0;
    x1 = lo_b;
    x2 = y2;
    x3 = lo_a;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return uint64_t(x0) | (uint64_t(x1) << 32);
}

// One wave per shot.  The block is found by binary search over the inclusive
// block prefix; inside the block each lane owns 16 consecutive entries, a wave
// prefix over lane totals finds the owning lane, which then scans its entries.
__global__ __launch_bounds__(kThreads) void k_shots(const float2 *__restrict__ psi,
                                                    const double *__restrict__ probs, int n, int64_t dim,
                                                    const uint64_t *__restrict__ cprefix, int64_t nb,
                                                    uint64_t seed, int64_t shot0, int64_t count, LayoutArg L,
                                                    uint64_t *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t sidx = (int64_t(blockIdx.x) * kThreads + threadIdx.x) >> 6;
  if (sidx >= count) return;  // whole waves exit together
  const uint64_t total = cprefix[nb - 1];
  const uint64_t r = philox_draw(seed, uint64_t(shot0 + sidx));
  const uint64_t t = __umul64hi(r, total);  // floor(r * T / 2^64) < T
  // smallest block b with cprefix[b] > t
  int64_t lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (cprefix[mid] > t)
      hi = mid;
    else
      lo = mid + 1;
  }
  const int64_t b = lo;
  const uint64_t tin = t - (b > 0 ? cprefix[b - 1] : 0ull);
  const int64_t base = b << kCdfBlockBits;
  uint64_t q[16];
  uint64_t mine = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int64_t x = base + lane * 16 + i;
    q[i] = (x < dim) ? q_at(psi, probs, x) : 0ull;
    mine += q[i];
  }
  // inclusive wave prefix of lane totals
  uint64_t incl = mine;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t up = __shfl_up(incl, off);
    if (lane >= off) incl += up;
  }
  const uint64_t excl = incl - mine;
  const unsigned long long owner_mask = __ballot(incl > tin);
  const int owner = __ffsll(owner_mask) - 1;  // the block total exceeds tin, so some lane owns it
  if (lane == owner) {
    uint64_t run = excl;
    int pick = 15;
    for (int i = 0; i < 16; ++i) {
      run += q[i];
      if (run > tin) {
        pick = i;
        break;
      }
    }
    const uint64_t y = uint64_t(base + lane * 16 + pick);
    out[sidx] = physical_to_logical(y, n, L);
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t launch_init_zero(float2 *psi, int n, hipStream_t st) {
  const int64_t dim = int64_t(1) << n;
  if (dim < 4) {
    hipLaunchKernelGGL(k_init_small, dim3(1), dim3(64), 0, st, psi, dim);
  } else {
    const int64_t n4 = dim / 2;
    hipLaunchKernelGGL(k_init_zero, dim3(grid_for(n4, kThreads, kFullGrid)), dim3(kThreads), 0, st,
                       reinterpret_cast<float4 *>(psi), n4, psi);
  }
  return hipGetLastError();
}

template <int K>
static hipError_t dense_valu_k(float2 *psi, int n, const int32_t *A, const float2 *m, hipStream_t st) {
  ValuArgs<K> a;
  for (int i = 0; i < (1 << (2 * K)); ++i) a.m[i] = m[i];
  for (int c = 0; c < (1 << K); ++c) {
    int64_t o = 0;
    for (int j = 0; j < K; ++j)
      if ((c >> j) & 1) o |= int64_t(1) << A[j];
    a.off[c] = o;
  }
  int s[K];
  for (int j = 0; j < K; ++j) s[j] = A[j];
  for (int i = 1; i < K; ++i)
    for (int j = i; j > 0 && s[j - 1] > s[j]; --j) {
      int t = s[j];
      s[j] = s[j - 1];
      s[j - 1] = t;
    }
  for (int j = 0; j < K; ++j) a.sorted[j] = s[j];
  const int64_t ngroups = int64_t(1) << (n - K);
  hipLaunchKernelGGL(k_dense_valu<K>, dim3(grid_for(ngroups, kThreads, kFullGrid)), dim3(kThreads), 0, st, psi,
                     ngroups, a);
  return hipGetLastError();
}

hipError_t launch_dense_valu(float2 *psi, int n, int k, const int32_t *A, const float2 *m, hipStream_t st) {
  switch (k) {
    case 1: return dense_valu_k<1>(psi, n, A, m, st);
    case 2: return dense_valu_k<2>(psi, n, A, m, st);
    case 3: return dense_valu_k<3>(psi, n, A, m, st);
    case 4: return dense_valu_k<4>(psi, n, A, m, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_1q_shuffle(float2 *psi, int n, int b, const float2 *m, hipStream_t st) {
  if (n < 1 || b < 0 || b > 6 || b >= n) return hipErrorInvalidValue;
  const int64_t nchunks = int64_t(1) << (n - 1);
  int64_t blocks = (nchunks + kThreads - 1) / kThreads;
  if (blocks > kFullGrid) blocks = kFullGrid;
  hipLaunchKernelGGL(k_1q_shuffle, dim3(unsigned(blocks)), dim3(kThreads), 0, st,
                     reinterpret_cast<float4 *>(psi), nchunks, b, m[0], m[1], m[2], m[3]);
  return hipGetLastError();
}

hipError_t launch_diag(float2 *psi, int n, int k, const int32_t *A, const float2 *d_dev, const float2 *d_host,
                       int nfix, const int32_t *fix_phys, int fix_val, hipStream_t st) {
  if (k < 1 || k > 8 || k > n || (!d_dev && (!d_host || k > 4)) || nfix < 0 || nfix > k || (nfix && !fix_phys))
    return hipErrorInvalidValue;
  DiagArgs a;
  std::memset(&a, 0, sizeof(a));
  a.k = k;
  if (!d_dev)
    for (int i = 0; i < (1 << k); ++i) a.small[i] = d_host[i];
  for (int j = 0; j < k; ++j) {
    a.tgt[j] = A[j];
    if (A[j] == 0) a.bit0 = 1 << j;
  }
  // fixed bits: distinct positions above physical bit 0, as ascending chunk-bit
  // positions with their values carried along
  std::pair<int, int> fx[8];
  for (int i = 0; i < nfix; ++i) {
    if (fix_phys[i] < 1 || fix_phys[i] >= n) return hipErrorInvalidValue;
    fx[i] = {fix_phys[i] - 1, (fix_val >> i) & 1};
  }
  std::sort(fx, fx + nfix);
  a.nfix = nfix;
  a.fixval = 0;
  for (int i = 0; i < nfix; ++i) {
    if (i > 0 && fx[i].first == fx[i - 1].first) return hipErrorInvalidValue;
    a.fix[i] = fx[i].first;
    a.fixval |= fx[i].second << i;
  }
  // three to five fixed bits, all at physical 13 or below, on states of 2^30
  // amplitudes or more: the fields [14, 19) and [24 - nfix, 29 - nfix) of the
  // work index are disjoint and inside its n - 1 - nfix bits, and the upper
  // one lands at physical bits 25..29 (every fixed bit sits below it)
  a.xhi = 0;
  if (n >= 30 && nfix >= 3 && nfix <= 5 && fx[nfix - 1].first <= 12) a.xhi = 24 - nfix;
  const int64_t nwork = (int64_t(1) << (n - 1)) >> nfix;
  if (a.xhi)
    hipLaunchKernelGGL((k_diag<true>), dim3(grid_for(nwork, kThreads, kFullGrid)), dim3(kThreads), 0, st,
                       reinterpret_cast<float4 *>(psi), nwork, d_dev, a);
  else
    hipLaunchKernelGGL((k_diag<false>), dim3(grid_for(nwork, kThreads, kFullGrid)), dim3(kThreads), 0, st,
                       reinterpret_cast<float4 *>(psi), nwork, d_dev, a);
  return hipGetLastError();
}

hipError_t launch_dense_generic(float2 *psi, int n, int k, const int32_t *A, const float2 *m_dev, hipStream_t st) {
  if (k < 1 || k > 8 || k > n) return hipErrorInvalidValue;
  GenericArgs a;
  a.k = k;
  int s[8];
  for (int j = 0; j < k; ++j) s[j] = a.tgt[j] = A[j];
  for (int i = 1; i < k; ++i)
    for (int j = i; j > 0 && s[j - 1] > s[j]; --j) {
      int t = s[j];
      s[j] = s[j - 1];
      s[j - 1] = t;
    }
  for (int j = 0; j < k; ++j) a.sorted[j] = s[j];
  for (int j = k; j < 8; ++j) a.sorted[j] = a.tgt[j] = 0;
  const int64_t ngroups = int64_t(1) << (n - k);
  hipLaunchKernelGGL(k_dense_generic, dim3(grid_for(ngroups, 1, 1 << 16)), dim3(kThreads), 0, st, psi, ngroups,
                     m_dev, a);
  return hipGetLastError();
}

hipError_t launch_swap_bits(float2 *psi, int n, int p, int q, hipStream_t st) {
  if (p == q || p < 0 || q < 0 || p >= n || q >= n) return hipErrorInvalidValue;
  if (p > q) {
    int t = p;
    p = q;
    q = t;
  }
  const int64_t m = int64_t(1) << (n - 2);
  hipLaunchKernelGGL(k_swap_bits, dim3(grid_for(m, kThreads, kFullGrid)), dim3(kThreads), 0, st, psi, m, p, q);
  return hipGetLastError();
}

hipError_t launch_probs(const float2 *psi, int n, double *out, int logical, const LayoutArg &L, hipStream_t st) {
  const int64_t dim = int64_t(1) << n;
  hipLaunchKernelGGL(k_probs, dim3(grid_for(dim, kThreads, kFullGrid)), dim3(kThreads), 0, st, psi, dim, n, out,
                     logical, L);
  return hipGetLastError();
}

hipError_t launch_norm(const float2 *psi, int n, double *partials, double *result, hipStream_t st) {
  const int64_t dim = int64_t(1) << n;
  const unsigned g = grid_for(dim, kThreads * 16, kNormPartials);
  hipLaunchKernelGGL(k_norm_partial, dim3(g), dim3(kThreads), 0, st, psi, dim, partials);
  hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(kThreads), 0, st, partials, int(g), result);
  return hipGetLastError();
}

hipError_t launch_cdf_build(const float2 *psi, const double *probs, int n, const Workspace &ws, hipStream_t st) {
  const int64_t dim = int64_t(1) << n;
  const int64_t nb = n > kCdfBlockBits ? (int64_t(1) << (n - kCdfBlockBits)) : 1;
  const int64_t gb = nb < (int64_t(1) << 20) ? nb : (int64_t(1) << 20);
  const int vec = (psi || (reinterpret_cast<uintptr_t>(probs) & 15) == 0) ? 1 : 0;
  unsigned *flag = cdf_flag(ws);
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, st, flag);
  hipLaunchKernelGGL(k_block_totals, dim3(unsigned(gb)), dim3(kThreads), 0, st, psi, probs, dim, nb, vec,
                     ws.blocksum, flag);
  const int64_t nc = (nb + 1023) / 1024;
  hipLaunchKernelGGL(k_scan_chunks, dim3(unsigned(nc)), dim3(kThreads), 0, st, ws.blocksum, nb, ws.chunksum, flag);
  if (nc > 1) {
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kThreads), 0, st, ws.chunksum, nc, flag);
    hipLaunchKernelGGL(k_scan_add, dim3(unsigned((nb + kThreads - 1) / kThreads)), dim3(kThreads), 0, st,
                       ws.blocksum, nb, ws.chunksum, flag);
  }
  return hipGetLastError();
}

hipError_t launch_shots(const float2 *psi, const double *probs, int n, const Workspace &ws, uint64_t seed,
                        int64_t shot0, int64_t count, const LayoutArg &L, hipStream_t st) {
  const int64_t dim = int64_t(1) << n;
  const int64_t nb = n > kCdfBlockBits ? (int64_t(1) << (n - kCdfBlockBits)) : 1;
  const int64_t threads = count * 64;
  hipLaunchKernelGGL(k_shots, dim3(unsigned((threads + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, psi,
                     probs, n, dim, ws.blocksum, nb, seed, shot0, count, L, ws.shots);
  return hipGetLastError();
}

}  // namespace sv
