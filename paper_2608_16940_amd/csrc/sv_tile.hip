// LDS-tiled kernels for gfx950.
//
// Dense fused gate on MFMA.  A fused k-qubit gate is a dense contraction
// (Eq. cost-formal: Theta(2^{N+k}) complex multiply-adds): every group of
// 2^k amplitudes that share the non-target bits is multiplied by G.  A
// workgroup owns one tile of 2^(K+M) amplitudes -- the K target bits plus the
// M lowest non-target physical bits -- so every global access is a contiguous
// run of at least 2^M amplitudes whatever the target positions are.  The tile
// is staged in LDS in "local" order (target bits lowest, in gate order, then
// the non-target bits), which makes each group contiguous; each wave then
// multiplies 32 groups at a time on the matrix cores:
//
//   * FP32, k = 4: the real embedding
//       [Re y; Im y] = [[Re G, -Im G], [Im G, Re G]] [Re x; Im x]
//     as a 2^(K+1) x 2^(K+1) by 2^(K+1) x 32 real GEMM (v_mfma_f32_32x32x2f32);
//   * FP32, k >= 5: the three-multiplication complex product
//       T1 = Gr Xr, T2 = Gi Xi, T3 = (Gr + Gi)(Xr + Xi),
//       Re y = T1 - T2, Im y = T3 - T1 - T2,
//     three 2^K x 2^K real GEMMs, 25% fewer MFMA cycles than the embedding;
//     only Gr and Gi are stored, Gr + Gi is one VALU add per step;
//   * BF16x3: each operand split x = hi + lo in bf16 and hi*hi + hi*lo +
//     lo*hi accumulated in FP32; G is split once on the host from FP64.  At
//     k = 4 the real embedding on v_mfma_f32_32x32x8bf16_1k (16 output rows
//     fill a 32-row tile only when embedded); at k >= 5 the four real GEMMs
//       Re y = Gr Xr - Gi Xi,  Im y = Gi Xr + Gr Xi
//     on gfx950's v_mfma_f32_32x32x16_bf16 (twice the rate of the 32x32x8
//     form), with only the Gr and Gi planes stored (half the embedding's
//     bytes) and -Xi formed by flipping sign bits.
//
// Operand layout.  The reduction ordering is free, so lane l of a wave holds
// group (l mod 32) and the contiguous half h = l / 32 of its inputs; MFMA step
// kk consumes the lane's kk-th input value.  The output rows are permuted on
// the host so that accumulator register r of output tile mt of lane l is the
// same contiguous half of the same group: results go back in place.
//
// The store side can read the tile with a different bit map (loc_out), which
// relabels bits inside the tile for free (the lazy relabel L' = alpha o L of
// Algorithm 2, restricted to the tile's bits).  Without a gate the same
// structure is an in-place bit permutation in one sweep (k_tile_permute).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sv_internal.h"
#include "sv_permute_host.h"

namespace sv {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ floatx16 mfma_bf16x16(uint4 a, uint4 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                  0, 0);
}
__device__ __forceinline__ uint4 flip_sign(uint4 x) {
  return make_uint4(x.x ^ 0x80008000u, x.y ^ 0x80008000u, x.z ^ 0x80008000u, x.w ^ 0x80008000u);
}

// Amplitudes are touched exactly once per sweep: stream them with
// non-temporal loads and stores so they do not displace cached operands.
__device__ __forceinline__ float4 ld_stream(const float2 *p) {
  const floatx4 v = __builtin_nontemporal_load(reinterpret_cast<const floatx4 *>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_stream(float2 *p, float2 a, float2 b) {
  const floatx4 v = {a.x, a.y, b.x, b.y};
  __builtin_nontemporal_store(v, reinterpret_cast<floatx4 *>(p));
}

struct TileArgs {
  float2 *psi;
  const void *op;
  int64_t ntiles;
  int s;
  int xs;             // workgroup-to-tile order (tile_of): 0 plain
  int lb_in, lb_out;  // local bit of tile-order bit 0 on load / store
  int sbit[24];
  int loc_in[24];
  int loc_out[24];
  int64_t goff_i[32];
  int32_t lam_i[32];
  int32_t lamo_i[32];
  int32_t pswz[7];  // k_tile_permute: LDS swizzle images of local bits 5..11 (lin_swz)
};

__device__ __forceinline__ int64_t insert_zero_bit(int64_t x, int p) {
  const int64_t low = x & ((int64_t(1) << p) - 1);
  return ((x >> p) << (p + 1)) | low;
}

// Tile taken by work index w (the workgroup index, plus multiples of the grid
// size when a workgroup loops).  Workgroups are handed to the eight XCDs in
// turn, so the three low bits of w name the XCD; with xs > 0 they become tile
// bits xs..xs+2 and bits 3..xs+2 of w move down, so that each XCD walks runs
// of 2^xs consecutive tiles.  A bijection on [0, ntiles) when ntiles is a
// power of two of at least 2^(xs+3) (the host checks).
__device__ __forceinline__ int64_t tile_of(int64_t w, int xs) {
  if (xs <= 0) return w;
  return ((w >> 3) & ((int64_t(1) << xs) - 1)) | ((w & 7) << xs) | ((w >> (xs + 3)) << (xs + 3));
}

// LDS address of local index lam (amplitude units).  The low K bits (position
// inside a group) are XOR-ed with a function of the group index so that the
// 32 groups a wave reads at once fall in 32 distinct 8-byte bank slots.
template <int K>
__device__ __forceinline__ int swz(int lam) {
  const int g = lam >> K;
  const int f = (K >= 5) ? (g & 31) : ((g >> 1) & ((1 << K) - 1));
  return lam ^ f;
}

__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float(unsigned(h) << 16); }

// BF16x3 split of one amplitude, packed in the 8 bytes of its LDS slot:
// (hi(re) | hi(im) << 16, lo(re) | lo(im) << 16) with hi = RNE bf16 of the
// value and lo = RNE bf16 of the residual.  Splitting once when the tile
// lands in LDS spares every wave that reads a group from repeating it.
__device__ __forceinline__ uint2 bf16x3_split(float re, float im) {
  const unsigned short hr = bf16_rne(re), hm = bf16_rne(im);
  const unsigned short lr = bf16_rne(re - bf16_to_f(hr)), lm = bf16_rne(im - bf16_to_f(hm));
  return make_uint2(unsigned(hr) | (unsigned(hm) << 16), unsigned(lr) | (unsigned(lm) << 16));
}

// Where a wave finds the gate operand: its own registers (loaded once per
// workgroup), the workgroup's LDS (loaded once, read per MFMA), or global
// memory through the caches (read per MFMA; only for the widest gates).
enum OpSrc { OP_REG = 0, OP_LDS = 1, OP_GLOBAL = 2 };
// Arithmetic scheme.
enum Alg { ALG_EMBED_F32 = 0, ALG_GAUSS_F32 = 1, ALG_EMBED_BF16X3 = 2, ALG_CPLX_BF16X3 = 3 };

template <int K, int PREC>
struct Scheme {
  static constexpr int alg = (PREC == SV_PREC_BF16X3) ? (K >= 5 ? ALG_CPLX_BF16X3 : ALG_EMBED_BF16X3)
                                                      : (K >= 5 ? ALG_GAUSS_F32 : ALG_EMBED_F32);
  // operand bytes (see pack_mfma_operand): two FP32 planes, four bf16 planes, or the embedding
  static constexpr int bytes = (alg == ALG_GAUSS_F32 || alg == ALG_CPLX_BF16X3) ? (1 << (2 * K + 3)) : (1 << (2 * K + 4));
};

// Reduction split: at k = 7 with the operand in LDS (128 KiB: one workgroup
// per CU) eight waves work on a tile, two per output tile, each over half of
// the reduction; the two partial sums meet in LDS (upper half first, then the
// lower half adds its own), so the matrix cores have two waves per SIMD to
// draw from instead of one.
template <int K, int PREC, int OPS>
struct KSplit {
  static constexpr int value = (K == 7 && OPS == OP_LDS) ? 2 : 1;
};

// Occupancy target (waves per SIMD the register budget is cut for).  FP32
// k=5 with the operand in LDS fits four 40 KiB workgroups per CU in 125
// VGPRs; the other k=5 forms would spill at that budget and keep three.
template <int K, int PREC, int OPS>
struct WavesPerSimd {
  static constexpr int value =
      K <= 4 ? 4 : (K == 5 ? ((PREC == SV_PREC_FP32 && OPS == OP_LDS) ? 4 : 3) : ((K == 7 && OPS == OP_LDS) ? 1 : 2)) *
                       KSplit<K, PREC, OPS>::value;
};

// Register prefetch of the next tile: measured at N=30 on MI355X, FP32 k=6
// 6.0 -> 4.1 ms, FP32 k=7 10.2 -> 9.7 ms, BF16x3 k=6 5.5 -> 5.3 ms, BF16x3 k=7
// (complex form, operand in LDS, one workgroup per CU) 4.3 -> 3.8 ms; the
// memory-bound k <= 5 sweeps are as fast or faster without it.
template <int K, int PREC>
struct Prefetch {
  static constexpr bool value = K >= 6;
};
constexpr int kPrefetchGridPerCU = 16;

template <int K, int M, int PREC, int OPS>
__global__ __launch_bounds__((256 * KSplit<K, PREC, OPS>::value), (WavesPerSimd<K, PREC, OPS>::value)) void k_tile_mfma(
    TileArgs a) {
  constexpr int KSP = KSplit<K, PREC, OPS>::value;
  constexpr int NT = 256 * KSP;         // four waves per reduction part
  constexpr int TB = (KSP == 2) ? 9 : 8;  // thread bits: tile-order bits 1..TB
  constexpr int S = K + M;
  constexpr int TILE = 1 << S;
  constexpr int CHUNKS = TILE / 2 / NT;  // 16-byte chunks per thread per tile
  constexpr int AH = 1 << (K - 1);       // amplitudes per lane half
  constexpr int ALG = Scheme<K, PREC>::alg;
  constexpr int NOPF = Scheme<K, PREC>::bytes / 4;  // operand size in floats
  constexpr int HALF = 1 << K;           // embedding: reals per lane half
  constexpr int KQ = HALF / 4;
  constexpr bool CPLX_ROWS = (ALG == ALG_GAUSS_F32 || ALG == ALG_CPLX_BF16X3);  // output rows are amplitudes
  constexpr int MTT = CPLX_ROWS ? (1 << K) / 32 : (2 << K) / 32;  // 32-row output tiles
  constexpr int NCB = (1 << M) / 32;     // 32-group column blocks per tile
  static_assert(MTT * NCB >= 4 && (MTT * NCB) % 4 == 0, "four waves share the (block, tile) pairs");
  constexpr int MPW = MTT * NCB / 4;     // output tiles per wave
  constexpr bool SHARED_GROUPS = NCB < 4;  // several waves work on the same groups
  // BF16x3 k >= 6: the cross terms hi*lo and lo*hi accumulate apart from
  // hi*hi (independent MFMA chains per output tile; 5-10% faster at N=30,
  // a third set costs occupancy); summed in FP32 before the store
  constexpr int BSETS = (ALG == ALG_CPLX_BF16X3 && K >= 6) ? 2 : 1;
  constexpr int NACC = (ALG == ALG_GAUSS_F32) ? 3 * MPW : (ALG == ALG_CPLX_BF16X3 ? 2 : 1) * BSETS * MPW;
  // BF16x3 complex form: the inputs are split into bf16 hi/lo once, as the
  // tile lands in LDS (the packed pair takes the float2's 8 bytes), and each
  // step gathers the halves of eight amplitudes from those pairs; the k = 4
  // embedding splits inside its product loop
  constexpr bool SPLIT_AT_LOAD = (ALG == ALG_CPLX_BF16X3);
  __shared__ float2 lds[TILE];
  __shared__ float opl_s[OPS == OP_LDS ? NOPF : 1];

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;

  int64_t goff_t = 0;
  int lam_t = 0, lamo_t = 0;
#pragma unroll
  for (int b = 1; b <= TB; ++b) {  // without branches, the kernel arguments load in a few batches
    const int on = (t >> (b - 1)) & 1;
    goff_t |= int64_t(on) << a.sbit[b];
    lam_t |= on << a.loc_in[b];
    lamo_t |= on << a.loc_out[b];
  }
  const int bin = 1 << a.lb_in, bout = 1 << a.lb_out;

  // wave -> reduction part, column block and its output tiles mt0 + j * (4 / NCB)
  const int ks = wave >> 2;
  const int cb = (wave & 3) % NCB;
  const int mt0 = (wave & 3) / NCB;
  constexpr int MT_STEP = 4 / NCB;

  // ---- operand
  const float *opf = reinterpret_cast<const float *>(a.op);
  constexpr int NREG = (OPS == OP_REG) ? NOPF / 64 : 1;
  float ra[NREG];
  (void)ra;
  if constexpr (OPS == OP_REG) {
    if constexpr (ALG == ALG_CPLX_BF16X3) {
      // 16 bytes (eight bf16) per lane and unit
      const float4 *op4 = reinterpret_cast<const float4 *>(a.op);
#pragma unroll
      for (int i = 0; i < NREG / 4; ++i) {
        const float4 t = op4[i * 64 + lane];
        ra[4 * i] = t.x;
        ra[4 * i + 1] = t.y;
        ra[4 * i + 2] = t.z;
        ra[4 * i + 3] = t.w;
      }
    } else if constexpr (ALG == ALG_EMBED_BF16X3) {
      // the bf16 operand holds one 8-byte group of four per lane: floats (2i, 2i + 1) of this lane
      const float2 *op2 = reinterpret_cast<const float2 *>(a.op);
#pragma unroll
      for (int i = 0; i < NREG / 2; ++i) {
        const float2 t = op2[i * 64 + lane];
        ra[2 * i] = t.x;
        ra[2 * i + 1] = t.y;
      }
    } else {
#pragma unroll
      for (int i = 0; i < NREG; ++i) ra[i] = opf[i * 64 + lane];
    }
  }
  // LDS operand.  At k = 5 (two 16-byte pieces per thread) it is loaded
  // straight into LDS, bypassing registers, so the tile loads that follow go
  // out at once instead of after the operand's round trip (copied through
  // registers, each piece waited for its load before the tile loads were
  // issued); its arrival is awaited before the first barrier.  Measured at
  // N=30: the k=5 FP32 sweep 3.22 -> 3.10 ms on average over 146 target
  // sets, BF16x3 2.98 -> 2.86; k = 4 was 1-3% slower with it and k = 6, 7
  // (a persistent grid, where the copy happens once) unchanged, so they copy.
  constexpr bool OP_EARLY = (OPS == OP_LDS) && K == 5 && (NOPF / 4 <= 2 * NT) && (NOPF / 4) % 64 == 0;
  if constexpr (OPS == OP_LDS) {
    const float4 *src = reinterpret_cast<const float4 *>(a.op);
    float4 *dst = reinterpret_cast<float4 *>(opl_s);
    if constexpr (OP_EARLY) {
      const int w0 = __builtin_amdgcn_readfirstlane(wave) * 64;  // this wave's first piece
#pragma unroll
      for (int i = 0; i < (NOPF / 4 + NT - 1) / NT; ++i)
        if (i * NT + w0 < NOPF / 4)  // whole waves: NOPF / 4 is a multiple of 64
          __builtin_amdgcn_global_load_lds(src + i * NT + w0 + lane,
                                           (__attribute__((address_space(3))) void *)(dst + i * NT + w0), 16, 0, 0);
    } else {
      for (int i = t; i < NOPF / 4; i += NT) dst[i] = src[i];
    }
  }
  const float *opsrc = (OPS == OP_LDS) ? static_cast<const float *>(opl_s) : opf;
  // operand float i of this lane (i indexes the lane-major packing)
  auto opv = [&](int i) -> float {
    if constexpr (OPS == OP_REG)
      return ra[i];
    else
      return opsrc[i * 64 + lane];
  };

  const int g = 32 * cb + (lane & 31);
  const int h = lane >> 5;
  const int gbase = g << K;

  // Compute-bound widths (Prefetch<>) run a persistent grid and load the next
  // tile into registers while the matrix cores work on this one; the others
  // take one tile per workgroup over a full grid.
  constexpr bool PF = Prefetch<K, PREC>::value;
  auto tile_base = [&](int64_t tl) {
    int64_t b0 = tl;
#pragma unroll
    for (int b = 0; b < S; ++b) b0 = insert_zero_bit(b0, a.sbit[b]);
    return b0;
  };
  float4 v[CHUNKS];  // this tile's 16-byte chunks (global -> LDS)
  int64_t nbase = 0;
  if (PF && int64_t(blockIdx.x) < a.ntiles) {
    nbase = tile_base(tile_of(blockIdx.x, a.xs));
#pragma unroll
    for (int i = 0; i < CHUNKS; ++i) v[i] = ld_stream(a.psi + nbase + goff_t + a.goff_i[i]);
  }
  for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const int64_t base = PF ? nbase : tile_base(tile_of(tile, a.xs));
    if (!PF) {
#pragma unroll
      for (int i = 0; i < CHUNKS; ++i) v[i] = ld_stream(a.psi + base + goff_t + a.goff_i[i]);
    }
#pragma unroll
    for (int i = 0; i < CHUNKS; ++i) {
      const int l0 = lam_t | a.lam_i[i];
      if constexpr (SPLIT_AT_LOAD) {
        uint2 *ldsu = reinterpret_cast<uint2 *>(lds);
        ldsu[swz<K>(l0)] = bf16x3_split(v[i].x, v[i].y);
        ldsu[swz<K>(l0 | bin)] = bf16x3_split(v[i].z, v[i].w);
      } else {
        lds[swz<K>(l0)] = make_float2(v[i].x, v[i].y);
        lds[swz<K>(l0 | bin)] = make_float2(v[i].z, v[i].w);
      }
    }
    if (OP_EARLY && tile == int64_t(blockIdx.x)) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the operand is in LDS
    __syncthreads();
    if (PF && tile + gridDim.x < a.ntiles) {
      nbase = tile_base(tile_of(tile + gridDim.x, a.xs));
#pragma unroll
      for (int i = 0; i < CHUNKS; ++i) v[i] = ld_stream(a.psi + nbase + goff_t + a.goff_i[i]);
    }

    floatx16 acc[NACC];
#pragma unroll
    for (int m = 0; m < NACC; ++m)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[m][r] = 0.f;

    if constexpr (ALG == ALG_GAUSS_F32) {
      // step kk uses amplitude (AH h + kk) of this lane's group
      // unroll depth of the product loop, measured at N=30 on MI355X: k = 5
      // rolled (5-7% faster than 8 steps at every target pattern), k = 6 and 7
      // with the operand in LDS fully unrolled (9% and 15% faster); the
      // cache-operand forms would spill fully unrolled and keep 8 steps
      constexpr int AHP = AH / KSP;  // steps of one reduction part
      constexpr int UNR = (K == 5) ? 1 : (OPS == OP_LDS ? AHP : 8);
#pragma unroll UNR
      for (int k2 = 0; k2 < AHP; ++k2) {
        const int kk = ks * AHP + k2;
        const float2 x = lds[swz<K>(gbase | (h * AH + kk))];
        const float xs = x.x + x.y;
#pragma unroll
        for (int j = 0; j < MPW; ++j) {
          const int mt = mt0 + j * MT_STEP;
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(opv((0 * MTT + mt) * AH + kk), x.x, acc[j], 0, 0, 0);
          acc[MPW + j] =
              __builtin_amdgcn_mfma_f32_32x32x2f32(opv((1 * MTT + mt) * AH + kk), x.y, acc[MPW + j], 0, 0, 0);
          // third Gauss operand Gr + Gi formed here: two planes keep the k=5 workgroup at 40 KiB of LDS
          acc[2 * MPW + j] = __builtin_amdgcn_mfma_f32_32x32x2f32(
              opv((0 * MTT + mt) * AH + kk) + opv((1 * MTT + mt) * AH + kk), xs, acc[2 * MPW + j], 0, 0, 0);
        }
      }
      if constexpr (SHARED_GROUPS) __syncthreads();  // sibling waves finished reading these groups
      // a split reduction: the upper part stores its partial sums, the lower part adds its own
#pragma unroll
      for (int part = KSP - 1; part >= 0; --part) {
        if (part < KSP - 1) __syncthreads();
        if (ks == part) {
#pragma unroll
          for (int j = 0; j < MPW; ++j) {
            const int mt = mt0 + j * MT_STEP;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const float t1 = acc[j][r], t2 = acc[MPW + j][r], t3 = acc[2 * MPW + j][r];
              float2 y = make_float2(t1 - t2, t3 - t1 - t2);
              const int ix = swz<K>(gbase | (h * AH + 16 * mt + r));
              if (part < KSP - 1) {
                const float2 q = lds[ix];
                y.x += q.x;
                y.y += q.y;
              }
              lds[ix] = y;
            }
          }
        }
      }
    } else if constexpr (ALG == ALG_EMBED_F32) {
      static_assert(KSP == 1, "the embedding forms (k = 4) keep one reduction part");
      // step kk uses real (HALF h + kk) of this lane's group
#pragma unroll
      for (int kk = 0; kk < HALF; ++kk) {
        const float2 x = lds[swz<K>(gbase | (h * AH + (kk >> 1)))];
        const float xv = (kk & 1) ? x.y : x.x;
#pragma unroll
        for (int j = 0; j < MPW; ++j) {
          const int mt = mt0 + j * MT_STEP;
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(opv(mt * HALF + kk), xv, acc[j], 0, 0, 0);
        }
      }
      if constexpr (SHARED_GROUPS) __syncthreads();
#pragma unroll
      for (int j = 0; j < MPW; ++j) {
        const int mt = mt0 + j * MT_STEP;
#pragma unroll
        for (int e = 0; e < 8; ++e)
          lds[swz<K>(gbase | (h * AH + 8 * mt + e))] = make_float2(acc[j][2 * e], acc[j][2 * e + 1]);
      }
    } else if constexpr (ALG == ALG_EMBED_BF16X3) {
      static_assert(KSP == 1, "the embedding forms (k = 4) keep one reduction part");
      // k = 4 only (the complex form takes k >= 5)
      const shortx4 *oph = reinterpret_cast<const shortx4 *>(opsrc);
#pragma unroll
      for (int kk = 0; kk < KQ; ++kk) {
        // four reals = two amplitudes (AH h + 2 kk, +1)
        shortx4 bh, bl;
        const float2 x0 = lds[swz<K>(gbase | (h * AH + 2 * kk))];
        const float2 x1 = lds[swz<K>(gbase | (h * AH + 2 * kk + 1))];
        const float xr[4] = {x0.x, x0.y, x1.x, x1.y};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const unsigned short hi = bf16_rne(xr[e]);
          const unsigned short lo = bf16_rne(xr[e] - bf16_to_f(hi));
          bh[e] = short(hi);
          bl[e] = short(lo);
        }
#pragma unroll
        for (int j = 0; j < MPW; ++j) {
          const int mt = mt0 + j * MT_STEP;
          shortx4 ah, al;
          if constexpr (OPS == OP_REG) {
            const int ih = 2 * (mt * KQ + kk), il = 2 * (MTT * KQ + mt * KQ + kk);
            ah = __builtin_bit_cast(shortx4, make_float2(ra[ih], ra[ih + 1]));
            al = __builtin_bit_cast(shortx4, make_float2(ra[il], ra[il + 1]));
          } else {
            ah = oph[(mt * KQ + kk) * 64 + lane];
            al = oph[(MTT * KQ + mt * KQ + kk) * 64 + lane];
          }
          constexpr int XS = (BSETS - 1) * MPW;  // cross-term accumulator offset
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, bh, acc[j], 0, 0, 0);
          acc[XS + j] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, bl, acc[XS + j], 0, 0, 0);
          acc[XS + j] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(al, bh, acc[XS + j], 0, 0, 0);
        }
      }
      if constexpr (SHARED_GROUPS) __syncthreads();
#pragma unroll
      for (int j = 0; j < MPW; ++j) {
        const int mt = mt0 + j * MT_STEP;
#pragma unroll
        for (int r = 0; r < 16; ++r)
          for (int t = 1; t < BSETS; ++t) acc[j][r] += acc[t * MPW + j][r];
#pragma unroll
        for (int e = 0; e < 8; ++e)
          lds[swz<K>(gbase | (h * AH + 8 * mt + e))] = make_float2(acc[j][2 * e], acc[j][2 * e + 1]);
      }
    } else {
      // complex form: step kk reduces over amplitudes AH h + 8 kk + e (e < 8) of this
      // lane's group; operand unit ((P MTT + mt) KS + kk) holds plane P in
      // (Gr hi, Gr lo, Gi hi, Gi lo) for those eight columns
      constexpr int KS = AH / 8;
      constexpr int KSS = KS / KSP;  // steps of one reduction part
      constexpr int UNR = (OPS == OP_LDS && K >= 6) ? KSS : (K == 5 ? 1 : 2);  // wider unrolls spill
      constexpr int XS = (BSETS - 1) * MPW;  // cross-term accumulator offset
      floatx16 *accR = acc, *accI = acc + BSETS * MPW;
      const uint2 *ldsu = reinterpret_cast<const uint2 *>(lds);
      auto opq = [&](int q) -> uint4 {
        if constexpr (OPS == OP_REG)
          return make_uint4(__float_as_uint(ra[4 * q]), __float_as_uint(ra[4 * q + 1]), __float_as_uint(ra[4 * q + 2]),
                            __float_as_uint(ra[4 * q + 3]));
        else
          return reinterpret_cast<const uint4 *>(opsrc)[q * 64 + lane];
      };
#pragma unroll UNR
      for (int k2 = 0; k2 < KSS; ++k2) {
        const int kk = ks * KSS + k2;
        uint2 sl[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) sl[e] = ldsu[swz<K>(gbase | (h * AH + 8 * kk + e))];
        // slot = (hi re | hi im << 16, lo re | lo im << 16): gather each half of eight amplitudes
        uint32_t rh[4], ih[4], rl[4], il[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const uint2 a0 = sl[2 * p], a1 = sl[2 * p + 1];
          rh[p] = (a0.x & 0xFFFFu) | (a1.x << 16);
          ih[p] = (a0.x >> 16) | (a1.x & 0xFFFF0000u);
          rl[p] = (a0.y & 0xFFFFu) | (a1.y << 16);
          il[p] = (a0.y >> 16) | (a1.y & 0xFFFF0000u);
        }
        const uint4 xrh = make_uint4(rh[0], rh[1], rh[2], rh[3]), xih = make_uint4(ih[0], ih[1], ih[2], ih[3]);
        const uint4 xrl = make_uint4(rl[0], rl[1], rl[2], rl[3]), xil = make_uint4(il[0], il[1], il[2], il[3]);
        const uint4 nxih = flip_sign(xih), nxil = flip_sign(xil);
#pragma unroll
        for (int j = 0; j < MPW; ++j) {
          const int mt = mt0 + j * MT_STEP;
          const uint4 grh = opq((0 * MTT + mt) * KS + kk), grl = opq((1 * MTT + mt) * KS + kk);
          const uint4 gih = opq((2 * MTT + mt) * KS + kk), gil = opq((3 * MTT + mt) * KS + kk);
          accR[j] = mfma_bf16x16(grh, xrh, accR[j]);
          accI[j] = mfma_bf16x16(gih, xrh, accI[j]);
          accR[j] = mfma_bf16x16(gih, nxih, accR[j]);
          accI[j] = mfma_bf16x16(grh, xih, accI[j]);
          accR[XS + j] = mfma_bf16x16(grh, xrl, accR[XS + j]);
          accI[XS + j] = mfma_bf16x16(gih, xrl, accI[XS + j]);
          accR[XS + j] = mfma_bf16x16(grl, xrh, accR[XS + j]);
          accI[XS + j] = mfma_bf16x16(gil, xrh, accI[XS + j]);
          accR[XS + j] = mfma_bf16x16(gih, nxil, accR[XS + j]);
          accI[XS + j] = mfma_bf16x16(grh, xil, accI[XS + j]);
          accR[XS + j] = mfma_bf16x16(gil, nxih, accR[XS + j]);
          accI[XS + j] = mfma_bf16x16(grl, xih, accI[XS + j]);
        }
      }
      if constexpr (SHARED_GROUPS) __syncthreads();
      // a split reduction: the upper part stores its partial sums, the lower part adds its own
#pragma unroll
      for (int part = KSP - 1; part >= 0; --part) {
        if (part < KSP - 1) __syncthreads();
        if (ks == part) {
#pragma unroll
          for (int j = 0; j < MPW; ++j) {
            const int mt = mt0 + j * MT_STEP;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              float re = accR[j][r], im = accI[j][r];
              if constexpr (BSETS > 1) {
                re += accR[XS + j][r];
                im += accI[XS + j][r];
              }
              const int ix = swz<K>(gbase | (h * AH + 16 * mt + r));
              if (part < KSP - 1) {
                const float2 q = lds[ix];
                re += q.x;
                im += q.y;
              }
              lds[ix] = make_float2(re, im);
            }
          }
        }
      }
    }
    __syncthreads();

    // ---- LDS -> global
#pragma unroll
    for (int i = 0; i < CHUNKS; ++i) {
      const int l0 = lamo_t | a.lamo_i[i];
      st_stream(a.psi + base + goff_t + a.goff_i[i], lds[swz<K>(l0)], lds[swz<K>(l0 | bout)]);
    }
    __syncthreads();
  }
}

// LDS address of local index l in the permutation tile: l ^ X(l >> 5), where
// X is linear over GF(2) (bit 5 + j of l contributes pswz[j] to the low five
// bits).  The map is a bijection and linear, so the address of a thread's
// part OR a chunk's part (disjoint bits) is the XOR of the parts' addresses.
__device__ __forceinline__ int lin_swz(int l, const int32_t *px) {
  int x = 0;
#pragma unroll
  for (int j = 0; j < 7; ++j) x ^= -((l >> (5 + j)) & 1) & px[j];  // no branches
  return l ^ x;
}

// In-place bit permutation of the tile's bits in one sweep.  The tile lands
// in LDS in tile order and leaves it through the permuted map, so the two
// phases read LDS along different bits; the host picks X so that the 64
// lanes of each wave instruction spread over all LDS banks in both phases
// (without it a wave's reads along high tile bits hit one bank 8 to 64
// times: one pass ran at 44% of HBM peak).  lam_i / lamo_i hold the chunks'
// swizzled addresses.
template <int S>
__global__ __launch_bounds__(256) void k_tile_permute(TileArgs a) {
  static_assert(S == 12, "the swizzle covers local bits 5..11");  // kPermTileBits
  constexpr int NT = 256;
  constexpr int CHUNKS = (1 << (S - 1)) / NT;
  __shared__ float2 lds[1 << S];
  const int t = threadIdx.x;
  int64_t goff_t = 0;
  int lamo_t = 0;
#pragma unroll
  for (int b = 1; b <= 8; ++b) {  // without branches, as in k_tile_mfma
    const int on = (t >> (b - 1)) & 1;
    goff_t |= int64_t(on) << a.sbit[b];
    lamo_t |= on << a.loc_out[b];
  }
  const int wr_t = lin_swz(2 * t, a.pswz);   // identity on load: local index 2t + 512 i
  const int rd_t = lin_swz(lamo_t, a.pswz);
  const int rd_b = lin_swz(1 << a.lb_out, a.pswz);
  for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    int64_t base = tile_of(tile, a.xs);
#pragma unroll
    for (int b = 0; b < S; ++b) base = insert_zero_bit(base, a.sbit[b]);
    float4 v[CHUNKS];
#pragma unroll
    for (int i = 0; i < CHUNKS; ++i) v[i] = ld_stream(a.psi + base + goff_t + a.goff_i[i]);
#pragma unroll
    for (int i = 0; i < CHUNKS; ++i) {
      const int l0 = wr_t ^ a.lam_i[i];
      lds[l0] = make_float2(v[i].x, v[i].y);
      lds[l0 ^ 1] = make_float2(v[i].z, v[i].w);  // X reads bits 5..11 only: f(l ^ 1) = f(l) ^ 1
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CHUNKS; ++i) {
      const int l0 = rd_t ^ a.lamo_i[i];
      st_stream(a.psi + base + goff_t + a.goff_i[i], lds[l0], lds[l0 ^ rd_b]);
    }
    __syncthreads();
  }
}

int64_t pdep_host(uint64_t v, const int *sbit, int s) {
  int64_t o = 0;
  for (int b = 0; b < s; ++b)
    if ((v >> b) & 1) o |= int64_t(1) << sbit[b];
  return o;
}
int32_t lam_host(uint64_t v, const int *loc, int s) {
  int32_t o = 0;
  for (int b = 0; b < s; ++b)
    if ((v >> b) & 1) o |= 1 << loc[b];
  return o;
}

// Default workgroup-to-tile order (SV_OPT_TILE_ORDER = -1).
constexpr int kDefaultTileOrder = 0;

void fill_args(const TilePlan &tp, int nt, int chunks, float2 *psi, const void *op, TileArgs *a) {
  std::memset(a, 0, sizeof(*a));
  a->psi = psi;
  a->op = op;
  a->s = tp.s;
  a->ntiles = int64_t(1) << (tp.n - tp.s);
  a->xs = tp.order < 0 ? kDefaultTileOrder : tp.order;
  if (a->xs > 0 && tp.n - tp.s < a->xs + 3) a->xs = 0;
  for (int b = 0; b < tp.s; ++b) {
    a->sbit[b] = tp.sbit[b];
    a->loc_in[b] = tp.loc_in[b];
    a->loc_out[b] = tp.loc_out[b];
  }
  a->lb_in = tp.loc_in[0];
  a->lb_out = tp.loc_out[0];
  for (int i = 0; i < chunks; ++i) {
    const uint64_t v = uint64_t(2) * uint64_t(i) * uint64_t(nt);
    a->goff_i[i] = pdep_host(v, tp.sbit, tp.s);
    a->lam_i[i] = lam_host(v, tp.loc_in, tp.s);
    a->lamo_i[i] = lam_host(v, tp.loc_out, tp.s);
  }
}

// One tile per workgroup: the dispatcher then walks memory in order, which
// measured faster than persistent workgroups striding over the state.
// A dispatch holds at most 2^32 - 1 work-items: 2^22 workgroups of 256 stay
// well inside it; the kernels loop over the remaining tiles.
unsigned grid_of(int64_t ntiles) { return unsigned(ntiles > (int64_t(1) << 22) ? (int64_t(1) << 22) : ntiles); }

template <int K, int M, int PREC, int OPS>
hipError_t tile_mfma_k(const TilePlan &tp, float2 *psi, const void *op, hipStream_t st) {
  constexpr int NT = 256 * KSplit<K, PREC, OPS>::value;
  constexpr int CHUNKS = (1 << (K + M)) / 2 / NT;
  TileArgs a;
  fill_args(tp, NT, CHUNKS, psi, op, &a);
  int64_t tiles = a.ntiles;
  if (Prefetch<K, PREC>::value) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    tiles = std::min<int64_t>(tiles, int64_t(cus) * kPrefetchGridPerCU);
  }
  hipLaunchKernelGGL((k_tile_mfma<K, M, PREC, OPS>), dim3(grid_of(tiles)), dim3(NT), 0, st, a);
  return hipGetLastError();
}

double re_of(const double *G, int D, int r, int c) { return G[2 * (r * D + c)]; }
double im_of(const double *G, int D, int r, int c) { return G[2 * (r * D + c) + 1]; }

// entry (orow, icol) of the real embedding [[Re G, -Im G], [Im G, Re G]] with
// interleaved (re, im) rows and columns
double embedded(const double *G, int K, int orow, int icol) {
  const int D = 1 << K;
  const int r = orow >> 1, po = orow & 1, c = icol >> 1, pi = icol & 1;
  const double gr = re_of(G, D, r, c), gi = im_of(G, D, r, c);
  return (po == pi) ? gr : (po == 0 ? -gi : gi);
}

uint16_t host_bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
float host_bf16_to_f(uint16_t h) {
  uint32_t u = uint32_t(h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// bf16 neighbour of h one unit in the last place toward +inf (dir > 0) or -inf.
uint16_t bf16_step(uint16_t h, int dir) {
  const bool neg = (h & 0x8000u) != 0;
  const uint16_t mag = h & 0x7FFFu;
  if (mag == 0) return uint16_t(dir > 0 ? 0x0001u : 0x8001u);
  return uint16_t((dir > 0) != neg ? h + 1 : h - 1);
}

// Split every component of G into bf16 hi + lo (round to nearest), then move
// a few lo values to their other bf16 neighbour (each stays within one unit
// of its exact residual) so that each column of hi + lo has the column norm
// of G in FP64.  Without this the split matrix's small departure from
// unitarity, sum_r |g'_rc|^2 != sum_r |g_rc|^2, is coherent within a fused
// block and shows as a norm drift that grows linearly with the number of
// sweeps; with it diag(G'^H G') matches diag(G^H G) to far below one unit.
// Out: hr, lr, hi_, li indexed r * D + c.
void split_bf16x3(int D, const double *G, uint16_t *hr, uint16_t *lr, uint16_t *hi_, uint16_t *li) {
  std::vector<double> val(2 * size_t(D)), hv(2 * size_t(D));
  std::vector<uint16_t> l16(2 * size_t(D));
  std::vector<char> used(2 * size_t(D));
  for (int c = 0; c < D; ++c) {
    double want = 0, have = 0;
    for (int r = 0; r < D; ++r)
      for (int part = 0; part < 2; ++part) {
        const int j = 2 * r + part;
        const double v = part ? im_of(G, D, r, c) : re_of(G, D, r, c);
        const uint16_t h = host_bf16_rne(float(v));
        const double hd = host_bf16_to_f(h);
        const uint16_t l = host_bf16_rne(float(v - hd));
        (part ? hi_ : hr)[r * D + c] = h;
        val[j] = v;
        hv[j] = hd;
        l16[j] = l;
        used[j] = 0;
        want += v * v;
        const double e = hd + double(host_bf16_to_f(l));
        have += e * e;
      }
    // greedy: take the re-rounding that brings the column norm closest to want
    for (int it = 0; it < 2 * D; ++it) {
      const double err = have - want;
      int best = -1;
      double best_abs = std::fabs(err), best_delta = 0;
      uint16_t best_l = 0;
      for (int j = 0; j < 2 * D; ++j) {
        if (used[j]) continue;
        const double t = val[j] - hv[j];
        const double lcur = host_bf16_to_f(l16[j]);
        if (lcur == t) continue;  // exact: nothing to trade
        const uint16_t alt = bf16_step(l16[j], t > lcur ? 1 : -1);
        const double lalt = host_bf16_to_f(alt);
        const double e0 = hv[j] + lcur, e1 = hv[j] + lalt;
        const double delta = e1 * e1 - e0 * e0;
        if (std::fabs(err + delta) < best_abs) {
          best_abs = std::fabs(err + delta);
          best = j;
          best_delta = delta;
          best_l = alt;
        }
      }
      if (best < 0) break;
      l16[best] = best_l;
      used[best] = 1;
      have += best_delta;
    }
    for (int r = 0; r < D; ++r) {
      lr[r * D + c] = l16[2 * r];
      li[r * D + c] = l16[2 * r + 1];
    }
  }
}

// Output-row order that makes accumulator register r of lane half h hold row
// (half * h + 16 mt + r): row i of 32x32 output tile mt is stored there.
int out_row(int half, int mt, int i) { return half * ((i >> 2) & 1) + 16 * mt + 4 * (i >> 3) + (i & 3); }

}  // namespace

int mfma_tile_M(int K) {
  switch (K) {
    case 4: return 7;
    case 5: return 7;
    case 6: return 6;
    case 7: return 5;
    default: return -1;
  }
}

bool make_gate_tile(int n, int K, const int32_t *A, uint64_t extra, TilePlan *tp) {
  const int M = mfma_tile_M(K);
  if (M < 0 || n < K + M) return false;
  tp->n = n;
  tp->K = K;
  tp->M = M;
  tp->s = K + M;
  uint64_t tmask = 0;
  for (int j = 0; j < K; ++j) tmask |= uint64_t(1) << A[j];
  if (extra & tmask) return false;
  uint64_t lowmask = extra;
  int got = __builtin_popcountll(extra);
  if (got > M) return false;
  // Workgroups are handed to the eight XCDs in turn, so the three lowest
  // tile-index bits pick the XCD.  Leaving the three lowest non-target bits
  // from bit 7 up out of the tile puts them there: each XCD then takes 1 KiB
  // pieces spread over every 8 KiB when the targets allow it.  Measured at
  // N=30: k=4 on bits 0-3 2.84 -> 2.61 ms, k=5 1-5% faster, no pattern slower.
  uint64_t reserve = 0;
  for (int p = 7, r = 0; p < n && r < 3; ++p)
    if (!((tmask >> p) & 1) && !((lowmask >> p) & 1)) {
      reserve |= uint64_t(1) << p;
      ++r;
    }
  if (n - K - __builtin_popcountll(reserve) < M) reserve = 0;
  for (int p = 0; p < n && got < M; ++p)
    if (!((tmask >> p) & 1) && !((lowmask >> p) & 1) && !((reserve >> p) & 1)) {
      lowmask |= uint64_t(1) << p;
      ++got;
    }
  tp->smask = tmask | lowmask;
  // 16-byte chunks pair amplitudes that differ in physical bit 0: it must be a tile bit
  if (!(tp->smask & 1)) return false;
  int b = 0, rank = 0;
  for (int p = 0; p < n; ++p) {
    if (!((tp->smask >> p) & 1)) continue;
    tp->sbit[b] = p;
    int loc = -1;
    for (int j = 0; j < K; ++j)
      if (A[j] == p) loc = j;
    if (loc < 0) loc = K + rank++;
    tp->loc_in[b] = loc;
    tp->loc_out[b] = loc;
    ++b;
  }
  return true;
}

size_t mfma_operand_bytes(int K, int prec) {
  (void)prec;
  if (K >= 5) return size_t(1) << (2 * K + 3);  // FP32 Gr, Gi or bf16 Gr, Gi hi and lo
  return size_t(1) << (2 * K + 4);              // the real embedding (FP32, or bf16 hi and lo)
}

void pack_mfma_operand(int K, int prec, const double *G, void *out) {
  const int D = 1 << K;
  const int HALF = 1 << K, AH = 1 << (K - 1);
  const int EMT = (2 << K) / 32;
  if (prec == SV_PREC_FP32 && K >= 5) {
    // two planes Gr, Gi (the kernel forms Gr + Gi); plane x, tile mt, step kk, lane l holds
    // X[out_row(AH, mt, l % 32)][AH * (l / 32) + kk]
    const int GMT = D / 32;
    float *o = static_cast<float *>(out);
    for (int x = 0; x < 2; ++x)
      for (int mt = 0; mt < GMT; ++mt)
        for (int kk = 0; kk < AH; ++kk)
          for (int l = 0; l < 64; ++l) {
            const int r = out_row(AH, mt, l & 31), c = AH * (l >> 5) + kk;
            const double gr = re_of(G, D, r, c), gi = im_of(G, D, r, c);
            const double val = (x == 0) ? gr : gi;
            o[((x * GMT + mt) * AH + kk) * 64 + l] = float(val);
          }
  } else if (prec == SV_PREC_FP32) {
    // embedding; tile mt, step kk, lane l holds R[out_row(HALF, mt, l % 32)][HALF * (l / 32) + kk]
    float *o = static_cast<float *>(out);
    for (int mt = 0; mt < EMT; ++mt)
      for (int kk = 0; kk < HALF; ++kk)
        for (int l = 0; l < 64; ++l)
          o[(mt * HALF + kk) * 64 + l] = float(embedded(G, K, out_row(HALF, mt, l & 31), HALF * (l >> 5) + kk));
  } else if (K >= 5) {
    // BF16x3 complex form: planes (Gr hi, Gr lo, Gi hi, Gi lo) of the split
    // (split_bf16x3); plane P, tile mt, step kk, lane l holds the eight bf16
    // P[out_row(AH, mt, l % 32)][AH * (l / 32) + 8 kk + e], e < 8
    const int GMT = D / 32, KS = AH / 8;
    uint16_t *o = static_cast<uint16_t *>(out);
    std::vector<uint16_t> sp(4 * size_t(D) * D);
    uint16_t *hr = sp.data(), *lr = hr + D * D, *hm = lr + D * D, *lm = hm + D * D;
    split_bf16x3(D, G, hr, lr, hm, lm);
    const uint16_t *plane[4] = {hr, lr, hm, lm};
    for (int P = 0; P < 4; ++P)
      for (int mt = 0; mt < GMT; ++mt)
        for (int kk = 0; kk < KS; ++kk)
          for (int l = 0; l < 64; ++l)
            for (int e = 0; e < 8; ++e) {
              const int r = out_row(AH, mt, l & 31), c = AH * (l >> 5) + 8 * kk + e;
              o[((((size_t(P) * GMT + mt) * KS + kk) * 64) + l) * 8 + e] = plane[P][r * D + c];
            }
  } else {
    // embedding [[Re, -Im], [Im, Re]] of the split planes (split_bf16x3), hi
    // and lo planes; four consecutive reductions per step
    const int KQ = HALF / 4;
    uint16_t *hi = static_cast<uint16_t *>(out);
    uint16_t *lo = hi + size_t(EMT) * KQ * 64 * 4;
    std::vector<uint16_t> sp(4 * size_t(D) * D);
    uint16_t *hr = sp.data(), *lr = hr + D * D, *hm = lr + D * D, *lm = hm + D * D;
    split_bf16x3(D, G, hr, lr, hm, lm);
    for (int mt = 0; mt < EMT; ++mt)
      for (int kk = 0; kk < KQ; ++kk)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 4; ++e) {
            const int orow = out_row(HALF, mt, l & 31), icol = HALF * (l >> 5) + 4 * kk + e;
            const int r = orow >> 1, po = orow & 1, c = icol >> 1, pi = icol & 1;
            uint16_t h16, l16;
            if (po == pi) {
              h16 = hr[r * D + c];
              l16 = lr[r * D + c];
            } else {
              const uint16_t sgn = (po == 0) ? 0x8000u : 0;  // -Im in the upper right block
              h16 = hm[r * D + c] ^ sgn;
              l16 = lm[r * D + c] ^ sgn;
            }
            const size_t idx = ((size_t(mt) * KQ + kk) * 64 + l) * 4 + e;
            hi[idx] = h16;
            lo[idx] = l16;
          }
  }
}

hipError_t launch_tile_mfma(const TilePlan &tp, int prec, int opsrc, float2 *psi, const void *op, hipStream_t st) {
  const bool bf = (prec == SV_PREC_BF16X3);
  int o = opsrc;
  if (o == SV_MFMA_OPERAND_AUTO)  // measured at N=30 on MI355X: LDS for every width (BF16x3 k=7: 3.8 vs 4.2 ms)
    o = SV_MFMA_OPERAND_LDS;
  switch (tp.K) {
    case 4:
      if (o == SV_MFMA_OPERAND_REGS) return bf ? tile_mfma_k<4, 7, SV_PREC_BF16X3, OP_REG>(tp, psi, op, st) : tile_mfma_k<4, 7, SV_PREC_FP32, OP_REG>(tp, psi, op, st);
      return bf ? tile_mfma_k<4, 7, SV_PREC_BF16X3, OP_LDS>(tp, psi, op, st) : tile_mfma_k<4, 7, SV_PREC_FP32, OP_LDS>(tp, psi, op, st);
    case 5:
      if (o == SV_MFMA_OPERAND_REGS) return bf ? tile_mfma_k<5, 7, SV_PREC_BF16X3, OP_REG>(tp, psi, op, st) : tile_mfma_k<5, 7, SV_PREC_FP32, OP_REG>(tp, psi, op, st);
      if (o == SV_MFMA_OPERAND_GLOBAL) return bf ? tile_mfma_k<5, 7, SV_PREC_BF16X3, OP_GLOBAL>(tp, psi, op, st) : tile_mfma_k<5, 7, SV_PREC_FP32, OP_GLOBAL>(tp, psi, op, st);
      return bf ? tile_mfma_k<5, 7, SV_PREC_BF16X3, OP_LDS>(tp, psi, op, st) : tile_mfma_k<5, 7, SV_PREC_FP32, OP_LDS>(tp, psi, op, st);
    case 6:  // no register form: REGS takes the automatic choice (LDS)
      if (o != SV_MFMA_OPERAND_GLOBAL) return bf ? tile_mfma_k<6, 6, SV_PREC_BF16X3, OP_LDS>(tp, psi, op, st) : tile_mfma_k<6, 6, SV_PREC_FP32, OP_LDS>(tp, psi, op, st);
      return bf ? tile_mfma_k<6, 6, SV_PREC_BF16X3, OP_GLOBAL>(tp, psi, op, st) : tile_mfma_k<6, 6, SV_PREC_FP32, OP_GLOBAL>(tp, psi, op, st);
    case 7:  // the two 64 KiB FP32 planes, or the four 32 KiB bf16 planes, and the 32 KiB
             // tile fill the 160 KiB of LDS; REGS takes the automatic choice (LDS)
      if (o != SV_MFMA_OPERAND_GLOBAL)
        return bf ? tile_mfma_k<7, 5, SV_PREC_BF16X3, OP_LDS>(tp, psi, op, st) : tile_mfma_k<7, 5, SV_PREC_FP32, OP_LDS>(tp, psi, op, st);
      return bf ? tile_mfma_k<7, 5, SV_PREC_BF16X3, OP_GLOBAL>(tp, psi, op, st) : tile_mfma_k<7, 5, SV_PREC_FP32, OP_GLOBAL>(tp, psi, op, st);
    default: return hipErrorInvalidValue;
  }
}

// Default workgroup-to-tile order of layout permutations: the XCD bits on
// tile-index bits 9..11.  Measured at N=30 over 36 exchange patterns: 159 ms
// in all against 183 ms in the plain order, faster on 26 of them (exchanging
// bits 20..23 with 0..3: 4.8 -> 2.9 ms).
constexpr int kPermuteTileOrder = 9;

hipError_t launch_tile_permute(const TilePlan &tp_in, float2 *psi, hipStream_t st) {
  constexpr int S = kPermTileBits;
  if (tp_in.s != S || tp_in.n < S) return hipErrorInvalidValue;
  constexpr int NT = 256;
  constexpr int CHUNKS = (1 << (S - 1)) / NT;
  TilePlan tp = tp_in;
  if (tp.order < 0) tp.order = kPermuteTileOrder;
  TileArgs a;
  fill_args(tp, NT, CHUNKS, psi, nullptr, &a);
  choose_perm_swizzle(tp.loc_out, a.pswz);
  for (int i = 0; i < CHUNKS; ++i) {
    a.lam_i[i] = lin_swz_host(a.lam_i[i], a.pswz);
    a.lamo_i[i] = lin_swz_host(a.lamo_i[i], a.pswz);
  }
  hipLaunchKernelGGL((k_tile_permute<S>), dim3(grid_of(a.ntiles)), dim3(NT), 0, st, a);
  return hipGetLastError();
}

}  // namespace sv
