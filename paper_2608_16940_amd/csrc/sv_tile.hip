// LDS-tiled kernels for gfx950.
//
// Dense fused gate on MFMA.  A fused k-qubit gate is a dense contraction
// (Eq. cost-formal: Theta(2^{N+k}) complex multiply-adds): every group of
// 2^k amplitudes that share the non-target bits is multiplied by G.  Here a
// workgroup owns a tile of 2^(K+M) amplitudes -- the K target bits plus the M
// lowest non-target physical bits -- so every global access is a contiguous
// run of at least 2^M amplitudes whatever the target positions are.  The tile
// is staged in LDS in "local" order (target bits lowest, in gate order, then
// the non-target bits), which makes each group contiguous; each wave then
// multiplies 32 groups at a time with the real embedding of G,
//   [Re out; Im out] = [[Re G, -Im G], [Im G, Re G]] [Re in; Im in],
// as a 2^(K+1) x 2^(K+1) by 2^(K+1) x 32 real GEMM on
// v_mfma_f32_32x32x2f32 (FP32) or v_mfma_f32_32x32x8bf16_1k (BF16x3 split).
//
// Operand layout.  The K (reduction) ordering is free, so lane l of a wave
// holds group (l mod 32) and the contiguous half h = l / 32 of its 2^(K+1)
// reals; MFMA step kk consumes the lane's kk-th real.  The output rows of the
// embedded matrix are permuted on the host so that accumulator register r of
// M-tile mt of lane l is output real (2^K h + 16 mt + r): a lane's results are
// the same contiguous half of the same group, written back in place.
//
// The store side can read the tile with a different bit map (loc_out), which
// relabels bits inside the tile for free (the lazy relabel L' = alpha o L of
// Algorithm 2, restricted to the tile's bits).  With no gate the same kernel is
// an in-place bit permutation in one sweep.
#include <cstring>

#include "sv_internal.h"

namespace sv {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

struct TileArgs {
  float2 *psi;
  const void *op;
  int64_t ntiles;
  int s;
  int lb_in, lb_out;  // local bit of tile-order bit 0 on load / store
  int sbit[24];
  int loc_in[24];
  int loc_out[24];
  int64_t goff_i[32];
  int32_t lam_i[32];
  int32_t lamo_i[32];
};

__device__ __forceinline__ int64_t insert_zero_bit(int64_t x, int p) {
  const int64_t low = x & ((int64_t(1) << p) - 1);
  return ((x >> p) << (p + 1)) | low;
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

template <int K, int M, int PREC>
__global__ __launch_bounds__(64 << (M - 5)) void k_tile_mfma(TileArgs a) {
  constexpr int WAVES = 1 << (M - 5);
  constexpr int NT = 64 * WAVES;
  constexpr int S = K + M;
  constexpr int TILE = 1 << S;
  constexpr int CHUNKS = 1 << (K - 2);  // 16-byte chunks per thread per tile
  constexpr int HALF = 1 << K;          // reals per lane half
  constexpr int MT = (2 << K) / 32;     // 32-row output tiles
  constexpr int AH = HALF / 2;          // amplitudes per lane half
  constexpr bool RESIDENT = (K <= 5);   // embedded operand held in registers
  __shared__ float2 lds[TILE];

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;

  int64_t goff_t = 0;
  int lam_t = 0, lamo_t = 0;
#pragma unroll
  for (int b = 1; b <= M + 1; ++b) {
    if ((t >> (b - 1)) & 1) {
      goff_t |= int64_t(1) << a.sbit[b];
      lam_t |= 1 << a.loc_in[b];
      lamo_t |= 1 << a.loc_out[b];
    }
  }
  const int bin = 1 << a.lb_in, bout = 1 << a.lb_out;

  // ---- operand
  constexpr int NRES = RESIDENT ? (PREC == SV_PREC_FP32 ? MT * HALF : MT * (HALF / 4) * 2) : 1;
  float ra[NRES];
  shortx4 rh[RESIDENT && PREC == SV_PREC_BF16X3 ? MT * (HALF / 4) : 1];
  shortx4 rl[RESIDENT && PREC == SV_PREC_BF16X3 ? MT * (HALF / 4) : 1];
  const float *opf = reinterpret_cast<const float *>(a.op);
  const shortx4 *oph = reinterpret_cast<const shortx4 *>(a.op);
  const shortx4 *opl = oph + MT * (HALF / 4) * 64;
  if constexpr (RESIDENT) {
    if constexpr (PREC == SV_PREC_FP32) {
#pragma unroll
      for (int i = 0; i < MT * HALF; ++i) ra[i] = opf[i * 64 + lane];
    } else {
#pragma unroll
      for (int i = 0; i < MT * (HALF / 4); ++i) {
        rh[i] = oph[i * 64 + lane];
        rl[i] = opl[i * 64 + lane];
      }
    }
  }
  (void)ra;

  const int g = 32 * wave + (lane & 31);
  const int h = lane >> 5;

  for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    int64_t base = tile;
#pragma unroll
    for (int b = 0; b < S; ++b) base = insert_zero_bit(base, a.sbit[b]);

    // ---- global -> LDS (each chunk: two consecutive amplitudes, 16 B)
#pragma unroll
    for (int i = 0; i < CHUNKS; ++i) {
      const float4 v = *reinterpret_cast<const float4 *>(a.psi + base + goff_t + a.goff_i[i]);
      const int l0 = lam_t | a.lam_i[i];
      lds[swz<K>(l0)] = make_float2(v.x, v.y);
      lds[swz<K>(l0 | bin)] = make_float2(v.z, v.w);
    }
    __syncthreads();

    // ---- 32 groups per wave: gather this lane's half group
    float bx[HALF];
#pragma unroll
    for (int e = 0; e < AH; ++e) {
      const float2 x = lds[swz<K>((g << K) | (h * AH + e))];
      bx[2 * e] = x.x;
      bx[2 * e + 1] = x.y;
    }
    floatx16 acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mt][r] = 0.f;

    if constexpr (PREC == SV_PREC_FP32) {
#pragma unroll
      for (int kk = 0; kk < HALF; ++kk) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          float av;
          if constexpr (RESIDENT)
            av = ra[mt * HALF + kk];
          else
            av = opf[(mt * HALF + kk) * 64 + lane];
          acc[mt] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bx[kk], acc[mt], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < HALF / 4; ++kk) {
        shortx4 bh, bl;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float x = bx[4 * kk + e];
          const unsigned short hi = bf16_rne(x);
          const unsigned short lo = bf16_rne(x - bf16_to_f(hi));
          bh[e] = short(hi);
          bl[e] = short(lo);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          shortx4 ah, al;
          if constexpr (RESIDENT) {
            ah = rh[mt * (HALF / 4) + kk];
            al = rl[mt * (HALF / 4) + kk];
          } else {
            ah = oph[(mt * (HALF / 4) + kk) * 64 + lane];
            al = opl[(mt * (HALF / 4) + kk) * 64 + lane];
          }
          acc[mt] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, bh, acc[mt], 0, 0, 0);
          acc[mt] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, bl, acc[mt], 0, 0, 0);
          acc[mt] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(al, bh, acc[mt], 0, 0, 0);
        }
      }
    }

    // ---- results back to the same LDS slots (this wave owns these groups)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int e = 0; e < 8; ++e)
        lds[swz<K>((g << K) | (h * AH + 8 * mt + e))] = make_float2(acc[mt][2 * e], acc[mt][2 * e + 1]);
    __syncthreads();

    // ---- LDS -> global
#pragma unroll
    for (int i = 0; i < CHUNKS; ++i) {
      const int l0 = lamo_t | a.lamo_i[i];
      const float2 x0 = lds[swz<K>(l0)];
      const float2 x1 = lds[swz<K>(l0 | bout)];
      *reinterpret_cast<float4 *>(a.psi + base + goff_t + a.goff_i[i]) = make_float4(x0.x, x0.y, x1.x, x1.y);
    }
    __syncthreads();
  }
}

// In-place bit permutation of the tile's bits in one sweep.
template <int S>
__global__ __launch_bounds__(256) void k_tile_permute(TileArgs a) {
  constexpr int NT = 256;
  constexpr int CHUNKS = (1 << (S - 1)) / NT;
  __shared__ float2 lds[1 << S];
  const int t = threadIdx.x;
  int64_t goff_t = 0;
  int lamo_t = 0;
#pragma unroll
  for (int b = 1; b <= 8; ++b) {
    if ((t >> (b - 1)) & 1) {
      goff_t |= int64_t(1) << a.sbit[b];
      lamo_t |= 1 << a.loc_out[b];
    }
  }
  const int bout = 1 << a.lb_out;
  for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    int64_t base = tile;
#pragma unroll
    for (int b = 0; b < S; ++b) base = insert_zero_bit(base, a.sbit[b]);
#pragma unroll
    for (int i = 0; i < CHUNKS; ++i) {
      const float4 v = *reinterpret_cast<const float4 *>(a.psi + base + goff_t + a.goff_i[i]);
      const int l0 = 2 * (i * NT + t);  // identity on load
      lds[l0] = make_float2(v.x, v.y);
      lds[l0 + 1] = make_float2(v.z, v.w);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CHUNKS; ++i) {
      const int l0 = lamo_t | a.lamo_i[i];
      const float2 x0 = lds[l0];
      const float2 x1 = lds[l0 | bout];
      *reinterpret_cast<float4 *>(a.psi + base + goff_t + a.goff_i[i]) = make_float4(x0.x, x0.y, x1.x, x1.y);
    }
    __syncthreads();
  }
}

int g_cu_count = 0;
int cu_count() {
  if (g_cu_count == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) ==
                                                 hipSuccess && v > 0)
      g_cu_count = v;
    else
      g_cu_count = 256;
  }
  return g_cu_count;
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

void fill_args(const TilePlan &tp, int nt, int chunks, float2 *psi, const void *op, TileArgs *a) {
  std::memset(a, 0, sizeof(*a));
  a->psi = psi;
  a->op = op;
  a->s = tp.s;
  a->ntiles = int64_t(1) << (tp.n - tp.s);
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

float embedded(const double *G, int K, int orow, int icol) {
  const int D = 1 << K;
  const int r = orow >> 1, po = orow & 1, c = icol >> 1, pi = icol & 1;
  const double gr = G[2 * (r * D + c)], gi = G[2 * (r * D + c) + 1];
  double v = (po == pi) ? gr : (po == 0 ? -gi : gi);
  return float(v);
}
double embedded64(const double *G, int K, int orow, int icol) {
  const int D = 1 << K;
  const int r = orow >> 1, po = orow & 1, c = icol >> 1, pi = icol & 1;
  const double gr = G[2 * (r * D + c)], gi = G[2 * (r * D + c) + 1];
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

template <int K, int M, int PREC>
hipError_t tile_mfma_k(const TilePlan &tp, float2 *psi, const void *op, hipStream_t st) {
  constexpr int NT = 64 << (M - 5);
  constexpr int CHUNKS = 1 << (K - 2);
  TileArgs a;
  fill_args(tp, NT, CHUNKS, psi, op, &a);
  const int per_cu = (NT >= 256) ? 3 : 8;
  int64_t grid = int64_t(cu_count()) * per_cu;
  if (grid > a.ntiles) grid = a.ntiles;
  hipLaunchKernelGGL((k_tile_mfma<K, M, PREC>), dim3(unsigned(grid)), dim3(NT), 0, st, a);
  return hipGetLastError();
}

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

bool make_gate_tile(int n, int K, const int32_t *A, TilePlan *tp) {
  const int M = mfma_tile_M(K);
  if (M < 0 || n < K + M) return false;
  tp->n = n;
  tp->K = K;
  tp->M = M;
  tp->s = K + M;
  uint64_t tmask = 0;
  for (int j = 0; j < K; ++j) tmask |= uint64_t(1) << A[j];
  uint64_t lowmask = 0;
  int got = 0;
  for (int p = 0; p < n && got < M; ++p)
    if (!((tmask >> p) & 1)) {
      lowmask |= uint64_t(1) << p;
      ++got;
    }
  tp->smask = tmask | lowmask;
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
  return size_t(1) << (2 * K + 4);
}

void pack_mfma_operand(int K, int prec, const double *G, void *out) {
  const int HALF = 1 << K;
  const int MT = (2 << K) / 32;
  if (prec == SV_PREC_FP32) {
    float *o = static_cast<float *>(out);
    for (int mt = 0; mt < MT; ++mt)
      for (int kk = 0; kk < HALF; ++kk)
        for (int l = 0; l < 64; ++l) {
          const int i = l & 31, kp = l >> 5;
          const int orow = HALF * ((i >> 2) & 1) + 16 * mt + 4 * (i >> 3) + (i & 3);
          const int icol = HALF * kp + kk;
          o[(mt * HALF + kk) * 64 + l] = embedded(G, K, orow, icol);
        }
  } else {
    uint16_t *hi = static_cast<uint16_t *>(out);
    uint16_t *lo = hi + size_t(MT) * (HALF / 4) * 64 * 4;
    for (int mt = 0; mt < MT; ++mt)
      for (int kk = 0; kk < HALF / 4; ++kk)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 4; ++e) {
            const int i = l & 31, kp = l >> 5;
            const int orow = HALF * ((i >> 2) & 1) + 16 * mt + 4 * (i >> 3) + (i & 3);
            const int icol = HALF * kp + 4 * kk + e;
            const double v = embedded64(G, K, orow, icol);
            const uint16_t h = host_bf16_rne(float(v));
            const uint16_t l16 = host_bf16_rne(float(v - double(host_bf16_to_f(h))));
            const size_t idx = ((size_t(mt) * (HALF / 4) + kk) * 64 + l) * 4 + e;
            hi[idx] = h;
            lo[idx] = l16;
          }
  }
}

hipError_t launch_tile_mfma(const TilePlan &tp, int prec, float2 *psi, const void *op, hipStream_t st) {
  const bool bf = (prec == SV_PREC_BF16X3);
  switch (tp.K) {
    case 4: return bf ? tile_mfma_k<4, 7, SV_PREC_BF16X3>(tp, psi, op, st) : tile_mfma_k<4, 7, SV_PREC_FP32>(tp, psi, op, st);
    case 5: return bf ? tile_mfma_k<5, 7, SV_PREC_BF16X3>(tp, psi, op, st) : tile_mfma_k<5, 7, SV_PREC_FP32>(tp, psi, op, st);
    case 6: return bf ? tile_mfma_k<6, 6, SV_PREC_BF16X3>(tp, psi, op, st) : tile_mfma_k<6, 6, SV_PREC_FP32>(tp, psi, op, st);
    case 7: return bf ? tile_mfma_k<7, 5, SV_PREC_BF16X3>(tp, psi, op, st) : tile_mfma_k<7, 5, SV_PREC_FP32>(tp, psi, op, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tile_permute(const TilePlan &tp, float2 *psi, hipStream_t st) {
  constexpr int S = 12;
  if (tp.s != S || tp.n < S) return hipErrorInvalidValue;
  constexpr int NT = 256;
  constexpr int CHUNKS = (1 << (S - 1)) / NT;
  TileArgs a;
  fill_args(tp, NT, CHUNKS, psi, nullptr, &a);
  int64_t grid = int64_t(cu_count()) * 4;
  if (grid > a.ntiles) grid = a.ntiles;
  hipLaunchKernelGGL((k_tile_permute<S>), dim3(unsigned(grid)), dim3(NT), 0, st, a);
  return hipGetLastError();
}

}  // namespace sv
