// Sampling from a caller's probability array without any allocation: the
// sampler's scratch (CDF block totals and their chunk totals, a shot chunk,
// the bad-input flag) lives in one file-scope device array instead of a
// caller workspace.  Every GPU the library runs on holds its own copy of the
// array until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
#include <mutex>

#include "sv_internal.h"

namespace sv {
namespace {

constexpr int kNoAllocMaxQubits = SV_NOALLOC_MAX_QUBITS;
constexpr int64_t kNoAllocShotChunk = SV_NOALLOC_SHOT_CHUNK;
constexpr size_t kNoAllocBlocks = size_t(1) << (kNoAllocMaxQubits - kCdfBlockBits);

constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Scratch layout: block totals | chunk totals | shot chunk | scalars.
constexpr size_t kOffBlocks = 0;
constexpr size_t kOffChunks = kOffBlocks + align256(kNoAllocBlocks * 8);
constexpr size_t kOffShots = kOffChunks + align256(((kNoAllocBlocks + 1023) / 1024) * 8);
constexpr size_t kOffScalars = kOffShots + align256(size_t(kNoAllocShotChunk) * 8);
constexpr size_t kScratchBytes = kOffScalars + align256(64 * 8);
static_assert(kScratchBytes == SV_NOALLOC_SCRATCH_BYTES, "scratch size in the header");

// 256-byte aligned, like a caller workspace.
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void *g_ptr[kMaxDevices];
hipError_t g_err[kMaxDevices];

// Device address of this device's scratch array, looked up once per device
// with that device current.
int scratch_for_current_device(char **out) {
  int dev = -1;
  SV_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index outside the scratch table");
    return SV_ERR_DEVICE;
  }
  std::call_once(g_once[dev], [dev]() {
    void *p = nullptr;
    g_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_ptr[dev] = (g_err[dev] == hipSuccess) ? p : nullptr;
  });
  if (g_err[dev] != hipSuccess || !g_ptr[dev]) {
    set_error(std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(g_err[dev]));
    return SV_ERR_DEVICE;
  }
  *out = static_cast<char *>(g_ptr[dev]);
  return SV_OK;
}

}  // namespace
}  // namespace sv

using namespace sv;

extern "C" int sv_sample_probs_noalloc(const double *probs_dev, int n, uint64_t seed, int64_t shots,
                                       uint64_t *out_host, void *stream) {
  return guard([&]() -> int {
    if (!probs_dev || (!out_host && shots > 0) || shots < 0) {
      set_error("bad argument");
      return SV_ERR_ARG;
    }
    if (n < SV_MIN_QUBITS || n > kNoAllocMaxQubits) {
      set_error("n outside [1, SV_NOALLOC_MAX_QUBITS] for the allocation-free sampler");
      return SV_ERR_ARG;
    }
    if (shots == 0) return SV_OK;
    char *base = nullptr;
    const int rc = scratch_for_current_device(&base);
    if (rc) return rc;
    Workspace ws;
    ws.blocksum = reinterpret_cast<uint64_t *>(base + kOffBlocks);
    ws.chunksum = reinterpret_cast<uint64_t *>(base + kOffChunks);
    ws.shots = reinterpret_cast<uint64_t *>(base + kOffShots);
    ws.scalars = reinterpret_cast<uint64_t *>(base + kOffScalars);
    return sample_impl(nullptr, probs_dev, n, ws, kNoAllocShotChunk, seed, shots, out_host, identity_layout(n),
                       static_cast<hipStream_t>(stream), SV_ERR_ARG);
  });
}
