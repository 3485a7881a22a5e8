// log rho without device allocation, for callers that cannot allocate (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
// kernels as tdo_log_rho (weight packing, the fused forward layers, the Hermitian
// log-sum-exp), with their work memory in a fixed array of the library's device image
// instead of the context's workspace.
//
// The array is a device symbol; host code never uses its name as an address.  Its
// device address is looked up once per device (hipGetSymbolAddress, with that device
// current) when a context is created on the device, and kept per device; every
// kernel argument that points into it is formed from that address.  Every call on a
// device shares the array, which keeps the last call's contents: each call writes all
// it reads (packed weights, then per chunk the residual buffers before the layers read
// them), so nothing needs clearing, and calls that overlap in time on one device race.
#include <algorithm>
#include <mutex>

#include "common.h"
#include "netapi.h"
#include "train.h"

namespace tdo {

namespace {

constexpr size_t kScratchBytes = TDO_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

}  // namespace

// Device address of this device's copy of the scratch array (once per device, with the
// device current; the caller's current device is restored).
int32_t noalloc_setup(int device) {
  TDO_CHECK(device >= 0 && device < kMaxDevices, TDO_EINVAL, "device %d outside [0, %d)", device, kMaxDevices);
  std::lock_guard<std::mutex> g(g_mu);
  if (g_scratch[device]) return TDO_OK;
  int cur = 0;
  TDO_HIP(hipGetDevice(&cur));
  TDO_HIP(hipSetDevice(device));
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  const hipError_t e2 = hipSetDevice(cur);
  TDO_CHECK(e == hipSuccess && p != nullptr, TDO_EHIP, "hipGetSymbolAddress of the scratch array failed: %s",
            hipGetErrorString(e));
  TDO_HIP(e2);
  g_scratch[device] = p;
  return TDO_OK;
}

}  // namespace tdo

using namespace tdo;

extern "C" int32_t tdo_log_rho_noalloc(tdo_ctx_t* ctx, const tdo_arch_t* arch, const float* params, int32_t n,
                                       const uint64_t* cfg, int64_t B, tdo_prec_t prec, float* log_rho,
                                       hipStream_t stream) {
  clear_error();
  TDO_CHECK(ctx != nullptr, TDO_EINVAL, "ctx is NULL");
  TDO_CHECK(prec == TDO_FP32 || prec == TDO_BF16, TDO_EINVAL, "unknown precision %d", (int)prec);
  NetPlan np;
  TDO_TRY(net_plan(&ctx->c, arch, n, prec == TDO_BF16, &np));
  np.prof = nullptr;  // per-kernel timing would create events
  TDO_CHECK(B >= 0, TDO_EINVAL, "B=%lld < 0", (long long)B);
  if (B == 0) return TDO_OK;
  TDO_CHECK(params && cfg && log_rho, TDO_EINVAL, "NULL buffer");
  const int dev = ctx->c.device;
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_mu);
    base = (dev >= 0 && dev < kMaxDevices) ? g_scratch[dev] : nullptr;
  }
  TDO_CHECK(base != nullptr, TDO_EINVAL, "no scratch address for device %d (the context was not set up)", dev);
  TDO_HIP(hipSetDevice(dev));
  // packed weights first, then per chunk two residual buffers and z
  Arena ar;
  size_t woff[4];
  carve_weights(np, ar, woff);
  const size_t fixed = ar.used;
  const size_t per_block = 32 * (size_t)np.D * 4;
  const size_t per_unit = 2 * per_block * (size_t)blocks_for(np, np.cpb) + (size_t)np.cpb * 16 + 3 * 256;
  TDO_CHECK(fixed + per_unit <= kScratchBytes, TDO_ENOMEM,
            "the packed weights (%zu bytes) leave no room for one block in the %zu-byte scratch", fixed,
            kScratchBytes);
  // entries per chunk: a multiple of the configurations per block that fits the scratch
  int64_t chunk = (int64_t)((kScratchBytes - fixed) / per_unit) * np.cpb;
  chunk = std::min<int64_t>(chunk, (B + np.cpb - 1) / np.cpb * np.cpb);
  const int64_t nblk = blocks_for(np, chunk);
  const size_t oxa = ar.take<float>((size_t)nblk * 32 * np.D);
  const size_t oxb = ar.take<float>((size_t)nblk * 32 * np.D);
  const size_t oz = ar.take<float>((size_t)chunk * 4);
  TDO_CHECK(ar.used <= kScratchBytes, TDO_ENOMEM, "scratch plan of %zu bytes exceeds %zu", ar.used, kScratchBytes);
  NetWeights w = weights_at(base, woff);
  TDO_TRY(pack_weights(np, params, &w, stream));
  for (int64_t e0 = 0; e0 < B; e0 += chunk) {
    const int64_t E = std::min(chunk, B - e0);
    TDO_TRY(run_forward(np, w, cfg + 2 * e0, E, nullptr, at<float>(base, oxa), at<float>(base, oxb), nullptr,
                        at<float>(base, oz), stream));
    TDO_TRY(launch_symmetrise(nullptr, E, at<float>(base, oz), log_rho + 2 * e0, stream));
  }
  return TDO_OK;
}
