// rpca_svd_noalloc: the randomized SVD on a file-scope device array instead
// of a workspace the library allocates, for callers that cannot allocate.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/rpca.h"
#include "internal.h"

namespace {

// Scratch of the allocation-free entry point: working buffers, then the LU
// arrival counters in the last kCounterBytes.  Every device the library runs
// on holds one copy until the process ends.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr size_t kCounterBytes = size_t(64) << 10;
static __device__ __align__(256) char scratch[kScratchBytes];

// The array's address on each device (host code must never use the symbol
// itself as a device address), looked up once per device with that device
// current.
constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void* g_ptr[kMaxDevices];
hipError_t g_err[kMaxDevices];

void lookup(int dev) {
  int cur = -1;
  g_err[dev] = hipGetDevice(&cur);
  if (g_err[dev] != hipSuccess) return;
  if (cur != dev && (g_err[dev] = hipSetDevice(dev)) != hipSuccess) return;
  void* p = nullptr;
  g_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_ptr[dev] = (g_err[dev] == hipSuccess) ? p : nullptr;
  if (cur != dev) (void)hipSetDevice(cur);
}

}  // namespace

extern "C" rpca_status rpca_svd_noalloc(rpca_ctx ctx, const rpca_matrix* A, int k, int l, int its,
                                        uint64_t seed, unsigned flags, float* U, int64_t ldu,
                                        double* S, float* V, int64_t ldv) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  const int dev = rpca::ctx_device(ctx);
  if (dev < 0 || dev >= kMaxDevices)
    return rpca::ctx_fail(ctx, RPCA_ERR_UNSUPPORTED, "rpca_svd_noalloc: device index above 63");
  std::call_once(g_once[dev], lookup, dev);
  if (g_err[dev] != hipSuccess || !g_ptr[dev])
    return rpca::ctx_fail(ctx, RPCA_ERR_HIP,
                          (std::string("rpca_svd_noalloc: hipGetSymbolAddress failed: ") +
                           hipGetErrorString(g_err[dev])).c_str());
  char* base = static_cast<char*>(g_ptr[dev]);
  return rpca::svd_on_workspace(ctx, A, k, l, its, seed, flags, U, ldu, S, V, ldv, base,
                                kScratchBytes - kCounterBytes,
                                reinterpret_cast<unsigned*>(base + kScratchBytes - kCounterBytes),
                                kCounterBytes / sizeof(unsigned));
}
