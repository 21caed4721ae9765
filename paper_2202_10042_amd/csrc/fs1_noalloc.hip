// fs1_noalloc.hip -- fs1_solve on a fixed device workspace, for callers that
// cannot allocate device memory during the call.
//
// The workspace is a file-scope device array (one copy per GPU, alive until
// the process ends).  Host code never uses the array's name as an address:
// its device address is taken once per device with hipGetSymbolAddress (with
// that device current) and kept.  Every call on a GPU shares that GPU's copy,
// so calls that overlap on one GPU (other streams, other host threads) race;
// the solve clears what must start at zero itself.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fs1.h"
#include "fs1_host.h"

namespace fs1 {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
int scratch_address(int dev, char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return host::hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return host::set_err(FS1_ERR_HIP, "hipGetSymbolAddress(scratch) gave no address");
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return FS1_OK;
}

}  // namespace
}  // namespace fs1

extern "C" int fs1_solve_noalloc(fs1_ctx* ctx, const double* mu, const double* nu, int64_t n,
                                 double eps, double tol, const fs1_opts* opts,
                                 fs1_result* out) {
  using namespace fs1::host;
  if (!ctx) return set_err(FS1_ERR_INVALID_ARG, "null context");
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != ctx->device)
    return set_err(FS1_ERR_INVALID_ARG,
                   "the context's device (%d) must be current (current device %d)", ctx->device,
                   dev);
  if (dev < 0 || dev >= fs1::kMaxDevices)
    return set_err(FS1_ERR_INVALID_ARG, "device %d beyond the %d supported", dev,
                   fs1::kMaxDevices);
  char* ws = nullptr;
  const int st = fs1::scratch_address(dev, &ws);
  if (st) return st;
  return solve_on(ctx, mu, nu, n, eps, tol, opts, out, ws, fs1::kScratchBytes);
}
