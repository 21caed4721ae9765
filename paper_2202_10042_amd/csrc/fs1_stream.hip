// fs1_stream.hip -- a STREAM-style device copy: the attainable-bandwidth
// reference beside which the half-iteration kernels' achieved bandwidth is
// reported (they read and write whole vectors once per half, as a copy does).
//
// Each workgroup of 256 threads moves 256 x U 16-byte vectors; every load of a
// thread is issued before its first store, and the k-th access of the
// workgroup's threads covers one contiguous 4 KiB span.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fs1.h"
#include "fs1_host.h"

namespace fs1 {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kCopyThreads = 256;
constexpr int kCopyUnroll = 4;

template <int U, bool NT>
__global__ __launch_bounds__(kCopyThreads) void k_stream_copy(const u32x4* __restrict__ src,
                                                              u32x4* __restrict__ dst,
                                                              int64_t nvec) {
  const int64_t base = int64_t(blockIdx.x) * (kCopyThreads * U) + threadIdx.x;
  u32x4 v[U];
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const int64_t k = base + int64_t(i) * kCopyThreads;
    if (k < nvec) {
      if constexpr (NT) {
        v[i] = __builtin_nontemporal_load(src + k);
      } else {
        v[i] = src[k];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const int64_t k = base + int64_t(i) * kCopyThreads;
    if (k < nvec) {
      if constexpr (NT) {
        __builtin_nontemporal_store(v[i], dst + k);
      } else {
        dst[k] = v[i];
      }
    }
  }
}

}  // namespace
}  // namespace fs1

using namespace fs1;
using namespace fs1::host;

extern "C" int fs1_stream_copy(fs1_ctx* ctx, const void* src, void* dst, int64_t bytes,
                               int flags) {
  if (!ctx) return set_err(FS1_ERR_INVALID_ARG, "null context");
  if (bytes < 0 || (bytes & 15) != 0)
    return set_err(FS1_ERR_INVALID_ARG, "bytes must be a non-negative multiple of 16");
  if (bytes == 0) return FS1_OK;
  if (!src || !dst) return set_err(FS1_ERR_INVALID_ARG, "null array");
  if (!aligned16(src) || !aligned16(dst))
    return set_err(FS1_ERR_INVALID_ARG, "device arrays must be 16-byte aligned");
  if (flags & ~1) return set_err(FS1_ERR_INVALID_ARG, "unknown flags %d", flags);
  const char* s = static_cast<const char*>(src);
  const char* d = static_cast<const char*>(dst);
  if (s < d + bytes && d < s + bytes) return set_err(FS1_ERR_INVALID_ARG, "src and dst overlap");
  const int64_t nvec = bytes / 16;
  const int64_t per_block = int64_t(kCopyThreads) * kCopyUnroll;
  const int64_t blocks = (nvec + per_block - 1) / per_block;
  if (blocks > int64_t(INT32_MAX)) return set_err(FS1_ERR_INVALID_ARG, "copy too large");
  const u32x4* sv = static_cast<const u32x4*>(src);
  u32x4* dv = static_cast<u32x4*>(dst);
  if (flags & 1) {
    k_stream_copy<kCopyUnroll, true><<<unsigned(blocks), kCopyThreads, 0, ctx->stream>>>(sv, dv,
                                                                                       nvec);
  } else {
    k_stream_copy<kCopyUnroll, false><<<unsigned(blocks), kCopyThreads, 0, ctx->stream>>>(sv, dv,
                                                                                        nvec);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "fs1_stream_copy launch");
  return FS1_OK;
}
