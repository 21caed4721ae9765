// fs1_host.h -- host-side pieces shared by the C ABI (fs1_api.cpp) and the
// serving loop (fs1_server.cpp): the context object, error reporting,
// workspace helpers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "fs1.h"
#include "fs1_batch.h"
#include "fs1_internal.h"

struct fs1_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  // caller's device allocator (fs1_ctx_create_with_allocator); null: hipMalloc
  fs1_alloc_fn alloc = nullptr;
  fs1_free_fn free = nullptr;
  void* alloc_user = nullptr;
  char* ws = nullptr;      // device workspace
  size_t ws_size = 0;
  fs1::Ctrl* hctrl = nullptr;  // pinned host mirror of the control block
  // diagnostic timing of the half-iteration kernels (fs1_ctx_set_profiling)
  int profiling = 0;
  std::vector<hipEvent_t> events;
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
  double prof_bytes = 0.0;
  // batched solves
  void* hstage = nullptr;   // pinned host staging (stop counters, states, lists)
  size_t hstage_size = 0;
  hipStream_t capture = nullptr;  // stream used only to capture iteration graphs
  hipEvent_t bev[2] = {nullptr, nullptr};
  // resident instances: one stream per workgroup size, beside the shared launches
  hipStream_t aux[2] = {nullptr, nullptr};
  hipEvent_t rev[3] = {nullptr, nullptr, nullptr};  // set-up done / each stream done
};

namespace fs1 {
namespace host {

// Record a message for fs1_last_error() and return `code`.
int set_err(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
const char* last_error_text();

bool aligned16(const void* p);
// Device memory of a context: from the caller's allocator when it gave one,
// else hipMalloc / hipFree.
int dev_alloc(fs1_ctx* c, size_t bytes, void** out);
void dev_free(fs1_ctx* c, void* p);
size_t round_up(size_t x, size_t a);
int ensure_ws(fs1_ctx* c, size_t bytes);
int ensure_hstage(fs1_ctx* c, size_t bytes);
int check_h_eps(int64_t n, double h, double eps);
// Capture `count` batched iterations over the groups into an executable graph.
int capture_iterations(fs1_ctx* ctx, const BatchBufs& z, const std::vector<BatchGroup>& groups,
                       int count, hipGraphExec_t* out);

// Body of fs1_solve.  fixed_ws == nullptr: workspace from the context (grown on
// demand); otherwise the solve runs on fixed_ws (device memory of fixed_cap
// bytes) and allocates nothing, failing with FS1_ERR_INVALID_ARG if the grid
// needs more.
// dev_out != nullptr: the asynchronous form (fs1_solve_async): no host
// synchronisation, every iteration's launches issued, the result written to
// dev_out (device memory) by a kernel; *out only reports argument errors.
int solve_on(fs1_ctx* ctx, const double* mu, const double* nu, int64_t n, double eps, double tol,
             const fs1_opts* opts_in, fs1_result* out, char* fixed_ws, size_t fixed_cap,
             fs1_result* dev_out = nullptr);

// Bump allocator over a workspace (a null base only measures).
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(char* b) : base(b) {}
  void* take(size_t bytes) {
    void* p = base ? base + off : nullptr;
    off = round_up(off + bytes, 256);
    return p;
  }
};

}  // namespace host

// FS-1 on grids (fs1_2d.hip): the bodies of fs1_kv_apply_2d / _nd and
// fs1_solve_2d / _nd (opts already defaulted, *out cleared).
int kv_apply_2d(fs1_ctx* ctx, const void* x, void* y, int64_t n1, int64_t n2, double h1,
                double h2, double eps, int dt);
int solve_2d(fs1_ctx* ctx, const double* mu, const double* nu, int64_t n1, int64_t n2, double h1,
             double h2, double eps, double tol, const fs1_opts& o, fs1_result* out);
int kv_apply_grid(fs1_ctx* ctx, const void* x, void* y, int nd, const int64_t* dims,
                  const double* h, double eps, int dt);
int solve_grid(fs1_ctx* ctx, const double* mu, const double* nu, int nd, const int64_t* dims,
               const double* h, double eps, double tol, const fs1_opts& o, fs1_result* out);

}  // namespace fs1

#define HIP_TRY(call)                                              \
  do {                                                             \
    hipError_t e_ = (call);                                        \
    if (e_ != hipSuccess) return ::fs1::host::hip_fail(e_, #call); \
  } while (0)
