// fs1_api.cpp -- the C ABI of libfs1 (include/fs1.h): argument validation,
// workspace, and the host loop of Algorithm 1 (FS-1).
//
// The solve loop launches, for every iteration l, the psi-half (K^T phi by the
// scans, psi = nu / K^T phi, the stopping-test error of (phi^l, psi^l)) and the
// phi-half (which closes the stopping test on the device and, unless it is met,
// computes phi = mu / K psi).  Once the test is met every later launch returns
// at once, so the host only has to look at the device flag every `sync_every`
// iterations; the iteration at which the solve stops does not depend on that
// interval.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fs1.h"
#include "fs1_batch.h"
#include "fs1_host.h"
#include "fs1_internal.h"
#include "fs1_tau.h"
#include "fs1_tune.h"

using namespace fs1;

namespace fs1 {
namespace host {

namespace {
thread_local std::string g_err;
}  // namespace

const char* last_error_text() { return g_err.c_str(); }

int set_err(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return set_err(FS1_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int dev_alloc(fs1_ctx* c, size_t bytes, void** out) {
  *out = nullptr;
  if (c->alloc) {
    void* p = c->alloc(bytes, c->alloc_user);
    if (!p) return set_err(FS1_ERR_NO_MEMORY, "the caller's allocator returned no memory for %zu bytes", bytes);
    if (!aligned16(p)) {
      c->free(p, c->alloc_user);
      return set_err(FS1_ERR_NO_MEMORY, "the caller's allocator returned memory that is not 16-byte aligned");
    }
    *out = p;
    return FS1_OK;
  }
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) {
    *out = nullptr;
    return set_err(FS1_ERR_NO_MEMORY, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  return FS1_OK;
}

void dev_free(fs1_ctx* c, void* p) {
  if (!p) return;
  if (c->free)
    c->free(p, c->alloc_user);
  else
    (void)hipFree(p);
}

// Grow the context workspace to at least `bytes` (stream-synchronised when the
// old buffer is released, because earlier asynchronous calls may still use it).
int ensure_ws(fs1_ctx* c, size_t bytes) {
  if (bytes <= c->ws_size) return FS1_OK;
  if (c->ws) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    dev_free(c, c->ws);
    c->ws = nullptr;
    c->ws_size = 0;
  }
  const size_t sz = round_up(bytes, size_t(1) << 20);
  void* p = nullptr;
  const int st = dev_alloc(c, sz, &p);
  if (st) return st;
  c->ws = static_cast<char*>(p);
  c->ws_size = sz;
  return FS1_OK;
}

// Pinned host staging of at least `bytes`.
int ensure_hstage(fs1_ctx* c, size_t bytes) {
  if (bytes <= c->hstage_size) return FS1_OK;
  if (c->hstage) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipHostFree(c->hstage));
    c->hstage = nullptr;
    c->hstage_size = 0;
  }
  const size_t sz = round_up(bytes, size_t(1) << 16);
  hipError_t e = hipHostMalloc(&c->hstage, sz, hipHostMallocDefault);
  if (e != hipSuccess) {
    c->hstage = nullptr;
    return set_err(FS1_ERR_NO_MEMORY, "hipHostMalloc(%zu) failed: %s", sz, hipGetErrorString(e));
  }
  c->hstage_size = sz;
  return FS1_OK;
}

int check_h_eps(int64_t n, double h, double eps) {
  if (n < 1) return set_err(FS1_ERR_INVALID_ARG, "n must be >= 1 (got %lld)", (long long)n);
  if (!(h > 0.0) || !std::isfinite(h)) return set_err(FS1_ERR_INVALID_ARG, "h must be finite and > 0");
  if (!(eps > 0.0) || !std::isfinite(eps))
    return set_err(FS1_ERR_INVALID_ARG, "eps must be finite and > 0");
  // exponents of lambda^D over the whole grid must fit the extended-range format
  if (double(n) * (h / eps) > 1.0e8)
    return set_err(FS1_ERR_INVALID_ARG, "n*h/eps = %g exceeds 1e8", double(n) * (h / eps));
  return FS1_OK;
}

int capture_iterations(fs1_ctx* ctx, const BatchBufs& z, const std::vector<BatchGroup>& groups,
                       int count, hipGraphExec_t* out) {
  *out = nullptr;
  if (!ctx->capture) HIP_TRY(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
  const hipError_t le =
      launch_batch_iterations(z, groups.data(), int(groups.size()), count, ctx->capture);
  hipGraph_t graph = nullptr;
  const hipError_t ce = hipStreamEndCapture(ctx->capture, &graph);
  if (le != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(le, "batched iteration capture");
  }
  if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
  const hipError_t ie = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    *out = nullptr;
    return hip_fail(ie, "hipGraphInstantiate");
  }
  return FS1_OK;
}

}  // namespace host
}  // namespace fs1

using namespace fs1::host;

namespace {

int kv_common(fs1_ctx* ctx, const void* x, void* y, int64_t n, double h, double eps, int dt,
              bool log) {
  if (!ctx) return set_err(FS1_ERR_INVALID_ARG, "null context");
  if (!x || !y) return set_err(FS1_ERR_INVALID_ARG, "null array");
  if (dt != FS1_F64 && dt != FS1_F32) return set_err(FS1_ERR_INVALID_ARG, "bad dtype %d", dt);
  if (!aligned16(x) || !aligned16(y))
    return set_err(FS1_ERR_INVALID_ARG, "device arrays must be 16-byte aligned");
  int st = check_h_eps(n, h, eps);
  if (st) return st;
  const size_t es = dt == FS1_F64 ? 8 : 4;
  const char* xb = static_cast<const char*>(x);
  const char* yb = static_cast<const char*>(y);
  if (xb < yb + n * es && yb < xb + n * es)
    return set_err(FS1_ERR_INVALID_ARG, "x and y must not overlap");
  const int R = pick_run_length(dt, log, h / eps);
  const int64_t C = int64_t(kBlock) * R;
  const int64_t nchunks = (n + C - 1) / C;
  if (nchunks > int64_t(INT32_MAX)) return set_err(FS1_ERR_INVALID_ARG, "n too large");
  Carve cv(nullptr);
  cv.take(nchunks * sizeof(ChunkAgg));
  cv.take(carry_buffer_bytes(nchunks));
  cv.take(2 * sizeof(int));
  st = ensure_ws(ctx, cv.off);
  if (st) return st;
  Carve w(ctx->ws);
  ChunkAgg* agg = static_cast<ChunkAgg*>(w.take(nchunks * sizeof(ChunkAgg)));
  ChunkAgg* carry = static_cast<ChunkAgg*>(w.take(carry_buffer_bytes(nchunks)));
  int* special = static_cast<int*>(w.take(2 * sizeof(int)));
  const ScanConsts k = make_scan_consts(h, eps, R);
  const CarryConsts kc = make_carry_consts(h, eps, C, nchunks);
  hipError_t e = log ? launch_kv_log(dt, x, y, n, k, kc, agg, carry, special, ctx->stream)
                     : launch_kv_plain(dt, x, y, n, k, kc, agg, carry, ctx->stream);
  if (e != hipSuccess) return hip_fail(e, log ? "fs1_kv_apply_log launch" : "fs1_kv_apply launch");
  return FS1_OK;
}

// FS1_FLAG_DEVICE_PARAMS: the per-instance eps and tol live in device memory;
// copy them to host vectors and point *eps, *tol there.
int host_params(fs1_ctx* ctx, const fs1_opts* opts, int32_t B, const double** eps,
                const double** tol, std::vector<double>& he, std::vector<double>& ht) {
  if (!ctx || !opts || !(opts->flags & FS1_FLAG_DEVICE_PARAMS) || B <= 0) return FS1_OK;
  if (!*eps || !*tol) return set_err(FS1_ERR_INVALID_ARG, "bad batch arguments");
  he.resize(size_t(B));
  ht.resize(size_t(B));
  HIP_TRY(hipMemcpyAsync(he.data(), *eps, size_t(B) * sizeof(double), hipMemcpyDeviceToHost,
                         ctx->stream));
  HIP_TRY(hipMemcpyAsync(ht.data(), *tol, size_t(B) * sizeof(double), hipMemcpyDeviceToHost,
                         ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  *eps = he.data();
  *tol = ht.data();
  return FS1_OK;
}

// Ragged batch in the log domain: every instance keeps its own lambda, run
// length, stopping test and iteration count; all of them advance in the same
// launches (fs1_batch.hip).
int batched_entry(fs1_ctx* ctx, const double* mu_packed, const double* nu_packed,
                  const int64_t* offsets, int32_t B, const double* eps, const double* tol,
                  const fs1_opts* opts, fs1_result* out, const BatchCfg* force);

// force (optional): the configuration of every instance (B entries; the
// tuner's measurements), else batch_config() per instance.
int batch_solve(fs1_ctx* ctx, const double* mu, const double* nu, const int64_t* offsets,
                int32_t B, const double* eps, const double* tol, const fs1_opts& o,
                fs1_result* out, const BatchCfg* force = nullptr) {
  const int dt = o.dtype;
  const size_t es = dt == FS1_F64 ? 8 : 4;
  hipStream_t s = ctx->stream;

  // run length of each instance, and whether one workgroup holds all of it
  // (resident: all its iterations in one launch): a function of (n, eps,
  // dtype) only, so an instance's arithmetic does not depend on the rest of
  // the batch
  std::vector<int> rlen(B), rthreads(B, 0);
  for (int32_t i = 0; i < B; ++i) {
    const int64_t n = offsets[i + 1] - offsets[i];
    const BatchCfg cfg = force ? force[i] : batch_config(dt, n, (1.0 / double(n)) / eps[i]);
    rlen[i] = cfg.R;
    rthreads[i] = cfg.nt;
  }
  std::vector<int> rs(rlen);
  std::sort(rs.begin(), rs.end(), [](int a, int b) { return a > b; });
  rs.erase(std::unique(rs.begin(), rs.end()), rs.end());
  std::vector<BatchGroup> groups;
  std::vector<std::vector<int>> members;  // instances of each group
  std::vector<InstInfo> info(B);
  int64_t chunk = 0, elem = 0;
  for (int r : rs) {
    BatchGroup g{r, nullptr, 0};
    members.emplace_back();
    const int64_t C = int64_t(kBlock) * r;
    for (int32_t i = 0; i < B; ++i) {
      if (rlen[i] != r) continue;
      const int64_t n = offsets[i + 1] - offsets[i];
      // a resident instance is allocated to exactly its workgroup's runs
      const int64_t nch = rthreads[i] ? rthreads[i] / kBlock : (n + C - 1) / C;
      if (chunk + nch > int64_t(INT32_MAX) / kBlock)
        return set_err(FS1_ERR_INVALID_ARG, "batch too large");
      info[i] = make_inst_info(mu + offsets[i], nu + offsets[i], elem, n, int(chunk), r,
                               1.0 / double(n), eps[i], tol[i], 0);
      info[i].nch = int32_t(nch);
      members.back().push_back(int(i));
      chunk += nch;
      elem += nch * C;
    }
    groups.push_back(g);
  }
  const int ngroups = int(groups.size());
  const int64_t nchunks = chunk, nruns = chunk * kBlock, nelem = elem;
  // resident classes (R, workgroup size), the larger workgroups first
  std::vector<ResGroup> rgroups;
  std::vector<int> rorder;  // instances of the classes, consecutive
  for (int nt : {1024, 256}) {
    for (int r : rs) {
      ResGroup g{r, nt, nullptr, 0};
      for (int32_t i = 0; i < B; ++i) {
        if (rthreads[i] == nt && rlen[i] == r) {
          rorder.push_back(int(i));
          ++g.count;
        }
      }
      if (g.count > 0) rgroups.push_back(g);
    }
  }
  const int nres = int(rorder.size());

  BatchBufs z{};
  ChunkRef* clist = nullptr;  // device chunk lists of the groups (running instances only)
  int* rlist = nullptr;       // device instance lists of the resident classes
  auto layout = [&](Carve& w) {
    z.inst = static_cast<InstInfo*>(w.take(size_t(B) * sizeof(InstInfo)));
    z.st = static_cast<InstState*>(w.take(size_t(B) * sizeof(InstState)));
    z.iter_base = static_cast<int*>(w.take(2 * sizeof(int)));
    z.mu64 = static_cast<double*>(w.take(nelem * sizeof(double)));
    z.nu64 = static_cast<double*>(w.take(nelem * sizeof(double)));
    z.mu32 = dt == FS1_F32 ? w.take(nelem * sizeof(float)) : nullptr;
    z.nu32 = dt == FS1_F32 ? w.take(nelem * sizeof(float)) : nullptr;
    z.vF = w.take(nelem * es);
    z.vG[0] = w.take(nelem * es);
    z.vG[1] = w.take(nelem * es);
    z.eF = static_cast<int*>(w.take(nruns * sizeof(int)));
    z.eG[0] = static_cast<int*>(w.take(nruns * sizeof(int)));
    z.eG[1] = static_cast<int*>(w.take(nruns * sizeof(int)));
    z.aggF = static_cast<ChunkAgg*>(w.take(nchunks * sizeof(ChunkAgg)));
    z.aggG = static_cast<ChunkAgg*>(w.take(nchunks * sizeof(ChunkAgg)));
    z.agg2 = w.take(nchunks * 48);
    z.part = static_cast<double*>(w.take(nchunks * sizeof(double)));
    z.part2 = static_cast<double*>(w.take(nchunks * sizeof(double)));
    z.part3 = static_cast<double*>(w.take(nchunks * sizeof(double)));
    clist = static_cast<ChunkRef*>(w.take(nchunks * sizeof(ChunkRef)));
    rlist = static_cast<int*>(w.take(size_t(std::max(nres, 1)) * sizeof(int)));
  };
  {
    Carve probe(nullptr);
    layout(probe);
    int st = ensure_ws(ctx, probe.off);
    if (st) return st;
    // pinned staging: stop counters, the per-instance states, the chunk lists
    st = ensure_hstage(ctx, 64 + size_t(B) * sizeof(InstState) +
                                size_t(nchunks) * sizeof(ChunkRef) + size_t(nres) * sizeof(int));
    if (st) return st;
    Carve w(ctx->ws);
    layout(w);
  }
  z.ndone = z.iter_base + 1;
  z.dtype = dt;
  z.itr_max = o.itr_max;
  z.check_every = o.check_every;
  z.nchunks = nchunks;
  z.nelem = nelem;

  std::vector<InstState> init(B);
  for (InstState& t : init) {
    std::memset(&t, 0, sizeof(t));
    t.stop_iter = -1;
    t.fail_iter = INT_MAX;
    t.last_check = -1;
    t.last_err = NAN;
  }
  HIP_TRY(hipMemcpyAsync(z.inst, info.data(), size_t(B) * sizeof(InstInfo),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(z.st, init.data(), size_t(B) * sizeof(InstState),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(z.iter_base, 0, 2 * sizeof(int), s));
  // `count` iterations per replay; every instance stops by iteration itr_max
  const int count = std::max(1, std::min(o.sync_every, o.itr_max + 1));
  const int64_t max_rounds = (int64_t(o.itr_max) + count) / count + 1;
  const bool use_graph = !(o.flags & FS1_FLAG_NO_GRAPH);
  hipGraphExec_t gexec = nullptr;
  struct GraphGuard {
    hipGraphExec_t* g;
    ~GraphGuard() {
      if (*g) (void)hipGraphExecDestroy(*g);
    }
  } guard{&gexec};
  auto capture = [&]() -> int {
    if (gexec) {
      (void)hipGraphExecDestroy(gexec);
      gexec = nullptr;
    }
    return use_graph ? capture_iterations(ctx, z, groups, count, &gexec) : FS1_OK;
  };
  for (hipEvent_t& e : ctx->bev)
    if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));

  char* hb = static_cast<char*>(ctx->hstage);
  int* hdone = reinterpret_cast<int*>(hb);
  InstState* hst = reinterpret_cast<InstState*>(hb + 64);
  ChunkRef* hlist = reinterpret_cast<ChunkRef*>(hb + 64 + size_t(B) * sizeof(InstState));
  // Launches run over the chunk records of the instances still running.  The
  // lists are rebuilt (and the graph recaptured) whenever an eighth of the
  // instances that were running at the last rebuild have stopped, so late
  // launches do not carry the chunks of finished instances.
  // all = true: every instance (set-up, finalisation); otherwise the chunks
  // of the shared launches: instances that are not resident and, once
  // `running` is set, have not stopped.
  auto build_lists = [&](bool all, bool running) -> int {
    if (running) {
      HIP_TRY(hipMemcpyAsync(hst, z.st, size_t(B) * sizeof(InstState), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
    }
    int64_t at = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      const int64_t start = at;
      for (int b : members[gi]) {
        if (!all && (rthreads[b] || (running && hst[b].done))) continue;
        for (int j = 0; j < info[b].nch; ++j) hlist[at++] = chunk_ref(info[b], b, j);
      }
      groups[gi].list = clist + start;
      groups[gi].nlist = int(at - start);
    }
    if (at > 0)
      HIP_TRY(hipMemcpyAsync(clist, hlist, size_t(at) * sizeof(ChunkRef), hipMemcpyHostToDevice,
                             s));
    // the pinned list is read by that copy: finish it before the host writes again
    HIP_TRY(hipStreamSynchronize(s));
    return FS1_OK;
  };
  int st = build_lists(true, false);
  if (st) return st;
  HIP_TRY(launch_batch_setup(z, groups.data(), ngroups, nullptr, B, s));
  // resident instances: their own launches on a second stream, beside the
  // shared launches of the others
  if (nres > 0) {
    int* hr = reinterpret_cast<int*>(hlist + nchunks);
    std::memcpy(hr, rorder.data(), size_t(nres) * sizeof(int));
    HIP_TRY(hipMemcpyAsync(rlist, hr, size_t(nres) * sizeof(int), hipMemcpyHostToDevice, s));
    int at = 0;
    for (ResGroup& g : rgroups) {
      g.ilist = rlist + at;
      at += g.count;
    }
    for (hipStream_t& a : ctx->aux)
      if (!a) HIP_TRY(hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
    for (hipEvent_t& e : ctx->rev)
      if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(ctx->rev[0], s));
    // the two workgroup sizes run side by side
    for (int k = 0; k < 2; ++k) {
      hipStream_t a = ctx->aux[k];
      HIP_TRY(hipStreamWaitEvent(a, ctx->rev[0], 0));
      for (const ResGroup& g : rgroups)
        if (g.nt == (k == 0 ? 1024 : 256)) HIP_TRY(launch_batch_resident(z, &g, 1, a));
      HIP_TRY(hipEventRecord(ctx->rev[1 + k], a));
    }
  }
  st = build_lists(false, false);
  if (st) return st;
  st = capture();
  if (st) return st;

  hdone[0] = hdone[1] = 0;
  int stopped = 0, stopped_at_rebuild = 0, running_at_rebuild = B;
  for (int64_t r = 0; r <= max_rounds; ++r) {
    if (gexec) {
      HIP_TRY(hipGraphLaunch(gexec, s));
    } else {
      HIP_TRY(launch_batch_iterations(z, groups.data(), ngroups, count, s));
    }
    HIP_TRY(hipMemcpyAsync(&hdone[r & 1], z.ndone, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(ctx->bev[r & 1], s));
    if (r > 0) {
      // one replay stays queued ahead of the host's look at the stop counter
      HIP_TRY(hipEventSynchronize(ctx->bev[(r - 1) & 1]));
      stopped = hdone[(r - 1) & 1];
      if (stopped >= B) break;
      if (stopped - stopped_at_rebuild >= std::max(1, running_at_rebuild / 8)) {
        st = build_lists(false, true);
        if (st) return st;
        st = capture();
        if (st) return st;
        stopped = hdone[r & 1];  // the queued replay has completed
        if (stopped >= B) break;
        stopped_at_rebuild = stopped;
        running_at_rebuild = B - stopped;
      }
    }
  }
  if (nres > 0) {
    // the shared launches may finish first: wait for the resident ones
    HIP_TRY(hipStreamWaitEvent(s, ctx->rev[1], 0));
    HIP_TRY(hipStreamWaitEvent(s, ctx->rev[2], 0));
    HIP_TRY(hipMemcpyAsync(&hdone[0], z.ndone, sizeof(int), hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  stopped = std::max(stopped, std::max(hdone[0], hdone[1]));
  if (stopped != B)
    return set_err(FS1_ERR_INTERNAL, "batched solve: %d of %d instances stopped", stopped, B);
  st = build_lists(true, false);
  if (st) return st;

  HIP_TRY(launch_batch_finalize(z, groups.data(), ngroups, nullptr, B, nullptr, s));
  InstState* hs = hst;
  HIP_TRY(hipMemcpyAsync(hs, z.st, size_t(B) * sizeof(InstState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int32_t i = 0; i < B; ++i) {
    const InstState& t = hs[i];
    fs1_result& r = out[i];
    if (t.invalid) {
      r.status = FS1_ERR_INVALID_ARG;
      continue;
    }
    if (t.fail) {
      r.iterations = t.fail_iter;
      r.status = FS1_ERR_NONFINITE;
      continue;
    }
    r.iterations = t.stop_iter >= 0 ? t.stop_iter : o.itr_max;
    r.w1 = t.w1;
    r.marginal_err = t.err;
    r.mu_err = t.mu_err;
    r.converged = !(t.err > tol[i]) ? 1 : 0;
    r.status = (std::isfinite(t.w1) && std::isfinite(t.err)) ? FS1_OK : FS1_ERR_NONFINITE;
  }
  return FS1_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* fs1_last_error(void) { return last_error_text(); }

const char* fs1_version(void) { return "fs1 0.1 (gfx950)"; }

int fs1_ctx_create(void* stream, fs1_ctx** out) {
  return fs1_ctx_create_with_allocator(stream, nullptr, nullptr, nullptr, out);
}

int fs1_ctx_create_with_allocator(void* stream, fs1_alloc_fn alloc, fs1_free_fn free_fn,
                                  void* user, fs1_ctx** out) {
  if (!out) return set_err(FS1_ERR_INVALID_ARG, "null output pointer");
  *out = nullptr;
  if (!alloc != !free_fn)
    return set_err(FS1_ERR_INVALID_ARG, "give both allocator callbacks or neither");
  fs1_ctx* c = new (std::nothrow) fs1_ctx();
  if (!c) return set_err(FS1_ERR_NO_MEMORY, "context allocation failed");
  c->stream = static_cast<hipStream_t>(stream);
  c->alloc = alloc;
  c->free = free_fn;
  c->alloc_user = user;
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipGetDevice");
  }
  e = hipHostMalloc(reinterpret_cast<void**>(&c->hctrl), sizeof(Ctrl), hipHostMallocDefault);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipHostMalloc");
  }
  *out = c;
  return FS1_OK;
}

int fs1_ctx_destroy(fs1_ctx* c) {
  if (!c) return FS1_OK;
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  for (hipStream_t a : c->aux)
    if (a) (void)hipStreamSynchronize(a);
  for (hipEvent_t e : c->bev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->rev)
    if (e) (void)hipEventDestroy(e);
  if (c->capture) (void)hipStreamDestroy(c->capture);
  for (hipStream_t a : c->aux)
    if (a) (void)hipStreamDestroy(a);
  if (c->hstage) (void)hipHostFree(c->hstage);
  if (c->ws) dev_free(c, c->ws);
  if (c->hctrl) (void)hipHostFree(c->hctrl);
  delete c;
  return FS1_OK;
}

int fs1_ctx_set_stream(fs1_ctx* c, void* stream) {
  if (!c) return set_err(FS1_ERR_INVALID_ARG, "null context");
  c->stream = static_cast<hipStream_t>(stream);
  return FS1_OK;
}

int fs1_ctx_set_profiling(fs1_ctx* c, int enable) {
  if (!c) return set_err(FS1_ERR_INVALID_ARG, "null context");
  c->profiling = enable > 0 ? enable : 0;
  c->prof_ms = 0.0;
  c->prof_launches = 0;
  c->prof_bytes = 0.0;
  return FS1_OK;
}

int fs1_ctx_kernel_stats(fs1_ctx* c, double* total_ms, int64_t* launches, double* alg_bytes) {
  if (!c) return set_err(FS1_ERR_INVALID_ARG, "null context");
  if (total_ms) *total_ms = c->prof_ms;
  if (launches) *launches = c->prof_launches;
  if (alg_bytes) *alg_bytes = c->prof_bytes;
  return FS1_OK;
}

int fs1_kv_apply(fs1_ctx* ctx, const void* x, void* y, int64_t n, double h, double eps, int dt) {
  return kv_common(ctx, x, y, n, h, eps, dt, false);
}

int fs1_kv_apply_log(fs1_ctx* ctx, const void* lx, void* ly, int64_t n, double h, double eps,
                     int dt) {
  return kv_common(ctx, lx, ly, n, h, eps, dt, true);
}

int fs1_opts_default(fs1_opts* o) {
  if (!o) return set_err(FS1_ERR_INVALID_ARG, "null opts");
  std::memset(o, 0, sizeof(*o));
  o->h = 0.0;
  o->itr_max = 10000;
  o->dtype = FS1_F64;
  o->domain = FS1_PLAIN;
  o->check_every = 1;
  o->sync_every = 16;
  o->flags = 0;
  o->potentials_out = nullptr;
  o->err_history = nullptr;
  o->tau = 1e3;
  return FS1_OK;
}

int fs1_solve(fs1_ctx* ctx, const double* mu, const double* nu, int64_t n, double eps, double tol,
              const fs1_opts* opts_in, fs1_result* out) {
  return fs1::host::solve_on(ctx, mu, nu, n, eps, tol, opts_in, out, nullptr, 0, nullptr);
}

int fs1_solve_async(fs1_ctx* ctx, const double* mu, const double* nu, int64_t n, double eps,
                    double tol, const fs1_opts* opts, fs1_result* out_dev) {
  if (!out_dev) return set_err(FS1_ERR_INVALID_ARG, "null result pointer");
  fs1_result host{};
  return fs1::host::solve_on(ctx, mu, nu, n, eps, tol, opts, &host, nullptr, 0, out_dev);
}

}  // extern "C"

namespace fs1 {
namespace host {

int solve_on(fs1_ctx* ctx, const double* mu, const double* nu, int64_t n, double eps, double tol,
             const fs1_opts* opts_in, fs1_result* out, char* fixed_ws, size_t fixed_cap,
             fs1_result* dev_out) {
  // dev_out: the asynchronous solve (no host synchronisation, every launch
  // issued, result written to device memory by a kernel)
  const bool async = dev_out != nullptr;
  if (!ctx) return set_err(FS1_ERR_INVALID_ARG, "null context");
  if (!out) return set_err(FS1_ERR_INVALID_ARG, "null result pointer");
  std::memset(out, 0, sizeof(*out));
  out->w1 = NAN;
  out->marginal_err = NAN;
  out->mu_err = NAN;
  auto finish = [&](int st) {
    out->status = st;
    return st;
  };
  fs1_opts o;
  fs1_opts_default(&o);
  if (opts_in) o = *opts_in;
  if (o.itr_max < 0) o.itr_max = 10000;
  if (o.check_every < 1) o.check_every = 1;
  if (o.sync_every < 1) o.sync_every = 16;
  const double h = o.h > 0.0 ? o.h : 1.0 / double(n);
  if (!mu || !nu) return finish(set_err(FS1_ERR_INVALID_ARG, "null marginal"));
  if (!aligned16(mu) || !aligned16(nu))
    return finish(set_err(FS1_ERR_INVALID_ARG, "device arrays must be 16-byte aligned"));
  if (o.dtype != FS1_F64 && o.dtype != FS1_F32)
    return finish(set_err(FS1_ERR_INVALID_ARG, "bad dtype %d", o.dtype));
  if (o.domain != FS1_PLAIN && o.domain != FS1_LOG && o.domain != FS1_ABSORB)
    return finish(set_err(FS1_ERR_INVALID_ARG, "bad domain %d", o.domain));
  const bool tau_mode = o.domain == FS1_ABSORB;
  if (tau_mode && !(o.tau > 0.0 && std::isfinite(o.tau)))
    return finish(set_err(FS1_ERR_INVALID_ARG, "tau must be finite and > 0"));
  if (tau_mode && (o.flags & FS1_FLAG_PERSISTENT))
    return finish(set_err(FS1_ERR_INVALID_ARG,
                          "the absorption variant has no persistent solver"));
  if (!(tol >= 0.0)) return finish(set_err(FS1_ERR_INVALID_ARG, "tol must be >= 0"));
  if ((o.flags & 1) && !o.potentials_out)
    return finish(set_err(FS1_ERR_INVALID_ARG, "potentials requested without an output array"));
  const bool warm = o.warm_m != nullptr || o.warm_e != nullptr;
  if (warm && (!o.warm_m || !o.warm_e))
    return finish(set_err(FS1_ERR_INVALID_ARG, "a warm start needs both warm_m and warm_e"));
  if (warm && tau_mode)
    return finish(set_err(FS1_ERR_INVALID_ARG, "no warm start in the absorption variant"));
  if ((o.state_m != nullptr) != (o.state_e != nullptr))
    return finish(set_err(FS1_ERR_INVALID_ARG, "the state output needs both state_m and state_e"));
  if ((warm && (!aligned16(o.warm_m) || !aligned16(o.warm_e))) ||
      (o.state_m && (!aligned16(o.state_m) || !aligned16(o.state_e))))
    return finish(set_err(FS1_ERR_INVALID_ARG, "device arrays must be 16-byte aligned"));
  if (async && (tau_mode || (o.flags & FS1_FLAG_PERSISTENT)))
    return finish(set_err(FS1_ERR_INVALID_ARG,
                          "the asynchronous solve has no absorption variant and no persistent "
                          "solver"));
  if (async && !aligned16(dev_out))
    return finish(set_err(FS1_ERR_INVALID_ARG, "device arrays must be 16-byte aligned"));
  int st = check_h_eps(n, h, eps);
  if (st) return finish(st);

  // the threshold variant stores its final state in the log domain's layout
  const bool absorb = o.domain == FS1_LOG || o.domain == FS1_ABSORB;
  const int dt = o.dtype;
  const size_t es = dt == FS1_F64 ? 8 : 4;
  int R = pick_run_length(dt, absorb, h / eps);
  // grids of at most 1024 runs: the whole solve in one resident workgroup
  int rr = (o.flags & (FS1_FLAG_GENERAL | FS1_FLAG_PERSISTENT | FS1_FLAG_NO_RESIDENT))
               ? 0
               : resident_run_length(n, R);
  // runs of 16 on 256 or 512 threads instead of runs of 8 on 1024 threads
  // (fewer waves in every workgroup-wide step): binary64 grids of 2049 to
  // 8192 entries (below 2049 entries runs of 8 on fewer threads are faster),
  // binary32 grids of 4097 to 8192 entries where its run length is 16.  The
  // threshold variant keeps runs of 8.
  if (rr == 8 && !tau_mode && n <= int64_t(512) * 16 &&
      ((dt == FS1_F64 && n > int64_t(256) * 8 && (!absorb || 15.0 * (h / eps) <= 600.0)) ||
       (dt == FS1_F32 && R == 16)))
    rr = 16;
  if (rr > 0) R = rr;
  const int res_threads = rr > 0 ? solve_resident_threads(n, R) : 0;
  // the fused one-launch-per-half path picks its own run length where it applies
  if (res_threads == 0 && absorb && !tau_mode &&
      !(o.flags & (FS1_FLAG_GENERAL | FS1_FLAG_PERSISTENT))) {
    const int rf = fused_run_length(dt, h / eps, n);
    if (rf > 0) R = rf;
  }
  const int64_t C = int64_t(kBlock) * R;
  // the resident workgroup's runs are allocated whole
  const int64_t nchunks = res_threads ? std::max(res_threads, kBlock) / kBlock : (n + C - 1) / C;
  if (nchunks > int64_t(INT32_MAX)) return finish(set_err(FS1_ERR_INVALID_ARG, "n too large"));
  const int64_t nruns = nchunks * kBlock;

  // workspace layout
  SolveBufs b{};
  TauBufs tb{};
  int* epoch = nullptr;  // persistent solve: per-chunk publication flags
  const int64_t npad = nchunks * C;  // vectors are allocated to whole chunks
  double* mu64 = nullptr;
  double* nu64 = nullptr;
  auto layout = [&](Carve& w) {
    b.vF = w.take(npad * es);
    b.vG[0] = w.take(npad * es);
    b.vG[1] = w.take(npad * es);
    b.eF = static_cast<int*>(w.take(nruns * sizeof(int)));
    b.eG[0] = static_cast<int*>(w.take(nruns * sizeof(int)));
    b.eG[1] = static_cast<int*>(w.take(nruns * sizeof(int)));
    b.xF = static_cast<ChunkExp*>(w.take(nchunks * sizeof(ChunkExp)));
    b.xG[0] = static_cast<ChunkExp*>(w.take(nchunks * sizeof(ChunkExp)));
    b.xG[1] = static_cast<ChunkExp*>(w.take(nchunks * sizeof(ChunkExp)));
    b.lanetab = w.take(kWave * 32);
    b.mu32 = dt == FS1_F32 ? w.take(npad * sizeof(float)) : nullptr;
    b.nu32 = dt == FS1_F32 ? w.take(npad * sizeof(float)) : nullptr;
    mu64 = static_cast<double*>(w.take(npad * sizeof(double)));
    nu64 = static_cast<double*>(w.take(npad * sizeof(double)));
    b.aggF = static_cast<ChunkAgg*>(w.take(nchunks * sizeof(ChunkAgg)));
    b.aggG = static_cast<ChunkAgg*>(w.take(nchunks * sizeof(ChunkAgg)));
    b.carry = static_cast<ChunkAgg*>(w.take(carry_buffer_bytes(nchunks)));
    b.agg2 = w.take(nchunks * 48);
    b.carry2 = w.take(nchunks * 48);
    b.part = static_cast<double*>(w.take(nchunks * sizeof(double)));
    b.part2 = static_cast<double*>(w.take(nchunks * sizeof(double)));
    b.dtab = static_cast<XF64*>(w.take(nchunks * sizeof(XF64)));
    b.ctrl = static_cast<Ctrl*>(w.take(sizeof(Ctrl)));
    if (tau_mode) {  // (the one-workgroup solver does not use them)
      tb.potF = static_cast<double*>(w.take(npad * sizeof(double)));
      tb.potG = static_cast<double*>(w.take(npad * sizeof(double)));
      tb.pmF = static_cast<double*>(w.take(nchunks * sizeof(double)));
      tb.pmG = static_cast<double*>(w.take(nchunks * sizeof(double)));
      tb.absorb = static_cast<int*>(w.take(sizeof(int)));
    }
    epoch = static_cast<int*>(w.take(size_t(std::max<int64_t>(nchunks, 1)) * sizeof(int)));
  };
  {
    Carve probe(nullptr);
    layout(probe);
    char* base = fixed_ws;
    if (fixed_ws) {
      if (probe.off > fixed_cap)
        return finish(set_err(FS1_ERR_INVALID_ARG,
                              "the solve needs %zu bytes of workspace, more than the %zu "
                              "bytes available",
                              probe.off, fixed_cap));
    } else {
      if (async && probe.off > ctx->ws_size) {
        // growing the workspace synchronises the stream: not under capture
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIP_TRY(hipStreamIsCapturing(ctx->stream, &cs));
        if (cs != hipStreamCaptureStatusNone)
          return finish(set_err(FS1_ERR_INVALID_ARG,
                                "the context's workspace (%zu bytes) is smaller than this solve "
                                "needs (%zu) and the stream is capturing: run the solve once "
                                "before the capture",
                                ctx->ws_size, probe.off));
      }
      st = ensure_ws(ctx, probe.off);
      if (st) return finish(st);
      base = ctx->ws;
    }
    Carve w(base);
    layout(w);
  }
  b.dtype = dt;
  b.absorb = absorb ? 1 : 0;
  b.n = n;
  b.nchunks = nchunks;
  b.R = R;
  b.npad = npad;
  b.mu_src = mu;
  b.nu_src = nu;
  b.mu = mu64;
  b.nu = nu64;
  b.err_hist = o.err_history;
  b.tau = tau_mode ? o.tau : 0.0;
  b.inv_eps = 1.0 / eps;
  hipStream_t s = ctx->stream;
  Ctrl* hc = ctx->hctrl;

  // a1: validate the marginals on the device (finite, >= 0, equal mass)
  if (async)
    HIP_TRY(launch_async_reset(b, o.err_history, o.itr_max, s));
  else
    HIP_TRY(hipMemsetAsync(b.ctrl, 0, sizeof(Ctrl), s));
  HIP_TRY(launch_setup(b, s));
  // a warm start writes the state now (and checks it with the marginals)
  if (warm) HIP_TRY(launch_warm(b, o.warm_m, o.warm_e, s));
  if (!async) {
    HIP_TRY(hipMemcpyAsync(hc, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hc->bad_input & 1)
      return finish(set_err(FS1_ERR_INVALID_ARG, "marginals must be finite and >= 0"));
    if (hc->bad_input & 2)
      return finish(set_err(FS1_ERR_INVALID_ARG,
                            "warm start: mantissas must be finite and >= 0, |exponents| <= 2^20, "
                            "and (plain domain) every scaling finite in the working precision"));
    if (!(hc->sum_mu > 0.0) || !(hc->sum_nu > 0.0))
      return finish(set_err(FS1_ERR_INVALID_ARG, "marginals must have positive mass"));
    if (std::fabs(hc->sum_mu - hc->sum_nu) > 1e-10 * hc->sum_mu)
      return finish(set_err(FS1_ERR_INVALID_ARG, "unequal masses: sum mu = %.17g, sum nu = %.17g",
                            hc->sum_mu, hc->sum_nu));
    if (o.err_history)
      HIP_TRY(hipMemsetAsync(o.err_history, 0xFF, sizeof(double) * (size_t(o.itr_max) + 1), s));
  }

  const ScanConsts k = make_scan_consts(h, eps, R);
  const CarryConsts kc = make_carry_consts(h, eps, C, nchunks);
  HIP_TRY(launch_init_state(b, k, warm, s));

  // diagnostic timing: events around every half-iteration kernel of a batch
  // (a fixed workspace means the caller cannot allocate: no timing events)
  const bool prof = ctx->profiling != 0 && !fixed_ws && !async;
  if (prof && ctx->events.size() < 4) {
    while (ctx->events.size() < 4) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e));
      ctx->events.push_back(e);
    }
  }
  // algorithmic bytes of one half-iteration kernel: read the vector fed to K,
  // read the marginal, write the new vector; a checked psi-half also reads the
  // old psi and the binary64 nu
  const double bytes_half = double(n) * 3.0 * double(es);
  const double bytes_check = double(n) * (double(es) + (dt == FS1_F64 ? 0.0 : 8.0));

  // Mid-size grids whose vectors fit in the registers of the co-resident
  // workgroups run all iterations in one cooperative launch.
  const bool resident = res_threads > 0 && usable_resident(b);
  // the absorption variant runs the general path where the grid does not fit
  // one workgroup
  const bool tau_general = tau_mode && !resident;
  const bool persistent =
      !resident && !tau_general && (o.flags & FS1_FLAG_PERSISTENT) && usable_persistent(b, h / eps);
  const bool fused = !resident && !persistent && !tau_general &&
                     !(o.flags & FS1_FLAG_GENERAL) && usable_fused(b, h / eps);
  // larger grids in the log domain: the streaming large-grid kernel
  const bool large = !resident && !persistent && !tau_general && !fused &&
                     !(o.flags & FS1_FLAG_GENERAL) && usable_large(b, h / eps);
  // the fused and large-grid paths, and the general path where
  // solve_tiled(), iterate on the tile layout
  const bool tiled =
      fused || large || (!resident && !persistent && !tau_general && solve_tiled(b));
  if (tau_general) {
    tb.tau = o.tau;
    tb.eps = eps;
    HIP_TRY(launch_tau_init(b, tb, s));
  }
  if (fused || persistent) HIP_TRY(launch_decay_table(b, k, s));
  if (fused) HIP_TRY(launch_fused_init(b, k, s));
  if (tiled) HIP_TRY(launch_relayout(b, true, 0, s));
  if (large) HIP_TRY(launch_large_pack(b, k, s));
  if (persistent || resident) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof) {
      e0 = ctx->events[0];
      e1 = ctx->events[1];
      HIP_TRY(hipEventRecord(e0, s));
    }
    if (resident) {
      HIP_TRY(launch_resident(b, k, o.itr_max, o.check_every, tol, s));
    } else {
      HIP_TRY(hipMemsetAsync(epoch, 0, size_t(nchunks) * sizeof(int), s));
      HIP_TRY(launch_persistent(b, k, o.itr_max, o.check_every, tol, epoch, s));
    }
    if (prof) HIP_TRY(hipEventRecord(e1, s));
  }
  if ((persistent || resident) && !async) {
    HIP_TRY(hipMemcpyAsync(hc, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hc->barrier_timeout)
      return finish(set_err(FS1_ERR_INTERNAL, "persistent solve: grid barrier timed out"));
    if (prof) {
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, ctx->events[0], ctx->events[1]));
      const int its = hc->fail ? hc->fail_iter : hc->iters_done;
      ctx->prof_ms += ms;
      ctx->prof_launches += 1;
      // per iteration: two halves, plus the checked psi-halves' extra reads
      const int checks = its > 0 ? (its - 1) / o.check_every + 1 : 0;
      ctx->prof_bytes += 2.0 * bytes_half * its + bytes_check * checks;
    }
  }

  // Algorithm 1: while l < itr_max and err(l) > tol
  int l = (persistent || resident) ? o.itr_max : 0;
  bool stopped = persistent || resident;
  int batch = 0;
  // diagnostic timing: the fused path's launches are short, so whole polling
  // batches are bracketed (back-to-back kernels run without gaps, and batch
  // time / launches is the average kernel duration without per-launch event
  // overhead); the general path's half-iteration kernel is bracketed alone,
  // in the first iteration of a timed batch (its carry kernels are not counted)
  const bool per_launch = !fused && !tau_general;
  while (l < o.itr_max && !stopped) {
    const int l0 = l;
    const int l_end = std::min(o.itr_max, l + o.sync_every);
    const bool timed = prof && (batch % ctx->profiling) == 0;
    if (timed && !per_launch) HIP_TRY(hipEventRecord(ctx->events[0], s));
    for (; l < l_end; ++l) {
      const int check = (l % o.check_every) == 0;
      if (fused) {
        HIP_TRY(launch_fused_half(b, k, l, check, tol, true, s));
        HIP_TRY(launch_fused_half(b, k, l, check, tol, false, s));
      } else if (large) {
        const bool ev = timed && l == l0;
        HIP_TRY(launch_large_half(b, k, kc, l, check, tol, true, s,
                                  ev ? ctx->events[0] : nullptr, ev ? ctx->events[1] : nullptr));
        HIP_TRY(launch_large_half(b, k, kc, l, check, tol, false, s,
                                  ev ? ctx->events[2] : nullptr, ev ? ctx->events[3] : nullptr));
      } else if (tau_general) {
        HIP_TRY(launch_tau_half(b, tb, k, kc, l, check, tol, true, s));
        HIP_TRY(launch_tau_half(b, tb, k, kc, l, check, tol, false, s));
      } else {
        const bool ev = timed && l == l0;
        HIP_TRY(launch_half_psi(b, k, kc, l, check, tol, s, ev ? ctx->events[0] : nullptr,
                                ev ? ctx->events[1] : nullptr));
        HIP_TRY(launch_half_phi(b, k, kc, l, check, tol, s, ev ? ctx->events[2] : nullptr,
                                ev ? ctx->events[3] : nullptr));
      }
    }
    if (timed && !per_launch) HIP_TRY(hipEventRecord(ctx->events[1], s));
    // (the asynchronous solve issues every launch: those after the stop
    // return at once)
    if (async) continue;
    HIP_TRY(hipMemcpyAsync(hc, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    stopped = hc->done != 0;
    // a batch in which the solve stopped contains launches that returned at
    // once; only batches in which every launch did its work are counted
    if (timed && !stopped) {
      float ms = 0.0f;
      if (per_launch) {
        float ms2 = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, ctx->events[0], ctx->events[1]));
        HIP_TRY(hipEventElapsedTime(&ms2, ctx->events[2], ctx->events[3]));
        ctx->prof_ms += double(ms) + double(ms2);
        ctx->prof_launches += 2;
        ctx->prof_bytes += 2.0 * bytes_half + ((l0 % o.check_every) == 0 ? bytes_check : 0.0);
      } else {
        HIP_TRY(hipEventElapsedTime(&ms, ctx->events[0], ctx->events[1]));
        ctx->prof_ms += ms;
        ctx->prof_launches += 2 * (l - l0);
        for (int i = l0; i < l; ++i)
          ctx->prof_bytes += 2.0 * bytes_half + ((i % o.check_every) == 0 ? bytes_check : 0.0);
      }
    }
    ++batch;
  }
  int gbuf = 0;
  int l_final = o.itr_max;
  if (async) {
    // the final psi's buffer is known on the device only: moved to buffer 0
    if (!persistent && !resident) HIP_TRY(launch_select_psi(b, o.itr_max, s));
  } else {
    HIP_TRY(hipMemcpyAsync(hc, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hc->fail) {
      out->iterations = hc->fail_iter;
      out->converged = 0;
      return finish(set_err(FS1_ERR_NONFINITE,
                            "a scaling became non-finite at iteration %d (abnormal termination)",
                            hc->fail_iter + 1));
    }
    if (hc->done && hc->stop_iter >= 0) l_final = hc->stop_iter;
    // the persistent and resident kernels leave their final psi in buffer 0
    gbuf = (persistent || resident) ? 0 : (l_final & 1);
  }

  if (tau_general) HIP_TRY(launch_tau_finish(b, tb, gbuf, s));
  if (large) HIP_TRY(launch_large_unpack(b, gbuf, s));
  if (tiled) HIP_TRY(launch_relayout(b, false, gbuf, s));
  HIP_TRY(launch_finalize(b, k, kc, gbuf, h, s));
  if (o.flags & 1) HIP_TRY(launch_potentials(b, gbuf, o.potentials_out, s));
  if (o.state_m) HIP_TRY(launch_state_out(b, gbuf, o.state_m, o.state_e, s));
  if (async) {
    HIP_TRY(launch_result(b, dev_out, tol, o.itr_max, s));
    return finish(FS1_OK);
  }
  HIP_TRY(hipMemcpyAsync(hc, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  out->w1 = hc->w1;
  out->marginal_err = hc->err_final;
  out->mu_err = hc->mu_err;
  out->iterations = l_final;
  out->converged = !(hc->err_final > tol) ? 1 : 0;
  out->absorptions = tau_mode ? hc->absorptions : 0;
  if (!std::isfinite(hc->w1) || !std::isfinite(hc->err_final)) {
    return finish(set_err(FS1_ERR_NONFINITE, "non-finite cost or marginal error"));
  }
  return finish(FS1_OK);
}

}  // namespace host
}  // namespace fs1

extern "C" {

int fs1_kv_apply_2d(fs1_ctx* ctx, const void* x, void* y, int64_t n1, int64_t n2, double h1,
                    double h2, double eps, int dt) {
  return fs1::kv_apply_2d(ctx, x, y, n1, n2, h1, h2, eps, dt);
}

int fs1_kv_apply_nd(fs1_ctx* ctx, const void* x, void* y, int ndim, const int64_t* dims,
                    const double* h, double eps, int dt) {
  return fs1::kv_apply_grid(ctx, x, y, ndim, dims, h, eps, dt);
}

// the defaulting and checks of the grid solves before their bodies
static bool grid_solve_prologue(fs1_ctx* ctx, const double* mu, const double* nu,
                                const fs1_opts* opts_in, fs1_result* out, fs1_opts* o,
                                int* st) {
  if (!ctx) {
    *st = set_err(FS1_ERR_INVALID_ARG, "null context");
    return false;
  }
  if (!out) {
    *st = set_err(FS1_ERR_INVALID_ARG, "null result pointer");
    return false;
  }
  std::memset(out, 0, sizeof(*out));
  out->w1 = NAN;
  out->marginal_err = NAN;
  out->mu_err = NAN;
  fs1_opts_default(o);
  if (opts_in) *o = *opts_in;
  if (o->itr_max < 0) o->itr_max = 10000;
  if (o->check_every < 1) o->check_every = 1;
  if (o->sync_every < 1) o->sync_every = 16;
  if ((mu && !aligned16(mu)) || (nu && !aligned16(nu))) {
    out->status = set_err(FS1_ERR_INVALID_ARG, "device arrays must be 16-byte aligned");
    *st = out->status;
    return false;
  }
  return true;
}

int fs1_solve_nd(fs1_ctx* ctx, const double* mu, const double* nu, int ndim, const int64_t* dims,
                 const double* h, double eps, double tol, const fs1_opts* opts_in,
                 fs1_result* out) {
  fs1_opts o;
  int st = FS1_OK;
  if (!grid_solve_prologue(ctx, mu, nu, opts_in, out, &o, &st)) return st;
  return fs1::solve_grid(ctx, mu, nu, ndim, dims, h, eps, tol, o, out);
}

int fs1_solve_2d(fs1_ctx* ctx, const double* mu, const double* nu, int64_t n1, int64_t n2,
                 double h1, double h2, double eps, double tol, const fs1_opts* opts_in,
                 fs1_result* out) {
  if (!ctx) return set_err(FS1_ERR_INVALID_ARG, "null context");
  if (!out) return set_err(FS1_ERR_INVALID_ARG, "null result pointer");
  std::memset(out, 0, sizeof(*out));
  out->w1 = NAN;
  out->marginal_err = NAN;
  out->mu_err = NAN;
  fs1_opts o;
  fs1_opts_default(&o);
  if (opts_in) o = *opts_in;
  if (o.itr_max < 0) o.itr_max = 10000;
  if (o.check_every < 1) o.check_every = 1;
  if (o.sync_every < 1) o.sync_every = 16;
  if ((mu && !aligned16(mu)) || (nu && !aligned16(nu))) {
    out->status = set_err(FS1_ERR_INVALID_ARG, "device arrays must be 16-byte aligned");
    return out->status;
  }
  return fs1::solve_2d(ctx, mu, nu, n1, n2, h1, h2, eps, tol, o, out);
}

int fs1_solve_batched(fs1_ctx* ctx, const double* mu_packed, const double* nu_packed,
                      const int64_t* offsets, int32_t B, const double* eps, const double* tol,
                      const fs1_opts* opts, fs1_result* out) {
  std::vector<double> he, ht;
  const int st = host_params(ctx, opts, B, &eps, &tol, he, ht);
  if (st) return st;
  return batched_entry(ctx, mu_packed, nu_packed, offsets, B, eps, tol, opts, out, nullptr);
}

int fs1_solve_batched_config(fs1_ctx* ctx, const double* mu_packed, const double* nu_packed,
                             const int64_t* offsets, int32_t B, const double* eps,
                             const double* tol, const fs1_opts* opts, const int32_t* run_length,
                             const int32_t* threads, fs1_result* out) {
  if (!ctx) return set_err(FS1_ERR_INVALID_ARG, "null context");
  std::vector<double> he, ht;
  const int pst = host_params(ctx, opts, B, &eps, &tol, he, ht);
  if (pst) return pst;
  const int dt = opts ? opts->dtype : FS1_F64;
  if (opts && opts->domain != FS1_LOG)
    return set_err(FS1_ERR_INVALID_ARG, "a forced configuration needs the log domain");
  if (B > 0 && (!run_length || !offsets))
    return set_err(FS1_ERR_INVALID_ARG, "bad batch arguments");
  std::vector<BatchCfg> cfg(size_t(std::max(B, 0)));
  for (int32_t i = 0; i < B; ++i) {
    const int r = run_length[i];
    const int nt = threads ? threads[i] : 0;
    if (nt == 0 ? !batch_shared_r_ok(dt, r) : !batch_resident_ok(dt, r, nt))
      return set_err(FS1_ERR_INVALID_ARG,
                     "instance %d: no batched kernels for run length %d on %d threads", i, r, nt);
    const int64_t n = offsets[i + 1] - offsets[i];
    if (eps && eps[i] > 0.0 && n > 0 && r > pick_run_length(dt, true, (1.0 / double(n)) / eps[i]))
      return set_err(FS1_ERR_INVALID_ARG, "instance %d: run length %d exceeds what h/eps allows",
                     i, r);
    if (nt > 0 && n > int64_t(nt) * r)
      return set_err(FS1_ERR_INVALID_ARG, "instance %d does not fit %d threads x %d", i, nt, r);
    cfg[size_t(i)] = BatchCfg{r, nt};
  }
  return batched_entry(ctx, mu_packed, nu_packed, offsets, B, eps, tol, opts, out, cfg.data());
}

}  // extern "C"

namespace {

int batched_entry(fs1_ctx* ctx, const double* mu_packed, const double* nu_packed,
                  const int64_t* offsets, int32_t B, const double* eps, const double* tol,
                  const fs1_opts* opts, fs1_result* out, const BatchCfg* force) {
  if (!ctx) return set_err(FS1_ERR_INVALID_ARG, "null context");
  if (B < 0 || (B > 0 && (!offsets || !eps || !tol || !out || !mu_packed || !nu_packed)))
    return set_err(FS1_ERR_INVALID_ARG, "bad batch arguments");
  if (B == 0) return FS1_OK;
  if (offsets[0] != 0) return set_err(FS1_ERR_INVALID_ARG, "offsets[0] must be 0");
  fs1_opts o;
  fs1_opts_default(&o);
  if (opts) o = *opts;
  if (o.itr_max < 0) o.itr_max = 10000;
  if (o.check_every < 1) o.check_every = 1;
  if (o.sync_every < 1) o.sync_every = 16;
  if (o.dtype != FS1_F64 && o.dtype != FS1_F32)
    return set_err(FS1_ERR_INVALID_ARG, "bad dtype %d", o.dtype);
  if (o.domain != FS1_PLAIN && o.domain != FS1_LOG)
    return set_err(FS1_ERR_INVALID_ARG, "bad domain %d", o.domain);
  if (!aligned16(mu_packed) || !aligned16(nu_packed))
    return set_err(FS1_ERR_INVALID_ARG, "device arrays must be 16-byte aligned");
  for (int32_t i = 0; i < B; ++i) {
    const int64_t n = offsets[i + 1] - offsets[i];
    if (n < 1) return set_err(FS1_ERR_INVALID_ARG, "instance %d is empty", i);
    if (n > int64_t(INT32_MAX) / 2) return set_err(FS1_ERR_INVALID_ARG, "instance %d too long", i);
    if (!(tol[i] >= 0.0)) return set_err(FS1_ERR_INVALID_ARG, "instance %d: tol must be >= 0", i);
    const int st = check_h_eps(n, 1.0 / double(n), eps[i]);
    if (st) return set_err(st, "instance %d: %s", i, std::string(last_error_text()).c_str());
  }
  for (int32_t i = 0; i < B; ++i) {
    std::memset(&out[i], 0, sizeof(out[i]));
    out[i].w1 = NAN;
    out[i].marginal_err = NAN;
    out[i].mu_err = NAN;
  }
  if (o.domain == FS1_PLAIN) {
    // the plain domain keeps Algorithm 1's unscaled arithmetic: one solve at a time
    fs1_opts so = o;
    so.h = 0.0;
    so.flags = 0;
    so.potentials_out = nullptr;
    so.err_history = nullptr;
    so.warm_m = nullptr;
    so.warm_e = nullptr;
    so.state_m = nullptr;
    so.state_e = nullptr;
    for (int32_t i = 0; i < B; ++i) {
      const int64_t a = offsets[i];
      if (!aligned16(mu_packed + a) || !aligned16(nu_packed + a)) {
        out[i].status = set_err(FS1_ERR_INVALID_ARG,
                                "plain domain: instance %d must start 16-byte aligned", i);
        continue;
      }
      fs1_solve(ctx, mu_packed + a, nu_packed + a, offsets[i + 1] - a, eps[i], tol[i], &so,
                &out[i]);
    }
    return FS1_OK;
  }
  return batch_solve(ctx, mu_packed, nu_packed, offsets, B, eps, tol, o, out, force);
}

}  // namespace
