// fs1_server.cpp -- request loop with continuous batching (include/fs1.h,
// fs1_server_*).
//
// The server owns one device pool, sized by the memory budget at creation,
// laid out as the batched solve's padded arrays (fs1_batch.h): element slots
// of 256 entries, chunk ids (each with its 256 per-run exponents and its chunk
// aggregates) and instance slots.  Three first-fit range allocators hand out
// those resources at admission and take them back at completion, so requests
// of any size come and go while others keep iterating.  A step is:
//   1. admit queued requests in order while they fit: stage their
//      descriptions, scatter them into their slots, pack their marginals,
//      validate them and publish their initial aggregates;
//   2. run iters_per_step iterations of every admitted request (one launch per
//      half-iteration and run-length class over the chunks of the admitted
//      requests, replayed from a graph that is recaptured when that set
//      changes);
//   3. read which requests stopped (a device ring written by the kernels that
//      stop them), finalise just those and turn them into completions.
// A request's iteration count starts at its admission (its l0), so its
// arithmetic is the same whenever it was admitted and whatever runs beside it.
#include <hip/hip_runtime.h>

#include <string>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

#include "fs1.h"
#include "fs1_batch.h"
#include "fs1_host.h"
#include "fs1_internal.h"
#include "fs1_tune.h"

using namespace fs1;
using namespace fs1::host;

namespace {

constexpr int kSlot = kBlock;  // entries per element slot (a chunk of R = 1)

// First-fit allocator of ranges [start, start + len) of [0, capacity).
class RangeAlloc {
 public:
  void reset(int64_t cap) {
    free_.clear();
    if (cap > 0) free_[0] = cap;
    used_ = 0;
  }
  int64_t alloc(int64_t len) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < len) continue;
      const int64_t start = it->first, rest = it->second - len;
      free_.erase(it);
      if (rest > 0) free_[start + len] = rest;
      used_ += len;
      return start;
    }
    return -1;
  }
  void release(int64_t start, int64_t len) {
    used_ -= len;
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        prev->second += len;
        return;
      }
    }
    free_[start] = len;
  }
  int64_t used() const { return used_; }

 private:
  std::map<int64_t, int64_t> free_;
  int64_t used_ = 0;
};

struct Request {
  int64_t ticket;
  const double* mu;
  const double* nu;
  int64_t n;
  double eps;
  double tol;
};

struct Active {
  int64_t ticket = -1;
  int R = 0;
  int64_t slot0 = 0, nslot = 0;
  int chunk0 = 0, nch = 0;
  double tol = 0.0;
  int64_t admitted_step = 0;
};

}  // namespace

struct fs1_server {
  fs1_ctx* ctx = nullptr;
  fs1_server_opts o{};
  char* mem = nullptr;
  int64_t nslots = 0;          // element slots; also the capacity of chunk ids
  size_t bytes_per_slot = 0;
  RangeAlloc slots, chunks;
  BatchBufs z{};
  ChunkRef* alist = nullptr;   // chunk lists of the admitted requests, per run length
  ChunkRef* wlist = nullptr;   // chunk lists of a set-up or a finalisation
  int* dilist = nullptr;       // instance list of a set-up or a finalisation
  InstInfo* dsinfo = nullptr;  // admission staging
  InstState* dsstate = nullptr;
  InstState* dgather = nullptr;  // finalised states
  char* hmem = nullptr;        // pinned host staging
  InstInfo* hsinfo = nullptr;
  InstState* hsstate = nullptr;
  InstState* hgather = nullptr;
  int* hilist = nullptr;
  ChunkRef* hlist = nullptr;
  int* hring = nullptr;
  int* hcount = nullptr;
  std::deque<Request> queue;
  std::vector<Active> act;     // by instance slot
  std::vector<char> retiring;  // by instance slot: stopped, being finalised
  std::vector<int> free_inst;
  std::map<int, std::vector<ChunkRef>> running;  // run length -> chunks of admitted requests
  std::vector<BatchGroup> groups;           // the launch groups over alist
  int64_t next_ticket = 0, steps = 0, completed_total = 0, consumed = 0, nactive = 0;
  int iter_base = 0;
  std::deque<fs1_completion> done;
  hipGraphExec_t gexec = nullptr;
  bool dirty = true;
  bool inflight = false;  // FS1_FLAG_SERVER_OVERLAP: iterations enqueued, not yet retired
};

namespace {

size_t elem_bytes(int dt) {
  const size_t es = dt == FS1_F64 ? 8 : 4;
  return 16 + (dt == FS1_F32 ? 8 : 0) + 3 * es;
}

// Carve the pool: element arrays (nslots * 256 entries), run arrays and chunk
// arrays (nslots chunk ids), instance arrays (max_active).
void carve(fs1_server* v, Carve& w) {
  const int dt = v->o.dtype;
  const size_t es = dt == FS1_F64 ? 8 : 4;
  const int64_t ne = v->nslots * kSlot, nc = v->nslots, nr = v->nslots * kBlock;
  const int64_t ni = v->o.max_active;
  BatchBufs& z = v->z;
  z.mu64 = static_cast<double*>(w.take(ne * 8));
  z.nu64 = static_cast<double*>(w.take(ne * 8));
  z.mu32 = dt == FS1_F32 ? w.take(ne * 4) : nullptr;
  z.nu32 = dt == FS1_F32 ? w.take(ne * 4) : nullptr;
  z.vF = w.take(ne * es);
  z.vG[0] = w.take(ne * es);
  z.vG[1] = w.take(ne * es);
  z.eF = static_cast<int*>(w.take(nr * 4));
  z.eG[0] = static_cast<int*>(w.take(nr * 4));
  z.eG[1] = static_cast<int*>(w.take(nr * 4));
  z.aggF = static_cast<ChunkAgg*>(w.take(nc * sizeof(ChunkAgg)));
  z.aggG = static_cast<ChunkAgg*>(w.take(nc * sizeof(ChunkAgg)));
  z.agg2 = w.take(nc * 48);
  z.part = static_cast<double*>(w.take(nc * 8));
  z.part2 = static_cast<double*>(w.take(nc * 8));
  z.part3 = static_cast<double*>(w.take(nc * 8));
  v->alist = static_cast<ChunkRef*>(w.take(nc * sizeof(ChunkRef)));
  v->wlist = static_cast<ChunkRef*>(w.take(nc * sizeof(ChunkRef)));
  z.inst = static_cast<InstInfo*>(w.take(ni * sizeof(InstInfo)));
  z.st = static_cast<InstState*>(w.take(ni * sizeof(InstState)));
  v->dsinfo = static_cast<InstInfo*>(w.take(ni * sizeof(InstInfo)));
  v->dsstate = static_cast<InstState*>(w.take(ni * sizeof(InstState)));
  v->dgather = static_cast<InstState*>(w.take(ni * sizeof(InstState)));
  v->dilist = static_cast<int*>(w.take(ni * 4));
  z.ring = static_cast<int*>(w.take(ni * 4));
  z.iter_base = static_cast<int*>(w.take(2 * sizeof(int)));
}

int64_t request_slots(int dt, int64_t n, double eps, int* R_out, int* nch_out) {
  const int R = shared_run_length(dt, n, (1.0 / double(n)) / eps);
  const int64_t C = int64_t(kBlock) * R;
  const int64_t nch = (n + C - 1) / C;
  *R_out = R;
  *nch_out = int(nch);
  return nch * R;  // element slots (a chunk is R slots); nch chunk ids
}

fs1_result to_result(const InstState& t, const Active& a, int itr_max) {
  fs1_result r;
  std::memset(&r, 0, sizeof(r));
  r.w1 = NAN;
  r.marginal_err = NAN;
  r.mu_err = NAN;
  if (t.invalid) {
    r.status = FS1_ERR_INVALID_ARG;
  } else if (t.fail) {
    r.iterations = t.fail_iter;
    r.status = FS1_ERR_NONFINITE;
  } else {
    r.iterations = t.stop_iter >= 0 ? t.stop_iter : itr_max;
    r.w1 = t.w1;
    r.marginal_err = t.err;
    r.mu_err = t.mu_err;
    r.converged = !(t.err > a.tol) ? 1 : 0;
    r.status = (std::isfinite(t.w1) && std::isfinite(t.err)) ? FS1_OK : FS1_ERR_NONFINITE;
  }
  return r;
}

// Launch lists per run length of the given chunk records, uploaded to `dev`.
int upload_groups(fs1_server* v, const std::map<int, std::vector<ChunkRef>>& by_r, ChunkRef* dev,
                  std::vector<BatchGroup>* out) {
  out->clear();
  int64_t at = 0;
  for (const auto& kv : by_r) {
    if (kv.second.empty()) continue;
    std::memcpy(v->hlist + at, kv.second.data(), kv.second.size() * sizeof(ChunkRef));
    BatchGroup g{kv.first, dev + at, int(kv.second.size())};
    out->push_back(g);
    at += int64_t(kv.second.size());
  }
  if (at > 0) {
    HIP_TRY(hipMemcpyAsync(dev, v->hlist, size_t(at) * sizeof(ChunkRef), hipMemcpyHostToDevice,
                           v->ctx->stream));
    // the pinned list is read by that copy: finish it before the host reuses it
    HIP_TRY(hipStreamSynchronize(v->ctx->stream));
  }
  return FS1_OK;
}

int admit(fs1_server* v) {
  const int dt = v->o.dtype;
  std::map<int, std::vector<ChunkRef>> fresh;
  int count = 0;
  while (!v->queue.empty() && !v->free_inst.empty()) {
    const Request& q = v->queue.front();
    int R, nch;
    const int64_t ns = request_slots(dt, q.n, q.eps, &R, &nch);
    const int64_t s0 = v->slots.alloc(ns);
    if (s0 < 0) break;
    const int64_t c0 = v->chunks.alloc(nch);
    if (c0 < 0) {
      v->slots.release(s0, ns);
      break;
    }
    const int b = v->free_inst.back();
    v->free_inst.pop_back();
    Active& a = v->act[b];
    a.ticket = q.ticket;
    a.R = R;
    a.slot0 = s0;
    a.nslot = ns;
    a.chunk0 = int(c0);
    a.nch = nch;
    a.tol = q.tol;
    a.admitted_step = v->steps;
    v->hsinfo[count] = make_inst_info(q.mu, q.nu, s0 * kSlot, q.n, int(c0), R,
                                      1.0 / double(q.n), q.eps, q.tol, v->iter_base);
    InstState& t = v->hsstate[count];
    std::memset(&t, 0, sizeof(t));
    t.stop_iter = -1;
    t.fail_iter = INT_MAX;
    t.last_check = -1;
    t.last_err = NAN;
    v->hilist[count] = b;
    std::vector<ChunkRef>& fl = fresh[R];
    std::vector<ChunkRef>& rl = v->running[R];
    for (int i = 0; i < nch; ++i) {
      const ChunkRef r = chunk_ref(v->hsinfo[count], b, i);
      fl.push_back(r);
      rl.push_back(r);
    }
    ++count;
    ++v->nactive;
    v->queue.pop_front();
  }
  if (count == 0) return FS1_OK;
  hipStream_t s = v->ctx->stream;
  HIP_TRY(hipMemcpyAsync(v->dsinfo, v->hsinfo, count * sizeof(InstInfo), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(v->dsstate, v->hsstate, count * sizeof(InstState), hipMemcpyHostToDevice,
                         s));
  HIP_TRY(hipMemcpyAsync(v->dilist, v->hilist, count * sizeof(int), hipMemcpyHostToDevice, s));
  HIP_TRY(launch_batch_admit(v->z, v->dsinfo, v->dsstate, v->dilist, count, s));
  std::vector<BatchGroup> g;
  int st = upload_groups(v, fresh, v->wlist, &g);  // (synchronises: staging reusable)
  if (st) return st;
  HIP_TRY(launch_batch_setup(v->z, g.data(), int(g.size()), v->dilist, count, s));
  v->dirty = true;
  return FS1_OK;
}

int run_iterations(fs1_server* v) {
  if (v->nactive == 0) return FS1_OK;
  const bool use_graph = !(v->o.flags & FS1_FLAG_NO_GRAPH);
  if (v->dirty) {
    if (v->gexec) {
      (void)hipGraphExecDestroy(v->gexec);
      v->gexec = nullptr;
    }
    int st = upload_groups(v, v->running, v->alist, &v->groups);
    if (st) return st;
    if (use_graph) {
      st = capture_iterations(v->ctx, v->z, v->groups, v->o.iters_per_step, &v->gexec);
      if (st) return st;
    }
    v->dirty = false;
  }
  if (v->gexec) {
    HIP_TRY(hipGraphLaunch(v->gexec, v->ctx->stream));
  } else {
    HIP_TRY(launch_batch_iterations(v->z, v->groups.data(), int(v->groups.size()),
                                    v->o.iters_per_step, v->ctx->stream));
  }
  v->iter_base += v->o.iters_per_step;
  return FS1_OK;
}

int retire(fs1_server* v, int32_t* produced) {
  hipStream_t s = v->ctx->stream;
  HIP_TRY(hipMemcpyAsync(v->hcount, v->z.ndone, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t total = *v->hcount;
  const int64_t fresh = total - v->consumed;
  if (fresh <= 0) return FS1_OK;
  const int cap = v->o.max_active;
  HIP_TRY(hipMemcpyAsync(v->hring, v->z.ring, size_t(cap) * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::map<int, std::vector<ChunkRef>> fin;
  int count = 0;
  for (int64_t k = v->consumed; k < total; ++k) {
    const int b = v->hring[k % cap];
    v->hilist[count++] = b;
    v->retiring[b] = 1;
  }
  // one stable pass per run length: the stopped requests' chunks go to the
  // finalisation lists (each request's in chunk order; a chunk's finalisation
  // reads only what earlier launches published, so the order across requests
  // does not matter), the others stay in the running lists in their order
  for (auto& kv : v->running) {
    std::vector<ChunkRef>& rl = kv.second;
    std::vector<ChunkRef>* l = nullptr;
    size_t w = 0;
    for (const ChunkRef& r : rl) {
      if (v->retiring[r.b]) {
        if (!l) l = &fin[kv.first];
        l->push_back(r);
      } else {
        rl[w++] = r;
      }
    }
    rl.resize(w);
  }
  v->consumed = total;
  HIP_TRY(hipMemcpyAsync(v->dilist, v->hilist, count * sizeof(int), hipMemcpyHostToDevice, s));
  std::vector<BatchGroup> g;
  int st = upload_groups(v, fin, v->wlist, &g);
  if (st) return st;
  HIP_TRY(launch_batch_finalize(v->z, g.data(), int(g.size()), v->dilist, count, v->dgather, s));
  HIP_TRY(hipMemcpyAsync(v->hgather, v->dgather, count * sizeof(InstState), hipMemcpyDeviceToHost,
                         s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < count; ++i) {
    const int b = v->hilist[i];
    Active& a = v->act[b];
    fs1_completion c;
    std::memset(&c, 0, sizeof(c));
    c.ticket = a.ticket;
    c.result = to_result(v->hgather[i], a, v->o.itr_max);
    c.admitted_step = a.admitted_step;
    c.completed_step = v->steps;
    v->done.push_back(c);
    // give the request's resources back (its chunks left the launches above)
    v->slots.release(a.slot0, a.nslot);
    v->chunks.release(a.chunk0, a.nch);
    v->retiring[b] = 0;
    a = Active{};
    v->free_inst.push_back(b);
    --v->nactive;
  }
  v->completed_total += count;
  v->dirty = true;
  if (produced) *produced = count;
  return FS1_OK;
}

}  // namespace

extern "C" {

int fs1_server_opts_default(fs1_server_opts* o) {
  if (!o) return set_err(FS1_ERR_INVALID_ARG, "null opts");
  std::memset(o, 0, sizeof(*o));
  o->hbm_budget = int64_t(1) << 30;
  o->max_active = 4096;
  o->dtype = FS1_F32;
  o->itr_max = 10000;
  o->check_every = 1;
  o->iters_per_step = 16;
  o->flags = 0;
  return FS1_OK;
}

int fs1_server_create(fs1_ctx* ctx, const fs1_server_opts* oin, fs1_server** out) {
  if (!ctx || !out) return set_err(FS1_ERR_INVALID_ARG, "null context or output pointer");
  *out = nullptr;
  fs1_server_opts o;
  fs1_server_opts_default(&o);
  if (oin) o = *oin;
  if (o.itr_max < 0) o.itr_max = 10000;
  if (o.dtype != FS1_F64 && o.dtype != FS1_F32)
    return set_err(FS1_ERR_INVALID_ARG, "bad dtype %d", o.dtype);
  if (o.max_active < 1 || o.check_every < 1 || o.iters_per_step < 1)
    return set_err(FS1_ERR_INVALID_ARG, "max_active, check_every, iters_per_step must be >= 1");
  if (o.hbm_budget < (int64_t(16) << 20))
    return set_err(FS1_ERR_INVALID_ARG, "hbm_budget must be at least 16 MiB");
  fs1_server* v = new (std::nothrow) fs1_server();
  if (!v) return set_err(FS1_ERR_NO_MEMORY, "server allocation failed");
  v->ctx = ctx;
  v->o = o;
  // slots that fit the budget: per slot 256 entries of every element array,
  // one chunk id (256 run exponents x 3, aggregates, shares, lists)
  v->bytes_per_slot = size_t(kSlot) * elem_bytes(o.dtype) + 3 * kBlock * 4 +
                      2 * sizeof(ChunkAgg) + 48 + 3 * 8 + 2 * sizeof(ChunkRef);
  const size_t fixed = size_t(o.max_active) * (2 * sizeof(InstInfo) + 3 * sizeof(InstState) + 8) +
                       (size_t(32) << 10);
  v->nslots = o.hbm_budget > int64_t(fixed)
                  ? int64_t((size_t(o.hbm_budget) - fixed) / (v->bytes_per_slot + 64))
                  : 0;
  if (v->nslots < 1) {
    delete v;
    return set_err(FS1_ERR_INVALID_ARG, "hbm_budget too small for max_active = %d",
                   o.max_active);
  }
  Carve probe(nullptr);
  carve(v, probe);
  {
    void* pool = nullptr;
    const int st = dev_alloc(ctx, probe.off, &pool);
    if (st) {
      delete v;
      return set_err(st, "server pool of %zu bytes: %s", probe.off,
                     std::string(last_error_text()).c_str());
    }
    v->mem = static_cast<char*>(pool);
  }
  hipError_t e = hipSuccess;
  Carve w(v->mem);
  carve(v, w);
  v->z.ndone = v->z.iter_base + 1;
  v->z.ring_cap = o.max_active;
  v->z.dtype = o.dtype;
  v->z.itr_max = o.itr_max;
  v->z.check_every = o.check_every;
  v->z.nchunks = v->nslots;
  v->z.nelem = v->nslots * kSlot;
  const size_t ni = size_t(o.max_active);
  const size_t hbytes = ni * (sizeof(InstInfo) + 2 * sizeof(InstState) + 2 * sizeof(int)) +
                        size_t(v->nslots) * sizeof(ChunkRef) + 256;
  e = hipHostMalloc(reinterpret_cast<void**>(&v->hmem), hbytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    dev_free(ctx, v->mem);
    delete v;
    return set_err(FS1_ERR_NO_MEMORY, "hipHostMalloc(%zu) failed: %s", hbytes,
                   hipGetErrorString(e));
  }
  char* h = v->hmem;
  v->hcount = reinterpret_cast<int*>(h);
  h += 64;
  v->hsinfo = reinterpret_cast<InstInfo*>(h);
  h += ni * sizeof(InstInfo);
  v->hsstate = reinterpret_cast<InstState*>(h);
  h += ni * sizeof(InstState);
  v->hgather = reinterpret_cast<InstState*>(h);
  h += ni * sizeof(InstState);
  v->hilist = reinterpret_cast<int*>(h);
  h += ni * sizeof(int);
  v->hring = reinterpret_cast<int*>(h);
  h += ni * sizeof(int);
  v->hlist = reinterpret_cast<ChunkRef*>(h);
  v->slots.reset(v->nslots);
  v->chunks.reset(v->nslots);
  v->act.assign(ni, Active{});
  v->retiring.assign(ni, 0);
  for (int b = o.max_active - 1; b >= 0; --b) v->free_inst.push_back(b);
  e = hipMemsetAsync(v->z.iter_base, 0, 2 * sizeof(int), ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    (void)hipHostFree(v->hmem);
    dev_free(ctx, v->mem);
    delete v;
    return hip_fail(e, "server initialisation");
  }
  *out = v;
  return FS1_OK;
}

int fs1_server_destroy(fs1_server* v) {
  if (!v) return FS1_OK;
  (void)hipStreamSynchronize(v->ctx->stream);
  if (v->gexec) (void)hipGraphExecDestroy(v->gexec);
  if (v->hmem) (void)hipHostFree(v->hmem);
  if (v->mem) dev_free(v->ctx, v->mem);
  delete v;
  return FS1_OK;
}

int fs1_server_submit(fs1_server* v, const double* mu, const double* nu, int64_t n, double eps,
                      double tol, int64_t* ticket) {
  if (!v) return set_err(FS1_ERR_INVALID_ARG, "null server");
  if (!mu || !nu) return set_err(FS1_ERR_INVALID_ARG, "null marginal");
  if (n > int64_t(INT32_MAX) / 2) return set_err(FS1_ERR_INVALID_ARG, "n too large");
  int st = check_h_eps(n, n > 0 ? 1.0 / double(n) : 1.0, eps);
  if (st) return st;
  if (!(tol >= 0.0)) return set_err(FS1_ERR_INVALID_ARG, "tol must be >= 0");
  int R, nch;
  const int64_t ns = request_slots(v->o.dtype, n, eps, &R, &nch);
  if (ns > v->nslots || nch > v->nslots)
    return set_err(FS1_ERR_INVALID_ARG, "request of n = %lld exceeds the server's budget",
                   (long long)n);
  Request q{v->next_ticket++, mu, nu, n, eps, tol};
  v->queue.push_back(q);
  if (ticket) *ticket = q.ticket;
  return FS1_OK;
}

int fs1_server_step(fs1_server* v, int32_t* completed) {
  if (!v) return set_err(FS1_ERR_INVALID_ARG, "null server");
  if (completed) *completed = 0;
  const bool overlap = (v->o.flags & FS1_FLAG_SERVER_OVERLAP) != 0;
  if (v->inflight) {
    // the previous call's iterations: wait for them and finalise what they stopped
    v->inflight = false;
    const int st = retire(v, completed);
    if (st) return st;
  }
  if (v->queue.empty() && v->nactive == 0) return FS1_OK;
  int st = admit(v);
  if (st) return st;
  st = run_iterations(v);
  if (st) return st;
  ++v->steps;
  if (overlap) {
    v->inflight = true;
    return FS1_OK;
  }
  return retire(v, completed);
}

int fs1_server_poll(fs1_server* v, fs1_completion* out, int32_t max, int32_t* count) {
  if (!v || !count || (max > 0 && !out)) return set_err(FS1_ERR_INVALID_ARG, "bad poll arguments");
  int32_t k = 0;
  while (k < max && !v->done.empty()) {
    out[k++] = v->done.front();
    v->done.pop_front();
  }
  *count = k;
  return FS1_OK;
}

int fs1_server_get_info(fs1_server* v, fs1_server_info* out) {
  if (!v || !out) return set_err(FS1_ERR_INVALID_ARG, "null server or output");
  out->queued = int64_t(v->queue.size());
  out->active = v->nactive;
  out->completed = v->completed_total;
  out->steps = v->steps;
  out->bytes_in_use = v->slots.used() * int64_t(v->bytes_per_slot);
  out->bytes_total = v->nslots * int64_t(v->bytes_per_slot);
  return FS1_OK;
}

}  // extern "C"
