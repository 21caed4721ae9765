// fs1_persist.hip -- the whole FS-1 iteration (Algorithm 1) in one cooperative
// launch, for grids whose scaling vectors fit in the registers of the
// co-resident workgroups.
//
// Every workgroup owns one chunk (256 threads x R elements) and keeps phi,
// psi and the marginals of its chunk in registers for the whole solve.  A
// half-iteration is
//   (1) the chunk's forward / backward recursion aggregates (Sec. 3,
//       eq. (recursion)) of the vector fed to K, published to global memory
//       with a per-chunk epoch flag (no central counter);
//   (2) a wait, by every workgroup, for the flags of all chunks;
//   (3) the chunk carries, recomputed by every workgroup from all published
//       aggregates, and the in-chunk recursions with those carries;
//   (4) the Sinkhorn update (Sec. 2: psi = nu / K^T phi, then phi = mu / K psi)
//       and, on checked iterations, the chunk's share of Algorithm 1's stopping
//       error.
// After the wait of each phi-half every workgroup sums the error shares in
// the same fixed order, so all of them take the same stop decision.
//
// Inside a chunk the recursions run in plain floating point relative to one
// power-of-two frame per chunk.  Every output of a chunk is within
// lambda^(chunk length) of the chunk's largest contribution, so this frame is
// exact up to rounding as long as chunk length * h/eps * log2(e) stays inside
// the exponent range of the working precision (checked on the host).
#include <climits>

#include "fs1_device.h"
#include "fs1_frame.h"
#include "fs1_internal.h"

namespace fs1 {

namespace {

constexpr int kCarryMaxP = 8;
constexpr int kMaxPersistChunks = kCarryMaxP * kBlock / 2;  // 1024: the carry prefetch's reach
// log2 span budget of the per-chunk frame (see the file comment)
constexpr double kFrameLog2Span64 = 900.0;
constexpr double kFrameLog2Span32 = 80.0;

struct PersistArgs {
  const double* mu;       // binary64 marginals: error terms; update when T = double
  const double* nu;
  const float* mu32;      // binary32 copies: update when T = float
  const float* nu32;
  void* vF;               // in: initial phi; out: final phi
  void* vG;               // in: initial psi; out: final psi
  int* eF;                // run exponents of phi / psi (in and out)
  int* eG;
  ChunkAgg* A0;           // chunk aggregates of phi (psi-halves)
  ChunkAgg* A1;           // chunk aggregates of psi (phi-halves)
  double* part;           // per-chunk stopping-error shares
  Ctrl* ctrl;
  int* epoch;             // per chunk: the last half whose aggregates it published
  double* err_hist;
  int64_t n;
  int nchunks;
  int itr_max;
  int check_every;
  double tol;
  const XF64* dtab;       // lambda^(chunk length * d), d < nchunks
};

// Publication of one half's chunk aggregates (and error shares) between
// co-resident workgroups (cooperative launch), without a central counter.
// Everything that crosses workgroups (aggregates, shares, flags) is written
// and read with device-scope atomics, which on gfx950 are loads and stores
// with the device-scope cache policy (sc1): they are performed at the
// device's coherence point, past the per-XCD L2, so the L2 write-back and
// invalidate of an agent-scope release or acquire fence -- which order
// ordinary accesses that may sit in L2 -- have nothing to order here (and
// cost 4.7x in solve time at N = 2^20).  Ordering of the device-scope
// accesses: every wave waits for its own stores to complete (vmcnt(0): the
// stores are acknowledged once performed at that point) before the
// workgroup barrier; only then does thread 0 store the workgroup's epoch flag
// `gen`.  The first wave polls, with a bounded spin, until every chunk's flag
// reaches `gen`; the loads that read the aggregates and shares are issued
// only after the flag loads that saw `gen` have returned (they depend on them
// through the loop exit and the barrier), and read the same coherence point.
// A wait that exceeds the bound sets ctrl->barrier_timeout; every workgroup
// that sees it (or times out itself) returns false, and the caller leaves its
// iteration loop, so after at most one bounded wait every workgroup runs to
// completion.
constexpr int kWaitStoresDone = 0x0F70;  // s_waitcnt vmcnt(0) expcnt(7) lgkmcnt(15)

__device__ __forceinline__ bool publish_sync(int* epoch, int gen, int nchunks, Ctrl* ctrl) {
  __shared__ int sok;
  __builtin_amdgcn_s_waitcnt(kWaitStoresDone);  // this wave's stores have completed
  __syncthreads();  // ... in every wave of the workgroup
  if (threadIdx.x == 0)
    __hip_atomic_store(&epoch[blockIdx.x], gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // the first wavefront polls every chunk's flag (relaxed device-coherent
  // loads, all of a round issued together) until all have reached gen
  if (threadIdx.x < kWave) {
    int ok = 1;
    unsigned spins = 0;
    for (;;) {
      int mn = INT_MAX;
      for (int c = threadIdx.x; c < nchunks; c += kWave)
        mn = min(mn, __hip_atomic_load(&epoch[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (__all(mn >= gen)) break;
      if (++spins > (1u << 22) ||
          __hip_atomic_load(&ctrl->barrier_timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        if (threadIdx.x == 0)
          __hip_atomic_store(&ctrl->barrier_timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (threadIdx.x == 0) sok = ok;
  }
  __syncthreads();
  return sok != 0;
}

// Device-coherent loads of aggregates published by this launch.
struct CoherentLoad {
  __device__ XF64 operator()(const XF64* p) const {
    XF64 v;
    v.m = __hip_atomic_load(const_cast<double*>(&p->m), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v.e = __hip_atomic_load(const_cast<int*>(&p->e), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v.pad = 0;
    return v;
  }
};

// Thread 0 stores the chunk's aggregates with device-coherent stores.
template <typename T>
__device__ __forceinline__ void publish_coherent(const FastDec<T>& D, const T* sf, const T* sb,
                                                 int ein, ChunkAgg* A) {
  if (threadIdx.x == 0) {
    XF64 f, b;
    chunk_aggs<T>(D, sf, sb, ein, f, b);
    ChunkAgg* p = A + blockIdx.x;
    __hip_atomic_store(&p->f.m, f.m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&p->f.e, f.e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&p->b.m, b.m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&p->b.e, b.e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Chunk carries from the prefetched segments with the decay table in LDS
// (lambda^(C d), C the chunk length; mantissas in tdm, exponents in tde): the
// forward carry of chunk b is the sum over c < b of lambda^(C (b-1-c)) F_c,
// the backward one the sum over c > b of lambda^(C (c-b-1)) B_c.  The terms
// are independent: each wave takes the largest exponent of its terms (an
// integer max), sums the terms aligned to it in binary64, and the two waves
// of a direction are combined in extended range (forward into scar[0],
// backward into scar[1]).
template <int CMAX>
__device__ __forceinline__ void carry_finish_lds(const CarryItems<CMAX>& it, int b,
                                                 const double* tdm, const int* tde, XF64* red4,
                                                 XF64* scar) {
  const bool fwd = threadIdx.x < kBlock / 2;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  double tm[CMAX];
  int te[CMAX];
  int emax = kExpZero;
#pragma unroll
  for (int i = 0; i < CMAX; ++i) {
    const int c = it.lo + i;
    if (c < it.hi && it.m[i] != 0.0) {
      const int d = fwd ? b - 1 - c : c - b - 1;
      tm[i] = it.m[i] * tdm[d];
      te[i] = it.e[i] + tde[d];
      emax = max(emax, te[i]);
    } else {
      tm[i] = 0.0;
      te[i] = kExpZero;
    }
  }
  emax = wave_max(emax);
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < CMAX; ++i) s += ldexp(tm[i], te[i] - emax);
  s = wave_sum(s);
  if (lane == 0) red4[w] = to64(xnorm(s, emax));
  __syncthreads();
  if (threadIdx.x == 0) {
    scar[0] = to64(xnorm(xadd(XF<double>{red4[0].m, red4[0].e}, XF<double>{red4[1].m, red4[1].e})));
    scar[1] = to64(xnorm(xadd(XF<double>{red4[2].m, red4[2].e}, XF<double>{red4[3].m, red4[3].e})));
  }
  __syncthreads();
}

template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_persist(PersistArgs a, ScanConsts k) {
  __shared__ T sf[kNW];
  __shared__ T sb[kNW];
  __shared__ int smax[kNW];
  __shared__ double red[kNW];
  __shared__ XF64 scar[2];
  __shared__ XF64 red4[kNW];
  __shared__ int sdec;
  __shared__ double tdm[kMaxPersistChunks];  // lambda^(C d), d = 0..nchunks-1
  __shared__ int tde[kMaxPersistChunks];

  const int lane = threadIdx.x & (kWave - 1);
  const int64_t run = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t base = run * R;
  const int64_t n = a.n;
  int gen = 0;  // halves published so far

  // register-resident state
  T ph[R], ps[R], pso[R], mu[R], nu[R];
  load_run<T, R>(static_cast<const T*>(a.vF), base, n, ph, T(0));
  load_run<T, R>(static_cast<const T*>(a.vG), base, n, ps, T(0));
  int eph = a.eF[run];
  int eps = a.eG[run];
  int epso = eps;
  if constexpr (sizeof(T) == 8) {
    load_run<T, R>(reinterpret_cast<const T*>(a.mu), base, n, mu, T(0));
    load_run<T, R>(reinterpret_cast<const T*>(a.nu), base, n, nu, T(0));
  } else {
    load_run<T, R>(reinterpret_cast<const T*>(a.mu32), base, n, mu, T(0));
    load_run<T, R>(reinterpret_cast<const T*>(a.nu32), base, n, nu, T(0));
  }
#pragma unroll
  for (int j = 0; j < R; ++j) pso[j] = ps[j];

  for (int d = threadIdx.x; d < a.nchunks; d += kBlock) {
    const XF64 p = a.dtab[d];
    tdm[d] = p.m;
    tde[d] = p.e;
  }  // read after local_scan's barrier
  const Lam<T> L = lam_of<T>(k);
  const FastDec<T> D = make_fast_dec<T>(k, lane);
  HalfState<T, R> hs;
  T y[R];
  int l = 0;
  int stop_iter = -1;
  bool failed = false;
  for (; l < a.itr_max; ++l) {
    const bool check = (l % a.check_every) == 0;
    // ---------------- psi-half: psi <- nu / K^T phi ----------------
    local_scan<T, R>(ph, eph, L, D, sf, sb, smax, hs);
    publish_coherent<T>(D, sf, sb, hs.ein, a.A0);
    if (!publish_sync(a.epoch, ++gen, a.nchunks, a.ctrl)) break;
    // the carry loads and the failure flag of the previous phi-half travel
    // together; that slot is written only before the wait, so every
    // workgroup reads the same value
    CarryItems<kCarryMaxP> items;
    carry_prefetch<kCarryMaxP>(a.A0, blockIdx.x, a.nchunks, items, CoherentLoad());
    if (threadIdx.x == 0)
      sdec = __hip_atomic_load(&a.ctrl->fail_half[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (sdec) {
      failed = true;
      break;
    }
    carry_finish_lds<kCarryMaxP>(items, blockIdx.x, tdm, tde, red4, scar);
    int eap = frame_apply<T, R>(L, D, sf, sb, scar, hs, y);
    if (check) {
      double s = 0.0;
      if constexpr (sizeof(T) == 8) {
        // binary64: the registers already hold nu
#pragma unroll
        for (int j = 0; j < R; ++j)
          if (base + j < n) s += fabs(ldexp(ps[j] * y[j], eps + eap) - nu[j]);
      } else {
        double nu64[R];
        load_run<double, R>(a.nu, base, n, nu64, 0.0);
#pragma unroll
        for (int j = 0; j < R; ++j)
          if (base + j < n) s += fabs(ldexp(double(ps[j]) * double(y[j]), eps + eap) - nu64[j]);
      }
      const double tot = block_sum<kNW>(s, red);
      if (threadIdx.x == 0)
        __hip_atomic_store(&a.part[blockIdx.x], tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    bool bad = false;
    T q[R];
    const int eq = update_run<T, R>(nu, y, eap, q, bad);
    if (bad) {
      atomicOr(&a.ctrl->fail_half[0], 1);
      atomicOr(&a.ctrl->fail, 1);
      atomicMin(&a.ctrl->fail_iter, l);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
      pso[j] = ps[j];
      ps[j] = q[j];
    }
    epso = eps;
    eps = eq;

    // ---------------- phi-half: phi <- mu / K psi ----------------
    local_scan<T, R>(ps, eps, L, D, sf, sb, smax, hs);
    publish_coherent<T>(D, sf, sb, hs.ein, a.A1);
    if (!publish_sync(a.epoch, ++gen, a.nchunks, a.ctrl)) break;
    // the carry loads, the failure flag of this iteration's psi-half (written
    // only before the wait) and the error shares of its stopping test travel
    // together; every thread sums its shares in chunk order and the block in
    // wave order, so every workgroup takes the same decision
    carry_prefetch<kCarryMaxP>(a.A1, blockIdx.x, a.nchunks, items, CoherentLoad());
    {
      double s = 0.0;
      if (check) {
#pragma unroll
        for (int i = 0; i < kMaxPersistChunks / kBlock; ++i) {
          const int c = int(threadIdx.x) + i * kBlock;
          if (c < a.nchunks)
            s += __hip_atomic_load(&a.part[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      if (threadIdx.x == 0)
        sdec = __hip_atomic_load(&a.ctrl->fail_half[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s = wave_sum(s);
      if (lane == 0) red[threadIdx.x / kWave] = s;
    }
    __syncthreads();
    if (sdec) {
      failed = true;
      break;
    }
    if (check) {
      double err = 0.0;
#pragma unroll
      for (int v = 0; v < kNW; ++v) err += red[v];
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.ctrl->last_err = err;
        a.ctrl->last_check = l;
        if (a.err_hist) a.err_hist[l] = err;
      }
      if (!(err > a.tol)) {
        // stop with (phi^l, psi^l): undo this iteration's psi update
#pragma unroll
        for (int j = 0; j < R; ++j) ps[j] = pso[j];
        eps = epso;
        stop_iter = l;
        break;
      }
    }
    carry_finish_lds<kCarryMaxP>(items, blockIdx.x, tdm, tde, red4, scar);
    eap = frame_apply<T, R>(L, D, sf, sb, scar, hs, y);
    bad = false;
    const int ef = update_run<T, R>(mu, y, eap, q, bad);
    if (bad) {
      atomicOr(&a.ctrl->fail_half[1], 1);
      atomicOr(&a.ctrl->fail, 1);
      atomicMin(&a.ctrl->fail_iter, l);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) ph[j] = q[j];
    eph = ef;
  }
  // final state for the finalisation kernels
  store_run<T, R>(static_cast<T*>(a.vF), base, n, ph);
  store_run<T, R>(static_cast<T*>(a.vG), base, n, ps);
  a.eF[run] = eph;
  a.eG[run] = eps;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.ctrl->iters_done = (stop_iter >= 0) ? stop_iter : l;
    if (stop_iter >= 0) {
      a.ctrl->done = 1;
      a.ctrl->stop_iter = stop_iter;
    }
    if (failed) a.ctrl->done = 1;
  }
}

template <typename T, int R>
hipError_t persist_t(const SolveBufs& b, const ScanConsts& k, int itr_max, int check_every,
                     double tol, int* epoch, hipStream_t s) {
  PersistArgs a{};
  a.mu = b.mu;
  a.nu = b.nu;
  a.mu32 = static_cast<const float*>(b.mu32);
  a.nu32 = static_cast<const float*>(b.nu32);
  a.vF = b.vF;
  a.vG = b.vG[0];
  a.eF = b.eF;
  a.eG = b.eG[0];
  a.A0 = b.aggF;
  a.A1 = b.aggG;
  a.part = b.part;
  a.ctrl = b.ctrl;
  a.epoch = epoch;
  a.err_hist = b.err_hist;
  a.n = b.n;
  a.nchunks = int(b.nchunks);
  a.itr_max = itr_max;
  a.check_every = check_every;
  a.tol = tol;
  a.dtab = b.dtab;
  ScanConsts kk = k;
  void* args[] = {&a, &kk};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_persist<T, R>),
                                    dim3(unsigned(b.nchunks)), dim3(kBlock), args, 0, s);
}

template <typename T, int R>
int max_coresident() {
  int dev = 0, ncu = 0, per = 0, coop = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
      !coop)
    return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per, reinterpret_cast<const void*>(&k_persist<T, R>), kBlock, 0) != hipSuccess)
    return 0;
  return per * ncu;
}

}  // namespace

bool usable_persistent(const SolveBufs& b, double c) {
  if (!b.absorb) return false;  // the plain domain keeps the paper's unscaled arithmetic
  const double span = double(kBlock) * double(b.R) * c * kLog2E;
  if (b.dtype == 0) {
    if (b.R != 8 || span > kFrameLog2Span64) return false;
  } else {
    if (b.R != 16 || span > kFrameLog2Span32) return false;
  }
  if (b.nchunks > kMaxPersistChunks) return false;
  const int cap = b.dtype == 0 ? max_coresident<double, 8>() : max_coresident<float, 16>();
  return b.nchunks <= cap;
}

hipError_t launch_persistent(const SolveBufs& b, const ScanConsts& k, int itr_max,
                             int check_every, double tol, int* epoch, hipStream_t s) {
  if (b.dtype == 0) return persist_t<double, 8>(b, k, itr_max, check_every, tol, epoch, s);
  return persist_t<float, 16>(b, k, itr_max, check_every, tol, epoch, s);
}

}  // namespace fs1
