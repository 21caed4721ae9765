// fs1_persist.hip -- the whole FS-1 iteration (Algorithm 1) in one cooperative
// launch, for grids whose scaling vectors fit in the registers of the
// co-resident workgroups.
//
// Every workgroup owns one chunk (256 threads x R elements) and keeps phi,
// psi and the marginals of its chunk in registers for the whole solve.  A
// half-iteration is
//   (1) the chunk's forward / backward recursion aggregates (Sec. 3,
//       eq. (recursion)) of the vector fed to K, published to global memory;
//   (2) one grid barrier;
//   (3) the chunk carries, recomputed by every workgroup from all published
//       aggregates, and the in-chunk recursions with those carries;
//   (4) the Sinkhorn update (Sec. 2: psi = nu / K^T phi, then phi = mu / K psi)
//       and, on checked iterations, the chunk's share of Algorithm 1's stopping
//       error.
// After the barrier of each phi-half every workgroup sums the error shares in
// the same fixed order, so all of them take the same stop decision.
//
// Inside a chunk the recursions run in plain floating point relative to one
// power-of-two frame per chunk.  Every output of a chunk is within
// lambda^(chunk length) of the chunk's largest contribution, so this frame is
// exact up to rounding as long as chunk length * h/eps * log2(e) stays inside
// the exponent range of the working precision (checked on the host).
#include <climits>

#include "fs1_device.h"
#include "fs1_internal.h"

namespace fs1 {

namespace {

constexpr int kNW = kBlock / kWave;
constexpr int kMaxPersistChunks = 2048;
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
  unsigned* bar;          // grid barrier: [0] arrivals, [1] generation
  double* err_hist;
  int64_t n;
  int nchunks;
  int itr_max;
  int check_every;
  double tol;
  Decay cpow[20];         // lambda^(chunk length * 2^s)
};

// Grid barrier over co-resident workgroups (cooperative launch).  The
// arriving thread publishes its workgroup's global writes (device-scope
// release), the last arrival advances the generation, and the others wait for
// it with a bounded spin: a wait that exceeds the bound sets
// ctrl->barrier_timeout and returns, so no wavefront can hang.
// Returns false (in every thread of the workgroup) once any workgroup has given
// up waiting; the caller then leaves its iteration loop, so after one bounded
// wait every workgroup runs to completion.
__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned nblocks, Ctrl* ctrl,
                                             int* sflag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const unsigned arrived =
        __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    if (arrived == nblocks) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(2);
        if (__hip_atomic_load(&ctrl->barrier_timeout, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT) ||
            ++spins > (1u << 22)) {
          __hip_atomic_store(&ctrl->barrier_timeout, 1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    __threadfence();
    *sflag = ok;
  }
  __syncthreads();
  return *sflag != 0;
}

template <typename T>
struct FastDec {
  T step[6];   // lambda^(R 2^s)
  T wave;      // lambda^(64 R)
  T lane_f;    // lambda^(lane R)
  T lane_b;    // lambda^((63 - lane) R)
};

template <typename T>
__device__ __forceinline__ T dec_val(const Decay& d) {
  return T(ldexp(d.m, d.e));
}

template <typename T>
__device__ __forceinline__ FastDec<T> make_fast_dec(const ScanConsts& k, int lane) {
  FastDec<T> D;
#pragma unroll
  for (int s = 0; s < 6; ++s) D.step[s] = dec_val<T>(k.lane[s]);
  D.wave = dec_val<T>(k.lane[6]);
  double mf = 1.0, mb = 1.0;
  int ef = 0, eb = 0;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    if ((lane >> s) & 1) {
      mf *= k.lane[s].m;
      ef += k.lane[s].e;
    }
    if (((kWave - 1 - lane) >> s) & 1) {
      mb *= k.lane[s].m;
      eb += k.lane[s].e;
    }
  }
  D.lane_f = T(ldexp(mf, ef));
  D.lane_b = T(ldexp(mb, eb));
  return D;
}

__device__ __forceinline__ int block_max_int(int v, int* sh) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d));
  if (lane == 0) sh[w] = v;
  __syncthreads();
  int r = sh[0];
#pragma unroll
  for (int i = 1; i < kNW; ++i) r = max(r, sh[i]);
  __syncthreads();
  return r;
}

// xfloat sum over the 64 lanes (same tree in every lane: every lane returns
// the same value).
__device__ __forceinline__ XF<double> wave_xsum(XF<double> v) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) {
    const XF<double> o = {__shfl_xor(v.m, d), __shfl_xor(v.e, d)};
    v = xadd(v, o);
  }
  return xnorm(v);
}

__device__ __forceinline__ XF<double> pow_bits(int64_t d, const Decay* p) {
  XF<double> r = {1.0, 0};
  for (int s = 0; d != 0 && s < 20; ++s, d >>= 1) {
    if (d & 1) r = {r.m * p[s].m, r.e + p[s].e};
  }
  return r;
}

// Forward carry into chunk b (state at the element before the chunk) from the
// forward aggregates of chunks 0..b-1, by one wavefront.
__device__ XF<double> carry_fwd(const ChunkAgg* A, int b, const PersistArgs& a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int seg = (b + kWave - 1) / kWave;
  const int lo = lane * seg;
  const int hi = min(lo + seg, b);
  XF<double> acc = xzero<double>();
  if (lo < hi) {
    const XF<double> cd = {a.cpow[0].m, a.cpow[0].e};
    for (int c = lo; c < hi; ++c) acc = xnorm(xadd(xmul(acc, cd), XF<double>{A[c].f.m, A[c].f.e}));
    acc = xmul(acc, pow_bits(b - hi, a.cpow));  // from the end of chunk hi-1 to the end of b-1
  }
  return wave_xsum(acc);
}

// Backward carry into chunk b (inclusive backward state at the element after
// the chunk) from the backward aggregates of chunks b+1..nchunks-1.
__device__ XF<double> carry_bwd(const ChunkAgg* A, int b, const PersistArgs& a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int first = b + 1;
  const int cnt = a.nchunks - first;
  const int seg = (cnt + kWave - 1) / kWave;
  const int lo = first + lane * seg;
  const int hi = min(lo + seg, a.nchunks);
  XF<double> acc = xzero<double>();
  if (cnt > 0 && lo < hi) {
    const XF<double> cd = {a.cpow[0].m, a.cpow[0].e};
    for (int c = hi - 1; c >= lo; --c)
      acc = xnorm(xadd(xmul(acc, cd), XF<double>{A[c].b.m, A[c].b.e}));
    acc = xmul(acc, pow_bits(lo - first, a.cpow));  // from the start of lo to the start of b+1
  }
  return wave_xsum(acc);
}

template <typename T, int R>
struct HalfState {
  T xf[R];     // input run in the chunk frame
  T exf, exb;  // wave-exclusive carries (chunk frame)
  int ein;     // chunk frame exponent of the input
};

// Phase 1 of a half: frame, thread aggregates, wave scans, chunk aggregates.
template <typename T, int R>
__device__ __forceinline__ void half_aggregate(const T (&x)[R], int ex, const Lam<T>& L,
                                               const FastDec<T>& D, T* sf, T* sb, int* smax,
                                               ChunkAgg* A, HalfState<T, R>& hs) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int eb = block_max_int(local_exponent<T, R>(x, ex), smax);
  hs.ein = (eb == kExpZero) ? 0 : eb;
#pragma unroll
  for (int j = 0; j < R; ++j) hs.xf[j] = ldx(x[j], ex - hs.ein);
  T f, b;
  run_aggs<T, R>(hs.xf, L, f, b);
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int d = 1 << s;
    const T of = __shfl_up(f, d);
    const T ob = __shfl_down(b, d);
    if (lane >= d) f = fma(D.step[s], of, f);
    if (lane + d < kWave) b = fma(D.step[s], ob, b);
  }
  T ef = __shfl_up(f, 1);
  T eb2 = __shfl_down(b, 1);
  hs.exf = (lane == 0) ? T(0) : ef;
  hs.exb = (lane == kWave - 1) ? T(0) : eb2;
  if (lane == kWave - 1) sf[w] = f;
  if (lane == 0) sb[w] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    T gf = T(0), gb = T(0);
#pragma unroll
    for (int v = 0; v < kNW; ++v) gf = fma(D.wave, gf, sf[v]);
#pragma unroll
    for (int v = kNW - 1; v >= 0; --v) gb = fma(D.wave, gb, sb[v]);
    const XF<T> xfw = xnorm(gf, hs.ein);
    const XF<T> xbw = xnorm(gb, hs.ein);
    A[blockIdx.x].f = to64(xfw);
    A[blockIdx.x].b = to64(xbw);
  }
}

// Phase 3 of a half: chunk carries (waves 0 and 1), frame alignment, in-chunk
// recursions.  Returns y = (K in) * 2^-eap in every thread's run.
template <typename T, int R>
__device__ __forceinline__ int half_apply(const ChunkAgg* A, const PersistArgs& a,
                                          const Lam<T>& L, const FastDec<T>& D, const T* sf,
                                          const T* sb, XF64* scar, HalfState<T, R>& hs,
                                          T (&y)[R]) {
  const int w = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int b = blockIdx.x;
  if (w == 0) {
    const XF<double> cf = carry_fwd(A, b, a);
    if (lane == 0) scar[0] = to64(cf);
  } else if (w == 1) {
    const XF<double> cb = carry_bwd(A, b, a);
    if (lane == 0) scar[1] = to64(cb);
  }
  __syncthreads();
  const XF64 cf = scar[0];
  const XF64 cb = scar[1];
  int eap = hs.ein;
  if (cf.m != 0.0) eap = max(eap, cf.e);
  if (cb.m != 0.0) eap = max(eap, cb.e);
  const int sh = hs.ein - eap;  // <= 0: rescale the chunk-frame quantities
  T accf = T(ldexp(cf.m, cf.e - eap));
  T accb = T(ldexp(cb.m, cb.e - eap));
  for (int v = 0; v < w; ++v) accf = fma(D.wave, accf, ldx(sf[v], sh));
  for (int v = kNW - 1; v > w; --v) accb = fma(D.wave, accb, ldx(sb[v], sh));
  const T tcf = fma(D.lane_f, accf, ldx(hs.exf, sh));
  const T tcb = fma(D.lane_b, accb, ldx(hs.exb, sh));
  T xf[R];
#pragma unroll
  for (int j = 0; j < R; ++j) xf[j] = ldx(hs.xf[j], sh);
  run_apply<T, R>(xf, tcf, tcb, L, y);
  return eap;
}

// New run values q = marg / y (zero marginal -> zero), renormalised so that the
// run maximum is in [1/2, 1); returns the run exponent (y is in frame eap).
template <typename T, int R>
__device__ __forceinline__ int update_run(const T (&mg)[R], const T (&y)[R], int eap, T (&q)[R],
                                          bool& bad) {
  T qm = T(0);
#pragma unroll
  for (int j = 0; j < R; ++j) {
    q[j] = (mg[j] == T(0)) ? T(0) : mg[j] / y[j];
    bad |= !isfinite(q[j]);
    if (isfinite(q[j])) qm = fmax(qm, q[j]);
  }
  int kq = 0;
  if (qm > T(0)) frx(qm, &kq);
#pragma unroll
  for (int j = 0; j < R; ++j) q[j] = ldx(q[j], -kq);
  return kq - eap;
}

template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_persist(PersistArgs a, ScanConsts k) {
  __shared__ T sf[kNW];
  __shared__ T sb[kNW];
  __shared__ int smax[kNW];
  __shared__ double red[kNW];
  __shared__ XF64 scar[2];
  __shared__ int sdec;
  __shared__ int sbar;

  const int lane = threadIdx.x & (kWave - 1);
  const int64_t run = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t base = run * R;
  const int64_t n = a.n;
  const unsigned nblocks = gridDim.x;

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
    half_aggregate<T, R>(ph, eph, L, D, sf, sb, smax, a.A0, hs);
    if (!grid_barrier(a.bar, nblocks, a.ctrl, &sbar)) break;
    // failures of the previous phi-half: that slot is written only before this
    // barrier, so every workgroup reads the same value
    if (threadIdx.x == 0)
      sdec = __hip_atomic_load(&a.ctrl->fail_half[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (sdec) {
      failed = true;
      break;
    }
    int eap = half_apply<T, R>(a.A0, a, L, D, sf, sb, scar, hs, y);
    if (check) {
      double s = 0.0;
      double nu64[R];
      load_run<double, R>(a.nu, base, n, nu64, 0.0);
#pragma unroll
      for (int j = 0; j < R; ++j)
        if (base + j < n) s += fabs(ldexp(double(ps[j]) * double(y[j]), eps + eap) - nu64[j]);
      const double tot = block_sum<kNW>(s, red);
      if (threadIdx.x == 0) a.part[blockIdx.x] = tot;
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
    half_aggregate<T, R>(ps, eps, L, D, sf, sb, smax, a.A1, hs);
    if (!grid_barrier(a.bar, nblocks, a.ctrl, &sbar)) break;
    // stopping test of iteration l (every workgroup sums the same shares in
    // the same order) and the failure flag
    if (threadIdx.x < kWave) {
      // failures of this iteration's psi-half (slot written only before the barrier)
      int dec = __hip_atomic_load(&a.ctrl->fail_half[0], __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT) ? 2 : 0;
      if (check && !dec) {
        double s = 0.0;
        for (int c = lane; c < a.nchunks; c += kWave) s += a.part[c];
#pragma unroll
        for (int d = kWave / 2; d >= 1; d >>= 1) s += __shfl_xor(s, d);
        if (lane == 0) {
          if (blockIdx.x == 0) {
            a.ctrl->last_err = s;
            a.ctrl->last_check = l;
            if (a.err_hist) a.err_hist[l] = s;
          }
          if (!(s > a.tol)) dec = 1;
        }
      }
      if (lane == 0) sdec = dec;
    }
    __syncthreads();
    if (sdec == 2) {
      failed = true;
      break;
    }
    if (sdec == 1) {
      // stop with (phi^l, psi^l): undo this iteration's psi update
#pragma unroll
      for (int j = 0; j < R; ++j) ps[j] = pso[j];
      eps = epso;
      stop_iter = l;
      break;
    }
    eap = half_apply<T, R>(a.A1, a, L, D, sf, sb, scar, hs, y);
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
                     double tol, unsigned* bar, hipStream_t s) {
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
  a.bar = bar;
  a.err_hist = b.err_hist;
  a.n = b.n;
  a.nchunks = int(b.nchunks);
  a.itr_max = itr_max;
  a.check_every = check_every;
  a.tol = tol;
  const double cl = k.c_log2e * double(kBlock) * double(R);
  for (int i = 0; i < 20; ++i) a.cpow[i] = make_decay(cl * double(1ll << i));
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
                             int check_every, double tol, unsigned* bar, hipStream_t s) {
  if (b.dtype == 0) return persist_t<double, 8>(b, k, itr_max, check_every, tol, bar, s);
  return persist_t<float, 16>(b, k, itr_max, check_every, tol, bar, s);
}

}  // namespace fs1
