// fs1_tau.hip -- the threshold form of the stabilisation on the
// multi-workgroup path (see fs1_tau.h).
//
//   k_tau_from_log : initial state, log layout -> scaled form, chunk maxima
//   k_tau_decide   : the absorption test at the top of an iteration
//   k_half_tau     : one half-iteration (pack, recursions with the chunk
//                    carries, stopping-error share, update, chunk maximum,
//                    aggregates of the new packed vector); the psi-half also
//                    performs the absorption when the test fired
//   k_tau_to_log   : final state back to the log layout
#include <algorithm>
#include <climits>

#include "fs1_device.h"
#include "fs1_internal.h"
#include "fs1_resident.h"
#include "fs1_tau.h"

namespace fs1 {

namespace {

constexpr int kNWt = kBlock / kWave;

// Workgroup maximum of non-negative values (valid in every thread).
__device__ __forceinline__ double chunk_max(double v, double* red) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) v = fmax(v, __shfl_xor(v, d));
  if (lane == 0) red[w] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int i = 1; i < kNWt; ++i) r = fmax(r, red[i]);
  __syncthreads();
  return r;
}

template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_tau_from_log(T* v, const int* e, double* pot,
                                                         double* pm) {
  __shared__ double red[kNWt];
  const int64_t run = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t base = run * R;
  T x[R];
  res_load<T, R>(v, base, x);
  const int E = e[run];
  double mx = 0.0;
  double z[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    x[j] = ldx(x[j], E);
    mx = fmax(mx, double(x[j]));
    z[j] = 0.0;
  }
  res_store<T, R>(v, base, x);
  res_store<double, R>(pot, base, z);
  mx = chunk_max(mx, red);
  if (threadIdx.x == 0) pm[blockIdx.x] = mx;
}

template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_tau_to_log(T* v, int* e, const double* pot,
                                                       double inv_eps) {
  const int64_t run = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t base = run * R;
  T x[R], y[R];
  double p[R];
  res_load<T, R>(v, base, x);
  res_load<double, R>(pot, base, p);
  const int E = tau_pack<T, R>(x, p, inv_eps, y);
  res_store<T, R>(v, base, y);
  e[run] = E;
}

// The test of the threshold form: largest scaled entry of phit and psit above
// tau.  Sets the flag read by the iteration's psi-half and counts absorptions.
__global__ __launch_bounds__(kCarryBlock) void k_tau_decide(const double* pmF, const double* pmG,
                                                            int64_t nchunks, double tau,
                                                            int* absorb, Ctrl* ctrl) {
  constexpr int NW = kCarryBlock / kWave;
  __shared__ double red[NW];
  if (ctrl->done || ctrl->fail) return;
  double m = 0.0;
  for (int64_t c = threadIdx.x; c < nchunks; c += kCarryBlock) m = fmax(m, fmax(pmF[c], pmG[c]));
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) m = fmax(m, __shfl_xor(m, d));
  if (lane == 0) red[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int i = 1; i < NW; ++i) r = fmax(r, red[i]);
    const int a = r > tau ? 1 : 0;
    *absorb = a;
    if (a) ctrl->absorptions += 1;
  }
}

enum TauMode { T_PSI = 0, T_PHI = 1 };

template <typename T>
struct TauHalfArgs {
  T* vin;              // scaled vector fed to K (phit / psit)
  double* pin;         // its potential (alpha / beta)
  T* vold;             // psi-half: psit^l (error term; absorbed in place)
  double* pout;        // potential of the output (beta / alpha)
  T* vout;             // the updated scaled vector
  const double* m64;   // marginal, binary64 (error; update when T = double)
  const float* m32;    // marginal, binary32 (update when T = float)
  const ChunkAgg* carry;
  ChunkAgg* agg_out;   // aggregates of the new packed vector
  double* part;        // per-chunk error shares
  double* pm_out;      // per-chunk maximum of the new scaled vector
  const int* absorb;
  Ctrl* ctrl;
  int64_t n;
  int l;
  int check;
  double eps;
  double inv_eps;
  CarryFix cfix;
};

template <typename T, int R>
__device__ __forceinline__ void absorb_run(T (&v)[R], double (&pot)[R], double eps) {
#pragma unroll
  for (int j = 0; j < R; ++j)
    if (v[j] > T(0)) {
      pot[j] += eps * log(double(v[j]));
      v[j] = T(1);
    }
}

template <typename T, int R, int MODE>
__global__ __launch_bounds__(kBlock) void k_half_tau(TauHalfArgs<T> a, ScanConsts k) {
  __shared__ ScanLds<S1<T>, kNWt> sh;
  __shared__ double red[kNWt];
  const int64_t run = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t base = run * R;
  const bool want_err = MODE == T_PSI && a.check;
  // every global load is issued before any of them is waited for
  const int done = a.ctrl->done;
  const int ab = MODE == T_PSI ? *a.absorb : 0;
  T x[R];
  double pin[R], pout[R];
  res_load<T, R>(a.vin, base, x);
  res_load<double, R>(a.pin, base, pin);
  res_load<double, R>(a.pout, base, pout);
  T old[R];
  if constexpr (MODE == T_PSI) res_load<T, R>(a.vold, base, old);
  double m64[R];
  if (want_err || sizeof(T) == 8) res_load<double, R>(a.m64, base, m64);
  T mg[R];
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int j = 0; j < R; ++j) mg[j] = T(m64[j]);
  } else {
    res_load<T, R>(reinterpret_cast<const T*>(a.m32), base, mg);
  }
  const ChunkAgg cg = chunk_carry(a.carry, a.cfix, blockIdx.x);
  if (done) return;
  if constexpr (MODE == T_PSI) {
    if (ab) {
      // absorption at the top of the iteration: phi = e^{alpha/eps} phit and
      // psi^l = e^{beta/eps} psit^l keep their values, so the packed input and
      // the error term do not change; psit^l is rewritten too, since a stop
      // at this iteration returns it with the new beta
      absorb_run<T, R>(x, pin, a.eps);
      absorb_run<T, R>(old, pout, a.eps);
      res_store<T, R>(a.vin, base, x);
      res_store<double, R>(a.pin, base, pin);
      res_store<T, R>(a.vold, base, old);
      res_store<double, R>(a.pout, base, pout);
    }
  }
  T xp[R];
  const int E = tau_pack<T, R>(x, pin, a.inv_eps, xp);
  const Lam<T> L = lam_of<T>(k);
  T af, abk;
  run_aggs<T, R>(xp, L, af, abk);
  Dec<T> dec[7];
  lane_decays<T>(k, dec);
  S1<T> cf, cb;
  block_scan<S1<T>, kNWt, T>(S1<T>{{af, E}}, S1<T>{{abk, E}}, dec, S1<T>{from64<T>(cg.f)},
                             S1<T>{from64<T>(cg.b)}, &cf, &cb, nullptr, nullptr, sh);
  const S1<T> lcf = cf.shift(step_decay<T>(k)), lcb = cb.shift(step_decay<T>(k));
  int eref = max(local_exponent<T, R>(xp, E), max(lcf.v.e, lcb.v.e));
  if (eref == kExpZero) eref = 0;
  T xf[R];
#pragma unroll
  for (int j = 0; j < R; ++j) xf[j] = ldx(xp[j], E - eref);
  T y[R];  // (K e^{pot/eps} vin)_j * 2^-eref
  run_apply<T, R>(xf, ldx(lcf.v.m, lcf.v.e - eref), ldx(lcb.v.m, lcb.v.e - eref), L, y);

  // error share sum_j | psi^l_j (K^T phi^l)_j - nu_j |, binary64
  if (want_err) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j)
      s += fabs(scale2(double(old[j]) * double(y[j]), double(eref) + pout[j] * a.inv_eps * kLog2E) -
                m64[j]);
    const double tot = block_sum<kNWt>(s, red);
    if (threadIdx.x == 0) a.part[blockIdx.x] = tot;
  }

  // update: out = marg / (e^{pout/eps} (K in))  (zero marginal -> zero)
  T q[R];
  bool bad = false;
  tau_update<T, R>(mg, y, eref, pout, a.inv_eps, q, bad);
  res_store<T, R>(a.vout, base, q);
  if (bad) {
    atomicOr(&a.ctrl->fail, 1);
    atomicMin(&a.ctrl->fail_iter, a.l);
  }
  double mx = 0.0;
#pragma unroll
  for (int j = 0; j < R; ++j)
    if (isfinite(q[j])) mx = fmax(mx, double(q[j]));
  mx = chunk_max(mx, red);
  if (threadIdx.x == 0) a.pm_out[blockIdx.x] = mx;
  // aggregates of the new packed vector (what the next half packs)
  T xq[R];
  const int Eo = tau_pack<T, R>(q, pout, a.inv_eps, xq);
  T nf, nb;
  run_aggs<T, R>(xq, L, nf, nb);
  S1<T> gf, gb;
  block_scan<S1<T>, kNWt, T>(S1<T>{{nf, Eo}}, S1<T>{{nb, Eo}}, dec, S1<T>::zero(), S1<T>::zero(),
                             nullptr, nullptr, &gf, &gb, sh);
  if (threadIdx.x == 0) {
    a.agg_out[blockIdx.x].f = to64(gf.v);
    a.agg_out[blockIdx.x].b = to64(gb.v);
  }
}

template <typename T, int R>
struct TauOps {
  static hipError_t init(const SolveBufs& b, const TauBufs& t, hipStream_t s) {
    const unsigned g = unsigned(b.nchunks);
    k_tau_from_log<T, R><<<g, kBlock, 0, s>>>(static_cast<T*>(b.vF), b.eF, t.potF, t.pmF);
    k_tau_from_log<T, R><<<g, kBlock, 0, s>>>(static_cast<T*>(b.vG[0]), b.eG[0], t.potG, t.pmG);
    return hipGetLastError();
  }
  static hipError_t half(const SolveBufs& b, const TauBufs& t, const ScanConsts& k,
                         const CarryConsts& kc, int l, int check, double tol, bool psi,
                         hipStream_t s) {
    TauHalfArgs<T> a{};
    a.cfix = carry_fix_of(kc);
    a.n = b.n;
    a.l = l;
    a.check = check;
    a.ctrl = b.ctrl;
    a.carry = b.carry;
    a.part = b.part;
    a.absorb = t.absorb;
    a.eps = t.eps;
    a.inv_eps = 1.0 / t.eps;
    const int cur = l & 1, nxt = (l + 1) & 1;
    const unsigned g = unsigned(b.nchunks);
    hipError_t e;
    if (psi) {
      k_tau_decide<<<1, kCarryBlock, 0, s>>>(t.pmF, t.pmG, b.nchunks, t.tau, t.absorb, b.ctrl);
      e = launch_solve_carry(1, b.aggF, b.carry, kc, b.ctrl, nullptr, nullptr, l, 0, tol, s);
      if (e != hipSuccess) return e;
      a.vin = static_cast<T*>(b.vF);
      a.pin = t.potF;
      a.vold = static_cast<T*>(b.vG[cur]);
      a.pout = t.potG;
      a.vout = static_cast<T*>(b.vG[nxt]);
      a.m64 = b.nu;
      a.m32 = static_cast<const float*>(b.nu32);
      a.agg_out = b.aggG;
      a.pm_out = t.pmG;
      k_half_tau<T, R, T_PSI><<<g, kBlock, 0, s>>>(a, k);
    } else {
      e = launch_solve_carry(2, b.aggG, b.carry, kc, b.ctrl, b.part, b.err_hist, l, check, tol, s);
      if (e != hipSuccess) return e;
      a.vin = static_cast<T*>(b.vG[nxt]);
      a.pin = t.potG;
      a.vold = nullptr;
      a.pout = t.potF;
      a.vout = static_cast<T*>(b.vF);
      a.m64 = b.mu;
      a.m32 = static_cast<const float*>(b.mu32);
      a.agg_out = b.aggF;
      a.pm_out = t.pmF;
      k_half_tau<T, R, T_PHI><<<g, kBlock, 0, s>>>(a, k);
    }
    return hipGetLastError();
  }
  static hipError_t finish(const SolveBufs& b, const TauBufs& t, int gbuf, hipStream_t s) {
    const unsigned g = unsigned(b.nchunks);
    const double ie = 1.0 / t.eps;
    k_tau_to_log<T, R><<<g, kBlock, 0, s>>>(static_cast<T*>(b.vF), b.eF, t.potF, ie);
    k_tau_to_log<T, R><<<g, kBlock, 0, s>>>(static_cast<T*>(b.vG[gbuf]), b.eG[gbuf], t.potG, ie);
    return hipGetLastError();
  }
};

template <typename F>
hipError_t tau_dispatch(const SolveBufs& b, F&& f) {
  if (b.dtype == 0) {
    if (b.R == 8) return f(TauOps<double, 8>{});
    if (b.R == 4) return f(TauOps<double, 4>{});
    return f(TauOps<double, 1>{});
  }
  switch (b.R) {
    case 16: return f(TauOps<float, 16>{});
    case 8: return f(TauOps<float, 8>{});
    case 4: return f(TauOps<float, 4>{});
    default: return f(TauOps<float, 1>{});
  }
}

}  // namespace

size_t tau_bytes(int64_t npad, int64_t nchunks) {
  return 2 * size_t(npad) * sizeof(double) + 2 * size_t(nchunks) * sizeof(double) + 256;
}

hipError_t launch_tau_init(const SolveBufs& b, const TauBufs& t, hipStream_t s) {
  return tau_dispatch(b, [&](auto ops) { return decltype(ops)::init(b, t, s); });
}

hipError_t launch_tau_half(const SolveBufs& b, const TauBufs& t, const ScanConsts& k,
                           const CarryConsts& kc, int l, int check, double tol, bool psi,
                           hipStream_t s) {
  return tau_dispatch(
      b, [&](auto ops) { return decltype(ops)::half(b, t, k, kc, l, check, tol, psi, s); });
}

hipError_t launch_tau_finish(const SolveBufs& b, const TauBufs& t, int gbuf, hipStream_t s) {
  return tau_dispatch(b, [&](auto ops) { return decltype(ops)::finish(b, t, gbuf, s); });
}

}  // namespace fs1
