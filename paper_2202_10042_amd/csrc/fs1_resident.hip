// fs1_resident.hip -- the whole FS-1 solve (Algorithm 1) in one workgroup and
// one launch, for grids of at most 1024 runs (n <= 1024 R).
//
// The workgroup keeps phi, psi and the marginals in registers for the whole
// solve (thread t owns entries [t R, t R + R)), so an iteration is two
// workgroup-wide evaluations of the recursions of Sec. 3, eq. (recursion)
// (wavefront scans and one LDS exchange each; there are no chunk carries),
// the Sinkhorn update of Sec. 2 (psi = nu / K^T phi, then phi = mu / K psi)
// and, on checked iterations, the stopping error of Algorithm 1: no global
// memory traffic and no kernel boundary per iteration.  The arithmetic is the
// general path's (per-run exponents renormalised every half in the log
// domain, plain floating point otherwise), so the results agree with it to
// rounding.
#include "fs1_device.h"
#include "fs1_internal.h"

namespace fs1 {

namespace {

struct ResidentArgs {
  const double* mu;       // binary64 marginals, zero-padded to NT * R
  const double* nu;
  const float* mu32;      // binary32 copies (T = float)
  const float* nu32;
  void* vF;               // in: initial phi; out: final phi (NT * R entries)
  void* vG;               // in: initial psi; out: final psi
  int* eF;                // run exponents (NT entries; the log domain only)
  int* eG;
  Ctrl* ctrl;
  double* err_hist;
  int itr_max;
  int check_every;
  double tol;
};

template <typename T, int R>
__device__ __forceinline__ void res_load(const T* p, int64_t base, T (&x)[R]) {
  if constexpr (R % Vec16<T>::n == 0) {
    load_run_z<T, R>(p, base, x);
  } else {
#pragma unroll
    for (int j = 0; j < R; ++j) x[j] = p[base + j];
  }
}

template <typename T, int R>
__device__ __forceinline__ void res_store(T* p, int64_t base, const T (&x)[R]) {
  if constexpr (R % Vec16<T>::n == 0) {
    store_run_z<T, R>(p, base, x);
  } else {
#pragma unroll
    for (int j = 0; j < R; ++j) p[base + j] = x[j];
  }
}

// y * 2^eref = K x over the whole workgroup (x_j * 2^E in this thread's run);
// returns eref (0 in the plain domain).
template <typename T, int R, bool ABSORB, int NW>
__device__ __forceinline__ int res_apply(const T (&x)[R], int E, const Lam<T>& L,
                                         const Dec<T>* dec, const Dec<T>& step,
                                         ScanLds<S1<T>, NW>& sh, T (&y)[R]) {
  T af, ab;
  run_aggs<T, R>(x, L, af, ab);
  S1<T> cf, cb;
  block_scan<S1<T>, NW, T>(S1<T>{{af, E}}, S1<T>{{ab, E}}, dec, S1<T>::zero(), S1<T>::zero(),
                           &cf, &cb, nullptr, nullptr, sh);
  // carries moved one step into the run, in extended range
  const S1<T> lcf = cf.shift(step), lcb = cb.shift(step);
  int eref = 0;
  if constexpr (ABSORB) {
    eref = max(local_exponent<T, R>(x, E), max(lcf.v.e, lcb.v.e));
    if (eref == kExpZero) eref = 0;
  }
  T xf[R];
#pragma unroll
  for (int j = 0; j < R; ++j) xf[j] = ldx(x[j], E - eref);
  run_apply<T, R>(xf, ldx(lcf.v.m, lcf.v.e - eref), ldx(lcb.v.m, lcb.v.e - eref), L, y);
  return eref;
}

// v = marg / (K in) in place (zero marginal -> zero scaling); in the log
// domain the power-of-two part of the run goes into its exponent.  Returns
// the run's new exponent.
template <typename T, int R, bool ABSORB>
__device__ __forceinline__ int res_update(const T (&mg)[R], const T (&y)[R], int eref,
                                          T (&v)[R], bool& bad) {
#pragma unroll
  for (int j = 0; j < R; ++j) {
    v[j] = (mg[j] == T(0)) ? T(0) : mg[j] / y[j];
    bad |= !isfinite(v[j]);
  }
  if constexpr (!ABSORB) {
    return 0;
  } else {
    T qm = T(0);
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (isfinite(v[j])) qm = fmax(qm, v[j]);
    int kq = 0;
    if (qm > T(0)) frx(qm, &kq);
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = ldx(v[j], -kq);
    return kq - eref;
  }
}

template <typename T, int R, bool ABSORB, int NT>
__global__ __launch_bounds__(NT) void k_resident(ResidentArgs a, ScanConsts k) {
  constexpr int NW = NT / kWave;
  __shared__ ScanLds<S1<T>, NW> sh;
  __shared__ double red[NW];
  __shared__ int sstop;
  const int t = threadIdx.x;
  const int64_t base = int64_t(t) * R;

  T ph[R], ps[R], mu[R], nu[R];
  res_load<T, R>(static_cast<const T*>(a.vF), base, ph);
  res_load<T, R>(static_cast<const T*>(a.vG), base, ps);
  int eph = ABSORB ? a.eF[t] : 0;
  int eps = ABSORB ? a.eG[t] : 0;
  if constexpr (sizeof(T) == 8) {
    res_load<T, R>(reinterpret_cast<const T*>(a.mu), base, mu);
    res_load<T, R>(reinterpret_cast<const T*>(a.nu), base, nu);
  } else {
    res_load<T, R>(reinterpret_cast<const T*>(a.mu32), base, mu);
    res_load<T, R>(reinterpret_cast<const T*>(a.nu32), base, nu);
  }
  const Lam<T> L = lam_of<T>(k);
  Dec<T> dec[7];
  lane_decays<T>(k, dec);
  const Dec<T> step = step_decay<T>(k);

  int l = 0;
  int stop_iter = -1, fail_iter = -1;
  T y[R];
  for (; l < a.itr_max; ++l) {
    // psi-half: K^T phi^l (K is symmetric)
    int eref = res_apply<T, R, ABSORB, NW>(ph, eph, L, dec, step, sh, y);
    if ((l % a.check_every) == 0) {
      // stopping test of Algorithm 1 on (phi^l, psi^l), binary64
      double nu64[R];
      if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int j = 0; j < R; ++j) nu64[j] = double(nu[j]);
      } else {
        res_load<double, R>(a.nu, base, nu64);
      }
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < R; ++j) s += fabs(ldexp(double(ps[j]) * double(y[j]), eps + eref) - nu64[j]);
      const double tot = block_sum<NW>(s, red);
      if (t == 0) {
        a.ctrl->last_err = tot;
        a.ctrl->last_check = l;
        if (a.err_hist) a.err_hist[l] = tot;
        sstop = !(tot > a.tol);
      }
      __syncthreads();
      if (sstop) {
        stop_iter = l;
        break;
      }
    }
    bool bad = false;
    eps = res_update<T, R, ABSORB>(nu, y, eref, ps, bad);
    // phi-half: K psi^{l+1}
    eref = res_apply<T, R, ABSORB, NW>(ps, eps, L, dec, step, sh, y);
    eph = res_update<T, R, ABSORB>(mu, y, eref, ph, bad);
    // a non-finite scaling in either half ends the solve (abnormal termination)
    if (__syncthreads_or(bad ? 1 : 0)) {
      fail_iter = l;
      break;
    }
  }
  res_store<T, R>(static_cast<T*>(a.vF), base, ph);
  res_store<T, R>(static_cast<T*>(a.vG), base, ps);
  if constexpr (ABSORB) {
    a.eF[t] = eph;
    a.eG[t] = eps;
  }
  if (t == 0) {
    a.ctrl->iters_done = (stop_iter >= 0) ? stop_iter : l;
    if (stop_iter >= 0) {
      a.ctrl->done = 1;
      a.ctrl->stop_iter = stop_iter;
    }
    if (fail_iter >= 0) {
      a.ctrl->done = 1;
      a.ctrl->fail = 1;
      a.ctrl->fail_iter = fail_iter;
    }
  }
}

template <typename T, int R, bool ABSORB>
hipError_t resident_t(const SolveBufs& b, const ScanConsts& k, int itr_max, int check_every,
                      double tol, hipStream_t s) {
  ResidentArgs a{};
  a.mu = b.mu;
  a.nu = b.nu;
  a.mu32 = static_cast<const float*>(b.mu32);
  a.nu32 = static_cast<const float*>(b.nu32);
  a.vF = b.vF;
  a.vG = b.vG[0];
  a.eF = b.eF;
  a.eG = b.eG[0];
  a.ctrl = b.ctrl;
  a.err_hist = b.err_hist;
  a.itr_max = itr_max;
  a.check_every = check_every;
  a.tol = tol;
  const int nt = resident_threads(b.n, R);
  if (nt == 256) {
    k_resident<T, R, ABSORB, 256><<<1, 256, 0, s>>>(a, k);
  } else if constexpr (R <= 8) {
    if (nt != 1024) return hipErrorInvalidValue;
    k_resident<T, R, ABSORB, 1024><<<1, 1024, 0, s>>>(a, k);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, bool ABSORB>
hipError_t resident_r(const SolveBufs& b, const ScanConsts& k, int itr_max, int check_every,
                      double tol, hipStream_t s) {
  if constexpr (sizeof(T) == 8) {
    switch (b.R) {
      case 8: return resident_t<T, 8, ABSORB>(b, k, itr_max, check_every, tol, s);
      case 1: return resident_t<T, 1, ABSORB>(b, k, itr_max, check_every, tol, s);
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (b.R) {
      case 16: return resident_t<T, 16, ABSORB>(b, k, itr_max, check_every, tol, s);
      case 8: return resident_t<T, 8, ABSORB>(b, k, itr_max, check_every, tol, s);
      case 4: return resident_t<T, 4, ABSORB>(b, k, itr_max, check_every, tol, s);
      case 1: return resident_t<T, 1, ABSORB>(b, k, itr_max, check_every, tol, s);
      default: return hipErrorInvalidValue;
    }
  }
}

}  // namespace

int resident_threads(int64_t n, int R) {
  if (n <= int64_t(256) * R) return 256;
  // 1024 threads leave at most 128 registers each: runs of up to 8
  if (R <= 8 && n <= int64_t(1024) * R) return 1024;
  return 0;
}

int resident_run_length(int64_t n, int rmax) {
  if (n <= int64_t(256) * rmax) return rmax;
  const int r = rmax < 8 ? rmax : 8;
  return n <= int64_t(1024) * r ? r : 0;
}

bool usable_resident(const SolveBufs& b) {
  const bool r_ok = b.dtype == 0 ? (b.R == 8 || b.R == 1)
                                 : (b.R == 16 || b.R == 8 || b.R == 4 || b.R == 1);
  const int nt = resident_threads(b.n, b.R);
  // the state must cover whole allocated runs: nt threads x R entries
  return r_ok && nt > 0 && b.npad == int64_t(nt) * b.R;
}

hipError_t launch_resident(const SolveBufs& b, const ScanConsts& k, int itr_max, int check_every,
                           double tol, hipStream_t s) {
  if (!usable_resident(b)) return hipErrorInvalidValue;
  if (b.dtype == 0)
    return b.absorb ? resident_r<double, true>(b, k, itr_max, check_every, tol, s)
                    : resident_r<double, false>(b, k, itr_max, check_every, tol, s);
  return b.absorb ? resident_r<float, true>(b, k, itr_max, check_every, tol, s)
                  : resident_r<float, false>(b, k, itr_max, check_every, tol, s);
}

}  // namespace fs1
