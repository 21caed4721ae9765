// fs1_resident.hip -- the whole FS-1 solve (Algorithm 1) of one grid in one
// workgroup and one launch, for grids of at most 1024 runs (n <= 1024 R).
//
// The workgroup keeps phi, psi and the marginals in registers for the whole
// solve (fs1_resident.h), so an iteration needs no global memory traffic and
// no kernel boundary.  The arithmetic is the general path's (per-run
// exponents renormalised every half in the log domain, plain floating point
// otherwise), so the results agree with it to rounding.
#include <algorithm>

#include "fs1_device.h"
#include "fs1_internal.h"
#include "fs1_resident.h"

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

template <typename T, int R, bool ABSORB, int NT>
__global__ __launch_bounds__(NT) void k_resident(ResidentArgs a, ScanConsts k) {
  __shared__ ResidentLds<T, NT / kWave> S;
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
  Ctrl* ctrl = a.ctrl;
  double* hist = a.err_hist;
  const ResidentEnd end = resident_iterate<T, R, ABSORB, NT>(
      ph, eph, ps, eps, mu, nu, a.nu + base, k, a.tol, a.itr_max, a.check_every, S,
      [&](int l, double err) {
        ctrl->last_err = err;
        ctrl->last_check = l;
        if (hist) hist[l] = err;
      });
  res_store<T, R>(static_cast<T*>(a.vF), base, ph);
  res_store<T, R>(static_cast<T*>(a.vG), base, ps);
  if constexpr (ABSORB) {
    a.eF[t] = eph;
    a.eG[t] = eps;
  }
  if (t == 0) {
    ctrl->iters_done = (end.stop_iter >= 0) ? end.stop_iter : end.l;
    if (end.stop_iter >= 0) {
      ctrl->done = 1;
      ctrl->stop_iter = end.stop_iter;
    }
    if (end.fail_iter >= 0) {
      ctrl->done = 1;
      ctrl->fail = 1;
      ctrl->fail_iter = end.fail_iter;
    }
  }
}

// The threshold form of the stabilisation (fs1_resident.h): the state enters
// as the plain iteration's initial vectors (exponents 0, potentials 0) and
// leaves in the log domain's layout (per-run exponents) for the common
// finalisation.
template <typename T, int R, int NT>
__global__ __launch_bounds__(NT) void k_resident_tau(ResidentArgs a, ScanConsts k, double tau,
                                                     double eps) {
  __shared__ ResidentLds<T, NT / kWave> S;
  const int t = threadIdx.x;
  const int64_t base = int64_t(t) * R;
  T pt[R], qt[R], mu[R], nu[R];
  double al[R], be[R];
  res_load<T, R>(static_cast<const T*>(a.vF), base, pt);
  res_load<T, R>(static_cast<const T*>(a.vG), base, qt);
  const int e0f = a.eF[t], e0g = a.eG[t];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    pt[j] = ldx(pt[j], e0f);
    qt[j] = ldx(qt[j], e0g);
    al[j] = 0.0;
    be[j] = 0.0;
  }
  if constexpr (sizeof(T) == 8) {
    res_load<T, R>(reinterpret_cast<const T*>(a.mu), base, mu);
    res_load<T, R>(reinterpret_cast<const T*>(a.nu), base, nu);
  } else {
    res_load<T, R>(reinterpret_cast<const T*>(a.mu32), base, mu);
    res_load<T, R>(reinterpret_cast<const T*>(a.nu32), base, nu);
  }
  Ctrl* ctrl = a.ctrl;
  double* hist = a.err_hist;
  int nabs = 0;
  const ResidentEnd end = resident_iterate_tau<T, R, NT>(
      pt, al, qt, be, mu, nu, a.nu + base, k, a.tol, tau, eps, a.itr_max, a.check_every, S,
      [&](int l, double err) {
        ctrl->last_err = err;
        ctrl->last_check = l;
        if (hist) hist[l] = err;
      },
      &nabs);
  // final state in the log domain's layout: each run's values e^{pot/eps} v
  // with one shared exponent
  T x[R];
  const int ef = tau_pack<T, R>(pt, al, 1.0 / eps, x);
  res_store<T, R>(static_cast<T*>(a.vF), base, x);
  a.eF[t] = ef;
  const int eg = tau_pack<T, R>(qt, be, 1.0 / eps, x);
  res_store<T, R>(static_cast<T*>(a.vG), base, x);
  a.eG[t] = eg;
  if (t == 0) {
    ctrl->iters_done = (end.stop_iter >= 0) ? end.stop_iter : end.l;
    ctrl->absorptions = nabs;
    if (end.stop_iter >= 0) {
      ctrl->done = 1;
      ctrl->stop_iter = end.stop_iter;
    }
    if (end.fail_iter >= 0) {
      ctrl->done = 1;
      ctrl->fail = 1;
      ctrl->fail_iter = end.fail_iter;
    }
  }
}

// run lengths the threshold variant is built for (binary64 runs of 16 are
// chosen only for the log and plain domains)
template <typename T, int R>
constexpr bool kTauRuns = !(sizeof(T) == 8 && R == 16);

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
  const int nt = solve_resident_threads(b.n, R);
  const bool tau_mode = b.tau > 0.0;
  const double eps = 1.0 / b.inv_eps;
  if (nt == kWave) {
    if constexpr (kTauRuns<T, R>) {
      if (tau_mode && ABSORB) {
        k_resident_tau<T, R, kWave><<<1, kWave, 0, s>>>(a, k, b.tau, eps);
        return hipGetLastError();
      }
    }
    if (tau_mode) return hipErrorInvalidValue;
    k_resident<T, R, ABSORB, kWave><<<1, kWave, 0, s>>>(a, k);
  } else if (nt == 256) {
    if constexpr (kTauRuns<T, R>) {
      if (tau_mode && ABSORB) {
        k_resident_tau<T, R, 256><<<1, 256, 0, s>>>(a, k, b.tau, eps);
        return hipGetLastError();
      }
    }
    if (tau_mode) return hipErrorInvalidValue;
    k_resident<T, R, ABSORB, 256><<<1, 256, 0, s>>>(a, k);
  } else if (nt == 512) {
    // runs of 16 in the log or plain domain only
    if constexpr (R == 16) {
      if (tau_mode) return hipErrorInvalidValue;
      k_resident<T, R, ABSORB, 512><<<1, 512, 0, s>>>(a, k);
    } else {
      return hipErrorInvalidValue;
    }
  } else if constexpr (R <= 8) {
    if (nt != 1024) return hipErrorInvalidValue;
    if (tau_mode && ABSORB)
      k_resident_tau<T, R, 1024><<<1, 1024, 0, s>>>(a, k, b.tau, eps);
    else
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
      case 16: return resident_t<T, 16, ABSORB>(b, k, itr_max, check_every, tol, s);
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

int solve_resident_threads(int64_t n, int R) {
  // a grid of at most 64 runs is one wavefront: its scans and reductions never
  // leave the wave's registers
  if (n <= int64_t(kWave) * R) return kWave;
  if (n <= int64_t(256) * R) return 256;
  // runs of 16 (chosen up to 8192 entries): 512 threads
  if (R == 16 && n <= int64_t(512) * R) return 512;
  return resident_threads(n, R);
}

int resident_run_length(int64_t n, int rmax) {
  if (n <= int64_t(256) * rmax) return rmax;
  const int r = rmax < 8 ? rmax : 8;
  return n <= int64_t(1024) * r ? r : 0;
}

bool usable_resident(const SolveBufs& b) {
  const bool r_ok = b.dtype == 0 ? (b.R == 16 || b.R == 8 || b.R == 1)
                                 : (b.R == 16 || b.R == 8 || b.R == 4 || b.R == 1);
  const int nt = solve_resident_threads(b.n, b.R);
  // the allocation is whole chunks (at least one): nt threads x R entries
  // rounded up to a chunk
  return r_ok && nt > 0 && b.npad == int64_t(std::max(nt, kBlock)) * b.R;
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
