// fs1_resident.h -- the FS-1 iteration (Algorithm 1) run by one workgroup
// on a grid it holds entirely in registers (device helpers shared by the
// single-pair resident solver and the batched one).
//
// Thread t owns entries [t R, t R + R).  An iteration is two workgroup-wide
// evaluations of the recursions of Sec. 3, eq. (recursion) (wavefront scans
// and one LDS exchange each, no chunk carries), the Sinkhorn update of Sec. 2
// (psi = nu / K^T phi, then phi = mu / K psi) and, on checked iterations, the
// stopping error of Algorithm 1.  The arithmetic is the general path's:
// per-run exponents renormalised every half in the log domain (ABSORB),
// plain floating point otherwise.
#pragma once

#include "fs1_device.h"
#include "fs1_internal.h"

namespace fs1 {

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

// How the iteration ended: l = completed iterations, stop_iter = l with
// err(l) <= tol (-1 if none), fail_iter = iteration whose update produced a
// non-finite scaling (-1 if none).
struct ResidentEnd {
  int l;
  int stop_iter;
  int fail_iter;
};

template <typename T, int NW>
struct ResidentLds {
  ScanLds<S1<T>, NW> sh;
  double red[NW];
  int stop;
};

// Algorithm 1 from the state (ph, eph), (ps, eps): while l < itr_max and
// err(l) > tol.  On return (ph, ps) is the final state: (phi^l, psi^l) at a
// stop, (phi^itr_max, psi^itr_max) at the cap.  nu64 points at this thread's
// binary64 nu (read on checked iterations when T = float); on_check(l, err)
// runs in thread 0 after every evaluated error.
template <typename T, int R, bool ABSORB, int NT, typename OnCheck>
__device__ __forceinline__ ResidentEnd resident_iterate(T (&ph)[R], int& eph, T (&ps)[R],
                                                        int& eps, const T (&mu)[R],
                                                        const T (&nu)[R], const double* nu64,
                                                        const ScanConsts& k, double tol,
                                                        int itr_max, int check_every,
                                                        ResidentLds<T, NT / kWave>& S,
                                                        OnCheck on_check) {
  constexpr int NW = NT / kWave;
  const Lam<T> L = lam_of<T>(k);
  Dec<T> dec[7];
  lane_decays<T>(k, dec);
  const Dec<T> step = step_decay<T>(k);
  ResidentEnd end{0, -1, -1};
  T y[R];
  int l = 0;
  for (; l < itr_max; ++l) {
    // psi-half: K^T phi^l (K is symmetric)
    int eref = res_apply<T, R, ABSORB, NW>(ph, eph, L, dec, step, S.sh, y);
    if ((l % check_every) == 0) {
      // stopping test of Algorithm 1 on (phi^l, psi^l), binary64
      double nv[R];
      if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int j = 0; j < R; ++j) nv[j] = double(nu[j]);
      } else {
        res_load<double, R>(nu64, 0, nv);
      }
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < R; ++j) s += fabs(ldexp(double(ps[j]) * double(y[j]), eps + eref) - nv[j]);
      const double tot = block_sum<NW>(s, S.red);
      if (threadIdx.x == 0) {
        on_check(l, tot);
        S.stop = !(tot > tol);
      }
      __syncthreads();
      if (S.stop) {
        end.stop_iter = l;
        break;
      }
    }
    bool bad = false;
    eps = res_update<T, R, ABSORB>(nu, y, eref, ps, bad);
    // phi-half: K psi^{l+1}
    eref = res_apply<T, R, ABSORB, NW>(ps, eps, L, dec, step, S.sh, y);
    eph = res_update<T, R, ABSORB>(mu, y, eref, ph, bad);
    // a non-finite scaling in either half ends the solve (abnormal termination)
    if (__syncthreads_or(bad ? 1 : 0)) {
      end.fail_iter = l;
      break;
    }
  }
  end.l = l;
  return end;
}

}  // namespace fs1
