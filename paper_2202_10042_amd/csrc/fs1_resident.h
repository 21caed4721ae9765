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

// ---------------------------------------------------------------------------
// The threshold form of the stabilisation (Sec. 2 and Sec. 3 remarks): the
// scalings are phi = e^{alpha/eps} phit and psi = e^{beta/eps} psit with
// binary64 potentials and scaled vectors in T; whenever the largest scaled
// entry exceeds tau both vectors are absorbed (alpha += eps ln phit, phit = 1;
// zero entries stay zero).  A product with the rescaled kernel
// diag(e^{alpha/eps}) K diag(e^{beta/eps}) is the product of K with
// e^{pot/eps} v, which each run packs into its shared exponent; the run
// recursions then cover the coefficients lambda e^{(beta_{i+1}-beta_i)/eps} of
// the remark exactly.
// ---------------------------------------------------------------------------

// x_j 2^E = v_j e^{pot_j / eps} over this thread's run (E shared by the run;
// 0 for a run of zeros)
template <typename T, int R>
__device__ __forceinline__ int tau_pack(const T (&v)[R], const double (&pot)[R], double inv_eps,
                                        T (&x)[R]) {
  double m[R];
  int k[R];
  int E = kExpZero;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const double t = pot[j] * inv_eps * kLog2E;
    const double fl = floor(t);
    k[j] = int(fl);
    m[j] = double(v[j]) * exp2(t - fl);
    if (v[j] > T(0)) E = max(E, k[j]);
  }
  if (E == kExpZero) E = 0;
#pragma unroll
  for (int j = 0; j < R; ++j) x[j] = (v[j] > T(0)) ? T(ldexp(m[j], k[j] - E)) : T(0);
  return E;
}

// 2^(u) * a for a binary64 a and a real exponent u (u may exceed the range of
// 2^u in binary64 while the product does not)
__device__ __forceinline__ double scale2(double a, double u) {
  const double fl = floor(u);
  return ldexp(a * exp2(u - fl), int(fl));
}

template <int NW>
__device__ __forceinline__ double block_max(double v, double* sh) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d));
  if constexpr (NW == 1) return v;  // one wavefront: every lane holds the maximum
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) r = fmax(r, sh[i]);
  __syncthreads();
  return r;  // in every thread
}

template <typename T, int R>
__device__ __forceinline__ void tau_absorb(T (&v)[R], double (&pot)[R], double eps) {
#pragma unroll
  for (int j = 0; j < R; ++j)
    if (v[j] > T(0)) {
      pot[j] += eps * log(double(v[j]));
      v[j] = T(1);
    }
}

// v_j = marg_j / (e^{pot_j/eps} y_j 2^eref), formed in binary64
template <typename T, int R>
__device__ __forceinline__ void tau_update(const T (&mg)[R], const T (&y)[R], int eref,
                                           const double (&pot)[R], double inv_eps, T (&v)[R],
                                           bool& bad) {
#pragma unroll
  for (int j = 0; j < R; ++j) {
    if (mg[j] == T(0)) {
      v[j] = T(0);
      continue;
    }
    const double q = scale2(double(mg[j]) / double(y[j]), -(double(eref) + pot[j] * inv_eps * kLog2E));
    v[j] = T(q);
    bad |= !isfinite(v[j]);
  }
}

// Algorithm 1 with the threshold stabilisation, from (pt, al), (qt, be);
// the absorption test runs at the top of every iteration.  On return the
// state is the one Algorithm 1 returns; *nabs counts the absorptions.
template <typename T, int R, int NT, typename OnCheck>
__device__ __forceinline__ ResidentEnd resident_iterate_tau(
    T (&pt)[R], double (&al)[R], T (&qt)[R], double (&be)[R], const T (&mu)[R], const T (&nu)[R],
    const double* nu64, const ScanConsts& k, double tol, double tau, double eps, int itr_max,
    int check_every, ResidentLds<T, NT / kWave>& S, OnCheck on_check, int* nabs) {
  constexpr int NW = NT / kWave;
  const double inv_eps = 1.0 / eps;
  const Lam<T> L = lam_of<T>(k);
  Dec<T> dec[7];
  lane_decays<T>(k, dec);
  const Dec<T> step = step_decay<T>(k);
  ResidentEnd end{0, -1, -1};
  T x[R], y[R];
  int l = 0, na = 0;
  for (; l < itr_max; ++l) {
    double mx = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) mx = fmax(mx, fmax(fabs(double(pt[j])), fabs(double(qt[j]))));
    if (block_max<NW>(mx, S.red) > tau) {
      tau_absorb<T, R>(pt, al, eps);
      tau_absorb<T, R>(qt, be, eps);
      ++na;
    }
    // psi-half: Kt^T phit = e^{beta/eps} K (e^{alpha/eps} phit)
    int E = tau_pack<T, R>(pt, al, inv_eps, x);
    int eref = res_apply<T, R, true, NW>(x, E, L, dec, step, S.sh, y);
    if ((l % check_every) == 0) {
      double nv[R];
      if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int j = 0; j < R; ++j) nv[j] = double(nu[j]);
      } else {
        res_load<double, R>(nu64, 0, nv);
      }
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < R; ++j)
        s += fabs(scale2(double(qt[j]) * double(y[j]), double(eref) + be[j] * inv_eps * kLog2E) -
                  nv[j]);
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
    tau_update<T, R>(nu, y, eref, be, inv_eps, qt, bad);
    // phi-half: Kt psit = e^{alpha/eps} K (e^{beta/eps} psit)
    E = tau_pack<T, R>(qt, be, inv_eps, x);
    eref = res_apply<T, R, true, NW>(x, E, L, dec, step, S.sh, y);
    tau_update<T, R>(mu, y, eref, al, inv_eps, pt, bad);
    if (__syncthreads_or(bad ? 1 : 0)) {
      end.fail_iter = l;
      break;
    }
  }
  end.l = l;
  *nabs = na;
  return end;
}

}  // namespace fs1
