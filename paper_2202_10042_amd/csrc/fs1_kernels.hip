// fs1_kernels.hip -- HIP kernels of the FS-1 hot path for gfx950.
//
// Kernel map (one "chunk" = one 256-thread block of R-element runs):
//   k_agg        chunk aggregates of a vector (forward / backward recursion
//                states, Sec. 3 eq. (recursion)), from plain, scaled or log
//                values
//   k_carry      single-block scan of the chunk aggregates -> chunk carries;
//                in a solve it also closes the stopping test of Algorithm 1
//   k_kv_apply   K x (plain) or ln K e^x (log-sum-exp semiring)
//   k_half       one half of the Sinkhorn update (Sec. 2: psi = nu / K^T phi,
//                then phi = mu / K psi), fused with the marginal error of
//                Algorithm 1's stopping test and with the chunk aggregates the
//                next half needs
//   k_cost_*     the returned double sum of Algorithm 1,
//                sum_{i,j} phi_i psi_j lambda^{|i-j|} |i-j| h, by a two-state
//                recursion (distance-weighted lower / upper parts) and a
//                binary64 reduction
//   k_setup, k_init, k_sum, k_potentials: validation, initial state
//                (phi = psi = 1/n), reductions, ln phi / ln psi.
#include <algorithm>
#include <climits>
#include <cmath>

#include "fs1.h"
#include "fs1_device.h"
#include "fs1_internal.h"
#include "fs1_tau.h"
#include "fs1_tile.h"

namespace fs1 {

// ===========================================================================
// Host helpers
// ===========================================================================
Decay make_decay(double D, double c) {
  // lambda^D = 2^-t, t = D c log2(e) >= 0:  2^(k - t) * 2^-k with k = ceil(t).
  // t is formed as an unevaluated sum t_hi + t_lo (the product D c is exact as
  // hi + lo for integer D, log2(e) is split into two doubles), so lambda^D keeps
  // full relative precision however large D c gets.
  constexpr double kL2eHi = 1.4426950408889634;     // log2(e) rounded
  constexpr double kL2eLo = 2.0355273740931033e-17;  // log2(e) - kL2eHi
  const double p_hi = D * c;
  const double p_lo = std::fma(D, c, -p_hi);
  const double t_hi = p_hi * kL2eHi;
  const double t_lo = std::fma(p_hi, kL2eHi, -t_hi) + (p_hi * kL2eLo + p_lo * kL2eHi);
  double k = std::ceil(t_hi);
  double f = (k - t_hi) - t_lo;  // k - t_hi is exact
  if (f < 0.0) {
    k += 1.0;
    f += 1.0;
  } else if (f >= 1.0) {
    k -= 1.0;
    f -= 1.0;
  }
  Decay d;
  d.m = std::exp2(f);
  d.e = -int(k);
  d.pad = 0;
  return d;
}

ScanConsts make_scan_consts(double h, double eps, int R) {
  ScanConsts k{};
  const double c = h / eps;
  k.lam = std::exp(-c);
  k.mu = -std::expm1(-c);
  k.use_mu = k.lam > 0.5 ? 1 : 0;
  k.c = c;
  k.c_log2e = c * kLog2E;
  k.R = R;
  for (int s = 0; s < 7; ++s) k.lane[s] = make_decay(double(R) * double(1 << s), c);
  k.chunk = make_decay(double(kBlock) * double(R), c);
  k.step1 = make_decay(1.0, c);
  return k;
}

CarryConsts make_carry_consts(double h, double eps, int64_t chunk_len, int64_t nchunks) {
  CarryConsts kc{};
  kc.nchunks = nchunks;
  kc.group = (nchunks + kCarryBlock - 1) / kCarryBlock;
  kc.chunk_len = chunk_len;
  kc.chunk = make_decay(double(chunk_len), h / eps);
  for (int s = 0; s < 7; ++s)
    kc.step[s] = make_decay(double(kc.group) * double(chunk_len) * double(1 << s), h / eps);
  for (int s = 0; s < 11; ++s) kc.cpow[s] = make_decay(double(chunk_len) * double(1 << s), h / eps);
  for (int s = 0; s < 7; ++s)
    kc.gstep[s] = make_decay(double(kCarryBlock) * double(chunk_len) * double(1 << s), h / eps);
  const int64_t ng = (nchunks + kCarryBlock - 1) / kCarryBlock;
  kc.two_level = (nchunks > kCarryBlock && ng <= kCarryBlock) ? 1 : 0;
  return kc;
}

CarryFix carry_fix_of(const CarryConsts& kc) {
  CarryFix f{};
  f.nchunks = kc.nchunks;
  f.two_level = kc.two_level;
  for (int s = 0; s < 11; ++s) f.cpow[s] = kc.cpow[s];
  return f;
}

namespace {
int64_t carry_groups(int64_t nchunks) { return (nchunks + kCarryBlock - 1) / kCarryBlock; }
}  // namespace

size_t carry_buffer_bytes(int64_t nchunks) {
  const int64_t g = carry_groups(nchunks);
  return size_t(nchunks + 2 * g) * sizeof(ChunkAgg) + size_t(g) * sizeof(double);
}

int pick_run_length(int dtype, bool absorb, double c) {
  // In scaled (log-domain) arithmetic every output of a run is within
  // lambda^(R-1) of the largest contribution to the run, so (R-1) h/eps must
  // stay well inside the exponent range of the working precision.
  if (dtype == 0) return (!absorb || 7.0 * c <= 600.0) ? 8 : 1;
  if (!absorb || 15.0 * c <= 60.0) return 16;
  if (7.0 * c <= 60.0) return 8;
  if (3.0 * c <= 60.0) return 4;
  return 1;
}

// ===========================================================================
// k_agg: chunk aggregates of a vector
// ===========================================================================
// IN_LOG with `special` set: special[0] |= 1 if an input is +inf, special[1]
// |= 1 if one is NaN (both zero before the launch).
template <typename T, int R, int IN>
__global__ __launch_bounds__(kBlock) void k_agg(const T* __restrict__ v, const int* __restrict__ ex,
                                                int64_t n, ScanConsts k,
                                                ChunkAgg* __restrict__ agg,
                                                int* __restrict__ special = nullptr) {
  __shared__ ScanLds<S1<T>, kBlock / kWave> sh;
  const int64_t run = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  T x[R];
  int E;
  load_input<T, R, IN>(v, ex, run, n, x, E);
  if constexpr (IN == IN_LOG) {
    // a finite logarithm maps to a value of at most 2 in its run's frame, so
    // only +inf and NaN inputs give +inf or NaN here
    bool pinf = false, nan = false;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      pinf |= isinf(x[j]) && x[j] > T(0);
      nan |= isnan(x[j]);
    }
    if (special && pinf) atomicOr(&special[0], 1);
    if (special && nan) atomicOr(&special[1], 1);
  }
  const Lam<T> L = lam_of<T>(k);
  T af, ab;
  run_aggs<T, R>(x, L, af, ab);
  Dec<T> dec[7];
  lane_decays<T>(k, dec);
  S1<T> gf, gb;
  block_scan<S1<T>, kBlock / kWave, T>(S1<T>{{af, E}}, S1<T>{{ab, E}}, dec, S1<T>::zero(),
                                       S1<T>::zero(), nullptr, nullptr, &gf, &gb, sh);
  if (threadIdx.x == 0) {
    agg[blockIdx.x].f = to64(gf.v);
    agg[blockIdx.x].b = to64(gb.v);
  }
}

// ===========================================================================
// k_carry: single-block scan of chunk aggregates -> chunk carries
//   MODE 0: plain.  MODE 1: psi-half of a solve (skip when stopped).
//   MODE 2: phi-half of a solve: close the stopping test of iteration l.
// ===========================================================================
template <int MODE>
__global__ __launch_bounds__(kCarryBlock) void k_carry(const ChunkAgg* __restrict__ agg,
                                                       ChunkAgg* __restrict__ carry,
                                                       CarryConsts kc, Ctrl* ctrl,
                                                       const double* __restrict__ part,
                                                       double* err_hist, int l, int check,
                                                       double tol) {
  constexpr int NW = kCarryBlock / kWave;
  __shared__ ScanLds<S1<double>, NW> sh;
  __shared__ double red[NW];
  __shared__ int stop;
  const int t = threadIdx.x;
  const int64_t g0 = int64_t(t) * kc.group;
  const int64_t g1 = (g0 + kc.group < kc.nchunks) ? g0 + kc.group : kc.nchunks;

  if constexpr (MODE != 0) {
    if (ctrl->done) return;
    if (ctrl->fail) {
      if (t == 0) ctrl->done = 1;
      return;
    }
  }
  if constexpr (MODE == 2) {
    if (check) {
      double s = 0.0;
      for (int64_t c = g0; c < g1; ++c) s += part[c];
      const double tot = block_sum<NW>(s, red);
      if (t == 0) {
        ctrl->last_err = tot;
        ctrl->last_check = l;
        if (err_hist) err_hist[l] = tot;
        stop = !(tot > tol);
        if (stop) {
          ctrl->done = 1;
          ctrl->stop_iter = l;
        }
      }
      __syncthreads();
      if (stop) return;
    }
  }

  const Dec<double> cdec = dec_of<double>(kc.chunk, double(kc.chunk_len));
  S1<double> gf = S1<double>::zero(), gb = S1<double>::zero();
  for (int64_t c = g0; c < g1; ++c)
    gf = gf.shift(cdec).add(S1<double>{{agg[c].f.m, agg[c].f.e}}).norm();
  for (int64_t c = g1 - 1; c >= g0; --c)
    gb = gb.shift(cdec).add(S1<double>{{agg[c].b.m, agg[c].b.e}}).norm();
  // Every group spans `group` chunks in the block scan.  Only the last
  // non-empty group can be cut short by nchunks; its forward aggregate feeds
  // only later groups, which are empty, and its backward aggregate (state at
  // the group start) is unaffected by the empty tail.
  Dec<double> dec[7];
#pragma unroll
  for (int s = 0; s < 7; ++s)
    dec[s] = dec_of<double>(kc.step[s], double(kc.group) * double(kc.chunk_len) * double(1 << s));
  S1<double> cf, cb;
  block_scan<S1<double>, NW, double>(gf, gb, dec, S1<double>::zero(), S1<double>::zero(), &cf,
                                     &cb, nullptr, nullptr, sh);
  S1<double> run = cf;
  for (int64_t c = g0; c < g1; ++c) {
    carry[c].f = to64(run.v);
    run = run.shift(cdec).add(S1<double>{{agg[c].f.m, agg[c].f.e}}).norm();
  }
  run = cb;
  for (int64_t c = g1 - 1; c >= g0; --c) {
    carry[c].b = to64(run.v);
    run = run.shift(cdec).add(S1<double>{{agg[c].b.m, agg[c].b.e}}).norm();
  }
}

// ---------------------------------------------------------------------------
// Two-level carries for more than 1024 chunks: every group of 1024 chunks is
// scanned by its own workgroup (one chunk per thread, so the work is log-deep
// instead of the single-block scan's serial walk over `group` chunks per
// thread), then one workgroup scans the group aggregates; each chunk kernel
// adds its group's carry moved to it when it loads its own (chunk_carry).
// Same semantics and modes as k_carry.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(kCarryBlock) void k_carry_groups(
    const ChunkAgg* __restrict__ agg, ChunkAgg* __restrict__ carry, ChunkAgg* __restrict__ gagg,
    double* __restrict__ gpart, CarryConsts kc, const Ctrl* ctrl,
    const double* __restrict__ part, int check) {
  constexpr int NW = kCarryBlock / kWave;
  __shared__ ScanLds<S1<double>, NW> sh;
  __shared__ double red[NW];
  if constexpr (MODE != 0) {
    if (ctrl->done || ctrl->fail) return;
  }
  const int64_t c = int64_t(blockIdx.x) * kCarryBlock + threadIdx.x;
  const bool in = c < kc.nchunks;
  if constexpr (MODE == 2) {
    if (check) {
      const double tot = block_sum<NW>(in ? part[c] : 0.0, red);
      if (threadIdx.x == 0) gpart[blockIdx.x] = tot;
    }
  }
  S1<double> f = S1<double>::zero(), b = S1<double>::zero();
  if (in) {
    f = S1<double>{{agg[c].f.m, agg[c].f.e}};
    b = S1<double>{{agg[c].b.m, agg[c].b.e}};
  }
  Dec<double> dec[7];
#pragma unroll
  for (int s = 0; s < 7; ++s) dec[s] = dec_of<double>(kc.cpow[s], double(kc.chunk_len) * double(1 << s));
  // (the last group's zero tail only moves its forward aggregate, which feeds
  // no later group)
  S1<double> cf, cb, af, ab;
  block_scan<S1<double>, NW, double>(f, b, dec, S1<double>::zero(), S1<double>::zero(), &cf, &cb,
                                     &af, &ab, sh);
  if (in) {
    carry[c].f = to64(cf.v);
    carry[c].b = to64(cb.v);
  }
  if (threadIdx.x == 0) {
    gagg[blockIdx.x].f = to64(af.v);
    gagg[blockIdx.x].b = to64(ab.v);
  }
}

template <int MODE>
__global__ __launch_bounds__(kCarryBlock) void k_carry_top(const ChunkAgg* __restrict__ gagg,
                                                           ChunkAgg* __restrict__ gcarry,
                                                           int ngroups, CarryConsts kc, Ctrl* ctrl,
                                                           const double* __restrict__ gpart,
                                                           double* err_hist, int l, int check,
                                                           double tol) {
  constexpr int NW = kCarryBlock / kWave;
  __shared__ ScanLds<S1<double>, NW> sh;
  __shared__ double red[NW];
  __shared__ int stop;
  const int t = threadIdx.x;
  if constexpr (MODE != 0) {
    if (ctrl->done) return;
    if (ctrl->fail) {
      if (t == 0) ctrl->done = 1;
      return;
    }
  }
  if constexpr (MODE == 2) {
    if (check) {
      const double tot = block_sum<NW>(t < ngroups ? gpart[t] : 0.0, red);
      if (t == 0) {
        ctrl->last_err = tot;
        ctrl->last_check = l;
        if (err_hist) err_hist[l] = tot;
        stop = !(tot > tol);
        if (stop) {
          ctrl->done = 1;
          ctrl->stop_iter = l;
        }
      }
      __syncthreads();
      if (stop) return;
    }
  }
  S1<double> f = S1<double>::zero(), b = S1<double>::zero();
  if (t < ngroups) {
    f = S1<double>{{gagg[t].f.m, gagg[t].f.e}};
    b = S1<double>{{gagg[t].b.m, gagg[t].b.e}};
  }
  Dec<double> dec[7];
#pragma unroll
  for (int s = 0; s < 7; ++s)
    dec[s] = dec_of<double>(kc.gstep[s], double(kCarryBlock) * double(kc.chunk_len) * double(1 << s));
  S1<double> cf, cb;
  block_scan<S1<double>, NW, double>(f, b, dec, S1<double>::zero(), S1<double>::zero(), &cf, &cb,
                                     nullptr, nullptr, sh);
  if (t < ngroups) {
    gcarry[t].f = to64(cf.v);
    gcarry[t].b = to64(cb.v);
  }
}

// Chunk carries from chunk aggregates (single-block scan up to 1024 chunks,
// two-level scan beyond).  `carry` holds carry_buffer_bytes(nchunks).
template <int MODE>
hipError_t launch_carry(const ChunkAgg* agg, ChunkAgg* carry, const CarryConsts& kc, Ctrl* ctrl,
                        const double* part, double* err_hist, int l, int check, double tol,
                        hipStream_t s) {
  if (!kc.two_level) {
    k_carry<MODE><<<1, kCarryBlock, 0, s>>>(agg, carry, kc, ctrl, part, err_hist, l, check, tol);
    return hipGetLastError();
  }
  const int64_t ng = carry_groups(kc.nchunks);
  ChunkAgg* gagg = carry + kc.nchunks;
  ChunkAgg* gcar = gagg + ng;
  double* gpart = reinterpret_cast<double*>(gcar + ng);
  k_carry_groups<MODE><<<unsigned(ng), kCarryBlock, 0, s>>>(agg, carry, gagg, gpart, kc, ctrl, part,
                                                           check);
  k_carry_top<MODE><<<1, kCarryBlock, 0, s>>>(gagg, gcar, int(ng), kc, ctrl, gpart, err_hist, l,
                                              check, tol);
  return hipGetLastError();
}

// The first level of the two-level carries alone (the chunk kernel folds the
// groups' aggregates and takes the stopping decision itself).
hipError_t launch_carry_groups(int mode, const ChunkAgg* agg, ChunkAgg* carry,
                               const CarryConsts& kc, Ctrl* ctrl, const double* part, int check,
                               hipStream_t s) {
  if (!kc.two_level) return hipErrorInvalidValue;
  const int64_t ng = carry_groups(kc.nchunks);
  ChunkAgg* gagg = carry + kc.nchunks;
  double* gpart = reinterpret_cast<double*>(gagg + 2 * ng);
  if (mode == 1)
    k_carry_groups<1><<<unsigned(ng), kCarryBlock, 0, s>>>(agg, carry, gagg, gpart, kc, ctrl,
                                                          part, check);
  else
    k_carry_groups<2><<<unsigned(ng), kCarryBlock, 0, s>>>(agg, carry, gagg, gpart, kc, ctrl,
                                                          part, check);
  return hipGetLastError();
}

hipError_t launch_solve_carry(int mode, const ChunkAgg* agg, ChunkAgg* carry,
                              const CarryConsts& kc, Ctrl* ctrl, const double* part,
                              double* err_hist, int l, int check, double tol, hipStream_t s) {
  if (mode == 1) return launch_carry<1>(agg, carry, kc, ctrl, part, err_hist, l, check, tol, s);
  return launch_carry<2>(agg, carry, kc, ctrl, part, err_hist, l, check, tol, s);
}

// ===========================================================================
// k_kv_apply: y = K x (plain) or ly = ln K e^lx (log)
// ===========================================================================
// LOG: `special` as set by k_agg over the same input.  Every kernel entry is
// positive, so one +inf logarithm makes every output +inf and one NaN makes
// every output NaN; those outputs are written directly.
template <typename T, int R, bool LOG>
__global__ __launch_bounds__(kBlock) void k_kv_apply(const T* __restrict__ x_in,
                                                     T* __restrict__ y_out, int64_t n,
                                                     ScanConsts k,
                                                     const ChunkAgg* __restrict__ carry,
                                                     CarryFix cfix,
                                                     const int* __restrict__ special = nullptr) {
  __shared__ ScanLds<S1<T>, kBlock / kWave> sh;
  const int64_t run = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if constexpr (LOG) {
    const int sp_nan = special[1], sp_inf = special[0];
    if (sp_nan | sp_inf) {
      T y[R];
#pragma unroll
      for (int j = 0; j < R; ++j) y[j] = sp_nan ? T(NAN) : T(INFINITY);
      store_run<T, R>(y_out, run * R, n, y);
      return;
    }
  }
  T x[R];
  int E;
  load_input<T, R, LOG ? IN_LOG : IN_PLAIN>(x_in, nullptr, run, n, x, E);
  const Lam<T> L = lam_of<T>(k);
  T af, ab;
  run_aggs<T, R>(x, L, af, ab);
  Dec<T> dec[7];
  lane_decays<T>(k, dec);
  const ChunkAgg cg = chunk_carry(carry, cfix, blockIdx.x);
  S1<T> cf, cb;
  block_scan<S1<T>, kBlock / kWave, T>(S1<T>{{af, E}}, S1<T>{{ab, E}}, dec,
                                       S1<T>{from64<T>(cg.f)}, S1<T>{from64<T>(cg.b)}, &cf, &cb,
                                       nullptr, nullptr, sh);
  // carries moved one step into the run, in extended range
  const S1<T> lcf = cf.shift(step_decay<T>(k)), lcb = cb.shift(step_decay<T>(k));
  int eref = 0;
  if constexpr (LOG) {
    eref = max(local_exponent<T, R>(x, E), max(lcf.v.e, lcb.v.e));
    if (eref == kExpZero) eref = 0;
  }
  T xf[R];
#pragma unroll
  for (int j = 0; j < R; ++j) xf[j] = ldx(x[j], E - eref);
  T y[R];
  run_apply<T, R>(xf, ldx(lcf.v.m, lcf.v.e - eref), ldx(lcb.v.m, lcb.v.e - eref), L, y);
  if constexpr (LOG) {
    // ln y = (log2 f + k + eref) ln 2 with y = f 2^k, f in [1/2, 1): only the
    // mantissa goes through the logarithm, so outputs far below the run's
    // frame keep their absolute precision
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const T yy = y[j];
      if (yy > T(0) && isfinite(yy)) {
        int ke;
        const T fm = frx(yy, &ke);
        if constexpr (sizeof(T) == 8) {
          y[j] = (log2(fm) + double(ke + eref)) * kLn2;
        } else {
          y[j] = float((double(log2f(fm)) + double(ke + eref)) * kLn2);
        }
      } else {
        y[j] = T(log2(double(yy)));  // -inf, +inf or NaN
      }
    }
  }
  store_run<T, R>(y_out, run * R, n, y);
}

// ===========================================================================
// k_half: one half of the Sinkhorn update (Sec. 2), fused with the error of
// Algorithm 1's stopping test and with the aggregates of the new vector.
//   MODE_PSI: psi^{l+1} = nu / (K^T phi^l); when `check`, also
//             err(l) = sum |psi^l (K^T phi^l) - nu| (per-chunk partials)
//   MODE_PHI: phi^{l+1} = mu / (K psi^{l+1})
//   MODE_ERR: only sum |own * (K in) - marg| (finalisation)
// State layout: value_j = v_j * 2^(ex[run of j]); with ABSORB = false the run
// exponents are identically 0 and the iteration is Algorithm 1 in plain
// floating point.
// ===========================================================================
enum HalfMode { MODE_PSI = 0, MODE_PHI = 1, MODE_ERR = 2 };

template <typename T>
struct HalfArgs {
  const T* vin;        // vector fed to K
  const int* ein;
  const double* m64;   // marginal, binary64 (error; update when T = double)
  const float* m32;    // marginal, binary32 copy (update when T = float)
  T* vout;             // updated vector
  int* eout;
  const T* vown;       // own vector for the error term
  const int* eown;
  const ChunkAgg* carry;
  ChunkAgg* agg_out;
  double* part;
  Ctrl* ctrl;
  int64_t n;
  int l;
  int check;
  CarryFix cfix;
};

// Solve vectors are allocated to whole chunks and hold zeros past n: runs are
// read and written as whole 16-byte vectors where the run length allows.
template <typename T, int R>
__device__ __forceinline__ void solve_load(const T* p, int64_t base, int64_t n, T (&x)[R]) {
  if constexpr (R % Vec16<T>::n == 0) {
    load_run_z<T, R>(p, base, x);
  } else {
    load_run<T, R>(p, base, n, x, T(0));
  }
}
template <typename T, int R>
__device__ __forceinline__ void solve_store(T* p, int64_t base, int64_t n, const T (&x)[R]) {
  if constexpr (R % Vec16<T>::n == 0) {
    store_run_z<T, R>(p, base, x);
  } else {
    store_run<T, R>(p, base, n, x);
  }
}

// TILE: the solve vectors and marginal copies are in the tile layout of
// fs1_tile.h (the iterations of the general path); otherwise in runs (the
// finalisation, and run lengths that are not whole 16-byte vectors).
template <typename T, int R, bool TILE, bool ABSORB, int MODE>
__device__ __forceinline__ void half_load(const T* p, int64_t run, int64_t n, T (&x)[R]) {
  if constexpr (TILE) {
    tile_load<T, R>(p, run, int(threadIdx.x & (kWave - 1)), x);
  } else {
    solve_load<T, R>(p, run * R, n, x);
  }
}

template <typename T, int R, bool ABSORB, int MODE, bool TILE = false>
__global__ __launch_bounds__(kBlock) void k_half(HalfArgs<T> a, ScanConsts k) {
  __shared__ ScanLds<S1<T>, kBlock / kWave> sh;
  __shared__ double red[kBlock / kWave];
  const int64_t run = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t base = run * R;
  const int64_t n = a.n;
  const bool want_err = (MODE == MODE_ERR) || (MODE == MODE_PSI && a.check);
  // every global load is issued before any of them is waited for
  int done = 0;
  if constexpr (MODE != MODE_ERR) done = a.ctrl->done;
  T x[R];
  half_load<T, R, TILE, ABSORB, MODE>(a.vin, run, n, x);
  const int E = ABSORB ? a.ein[run] : 0;
  T own[R];
  int eo = 0;
  if (want_err) {
    half_load<T, R, TILE, ABSORB, MODE>(a.vown, run, n, own);
    eo = ABSORB ? a.eown[run] : 0;
  }
  double m64[R];
  if (want_err || sizeof(T) == 8) half_load<double, R, TILE, ABSORB, MODE>(a.m64, run, n, m64);
  T mg[R];
  if constexpr (MODE != MODE_ERR) {
    if constexpr (sizeof(T) == 8) {
#pragma unroll
      for (int j = 0; j < R; ++j) mg[j] = T(m64[j]);
    } else {
      half_load<T, R, TILE, ABSORB, MODE>(reinterpret_cast<const T*>(a.m32), run, n, mg);
    }
  }
  const ChunkAgg cg = chunk_carry(a.carry, a.cfix, blockIdx.x);
  if (done) return;
  const Lam<T> L = lam_of<T>(k);
  T af, ab;
  run_aggs<T, R>(x, L, af, ab);
  Dec<T> dec[7];
  lane_decays<T>(k, dec);
  S1<T> cf, cb;
  block_scan<S1<T>, kBlock / kWave, T>(S1<T>{{af, E}}, S1<T>{{ab, E}}, dec,
                                       S1<T>{from64<T>(cg.f)}, S1<T>{from64<T>(cg.b)}, &cf, &cb,
                                       nullptr, nullptr, sh);
  const S1<T> lcf = cf.shift(step_decay<T>(k)), lcb = cb.shift(step_decay<T>(k));
  int eref = 0;
  if constexpr (ABSORB) {
    eref = max(local_exponent<T, R>(x, E), max(lcf.v.e, lcb.v.e));
    if (eref == kExpZero) eref = 0;
  }
  T xf[R];
#pragma unroll
  for (int j = 0; j < R; ++j) xf[j] = ldx(x[j], E - eref);
  T y[R];  // (K in)_j * 2^-eref
  run_apply<T, R>(xf, ldx(lcf.v.m, lcf.v.e - eref), ldx(lcb.v.m, lcb.v.e - eref), L, y);

  // error term sum_j | own_j (K in)_j - marg_j |, binary64 (entries past n
  // are zero and add nothing)
  if (want_err) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const double pr = ldexp(double(own[j]) * double(y[j]), eo + eref);
      s += fabs(pr - m64[j]);
    }
    const double tot = block_sum<kBlock / kWave>(s, red);
    if (threadIdx.x == 0) a.part[blockIdx.x] = tot;
  }
  if constexpr (MODE == MODE_ERR) return;

  // update: out_j = marg_j / (K in)_j  (zero marginal -> zero scaling)
  T q[R];
  bool bad = false;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    q[j] = (mg[j] == T(0)) ? T(0) : mg[j] / y[j];
    bad |= !isfinite(q[j]);
  }
  int Eo = 0;
  if constexpr (ABSORB) {
    // absorb the power-of-two part of the new run into its exponent
    T qm = T(0);
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (isfinite(q[j])) qm = fmax(qm, q[j]);
    int kq = 0;
    if (qm > T(0)) frx(qm, &kq);
#pragma unroll
    for (int j = 0; j < R; ++j) q[j] = ldx(q[j], -kq);
    Eo = kq - eref;
    a.eout[run] = Eo;
  }
  if constexpr (TILE) {
    tile_store<T, R>(a.vout, run, int(threadIdx.x & (kWave - 1)), q);
  } else {
    solve_store<T, R>(a.vout, base, n, q);
  }
  if (bad) {
    atomicOr(&a.ctrl->fail, 1);
    atomicMin(&a.ctrl->fail_iter, a.l);
  }
  // aggregates of the new vector for the next half
  T nf, nb;
  run_aggs<T, R>(q, L, nf, nb);
  S1<T> gf, gb;
  block_scan<S1<T>, kBlock / kWave, T>(S1<T>{{nf, Eo}}, S1<T>{{nb, Eo}}, dec, S1<T>::zero(),
                                       S1<T>::zero(), nullptr, nullptr, &gf, &gb, sh);
  if (threadIdx.x == 0) {
    a.agg_out[blockIdx.x].f = to64(gf.v);
    a.agg_out[blockIdx.x].b = to64(gb.v);
  }
}

// ===========================================================================
// Transport cost (two-state recursions of fs1_device.h)
// ===========================================================================
template <typename T, int R, bool ABSORB>
__global__ __launch_bounds__(kBlock) void k_cost_agg(const T* __restrict__ v,
                                                     const int* __restrict__ ex, int64_t n,
                                                     ScanConsts k, ChunkAgg2* __restrict__ agg) {
  __shared__ ScanLds<S2<T>, kBlock / kWave> sh;
  const int64_t run = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  T x[R];
  int E;
  load_input<T, R, ABSORB ? IN_SCALED : IN_PLAIN>(v, ex, run, n, x, E);
  const Lam<T> L = lam_of<T>(k);
  T fp, fd, bp, bd;
  run_aggs2<T, R>(x, L, fp, fd, bp, bd);
  Dec<T> dec[7];
  lane_decays<T>(k, dec);
  S2<T> gf, gb;
  block_scan<S2<T>, kBlock / kWave, T>(S2<T>::of(fp, fd, E), S2<T>::of(bp, bd, E), dec,
                                       S2<T>::zero(), S2<T>::zero(), nullptr, nullptr, &gf, &gb,
                                       sh);
  if (threadIdx.x == 0) {
    ChunkAgg2 o;
    s2_put_fwd(o, gf);
    s2_put_bwd(o, gb);
    agg[blockIdx.x] = o;
  }
}

__global__ __launch_bounds__(kCarryBlock) void k_cost_carry(const ChunkAgg2* __restrict__ agg,
                                                            ChunkAgg2* __restrict__ carry,
                                                            CarryConsts kc) {
  constexpr int NW = kCarryBlock / kWave;
  __shared__ ScanLds<S2<double>, NW> sh;
  const int t = threadIdx.x;
  const int64_t g0 = int64_t(t) * kc.group;
  const int64_t g1 = (g0 + kc.group < kc.nchunks) ? g0 + kc.group : kc.nchunks;
  const Dec<double> cdec = dec_of<double>(kc.chunk, double(kc.chunk_len));
  S2<double> gf = S2<double>::zero(), gb = S2<double>::zero();
  for (int64_t c = g0; c < g1; ++c)
    gf = gf.shift(cdec).add(s2_fwd<double>(agg[c])).norm();
  // (a group cut short by nchunks only feeds empty groups; see k_carry)
  for (int64_t c = g1 - 1; c >= g0; --c)
    gb = gb.shift(cdec).add(s2_bwd<double>(agg[c])).norm();
  Dec<double> dec[7];
#pragma unroll
  for (int s = 0; s < 7; ++s)
    dec[s] = dec_of<double>(kc.step[s], double(kc.group) * double(kc.chunk_len) * double(1 << s));
  S2<double> cf, cb;
  block_scan<S2<double>, NW, double>(gf, gb, dec, S2<double>::zero(), S2<double>::zero(), &cf,
                                     &cb, nullptr, nullptr, sh);
  S2<double> r = cf;
  for (int64_t c = g0; c < g1; ++c) {
    s2_put_fwd(carry[c], r);
    r = r.shift(cdec).add(s2_fwd<double>(agg[c])).norm();
  }
  r = cb;
  for (int64_t c = g1 - 1; c >= g0; --c) {
    s2_put_bwd(carry[c], r);
    r = r.shift(cdec).add(s2_bwd<double>(agg[c])).norm();
  }
}

template <typename T, int R, bool ABSORB>
__global__ __launch_bounds__(kBlock) void k_cost_apply(const T* __restrict__ vphi,
                                                       const int* __restrict__ ephi,
                                                       const T* __restrict__ vpsi,
                                                       const int* __restrict__ epsi, int64_t n,
                                                       ScanConsts k,
                                                       const ChunkAgg2* __restrict__ carry,
                                                       double* __restrict__ part) {
  __shared__ ScanLds<S2<T>, kBlock / kWave> sh;
  __shared__ double red[kBlock / kWave];
  const int64_t run = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t base = run * R;
  T x[R];
  int E;
  load_input<T, R, ABSORB ? IN_SCALED : IN_PLAIN>(vpsi, epsi, run, n, x, E);
  const Lam<T> L = lam_of<T>(k);
  T fp, fd, bp, bd;
  run_aggs2<T, R>(x, L, fp, fd, bp, bd);
  Dec<T> dec[7];
  lane_decays<T>(k, dec);
  const ChunkAgg2 cg = carry[blockIdx.x];
  S2<T> cf, cb;
  block_scan<S2<T>, kBlock / kWave, T>(S2<T>::of(fp, fd, E), S2<T>::of(bp, bd, E), dec,
                                       s2_fwd<T>(cg), s2_bwd<T>(cg), &cf, &cb, nullptr, nullptr,
                                       sh);
  // carries moved one step into the run (extended range)
  const S2<T> lcf = cf.shift(step_decay<T>(k)), lcb = cb.shift(step_decay<T>(k));
  const int eref = cost_frame<T, R>(lcf, lcb, local_exponent<T, R>(x, E), k);
  T xf[R];
#pragma unroll
  for (int j = 0; j < R; ++j) xf[j] = ldx(x[j], E - eref);
  T w[R];
  run_cost<T, R>(xf, ldx(lcf.p.m, lcf.p.e - eref), ldx(lcf.d.m, lcf.d.e - eref),
                 ldx(lcb.p.m, lcb.p.e - eref), ldx(lcb.d.m, lcb.d.e - eref), L, w);
  T ph[R];
  load_run<T, R>(vphi, base, n, ph, T(0));
  const int ep = ABSORB ? ephi[run] : 0;
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < R; ++j)
    if (base + j < n) s += ldexp(double(ph[j]) * double(w[j]), ep + eref);
  const double tot = block_sum<kBlock / kWave>(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// ===========================================================================
// Small kernels: setup, initial state, reductions, potentials
// ===========================================================================
__global__ __launch_bounds__(256) void k_setup(const double* __restrict__ mu,
                                               const double* __restrict__ nu, int64_t n,
                                               int64_t npad, double* __restrict__ mu64,
                                               double* __restrict__ nu64,
                                               float* __restrict__ mu32,
                                               float* __restrict__ nu32, Ctrl* ctrl) {
  __shared__ double red[4];
  double sm = 0.0, sn = 0.0;
  int bad = 0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < npad;
       i += int64_t(gridDim.x) * blockDim.x) {
    double a = 0.0, b = 0.0;  // zero padding past n
    if (i < n) {
      a = mu[i];
      b = nu[i];
    }
    bad |= !(isfinite(a) && a >= 0.0) || !(isfinite(b) && b >= 0.0);
    sm += a;
    sn += b;
    mu64[i] = a;
    nu64[i] = b;
    if (mu32) {
      mu32[i] = float(a);
      nu32[i] = float(b);
    }
  }
  const double tm = block_sum<4>(sm, red);
  const double tn = block_sum<4>(sn, red);
  if (bad) atomicOr(&ctrl->bad_input, 1);
  if (threadIdx.x == 0) {
    atomicAdd(&ctrl->sum_mu, tm);
    atomicAdd(&ctrl->sum_nu, tn);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_init(T* __restrict__ vf, T* __restrict__ vg, int* ef,
                                              int* eg, int64_t n, int64_t npad, int64_t nruns,
                                              Ctrl* ctrl) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const T v = T(1.0 / double(n));
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < npad; i += stride) {
    vf[i] = i < n ? v : T(0);
    vg[i] = i < n ? v : T(0);
  }
  if (ef) {
    for (int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < nruns; r += stride) {
      ef[r] = 0;
      eg[r] = 0;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->done = 0;
    ctrl->stop_iter = -1;
    ctrl->fail = 0;
    ctrl->fail_iter = INT_MAX;
    ctrl->last_check = -1;
    ctrl->last_err = NAN;
    ctrl->barrier_timeout = 0;
    ctrl->iters_done = 0;
    ctrl->fail_half[0] = 0;
    ctrl->fail_half[1] = 0;
  }
}

// Warm start: (phi, psi) from split scalings m 2^e (Algorithm 1 started from a
// given pair instead of 1/n).  One thread per run of the solve's layout.  With
// per-run exponents (ef, eg non-null) a run takes the largest exponent of its
// entries and holds the mantissas shifted to it (exact, up to entries below
// the working precision of the run); in plain arithmetic the values are
// m 2^e themselves.  Entries past n are zero.  Invalid input (m not finite or
// negative, |e| > 2^20, a plain value that overflows) sets bit 1 of
// ctrl->bad_input.
template <typename T>
__global__ __launch_bounds__(256) void k_warm(const double* __restrict__ m,
                                              const int* __restrict__ e, int64_t n, int R,
                                              int64_t nruns, T* __restrict__ vf,
                                              T* __restrict__ vg, int* ef, int* eg,
                                              Ctrl* ctrl) {
  constexpr int kMaxExp = 1 << 20;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  int bad = 0;
  for (int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < nruns; r += stride) {
    const int64_t base = r * R;
    for (int side = 0; side < 2; ++side) {
      const double* ms = m + side * n;
      const int* es = e + side * n;
      T* v = side ? vg : vf;
      int* ex = side ? eg : ef;
      int E = kExpZero;
      for (int j = 0; j < R && base + j < n; ++j) {
        const double mm = ms[base + j];
        const int ee = es[base + j];
        if (!(isfinite(mm) && mm >= 0.0) || ee > kMaxExp || ee < -kMaxExp) {
          bad = 1;
        } else if (mm > 0.0) {
          int k;
          frexp(mm, &k);
          E = max(E, ee + k);
        }
      }
      if (E == kExpZero) E = 0;
      for (int j = 0; j < R; ++j) {
        const int64_t i = base + j;
        T val = T(0);
        if (i < n) {
          const double mm = ms[i];
          const int ee = es[i];
          if (isfinite(mm) && mm > 0.0 && ee <= kMaxExp && ee >= -kMaxExp) {
            val = ex ? T(ldexp(mm, ee - E)) : T(ldexp(mm, ee));
            if (!isfinite(val)) bad = 1;
          }
        }
        v[i] = val;
      }
      if (ex) ex[r] = E;
    }
  }
  if (bad) atomicOr(&ctrl->bad_input, 2);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->done = 0;
    ctrl->stop_iter = -1;
    ctrl->fail = 0;
    ctrl->fail_iter = INT_MAX;
    ctrl->last_check = -1;
    ctrl->last_err = NAN;
    ctrl->barrier_timeout = 0;
    ctrl->iters_done = 0;
    ctrl->fail_half[0] = 0;
    ctrl->fail_half[1] = 0;
  }
}

// Final (phi or psi) in split form: m[i] = v[i], e[i] = the run exponent (0 in
// plain arithmetic); the vector in runs of R.
template <typename T>
__global__ __launch_bounds__(256) void k_state_out(const T* __restrict__ v,
                                                   const int* __restrict__ ex, int R, int64_t n,
                                                   double* __restrict__ m, int* __restrict__ e) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    m[i] = double(v[i]);
    e[i] = ex ? ex[i / R] : 0;
  }
}

// ---------------------------------------------------------------------------
// The asynchronous solve (no host synchronisation; capturable in a graph):
// control-block reset, error-history fill, the final psi moved to buffer 0,
// and the result written to device memory -- all as kernels.
// ---------------------------------------------------------------------------
__global__ void k_ctrl_reset(Ctrl* c) {
  int* p = reinterpret_cast<int*>(c);
  for (int i = threadIdx.x; i < int(sizeof(Ctrl) / sizeof(int)); i += blockDim.x) p[i] = 0;
}

__global__ __launch_bounds__(256) void k_fill_nan(double* p, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    p[i] = NAN;
}

// Iterations Algorithm 1 completed: the stopping iteration, else itr_max.
__device__ __forceinline__ int completed_iterations(const Ctrl* c, int itr_max) {
  return (c->done && c->stop_iter >= 0) ? c->stop_iter : itr_max;
}

// When the final psi is in buffer 1 (an odd number of completed iterations),
// copy it (values, run exponents, chunk exponents) to buffer 0.
__global__ __launch_bounds__(256) void k_select_psi(uint4* __restrict__ v0,
                                                    const uint4* __restrict__ v1, int64_t nv,
                                                    int* __restrict__ e0,
                                                    const int* __restrict__ e1, int64_t ne,
                                                    ChunkExp* __restrict__ x0,
                                                    const ChunkExp* __restrict__ x1, int64_t nx,
                                                    const Ctrl* ctrl, int itr_max) {
  if ((completed_iterations(ctrl, itr_max) & 1) == 0) return;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nv; i += stride)
    v0[i] = v1[i];
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < ne; i += stride)
    e0[i] = e1[i];
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nx; i += stride)
    x0[i] = x1[i];
}

// The solve's result, as fs1_solve would return it, into device memory.
__global__ void k_result(const Ctrl* c, fs1_result* out, double tol, int itr_max) {
  if (threadIdx.x != 0) return;
  fs1_result r;
  r.w1 = c->w1;
  r.marginal_err = c->err_final;
  r.mu_err = c->mu_err;
  r.iterations = completed_iterations(c, itr_max);
  r.converged = !(c->err_final > tol) ? 1 : 0;
  r.absorptions = 0;
  r.status = FS1_OK;
  const bool invalid = (c->bad_input != 0) || !(c->sum_mu > 0.0) || !(c->sum_nu > 0.0) ||
                       fabs(c->sum_mu - c->sum_nu) > 1e-10 * c->sum_mu;
  if (invalid) {
    r.status = FS1_ERR_INVALID_ARG;
    r.iterations = 0;
  } else if (c->fail) {
    r.status = FS1_ERR_NONFINITE;
    r.iterations = c->fail_iter;
  } else if (!isfinite(c->w1) || !isfinite(c->err_final)) {
    r.status = FS1_ERR_NONFINITE;
  }
  if (r.status != FS1_OK) {
    r.converged = 0;
    if (invalid) r.w1 = r.marginal_err = r.mu_err = NAN;
  }
  *out = r;
}

hipError_t launch_async_reset(const SolveBufs& b, double* err_hist, int itr_max, hipStream_t s) {
  k_ctrl_reset<<<1, 64, 0, s>>>(b.ctrl);
  if (err_hist) {
    const int64_t nh = int64_t(itr_max) + 1;
    k_fill_nan<<<unsigned(std::min<int64_t>((nh + 255) / 256, 1024)), 256, 0, s>>>(err_hist, nh);
  }
  return hipGetLastError();
}

hipError_t launch_select_psi(const SolveBufs& b, int itr_max, hipStream_t s) {
  const int64_t es = b.dtype == 0 ? 8 : 4;
  const int64_t nv = b.npad * es / 16;
  const int64_t ne = b.nchunks * kBlock;
  const unsigned g = unsigned(std::min<int64_t>((nv + 255) / 256, 8192));
  k_select_psi<<<g, 256, 0, s>>>(static_cast<uint4*>(b.vG[0]), static_cast<const uint4*>(b.vG[1]),
                                 nv, b.eG[0], b.eG[1], ne, b.xG[0], b.xG[1], b.nchunks, b.ctrl,
                                 itr_max);
  return hipGetLastError();
}

hipError_t launch_result(const SolveBufs& b, fs1_result* out, double tol, int itr_max,
                         hipStream_t s) {
  k_result<<<1, 64, 0, s>>>(b.ctrl, out, tol, itr_max);
  return hipGetLastError();
}

// out = scale * sum(part[0..np)) in a fixed order
__global__ __launch_bounds__(1024) void k_sum(const double* __restrict__ part, int64_t np,
                                              double scale, double* out) {
  __shared__ double red[16];
  const int64_t per = (np + 1023) / 1024;
  const int64_t a = int64_t(threadIdx.x) * per;
  const int64_t b = (a + per < np) ? a + per : np;
  double s = 0.0;
  for (int64_t i = a; i < b; ++i) s += part[i];
  const double t = block_sum<16>(s, red);
  if (threadIdx.x == 0) *out = t * scale;
}

template <typename T>
__global__ __launch_bounds__(256) void k_potentials(const T* __restrict__ v,
                                                    const int* __restrict__ ex, int R,
                                                    int64_t n, double* __restrict__ out) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double x = double(v[i]);
    const int e = ex ? ex[i / R] : 0;
    if (x > 0.0 && isfinite(x)) {
      int k;
      const double f = frexp(x, &k);
      out[i] = log(f) + double(k + e) * kLn2;
    } else {
      out[i] = (x == 0.0) ? -INFINITY : NAN;
    }
  }
}

// ===========================================================================
// Launchers
// ===========================================================================
static inline unsigned grid_of(int64_t nchunks) { return unsigned(nchunks); }

template <typename T, int R>
static hipError_t kv_plain_t(const void* x, void* y, int64_t n, const ScanConsts& k,
                             const CarryConsts& kc, ChunkAgg* agg, ChunkAgg* carry,
                             hipStream_t s) {
  const unsigned g = grid_of(kc.nchunks);
  k_agg<T, R, IN_PLAIN><<<g, kBlock, 0, s>>>(static_cast<const T*>(x), nullptr, n, k, agg);
  {
    const hipError_t e = launch_carry<0>(agg, carry, kc, nullptr, nullptr, nullptr, 0, 0, 0.0, s);
    if (e != hipSuccess) return e;
  }
  k_kv_apply<T, R, false><<<g, kBlock, 0, s>>>(static_cast<const T*>(x), static_cast<T*>(y), n,
                                               k, carry, carry_fix_of(kc));
  return hipGetLastError();
}

__global__ void k_zero_ints(int* p, int count) {
  if (int(threadIdx.x) < count) p[threadIdx.x] = 0;
}

template <typename T, int R>
static hipError_t kv_log_t(const void* x, void* y, int64_t n, const ScanConsts& k,
                           const CarryConsts& kc, ChunkAgg* agg, ChunkAgg* carry, int* special,
                           hipStream_t s) {
  const unsigned g = grid_of(kc.nchunks);
  // (a kernel, not a memset: the call may be captured into a graph)
  k_zero_ints<<<1, 64, 0, s>>>(special, 2);
  k_agg<T, R, IN_LOG><<<g, kBlock, 0, s>>>(static_cast<const T*>(x), nullptr, n, k, agg,
                                           special);
  {
    const hipError_t e = launch_carry<0>(agg, carry, kc, nullptr, nullptr, nullptr, 0, 0, 0.0, s);
    if (e != hipSuccess) return e;
  }
  k_kv_apply<T, R, true><<<g, kBlock, 0, s>>>(static_cast<const T*>(x), static_cast<T*>(y), n,
                                              k, carry, carry_fix_of(kc), special);
  return hipGetLastError();
}

hipError_t launch_kv_plain(int dtype, const void* x, void* y, int64_t n, const ScanConsts& k,
                           const CarryConsts& kc, ChunkAgg* agg, ChunkAgg* carry,
                           hipStream_t s) {
  if (dtype == 0) {
    if (k.R == 8) return kv_plain_t<double, 8>(x, y, n, k, kc, agg, carry, s);
    return kv_plain_t<double, 1>(x, y, n, k, kc, agg, carry, s);
  }
  switch (k.R) {
    case 16: return kv_plain_t<float, 16>(x, y, n, k, kc, agg, carry, s);
    case 8: return kv_plain_t<float, 8>(x, y, n, k, kc, agg, carry, s);
    case 4: return kv_plain_t<float, 4>(x, y, n, k, kc, agg, carry, s);
    default: return kv_plain_t<float, 1>(x, y, n, k, kc, agg, carry, s);
  }
}

hipError_t launch_kv_log(int dtype, const void* x, void* y, int64_t n, const ScanConsts& k,
                         const CarryConsts& kc, ChunkAgg* agg, ChunkAgg* carry, int* special,
                         hipStream_t s) {
  if (dtype == 0) {
    if (k.R == 8) return kv_log_t<double, 8>(x, y, n, k, kc, agg, carry, special, s);
    return kv_log_t<double, 1>(x, y, n, k, kc, agg, carry, special, s);
  }
  switch (k.R) {
    case 16: return kv_log_t<float, 16>(x, y, n, k, kc, agg, carry, special, s);
    case 8: return kv_log_t<float, 8>(x, y, n, k, kc, agg, carry, special, s);
    case 4: return kv_log_t<float, 4>(x, y, n, k, kc, agg, carry, special, s);
    default: return kv_log_t<float, 1>(x, y, n, k, kc, agg, carry, special, s);
  }
}

// ---------------------------------------------------------------------------
// Solve launchers: dispatch on (dtype, R, absorb)
// ---------------------------------------------------------------------------
template <typename T, int R, bool AB>
struct SolveOps {
  // run lengths of whole 16-byte vectors can take the tile layout (the fused
  // path always does); the general path iterates on it in binary64, where it
  // measured faster (N = 1e8: 1.257 against 1.280 ms per iteration; binary32
  // measured 0.768 against 0.745 and keeps runs)
  static constexpr bool kTileable = R % Vec16<T>::n == 0;
  static constexpr bool kTile = kTileable && sizeof(T) == 8;
  static hipError_t setup_aggF(const SolveBufs& b, const ScanConsts& k, hipStream_t s) {
    k_agg<T, R, AB ? IN_SCALED : IN_PLAIN><<<grid_of(b.nchunks), kBlock, 0, s>>>(
        static_cast<const T*>(b.vF), b.eF, b.n, k, b.aggF);
    return hipGetLastError();
  }
  static HalfArgs<T> args(const SolveBufs& b, const CarryConsts& kc, int mode, int l, int check,
                          int gbuf) {
    HalfArgs<T> a{};
    a.cfix = carry_fix_of(kc);
    a.n = b.n;
    a.l = l;
    a.check = check;
    a.ctrl = b.ctrl;
    a.carry = b.carry;
    a.part = b.part;
    if (mode == MODE_PSI) {
      const int cur = l & 1, nxt = (l + 1) & 1;
      a.vin = static_cast<const T*>(b.vF);
      a.ein = b.eF;
      a.m64 = b.nu;
      a.m32 = static_cast<const float*>(b.nu32);
      a.vout = static_cast<T*>(b.vG[nxt]);
      a.eout = b.eG[nxt];
      a.vown = static_cast<const T*>(b.vG[cur]);
      a.eown = b.eG[cur];
      a.agg_out = b.aggG;
    } else {
      const int nxt = (l + 1) & 1;
      a.vin = static_cast<const T*>(b.vG[nxt]);
      a.ein = b.eG[nxt];
      a.m64 = b.mu;
      a.m32 = static_cast<const float*>(b.mu32);
      a.vout = static_cast<T*>(b.vF);
      a.eout = b.eF;
      a.agg_out = b.aggF;
    }
    (void)gbuf;
    return a;
  }
  static hipError_t half_psi(const SolveBufs& b, const ScanConsts& k, const CarryConsts& kc,
                             int l, int check, double tol, hipStream_t s, hipEvent_t ev0,
                             hipEvent_t ev1) {
    {
      const hipError_t e =
          launch_carry<1>(b.aggF, b.carry, kc, b.ctrl, nullptr, nullptr, l, 0, tol, s);
      if (e != hipSuccess) return e;
    }
    if (ev0) (void)hipEventRecord(ev0, s);
    k_half<T, R, AB, MODE_PSI, kTile><<<grid_of(b.nchunks), kBlock, 0, s>>>(
        args(b, kc, MODE_PSI, l, check, 0), k);
    if (ev1) (void)hipEventRecord(ev1, s);
    return hipGetLastError();
  }
  static hipError_t half_phi(const SolveBufs& b, const ScanConsts& k, const CarryConsts& kc,
                             int l, int check, double tol, hipStream_t s, hipEvent_t ev0,
                             hipEvent_t ev1) {
    {
      const hipError_t e =
          launch_carry<2>(b.aggG, b.carry, kc, b.ctrl, b.part, b.err_hist, l, check, tol, s);
      if (e != hipSuccess) return e;
    }
    if (ev0) (void)hipEventRecord(ev0, s);
    k_half<T, R, AB, MODE_PHI, kTile><<<grid_of(b.nchunks), kBlock, 0, s>>>(
        args(b, kc, MODE_PHI, l, check, 0), k);
    if (ev1) (void)hipEventRecord(ev1, s);
    return hipGetLastError();
  }
  static hipError_t finalize(const SolveBufs& b, const ScanConsts& k, const CarryConsts& kc,
                             int gbuf, double h, hipStream_t s) {
    const unsigned g = grid_of(b.nchunks);
    const T* vF = static_cast<const T*>(b.vF);
    const T* vG = static_cast<const T*>(b.vG[gbuf]);
    const int* eF = b.eF;
    const int* eG = b.eG[gbuf];
    // nu side: | psi (K^T phi) - nu |
    k_agg<T, R, AB ? IN_SCALED : IN_PLAIN><<<g, kBlock, 0, s>>>(vF, eF, b.n, k, b.aggF);
    {
      const hipError_t e =
          launch_carry<0>(b.aggF, b.carry, kc, nullptr, nullptr, nullptr, 0, 0, 0.0, s);
      if (e != hipSuccess) return e;
    }
    HalfArgs<T> a{};
    a.cfix = carry_fix_of(kc);
    a.n = b.n;
    a.ctrl = b.ctrl;
    a.carry = b.carry;
    a.part = b.part;
    a.vin = vF;
    a.ein = eF;
    a.vown = vG;
    a.eown = eG;
    a.m64 = b.nu;
    k_half<T, R, AB, MODE_ERR><<<g, kBlock, 0, s>>>(a, k);
    k_sum<<<1, 1024, 0, s>>>(b.part, b.nchunks, 1.0, &b.ctrl->err_final);
    // mu side: | phi (K psi) - mu |
    k_agg<T, R, AB ? IN_SCALED : IN_PLAIN><<<g, kBlock, 0, s>>>(vG, eG, b.n, k, b.aggG);
    {
      const hipError_t e =
          launch_carry<0>(b.aggG, b.carry, kc, nullptr, nullptr, nullptr, 0, 0, 0.0, s);
      if (e != hipSuccess) return e;
    }
    a.vin = vG;
    a.ein = eG;
    a.vown = vF;
    a.eown = eF;
    a.m64 = b.mu;
    k_half<T, R, AB, MODE_ERR><<<g, kBlock, 0, s>>>(a, k);
    k_sum<<<1, 1024, 0, s>>>(b.part, b.nchunks, 1.0, &b.ctrl->mu_err);
    // transport cost
    ChunkAgg2* agg2 = static_cast<ChunkAgg2*>(b.agg2);
    ChunkAgg2* car2 = static_cast<ChunkAgg2*>(b.carry2);
    k_cost_agg<T, R, AB><<<g, kBlock, 0, s>>>(vG, eG, b.n, k, agg2);
    k_cost_carry<<<1, kCarryBlock, 0, s>>>(agg2, car2, kc);
    k_cost_apply<T, R, AB><<<g, kBlock, 0, s>>>(vF, eF, vG, eG, b.n, k, car2, b.part);
    k_sum<<<1, 1024, 0, s>>>(b.part, b.nchunks, h, &b.ctrl->w1);
    return hipGetLastError();
  }
  static hipError_t relayout(const SolveBufs& b, bool to_tiles, int gbuf, hipStream_t s) {
    if constexpr (kTileable) {
      const unsigned g = grid_of(b.nchunks);
      T* v[2] = {static_cast<T*>(b.vF), static_cast<T*>(b.vG[gbuf])};
      double* m[2] = {const_cast<double*>(b.mu), const_cast<double*>(b.nu)};
      for (int i = 0; i < 2; ++i) {
        if (to_tiles) {
          k_relayout<T, R, true><<<g, kBlock, 0, s>>>(v[i]);
          k_relayout<double, R, true><<<g, kBlock, 0, s>>>(m[i]);
        } else {
          k_relayout<T, R, false><<<g, kBlock, 0, s>>>(v[i]);
          k_relayout<double, R, false><<<g, kBlock, 0, s>>>(m[i]);
        }
      }
      if constexpr (sizeof(T) == 4) {
        float* m32[2] = {static_cast<float*>(b.mu32), static_cast<float*>(b.nu32)};
        for (int i = 0; i < 2; ++i) {
          if (to_tiles)
            k_relayout<float, R, true><<<g, kBlock, 0, s>>>(m32[i]);
          else
            k_relayout<float, R, false><<<g, kBlock, 0, s>>>(m32[i]);
        }
      }
    }
    return hipGetLastError();
  }
  static hipError_t init(const SolveBufs& b, const ScanConsts& k, bool warm, hipStream_t s) {
    if (!warm) {
      const int64_t nruns = b.nchunks * kBlock;
      const unsigned g =
          unsigned(std::min<int64_t>((std::max(b.npad, nruns) + 255) / 256, 4096));
      k_init<T><<<g, 256, 0, s>>>(static_cast<T*>(b.vF), static_cast<T*>(b.vG[0]),
                                  AB ? b.eF : nullptr, AB ? b.eG[0] : nullptr, b.n, b.npad,
                                  nruns, b.ctrl);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return setup_aggF(b, k, s);
  }
  static hipError_t warm(const SolveBufs& b, const double* m, const int* e, hipStream_t s) {
    const int64_t nruns = b.nchunks * kBlock;
    const unsigned g = unsigned(std::min<int64_t>((nruns + 255) / 256, 4096));
    k_warm<T><<<g, 256, 0, s>>>(m, e, b.n, R, nruns, static_cast<T*>(b.vF),
                                static_cast<T*>(b.vG[0]), AB ? b.eF : nullptr,
                                AB ? b.eG[0] : nullptr, b.ctrl);
    return hipGetLastError();
  }
  static hipError_t state_out(const SolveBufs& b, int gbuf, double* m, int* e, hipStream_t s) {
    const unsigned g = unsigned(std::min<int64_t>((b.n + 255) / 256, 4096));
    k_state_out<T><<<g, 256, 0, s>>>(static_cast<const T*>(b.vF), AB ? b.eF : nullptr, R, b.n,
                                      m, e);
    k_state_out<T><<<g, 256, 0, s>>>(static_cast<const T*>(b.vG[gbuf]),
                                      AB ? b.eG[gbuf] : nullptr, R, b.n, m + b.n, e + b.n);
    return hipGetLastError();
  }
  static hipError_t potentials(const SolveBufs& b, int gbuf, double* out, hipStream_t s) {
    const unsigned g = unsigned(std::min<int64_t>((b.n + 255) / 256, 4096));
    k_potentials<T><<<g, 256, 0, s>>>(static_cast<const T*>(b.vF), AB ? b.eF : nullptr, R, b.n,
                                      out);
    k_potentials<T><<<g, 256, 0, s>>>(static_cast<const T*>(b.vG[gbuf]),
                                      AB ? b.eG[gbuf] : nullptr, R, b.n, out + b.n);
    return hipGetLastError();
  }
};

// Call F with the SolveOps instantiation matching the solve's configuration.
template <typename F>
static hipError_t dispatch(const SolveBufs& b, F&& f) {
  if (b.dtype == 0) {
    if (b.R == 16)
      return b.absorb ? f(SolveOps<double, 16, true>{}) : f(SolveOps<double, 16, false>{});
    if (b.R == 8) return b.absorb ? f(SolveOps<double, 8, true>{}) : f(SolveOps<double, 8, false>{});
    if (b.R == 4) return b.absorb ? f(SolveOps<double, 4, true>{}) : f(SolveOps<double, 4, false>{});
    return b.absorb ? f(SolveOps<double, 1, true>{}) : f(SolveOps<double, 1, false>{});
  }
  switch (b.R) {
    case 16:
      return b.absorb ? f(SolveOps<float, 16, true>{}) : f(SolveOps<float, 16, false>{});
    case 8:
      return b.absorb ? f(SolveOps<float, 8, true>{}) : f(SolveOps<float, 8, false>{});
    case 4:
      return b.absorb ? f(SolveOps<float, 4, true>{}) : f(SolveOps<float, 4, false>{});
    default:
      return b.absorb ? f(SolveOps<float, 1, true>{}) : f(SolveOps<float, 1, false>{});
  }
}

hipError_t launch_setup(const SolveBufs& b, hipStream_t s) {
  const unsigned g = unsigned(std::min<int64_t>((b.npad + 255) / 256, 2048));
  k_setup<<<g, 256, 0, s>>>(b.mu_src, b.nu_src, b.n, b.npad, const_cast<double*>(b.mu),
                            const_cast<double*>(b.nu), static_cast<float*>(b.mu32),
                            static_cast<float*>(b.nu32), b.ctrl);
  return hipGetLastError();
}

bool solve_tiled(const SolveBufs& b) {
  return b.dtype == 0 && b.R % 2 == 0;
}

hipError_t launch_relayout(const SolveBufs& b, bool to_tiles, int gbuf, hipStream_t s) {
  return dispatch(b, [&](auto ops) { return decltype(ops)::relayout(b, to_tiles, gbuf, s); });
}

hipError_t launch_init_state(const SolveBufs& b, const ScanConsts& k, bool warm, hipStream_t s) {
  return dispatch(b, [&](auto ops) { return decltype(ops)::init(b, k, warm, s); });
}

hipError_t launch_warm(const SolveBufs& b, const double* m, const int* e, hipStream_t s) {
  return dispatch(b, [&](auto ops) { return decltype(ops)::warm(b, m, e, s); });
}

hipError_t launch_state_out(const SolveBufs& b, int gbuf, double* m, int* e, hipStream_t s) {
  return dispatch(b, [&](auto ops) { return decltype(ops)::state_out(b, gbuf, m, e, s); });
}

hipError_t launch_half_psi(const SolveBufs& b, const ScanConsts& k, const CarryConsts& kc, int l,
                           int check, double tol, hipStream_t s, hipEvent_t ev0,
                           hipEvent_t ev1) {
  return dispatch(
      b, [&](auto ops) { return decltype(ops)::half_psi(b, k, kc, l, check, tol, s, ev0, ev1); });
}

hipError_t launch_half_phi(const SolveBufs& b, const ScanConsts& k, const CarryConsts& kc, int l,
                           int check, double tol, hipStream_t s, hipEvent_t ev0,
                           hipEvent_t ev1) {
  return dispatch(
      b, [&](auto ops) { return decltype(ops)::half_phi(b, k, kc, l, check, tol, s, ev0, ev1); });
}

hipError_t launch_finalize(const SolveBufs& b, const ScanConsts& k, const CarryConsts& kc,
                           int gbuf, double h, hipStream_t s) {
  return dispatch(b, [&](auto ops) { return decltype(ops)::finalize(b, k, kc, gbuf, h, s); });
}

hipError_t launch_potentials(const SolveBufs& b, int gbuf, double* out, hipStream_t s) {
  return dispatch(b, [&](auto ops) { return decltype(ops)::potentials(b, gbuf, out, s); });
}

}  // namespace fs1
