// fs1_device.h -- device building blocks of the FS-1 scans (gfx950, wave64).
//
// Every K x of the method is the sum of two first-order recursions (Sec. 3,
// eq. (recursion)): the lower part p_k = lambda p_{k-1} + x_k and the strict
// upper part q_k = lambda (q_{k+1} + x_{k+1}).  A recursion x -> lambda x + b is
// an affine map; a run of L steps composes to x -> lambda^L x + (local sum),
// so the recursion is a scan over (lambda^L, local sum) pairs.  The scan here is
// hierarchical:
//   thread run of R consecutive elements (plain FMA recursion, as in the paper)
//   -> wavefront scan of the 64 run aggregates (Hillis-Steele over lanes)
//   -> block combine of the wavefront aggregates through LDS
//   -> chunk carries from the single-block carry kernel.
// Every quantity above the thread run is an extended-range number m * 2^e
// (mantissa in binary64 or binary32, int exponent).  The decay lambda^D between
// levels is one such number computed from D * h/eps, so lambda^D never
// underflows even when D h / eps is in the thousands (the concern of the Sec. 3
// remark on forming lambda^m); contributions are dropped only when they are
// below the working precision of the sum they join.
#pragma once

#include "fs1_internal.h"

namespace fs1 {

static constexpr double kLog2E = 1.4426950408889634074;
static constexpr double kLog2ELo = 2.0355273740931033e-17;  // log2(e) - kLog2E
static constexpr double kLn2 = 0.69314718055994530942;

// ---------------------------------------------------------------------------
// Extended-range numbers
// ---------------------------------------------------------------------------
template <typename T>
struct XF {
  T m;
  int e;
};

__device__ __forceinline__ double ldx(double m, int e) { return ldexp(m, e); }
__device__ __forceinline__ float ldx(float m, int e) { return ldexpf(m, e); }
__device__ __forceinline__ double frx(double m, int* e) { return frexp(m, e); }
__device__ __forceinline__ float frx(float m, int* e) { return frexpf(m, e); }

template <typename T>
__device__ __forceinline__ XF<T> xzero() {
  return {T(0), kExpZero};
}

template <typename T>
__device__ __forceinline__ XF<T> xnorm(T m, int e) {
  if (m == T(0)) return xzero<T>();
  if (!isfinite(m)) return {m, 0};
  int k;
  T f = frx(m, &k);
  return {f, e + k};
}

template <typename T>
__device__ __forceinline__ XF<T> xnorm(XF<T> a) {
  return xnorm(a.m, a.e);
}

template <typename T>
__device__ __forceinline__ XF<T> xadd(XF<T> a, XF<T> b) {
  const int e = max(a.e, b.e);
  return {ldx(a.m, a.e - e) + ldx(b.m, b.e - e), e};
}

template <typename T>
__device__ __forceinline__ XF<T> xmul(XF<T> a, XF<T> d) {
  if (a.m == T(0)) return xzero<T>();
  return {a.m * d.m, a.e + d.e};
}

template <typename T>
__device__ __forceinline__ XF<T> from64(const XF64& a) {
  return {T(a.m), a.e};
}

__device__ __forceinline__ XF64 to64(XF<double> a) { return {a.m, a.e, 0}; }
__device__ __forceinline__ XF64 to64(XF<float> a) { return {double(a.m), a.e, 0}; }

// Value of an extended number as a plain T (may overflow / underflow).
template <typename T>
__device__ __forceinline__ T xval(XF<T> a) {
  return ldx(a.m, a.e);
}

// ---------------------------------------------------------------------------
// Wavefront data movement without the LDS crossbar: DPP row shifts (within
// rows of 16 lanes), whole-wave shifts by one lane, and readlane.  A lane with
// no source lane reads `old`.
// ---------------------------------------------------------------------------
constexpr int kDppRowShr = 0x110;   // + n: lane i reads lane i - n of its row
constexpr int kDppRowShl = 0x100;   // + n: lane i reads lane i + n of its row
constexpr int kDppWaveShr1 = 0x138; // lane i reads lane i - 1
constexpr int kDppWaveShl1 = 0x130; // lane i reads lane i + 1

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v, int old) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v, float old = 0.0f) {
  return __int_as_float(dpp_i32<CTRL>(__float_as_int(v), __float_as_int(old)));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v, double old = 0.0) {
  const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned long long o = static_cast<unsigned long long>(__double_as_longlong(old));
  const unsigned lo = unsigned(dpp_i32<CTRL>(int(unsigned(u)), int(unsigned(o))));
  const unsigned hi = unsigned(dpp_i32<CTRL>(int(unsigned(u >> 32)), int(unsigned(o >> 32))));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}
template <int CTRL>
__device__ __forceinline__ int dpp(int v, int old = 0) {
  return dpp_i32<CTRL>(v, old);
}

__device__ __forceinline__ int lane_read(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float lane_read(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_read(double v, int l) {
  const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(unsigned(u)), l));
  const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(unsigned(u >> 32)), l));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// Sum over the 64 lanes, the same value in every lane, in a fixed order: each
// row of 16 lanes by four shifted adds (its total lands in its last lane), then
// the four row totals.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dpp<kDppRowShr + 1>(v);
  v += dpp<kDppRowShr + 2>(v);
  v += dpp<kDppRowShr + 4>(v);
  v += dpp<kDppRowShr + 8>(v);
  return (lane_read(v, 15) + lane_read(v, 31)) + (lane_read(v, 47) + lane_read(v, 63));
}

__device__ __forceinline__ int wave_max(int v) {
  v = max(v, dpp<kDppRowShr + 1>(v, v));
  v = max(v, dpp<kDppRowShr + 2>(v, v));
  v = max(v, dpp<kDppRowShr + 4>(v, v));
  v = max(v, dpp<kDppRowShr + 8>(v, v));
  return max(max(lane_read(v, 15), lane_read(v, 31)), max(lane_read(v, 47), lane_read(v, 63)));
}

// An extended number moved by DPP: a lane without a source lane reads zero.
template <int CTRL, typename T>
__device__ __forceinline__ XF<T> xmove(XF<T> v) {
  return {dpp<CTRL>(v.m, T(0)), dpp<CTRL>(v.e, kExpZero)};
}
template <typename T>
__device__ __forceinline__ XF<T> xlane(XF<T> v, int l) {
  return {lane_read(v.m, l), lane_read(v.e, l)};
}

// ---------------------------------------------------------------------------
// Decays lambda^D
// ---------------------------------------------------------------------------
template <typename T>
struct Dec {
  T m;
  int e;
  double dist;  // D (elements), used by the two-state cost recursion
};

template <typename T>
__device__ __forceinline__ Dec<T> dec_of(const Decay& d, double dist) {
  return {T(d.m), d.e, dist};
}

// ---------------------------------------------------------------------------
// The lambda-recursion step in the working precision.
//   lambda a + x:  fma(lambda, a, x), or (a + x) - mu a with mu = 1 - lambda when
//   lambda > 1/2, so that a binary32 lambda near 1 does not perturb h/eps.
// ---------------------------------------------------------------------------
template <typename T>
struct Lam {
  T lam;
  T mu;
  bool use_mu;
  __device__ __forceinline__ T axpy(T a, T x) const {
    return use_mu ? fma(-mu, a, a + x) : fma(lam, a, x);
  }
  __device__ __forceinline__ T mul(T a) const { return use_mu ? fma(-mu, a, a) : lam * a; }
};

// The same step with the choice made at compile time (kernels instantiated
// for both forms, so the unrolled recursions carry no select per step).
template <typename T, bool MU>
struct LamC {
  T lam;
  T mu;
  __device__ __forceinline__ T axpy(T a, T x) const {
    if constexpr (MU) {
      return fma(-mu, a, a + x);
    } else {
      return fma(lam, a, x);
    }
  }
  __device__ __forceinline__ T mul(T a) const {
    if constexpr (MU) {
      return fma(-mu, a, a);
    } else {
      return lam * a;
    }
  }
};

template <typename T, bool MU>
__device__ __forceinline__ LamC<T, MU> lamc_of(const ScanConsts& k) {
  return LamC<T, MU>{T(k.lam), T(k.mu)};
}

template <typename T>
__device__ __forceinline__ Lam<T> lam_of(const ScanConsts& k) {
  Lam<T> l;
  l.lam = T(k.lam);
  l.mu = T(k.mu);
  l.use_mu = k.use_mu != 0;
  return l;
}

// ---------------------------------------------------------------------------
// One-state scan element (the K x recursions): an extended number.
// Shifting a state by D elements with zero input multiplies it by lambda^D.
// ---------------------------------------------------------------------------
template <typename T>
struct S1 {
  XF<T> v;
  __device__ __forceinline__ static S1 zero() { return {xzero<T>()}; }
  __device__ __forceinline__ S1 shift(const Dec<T>& d) const { return {xmul(v, XF<T>{d.m, d.e})}; }
  __device__ __forceinline__ S1 add(const S1& o) const { return {xadd(v, o.v)}; }
  __device__ __forceinline__ S1 norm() const { return {xnorm(v)}; }
  template <int CTRL>
  __device__ __forceinline__ S1 move() const {
    return {xmove<CTRL>(v)};
  }
  __device__ __forceinline__ S1 lane(int l) const { return {xlane(v, l)}; }
};

// ---------------------------------------------------------------------------
// Two-state scan element for the transport cost: (p, D) with
//   p_i = sum_{j<=i} x_j lambda^{i-j},  D_i = sum_{j<=i} x_j lambda^{i-j} (i-j)
// (and the mirrored pair backwards).  Shifting by D elements with zero input:
//   (p, D) -> (lambda^D p, lambda^D (D + D_elems p)).
// Each component is its own extended number: D can sit far below p (by the
// factor lambda when h/eps is large), beyond the range of one shared exponent.
// ---------------------------------------------------------------------------
template <typename T>
struct S2 {
  XF<T> p;
  XF<T> d;
  __device__ __forceinline__ static S2 zero() { return {xzero<T>(), xzero<T>()}; }
  __device__ __forceinline__ static S2 of(T p, T d, int e) { return {xnorm(p, e), xnorm(d, e)}; }
  __device__ __forceinline__ S2 shift(const Dec<T>& dc) const {
    const XF<T> lam = {dc.m, dc.e};
    const XF<T> dp = xadd(d, XF<T>{p.m * T(dc.dist), p.e});
    return {xmul(p, lam), xmul(dp, lam)};
  }
  __device__ __forceinline__ S2 add(const S2& o) const { return {xadd(p, o.p), xadd(d, o.d)}; }
  __device__ __forceinline__ S2 norm() const { return {xnorm(p), xnorm(d)}; }
  template <int CTRL>
  __device__ __forceinline__ S2 move() const {
    return {xmove<CTRL>(p), xmove<CTRL>(d)};
  }
  __device__ __forceinline__ S2 lane(int l) const { return {xlane(p, l), xlane(d, l)}; }
};

// Carry of chunk c from the carry buffer: under the two-level scan the stored
// value covers the chunk's own group of 1024 chunks, and the group's carry
// (stored after the chunk carries) is added, moved to the chunk: forward by
// j chunks, backward by (chunks in the group) - 1 - j.
__device__ __forceinline__ ChunkAgg chunk_carry(const ChunkAgg* carry, const CarryFix& cf,
                                                int64_t c) {
  ChunkAgg lc = carry[c];
  if (!cf.two_level) return lc;
  constexpr int64_t G = kCarryBlock;
  const int64_t ng = (cf.nchunks + G - 1) / G;
  const int64_t g = c / G, j = c - g * G;
  const int64_t gact = min(G, cf.nchunks - g * G);
  const ChunkAgg gc = carry[cf.nchunks + ng + g];
  XF<double> pf = {1.0, 0}, pb = {1.0, 0};
#pragma unroll
  for (int s = 0; s < 11; ++s) {
    if ((j >> s) & 1) pf = {pf.m * cf.cpow[s].m, pf.e + cf.cpow[s].e};
    if (((gact - 1 - j) >> s) & 1) pb = {pb.m * cf.cpow[s].m, pb.e + cf.cpow[s].e};
  }
  const XF<double> f = xadd(XF<double>{lc.f.m, lc.f.e}, xmul(XF<double>{gc.f.m, gc.f.e}, pf));
  const XF<double> b = xadd(XF<double>{lc.b.m, lc.b.e}, xmul(XF<double>{gc.b.m, gc.b.e}, pb));
  lc.f = to64(xnorm(f));
  lc.b = to64(xnorm(b));
  return lc;
}

// lambda^(l * unit) from the binary expansion of l (unit = the lane span).
template <typename T>
__device__ __forceinline__ Dec<T> lane_pow(int l, const Dec<T>* dec) {
  Dec<T> r = {T(1), 0, 0.0};
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    if ((l >> s) & 1) {
      r.m *= dec[s].m;
      r.e += dec[s].e;
      r.dist += dec[s].dist;
    }
  }
  return r;
}

// ---------------------------------------------------------------------------
// Block scan.  Each thread contributes the aggregates of its run:
//   tf: forward state at the run's last element (run fed with zero),
//   tb: inclusive backward state at the run's first element.
// dec[s] = lambda^(run span * 2^s) for s = 0..5 and dec[6] = lambda^(wave span).
// With block carries bcf (forward state just before the block) and bcb
// (inclusive backward state just after the block) it returns each thread's
// carries: cf = forward state just before its run, cb = inclusive backward
// state just after its run.  It can also return the block aggregates.
// ---------------------------------------------------------------------------
template <typename S, int NW>
struct ScanLds {
  S f[NW];
  S b[NW];
};

template <typename S, int NW, typename T>
__device__ __forceinline__ void block_scan(S tf, S tb, const Dec<T>* dec, const S& bcf,
                                           const S& bcb, S* cf, S* cb, S* agg_f, S* agg_b,
                                           ScanLds<S, NW>& sh) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  S incf = tf.norm();
  S incb = tb.norm();
  // within rows of 16 lanes (DPP row shifts; a lane without a source adds zero)
  incf = incf.add(incf.template move<kDppRowShr + 1>().shift(dec[0]));
  incb = incb.add(incb.template move<kDppRowShl + 1>().shift(dec[0]));
  incf = incf.add(incf.template move<kDppRowShr + 2>().shift(dec[1]));
  incb = incb.add(incb.template move<kDppRowShl + 2>().shift(dec[1]));
  incf = incf.add(incf.template move<kDppRowShr + 4>().shift(dec[2]));
  incb = incb.add(incb.template move<kDppRowShl + 4>().shift(dec[2]));
  incf = incf.add(incf.template move<kDppRowShr + 8>().shift(dec[3]));
  incb = incb.add(incb.template move<kDppRowShl + 8>().shift(dec[3]));
  incf = incf.norm();
  incb = incb.norm();
  if (!cf && agg_f) {
    // totals only: the wavefront's forward total is its last lane's value
    // after the cross-row step below and the backward total its first lane's,
    // formed here directly by the same operations in the same order (the
    // lane power there is lambda^(16 R) = dec[4] for both), without the
    // per-lane step that only the prefixes need
    const S p15 = incf.lane(15);
    const S p31 = incf.lane(31).add(p15.shift(dec[4])).norm();
    const S p47 = incf.lane(47).add(p31.shift(dec[4])).norm();
    const S wf = incf.lane(kWave - 1).add(p47.shift(dec[4])).norm();
    const S s48 = incb.lane(48);
    const S s32 = incb.lane(32).add(s48.shift(dec[4])).norm();
    const S s16 = incb.lane(16).add(s32.shift(dec[4])).norm();
    const S wb = incb.lane(0).add(s16.shift(dec[4])).norm();
    if constexpr (NW == 1) {
      *agg_f = wf.norm();
      *agg_b = wb.norm();
      return;
    }
    if (lane == 0) {
      sh.f[w] = wf;
      sh.b[w] = wb;
    }
    __syncthreads();
    S af = S::zero();
    S ab = S::zero();
    for (int v = 0; v < NW; ++v) af = af.shift(dec[6]).add(sh.f[v]);
    for (int v = NW - 1; v >= 0; --v) ab = ab.shift(dec[6]).add(sh.b[v]);
    *agg_f = af.norm();
    *agg_b = ab.norm();
    __syncthreads();
    return;
  }
  // across rows: the rows before (after) a row enter through the last (first)
  // lane of its neighbour row, read once per wavefront
  const int row = lane >> 4;
  {
    const S p15 = incf.lane(15);
    const S p31 = incf.lane(31).add(p15.shift(dec[4])).norm();
    const S p47 = incf.lane(47).add(p31.shift(dec[4])).norm();
    const S c = row == 0 ? S::zero() : (row == 1 ? p15 : (row == 2 ? p31 : p47));
    incf = incf.add(c.shift(lane_pow((lane & 15) + 1, dec))).norm();
  }
  {
    const S s48 = incb.lane(48);
    const S s32 = incb.lane(32).add(s48.shift(dec[4])).norm();
    const S s16 = incb.lane(16).add(s32.shift(dec[4])).norm();
    const S c = row == 3 ? S::zero() : (row == 2 ? s48 : (row == 1 ? s32 : s16));
    incb = incb.add(c.shift(lane_pow(16 - (lane & 15), dec))).norm();
  }
  // exclusive values: the neighbouring lane's inclusive value (zero at the ends)
  const S exf = incf.template move<kDppWaveShr1>();
  const S exb = incb.template move<kDppWaveShl1>();
  if constexpr (NW == 1) {
    // one wavefront: its totals are read from its end lanes, no LDS exchange
    if (cf) {
      *cf = bcf.shift(lane_pow(lane, dec)).add(exf).norm();
      *cb = bcb.shift(lane_pow(kWave - 1 - lane, dec)).add(exb).norm();
    }
    if (agg_f) {
      *agg_f = incf.lane(kWave - 1).norm();
      *agg_b = incb.lane(0).norm();
    }
    return;
  }
  if (lane == kWave - 1) sh.f[w] = incf;
  if (lane == 0) sh.b[w] = incb;
  __syncthreads();
  if (cf) {
    S accf = bcf;
    for (int v = 0; v < w; ++v) accf = accf.shift(dec[6]).add(sh.f[v]);
    S accb = bcb;
    for (int v = NW - 1; v > w; --v) accb = accb.shift(dec[6]).add(sh.b[v]);
    *cf = accf.shift(lane_pow(lane, dec)).add(exf).norm();
    *cb = accb.shift(lane_pow(kWave - 1 - lane, dec)).add(exb).norm();
  }
  if (agg_f) {
    S af = S::zero();
    S ab = S::zero();
    for (int v = 0; v < NW; ++v) af = af.shift(dec[6]).add(sh.f[v]);
    for (int v = NW - 1; v >= 0; --v) ab = ab.shift(dec[6]).add(sh.b[v]);
    *agg_f = af.norm();
    *agg_b = ab.norm();
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Deterministic block sum of a double (fixed reduction order).
// ---------------------------------------------------------------------------
template <int NW>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  v = wave_sum(v);
  if constexpr (NW == 1) return v;  // one wavefront: every lane holds the sum
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NW; ++i) t += sh[i];
  }
  __syncthreads();
  return t;  // valid in thread 0
}

// ---------------------------------------------------------------------------
// Run loads and stores (R consecutive elements per thread).  The vector path
// needs 16-byte aligned arrays (checked by the host); the tail run is guarded.
// ---------------------------------------------------------------------------
template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int n = 2;
};
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int n = 4;
};

// The vector-or-guarded choice is made per wavefront (a ballot over the
// active lanes), not per lane: a divergent choice would run both sides and
// make the guarded side wait for every load still in flight, since both write
// the same registers.
template <typename T, int R>
__device__ __forceinline__ void load_run(const T* __restrict__ p, int64_t base, int64_t n,
                                         T (&x)[R], T fill) {
  constexpr int V = Vec16<T>::n;
  if constexpr (R % V == 0) {
    if (__builtin_amdgcn_ballot_w64(base + R > n) == 0) {
      using VT = typename Vec16<T>::type;
      const VT* q = reinterpret_cast<const VT*>(p + base);
#pragma unroll
      for (int i = 0; i < R / V; ++i) {
        const VT v = q[i];
        if constexpr (V == 2) {
          x[2 * i] = v.x;
          x[2 * i + 1] = v.y;
        } else {
          x[4 * i] = v.x;
          x[4 * i + 1] = v.y;
          x[4 * i + 2] = v.z;
          x[4 * i + 3] = v.w;
        }
      }
      return;
    }
  }
#pragma unroll
  for (int j = 0; j < R; ++j) x[j] = (base + j < n) ? p[base + j] : fill;
}

template <typename T, int R>
__device__ __forceinline__ void store_run(T* __restrict__ p, int64_t base, int64_t n,
                                          const T (&x)[R]) {
  constexpr int V = Vec16<T>::n;
  if constexpr (R % V == 0) {
    if (__builtin_amdgcn_ballot_w64(base + R > n) == 0) {
      using VT = typename Vec16<T>::type;
      VT* q = reinterpret_cast<VT*>(p + base);
#pragma unroll
      for (int i = 0; i < R / V; ++i) {
        VT v;
        if constexpr (V == 2) {
          v.x = x[2 * i];
          v.y = x[2 * i + 1];
        } else {
          v.x = x[4 * i];
          v.y = x[4 * i + 1];
          v.z = x[4 * i + 2];
          v.w = x[4 * i + 3];
        }
        q[i] = v;
      }
      return;
    }
  }
#pragma unroll
  for (int j = 0; j < R; ++j)
    if (base + j < n) p[base + j] = x[j];
}

// Run loads and stores on arrays allocated to whole chunks whose entries past
// n hold zeros (every run of the grid lies inside the allocation): plain
// 16-byte vector accesses, with no branch or select that would make the
// kernel wait for a load before it needs the value.
template <typename T, int R>
__device__ __forceinline__ void load_run_z(const T* __restrict__ p, int64_t base, T (&x)[R]) {
  constexpr int V = Vec16<T>::n;
  static_assert(R % V == 0, "padded runs are whole 16-byte vectors");
  using VT = typename Vec16<T>::type;
  const VT* q = reinterpret_cast<const VT*>(p + base);
#pragma unroll
  for (int i = 0; i < R / V; ++i) {
    const VT v = q[i];
    if constexpr (V == 2) {
      x[2 * i] = v.x;
      x[2 * i + 1] = v.y;
    } else {
      x[4 * i] = v.x;
      x[4 * i + 1] = v.y;
      x[4 * i + 2] = v.z;
      x[4 * i + 3] = v.w;
    }
  }
}

template <typename T, int R>
__device__ __forceinline__ void store_run_z(T* __restrict__ p, int64_t base, const T (&x)[R]) {
  constexpr int V = Vec16<T>::n;
  static_assert(R % V == 0, "padded runs are whole 16-byte vectors");
  using VT = typename Vec16<T>::type;
  VT* q = reinterpret_cast<VT*>(p + base);
#pragma unroll
  for (int i = 0; i < R / V; ++i) {
    VT v;
    if constexpr (V == 2) {
      v.x = x[2 * i];
      v.y = x[2 * i + 1];
    } else {
      v.x = x[4 * i];
      v.y = x[4 * i + 1];
      v.z = x[4 * i + 2];
      v.w = x[4 * i + 3];
    }
    q[i] = v;
  }
}

// ===========================================================================
// Device helpers
// ===========================================================================
enum InMode { IN_PLAIN = 0, IN_SCALED = 1, IN_LOG = 2 };

template <typename T, int R>
__device__ __forceinline__ void load_log_run(const T* __restrict__ lx, int64_t base, int64_t n,
                                             T (&x)[R], int& E) {
  T raw[R];
  load_run<T, R>(lx, base, n, raw, T(-INFINITY));
  // t = lx log2(e) as t + te with log2(e) split into two doubles: the rounding
  // of the product alone would be an absolute error of about u |lx| in the
  // exponent, large against the output when lx is far from ln y
  double t[R], te[R];
  double tmax = -INFINITY;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const double v = double(raw[j]);
    t[j] = v * kLog2E;
    te[j] = isfinite(t[j]) ? fma(v, kLog2E, -t[j]) + v * kLog2ELo : 0.0;
    if (isfinite(t[j])) tmax = fmax(tmax, t[j]);
  }
  double Ed = (tmax == -INFINITY) ? 0.0 : floor(tmax);
  Ed = fmin(fmax(Ed, -4.0e8), 4.0e8);
  E = int(Ed);
  // 2^(t_j - E) = 2^frac(t_j) * 2^(floor(t_j) - E): only the exact fractional
  // part goes through the exponential, so entries far below the run maximum
  // keep their relative precision
#pragma unroll
  for (int j = 0; j < R; ++j) {
    if (isfinite(t[j])) {
      const double k = floor(t[j]);
      const double f = (t[j] - k) + te[j];  // t - k exact, in [0, 1)
      const int sh = int(fmax(k - Ed, -2000.0));
      if constexpr (sizeof(T) == 8) {
        x[j] = ldexp(exp2(f), sh);
      } else {
        x[j] = ldexpf(exp2f(float(f)), sh);
      }
    } else {
      x[j] = T(exp2(t[j]));  // 0 for -inf; +inf or NaN propagate
    }
  }
}

template <typename T, int R, int IN>
__device__ __forceinline__ void load_input(const T* __restrict__ v, const int* __restrict__ ex,
                                           int64_t run, int64_t n, T (&x)[R], int& E) {
  const int64_t base = run * R;
  if constexpr (IN == IN_LOG) {
    load_log_run<T, R>(v, base, n, x, E);
  } else {
    load_run<T, R>(v, base, n, x, T(0));
    E = (IN == IN_SCALED) ? ex[run] : 0;
  }
}

template <typename T, int R, typename LT>
__device__ __forceinline__ void run_aggs(const T (&x)[R], const LT& L, T& af, T& ab) {
  T a = T(0), b = T(0);
#pragma unroll
  for (int j = 0; j < R; ++j) a = L.axpy(a, x[j]);
#pragma unroll
  for (int j = R - 1; j >= 0; --j) b = L.axpy(b, x[j]);
  af = a;
  ab = b;
}

template <typename T>
__device__ __forceinline__ void lane_decays(const ScanConsts& k, Dec<T> (&dec)[7]) {
#pragma unroll
  for (int s = 0; s < 7; ++s) dec[s] = dec_of<T>(k.lane[s], double(k.R) * double(1 << s));
}

// Largest exponent of the local values: values < 2^eloc.
template <typename T, int R>
__device__ __forceinline__ int local_exponent(const T (&x)[R], int E) {
  T mx = T(0);
#pragma unroll
  for (int j = 0; j < R; ++j) mx = fmax(mx, x[j]);
  if (!(mx > T(0))) return kExpZero;
  if (!isfinite(mx)) return E;
  int k;
  frx(mx, &k);
  return E + k;
}

// Both recursions of eq. (recursion) over one run, in the run's frame:
// y_k = p_k + q_k.  The carries come in already moved one step into the run:
// lcf = lambda * (forward state before the run), lcb = lambda * (inclusive
// backward state after the run).  Callers form them in extended range
// (step_in), so a lambda below the working precision's normal range (large
// h/eps, where runs have length 1) never multiplies a plain value.
template <typename T, int R, typename LT>
__device__ __forceinline__ void run_apply(const T (&xf)[R], T lcf, T lcb, const LT& L,
                                          T (&y)[R]) {
  T A = lcf + xf[0];
  y[0] = A;
#pragma unroll
  for (int j = 1; j < R; ++j) {
    A = L.axpy(A, xf[j]);
    y[j] = A;
  }
  T B = lcb;
  y[R - 1] += B;
  T P = B + xf[R - 1];
#pragma unroll
  for (int j = R - 2; j >= 0; --j) {
    B = L.mul(P);
    y[j] += B;
    P = B + xf[j];
  }
}

// lambda^1 as a decay (one grid step)
template <typename T>
__device__ __forceinline__ Dec<T> step_decay(const ScanConsts& k) {
  return dec_of<T>(k.step1, 1.0);
}

// ---------------------------------------------------------------------------
// Transport cost: W = h sum_i phi_i (D_i + E_i), with
//   D_i = sum_{j<i} psi_j lambda^{i-j} (i-j),  E_i = sum_{j>i} psi_j lambda^{j-i} (j-i).
// Forward pair (p, D): D <- lambda (D + p), p <- lambda p + psi_j; the
// backward pair mirrors it.  These follow from splitting |i-j| in the double
// sum of Algorithm 1's return into j < i and j > i.
// ---------------------------------------------------------------------------
// Forward and backward two-state aggregates (or carries) of one chunk, with
// the exponents of p and D.
struct ChunkAgg2 {
  double fp, fd;
  int fpe, fde;
  double bp, bd;
  int bpe, bde;
};

template <typename T>
__device__ __forceinline__ S2<T> s2_fwd(const ChunkAgg2& a) {
  return {{T(a.fp), a.fpe}, {T(a.fd), a.fde}};
}
template <typename T>
__device__ __forceinline__ S2<T> s2_bwd(const ChunkAgg2& a) {
  return {{T(a.bp), a.bpe}, {T(a.bd), a.bde}};
}
template <typename T>
__device__ __forceinline__ S2<T> s2_cast(const S2<double>& s) {
  return {{T(s.p.m), s.p.e}, {T(s.d.m), s.d.e}};
}
template <typename T>
__device__ __forceinline__ void s2_put_fwd(ChunkAgg2& o, const S2<T>& s) {
  o.fp = double(s.p.m);
  o.fpe = s.p.e;
  o.fd = double(s.d.m);
  o.fde = s.d.e;
}
template <typename T>
__device__ __forceinline__ void s2_put_bwd(ChunkAgg2& o, const S2<T>& s) {
  o.bp = double(s.p.m);
  o.bpe = s.p.e;
  o.bd = double(s.d.m);
  o.bde = s.d.e;
}

// Frame of a run's cost outputs w = D + E: the shifted carries' D parts and,
// within runs of R > 1, lambda times the largest local value (bounded so that
// the local values themselves stay finite in the frame).
template <typename T, int R>
__device__ __forceinline__ int cost_frame(const S2<T>& lcf, const S2<T>& lcb, int eloc,
                                          const ScanConsts& k) {
  int eref = max(lcf.d.e, lcb.d.e);
  if (R > 1 && eloc != kExpZero) eref = max(eref, eloc + max(k.step1.e + 1, -60));
  return eref == kExpZero ? 0 : eref;
}

template <typename T, int R>
__device__ __forceinline__ void run_aggs2(const T (&x)[R], const Lam<T>& L, T& fp, T& fd, T& bp,
                                          T& bd) {
  T p = T(0), d = T(0);
#pragma unroll
  for (int j = 0; j < R; ++j) {
    d = L.mul(d + p);
    p = L.axpy(p, x[j]);
  }
  T q = T(0), e = T(0);
#pragma unroll
  for (int j = R - 1; j >= 0; --j) {
    e = L.mul(e + q);
    q = L.axpy(q, x[j]);
  }
  fp = p;
  fd = d;
  bp = q;
  bd = e;
}

// w_k = D_k + E_k over one run, in the run's frame, from the two-state carries
// moved one step into the run (S2::shift by lambda^1, in extended range):
// (lfp, lfd) = lambda (p, D + p) of the state before the run, (lbp, lbd) the
// same of the inclusive backward state after the run.
template <typename T, int R>
__device__ __forceinline__ void run_cost(const T (&xf)[R], T lfp, T lfd, T lbp, T lbd,
                                         const Lam<T>& L, T (&w)[R]) {
  T p = lfp + xf[0], d = lfd;
  w[0] = d;
#pragma unroll
  for (int j = 1; j < R; ++j) {
    d = L.mul(d + p);
    p = L.axpy(p, xf[j]);
    w[j] = d;
  }
  T q = lbp + xf[R - 1], e = lbd;
  w[R - 1] += e;
#pragma unroll
  for (int j = R - 2; j >= 0; --j) {
    e = L.mul(e + q);
    q = L.axpy(q, xf[j]);
    w[j] += e;
  }
}

}  // namespace fs1
