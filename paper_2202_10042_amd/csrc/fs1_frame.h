// fs1_frame.h -- chunk-local FS-1 recursions in plain arithmetic on a
// power-of-two frame (device helpers shared by the fused and the persistent
// solvers).
//
// Every output of a chunk of length C is within lambda^C of the chunk's
// largest contribution (K has positive entries and lambda^{|i-j|} >= lambda^C
// inside the chunk), so scaling every value of the chunk by one power of two
// -- the frame -- and running the recursions of Sec. 3, eq. (recursion) in
// plain floating point loses nothing but rounding, provided
// C * h/eps * log2(e) stays well inside the exponent range of the working
// precision (the host checks this before choosing these kernels).  Values
// that underflow in the frame are below the working precision of every output
// they reach.  Carries between chunks are extended-range numbers.
#pragma once

#include "fs1_device.h"
#include "fs1_internal.h"

namespace fs1 {

constexpr int kNW = kBlock / kWave;

template <typename T>
struct FastDec {
  T step[6];   // lambda^(R 2^s)
  T wave;      // lambda^(64 R)
  T lane_f;    // lambda^(lane R)
  T lane_b;    // lambda^((63 - lane) R)
  T row_f;     // lambda^(((lane mod 16) + 1) R): from the last lane of the row before
  T row_b;     // lambda^((16 - lane mod 16) R): from the first lane of the row after
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
  const int nf = (lane & 15) + 1, nb = 16 - (lane & 15);  // both in [1, 16]
  mf = mb = 1.0;
  ef = eb = 0;
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    if ((nf >> s) & 1) {
      mf *= k.lane[s].m;
      ef += k.lane[s].e;
    }
    if ((nb >> s) & 1) {
      mb *= k.lane[s].m;
      eb += k.lane[s].e;
    }
  }
  D.row_f = T(ldexp(mf, ef));
  D.row_b = T(ldexp(mb, eb));
  return D;
}

// Inclusive decayed scans over the 64 lanes of a wavefront, forward
// (f_i = sum_{k <= i} lambda^{(i-k) R} v_k) and backward
// (b_i = sum_{k >= i} lambda^{(k-i) R} v_k): within each row of 16 lanes by
// shifted multiply-adds, then the rows before (after) a row enter through
// its first (last) lane's neighbour, read once per wavefront.
template <typename T>
__device__ __forceinline__ T wave_fscan(T f, const FastDec<T>& D, int lane) {
  f = fma(D.step[0], dpp<kDppRowShr + 1>(f), f);
  f = fma(D.step[1], dpp<kDppRowShr + 2>(f), f);
  f = fma(D.step[2], dpp<kDppRowShr + 4>(f), f);
  f = fma(D.step[3], dpp<kDppRowShr + 8>(f), f);
  const T p15 = lane_read(f, 15);
  const T p31 = fma(D.step[4], p15, lane_read(f, 31));
  const T p47 = fma(D.step[4], p31, lane_read(f, 47));
  const int row = lane >> 4;
  const T c = row == 0 ? T(0) : (row == 1 ? p15 : (row == 2 ? p31 : p47));
  return fma(D.row_f, c, f);
}

template <typename T>
__device__ __forceinline__ T wave_bscan(T b, const FastDec<T>& D, int lane) {
  b = fma(D.step[0], dpp<kDppRowShl + 1>(b), b);
  b = fma(D.step[1], dpp<kDppRowShl + 2>(b), b);
  b = fma(D.step[2], dpp<kDppRowShl + 4>(b), b);
  b = fma(D.step[3], dpp<kDppRowShl + 8>(b), b);
  const T s48 = lane_read(b, 48);
  const T s32 = fma(D.step[4], s48, lane_read(b, 32));
  const T s16 = fma(D.step[4], s32, lane_read(b, 16));
  const int row = lane >> 4;
  const T c = row == 3 ? T(0) : (row == 2 ? s48 : (row == 1 ? s32 : s16));
  return fma(D.row_b, c, b);
}

__device__ __forceinline__ int block_max_int(int v, int* sh) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  v = wave_max(v);
  if (lane == 0) sh[w] = v;
  __syncthreads();
  int r = sh[0];
#pragma unroll
  for (int i = 1; i < kNW; ++i) r = max(r, sh[i]);
  __syncthreads();
  return r;
}

// xfloat sum over the 64 lanes (every lane returns the same value): each row
// by shifted adds (lanes without a source read a zero), then the four row
// totals in order.
template <int CTRL>
__device__ __forceinline__ XF<double> xdpp(XF<double> v) {
  return {dpp<CTRL>(v.m, 0.0), dpp<CTRL>(v.e, kExpZero)};
}

__device__ __forceinline__ XF<double> wave_xsum(XF<double> v) {
  v = xnorm(xadd(v, xdpp<kDppRowShr + 1>(v)));
  v = xnorm(xadd(v, xdpp<kDppRowShr + 2>(v)));
  v = xnorm(xadd(v, xdpp<kDppRowShr + 4>(v)));
  v = xnorm(xadd(v, xdpp<kDppRowShr + 8>(v)));
  XF<double> r[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) r[q] = {lane_read(v.m, 16 * q + 15), lane_read(v.e, 16 * q + 15)};
  return xnorm(xadd(xnorm(xadd(r[0], r[1])), xnorm(xadd(r[2], r[3]))));
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
__device__ __forceinline__ XF<double> carry_fwd(const ChunkAgg* A, int b, const Decay* cpow) {
  const int lane = threadIdx.x & (kWave - 1);
  const int seg = (b + kWave - 1) / kWave;
  const int lo = lane * seg;
  const int hi = min(lo + seg, b);
  XF<double> acc = xzero<double>();
  if (lo < hi) {
    const XF<double> cd = {cpow[0].m, cpow[0].e};
    for (int c = lo; c < hi; ++c) acc = xnorm(xadd(xmul(acc, cd), XF<double>{A[c].f.m, A[c].f.e}));
    acc = xmul(acc, pow_bits(b - hi, cpow));  // from the end of chunk hi-1 to the end of b-1
  }
  return wave_xsum(acc);
}

// Backward carry into chunk b (inclusive backward state at the element after
// the chunk) from the backward aggregates of chunks b+1..nchunks-1.
__device__ __forceinline__ XF<double> carry_bwd(const ChunkAgg* A, int b, int nchunks,
                                                const Decay* cpow) {
  const int lane = threadIdx.x & (kWave - 1);
  const int first = b + 1;
  const int cnt = nchunks - first;
  const int seg = (cnt + kWave - 1) / kWave;
  const int lo = first + lane * seg;
  const int hi = min(lo + seg, nchunks);
  XF<double> acc = xzero<double>();
  if (cnt > 0 && lo < hi) {
    const XF<double> cd = {cpow[0].m, cpow[0].e};
    for (int c = hi - 1; c >= lo; --c)
      acc = xnorm(xadd(xmul(acc, cd), XF<double>{A[c].b.m, A[c].b.e}));
    acc = xmul(acc, pow_bits(lo - first, cpow));  // from the start of lo to the start of b+1
  }
  return wave_xsum(acc);
}

// Chunk carries computed by the whole workgroup.  Threads 0..127 build the
// forward carry of chunk b from chunks 0..b-1, threads 128..255 the backward
// carry from chunks b+1..nchunks-1; each thread takes a contiguous segment of
// at most CMAX chunks, whose aggregates are loaded at kernel start
// (carry_prefetch) so that the loads overlap the chunk's own scans.
template <int CMAX>
struct CarryItems {
  double m[CMAX];
  int e[CMAX];
  int lo, hi;  // segment [lo, hi)
};

// Decays lambda^(C d) of the items of a segment (carry_table).
template <int CMAX>
struct CarryDecays {
  double m[CMAX];
  int e[CMAX];
};

// Plain loads of published aggregates (a previous launch wrote them).
struct PlainLoad {
  __device__ XF64 operator()(const XF64* p) const { return *p; }
};

template <int CMAX, typename Load = PlainLoad>
__device__ __forceinline__ void carry_prefetch(const ChunkAgg* A, int b, int nchunks,
                                               CarryItems<CMAX>& it, Load load = Load()) {
  const bool fwd = threadIdx.x < kBlock / 2;
  const int u = threadIdx.x & (kBlock / 2 - 1);
  const int first = fwd ? 0 : b + 1;
  const int cnt = fwd ? b : nchunks - b - 1;
  const int seg = (cnt + kBlock / 2 - 1) / (kBlock / 2);
  it.lo = first + u * seg;
  it.hi = min(it.lo + seg, first + cnt);
#pragma unroll
  for (int i = 0; i < CMAX; ++i) {
    const int c = it.lo + i;
    if (c < it.hi) {
      const XF64 v = load(fwd ? &A[c].f : &A[c].b);
      it.m[i] = v.m;
      it.e[i] = v.e;
    } else {
      it.m[i] = 0.0;
      it.e[i] = kExpZero;
    }
  }
}

// The decays of a prefetched segment from the table tab[d] = lambda^(C d)
// (C the chunk length): d = b-1-c forward, c-b-1 backward.
template <int CMAX>
__device__ __forceinline__ void carry_table(const XF64* tab, int b, const CarryItems<CMAX>& it,
                                            CarryDecays<CMAX>& dc) {
  const bool fwd = threadIdx.x < kBlock / 2;
#pragma unroll
  for (int i = 0; i < CMAX; ++i) {
    const int c = it.lo + i;
    if (c < it.hi) {
      const XF64 t = tab[fwd ? b - 1 - c : c - b - 1];
      dc.m[i] = t.m;
      dc.e[i] = t.e;
    } else {
      dc.m[i] = 0.0;
      dc.e[i] = 0;
    }
  }
}

// Combine the prefetched segments: forward carry into scar[0], backward into
// scar[1] (both extended-range, normalised).
template <int CMAX>
__device__ __forceinline__ void carry_finish(const CarryItems<CMAX>& it, int b,
                                             const Decay* cpow, XF64* red4, XF64* scar) {
  const bool fwd = threadIdx.x < kBlock / 2;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const XF<double> cd = {cpow[0].m, cpow[0].e};
  XF<double> acc = xzero<double>();
  if (it.lo < it.hi) {
    if (fwd) {
#pragma unroll
      for (int i = 0; i < CMAX; ++i)
        if (it.lo + i < it.hi) acc = xnorm(xadd(xmul(acc, cd), XF<double>{it.m[i], it.e[i]}));
      acc = xmul(acc, pow_bits(b - it.hi, cpow));  // end of chunk hi-1 -> end of chunk b-1
    } else {
#pragma unroll
      for (int i = CMAX - 1; i >= 0; --i)
        if (it.lo + i < it.hi) acc = xnorm(xadd(xmul(acc, cd), XF<double>{it.m[i], it.e[i]}));
      acc = xmul(acc, pow_bits(it.lo - (b + 1), cpow));  // start of lo -> start of b+1
    }
  }
  acc = wave_xsum(acc);
  if (lane == 0) red4[w] = to64(acc);
  __syncthreads();
  if (threadIdx.x == 0) {
    scar[0] = to64(xnorm(xadd(XF<double>{red4[0].m, red4[0].e}, XF<double>{red4[1].m, red4[1].e})));
    scar[1] = to64(xnorm(xadd(XF<double>{red4[2].m, red4[2].e}, XF<double>{red4[3].m, red4[3].e})));
  }
  __syncthreads();
}

// Combine the prefetched segments with their table decays (carry_table):
// the forward carry of chunk b is the sum over c < b of
// lambda^(C (b-1-c)) F_c, the backward one the sum over c > b of
// lambda^(C (c-b-1)) B_c.  The terms are independent: each wave takes the
// largest exponent of its terms (an integer max), sums the terms aligned to
// it in binary64, and the two waves of a direction are combined in extended
// range (forward into scar[0], backward into scar[1]).
template <int CMAX>
__device__ __forceinline__ void carry_finish_tab(const CarryItems<CMAX>& it,
                                                 const CarryDecays<CMAX>& dc, XF64* red4,
                                                 XF64* scar) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  double tm[CMAX];
  int te[CMAX];
  int emax = kExpZero;
#pragma unroll
  for (int i = 0; i < CMAX; ++i) {
    if (it.lo + i < it.hi && it.m[i] != 0.0) {
      tm[i] = it.m[i] * dc.m[i];
      te[i] = it.e[i] + dc.e[i];
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
struct HalfState {
  T xf[R];     // input run in the chunk frame
  T exf, exb;  // wave-exclusive carries (chunk frame)
  int ein;     // chunk frame exponent of the input
};

// Frame, thread aggregates and wave scans of a chunk's runs (x_j 2^ex per
// run): fills hs and the per-wave aggregates sf / sb (LDS, chunk frame).
template <typename T, int R>
__device__ __forceinline__ void local_scan(const T (&x)[R], int ex, const Lam<T>& L,
                                           const FastDec<T>& D, T* sf, T* sb, int* smax,
                                           HalfState<T, R>& hs) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int eb = block_max_int(local_exponent<T, R>(x, ex), smax);
  // an all-zero chunk keeps the zero exponent: its frame then comes from the
  // carries alone (see frame_apply)
  hs.ein = eb;
#pragma unroll
  for (int j = 0; j < R; ++j) hs.xf[j] = (eb == kExpZero) ? T(0) : ldx(x[j], ex - hs.ein);
  T f, b;
  run_aggs<T, R>(hs.xf, L, f, b);
  f = wave_fscan<T>(f, D, lane);
  b = wave_bscan<T>(b, D, lane);
  // exclusive values: the neighbouring lane's inclusive value (0 at the ends)
  hs.exf = dpp<kDppWaveShr1>(f);
  hs.exb = dpp<kDppWaveShl1>(b);
  if (lane == kWave - 1) sf[w] = f;
  if (lane == 0) sb[w] = b;
  __syncthreads();
}

// The chunk's forward / backward aggregates (extended range, normalised) from
// the per-wave aggregates.
template <typename T>
__device__ __forceinline__ void chunk_aggs(const FastDec<T>& D, const T* sf, const T* sb, int ein,
                                           XF64& f, XF64& b) {
  T gf = T(0), gb = T(0);
#pragma unroll
  for (int v = 0; v < kNW; ++v) gf = fma(D.wave, gf, sf[v]);
#pragma unroll
  for (int v = kNW - 1; v >= 0; --v) gb = fma(D.wave, gb, sb[v]);
  f = to64(xnorm(gf, ein));
  b = to64(xnorm(gb, ein));
}

// Thread 0 stores the chunk's aggregates to A[blockIdx.x].
template <typename T>
__device__ __forceinline__ void publish(const FastDec<T>& D, const T* sf, const T* sb, int ein,
                                        ChunkAgg* A) {
  if (threadIdx.x == 0) chunk_aggs<T>(D, sf, sb, ein, A[blockIdx.x].f, A[blockIdx.x].b);
}

// Phase 3 of a half: chunk carries (waves 0 and 1), frame alignment, in-chunk
// recursions.  Returns y = (K in) * 2^-eap in every thread's run.
template <typename T, int R>
__device__ __forceinline__ int half_apply(const ChunkAgg* A, int nchunks, const Decay* cpow,
                                          const Lam<T>& L, const FastDec<T>& D, const T* sf,
                                          const T* sb, XF64* scar, HalfState<T, R>& hs,
                                          T (&y)[R]) {
  const int w = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int b = blockIdx.x;
  if (w == 0) {
    const XF<double> cf = carry_fwd(A, b, cpow);
    if (lane == 0) scar[0] = to64(cf);
  } else if (w == 1) {
    const XF<double> cb = carry_bwd(A, b, nchunks, cpow);
    if (lane == 0) scar[1] = to64(cb);
  }
  __syncthreads();
  const XF64 cf = scar[0];
  const XF64 cb = scar[1];
  int eap = hs.ein;
  if (cf.m != 0.0) eap = max(eap, cf.e);
  if (cb.m != 0.0) eap = max(eap, cb.e);
  if (eap == kExpZero) eap = 0;  // nothing nonzero reaches this chunk
  const int sh = (hs.ein == kExpZero) ? 0 : hs.ein - eap;  // <= 0: rescale the chunk-frame quantities
  T accf = T(ldexp(cf.m, cf.e - eap));
  T accb = T(ldexp(cb.m, cb.e - eap));
  for (int v = 0; v < w; ++v) accf = fma(D.wave, accf, ldx(sf[v], sh));
  for (int v = kNW - 1; v > w; --v) accb = fma(D.wave, accb, ldx(sb[v], sh));
  const T tcf = fma(D.lane_f, accf, ldx(hs.exf, sh));
  const T tcb = fma(D.lane_b, accb, ldx(hs.exb, sh));
  T xf[R];
#pragma unroll
  for (int j = 0; j < R; ++j) xf[j] = ldx(hs.xf[j], sh);
  run_apply<T, R>(xf, L.mul(tcf), L.mul(tcb), L, y);
  return eap;
}

// As half_apply, with the chunk carries already in scar (carry_finish).
template <typename T, int R>
__device__ __forceinline__ int frame_apply(const Lam<T>& L, const FastDec<T>& D, const T* sf,
                                           const T* sb, const XF64* scar, HalfState<T, R>& hs,
                                           T (&y)[R]) {
  const int w = threadIdx.x / kWave;
  const XF64 cf = scar[0];
  const XF64 cb = scar[1];
  int eap = hs.ein;
  if (cf.m != 0.0) eap = max(eap, cf.e);
  if (cb.m != 0.0) eap = max(eap, cb.e);
  if (eap == kExpZero) eap = 0;  // nothing nonzero reaches this chunk
  const int sh = (hs.ein == kExpZero) ? 0 : hs.ein - eap;  // chunk-local values are all zero then
  T accf = T(ldexp(cf.m, cf.e - eap));
  T accb = T(ldexp(cb.m, cb.e - eap));
  for (int v = 0; v < w; ++v) accf = fma(D.wave, accf, ldx(sf[v], sh));
  for (int v = kNW - 1; v > w; --v) accb = fma(D.wave, accb, ldx(sb[v], sh));
  const T tcf = fma(D.lane_f, accf, ldx(hs.exf, sh));
  const T tcb = fma(D.lane_b, accb, ldx(hs.exb, sh));
  T xf[R];
#pragma unroll
  for (int j = 0; j < R; ++j) xf[j] = ldx(hs.xf[j], sh);
  run_apply<T, R>(xf, L.mul(tcf), L.mul(tcb), L, y);
  return eap;
}

// 1 / y from the hardware reciprocal refined by Newton steps
// (r <- r + r (1 - y r)): two steps in binary64, one in binary32.
__device__ __forceinline__ double recip(double y) {
  double r = __builtin_amdgcn_rcp(y);
  double e = fma(-y, r, 1.0);
  r = fma(r, e, r);
  e = fma(-y, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float recip(float y) {
  float r = __builtin_amdgcn_rcpf(y);
  const float e = fmaf(-y, r, 1.0f);
  return fmaf(r, e, r);
}

// New values q = marg / y on the chunk frame (y is (K in) * 2^-eap, so the new
// vector is q * 2^-eap; zero marginal -> zero scaling).
template <typename T, int R>
__device__ __forceinline__ void update_frame(const T (&mg)[R], const T (&y)[R], T (&q)[R],
                                             bool& bad) {
#pragma unroll
  for (int j = 0; j < R; ++j) {
    q[j] = (mg[j] == T(0)) ? T(0) : mg[j] * recip(y[j]);
    bad |= !isfinite(q[j]);
  }
}

// Chunk aggregates of values given on one frame (exponent e for the whole
// chunk), by weighted reductions instead of scans: the forward aggregate is
// sum_t af(t) lambda^{(255 - t) R}, the backward one sum_t ab(t) lambda^{t R}.
// With `part` non-null the same reduction also sums each thread's `err` (in a
// fixed order) and thread 0 stores the total to part[blockIdx.x].
template <typename T, int R>
__device__ __forceinline__ void publish_frame(const T (&q)[R], int e, const Lam<T>& L,
                                              const FastDec<T>& D, T* sf, T* sb, ChunkAgg* A,
                                              double err = 0.0, double* sred = nullptr,
                                              double* part = nullptr) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  T f, b;
  run_aggs<T, R>(q, L, f, b);
  f *= D.lane_b;
  b *= D.lane_f;
  f = wave_sum(f);
  b = wave_sum(b);
  if (part) err = wave_sum(err);
  if (lane == 0) {
    sf[w] = f;
    sb[w] = b;
    if (part) sred[w] = err;
  }
  __syncthreads();
  publish<T>(D, sf, sb, e, A);
  if (part && threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int v = 0; v < kNW; ++v) t += sred[v];
    part[blockIdx.x] = t;
  }
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

}  // namespace fs1
