// fs1_batch.hip -- many independent FS-1 solves (Algorithm 1) of different
// lengths in the same launches.
//
// Layout (fs1_batch.h): instance b owns chunks [chunk0_b, chunk0_b + nch_b) of
// the padded work arrays; entries past n_b are zero and stay zero (a zero
// marginal gives a zero scaling, and every store writes whole runs).  A
// launch runs one workgroup per chunk record of its list.  A workgroup issues
// all its loads at once (its record tells it where everything is), computes
// its chunk carries from its instance's chunk aggregates, runs the
// extended-range scans of eq. (recursion) with its instance's lambda, and
// takes its instance's stop decision last, before storing anything (all
// workgroups of an instance sum the same error shares with the same tree, so
// they decide alike).  An instance thus executes the same arithmetic whatever
// else is in the batch and wherever it sits.  Iterations are counted on the
// device (iter_base), so a fixed number of iterations can be captured in a
// HIP graph and replayed until every instance has stopped.
#include <climits>

#include "fs1_batch.h"
#include "fs1_device.h"
#include "fs1_frame.h"
#include "fs1_internal.h"
#include "fs1_resident.h"
#include "fs1_xcd.h"

namespace fs1 {

namespace {

constexpr int kCarryItems = 8;                             // chunks per carry thread
constexpr int kPrefetchChunks = kCarryItems * kBlock / 2;  // 1024

enum BMode { B_PSI = 0, B_PHI = 1, B_ERR = 2 };
// which of two buffers a kernel reads
enum BSel { SEL_0 = 0, SEL_FINAL = 1, SEL_NEXT = 2, SEL_CUR = 3 };

// sum over the 64 lanes, the same in every lane: rows by DPP shifts, then the
// four row totals in order
__device__ __forceinline__ S2<double> s2_wave_sum(S2<double> v) {
  v = v.add(v.move<kDppRowShr + 1>());
  v = v.add(v.move<kDppRowShr + 2>());
  v = v.add(v.move<kDppRowShr + 4>());
  v = v.add(v.move<kDppRowShr + 8>()).norm();
  return v.lane(15).add(v.lane(31)).norm().add(v.lane(47).add(v.lane(63)).norm()).norm();
}

// Carries of chunk j of an instance from its chunk aggregates A[0..nch), for
// instances of more than kPrefetchChunks chunks: wave 0 the forward carry,
// wave 1 the backward one.
__device__ __forceinline__ void inst_carries(const ChunkAgg* A, int j, int nch, const Decay* cpow,
                                             XF64* scar) {
  const int w = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (w == 0) {
    XF<double> acc = xzero<double>();
    for (int i = lane; i < j; i += kWave) {
      const XF64 v = A[i].f;
      acc = xadd(acc, xmul(XF<double>{v.m, v.e}, pow_bits(j - 1 - i, cpow)));
    }
    acc = wave_xsum(acc);
    if (lane == 0) scar[0] = to64(acc);
  } else if (w == 1) {
    XF<double> acc = xzero<double>();
    for (int i = j + 1 + lane; i < nch; i += kWave) {
      const XF64 v = A[i].b;
      acc = xadd(acc, xmul(XF<double>{v.m, v.e}, pow_bits(i - j - 1, cpow)));
    }
    acc = wave_xsum(acc);
    if (lane == 0) scar[1] = to64(acc);
  }
  __syncthreads();
}

// Chunk carries of chunk b of an instance from the prefetched aggregates of
// its other chunks (carry_prefetch; threads 0..127 forward, 128..255
// backward): each thread folds its segment in extended range as carry_finish
// does, then each wavefront aligns its lanes' partial sums to their largest
// exponent (an integer maximum) and adds them in binary64 in a fixed tree;
// a wavefront without a term skips that.  Forward carry into scar[0] (waves 0
// and 1), backward into scar[1] (waves 2 and 3).
template <int CMAX>
__device__ __forceinline__ void bcarry_finish(const CarryItems<CMAX>& it, int b,
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
  const bool has = acc.m != 0.0;
  XF64 tot{0.0, kExpZero, 0};
  if (__ballot(has) != 0) {
    const int emax = wave_max(has ? acc.e : kExpZero);
    tot = XF64{wave_sum(has ? ldexp(acc.m, acc.e - emax) : 0.0), emax, 0};
  }
  if (lane == 0) red4[w] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    scar[0] = to64(xnorm(xadd(XF<double>{red4[0].m, red4[0].e}, XF<double>{red4[1].m, red4[1].e})));
    scar[1] = to64(xnorm(xadd(XF<double>{red4[2].m, red4[2].e}, XF<double>{red4[3].m, red4[3].e})));
  }
  __syncthreads();
}

struct BArgs {
  const InstInfo* inst;
  InstState* st;
  const ChunkRef* list;
  const int* iter_base;
  int* ndone;
  int* ring;
  int ring_cap;
  const void* vin[2];     // vector fed to K
  const int* ein[2];
  const void* vown[2];    // own vector of the error term
  const int* eown[2];
  void* vout[2];          // updated vector
  int* eout[2];
  const double* m64;      // padded marginal, binary64
  const float* m32;       // padded marginal, binary32
  const ChunkAgg* A_in;   // chunk aggregates of vin
  ChunkAgg* A_out;        // chunk aggregates of vout (or of vin for k_bpublish)
  double* part;
  int l_local;            // iteration = *iter_base + l_local - l0
  int itr_max;
  int check_every;
  int sel_in, sel_own, sel_out;
};

// psi buffer holding the returned state: the one of the stopping iteration,
// else of itr_max
__device__ __forceinline__ int final_buf(const InstState& s, int itr_max) {
  return (s.stop_iter >= 0) ? (s.stop_iter & 1) : (itr_max & 1);
}

__device__ __forceinline__ int pick(int sel, int l, const InstState& s, int itr_max) {
  switch (sel) {
    case SEL_FINAL: return final_buf(s, itr_max);
    case SEL_NEXT: return (l + 1) & 1;
    case SEL_CUR: return l & 1;
    default: return 0;
  }
}

// Runs of the padded arrays: whole 16-byte vectors where the run length
// allows (entries past n are zero), element by element otherwise.
template <typename T, int R>
__device__ __forceinline__ void bload(const T* p, int64_t base, int64_t lim, T (&x)[R]) {
  if constexpr (R % Vec16<T>::n == 0) {
    load_run_z<T, R>(p, base, x);
  } else {
    load_run<T, R>(p, base, lim, x, T(0));
  }
}
template <typename T, int R>
__device__ __forceinline__ void bstore(T* p, int64_t base, const T (&x)[R]) {
  if constexpr (R % Vec16<T>::n == 0) {
    store_run_z<T, R>(p, base, x);
  } else {
#pragma unroll
    for (int j = 0; j < R; ++j) p[base + j] = x[j];
  }
}

// One half of the Sinkhorn update (Sec. 2) for the chunks of a list:
//   B_PSI: psi^{l+1} = nu / K^T phi^l, error share of (phi^l, psi^l) when checked;
//   B_PHI: stopping test of iteration l, then phi^{l+1} = mu / K psi^{l+1};
//   B_ERR: error share only (finalisation).
template <typename T, int R, int MODE>
__global__ __launch_bounds__(kBlock) void k_bhalf(BArgs a) {
  __shared__ ScanLds<S1<T>, kNW> sh;
  __shared__ double red[kNW];
  __shared__ XF64 scar[2];
  __shared__ XF64 red4[kNW];
  __shared__ int sdec;
  // every XCD a contiguous range of the list: an instance's consecutive
  // chunks read the same published aggregates from one L2
  const ChunkRef r = a.list[xcd_contiguous(blockIdx.x, gridDim.x)];
  const InstInfo& in = a.inst[r.b];
  InstState& st = a.st[r.b];
  const int lane = threadIdx.x & (kWave - 1);
  const int l = (MODE == B_ERR) ? 0 : *a.iter_base + a.l_local - r.l0;
  const bool checked = (l % a.check_every) == 0;
  const bool want_err = (MODE == B_ERR) || (MODE == B_PSI && checked);

  // Every global load is issued here, before any is waited for: the stop
  // flags and error shares (needed last), the instance's chunk aggregates
  // (needed first, for the carries), the chunk's own data.
  int done = 0, fail = 0;
  double shv = 0.0;  // this thread's part of the instance's error (phi-half)
  if constexpr (MODE != B_ERR) {
    if (threadIdx.x == 0) {
      done = st.done;
      fail = st.fail;
    }
    if (MODE == B_PHI && checked)
      for (int i = threadIdx.x; i < r.nch; i += kBlock) shv += a.part[r.chunk0 + i];
  }
  const bool pre = r.nch <= kPrefetchChunks;
  CarryItems<kCarryItems> items;
  if (pre) carry_prefetch<kCarryItems>(a.A_in + r.chunk0, r.j, r.nch, items);
  const int64_t base = r.base + int64_t(threadIdx.x) * R;
  const int64_t run = int64_t(r.c) * kBlock + threadIdx.x;
  const int si = pick(a.sel_in, l, st, a.itr_max);
  T x[R];
  bload<T, R>(static_cast<const T*>(a.vin[si]), base, r.lim, x);
  const int E = a.ein[si][run];
  T own[R];
  int eo = 0;
  if (want_err) {
    const int so = pick(a.sel_own, l, st, a.itr_max);
    bload<T, R>(static_cast<const T*>(a.vown[so]), base, r.lim, own);
    eo = a.eown[so][run];
  }
  // binary64 marginal: the error term, and the update when T = double; the
  // binary32 copy is its rounding, loaded only when the error is not due
  double m64[R];
  T mg[R];
  if (want_err || sizeof(T) == 8) bload<double, R>(a.m64, base, r.lim, m64);
  if constexpr (MODE != B_ERR) {
    if (sizeof(T) == 8 || want_err) {
#pragma unroll
      for (int i = 0; i < R; ++i) mg[i] = T(m64[i]);
    } else {
      bload<T, R>(reinterpret_cast<const T*>(a.m32), base, r.lim, mg);
    }
  }

  // chunk carries first: they need only the aggregates
  if (pre) {
    bcarry_finish<kCarryItems>(items, r.j, in.cpow, red4, scar);
  } else {
    inst_carries(a.A_in + r.chunk0, r.j, r.nch, in.cpow, scar);
  }
  const ScanConsts& k = in.k;
  const Lam<T> L = lam_of<T>(k);
  T af, ab;
  run_aggs<T, R>(x, L, af, ab);
  Dec<T> dec[7];
  lane_decays<T>(k, dec);
  const XF64 cf64 = scar[0], cb64 = scar[1];
  S1<T> cf, cb;
  block_scan<S1<T>, kNW, T>(S1<T>{{af, E}}, S1<T>{{ab, E}}, dec, S1<T>{from64<T>(cf64)},
                            S1<T>{from64<T>(cb64)}, &cf, &cb, nullptr, nullptr, sh);
  // carries moved one step into the run, in extended range
  const S1<T> lcf = cf.shift(step_decay<T>(k)), lcb = cb.shift(step_decay<T>(k));
  int eref = max(local_exponent<T, R>(x, E), max(lcf.v.e, lcb.v.e));
  if (eref == kExpZero) eref = 0;
  T xf[R];
#pragma unroll
  for (int i = 0; i < R; ++i) xf[i] = ldx(x[i], E - eref);
  T y[R];  // (K vin)_i * 2^-eref
  run_apply<T, R>(xf, ldx(lcf.v.m, lcf.v.e - eref), ldx(lcb.v.m, lcb.v.e - eref), L, y);

  if (want_err) {
    // padding is zero and adds nothing
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) s += fabs(ldexp(double(own[i]) * double(y[i]), eo + eref) - m64[i]);
    const double tot = block_sum<kNW>(s, red);
    if (threadIdx.x == 0) a.part[r.c] = tot;
  }
  if constexpr (MODE == B_ERR) return;

  // Stop decision of Algorithm 1, taken before anything is stored.
  // 3: already stopped; 4: l reached itr_max; 2: a scaling became
  // non-finite; 1: err(l) <= tol.
  const bool test = MODE == B_PHI && checked;
  if (test) {
    double e = shv;
    e = wave_sum(e);
    if (lane == 0) red[threadIdx.x / kWave] = e;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int dec = 0;
    if (done) {
      dec = 3;
    } else if (l >= a.itr_max) {
      dec = 4;
    } else if (fail) {
      dec = 2;
    } else if (test) {
      double e = 0.0;
#pragma unroll
      for (int v = 0; v < kNW; ++v) e += red[v];
      if (r.j == 0) {
        st.last_err = e;
        st.last_check = l;
      }
      if (!(e > in.tol)) dec = 1;
    }
    sdec = dec;
  }
  __syncthreads();
  if (sdec) {
    if (r.j == 0 && threadIdx.x == 0 && sdec != 3) {
      if (sdec == 1) st.stop_iter = l;
      if (sdec == 4) st.capped = 1;
      st.done = 1;
      const int pos = atomicAdd(a.ndone, 1);
      if (a.ring) a.ring[pos % a.ring_cap] = r.b;
    }
    return;
  }

  // update: out = marg / (K vin)  (zero marginal -> zero scaling), with the
  // power-of-two part of the run absorbed into its exponent
  T q[R];
  bool bad = false;
  T qm = T(0);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    q[i] = (mg[i] == T(0)) ? T(0) : mg[i] / y[i];
    bad |= !isfinite(q[i]);
    if (isfinite(q[i])) qm = fmax(qm, q[i]);
  }
  int kq = 0;
  if (qm > T(0)) frx(qm, &kq);
#pragma unroll
  for (int i = 0; i < R; ++i) q[i] = ldx(q[i], -kq);
  const int Eo = kq - eref;
  const int sw = pick(a.sel_out, l, st, a.itr_max);
  bstore<T, R>(static_cast<T*>(a.vout[sw]), base, q);
  a.eout[sw][run] = Eo;
  if (bad) {
    atomicOr(&st.fail, 1);
    atomicMin(&st.fail_iter, l);
  }
  T nf, nb;
  run_aggs<T, R>(q, L, nf, nb);
  S1<T> gf, gb;
  block_scan<S1<T>, kNW, T>(S1<T>{{nf, Eo}}, S1<T>{{nb, Eo}}, dec, S1<T>::zero(), S1<T>::zero(),
                            nullptr, nullptr, &gf, &gb, sh);
  if (threadIdx.x == 0) {
    a.A_out[r.c].f = to64(gf.v);
    a.A_out[r.c].b = to64(gb.v);
  }
}

// Chunk aggregates of a stored vector (initial phi; final psi).
template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_bpublish(BArgs a) {
  __shared__ ScanLds<S1<T>, kNW> sh;
  const ChunkRef r = a.list[blockIdx.x];
  const InstInfo& in = a.inst[r.b];
  const int si = pick(a.sel_in, 0, a.st[r.b], a.itr_max);
  const int64_t base = r.base + int64_t(threadIdx.x) * R;
  const int64_t run = int64_t(r.c) * kBlock + threadIdx.x;
  T x[R];
  bload<T, R>(static_cast<const T*>(a.vin[si]), base, r.lim, x);
  const int E = a.ein[si][run];
  const Lam<T> L = lam_of<T>(in.k);
  T af, ab;
  run_aggs<T, R>(x, L, af, ab);
  Dec<T> dec[7];
  lane_decays<T>(in.k, dec);
  S1<T> gf, gb;
  block_scan<S1<T>, kNW, T>(S1<T>{{af, E}}, S1<T>{{ab, E}}, dec, S1<T>::zero(), S1<T>::zero(),
                            nullptr, nullptr, &gf, &gb, sh);
  if (threadIdx.x == 0) {
    a.A_out[r.c].f = to64(gf.v);
    a.A_out[r.c].b = to64(gb.v);
  }
}

// ---------------------------------------------------------------------------
// Transport cost per instance: w1 = h sum_i phi_i (D_i + E_i) with the
// two-state recursions over the final psi.
// ---------------------------------------------------------------------------
template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_bcost_agg(BArgs a, ChunkAgg2* agg2) {
  __shared__ ScanLds<S2<T>, kNW> sh;
  const ChunkRef r = a.list[blockIdx.x];
  const InstInfo& in = a.inst[r.b];
  const int si = final_buf(a.st[r.b], a.itr_max);
  const int64_t base = r.base + int64_t(threadIdx.x) * R;
  const int64_t run = int64_t(r.c) * kBlock + threadIdx.x;
  T x[R];
  bload<T, R>(static_cast<const T*>(a.vin[si]), base, r.lim, x);
  const int E = a.ein[si][run];
  const Lam<T> L = lam_of<T>(in.k);
  T fp, fd, bp, bd;
  run_aggs2<T, R>(x, L, fp, fd, bp, bd);
  Dec<T> dec[7];
  lane_decays<T>(in.k, dec);
  S2<T> gf, gb;
  block_scan<S2<T>, kNW, T>(S2<T>::of(fp, fd, E), S2<T>::of(bp, bd, E), dec, S2<T>::zero(),
                            S2<T>::zero(), nullptr, nullptr, &gf, &gb, sh);
  if (threadIdx.x == 0) {
    ChunkAgg2 o;
    s2_put_fwd(o, gf);
    s2_put_bwd(o, gb);
    agg2[r.c] = o;
  }
}

template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_bcost_apply(BArgs a, const ChunkAgg2* agg2) {
  __shared__ ScanLds<S2<T>, kNW> sh;
  __shared__ double red[kNW];
  __shared__ S2<double> scar[2];
  const ChunkRef r = a.list[blockIdx.x];
  const InstInfo& in = a.inst[r.b];
  const int w = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int si = final_buf(a.st[r.b], a.itr_max);
  const int64_t base = r.base + int64_t(threadIdx.x) * R;
  const int64_t run = int64_t(r.c) * kBlock + threadIdx.x;
  // chunk carries of the two-state recursion: a state moved by D elements
  // with zero input is (p, d) -> lambda^D (p, d + D p)
  const double C = double(kBlock) * R;
  const ChunkAgg2* A2 = agg2 + r.chunk0;
  if (w == 0) {
    S2<double> acc = S2<double>::zero();
    for (int i = lane; i < r.j; i += kWave) {
      const XF<double> p = pow_bits(r.j - 1 - i, in.cpow);
      acc = acc.add(s2_fwd<double>(A2[i]).shift(Dec<double>{p.m, p.e, C * double(r.j - 1 - i)}));
    }
    acc = s2_wave_sum(acc);
    if (lane == 0) scar[0] = acc;
  } else if (w == 1) {
    S2<double> acc = S2<double>::zero();
    for (int i = r.j + 1 + lane; i < r.nch; i += kWave) {
      const XF<double> p = pow_bits(i - r.j - 1, in.cpow);
      acc = acc.add(s2_bwd<double>(A2[i]).shift(Dec<double>{p.m, p.e, C * double(i - r.j - 1)}));
    }
    acc = s2_wave_sum(acc);
    if (lane == 0) scar[1] = acc;
  }
  T x[R];
  bload<T, R>(static_cast<const T*>(a.vin[si]), base, r.lim, x);
  const int E = a.ein[si][run];
  const Lam<T> L = lam_of<T>(in.k);
  T fp, fd, bp, bd;
  run_aggs2<T, R>(x, L, fp, fd, bp, bd);
  Dec<T> dec[7];
  lane_decays<T>(in.k, dec);
  __syncthreads();
  const S2<double> c0 = scar[0], c1 = scar[1];
  S2<T> cf, cb;
  block_scan<S2<T>, kNW, T>(S2<T>::of(fp, fd, E), S2<T>::of(bp, bd, E), dec, s2_cast<T>(c0),
                            s2_cast<T>(c1), &cf, &cb, nullptr, nullptr, sh);
  const S2<T> lcf = cf.shift(step_decay<T>(in.k)), lcb = cb.shift(step_decay<T>(in.k));
  const int eref = cost_frame<T, R>(lcf, lcb, local_exponent<T, R>(x, E), in.k);
  T xf[R];
#pragma unroll
  for (int i = 0; i < R; ++i) xf[i] = ldx(x[i], E - eref);
  T wv[R];
  run_cost<T, R>(xf, ldx(lcf.p.m, lcf.p.e - eref), ldx(lcf.d.m, lcf.d.e - eref),
                 ldx(lcb.p.m, lcb.p.e - eref), ldx(lcb.d.m, lcb.d.e - eref), L, wv);
  T ph[R];
  bload<T, R>(static_cast<const T*>(a.vown[0]), base, r.lim, ph);
  const int ep = a.eown[0][run];
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < R; ++i) s += ldexp(double(ph[i]) * double(wv[i]), ep + eref);
  const double tot = block_sum<kNW>(s, red);
  if (threadIdx.x == 0) a.part[r.c] = tot;
}

// ---------------------------------------------------------------------------
// Set-up and finalisation
// ---------------------------------------------------------------------------
// Pack the caller's marginals chunk-aligned (binary64, plus binary32 copies),
// set phi = psi = 1/n with exponent 0 and zeros past n, and write per-chunk
// masses.
template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_bsetup(BArgs a, double* mu64, double* nu64, float* mu32,
                                                   float* nu32, T* vF, T* vG0, int* eF,
                                                   int* eG0, double* pmu, double* pnu) {
  __shared__ double red[kNW];
  const ChunkRef r = a.list[blockIdx.x];
  const InstInfo& in = a.inst[r.b];
  const int64_t local0 = int64_t(r.j) * kBlock * R + int64_t(threadIdx.x) * R;
  const int64_t base = r.base + int64_t(threadIdx.x) * R;
  const T init = T(1.0 / double(in.n));
  double sm = 0.0, sn = 0.0;
  int bad = 0;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int64_t loc = local0 + i;
    double u = 0.0, v = 0.0;
    if (loc < in.n) {
      u = in.src_mu[loc];
      v = in.src_nu[loc];
      bad |= !(isfinite(u) && u >= 0.0) || !(isfinite(v) && v >= 0.0);
    }
    mu64[base + i] = u;
    nu64[base + i] = v;
    if (mu32) {
      mu32[base + i] = float(u);
      nu32[base + i] = float(v);
    }
    vF[base + i] = (loc < in.n) ? init : T(0);
    vG0[base + i] = (loc < in.n) ? init : T(0);
    sm += u;
    sn += v;
  }
  const int64_t run = int64_t(r.c) * kBlock + threadIdx.x;
  eF[run] = 0;
  eG0[run] = 0;
  const double tm = block_sum<kNW>(sm, red);
  const double tn = block_sum<kNW>(sn, red);
  if (bad) atomicOr(&a.st[r.b].bad_input, 1);
  if (threadIdx.x == 0) {
    pmu[r.c] = tm;
    pnu[r.c] = tn;
  }
}

// Per instance (one thread each): masses positive, finite and equal to
// 1e-10 relative; otherwise the instance is stopped before its first iteration.
__global__ void k_bvalidate(const InstInfo* inst, InstState* st, const double* pmu,
                            const double* pnu, const int* ilist, int count, int* ndone,
                            int* ring, int ring_cap) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int b = ilist ? ilist[t] : t;
  const InstInfo& in = inst[b];
  double sm = 0.0, sn = 0.0;
  for (int i = 0; i < in.nch; ++i) {
    sm += pmu[in.chunk0 + i];
    sn += pnu[in.chunk0 + i];
  }
  InstState& s = st[b];
  s.sum_mu = sm;
  s.sum_nu = sn;
  const bool ok = !s.bad_input && isfinite(sm) && isfinite(sn) && sm > 0.0 && sn > 0.0 &&
                  fabs(sm - sn) <= 1e-10 * sm;
  if (!ok) {
    s.invalid = 1;
    s.done = 1;
    const int pos = atomicAdd(ndone, 1);
    if (ring) ring[pos % ring_cap] = b;
  }
}

__global__ void k_badvance(int* iter_base, int by) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *iter_base += by;
}

// Per instance fixed-order sums of the per-chunk shares.
__global__ void k_bfinal(const InstInfo* inst, InstState* st, const double* perr,
                         const double* pmu, const double* pcost, const int* ilist, int count,
                         InstState* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int b = ilist ? ilist[t] : t;
  const InstInfo& in = inst[b];
  double e = 0.0, m = 0.0, w = 0.0;
  for (int i = 0; i < in.nch; ++i) {
    e += perr[in.chunk0 + i];
    m += pmu[in.chunk0 + i];
    w += pcost[in.chunk0 + i];
  }
  st[b].err = e;
  st[b].mu_err = m;
  st[b].w1 = w * in.h;
  if (out) out[t] = st[b];
}

// Admission: one thread per new instance copies its staged description and
// state into its slot.
__global__ void k_badmit(const InstInfo* sinfo, const InstState* sstate, const int* idx,
                         int count, InstInfo* inst, InstState* st) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  inst[idx[t]] = sinfo[t];
  st[idx[t]] = sstate[t];
}

// ---------------------------------------------------------------------------
// Resident instances (at most 1024 runs): one workgroup runs every iteration
// of its instance with the state in registers (fs1_resident.h), then leaves
// the final state where the finalisation kernels read it: phi in vF, psi in
// the buffer final_buf() names.
// ---------------------------------------------------------------------------
struct BResArgs {
  const InstInfo* inst;
  InstState* st;
  const int* ilist;       // instances of this launch, one per workgroup
  int* ndone;
  int* ring;
  int ring_cap;
  void* vF;
  void* vG[2];
  int* eF;
  int* eG[2];
  const double* mu64;
  const double* nu64;
  const float* mu32;
  const float* nu32;
  int itr_max;
  int check_every;
};

template <typename T, int R, int NT>
__global__ __launch_bounds__(NT) void k_bresident(BResArgs a) {
  __shared__ ResidentLds<T, NT / kWave> S;
  const int b = a.ilist[blockIdx.x];
  const InstInfo& in = a.inst[b];
  InstState& st = a.st[b];
  if (st.done) return;  // stopped at set-up (invalid input); the same value in every thread
  const int t = threadIdx.x;
  const int64_t base = in.base + int64_t(t) * R;
  const int64_t run = int64_t(in.chunk0) * kBlock + t;
  T ph[R], ps[R], mu[R], nu[R];
  res_load<T, R>(static_cast<const T*>(a.vF), base, ph);
  res_load<T, R>(static_cast<const T*>(a.vG[0]), base, ps);
  int eph = a.eF[run];
  int eps = a.eG[0][run];
  if constexpr (sizeof(T) == 8) {
    res_load<T, R>(reinterpret_cast<const T*>(a.mu64), base, mu);
    res_load<T, R>(reinterpret_cast<const T*>(a.nu64), base, nu);
  } else {
    res_load<T, R>(reinterpret_cast<const T*>(a.mu32), base, mu);
    res_load<T, R>(reinterpret_cast<const T*>(a.nu32), base, nu);
  }
  InstState* sp = &st;
  const ResidentEnd end = resident_iterate<T, R, true, NT>(
      ph, eph, ps, eps, mu, nu, a.nu64 + base, in.k, in.tol, a.itr_max, a.check_every, S,
      [&](int l, double err) {
        sp->last_err = err;
        sp->last_check = l;
      });
  const int fb = (end.stop_iter >= 0) ? (end.stop_iter & 1) : (a.itr_max & 1);
  res_store<T, R>(static_cast<T*>(a.vF), base, ph);
  res_store<T, R>(static_cast<T*>(a.vG[fb]), base, ps);
  a.eF[run] = eph;
  a.eG[fb][run] = eps;
  if (t == 0) {
    if (end.fail_iter >= 0) {
      st.fail = 1;
      st.fail_iter = end.fail_iter;
    } else if (end.stop_iter >= 0) {
      st.stop_iter = end.stop_iter;
    } else {
      st.capped = 1;
    }
    st.done = 1;
    const int pos = atomicAdd(a.ndone, 1);
    if (a.ring) a.ring[pos % a.ring_cap] = b;
  }
}

template <typename T, int R, int NT>
hipError_t bresident_t(const BResArgs& a, int count, hipStream_t s) {
  k_bresident<T, R, NT><<<unsigned(count), NT, 0, s>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t bresident(const BResArgs& a, int R, int nt, int count, hipStream_t s) {
  if (nt == 256) {
    switch (R) {
      case 16:
        if constexpr (sizeof(T) == 4) return bresident_t<T, 16, 256>(a, count, s);
        return hipErrorInvalidValue;
      case 8: return bresident_t<T, 8, 256>(a, count, s);
      case 4:
        if constexpr (sizeof(T) == 4) return bresident_t<T, 4, 256>(a, count, s);
        return hipErrorInvalidValue;
      case 1: return bresident_t<T, 1, 256>(a, count, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (nt == 1024) {
    switch (R) {
      case 8: return bresident_t<T, 8, 1024>(a, count, s);
      case 4:
        if constexpr (sizeof(T) == 4) return bresident_t<T, 4, 1024>(a, count, s);
        return hipErrorInvalidValue;
      case 1: return bresident_t<T, 1, 1024>(a, count, s);
      default: return hipErrorInvalidValue;
    }
  }
  return hipErrorInvalidValue;
}

template <typename T, int R>
struct BatchOps {
  static BArgs base(const BatchBufs& z, const BatchGroup& g) {
    BArgs a{};
    a.inst = z.inst;
    a.st = z.st;
    a.list = g.list;
    a.iter_base = z.iter_base;
    a.ndone = z.ndone;
    a.ring = z.ring;
    a.ring_cap = z.ring_cap;
    a.itr_max = z.itr_max;
    a.check_every = z.check_every;
    return a;
  }
  static unsigned grid(const BatchGroup& g) { return unsigned(g.nlist); }
  static void set_phi_in(BArgs& a, const BatchBufs& z) {
    a.vin[0] = a.vin[1] = z.vF;
    a.ein[0] = a.ein[1] = z.eF;
  }
  static void set_psi_in(BArgs& a, const BatchBufs& z, int sel) {
    a.vin[0] = z.vG[0];
    a.vin[1] = z.vG[1];
    a.ein[0] = z.eG[0];
    a.ein[1] = z.eG[1];
    a.sel_in = sel;
  }
  static hipError_t setup(const BatchBufs& z, const BatchGroup& g, hipStream_t s) {
    BArgs a = base(z, g);
    k_bsetup<T, R><<<grid(g), kBlock, 0, s>>>(
        a, z.mu64, z.nu64, static_cast<float*>(z.mu32), static_cast<float*>(z.nu32),
        static_cast<T*>(z.vF), static_cast<T*>(z.vG[0]), z.eF, z.eG[0], z.part, z.part2);
    return hipGetLastError();
  }
  static hipError_t publish_phi(const BatchBufs& z, const BatchGroup& g, hipStream_t s) {
    BArgs a = base(z, g);
    set_phi_in(a, z);
    a.A_out = z.aggF;
    k_bpublish<T, R><<<grid(g), kBlock, 0, s>>>(a);
    return hipGetLastError();
  }
  static hipError_t half(const BatchBufs& z, const BatchGroup& g, bool psi, int l_local,
                         hipStream_t s) {
    BArgs a = base(z, g);
    a.l_local = l_local;
    a.part = z.part;
    if (psi) {
      // psi^{l+1} = nu / K^T phi^l into buffer (l+1)&1; error of (phi^l, psi^l)
      set_phi_in(a, z);
      a.vown[0] = z.vG[0];
      a.vown[1] = z.vG[1];
      a.eown[0] = z.eG[0];
      a.eown[1] = z.eG[1];
      a.sel_own = SEL_CUR;
      a.vout[0] = z.vG[0];
      a.vout[1] = z.vG[1];
      a.eout[0] = z.eG[0];
      a.eout[1] = z.eG[1];
      a.sel_out = SEL_NEXT;
      a.m64 = z.nu64;
      a.m32 = static_cast<const float*>(z.nu32);
      a.A_in = z.aggF;
      a.A_out = z.aggG;
      k_bhalf<T, R, B_PSI><<<grid(g), kBlock, 0, s>>>(a);
    } else {
      // phi^{l+1} = mu / K psi^{l+1}
      set_psi_in(a, z, SEL_NEXT);
      a.vout[0] = a.vout[1] = z.vF;
      a.eout[0] = a.eout[1] = z.eF;
      a.m64 = z.mu64;
      a.m32 = static_cast<const float*>(z.mu32);
      a.A_in = z.aggG;
      a.A_out = z.aggF;
      k_bhalf<T, R, B_PHI><<<grid(g), kBlock, 0, s>>>(a);
    }
    return hipGetLastError();
  }
  static hipError_t finalize(const BatchBufs& z, const BatchGroup& g, hipStream_t s) {
    const unsigned gr = grid(g);
    // aggregates of the final phi (a resident instance leaves them stale; for
    // the others this recomputes what the last phi-half published, bit for bit)
    BArgs p0 = base(z, g);
    set_phi_in(p0, z);
    p0.A_out = z.aggF;
    k_bpublish<T, R><<<gr, kBlock, 0, s>>>(p0);
    // nu side: | psi (K^T phi) - nu |
    BArgs a = base(z, g);
    set_phi_in(a, z);
    a.vown[0] = z.vG[0];
    a.vown[1] = z.vG[1];
    a.eown[0] = z.eG[0];
    a.eown[1] = z.eG[1];
    a.sel_own = SEL_FINAL;
    a.m64 = z.nu64;
    a.A_in = z.aggF;
    a.part = z.part;
    k_bhalf<T, R, B_ERR><<<gr, kBlock, 0, s>>>(a);
    // aggregates of the final psi, then mu side: | phi (K psi) - mu |
    BArgs p = base(z, g);
    set_psi_in(p, z, SEL_FINAL);
    p.A_out = z.aggG;
    k_bpublish<T, R><<<gr, kBlock, 0, s>>>(p);
    BArgs m = base(z, g);
    set_psi_in(m, z, SEL_FINAL);
    m.vown[0] = m.vown[1] = z.vF;
    m.eown[0] = m.eown[1] = z.eF;
    m.m64 = z.mu64;
    m.A_in = z.aggG;
    m.part = z.part2;
    k_bhalf<T, R, B_ERR><<<gr, kBlock, 0, s>>>(m);
    // transport cost
    BArgs w = base(z, g);
    set_psi_in(w, z, SEL_FINAL);
    w.vown[0] = w.vown[1] = z.vF;
    w.eown[0] = w.eown[1] = z.eF;
    w.part = z.part3;
    k_bcost_agg<T, R><<<gr, kBlock, 0, s>>>(w, static_cast<ChunkAgg2*>(z.agg2));
    k_bcost_apply<T, R><<<gr, kBlock, 0, s>>>(w, static_cast<const ChunkAgg2*>(z.agg2));
    return hipGetLastError();
  }
};

template <typename F>
hipError_t bdispatch(int dtype, int R, F&& f) {
  if (dtype == 0) {
    switch (R) {
      case 8: return f(BatchOps<double, 8>{});
      case 1: return f(BatchOps<double, 1>{});
      default: return hipErrorInvalidValue;
    }
  }
  switch (R) {
    case 16: return f(BatchOps<float, 16>{});
    case 8: return f(BatchOps<float, 8>{});
    case 4: return f(BatchOps<float, 4>{});
    case 1: return f(BatchOps<float, 1>{});
    default: return hipErrorInvalidValue;
  }
}

bool group_empty(const BatchGroup& g) { return g.nlist == 0; }

}  // namespace

InstInfo make_inst_info(const double* mu, const double* nu, int64_t base, int64_t n, int chunk0,
                        int R, double h, double eps, double tol, int l0) {
  InstInfo in{};
  const int64_t C = int64_t(kBlock) * R;
  in.src_mu = mu;
  in.src_nu = nu;
  in.base = base;
  in.n = int32_t(n);
  in.nch = int32_t((n + C - 1) / C);
  in.chunk0 = chunk0;
  in.l0 = l0;
  in.h = h;
  in.tol = tol;
  in.k = make_scan_consts(h, eps, R);
  for (int s = 0; s < kInstPow; ++s) in.cpow[s] = make_decay(double(C) * double(1ll << s), h / eps);
  return in;
}

ChunkRef chunk_ref(const InstInfo& in, int b, int j) {
  ChunkRef r{};
  const int64_t C = int64_t(kBlock) * in.k.R;
  r.base = in.base + int64_t(j) * C;
  r.lim = in.base + in.n;
  r.c = in.chunk0 + j;
  r.b = b;
  r.j = j;
  r.nch = in.nch;
  r.chunk0 = in.chunk0;
  r.l0 = in.l0;
  return r;
}

hipError_t launch_batch_setup(const BatchBufs& z, const BatchGroup* groups, int ngroups,
                              const int* ilist, int count, hipStream_t s) {
  for (int i = 0; i < ngroups; ++i) {
    const BatchGroup& g = groups[i];
    if (group_empty(g)) continue;
    const hipError_t e =
        bdispatch(z.dtype, g.R, [&](auto ops) { return decltype(ops)::setup(z, g, s); });
    if (e != hipSuccess) return e;
  }
  if (count > 0)
    k_bvalidate<<<unsigned((count + 255) / 256), 256, 0, s>>>(
        z.inst, z.st, z.part, z.part2, ilist, count, z.ndone, z.ring, z.ring_cap);
  for (int i = 0; i < ngroups; ++i) {
    const BatchGroup& g = groups[i];
    if (group_empty(g)) continue;
    const hipError_t e =
        bdispatch(z.dtype, g.R, [&](auto ops) { return decltype(ops)::publish_phi(z, g, s); });
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_batch_iterations(const BatchBufs& z, const BatchGroup* groups, int ngroups,
                                   int count, hipStream_t s) {
  for (int l = 0; l < count; ++l) {
    for (int psi = 1; psi >= 0; --psi) {
      for (int i = 0; i < ngroups; ++i) {
        const BatchGroup& g = groups[i];
        if (group_empty(g)) continue;
        const hipError_t e = bdispatch(
            z.dtype, g.R, [&](auto ops) { return decltype(ops)::half(z, g, psi != 0, l, s); });
        if (e != hipSuccess) return e;
      }
    }
  }
  k_badvance<<<1, kWave, 0, s>>>(z.iter_base, count);
  return hipGetLastError();
}

hipError_t launch_batch_finalize(const BatchBufs& z, const BatchGroup* groups, int ngroups,
                                 const int* ilist, int count, InstState* out, hipStream_t s) {
  for (int i = 0; i < ngroups; ++i) {
    const BatchGroup& g = groups[i];
    if (group_empty(g)) continue;
    const hipError_t e =
        bdispatch(z.dtype, g.R, [&](auto ops) { return decltype(ops)::finalize(z, g, s); });
    if (e != hipSuccess) return e;
  }
  if (count > 0)
    k_bfinal<<<unsigned((count + 255) / 256), 256, 0, s>>>(z.inst, z.st, z.part, z.part2,
                                                          z.part3, ilist, count, out);
  return hipGetLastError();
}

hipError_t launch_batch_resident(const BatchBufs& z, const ResGroup* groups, int ngroups,
                                 hipStream_t s) {
  BResArgs a{};
  a.inst = z.inst;
  a.st = z.st;
  a.ndone = z.ndone;
  a.ring = z.ring;
  a.ring_cap = z.ring_cap;
  a.vF = z.vF;
  a.vG[0] = z.vG[0];
  a.vG[1] = z.vG[1];
  a.eF = z.eF;
  a.eG[0] = z.eG[0];
  a.eG[1] = z.eG[1];
  a.mu64 = z.mu64;
  a.nu64 = z.nu64;
  a.mu32 = static_cast<const float*>(z.mu32);
  a.nu32 = static_cast<const float*>(z.nu32);
  a.itr_max = z.itr_max;
  a.check_every = z.check_every;
  for (int i = 0; i < ngroups; ++i) {
    const ResGroup& g = groups[i];
    if (g.count <= 0) continue;
    a.ilist = g.ilist;
    const hipError_t e = z.dtype == 0 ? bresident<double>(a, g.R, g.nt, g.count, s)
                                      : bresident<float>(a, g.R, g.nt, g.count, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_batch_admit(const BatchBufs& z, const InstInfo* sinfo, const InstState* sstate,
                              const int* idx, int count, hipStream_t s) {
  if (count > 0)
    k_badmit<<<unsigned((count + 255) / 256), 256, 0, s>>>(sinfo, sstate, idx, count, z.inst,
                                                          z.st);
  return hipGetLastError();
}

}  // namespace fs1
