// fs1_large.hip -- the half-iteration kernel of large grids in the log domain.
//
// Grids of more than 1024 chunks stream every vector through HBM once per
// half: read the vector fed to K, the marginal (and, on checked psi-halves,
// the old psi), write the new vector.  k_large does the whole half in one
// pass over the chunk, on the chunk frame of fs1_frame.h (the in-chunk
// recursions of Sec. 3, eq. (recursion), in plain arithmetic on one power of
// two per chunk).  Its chunk carries come in two parts: those within its group
// of 1024 chunks from k_carry_groups (the scan of the previous half's chunk
// aggregates inside each group), and the groups' part, which every workgroup
// folds itself from the groups' aggregates (a few dozen independent terms;
// the phi-half of a checked iteration also sums the groups' error shares and
// takes Algorithm 1's stop decision here, before any store), so no top-level
// carry launch sits between the halves:
//   * every vector of a chunk shares one exponent, so no per-run exponent is
//     read or written (one pair of ints per chunk instead);
//   * the producer of a vector records, beside that exponent, the largest
//     exponent of the chunk's values, which is the frame its consumer needs:
//     no block-wide maximum at the start of a half;
//   * the update uses the refined reciprocal of fs1_frame.h;
//   * the new vector's chunk aggregates, its frame and the stopping-test
//     error share leave the chunk in one reduction at the end.
// The stop and failure flags are read first: a launch after the stop reads
// nothing else.
// Vectors and marginals are in the tile layout of fs1_tile.h.
#include "fs1_device.h"
#include "fs1_frame.h"
#include "fs1_internal.h"
#include "fs1_tile.h"

namespace fs1 {

namespace {

enum LargeMode { L_PSI = 0, L_PHI = 1 };

struct LargeArgs {
  const void* vin;          // vector fed to K (tile layout)
  const ChunkExp* xin;      // its chunk exponents
  const double* m64;        // marginal, binary64 (error; update when T = double)
  const float* m32;         // marginal, binary32 (update when T = float)
  void* vout;               // new vector
  ChunkExp* xout;
  const void* vown;         // old psi (error term of checked psi-halves)
  const ChunkExp* xown;
  const ChunkAgg* carry;    // carries of vin within each group of 1024 chunks
  const ChunkAgg* gagg;     // the groups' aggregates (the same carry kernel)
  const double* gpart;      // the groups' error shares (phi-half of a checked iteration)
  const void* lanetab;      // LaneDec<T>[64]: the lane-dependent decays
  ChunkAgg* A_out;          // chunk aggregates of vout
  double* part;             // per-chunk error shares
  double* err_hist;
  Ctrl* ctrl;
  double tol;
  int l;
  int check;
  int ngroups;
  CarryFix cfix;
  Decay gpow[10];           // lambda^(1024 C 2^s): moves between groups
};

// The carries of chunk b: its group's carries, folded here from the groups'
// aggregates as independent terms (forward by wave 0, backward by wave 1,
// into sg), and its carries within the group (from the carry kernel), to which
// the group's are added moved to the chunk (after a barrier).
__device__ __forceinline__ void group_fold(const LargeArgs& a, int b, XF64* sg) {
  const int w = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int g = b / kCarryBlock;
  if (w == 0) {
    XF<double> acc = xzero<double>();
    for (int i = lane; i < g; i += kWave) {
      const XF64 v = a.gagg[i].f;
      if (v.m != 0.0) acc = xnorm(xadd(acc, xmul(XF<double>{v.m, v.e}, pow_bits(g - 1 - i, a.gpow))));
    }
    acc = wave_xsum(acc);
    if (lane == 0) sg[0] = to64(acc);
  } else if (w == 1) {
    XF<double> acc = xzero<double>();
    for (int i = g + 1 + lane; i < a.ngroups; i += kWave) {
      const XF64 v = a.gagg[i].b;
      if (v.m != 0.0) acc = xnorm(xadd(acc, xmul(XF<double>{v.m, v.e}, pow_bits(i - g - 1, a.gpow))));
    }
    acc = wave_xsum(acc);
    if (lane == 0) sg[1] = to64(acc);
  }
}

__device__ __forceinline__ ChunkAgg chunk_carry_folded(const LargeArgs& a, int b, const ChunkAgg& lc,
                                                       const XF64* sg) {
  const int64_t g = b / kCarryBlock, j = b - g * kCarryBlock;
  const int64_t gact = min(int64_t(kCarryBlock), a.cfix.nchunks - g * kCarryBlock);
  XF<double> pf = {1.0, 0}, pb = {1.0, 0};
#pragma unroll
  for (int s = 0; s < 11; ++s) {
    if ((j >> s) & 1) pf = {pf.m * a.cfix.cpow[s].m, pf.e + a.cfix.cpow[s].e};
    if (((gact - 1 - j) >> s) & 1) pb = {pb.m * a.cfix.cpow[s].m, pb.e + a.cfix.cpow[s].e};
  }
  const XF<double> f = xadd(XF<double>{lc.f.m, lc.f.e}, xmul(XF<double>{sg[0].m, sg[0].e}, pf));
  const XF<double> bk = xadd(XF<double>{lc.b.m, lc.b.e}, xmul(XF<double>{sg[1].m, sg[1].e}, pb));
  ChunkAgg r;
  r.f = to64(xnorm(f));
  r.b = to64(xnorm(bk));
  return r;
}

// The lane-dependent decays of FastDec (fs1_frame.h), formed once per solve.
template <typename T>
struct LaneDec {
  T lane_f, lane_b, row_f, row_b;
};

template <typename T>
__global__ void k_lane_table(ScanConsts k, LaneDec<T>* tab) {
  const int lane = threadIdx.x & (kWave - 1);
  const FastDec<T> D = make_fast_dec<T>(k, lane);
  tab[lane] = LaneDec<T>{D.lane_f, D.lane_b, D.row_f, D.row_b};
}

template <typename T>
__device__ __forceinline__ FastDec<T> fast_dec_of(const ScanConsts& k, const LaneDec<T>& t) {
  FastDec<T> D;
#pragma unroll
  for (int s = 0; s < 6; ++s) D.step[s] = dec_val<T>(k.lane[s]);
  D.wave = dec_val<T>(k.lane[6]);
  D.lane_f = t.lane_f;
  D.lane_b = t.lane_b;
  D.row_f = t.row_f;
  D.row_b = t.row_b;
  return D;
}

// MU: the lambda step in the (a + x) - mu a form (lambda > 1/2), else fma.
template <typename T, int R, int MODE, bool MU>
__global__ __launch_bounds__(kBlock) void k_large(LargeArgs a, ScanConsts k) {
  __shared__ T sf[kNW];     // wave aggregates of the input (read by every wave)
  __shared__ T sb[kNW];
  __shared__ T pf[kNW];     // wave aggregates of the new vector (separate arrays:
  __shared__ T pb[kNW];     // a wave may publish while another still reads sf, sb)
  __shared__ double sred[kNW];
  __shared__ int smax[kNW];
  __shared__ XF64 sg[2];      // the group's carries
  __shared__ double serr;     // err(l) (phi-half of a checked iteration)
  // stopped by an earlier launch (stopping test met, or a failure seen: the
  // first launch after a failure records the stop)
  if (a.ctrl->done) return;
  if (a.ctrl->fail) {
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctrl->done = 1;
    return;
  }
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int b = blockIdx.x;
  const int64_t run = int64_t(b) * kBlock + threadIdx.x;
  const bool want_err = MODE == L_PSI && a.check;

  const ChunkExp xi = a.xin[b];
  T x[R];
  tile_load<T, R>(static_cast<const T*>(a.vin), run, lane, x);
  T own[R];
  ChunkExp xo{0, kExpZero};
  if (want_err) {
    tile_load<T, R>(static_cast<const T*>(a.vown), run, lane, own);
    xo = a.xown[b];
  }
  double m64[R];
  if (want_err || sizeof(T) == 8) tile_load<double, R>(a.m64, run, lane, m64);
  T mg[R];
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int j = 0; j < R; ++j) mg[j] = T(m64[j]);
  } else {
    tile_load<T, R>(reinterpret_cast<const T*>(a.m32), run, lane, mg);
  }
  const ChunkAgg lc = a.carry[b];
  const LaneDec<T> ld = static_cast<const LaneDec<T>*>(a.lanetab)[lane];
  // the groups' part of the carries, and the stopping-test sum of the groups'
  // error shares (every workgroup adds them in the same order)
  group_fold(a, b, sg);
  if (MODE == L_PHI && a.check && w == 2) {
    double e = 0.0;
    for (int i = lane; i < a.ngroups; i += kWave) e += a.gpart[i];
    e = wave_sum(e);
    if (lane == 0) serr = e;
  }

  const LamC<T, MU> L = lamc_of<T, MU>(k);
  const FastDec<T> D = fast_dec_of<T>(k, ld);
  // the input on its chunk frame (values below 1; an all-zero chunk has no
  // frame and contributes nothing)
  const bool zin = xi.frame == kExpZero;
  T xf[R];
#pragma unroll
  for (int j = 0; j < R; ++j) xf[j] = zin ? T(0) : ldx(x[j], xi.store - xi.frame);
  T f, g;
  run_aggs<T, R>(xf, L, f, g);
  f = wave_fscan<T>(f, D, lane);
  g = wave_bscan<T>(g, D, lane);
  const T exf = dpp<kDppWaveShr1>(f);
  const T exb = dpp<kDppWaveShl1>(g);
  if (lane == kWave - 1) sf[w] = f;
  if (lane == 0) sb[w] = g;
  __syncthreads();

  // Stop decision of Algorithm 1 for iteration l, taken before anything is
  // stored: every workgroup has the same sum.
  if (MODE == L_PHI && a.check) {
    const double e = serr;
    const bool stop = !(e > a.tol);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.ctrl->last_err = e;
      a.ctrl->last_check = a.l;
      if (a.err_hist) a.err_hist[a.l] = e;
      if (stop) {
        a.ctrl->stop_iter = a.l;
        a.ctrl->done = 1;
      }
    }
    if (stop) return;
  }
  const ChunkAgg cg = chunk_carry_folded(a, b, lc, sg);

  // output frame: the larger of the input frame and the carries' exponents
  int eap = zin ? kExpZero : xi.frame;
  if (cg.f.m != 0.0) eap = max(eap, cg.f.e);
  if (cg.b.m != 0.0) eap = max(eap, cg.b.e);
  if (eap == kExpZero) eap = 0;  // nothing nonzero reaches this chunk
  const int sh = zin ? 0 : xi.frame - eap;  // <= 0
  T accf = T(ldexp(cg.f.m, cg.f.e - eap));
  T accb = T(ldexp(cg.b.m, cg.b.e - eap));
  for (int v = 0; v < w; ++v) accf = fma(D.wave, accf, ldx(sf[v], sh));
  for (int v = kNW - 1; v > w; --v) accb = fma(D.wave, accb, ldx(sb[v], sh));
  const T tcf = fma(D.lane_f, accf, ldx(exf, sh));
  const T tcb = fma(D.lane_b, accb, ldx(exb, sh));
#pragma unroll
  for (int j = 0; j < R; ++j) xf[j] = ldx(xf[j], sh);
  T y[R];  // (K in)_j * 2^-eap
  run_apply<T, R>(xf, L.mul(tcf), L.mul(tcb), L, y);

  // share of the stopping error of (phi^l, psi^l) (entries past n are zero)
  double es = 0.0;
  if (want_err) {
#pragma unroll
    for (int j = 0; j < R; ++j)
      es += fabs(ldexp(double(own[j]) * double(y[j]), xo.store + eap) - m64[j]);
  }

  // update: the new vector is q * 2^-eap (zero marginal -> zero scaling)
  T q[R];
  bool bad = false;
  update_frame<T, R>(mg, y, q, bad);
  if (bad) {
    atomicOr(&a.ctrl->fail, 1);
    atomicMin(&a.ctrl->fail_iter, a.l);
  }
  tile_store_nt<T, R>(static_cast<T*>(a.vout), run, lane, q);
  T qm = T(0);
#pragma unroll
  for (int j = 0; j < R; ++j)
    if (isfinite(q[j])) qm = fmax(qm, q[j]);
  int kq = kExpZero;
  if (qm > T(0)) frx(qm, &kq);

  // chunk aggregates of the new vector (weighted reductions on the frame
  // -eap), the largest exponent of its values and the error share
  T nf, nb;
  run_aggs<T, R>(q, L, nf, nb);
  nf = wave_sum(nf * D.lane_b);
  nb = wave_sum(nb * D.lane_f);
  kq = wave_max(kq);
  if (want_err) es = wave_sum(es);
  if (lane == 0) {
    pf[w] = nf;
    pb[w] = nb;
    smax[w] = kq;
    sred[w] = es;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    chunk_aggs<T>(D, pf, pb, -eap, a.A_out[b].f, a.A_out[b].b);
    int km = smax[0];
#pragma unroll
    for (int v = 1; v < kNW; ++v) km = max(km, smax[v]);
    a.xout[b] = ChunkExp{-eap, km == kExpZero ? kExpZero : km - eap};
    if (want_err) {
      double t = 0.0;
#pragma unroll
      for (int v = 0; v < kNW; ++v) t += sred[v];
      a.part[b] = t;
    }
  }
}

// A vector in per-run exponents (tile layout) -> one exponent per chunk:
// every run is rescaled to the chunk's largest exponent, so the values stay
// below 1 and the chunk's frame is that exponent.  With A non-null the
// chunk's aggregates are published too, by the same weighted reductions that
// k_large publishes its new vectors with: a vector handed from one solve to
// the next by the warm start gives the aggregates the continuing solve had,
// bit for bit (the representations differ by a power of two, which every
// step of the reduction carries exactly).
template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_large_pack(T* __restrict__ v,
                                                       const int* __restrict__ ex,
                                                       ChunkExp* __restrict__ xout,
                                                       ChunkAgg* __restrict__ A,
                                                       const void* __restrict__ lanetab,
                                                       ScanConsts k) {
  __shared__ int smax[kNW];
  __shared__ T pf[kNW];
  __shared__ T pb[kNW];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t run = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  T x[R];
  tile_load<T, R>(v, run, lane, x);
  const int e = ex[run];
  const int eb = block_max_int(local_exponent<T, R>(x, e), smax);
#pragma unroll
  for (int j = 0; j < R; ++j) x[j] = (eb == kExpZero) ? T(0) : ldx(x[j], e - eb);
  tile_store<T, R>(v, run, lane, x);
  if (threadIdx.x == 0) xout[blockIdx.x] = ChunkExp{eb == kExpZero ? 0 : eb, eb};
  if (A) {
    const LaneDec<T> ld = static_cast<const LaneDec<T>*>(lanetab)[lane];
    const FastDec<T> D = fast_dec_of<T>(k, ld);
    const Lam<T> L = lam_of<T>(k);
    T nf, nb;
    run_aggs<T, R>(x, L, nf, nb);
    nf = wave_sum(nf * D.lane_b);
    nb = wave_sum(nb * D.lane_f);
    if (lane == 0) {
      pf[w] = nf;
      pb[w] = nb;
    }
    __syncthreads();
    if (threadIdx.x == 0) chunk_aggs<T>(D, pf, pb, eb == kExpZero ? 0 : eb, A[blockIdx.x].f,
                                        A[blockIdx.x].b);
  }
}

// One exponent per chunk -> per-run exponents (for the finalisation).
__global__ __launch_bounds__(kBlock) void k_large_unpack(const ChunkExp* __restrict__ xin,
                                                         int* __restrict__ ex) {
  const int64_t run = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  ex[run] = xin[blockIdx.x].store;
}

template <typename T, int R>
struct LargeOps {
  static hipError_t half(const SolveBufs& b, const ScanConsts& k, const CarryConsts& kc, int l,
                         int check, double tol, bool psi, hipStream_t s, hipEvent_t ev0,
                         hipEvent_t ev1) {
    LargeArgs a{};
    a.cfix = carry_fix_of(kc);
    a.carry = b.carry;
    a.ngroups = int((kc.nchunks + kCarryBlock - 1) / kCarryBlock);
    a.gagg = b.carry + kc.nchunks;
    a.gpart = reinterpret_cast<const double*>(b.carry + kc.nchunks + 2 * a.ngroups);
    for (int s2 = 0; s2 < 10; ++s2)
      a.gpow[s2] = make_decay(double(kCarryBlock) * double(kc.chunk_len) * double(1 << s2),
                              k.c);
    a.lanetab = b.lanetab;
    a.part = b.part;
    a.err_hist = b.err_hist;
    a.tol = tol;
    a.ctrl = b.ctrl;
    a.l = l;
    a.check = check;
    const int cur = l & 1, nxt = (l + 1) & 1;
    hipError_t e;
    if (psi) {
      // carries of phi^l within the groups (skipped once stopped)
      e = launch_carry_groups(1, b.aggF, b.carry, kc, b.ctrl, nullptr, 0, s);
      a.vin = b.vF;
      a.xin = b.xF;
      a.m64 = b.nu;
      a.m32 = static_cast<const float*>(b.nu32);
      a.vout = b.vG[nxt];
      a.xout = b.xG[nxt];
      a.vown = b.vG[cur];
      a.xown = b.xG[cur];
      a.A_out = b.aggG;
    } else {
      // the groups' shares of the stopping error of iteration l, and the
      // carries of psi^{l+1} within the groups; k_large takes the decision
      e = launch_carry_groups(2, b.aggG, b.carry, kc, b.ctrl, b.part, check, s);
      a.vin = b.vG[nxt];
      a.xin = b.xG[nxt];
      a.m64 = b.mu;
      a.m32 = static_cast<const float*>(b.mu32);
      a.vout = b.vF;
      a.xout = b.xF;
      a.A_out = b.aggF;
    }
    if (e != hipSuccess) return e;
    if (ev0) (void)hipEventRecord(ev0, s);
    const unsigned g = unsigned(b.nchunks);
    if (k.use_mu) {
      if (psi)
        k_large<T, R, L_PSI, true><<<g, kBlock, 0, s>>>(a, k);
      else
        k_large<T, R, L_PHI, true><<<g, kBlock, 0, s>>>(a, k);
    } else {
      if (psi)
        k_large<T, R, L_PSI, false><<<g, kBlock, 0, s>>>(a, k);
      else
        k_large<T, R, L_PHI, false><<<g, kBlock, 0, s>>>(a, k);
    }
    if (ev1) (void)hipEventRecord(ev1, s);
    return hipGetLastError();
  }
  static hipError_t pack(const SolveBufs& b, const ScanConsts& k, hipStream_t s) {
    k_lane_table<T><<<1, kWave, 0, s>>>(k, static_cast<LaneDec<T>*>(b.lanetab));
    k_large_pack<T, R><<<unsigned(b.nchunks), kBlock, 0, s>>>(static_cast<T*>(b.vF), b.eF, b.xF,
                                                              b.aggF, b.lanetab, k);
    k_large_pack<T, R><<<unsigned(b.nchunks), kBlock, 0, s>>>(
        static_cast<T*>(b.vG[0]), b.eG[0], b.xG[0], nullptr, b.lanetab, k);
    return hipGetLastError();
  }
};

bool large_frame_fits(int dtype, int R, double c) {
  // the chunk frame spans lambda^(chunk length) = 2^-(256 R c log2 e)
  const double span = double(kBlock) * double(R) * c * kLog2E;
  return span <= (dtype == 0 ? 900.0 : 80.0);
}

template <typename F>
hipError_t large_dispatch(const SolveBufs& b, F&& f) {
  if (b.dtype == 0) return b.R == 16 ? f(LargeOps<double, 16>{}) : f(LargeOps<double, 8>{});
  return b.R == 8 ? f(LargeOps<float, 8>{}) : f(LargeOps<float, 16>{});
}

}  // namespace

bool usable_large(const SolveBufs& b, double c) {
  if (!b.absorb || !(b.R == 8 || b.R == 16)) return false;
  return large_frame_fits(b.dtype, b.R, c);
}

hipError_t launch_large_pack(const SolveBufs& b, const ScanConsts& k, hipStream_t s) {
  return large_dispatch(b, [&](auto ops) { return decltype(ops)::pack(b, k, s); });
}

hipError_t launch_large_unpack(const SolveBufs& b, int gbuf, hipStream_t s) {
  k_large_unpack<<<unsigned(b.nchunks), kBlock, 0, s>>>(b.xF, b.eF);
  k_large_unpack<<<unsigned(b.nchunks), kBlock, 0, s>>>(b.xG[gbuf], b.eG[gbuf]);
  return hipGetLastError();
}

hipError_t launch_large_half(const SolveBufs& b, const ScanConsts& k, const CarryConsts& kc,
                             int l, int check, double tol, bool psi, hipStream_t s,
                             hipEvent_t ev0, hipEvent_t ev1) {
  return large_dispatch(b, [&](auto ops) {
    return decltype(ops)::half(b, k, kc, l, check, tol, psi, s, ev0, ev1);
  });
}

}  // namespace fs1
