// fs1_fused.hip -- one kernel launch per half-iteration of Algorithm 1.
//
// Each workgroup owns one chunk.  A launch of k_fused
//   * recomputes its chunk carries from the chunk aggregates the previous
//     launch published (the whole workgroup, as independent terms weighted by
//     the per-solve table of decays lambda^(C d), in extended range), while
//     the chunk's own data is still arriving,
//   * runs the in-chunk recursions of Sec. 3, eq. (recursion) on a per-chunk
//     frame (fs1_frame.h),
//   * writes its share of the stopping error (psi-half of checked iterations),
//   * takes the stop decision of Algorithm 1 for the current iteration (every
//     workgroup sums the previous launch's per-chunk error shares in the same
//     fixed order, so all of them decide alike) -- last, so that its loads are
//     hidden behind the arithmetic -- and unless it stops,
//   * applies the Sinkhorn update of Sec. 2 (psi = nu / K^T phi, or
//     phi = mu / K psi), stores it and publishes the chunk aggregates of the
//     new vector for the next launch.
// Launches after the stop still do the arithmetic but store nothing.  Kernel
// boundaries order everything: no inter-workgroup waiting.  The vectors and
// marginals are in the tile layout of fs1_tile.h throughout the fused
// iterations (converted in place before the first launch and after the last).
#include "fs1_device.h"
#include "fs1_frame.h"
#include "fs1_internal.h"
#include "fs1_tile.h"

namespace fs1 {

namespace {

constexpr int kCarryMax = 8;                      // chunks per carry thread
constexpr int kMaxFusedChunks = kCarryMax * kBlock / 2;  // 1024
constexpr double kFrameLog2Span64 = 900.0;
constexpr double kFrameLog2Span32 = 80.0;

enum FusedMode { F_PSI = 0, F_PHI = 1, F_ERR = 2 };


struct FusedArgs {
  const void* vin;        // vector fed to K (values, per-run exponents)
  const int* ein;
  const double* m64;      // marginal, binary64 (error; update when T = double)
  const float* m32;       // marginal, binary32 (update when T = float)
  void* vout;             // updated vector
  int* eout;
  const void* vown;       // own vector of the error term
  const int* eown;
  const ChunkAgg* A_in;   // chunk aggregates of vin
  ChunkAgg* A_out;        // chunk aggregates of vout
  double* part;           // per-chunk error shares
  Ctrl* ctrl;
  double* err_hist;
  int64_t n;
  int nchunks;
  int l;
  int check;
  double tol;
  const XF64* dtab;       // lambda^(chunk length * d), d < nchunks
};

template <typename T, int R, int MODE>
__global__ __launch_bounds__(kBlock) void k_fused(FusedArgs a, ScanConsts k) {
  __shared__ T sf[kNW];
  __shared__ T sb[kNW];
  __shared__ int smax[kNW];
  __shared__ double red[kNW];
  __shared__ XF64 scar[2];
  __shared__ XF64 red4[kNW];
  __shared__ int sdec;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t run = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const bool want_err = (MODE == F_ERR) || (MODE == F_PSI && a.check);

  // Every global load of the launch is issued here, before any use, oldest
  // first: the stop flags and error shares (needed last), the chunk
  // aggregates (needed first, for the carries), the chunk's own data.  The
  // flags were written by earlier launches (kernel boundaries order them).
  int done = 0, fail = 0;
  double sh4[kMaxFusedChunks / kBlock];  // this thread's error shares, chunks tid + 256 i
  if constexpr (MODE != F_ERR) {
    if (threadIdx.x == 0) {
      done = a.ctrl->done;
      fail = a.ctrl->fail;
    }
    if (MODE == F_PHI && a.check) {
#pragma unroll
      for (int i = 0; i < kMaxFusedChunks / kBlock; ++i) {
        const int c = int(threadIdx.x) + i * kBlock;
        sh4[i] = c < a.nchunks ? a.part[c] : 0.0;
      }
    }
  }
  CarryItems<kCarryMax> items;
  carry_prefetch<kCarryMax>(a.A_in, blockIdx.x, a.nchunks, items);
  CarryDecays<kCarryMax> decs;
  carry_table<kCarryMax>(a.dtab, blockIdx.x, items, decs);
  // (every vector is allocated to whole chunks and zero past n, in the tile
  // layout of fs1_tile.h: plain vector loads)
  T x[R];
  tile_load<T, R>(static_cast<const T*>(a.vin), run, lane, x);
  const int ex = a.ein[run];
  T own[R];
  double m64[R];
  int eo = 0;
  if constexpr (MODE != F_PHI) {
    // issued on every psi-half (from the input vector where no error is due:
    // the same lines as x), so that the number of loads behind the chunk
    // aggregates does not depend on the check and the carries below wait for
    // the aggregates only
    const T* vo = static_cast<const T*>(want_err ? a.vown : a.vin);
    tile_load<T, R>(vo, run, lane, own);
    eo = (want_err ? a.eown : a.ein)[run];
  }
  // (binary32: on every psi-half, used where the error is due, for the same
  // reason as the own vector)
  if (MODE != F_PHI || sizeof(T) == 8) tile_load<double, R>(a.m64, run, lane, m64);
  T mg[R];
  if constexpr (MODE != F_ERR) {
    if constexpr (sizeof(T) == 8) {
#pragma unroll
      for (int j = 0; j < R; ++j) mg[j] = T(m64[j]);
    } else {
      tile_load<T, R>(reinterpret_cast<const T*>(a.m32), run, lane, mg);
    }
  }
  // every load is in flight before the carry arithmetic starts: keep the
  // instruction scheduler from moving that arithmetic above the data loads
  __builtin_amdgcn_sched_barrier(0);

  // chunk carries first: they need only the aggregates, so this work runs
  // while the chunk's own data is still arriving
  carry_finish_tab<kCarryMax>(items, decs, red4, scar);
  const Lam<T> L = lam_of<T>(k);
  const FastDec<T> D = make_fast_dec<T>(k, lane);
  HalfState<T, R> hs;
  local_scan<T, R>(x, ex, L, D, sf, sb, smax, hs);
  T y[R];
  const int eap = frame_apply<T, R>(L, D, sf, sb, scar, hs, y);

  // this thread's share of the stopping error (entries past n are zero and
  // add nothing); reduced with the chunk aggregates at the end
  double es = 0.0;
  if (want_err) {
#pragma unroll
    for (int j = 0; j < R; ++j) es += fabs(ldexp(double(own[j]) * double(y[j]), eo + eap) - m64[j]);
  }
  if constexpr (MODE == F_ERR) {
    const double tot = block_sum<kNW>(es, red);
    if (threadIdx.x == 0) a.part[blockIdx.x] = tot;
    return;
  }

  // Stop decision of Algorithm 1, taken before anything is stored.
  // 3: already stopped; 2: a scaling became non-finite; 1: err(l) <= tol.
  // Every workgroup sums the same shares with the same tree, so all decide
  // alike.
  if (MODE == F_PHI && a.check) {
    double e = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxFusedChunks / kBlock; ++i) e += sh4[i];
    e = wave_sum(e);
    if (lane == 0) red[threadIdx.x / kWave] = e;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int dec = 0;
    if (done) {
      dec = 3;
    } else if (fail) {
      dec = 2;
    } else if (MODE == F_PHI && a.check) {
      double e = 0.0;
#pragma unroll
      for (int v = 0; v < kNW; ++v) e += red[v];
      if (blockIdx.x == 0) {
        a.ctrl->last_err = e;
        a.ctrl->last_check = a.l;
        if (a.err_hist) a.err_hist[a.l] = e;
      }
      if (!(e > a.tol)) dec = 1;
    }
    sdec = dec;
  }
  __syncthreads();
  if (sdec) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && sdec != 3) {
      if (sdec == 1) a.ctrl->stop_iter = a.l;
      a.ctrl->done = 1;
    }
    return;
  }

  // the new vector is q * 2^-eap: every run of the chunk gets exponent -eap
  T q[R];
  bool bad = false;
  update_frame<T, R>(mg, y, q, bad);
  if (bad) {
    atomicOr(&a.ctrl->fail, 1);
    atomicMin(&a.ctrl->fail_iter, a.l);
  }
  tile_store_nt<T, R>(static_cast<T*>(a.vout), run, lane, q);
  __builtin_nontemporal_store(-eap, &a.eout[run]);
  // aggregates of the new vector for the next launch, and the error share
  publish_frame<T, R>(q, -eap, L, D, sf, sb, a.A_out, es, red, want_err ? a.part : nullptr);
}

// Chunk aggregates of a stored vector (initial or warm-start state), by the
// same weighted reductions that k_fused publishes with (publish_frame), on the
// chunk's frame: the values of a vector handed from one solve to the next by
// the warm start give the aggregates the continuing solve had, bit for bit
// (the two representations differ by a power of two per run, which every
// step of the reduction carries exactly).
template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_publish(const T* __restrict__ v,
                                                    const int* __restrict__ ex, int64_t n,
                                                    ScanConsts k, ChunkAgg* A) {
  __shared__ T sf[kNW];
  __shared__ T sb[kNW];
  __shared__ int smax[kNW];
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t run = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  T x[R];
  load_run_z<T, R>(v, run * R, x);
  const int e = ex[run];
  const int eb = block_max_int(local_exponent<T, R>(x, e), smax);
  T xf[R];
#pragma unroll
  for (int j = 0; j < R; ++j) xf[j] = (eb == kExpZero) ? T(0) : ldx(x[j], e - eb);
  const Lam<T> L = lam_of<T>(k);
  const FastDec<T> D = make_fast_dec<T>(k, lane);
  publish_frame<T, R>(xf, eb == kExpZero ? 0 : eb, L, D, sf, sb, A);
}

template <typename T, int R>
struct FusedOps {
  static FusedArgs base_args(const SolveBufs& b, const ScanConsts& k, double tol) {
    FusedArgs a{};
    a.part = b.part;
    a.ctrl = b.ctrl;
    a.err_hist = b.err_hist;
    a.n = b.n;
    a.nchunks = int(b.nchunks);
    a.tol = tol;
    a.dtab = b.dtab;
    return a;
  }
  static hipError_t half(const SolveBufs& b, const ScanConsts& k, int l, int check, double tol,
                         bool psi, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    FusedArgs a = base_args(b, k, tol);
    a.l = l;
    a.check = check;
    const int cur = l & 1, nxt = (l + 1) & 1;
    if (psi) {
      a.vin = b.vF;
      a.ein = b.eF;
      a.m64 = b.nu;
      a.m32 = static_cast<const float*>(b.nu32);
      a.vout = b.vG[nxt];
      a.eout = b.eG[nxt];
      a.vown = b.vG[cur];
      a.eown = b.eG[cur];
      a.A_in = b.aggF;
      a.A_out = b.aggG;
    } else {
      a.vin = b.vG[nxt];
      a.ein = b.eG[nxt];
      a.m64 = b.mu;
      a.m32 = static_cast<const float*>(b.mu32);
      a.vout = b.vF;
      a.eout = b.eF;
      a.A_in = b.aggG;
      a.A_out = b.aggF;
    }
    if (ev0) (void)hipEventRecord(ev0, s);
    if (psi)
      k_fused<T, R, F_PSI><<<unsigned(b.nchunks), kBlock, 0, s>>>(a, k);
    else
      k_fused<T, R, F_PHI><<<unsigned(b.nchunks), kBlock, 0, s>>>(a, k);
    if (ev1) (void)hipEventRecord(ev1, s);
    return hipGetLastError();
  }
  static hipError_t publish_state(const SolveBufs& b, const ScanConsts& k, const void* v,
                                   const int* ex, ChunkAgg* A, hipStream_t s) {
    k_publish<T, R><<<unsigned(b.nchunks), kBlock, 0, s>>>(static_cast<const T*>(v), ex, b.n, k, A);
    return hipGetLastError();
  }
};

}  // namespace

namespace {
bool frame_fits(int dtype, int R, double c) {
  const double span = double(kBlock) * double(R) * c * kLog2E;
  return span <= (dtype == 0 ? kFrameLog2Span64 : kFrameLog2Span32);
}
}  // namespace

int fused_run_length(int dtype, double c, int64_t n) {
  // Two workgroups per compute unit run at once, so up to 512 chunks form one
  // wave of the grid; within that the run length with more chunks wins (N =
  // 2^20 in binary32: 15.3 us per iteration with 512 chunks, 15.8 with 256).
  // Past one wave more chunks lose, because every workgroup folds all chunk
  // aggregates into its carries (binary64 at N = 2^20: 20.2 us per iteration
  // with 512 chunks, 25.7 with 1024), so the longest run that fits is taken.
  // A run length is usable only where its chunk frame fits the working
  // precision.
  constexpr int64_t kOneWave = 512;
  const int cand[2] = {dtype == 0 ? 8 : 16, dtype == 0 ? 4 : 8};
  int best = 0;
  int64_t best_n = 0;
  for (int R : cand) {
    const int64_t nch = (n + int64_t(kBlock) * R - 1) / (int64_t(kBlock) * R);
    if (nch <= kOneWave && nch > best_n && frame_fits(dtype, R, c)) {
      best = R;
      best_n = nch;
    }
  }
  if (best) return best;
  for (int R : cand) {
    const int64_t nch = (n + int64_t(kBlock) * R - 1) / (int64_t(kBlock) * R);
    if (nch <= kMaxFusedChunks && frame_fits(dtype, R, c)) return R;
  }
  return 0;
}

bool usable_fused(const SolveBufs& b, double c) {
  if (!b.absorb) return false;  // the plain domain keeps the paper's unscaled arithmetic
  if (b.nchunks > kMaxFusedChunks || !frame_fits(b.dtype, b.R, c)) return false;
  return b.dtype == 0 ? (b.R == 4 || b.R == 8) : (b.R == 8 || b.R == 16);
}

template <typename F>
hipError_t fused_dispatch(const SolveBufs& b, F&& f) {
  if (b.dtype == 0) return b.R == 4 ? f(FusedOps<double, 4>{}) : f(FusedOps<double, 8>{});
  return b.R == 8 ? f(FusedOps<float, 8>{}) : f(FusedOps<float, 16>{});
}

namespace {
struct DecayTableArgs {
  XF64* tab;
  int n;
  Decay cpow[20];  // lambda^(chunk length * 2^s)
};

__global__ __launch_bounds__(kBlock) void k_decay_table(DecayTableArgs a) {
  const int d = int(blockIdx.x) * kBlock + int(threadIdx.x);
  if (d < a.n) a.tab[d] = to64(xnorm(pow_bits(d, a.cpow)));
}
}  // namespace

hipError_t launch_decay_table(const SolveBufs& b, const ScanConsts& k, hipStream_t s) {
  DecayTableArgs a{};
  a.tab = b.dtab;
  a.n = int(b.nchunks);
  for (int i = 0; i < 20; ++i)
    a.cpow[i] = make_decay(double(kBlock) * double(b.R) * double(1ll << i), k.c);
  k_decay_table<<<unsigned((b.nchunks + kBlock - 1) / kBlock), kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_fused_init(const SolveBufs& b, const ScanConsts& k, hipStream_t s) {
  return fused_dispatch(
      b, [&](auto ops) { return decltype(ops)::publish_state(b, k, b.vF, b.eF, b.aggF, s); });
}

hipError_t launch_fused_half(const SolveBufs& b, const ScanConsts& k, int l, int check,
                             double tol, bool psi, hipStream_t s, hipEvent_t ev0,
                             hipEvent_t ev1) {
  return fused_dispatch(
      b, [&](auto ops) { return decltype(ops)::half(b, k, l, check, tol, psi, s, ev0, ev1); });
}

}  // namespace fs1
