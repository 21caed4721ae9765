// fs1_2d.hip -- FS-1 on grids (Sec. 4, Algorithm 2): n1 x n2, and up to four axes.
//
// Layout: column-major, entry (i, j) at i + n1 j; i runs along the first axis
// (spacing h1, lambda1 = e^{-h1/eps}), j along the second (h2, lambda2).  The
// kernel is the Kronecker product K = K2 (x) K1 (the block matrix of Sec. 4),
// so K x is the 1-D recursions of Sec. 3 along every column (first axis) and
// then the recursions of eq. (2d recursion) across the columns, which are the
// same 1-D recursions along every row (second axis).  Each pass runs one
// workgroup per line: a column is contiguous, a row is strided by n1.  A line
// of up to 1024 R entries is held by one workgroup (thread t owns the line
// positions [t R, t R + R)) and scanned with the extended-range block scan of
// the 1-D path; there are no chunk carries.  On strided axes with short lines
// a workgroup takes 16 adjacent lines instead, so that its loads read whole
// cache lines, and every XCD takes a contiguous range of lines.
//
// The same passes serve grids of up to four axes (Sec. 4 says the
// construction extends to higher dimensions): axis a of an n_0 x ... grid
// (first axis fastest) has lines whose entries lie s_a = n_0 ... n_{a-1}
// apart, and K = K_{D-1} (x) ... (x) K_0 is one pass per axis.
//
// The transport cost splits along the axes: with C_a the 1-D kernel
// lambda_a^{|d|} |d| of axis a,
//   W = h1 <phi, (K2 (x) C1) psi> + h2 <phi, (C2 (x) K1) psi>
// (on D axes, one such term per axis), and C_a x is the two-state recursion
// of the 1-D cost.
//
// Plain domain (Algorithm 2 as written): scalings are plain numbers, and a
// non-finite or zero-denominator scaling ends the solve.
//
// Log domain (the stabilised form, Sec. 3 remark carried to Algorithm 2): every
// scaling entry is a mantissa and an int32 binary exponent, so its logarithm
// is ln m + e ln 2 and no product underflows however small eps is.  A pass
// takes the largest exponent of each thread's R entries as the exponent of its
// run and scans in extended range, as the 1-D log domain does; its output is
// a mantissa per entry beside the run's frame exponent, and the update
// normalises every new scaling entry to its own exponent.
#include <cmath>
#include <cstring>

#include "fs1_device.h"
#include "fs1_host.h"
#include "fs1_internal.h"
#include "fs1_xcd.h"

namespace fs1 {

namespace {

constexpr int kR2 = 8;  // entries per thread of a line
constexpr int kGroup = 16;  // adjacent lines per workgroup on strided axes (128 B in binary64)
constexpr int kGroupLong = 4;  // the same for lines of 33 .. 256 runs
constexpr int kContThreads = 256;  // workgroup of the grouped short contiguous lines

enum LineMode { L_APPLY = 0, L_COST = 1, L_UPDATE = 2, L_ERR = 3, L_DOT = 4, L_COSTDOT = 5 };

struct LineArgs {
  const void* x;        // input of the pass
  void* y;              // output (APPLY, COST, UPDATE)
  const void* own;      // ERR, DOT, COSTDOT, checked UPDATE: the vector the product multiplies
  const int* xe;        // log domain: binary exponents of x, y and own (one per entry)
  int* ye;
  const int* owne;
  const double* m64;    // marginal, binary64 (UPDATE with T = double; ERR; checked UPDATE)
  const float* m32;     // marginal, binary32 (UPDATE with T = float)
  double* part;         // per-line shares (ERR, DOT, COSTDOT, checked UPDATE)
  Ctrl* ctrl;
  int64_t inner;        // line L's first entry: (L mod inner) + (L div inner) outer
  int64_t outer;
  int64_t stride;       // offset between consecutive entries of a line
  int len;              // entries per line
  int l;                // iteration (failure record)
  int check;            // UPDATE: also the error share of Algorithm 2's stopping test
  int guard;            // return at once once the solve has stopped or failed
  // decide: first take the stop decision of iteration l from the nparts
  // shares in part (every workgroup sums them in the same order; workgroup 0
  // records it) and return at once when it stops
  int decide;
  int nparts;
  double tol;
  double* err_hist;
};

// The scan of block_scan (same contract: cf the forward state just before a
// thread's run, cb the inclusive backward state just after it) for GL lines
// per workgroup, line gi held by the threads gi + GL q (q < NQ, in line
// order): Hillis-Steele steps over q in LDS, the step of distance 2^s
// weighted by dec[s] = lambda^(R 2^s).
template <typename S, int NQ, int GL>
struct GroupLds {
  S f[NQ][GL];
  S b[NQ][GL];
};

template <typename S, int NQ, int GL, typename T>
__device__ __forceinline__ void group_scan(S tf, S tb, const Dec<T>* dec, int gi, int q, S* cf,
                                           S* cb, GroupLds<S, NQ, GL>& g) {
  S f = tf.norm();
  S b = tb.norm();
#pragma unroll
  for (int s = 0; (1 << s) < NQ; ++s) {
    const int d = 1 << s;
    g.f[q][gi] = f;
    g.b[q][gi] = b;
    __syncthreads();
    if (q >= d) f = f.add(g.f[q - d][gi].shift(dec[s])).norm();
    if (q + d < NQ) b = b.add(g.b[q + d][gi].shift(dec[s])).norm();
    __syncthreads();
  }
  g.f[q][gi] = f;
  g.b[q][gi] = b;
  __syncthreads();
  *cf = q > 0 ? g.f[q - 1][gi] : S::zero();
  *cb = q + 1 < NQ ? g.b[q + 1][gi] : S::zero();
  __syncthreads();
}

// SC: the log domain (mantissas with per-entry exponents xe, ye, owne).
// GL: lines per workgroup.  GL = 1: one line per workgroup, thread t holding
// its positions [t R, t R + R).  GL > 1 (strided axes whose line starts are a
// multiple of GL entries apart): GL adjacent lines, line gi held by the
// threads gi + GL q, so that the GL lanes of one load read GL adjacent
// entries (kGroup = 16: one whole cache line in binary64; kGroupLong = 4 for
// lines of up to 256 runs, a quarter line, the rest of which the next groups
// on the same XCD read from its L2).  CONT (short contiguous lines, the first
// axis): GL lines one after another, line gi held by the threads gi NQ + q,
// so that a workgroup streams GL lines instead of one.
template <typename T, int R, int NT, int MODE, bool SC, int GL = 1, bool CONT = false>
__global__ __launch_bounds__(NT) void k_line(LineArgs a, ScanConsts k) {
  constexpr int NW = NT / kWave;
  constexpr int NQ = NT / GL;            // threads per line
  constexpr int NQG = GL == 1 ? 1 : NQ;  // size of the grouped scan's LDS
  constexpr bool kCostMode = MODE == L_COST || MODE == L_COSTDOT;
  __shared__ ScanLds<S1<T>, NW> sh;
  __shared__ ScanLds<S2<T>, NW> sh2;
  __shared__ GroupLds<S1<T>, kCostMode ? 1 : NQG, GL> gsh;
  __shared__ GroupLds<S2<T>, kCostMode ? NQG : 1, GL> gsh2;
  __shared__ double red[NW];
  __shared__ double gred[GL == 1 ? 1 : NT];
  __shared__ int sstop;
  if (a.guard && (a.ctrl->done || a.ctrl->fail)) return;  // the same value in every thread
  if (a.decide) {
    double s = 0.0;
    for (int i = threadIdx.x; i < a.nparts; i += NT) s += a.part[i];
    const double tot = block_sum<NW>(s, red);  // valid in thread 0
    if (threadIdx.x == 0) {
      sstop = !(tot > a.tol);
      if (blockIdx.x == 0) {
        a.ctrl->last_err = tot;
        a.ctrl->last_check = a.l;
        if (a.err_hist) a.err_hist[a.l] = tot;
        if (sstop) {
          a.ctrl->stop_iter = a.l;
          a.ctrl->done = 1;
        }
      }
    }
    __syncthreads();
    if (sstop) return;
  }
  // every XCD a contiguous range of lines: the adjacent lines of a strided
  // axis, whose entries share cache lines, run in one L2
  // line within the workgroup, and thread of its line
  const int gi = GL == 1 ? 0 : (CONT ? int(threadIdx.x) / NQ : int(threadIdx.x) % GL);
  const int tq = GL == 1 ? int(threadIdx.x) : (CONT ? int(threadIdx.x) % NQ : int(threadIdx.x) / GL);
  const uint32_t line = xcd_contiguous(blockIdx.x, gridDim.x) * GL + uint32_t(gi);
  const uint32_t inner = uint32_t(a.inner);
  const int64_t base = int64_t(line % inner) + int64_t(line / inner) * a.outer;
  const int p0 = tq * R;
  const T* xin = static_cast<const T*>(a.x);
  T x[R];
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = (p0 + r < a.len) ? xin[base + int64_t(p0 + r) * a.stride] : T(0);
  // log domain: the run's exponent E is the largest of its entries' (zeros
  // excluded), and the run's values are the mantissas moved to it
  int E = 0;
  if constexpr (SC) {
    int xe[R];
    int emax = kExpZero;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      xe[r] = (p0 + r < a.len) ? a.xe[base + int64_t(p0 + r) * a.stride] : 0;
      if (x[r] != T(0)) emax = max(emax, xe[r]);
    }
    E = (emax == kExpZero) ? 0 : emax;
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = (x[r] == T(0)) ? T(0) : ldx(x[r], xe[r] - E);
  }
  const Lam<T> L = lam_of<T>(k);
  Dec<T> dec[7];
  lane_decays<T>(k, dec);
  const Dec<T> step = step_decay<T>(k);
  T y[R];
  int eref = 0;
  if constexpr (MODE == L_COST || MODE == L_COSTDOT) {
    // (C x)_i = sum_k lambda^{|i-k|} |i-k| x_k: the two-state recursion
    T fp, fd, bp, bd;
    run_aggs2<T, R>(x, L, fp, fd, bp, bd);
    S2<T> cf, cb;
    if constexpr (GL == 1) {
      block_scan<S2<T>, NW, T>(S2<T>::of(fp, fd, E), S2<T>::of(bp, bd, E), dec, S2<T>::zero(),
                               S2<T>::zero(), &cf, &cb, nullptr, nullptr, sh2);
    } else {
      group_scan<S2<T>, NQ, GL, T>(S2<T>::of(fp, fd, E), S2<T>::of(bp, bd, E), dec, gi, tq,
                                   &cf, &cb, gsh2);
    }
    const S2<T> lcf = cf.shift(step), lcb = cb.shift(step);
    eref = cost_frame<T, R>(lcf, lcb, local_exponent<T, R>(x, E), k);
    T xf[R];
#pragma unroll
    for (int r = 0; r < R; ++r) xf[r] = ldx(x[r], E - eref);
    run_cost<T, R>(xf, ldx(lcf.p.m, lcf.p.e - eref), ldx(lcf.d.m, lcf.d.e - eref),
                   ldx(lcb.p.m, lcb.p.e - eref), ldx(lcb.d.m, lcb.d.e - eref), L, y);
  } else {
    // (K x)_i = sum_k lambda^{|i-k|} x_k: the forward and backward recursions
    T af, ab;
    run_aggs<T, R>(x, L, af, ab);
    S1<T> cf, cb;
    if constexpr (GL == 1) {
      block_scan<S1<T>, NW, T>(S1<T>{{af, E}}, S1<T>{{ab, E}}, dec, S1<T>::zero(),
                               S1<T>::zero(), &cf, &cb, nullptr, nullptr, sh);
    } else {
      group_scan<S1<T>, NQ, GL, T>(S1<T>{{af, E}}, S1<T>{{ab, E}}, dec, gi, tq, &cf, &cb, gsh);
    }
    const S1<T> lcf = cf.shift(step), lcb = cb.shift(step);
    if constexpr (SC) {
      // the product on the run's frame: the largest of the run's and the
      // carries' exponents
      eref = max(local_exponent<T, R>(x, E), max(lcf.v.e, lcb.v.e));
      if (eref == kExpZero) eref = 0;
      T xf[R];
#pragma unroll
      for (int r = 0; r < R; ++r) xf[r] = ldx(x[r], E - eref);
      run_apply<T, R>(xf, ldx(lcf.v.m, lcf.v.e - eref), ldx(lcb.v.m, lcb.v.e - eref), L, y);
    } else {
      run_apply<T, R>(x, ldx(lcf.v.m, lcf.v.e), ldx(lcb.v.m, lcb.v.e), L, y);
    }
  }
  // y * 2^eref is the product at this thread's positions (plain domain: eref
  // = 0 except for the cost recursion's frame)
  T* yout = static_cast<T*>(a.y);
  if constexpr (MODE == L_APPLY || MODE == L_COST) {
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (p0 + r < a.len) {
        const int64_t q = base + int64_t(p0 + r) * a.stride;
        if constexpr (SC) {
          yout[q] = y[r];
          a.ye[q] = eref;
        } else {
          yout[q] = ldx(y[r], eref);
        }
      }
    return;
  }
  // a line's share of a sum: the sum of its threads' parts, in part[line]
  auto line_share = [&](double s) {
    if constexpr (GL == 1) {
      const double tot = block_sum<NW>(s, red);
      if (threadIdx.x == 0) a.part[line] = tot;
    } else {
      gred[threadIdx.x] = s;
      __syncthreads();
      if (tq == 0) {
        double tot = 0.0;
        for (int v = 0; v < NQ; ++v) tot += gred[CONT ? gi * NQ + v : v * GL + gi];
        a.part[line] = tot;
      }
    }
  };
  const T* own = static_cast<const T*>(a.own);
  // exponent of own at position q, beside the product's eref
  auto own_exp = [&](int64_t q) { return SC ? a.owne[q] + eref : eref; };
  if constexpr (MODE == L_DOT || MODE == L_COSTDOT) {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (p0 + r < a.len) {
        const int64_t q = base + int64_t(p0 + r) * a.stride;
        s += ldexp(double(own[q]) * double(y[r]), own_exp(q));
      }
    line_share(s);
    return;
  }
  // ERR, UPDATE: | own * (K x) - marg | and marg / (K x)
  const bool want_err = (MODE == L_ERR) || a.check;
  if (want_err) {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (p0 + r < a.len) {
        const int64_t q = base + int64_t(p0 + r) * a.stride;
        s += fabs(ldexp(double(own[q]) * double(y[r]), own_exp(q)) - a.m64[q]);
      }
    line_share(s);
  }
  if constexpr (MODE == L_UPDATE) {
    bool bad = false;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (p0 + r < a.len) {
        const int64_t q = base + int64_t(p0 + r) * a.stride;
        const T mg = (sizeof(T) == 8) ? T(a.m64[q]) : T(a.m32[q]);
        const T v = (mg == T(0)) ? T(0) : mg / y[r];
        bad |= !isfinite(v);
        if constexpr (SC) {
          // marg / (y 2^eref) = v 2^-eref, normalised entry by entry
          int kv = 0;
          const T vm = (v == T(0) || !isfinite(v)) ? v : frx(v, &kv);
          yout[q] = vm;
          a.ye[q] = (v == T(0)) ? 0 : kv - eref;
        } else {
          yout[q] = v;
        }
      }
    if (bad) {
      atomicOr(&a.ctrl->fail, 1);
      atomicMin(&a.ctrl->fail_iter, a.l);
    }
  }
}

// out[0] = scale * (fixed-order sum of part[0..n))
__global__ __launch_bounds__(256) void k_sum2(const double* part, int n, double scale,
                                              double* out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  const double tot = block_sum<4>(s, red);
  if (threadIdx.x == 0) out[0] = scale * tot;
}

template <typename T>
__global__ void k_fill2(T* a, T* b, int64_t n, T v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    a[i] = v;
    b[i] = v;
  }
}

// F = ln phi, G = ln psi (binary64; -inf where a scaling is zero); in the log
// domain the entries are m 2^e with their exponents in ea, eb
template <typename T>
__global__ void k_log2(const T* a, const T* b, const int* ea, const int* eb, int64_t n,
                       double* out) {
  constexpr double kLn2 = 0.69314718055994530942;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    out[i] = log(double(a[i])) + (ea ? double(ea[i]) * kLn2 : 0.0);
    out[n + i] = log(double(b[i])) + (eb ? double(eb[i]) * kLn2 : 0.0);
  }
}

__global__ void k_zero_int(int* a, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

// ---------------------------------------------------------------------------
// Small grids (n1 n2 <= 4096, short lines): the whole of Algorithm 2 in one
// workgroup of NT threads (the fewest of 64, 256, 1024 that hold the grid at 4
// entries each; in the plain domain up to 8192 points at 8 entries on 1024
// threads, where the three LDS arrays fit).  Thread t keeps the entries
// t + NT r (r < P) of phi, psi, mu and nu in registers; a product K v goes through three LDS arrays (columns
// padded to an odd length), one pass per axis, with the paper's sequential
// recursions along each line (Sec. 3: p_k = lambda p_{k-1} + x_k and the
// backward sum), the two directions of a line run side by side by two
// threads, so the arithmetic is the sequential algorithm's, line by line.
//
// SC (the log domain): every scaling entry, and every entry of a product, is
// an extended number (mantissa, int32 exponent), in registers and in two more
// LDS arrays of exponents, and the recursions run in extended arithmetic entry
// by entry with lambda itself extended, so nothing underflows however large
// h/eps is; the update normalises each new scaling entry as the per-line
// passes do.
// ---------------------------------------------------------------------------
constexpr int kRes2MaxThreads = 1024;
constexpr int kRes2Per = 4;  // entries per thread: n1 n2 <= 4 x threads (64, 256 or 1024)
// plain domain, 4097 .. 8192 grid points: 8 entries on each of 1024 threads
constexpr int kRes2PerWide = 8;

// Largest n1 + n2 for the one-workgroup solver (an iteration walks both line
// lengths sequentially, while the per-line launches take about 20 us (log
// domain) to 25 us (plain) an iteration at any of these sizes), measured on
// square and elongated grids at h/eps = 100: plain up to 16 x 256 wins, 8 x
// 500 loses; in the log domain the extended recursions cost more per entry
// (binary64 at 1024 threads runs groups of two to stay in registers).
constexpr int64_t kRes2MaxSpan = 384;       // plain domain
constexpr int64_t kRes2MaxSpanLog64 = 80;   // log domain, binary64
constexpr int64_t kRes2MaxSpanLog32 = 128;  // log domain, binary32

// LDS distance between columns: n1 made odd
__host__ __device__ inline int res2d_ld(int n1) { return n1 | 1; }

struct Res2Args {
  const double* mu;
  const double* nu;
  const float* mu32;
  const float* nu32;
  void* vF;      // in: initial phi; out: final phi
  void* vG;      // in: initial psi; out: final psi
  int* eF;       // log domain: exponents of vF and vG (in and out)
  int* eG;
  Ctrl* ctrl;
  double* err_hist;
  int n1, n2;
  int itr_max;
  int check_every;
  double tol;
  double lam1, lam2;
  Decay xlam1, xlam2;  // log domain: lambda1, lambda2 as extended numbers
};

// An LDS entry as an extended number: a zero mantissa takes the exponent of
// zero, so that it never sets the exponent of a sum.
template <typename T>
__device__ __forceinline__ XF<T> xentry(T m, int e) {
  return {m, m == T(0) ? kExpZero : e};
}

// One direction of a line's recursion, r_k = lambda r_{k-1} + x_k over the
// entries p0 + k step (k < len; step < 0 runs the line backwards), written to
// O.  A group of G entries at a time: the group's LDS loads are issued
// together, unconditionally, ahead of its dependent chain; the entries past
// the last whole group follow one at a time.
// SC: extended arithmetic, the exponents in XE / OE, lambda as xlam; the
// running sum is normalised once per group (a step multiplies the mantissa by
// lambda's, in [1, 2), and an addition at most doubles it, so G steps stay far
// inside the range of T).
template <typename T, int G, bool SC>
__device__ __forceinline__ void seq_scan(const T* X, const int* XE, T* O, int* OE, int p0,
                                         int step, int len, T lam, XF<T> xlam) {
  T r = T(0);
  XF<T> xr = xzero<T>();
  int k = 0;
  for (; k + G <= len; k += G) {
    T v[G];
    int ve[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      v[u] = X[p0 + (k + u) * step];
      if constexpr (SC) ve[u] = XE[p0 + (k + u) * step];
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      if constexpr (SC) {
        xr = xadd(xmul(xr, xlam), xentry(v[u], ve[u]));
        v[u] = xr.m;
        ve[u] = xr.e;
      } else {
        r = lam * r + v[u];
        v[u] = r;
      }
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      O[p0 + (k + u) * step] = v[u];
      if constexpr (SC) OE[p0 + (k + u) * step] = ve[u];
    }
    if constexpr (SC) xr = xnorm(xr);
  }
  for (; k < len; ++k) {
    const int q = p0 + k * step;
    if constexpr (SC) {
      xr = xadd(xmul(xr, xlam), xentry(X[q], XE[q]));
      O[q] = xr.m;
      OE[q] = xr.e;
    } else {
      r = lam * r + X[q];
      O[q] = r;
    }
  }
}

// The 1-D product along the lines of one axis, from X into Y and Z: for each
// line, one thread runs the forward recursion into Y and another the backward
// one (inclusive, s_k = lambda s_{k+1} + x_k) into Z, side by side; the
// product is then y_k = f_k + lambda s_{k+1} (Sec. 3: the backward sum of the
// paper is lambda s_{k+1}).  nlines lines of len entries, line L at L lstep,
// entries estep apart.
template <typename T, int NT, int G, bool SC>
__device__ __forceinline__ void seq_axis(const T* X, const int* XE, T* Y, int* YE, T* Z, int* ZE,
                                         int nlines, int lstep, int len, int estep, T lam,
                                         XF<T> xlam) {
  for (int w = threadIdx.x; w < 2 * nlines; w += NT) {
    const bool fw = w < nlines;
    const int L = fw ? w : w - nlines;
    seq_scan<T, G, SC>(X, XE, fw ? Y : Z, fw ? YE : ZE, L * lstep + (fw ? 0 : (len - 1) * estep),
                       fw ? estep : -estep, len, lam, xlam);
  }
}

// y_k = f_k + lambda s_{k+1} at LDS position q (s_{k+1} at q + estep; none at
// the line's last entry)
template <typename T>
__device__ __forceinline__ T seq_combine(const T* Y, const T* Z, int q, int estep, bool last,
                                         T lam) {
  return last ? Y[q] : Y[q] + lam * Z[q + estep];
}

template <typename T>
__device__ __forceinline__ XF<T> seq_combine_x(const T* Y, const int* YE, const T* Z,
                                               const int* ZE, int q, int estep, bool last,
                                               XF<T> lam) {
  const XF<T> f{Y[q], YE[q]};
  return last ? f : xadd(f, xmul(XF<T>{Z[q + estep], ZE[q + estep]}, lam));
}

constexpr int GX64 = 2;  // group of the binary64 log-domain recursions at 1024 threads

template <typename T, int NT, bool SC, int P>
__global__ __launch_bounds__(NT) void k_res2d(Res2Args a) {
  extern __shared__ __align__(16) unsigned char lds2[];
  __shared__ double red[NT / kWave];
  __shared__ int sstop;
  const int n = a.n1 * a.n2;
  // columns ld = n1 | 1 entries apart in LDS: an odd stride spreads the
  // lanes that walk different columns over the banks
  const int ld = res2d_ld(a.n1);
  const int nl = ld * a.n2;
  T* X = reinterpret_cast<T*>(lds2);
  T* Y = X + nl;
  T* Z = Y + nl;
  int* XE = reinterpret_cast<int*>(Z + nl);  // log domain only
  int* YE = XE + nl;
  int* ZE = YE + nl;
  const int t = threadIdx.x;
  // LDS position of the entries t + NT r, and whether each is the last of its
  // column / of its row
  int off[P];
  bool last1[P], last2[P];
#pragma unroll
  for (int r = 0; r < P; ++r) {
    const int e = t + NT * r;
    const int i = e % a.n1, j = e / a.n1;
    off[r] = i + ld * j;
    last1[r] = i + 1 == a.n1;
    last2[r] = j + 1 == a.n2;
  }
  const T lam1 = T(a.lam1), lam2 = T(a.lam2);
  const XF<T> xl1{T(a.xlam1.m), a.xlam1.e}, xl2{T(a.xlam2.m), a.xlam2.e};
  T ph[P], ps[P], mu[P], nu[P];
  int phe[P], pse[P];  // log domain: exponents of ph, ps
  // the stopping test's binary64 nu (binary64 scalings: nu itself)
  double nu64[sizeof(T) == 8 ? 1 : P];
#pragma unroll
  for (int r = 0; r < P; ++r) {
    const int e = t + NT * r;
    const bool in = e < n;
    ph[r] = in ? static_cast<const T*>(a.vF)[e] : T(0);
    ps[r] = in ? static_cast<const T*>(a.vG)[e] : T(0);
    phe[r] = (SC && in) ? a.eF[e] : 0;
    pse[r] = (SC && in) ? a.eG[e] : 0;
    if constexpr (sizeof(T) == 8) {
      mu[r] = in ? T(a.mu[e]) : T(0);
      nu[r] = in ? T(a.nu[e]) : T(0);
    } else {
      nu64[r] = in ? a.nu[e] : 0.0;
      mu[r] = in ? T(a.mu32[e]) : T(0);
      nu[r] = in ? T(a.nu32[e]) : T(0);
    }
  }
  // entries per group of the line recursions (binary64 in the log domain at
  // 1024 threads: fewer, which keeps the kernel within its 128 registers per
  // lane)
  constexpr int G = !SC ? (sizeof(T) == 8 ? 8 : 16)
                        : ((sizeof(T) == 8 && NT == kRes2MaxThreads) ? GX64 : 8);
  // K v (v = ph or ps with its exponents) at this thread's entries into
  // pm (and pe): the recursions along the columns (X -> Y, Z), their
  // combination into X, the recursions along the rows (X -> Y, Z), and the
  // combination of those at the thread's own entries
  T pm[P];
  int pe[P];
  auto product = [&](const T* v, const int* ve) {
#pragma unroll
    for (int r = 0; r < P; ++r) {
      const int e = t + NT * r;
      if (e < n) {
        X[off[r]] = v[r];
        if constexpr (SC) XE[off[r]] = ve[r];
      }
    }
    __syncthreads();
    seq_axis<T, NT, G, SC>(X, XE, Y, YE, Z, ZE, a.n2, ld, a.n1, 1, lam1, xl1);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < P; ++r) {
      const int e = t + NT * r;
      if (e < n) {
        if constexpr (SC) {
          const XF<T> c = seq_combine_x(Y, YE, Z, ZE, off[r], 1, last1[r], xl1);
          X[off[r]] = c.m;
          XE[off[r]] = c.e;
        } else {
          X[off[r]] = seq_combine(Y, Z, off[r], 1, last1[r], lam1);
        }
      }
    }
    __syncthreads();
    seq_axis<T, NT, G, SC>(X, XE, Y, YE, Z, ZE, a.n1, 1, a.n2, ld, lam2, xl2);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < P; ++r) {
      const int e = t + NT * r;
      if (e < n) {
        if constexpr (SC) {
          const XF<T> c = seq_combine_x(Y, YE, Z, ZE, off[r], ld, last2[r], xl2);
          pm[r] = c.m;
          pe[r] = c.e;
        } else {
          pm[r] = seq_combine(Y, Z, off[r], ld, last2[r], lam2);
          pe[r] = 0;
        }
      }
    }
  };
  // v <- marg / (K v'), entry by entry (normalised to its own exponent in
  // the log domain); returns whether any entry is not finite
  auto update = [&](T* v, int* ve, const T* marg) {
    bool bad = false;
#pragma unroll
    for (int r = 0; r < P; ++r) {
      const int e = t + NT * r;
      if (e < n) {
        const T q = (marg[r] == T(0)) ? T(0) : marg[r] / pm[r];
        bad |= !isfinite(q);
        if constexpr (SC) {
          int kq = 0;
          v[r] = (q == T(0) || !isfinite(q)) ? q : frx(q, &kq);
          ve[r] = (q == T(0)) ? 0 : kq - pe[r];
        } else {
          v[r] = q;
        }
      }
    }
    return bad;
  };
  int l = 0, stop_iter = -1, fail_iter = -1;
  for (; l < a.itr_max; ++l) {
    // psi-half: K^T phi^l (K is symmetric)
    product(ph, phe);
    if ((l % a.check_every) == 0) {
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const int e = t + NT * r;
        if (e < n) {
          double pv = double(ps[r]) * double(pm[r]);
          if constexpr (SC) pv = ldexp(pv, pse[r] + pe[r]);
          s += fabs(pv - (sizeof(T) == 8 ? double(nu[r]) : nu64[sizeof(T) == 8 ? 0 : r]));
        }
      }
      const double tot = block_sum<NT / kWave>(s, red);
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
    bool bad = update(ps, pse, nu);
    // phi-half: K psi^{l+1} (its first LDS writes go to X, which no thread
    // reads after the row recursions)
    product(ps, pse);
    bad |= update(ph, phe, mu);
    // a non-finite scaling in either half ends the solve (abnormal termination)
    if (__syncthreads_or(bad ? 1 : 0)) {
      fail_iter = l;
      break;
    }
  }
#pragma unroll
  for (int r = 0; r < P; ++r) {
    const int e = t + NT * r;
    if (e < n) {
      static_cast<T*>(a.vF)[e] = ph[r];
      static_cast<T*>(a.vG)[e] = ps[r];
      if constexpr (SC) {
        a.eF[e] = phe[r];
        a.eG[e] = pse[r];
      }
    }
  }
  if (t == 0) {
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

// LDS bytes of the one-workgroup solver, or 0 if the grid does not fit it on
// this device
int res2d_threads(int64_t n) {
  for (int nt : {64, 256, kRes2MaxThreads})
    if (n <= int64_t(nt) * kRes2Per) return nt;
  return 0;
}

// entries per thread: kRes2Per, or kRes2PerWide (plain domain, 1024 threads)
// for grids beyond 4 x 1024 points; 0 if the grid does not fit either
int res2d_per(int64_t n, bool log_domain) {
  if (res2d_threads(n) != 0) return kRes2Per;
  return (!log_domain && n <= int64_t(kRes2MaxThreads) * kRes2PerWide) ? kRes2PerWide : 0;
}

size_t res2d_lds(int64_t n1, int64_t n2, int dt, bool log_domain) {
  const int64_t n = n1 * n2;
  if (res2d_per(n, log_domain) == 0) return 0;
  // an iteration walks both line lengths sequentially: beyond this the
  // per-line launches (fixed cost per pass) are faster
  const int64_t span = !log_domain ? kRes2MaxSpan
                                   : (dt == FS1_F64 ? kRes2MaxSpanLog64 : kRes2MaxSpanLog32);
  if (n1 + n2 > span) return 0;
  // X, Y and Z (columns padded to an odd length), and in the log domain
  // their exponents
  const size_t bytes = size_t(3) * size_t(res2d_ld(int(n1))) * size_t(n2) *
                       ((dt == FS1_F64 ? 8 : 4) + (log_domain ? 4 : 0));
  int dev = 0, lim = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 0;
  // room for the kernel's own reduction arrays
  return bytes + 1024 <= size_t(lim) ? bytes : 0;
}

template <typename T, int NT, bool SC, int P>
hipError_t launch_res2d_t(const Res2Args& a, size_t lds, hipStream_t s) {
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k_res2d<T, NT, SC, P>),
        hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
  }
  k_res2d<T, NT, SC, P><<<1, NT, lds, s>>>(a);
  return hipGetLastError();
}

template <typename T, bool SC>
hipError_t launch_res2d(const Res2Args& a, size_t lds, hipStream_t s) {
  const int64_t n = int64_t(a.n1) * a.n2;
  if constexpr (!SC) {
    if (res2d_per(n, false) == kRes2PerWide)
      return launch_res2d_t<T, kRes2MaxThreads, SC, kRes2PerWide>(a, lds, s);
  }
  switch (res2d_threads(n)) {
    case 64: return launch_res2d_t<T, 64, SC, kRes2Per>(a, lds, s);
    case 256: return launch_res2d_t<T, 256, SC, kRes2Per>(a, lds, s);
    case kRes2MaxThreads: return launch_res2d_t<T, kRes2MaxThreads, SC, kRes2Per>(a, lds, s);
    default: return hipErrorInvalidValue;
  }
}

// One pass over the lines of one axis.  R: entries per thread (kR2, or 1 in
// the log domain where h/eps is too large for runs of kR2, as in 1-D).  The
// lines of axis a of a grid n_0 x ... (first axis fastest) start at
// (L mod s_a) + (L div s_a) s_a n_a, entries s_a = n_0 ... n_{a-1} apart.
struct Axis {
  int64_t nlines;
  int64_t inner;
  int64_t outer;
  int64_t stride;
  int len;
  int R;
  ScanConsts k;
};

template <typename T, int R, int MODE, bool SC>
hipError_t run_pass_r(const Axis& ax, const LineArgs& a, hipStream_t s) {
  const unsigned g = unsigned(ax.nlines);
  if (ax.inner == 1) {
    // short contiguous lines (the first axis): several one after another
    // per workgroup of kContThreads, each on the fewest threads that hold it,
    // where one line per workgroup would leave most of its lanes idle -- 16
    // or 32 threads' worth in a one-wavefront workgroup, with a group per
    // compute unit, or 128 threads' worth in a 256-thread workgroup, with
    // 2048 groups (measured: with fewer lines, or 64 threads' worth, the
    // one-line form's wavefront scan is faster than the group's LDS scan)
    constexpr int NTc = kContThreads;
    int nq = 16;
    while (int64_t(nq) * R < ax.len && nq < 128) nq *= 2;
    const int64_t gl = NTc / nq;
    const bool fits = int64_t(nq) * R >= ax.len && ax.nlines % gl == 0;
    if (fits && nq <= 32 && ax.nlines >= 256 * gl) {
      const unsigned gg = unsigned(ax.nlines / gl);
      if (nq == 16) {
        k_line<T, R, NTc, MODE, SC, NTc / 16, true><<<gg, NTc, 0, s>>>(a, ax.k);
      } else {
        k_line<T, R, NTc, MODE, SC, NTc / 32, true><<<gg, NTc, 0, s>>>(a, ax.k);
      }
      return hipGetLastError();
    }
    if (fits && nq == 128 && ax.nlines >= 2048 * gl) {
      k_line<T, R, NTc, MODE, SC, NTc / 128, true><<<unsigned(ax.nlines / gl), NTc, 0, s>>>(a,
                                                                                      ax.k);
      return hipGetLastError();
    }
  } else {
    // a strided axis with line starts a multiple of kGroup entries apart,
    // lines of at most 32 runs and enough lines for a group per compute unit:
    // kGroup adjacent lines per workgroup
    if (ax.inner % kGroup == 0 && ax.len <= 32 * R && ax.nlines >= int64_t(256) * kGroup) {
      const unsigned gg = unsigned(ax.nlines / kGroup);
      if (ax.len <= 8 * R) {
        k_line<T, R, 8 * kGroup, MODE, SC, kGroup><<<gg, 8 * kGroup, 0, s>>>(a, ax.k);
      } else {
        k_line<T, R, 32 * kGroup, MODE, SC, kGroup><<<gg, 32 * kGroup, 0, s>>>(a, ax.k);
      }
      return hipGetLastError();
    }
    // longer lines (up to 256 runs): kGroupLong adjacent lines per workgroup
    // (not the cost recursion, whose two-state scan would need twice the LDS)
    if constexpr (MODE != L_COST && MODE != L_COSTDOT) {
      if (ax.inner % kGroupLong == 0 && ax.len > 32 * R && ax.len <= 256 * R &&
          ax.nlines >= int64_t(256) * kGroupLong) {
        const unsigned gg = unsigned(ax.nlines / kGroupLong);
        if (ax.len <= 64 * R) {
          k_line<T, R, 64 * kGroupLong, MODE, SC, kGroupLong>
              <<<gg, 64 * kGroupLong, 0, s>>>(a, ax.k);
        } else if (ax.len <= 128 * R) {
          k_line<T, R, 128 * kGroupLong, MODE, SC, kGroupLong>
              <<<gg, 128 * kGroupLong, 0, s>>>(a, ax.k);
        } else {
          k_line<T, R, 256 * kGroupLong, MODE, SC, kGroupLong>
              <<<gg, 256 * kGroupLong, 0, s>>>(a, ax.k);
        }
        return hipGetLastError();
      }
    }
  }
  if (ax.len <= kWave * R) {
    // one wavefront: its scans and reductions stay in registers
    k_line<T, R, kWave, MODE, SC><<<g, kWave, 0, s>>>(a, ax.k);
  } else if (ax.len <= 256 * R) {
    k_line<T, R, 256, MODE, SC><<<g, 256, 0, s>>>(a, ax.k);
  } else {
    k_line<T, R, 1024, MODE, SC><<<g, 1024, 0, s>>>(a, ax.k);
  }
  return hipGetLastError();
}

template <typename T, int MODE, bool SC = false>
hipError_t run_pass(const Axis& ax, LineArgs a, hipStream_t s) {
  a.inner = ax.inner;
  a.outer = ax.outer;
  a.stride = ax.stride;
  a.len = ax.len;
  if constexpr (SC) {
    if (ax.R == 1) return run_pass_r<T, 1, MODE, SC>(ax, a, s);
  }
  return run_pass_r<T, kR2, MODE, SC>(ax, a, s);
}

// runtime mode -> the pass template
template <typename T, bool SC>
hipError_t run_mode(int mode, const Axis& ax, const LineArgs& a, hipStream_t s) {
  switch (mode) {
    case L_APPLY: return run_pass<T, L_APPLY, SC>(ax, a, s);
    case L_COST: return run_pass<T, L_COST, SC>(ax, a, s);
    case L_UPDATE: return run_pass<T, L_UPDATE, SC>(ax, a, s);
    case L_ERR: return run_pass<T, L_ERR, SC>(ax, a, s);
    case L_DOT: return run_pass<T, L_DOT, SC>(ax, a, s);
    default: return run_pass<T, L_COSTDOT, SC>(ax, a, s);
  }
}

constexpr int kMaxDim = 4;  // axes of a grid

struct Grid {
  int nd;
  int64_t n;
  int64_t max_lines;  // most lines of any axis
  Axis ax[kMaxDim];
};

// Entries per thread along an axis: kR2, except in the log domain where every
// output of a run must stay within lambda^(R-1) of its largest contribution
// inside the working precision (the 1-D bound on (R-1) h/eps), else 1.
int line_run_length(bool log_domain, int dt, double h, double eps) {
  if (!log_domain) return kR2;
  return pick_run_length(dt, true, h / eps) >= kR2 ? kR2 : 1;
}

Grid make_grid(int nd, const int64_t* dims, const double* h, double eps, bool log_domain = false,
               int dt = FS1_F64) {
  Grid g{};
  g.nd = nd;
  g.n = 1;
  for (int a = 0; a < nd; ++a) g.n *= dims[a];
  int64_t s = 1;
  for (int a = 0; a < nd; ++a) {
    const int r = line_run_length(log_domain, dt, h[a], eps);
    g.ax[a] = Axis{g.n / dims[a], s, s * dims[a], s, int(dims[a]), r,
                   make_scan_consts(h[a], eps, r)};
    g.max_lines = std::max(g.max_lines, g.ax[a].nlines);
    s *= dims[a];
  }
  return g;
}

int check_grid(int nd, const int64_t* dims, const double* h, double eps, bool log_domain = false,
               int dt = FS1_F64) {
  using host::set_err;
  const int64_t lmax = int64_t(1024) * kR2;
  if (nd < 1 || nd > kMaxDim)
    return set_err(FS1_ERR_INVALID_ARG, "ndim must be 1 .. %d (got %d)", kMaxDim, nd);
  if (!dims || !h) return set_err(FS1_ERR_INVALID_ARG, "null dims or spacings");
  if (!(eps > 0.0) || !std::isfinite(eps))
    return set_err(FS1_ERR_INVALID_ARG, "eps must be finite and > 0");
  int64_t n = 1;
  for (int a = 0; a < nd; ++a) {
    if (dims[a] < 1 || dims[a] > lmax)
      return set_err(FS1_ERR_INVALID_ARG, "grid side %d must be 1 .. %lld (got %lld)", a,
                     (long long)lmax, (long long)dims[a]);
    // one workgroup holds a line: 1024 entries where the runs have length 1
    if (log_domain && line_run_length(true, dt, h[a], eps) == 1 && dims[a] > 1024)
      return set_err(FS1_ERR_INVALID_ARG,
                     "log domain: h/eps too large for runs of %d along an axis of more than "
                     "1024 entries",
                     kR2);
    if (!(h[a] > 0.0) || !std::isfinite(h[a]))
      return set_err(FS1_ERR_INVALID_ARG, "spacings must be finite and > 0");
    if (double(dims[a]) * (h[a] / eps) > 1.0e8)
      return set_err(FS1_ERR_INVALID_ARG, "n h / eps exceeds 1e8 along an axis");
    n *= dims[a];
    // the lines of an axis are one launch's workgroups
    if (n > (int64_t(1) << 31) - 1)
      return set_err(FS1_ERR_INVALID_ARG, "the grid holds more than 2^31 - 1 points");
  }
  return FS1_OK;
}

// y = K x: the first axis from x into y, the others in place (a pass reads
// each entry of a line in the thread that writes it)
template <typename T>
hipError_t kvn(const Grid& g, const void* x, void* y, hipStream_t s) {
  LineArgs a{};
  for (int d = 0; d < g.nd; ++d) {
    a.x = d == 0 ? x : y;
    a.y = y;
    const hipError_t e = run_pass<T, L_APPLY>(g.ax[d], a, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

struct Bufs2 {
  void* vF;
  void* vG[2];
  void* t;
  int* eF;          // log domain: exponents of vF, vG, t (one per entry)
  int* eG[2];
  int* et;
  double* mu;       // caller's marginals, binary64
  double* nu;
  float* mu32;      // binary32 copies (T = float)
  float* nu32;
  double* part;     // per-line shares of the last axis (as many as the most lines)
  double* part2;
  double* sums;     // [0] err, [1] mu err, [2 + a] cost term of axis a
  Ctrl* ctrl;
};

// SC: the log domain, every vector with its per-entry exponents.
template <typename T, bool SC>
struct Ops2 {
  // x of a pass with its exponents
  static void in(LineArgs& a, const void* v, const int* e) {
    a.x = v;
    a.xe = e;
  }
  static void to(LineArgs& a, void* v, int* e) {
    a.y = v;
    a.ye = e;
  }
  static void with(LineArgs& a, const void* v, const int* e) {
    a.own = v;
    a.owne = e;
  }
  // The passes of a product K v (cost_axis >= 0: C along that axis instead
  // of K) from x: every axis but the last from x (first) or t into t, then
  // the last axis in mode `last` from t (or x for one axis), with the fields
  // of a that the last pass needs already set.  `a` arrives with the first
  // pass's fields (decide) and leaves them only to that pass.
  static hipError_t passes(const Grid& g, const Bufs2& b, LineArgs a, const void* x,
                           const int* xe, int cost_axis, int last, hipStream_t s) {
    LineArgs f = a;  // first pass: may decide; later passes never do
    for (int d = 0; d + 1 < g.nd; ++d) {
      LineArgs p = d == 0 ? f : a;
      if (d > 0) p.decide = 0;
      // a middle pass carries no last-pass work
      p.check = 0;
      in(p, d == 0 ? x : b.t, d == 0 ? xe : b.et);
      to(p, b.t, b.et);
      const hipError_t e = run_mode<T, SC>(d == cost_axis ? L_COST : L_APPLY, g.ax[d], p, s);
      if (e != hipSuccess) return e;
    }
    LineArgs p = a;
    if (g.nd > 1) p.decide = 0;
    in(p, g.nd == 1 ? x : b.t, g.nd == 1 ? xe : b.et);
    return run_mode<T, SC>(last, g.ax[g.nd - 1], p, s);
  }
  // psi^{l+1} = nu / K^T phi^l into vG[(l+1)&1] (and the error of (phi^l, psi^l) when checked)
  static hipError_t psi_half(const Grid& g, const Bufs2& b, int l, int check, hipStream_t s) {
    LineArgs a{};
    a.ctrl = b.ctrl;
    a.guard = 1;
    a.l = l;
    to(a, b.vG[(l + 1) & 1], b.eG[(l + 1) & 1]);
    with(a, b.vG[l & 1], b.eG[l & 1]);
    a.m64 = b.nu;
    a.m32 = b.nu32;
    a.part = b.part;
    a.check = check;
    return passes(g, b, a, b.vF, b.eF, -1, L_UPDATE, s);
  }
  // phi^{l+1} = mu / K psi^{l+1}; when checked, its first pass takes the stop
  // decision of iteration l from the psi-half's shares first
  static hipError_t phi_half(const Grid& g, const Bufs2& b, int l, int check, double tol,
                             double* err_hist, hipStream_t s) {
    LineArgs a{};
    a.ctrl = b.ctrl;
    a.guard = 1;
    a.l = l;
    a.decide = check;
    a.part = b.part;
    a.nparts = int(g.ax[g.nd - 1].nlines);
    a.tol = tol;
    a.err_hist = err_hist;
    to(a, b.vF, b.eF);
    a.m64 = b.mu;
    a.m32 = b.mu32;
    return passes(g, b, a, b.vG[(l + 1) & 1], b.eG[(l + 1) & 1], -1, L_UPDATE, s);
  }
  // final errors (both sides) and the transport cost of (phi, psi = vG[gbuf]):
  // one term per axis, h_a <phi, (.. C_a ..) psi>
  static hipError_t finalize(const Grid& g, const Bufs2& b, int gbuf, const double* h,
                             hipStream_t s) {
    const int nl = int(g.ax[g.nd - 1].nlines);
    LineArgs a{};
    a.ctrl = b.ctrl;
    // nu side: sum | psi (K^T phi) - nu |
    with(a, b.vG[gbuf], b.eG[gbuf]);
    a.m64 = b.nu;
    a.part = b.part;
    hipError_t e = passes(g, b, a, b.vF, b.eF, -1, L_ERR, s);
    if (e != hipSuccess) return e;
    k_sum2<<<1, 256, 0, s>>>(b.part, nl, 1.0, b.sums + 0);
    // mu side: sum | phi (K psi) - mu |
    with(a, b.vF, b.eF);
    a.m64 = b.mu;
    a.part = b.part2;
    e = passes(g, b, a, b.vG[gbuf], b.eG[gbuf], -1, L_ERR, s);
    if (e != hipSuccess) return e;
    k_sum2<<<1, 256, 0, s>>>(b.part2, nl, 1.0, b.sums + 1);
    // cost terms
    for (int c = 0; c < g.nd; ++c) {
      double* part = (c & 1) ? b.part2 : b.part;
      a.part = part;
      e = passes(g, b, a, b.vG[gbuf], b.eG[gbuf], c, c == g.nd - 1 ? L_COSTDOT : L_DOT, s);
      if (e != hipSuccess) return e;
      k_sum2<<<1, 256, 0, s>>>(part, nl, h[c], b.sums + 2 + c);
    }
    return hipGetLastError();
  }
};

template <typename F>
hipError_t dispatch2(int dt, bool log_domain, F&& f) {
  if (log_domain) return dt == 0 ? f(Ops2<double, true>{}) : f(Ops2<float, true>{});
  return dt == 0 ? f(Ops2<double, false>{}) : f(Ops2<float, false>{});
}

}  // namespace

int kv_apply_grid(fs1_ctx* ctx, const void* x, void* y, int nd, const int64_t* dims,
                  const double* h, double eps, int dt) {
  using namespace host;
  if (!ctx) return set_err(FS1_ERR_INVALID_ARG, "null context");
  if (!x || !y) return set_err(FS1_ERR_INVALID_ARG, "null array");
  if (dt != FS1_F64 && dt != FS1_F32) return set_err(FS1_ERR_INVALID_ARG, "bad dtype %d", dt);
  int st = check_grid(nd, dims, h, eps);
  if (st) return st;
  const Grid g = make_grid(nd, dims, h, eps);
  const size_t es = dt == FS1_F64 ? 8 : 4;
  const char* xb = static_cast<const char*>(x);
  const char* yb = static_cast<const char*>(y);
  if (xb < yb + g.n * es && yb < xb + g.n * es)
    return set_err(FS1_ERR_INVALID_ARG, "x and y must not overlap");
  const hipError_t e = dt == FS1_F64 ? kvn<double>(g, x, y, ctx->stream)
                                     : kvn<float>(g, x, y, ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "kernel application on a grid");
  return FS1_OK;
}

int kv_apply_2d(fs1_ctx* ctx, const void* x, void* y, int64_t n1, int64_t n2, double h1,
                double h2, double eps, int dt) {
  const int64_t dims[2] = {n1, n2};
  const double h[2] = {h1, h2};
  return kv_apply_grid(ctx, x, y, 2, dims, h, eps, dt);
}

int solve_grid(fs1_ctx* ctx, const double* mu, const double* nu, int nd, const int64_t* dims,
               const double* h, double eps, double tol, const fs1_opts& o, fs1_result* out) {
  using namespace host;
  auto finish = [&](int st) {
    out->status = st;
    return st;
  };
  if (!mu || !nu) return finish(set_err(FS1_ERR_INVALID_ARG, "null marginal"));
  if (o.dtype != FS1_F64 && o.dtype != FS1_F32)
    return finish(set_err(FS1_ERR_INVALID_ARG, "bad dtype %d", o.dtype));
  if (o.domain != FS1_PLAIN && o.domain != FS1_LOG)
    return finish(set_err(FS1_ERR_INVALID_ARG, "a grid solve runs in the plain or log domain"));
  const bool lg = o.domain == FS1_LOG;
  if (!(tol >= 0.0)) return finish(set_err(FS1_ERR_INVALID_ARG, "tol must be >= 0"));
  if ((o.flags & FS1_FLAG_POTENTIALS) && !o.potentials_out)
    return finish(set_err(FS1_ERR_INVALID_ARG, "potentials requested without an output array"));
  int st = check_grid(nd, dims, h, eps, o.domain == FS1_LOG, o.dtype);
  if (st) return finish(st);
  const int dt = o.dtype;
  const Grid g = make_grid(nd, dims, h, eps, lg, dt);
  const int64_t n = g.n;
  const size_t es = dt == FS1_F64 ? 8 : 4;
  const int64_t nl = g.max_lines;

  Bufs2 b{};
  auto layout = [&](Carve& w) {
    b.vF = w.take(size_t(n) * es);
    b.vG[0] = w.take(size_t(n) * es);
    b.vG[1] = w.take(size_t(n) * es);
    b.t = w.take(size_t(n) * es);
    if (lg) {
      b.eF = static_cast<int*>(w.take(size_t(n) * 4));
      b.eG[0] = static_cast<int*>(w.take(size_t(n) * 4));
      b.eG[1] = static_cast<int*>(w.take(size_t(n) * 4));
      b.et = static_cast<int*>(w.take(size_t(n) * 4));
    }
    b.mu = static_cast<double*>(w.take(size_t(n) * 8));
    b.nu = static_cast<double*>(w.take(size_t(n) * 8));
    b.mu32 = dt == FS1_F32 ? static_cast<float*>(w.take(size_t(n) * 4)) : nullptr;
    b.nu32 = dt == FS1_F32 ? static_cast<float*>(w.take(size_t(n) * 4)) : nullptr;
    b.part = static_cast<double*>(w.take(size_t(nl) * 8));
    b.part2 = static_cast<double*>(w.take(size_t(nl) * 8));
    b.sums = static_cast<double*>(w.take((2 + kMaxDim) * 8));
    b.ctrl = static_cast<Ctrl*>(w.take(sizeof(Ctrl)));
  };
  {
    Carve probe(nullptr);
    layout(probe);
    st = ensure_ws(ctx, probe.off);
    if (st) return finish(st);
    Carve w(ctx->ws);
    layout(w);
  }
  hipStream_t s = ctx->stream;
  Ctrl* hc = ctx->hctrl;
  // validation and copies of the marginals (the 1-D set-up kernel over n entries)
  SolveBufs sb{};
  sb.dtype = dt;
  sb.n = n;
  sb.npad = n;
  sb.mu_src = mu;
  sb.nu_src = nu;
  sb.mu = b.mu;
  sb.nu = b.nu;
  sb.mu32 = b.mu32;
  sb.nu32 = b.nu32;
  sb.ctrl = b.ctrl;
  HIP_TRY(hipMemsetAsync(b.ctrl, 0, sizeof(Ctrl), s));
  HIP_TRY(launch_setup(sb, s));
  HIP_TRY(hipMemcpyAsync(hc, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hc->bad_input)
    return finish(set_err(FS1_ERR_INVALID_ARG, "marginals must be finite and >= 0"));
  if (!(hc->sum_mu > 0.0) || !(hc->sum_nu > 0.0))
    return finish(set_err(FS1_ERR_INVALID_ARG, "marginals must have positive mass"));
  if (std::fabs(hc->sum_mu - hc->sum_nu) > 1e-10 * hc->sum_mu)
    return finish(set_err(FS1_ERR_INVALID_ARG, "unequal masses: sum mu = %.17g, sum nu = %.17g",
                          hc->sum_mu, hc->sum_nu));
  // control block: running, no stop, no failure
  Ctrl c0{};
  c0.stop_iter = -1;
  c0.fail_iter = INT32_MAX;
  c0.last_check = -1;
  c0.last_err = NAN;
  *hc = c0;
  HIP_TRY(hipMemcpyAsync(b.ctrl, hc, sizeof(Ctrl), hipMemcpyHostToDevice, s));
  if (o.err_history)
    HIP_TRY(hipMemsetAsync(o.err_history, 0xFF, sizeof(double) * (size_t(o.itr_max) + 1), s));
  const unsigned gf = unsigned((n + 255) / 256);
  if (dt == FS1_F64) {
    k_fill2<double><<<gf, 256, 0, s>>>(static_cast<double*>(b.vF), static_cast<double*>(b.vG[0]),
                                       n, 1.0 / double(n));
  } else {
    k_fill2<float><<<gf, 256, 0, s>>>(static_cast<float*>(b.vF), static_cast<float*>(b.vG[0]), n,
                                      float(1.0 / double(n)));
  }
  HIP_TRY(hipGetLastError());
  if (lg) {
    // phi = psi = 1/n as mantissas with exponent 0
    k_zero_int<<<gf, 256, 0, s>>>(b.eF, n);
    k_zero_int<<<gf, 256, 0, s>>>(b.eG[0], n);
    HIP_TRY(hipGetLastError());
  }
  // the ctrl upload reads the pinned mirror: finish it before the host reuses it
  HIP_TRY(hipStreamSynchronize(s));

  // small 2-D grids: every iteration in one workgroup; it leaves psi in buffer 0
  const size_t lds =
      (nd != 2 || (o.flags & FS1_FLAG_NO_RESIDENT)) ? 0 : res2d_lds(dims[0], dims[1], dt, lg);
  bool resident = false;
  if (lds > 0) {
    Res2Args ra{};
    ra.mu = b.mu;
    ra.nu = b.nu;
    ra.mu32 = b.mu32;
    ra.nu32 = b.nu32;
    ra.vF = b.vF;
    ra.vG = b.vG[0];
    ra.eF = b.eF;
    ra.eG = b.eG[0];
    ra.ctrl = b.ctrl;
    ra.err_hist = o.err_history;
    ra.n1 = int(dims[0]);
    ra.n2 = int(dims[1]);
    ra.itr_max = o.itr_max;
    ra.check_every = o.check_every;
    ra.tol = tol;
    ra.lam1 = std::exp(-h[0] / eps);
    ra.lam2 = std::exp(-h[1] / eps);
    ra.xlam1 = make_decay(1.0, h[0] / eps);
    ra.xlam2 = make_decay(1.0, h[1] / eps);
    hipError_t e;
    if (lg) {
      e = dt == FS1_F64 ? launch_res2d<double, true>(ra, lds, s)
                        : launch_res2d<float, true>(ra, lds, s);
    } else {
      e = dt == FS1_F64 ? launch_res2d<double, false>(ra, lds, s)
                        : launch_res2d<float, false>(ra, lds, s);
    }
    if (e != hipSuccess) return finish(hip_fail(e, "2-D one-workgroup solve"));
    resident = true;
  }
  // Algorithm 2: while l < itr_max and err(l) > tol
  int l = resident ? o.itr_max : 0;
  bool stopped = resident;
  while (l < o.itr_max && !stopped) {
    const int l_end = std::min(o.itr_max, l + o.sync_every);
    for (; l < l_end; ++l) {
      const int check = (l % o.check_every) == 0;
      HIP_TRY(dispatch2(dt, lg,
                        [&](auto ops) { return decltype(ops)::psi_half(g, b, l, check, s); }));
      HIP_TRY(dispatch2(dt, lg, [&](auto ops) {
        return decltype(ops)::phi_half(g, b, l, check, tol, o.err_history, s);
      }));
    }
    HIP_TRY(hipMemcpyAsync(hc, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    stopped = hc->done != 0 || hc->fail != 0;
  }
  HIP_TRY(hipMemcpyAsync(hc, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hc->fail) {
    out->iterations = hc->fail_iter;
    out->converged = 0;
    return finish(set_err(FS1_ERR_NONFINITE,
                          "a scaling became non-finite at iteration %d (abnormal termination)",
                          hc->fail_iter + 1));
  }
  const int l_final = (hc->done && hc->stop_iter >= 0) ? hc->stop_iter : o.itr_max;
  const int gbuf = resident ? 0 : (l_final & 1);
  HIP_TRY(dispatch2(dt, lg,
                    [&](auto ops) { return decltype(ops)::finalize(g, b, gbuf, h, s); }));
  if (o.flags & FS1_FLAG_POTENTIALS) {
    const int* ea = lg ? b.eF : nullptr;
    const int* eb = lg ? b.eG[gbuf] : nullptr;
    if (dt == FS1_F64) {
      k_log2<double><<<gf, 256, 0, s>>>(static_cast<const double*>(b.vF),
                                        static_cast<const double*>(b.vG[gbuf]), ea, eb, n,
                                        o.potentials_out);
    } else {
      k_log2<float><<<gf, 256, 0, s>>>(static_cast<const float*>(b.vF),
                                       static_cast<const float*>(b.vG[gbuf]), ea, eb, n,
                                       o.potentials_out);
    }
    HIP_TRY(hipGetLastError());
  }
  double sums[2 + kMaxDim];
  HIP_TRY(hipMemcpyAsync(sums, b.sums, sizeof(double) * (2 + nd), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  out->marginal_err = sums[0];
  out->mu_err = sums[1];
  out->w1 = 0.0;
  for (int a = 0; a < nd; ++a) out->w1 += sums[2 + a];
  out->iterations = l_final;
  out->converged = !(sums[0] > tol) ? 1 : 0;
  return finish((std::isfinite(out->w1) && std::isfinite(out->marginal_err)) ? FS1_OK
                                                                             : FS1_ERR_NONFINITE);
}

int solve_2d(fs1_ctx* ctx, const double* mu, const double* nu, int64_t n1, int64_t n2, double h1,
             double h2, double eps, double tol, const fs1_opts& o, fs1_result* out) {
  const int64_t dims[2] = {n1, n2};
  const double h[2] = {h1, h2};
  return solve_grid(ctx, mu, nu, 2, dims, h, eps, tol, o, out);
}

}  // namespace fs1
