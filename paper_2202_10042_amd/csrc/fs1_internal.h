// fs1_internal.h -- declarations shared by the HIP kernels (fs1_kernels.hip)
// and the host driver (fs1_api.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fs1.h"

namespace fs1 {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kBlock = 256;      // threads per chunk block (4 waves)
constexpr int kCarryBlock = 1024;  // threads of the single-block carry scan
constexpr int kExpZero = -(1 << 30);  // exponent of an exact zero in extended floats

// Extended-range number m * 2^e stored in memory (aggregates, carries).
struct XF64 {
  double m;
  int e;
  int pad;
};

// Forward and backward aggregate (or carry) of one chunk.
//  f: forward state (lower part p of eq. (recursion)) at the chunk's last element
//     when the chunk is fed with zero from the left -- or, as a carry, the
//     forward state at the element just before the chunk;
//  b: inclusive backward state sum_{j>=k} x_j lambda^{j-k} at the chunk's first
//     element k -- or, as a carry, that state at the element just after the chunk.
struct ChunkAgg {
  XF64 f;
  XF64 b;
};

// lambda^D for a fixed distance D, as mantissa * 2^exponent (mantissa in [1,2)).
struct Decay {
  double m;
  int e;
  int pad;
};

// Per-launch constants of the chunk kernels.
struct ScanConsts {
  double lam;        // lambda = exp(-h/eps)
  double mu;         // 1 - lambda (used when lambda > 1/2: lam*a + x = (a+x) - mu*a)
  double c;          // h / eps
  double c_log2e;    // (h/eps) * log2(e): log2 of 1/lambda
  int use_mu;        // 1 when lambda > 1/2
  int R;             // elements per thread run
  Decay lane[7];     // lambda^(R * 2^s), s = 0..6 (s = 6: one wavefront span)
  Decay chunk;       // lambda^(chunk length)
  Decay step1;       // lambda itself (one grid step), in extended range
};

// Constants of the carry scan over chunk aggregates: the single-block scan
// (group chunks per thread) for up to 1024 chunks per thread group, and the
// two-level scan (groups of 1024 chunks, then the groups) beyond.
struct CarryConsts {
  int64_t nchunks;
  int64_t group;     // chunks per thread (single-block scan)
  int64_t chunk_len; // elements per chunk
  Decay chunk;       // lambda^(chunk length)
  Decay step[7];     // lambda^(group * chunk length * 2^s), s = 0..6
  Decay cpow[11];    // lambda^(chunk length * 2^s), s = 0..10
  Decay gstep[7];    // lambda^(1024 * chunk length * 2^s), s = 0..6
  int two_level;     // 1: carries from groups of 1024 chunks, then across groups
  int pad;
};

// What a chunk kernel needs to complete its carry under the two-level scan:
// the group's carry (stored after the chunk carries) moved to the chunk.
struct CarryFix {
  int64_t nchunks;
  int two_level;
  int pad;
  Decay cpow[11];    // lambda^(chunk length * 2^s)
};
CarryFix carry_fix_of(const CarryConsts& kc);

// Bytes of the carry buffer for nchunks chunks: the carries, then the group
// aggregates, group carries and group error shares of the two-level scan.
size_t carry_buffer_bytes(int64_t nchunks);

// Device-side control block of one solve.
struct Ctrl {
  int done;          // 1 once the stopping test is met or a failure is seen
  int stop_iter;     // iteration l at which err(l) <= tol was found (-1 if none)
  int fail;          // a scaling became non-finite
  int fail_iter;     // first iteration whose update produced a non-finite value
  int last_check;    // last iteration whose error was evaluated (-1 if none)
  int barrier_timeout;  // persistent solve: a grid barrier wait gave up
  int iters_done;    // persistent solve: completed iterations at exit
  int fail_half[2];  // persistent solve: failure seen in a psi-half [0] / phi-half [1]
  int absorptions;   // threshold stabilisation: how many times the tau test fired
  double last_err;   // err at last_check
  double w1;         // transport cost (finalisation)
  double err_final;  // nu-side marginal error (finalisation)
  double mu_err;     // mu-side marginal error (finalisation)
  double sum_mu;     // setup: sum of mu
  double sum_nu;     // setup: sum of nu
  int bad_input;     // setup: a marginal entry is negative or non-finite
  int pad2[3];
};

// ---------------------------------------------------------------------------
// Host-side helpers (fs1_kernels.hip)
// ---------------------------------------------------------------------------
Decay make_decay(double D, double c);  // lambda^D = exp(-D c), D a whole number
ScanConsts make_scan_consts(double h, double eps, int R);
CarryConsts make_carry_consts(double h, double eps, int64_t chunk_len, int64_t nchunks);
int pick_run_length(int dtype, bool absorb, double c);  // R for a solve / log apply

// ---------------------------------------------------------------------------
// Launchers (fs1_kernels.hip).  All asynchronous on `s`; return hipError_t.
// ---------------------------------------------------------------------------
// Kernel application, plain values (dtype 0 = double, 1 = float).
hipError_t launch_kv_plain(int dtype, const void* x, void* y, int64_t n, const ScanConsts& k,
                           const CarryConsts& kc, ChunkAgg* agg, ChunkAgg* carry,
                           hipStream_t s);
// Kernel application on logarithms.  special: two ints of scratch (whether an
// input is +inf, whether one is NaN).
hipError_t launch_kv_log(int dtype, const void* lx, void* ly, int64_t n, const ScanConsts& k,
                         const CarryConsts& kc, ChunkAgg* agg, ChunkAgg* carry, int* special,
                         hipStream_t s);

// One exponent for a whole chunk of a vector (the large-grid solver): the
// values are v_j * 2^store, all below 2^frame (frame = kExpZero: all zero).
struct ChunkExp {
  int store;
  int frame;
};

// One solve's device buffers.
struct SolveBufs {
  int dtype;          // 0 double, 1 float
  int absorb;         // 1: log-domain (per-run exponents renormalised every half)
  int64_t n;
  int64_t nchunks;
  int64_t npad;       // nchunks * chunk length: every vector is allocated to whole chunks
  int R;
  const double* mu_src;  // the caller's marginals (read by the set-up only)
  const double* nu_src;
  const double* mu;   // binary64 copies, zero-padded to npad
  const double* nu;
  void* mu32;         // float copies (dtype 1), zero-padded
  void* nu32;
  void* vF;           // phi values (npad)
  void* vG[2];        // psi values, double-buffered (npad)
  int* eF;            // phi run exponents (nruns)
  int* eG[2];         // psi run exponents
  ChunkExp* xF;       // phi chunk exponents (large-grid solver; nchunks)
  ChunkExp* xG[2];    // psi chunk exponents
  void* lanetab;      // lane-dependent decays of the large-grid solver (64 x 32 bytes)
  ChunkAgg* aggF;     // chunk aggregates of phi
  ChunkAgg* aggG;     // chunk aggregates of psi
  ChunkAgg* carry;    // chunk carries of the current half
  void* agg2;         // two-state chunk aggregates (transport cost)
  void* carry2;       // two-state chunk carries (transport cost)
  XF64* dtab;         // lambda^(chunk length * d), d < nchunks (fused / persistent carries)
  double* part;       // per-chunk partial sums (error / cost)
  double* part2;      // second partial array (mu-side error)
  Ctrl* ctrl;
  double* err_hist;   // optional (itr_max + 1)
  double tau;         // > 0: the threshold-absorption variant (resident solver)
  double inv_eps;     // 1 / eps
};

// Resident solve: the whole solve in one workgroup and one launch, for n <=
// 1024 R.  resident_run_length() gives the run length to use for a grid of n
// whose exponent margin allows runs up to rmax (0: the grid does not fit),
// resident_threads() the workgroup size (256 or 1024, 0 if n does not fit);
// the vectors must be allocated to exactly that many runs.
int resident_run_length(int64_t n, int rmax);
int resident_threads(int64_t n, int R);
// The single solve's workgroup: one wavefront (64 threads) when n <= 64 R,
// 256 threads when n <= 256 R, 512 threads for runs of 16 up to 512 R, else
// resident_threads(); its allocation is max(threads, 256) runs.
int solve_resident_threads(int64_t n, int R);
bool usable_resident(const SolveBufs& b);
hipError_t launch_resident(const SolveBufs& b, const ScanConsts& k, int itr_max, int check_every,
                           double tol, hipStream_t s);

// Persistent solve (all iterations in one cooperative launch; state kept in
// registers).  usable_persistent() tells whether the configuration fits.
bool usable_persistent(const SolveBufs& b, double c);
// epoch: nchunks ints, zero before the launch (per-chunk publication flags)
hipError_t launch_persistent(const SolveBufs& b, const ScanConsts& k, int itr_max,
                             int check_every, double tol, int* epoch, hipStream_t s);

// One launch per half-iteration with in-kernel chunk carries (log domain,
// chunk frame valid, moderate chunk count).
bool usable_fused(const SolveBufs& b, double c);
// Run length for the fused path at this size (0: the fused path does not apply).
int fused_run_length(int dtype, double c, int64_t n);
hipError_t launch_fused_init(const SolveBufs& b, const ScanConsts& k, hipStream_t s);
// b.dtab[d] = lambda^(kBlock * b.R * d) for d < b.nchunks (fused and persistent solvers)
hipError_t launch_decay_table(const SolveBufs& b, const ScanConsts& k, hipStream_t s);
hipError_t launch_fused_half(const SolveBufs& b, const ScanConsts& k, int l, int check,
                             double tol, bool psi, hipStream_t s, hipEvent_t ev0 = nullptr,
                             hipEvent_t ev1 = nullptr);

// The solve's chunk-carry launches (fs1_kernels.hip): mode 1 for a psi-half
// (returns at once when the solve has stopped), mode 2 for a phi-half (closes
// the stopping test of iteration l first).
// k_carry_groups alone (two-level carries; the chunk kernel does the rest).
hipError_t launch_carry_groups(int mode, const ChunkAgg* agg, ChunkAgg* carry,
                               const CarryConsts& kc, Ctrl* ctrl, const double* part, int check,
                               hipStream_t s);
hipError_t launch_solve_carry(int mode, const ChunkAgg* agg, ChunkAgg* carry,
                              const CarryConsts& kc, Ctrl* ctrl, const double* part,
                              double* err_hist, int l, int check, double tol, hipStream_t s);

// Large grids in the log domain (more chunks than the fused path takes, chunk
// frame valid): one k_large launch per half-iteration after the carry
// kernels, vectors in the tile layout with one exponent per chunk.
// launch_large_pack turns vF / vG[0] (per-run exponents) into that form
// before the first half, launch_large_unpack writes the per-run exponents of
// vF / vG[gbuf] back from it after the last.
bool usable_large(const SolveBufs& b, double c);
hipError_t launch_large_pack(const SolveBufs& b, const ScanConsts& k, hipStream_t s);
hipError_t launch_large_unpack(const SolveBufs& b, int gbuf, hipStream_t s);
hipError_t launch_large_half(const SolveBufs& b, const ScanConsts& k, const CarryConsts& kc,
                             int l, int check, double tol, bool psi, hipStream_t s,
                             hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

hipError_t launch_setup(const SolveBufs& b, hipStream_t s);
// Initial state phi = psi = 1/n (warm = false) and phi's chunk aggregates;
// with warm = true only the aggregates (launch_warm has written the state).
hipError_t launch_init_state(const SolveBufs& b, const ScanConsts& k, bool warm, hipStream_t s);
// Warm start from split scalings (m: 2n doubles, e: 2n ints; phi then psi);
// bad input sets bit 1 of ctrl->bad_input.  Resets the control block's
// iteration fields as the initial state does.
hipError_t launch_warm(const SolveBufs& b, const double* m, const int* e, hipStream_t s);
// The asynchronous solve: the control block reset and the error history set
// to NaN by kernels (no memset node in a captured graph); the final psi moved
// to buffer 0 when the device-side iteration count is odd; the result written
// to device memory.
hipError_t launch_async_reset(const SolveBufs& b, double* err_hist, int itr_max, hipStream_t s);
hipError_t launch_select_psi(const SolveBufs& b, int itr_max, hipStream_t s);
hipError_t launch_result(const SolveBufs& b, fs1_result* out, double tol, int itr_max,
                         hipStream_t s);
// Final phi and psi = vG[gbuf] (run layout) in split form into m, e (2n each).
hipError_t launch_state_out(const SolveBufs& b, int gbuf, double* m, int* e, hipStream_t s);
// The fused path iterates on vectors in the tile layout of fs1_tile.h, and so
// does the general path where solve_tiled() (binary64, run length a whole
// number of 16-byte vectors): launch_relayout turns vF, vG[gbuf] and the
// marginal copies (mu, nu and their binary32 copies) into tiles (to_tiles) or
// back, in place.
bool solve_tiled(const SolveBufs& b);
hipError_t launch_relayout(const SolveBufs& b, bool to_tiles, int gbuf, hipStream_t s);
// psi-half of iteration l: psi^{l+1} = nu / (K^T phi^l); error of (phi^l, psi^l)
// when `check`.
// ev0 / ev1 (optional): events recorded just before and just after the
// half-iteration kernel itself (diagnostic timing).
hipError_t launch_half_psi(const SolveBufs& b, const ScanConsts& k, const CarryConsts& kc,
                           int l, int check, double tol, hipStream_t s,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// phi-half of iteration l: phi^{l+1} = mu / (K psi^{l+1}); finalises the error of
// iteration l (when checked) and sets the stop flag.
hipError_t launch_half_phi(const SolveBufs& b, const ScanConsts& k, const CarryConsts& kc,
                           int l, int check, double tol, hipStream_t s,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Final marginal errors and transport cost of (phi, psi = vG[gbuf]).
hipError_t launch_finalize(const SolveBufs& b, const ScanConsts& k, const CarryConsts& kc,
                           int gbuf, double h, hipStream_t s);
// Potentials F = ln phi, G = ln psi into out[0..n), out[n..2n).
hipError_t launch_potentials(const SolveBufs& b, int gbuf, double* out, hipStream_t s);

}  // namespace fs1
