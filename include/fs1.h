/*
 * fs1.h -- C ABI of libfs1: FS-1 Sinkhorn iterations for the Wasserstein-1
 * metric on a uniform 1-D grid, on AMD Instinct MI355X (gfx950).
 *
 * Method: Liao, Chen, Wang, Bai, Jin, Wu, "Fast Sinkhorn I: an O(N) algorithm
 * for the Wasserstein-1 metric" (arXiv 2202.10042).  On a uniform grid of
 * spacing h the Gibbs kernel is K_ij = lambda^{|i-j|}, lambda = exp(-h/eps)
 * (Sec. 2, scaling form of the entropic problem; Sec. 3, eq. (NBS_summation)),
 * so every K x is the sum of a forward and a backward first-order recursion
 * (Sec. 3, eq. (recursion)).  libfs1 evaluates those recursions as parallel
 * scans on the GPU.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns an int status: FS1_OK (0) or a negative fs1_status.
 *    No C++ exception crosses this boundary.  After a non-zero status,
 *    fs1_last_error() returns a message for the calling thread.
 *  - Array arguments named as device arrays are device pointers (HIP global
 *    memory) owned by the caller; libfs1 never frees or retains them past the
 *    call.  Host arrays are named as such.
 *  - Device arrays must be 16-byte aligned (any fresh HIP or PyTorch
 *    allocation is); otherwise FS1_ERR_INVALID_ARG.
 *  - Work is ordered on the stream given to fs1_ctx_create (0 = the null
 *    stream).  kv_apply calls are asynchronous; solve calls block until their
 *    result is written to the host struct.
 *  - Argument validation happens before any launch; a failed validation
 *    launches nothing and writes nothing.
 *  - A context is used by one host thread at a time.  Different contexts may
 *    be used concurrently on different streams.
 *  - Indices run 0..n-1 (the paper's 1..N).
 */
#ifndef FS1_H
#define FS1_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FS1_OK = 0,
    FS1_ERR_INVALID_ARG = -1, /* bad size, pointer, alignment, h, eps, tol or marginal */
    FS1_ERR_NONFINITE = -2,   /* a scaling became non-finite ("abnormal termination",
                                 Sec. 5.2 and 5.4 of the paper) */
    FS1_ERR_HIP = -3,         /* a HIP runtime call failed */
    FS1_ERR_NO_MEMORY = -4,   /* device or host allocation failed */
    FS1_ERR_INTERNAL = -5     /* a device-side consistency check failed */
} fs1_status;

typedef enum {
    FS1_F64 = 0, /* binary64 storage and scans */
    FS1_F32 = 1  /* binary32 storage and scans; marginal error, cost and the
                    accumulations that feed them stay binary64 */
} fs1_dtype;

typedef enum {
    FS1_PLAIN = 0, /* Algorithm 1 as printed: scalings phi, psi in plain floating
                      point; overflow/underflow ends the solve with
                      FS1_ERR_NONFINITE */
    FS1_LOG = 1,   /* log-domain stabilised FS-1: phi and psi are kept as
                      e^{alpha} * phi~ with the power-of-two part absorbed into a
                      per-run exponent at every half-iteration (the absorption of
                      the Sec. 2 and Sec. 3 remarks, threshold tau -> 0); results
                      equal the plain iteration in exact arithmetic */
    FS1_ABSORB = 2 /* the stabilised FS-1 of the Sec. 2 and Sec. 3 remarks with
                      a finite threshold: scaled vectors phit, psit in the
                      working precision and binary64 potentials alpha, beta
                      (phi = e^{alpha/eps} phit), both absorbed whenever the
                      largest scaled entry exceeds opts->tau; fs1_solve only;
                      grids of at most 1024 runs in one workgroup, larger ones
                      (or FS1_FLAG_GENERAL / FS1_FLAG_NO_RESIDENT) on the
                      general path; FS1_FLAG_PERSISTENT is FS1_ERR_INVALID_ARG */
} fs1_domain;

typedef struct fs1_ctx fs1_ctx;

/* Device memory from the caller's allocator (e.g. a framework's caching
 * allocator): alloc returns `bytes` of device memory on the context's device,
 * 16-byte aligned, usable on the context's stream (NULL when it has none);
 * free gives back a block alloc returned.  Both are called on the host thread
 * that makes the library call. */
typedef void *(*fs1_alloc_fn)(size_t bytes, void *user);
typedef void (*fs1_free_fn)(void *ptr, void *user);

/* Create a context bound to a HIP stream (hipStream_t passed as void*; NULL =
 * null stream) on the device current at the time of the call.  The context
 * owns its workspace (grown on demand, freed by fs1_ctx_destroy). */
int fs1_ctx_create(void *stream, fs1_ctx **out);
/* As fs1_ctx_create, with every device allocation of the context -- the
 * solve workspace (O(n) scalars plus O(n / chunk) carry words, grown on demand;
 * the old block is freed after the stream has finished with it) and the pool
 * of a server created on it -- taken from alloc and given back through
 * free_fn (by fs1_ctx_destroy, fs1_server_destroy or a workspace regrowth).
 * alloc and free_fn are both given or both NULL (then hipMalloc / hipFree);
 * otherwise FS1_ERR_INVALID_ARG.  Pinned host staging still comes from HIP. */
int fs1_ctx_create_with_allocator(void *stream, fs1_alloc_fn alloc, fs1_free_fn free_fn,
                                  void *user, fs1_ctx **out);
int fs1_ctx_destroy(fs1_ctx *ctx);
/* Rebind the context to another stream (e.g. the caller's current stream). */
int fs1_ctx_set_stream(fs1_ctx *ctx, void *stream);

/* Diagnostic timing for benchmarks.  With enable = k > 0, fs1_solve records
 * HIP events on the context stream around every k-th polling batch of
 * half-iteration launches (sync_every iterations; the psi = nu / K^T phi and
 * phi = mu / K psi updates) in which every launch did its work, and
 * accumulates the batch durations, the number of half-iteration launches and
 * their algorithmic bytes (read the vector fed to K, read the marginal, write
 * the new vector; checked psi-halves also read the old psi and, in binary32
 * mode, the binary64 nu).  The persistent solver is timed as one launch.
 * enable = 0 turns timing off.  Every call resets the counters.  Results of
 * the solve do not change. */
int fs1_ctx_set_profiling(fs1_ctx *ctx, int enable);
/* Accumulated half-iteration kernel time (ms), number of timed launches and
 * algorithmic bytes since profiling was last enabled.  Any pointer may be NULL. */
int fs1_ctx_kernel_stats(fs1_ctx *ctx, double *total_ms, int64_t *launches,
                         double *alg_bytes);

/* Diagnostic STREAM-style copy of `bytes` bytes from src to dst (device
 * arrays, 16-byte aligned, not overlapping; bytes a multiple of 16), the
 * attainable-bandwidth reference for the half-iteration kernels, which read
 * and write whole vectors once per half as a copy does.  flags bit 0: use
 * non-temporal loads and stores.  Asynchronous on the context stream.  Not part
 * of the method. */
int fs1_stream_copy(fs1_ctx *ctx, const void *src, void *dst, int64_t bytes, int flags);

/* Thread-local message describing the last failure on this host thread. */
const char *fs1_last_error(void);
/* Library version string. */
const char *fs1_version(void);

/* ------------------------------------------------------------------------ */
/* Kernel application (Sec. 3: K psi split into the lower part p and the     */
/* strict upper part q, each a first-order recursion; eq. (recursion)).      */
/* ------------------------------------------------------------------------ */

/* y_i = sum_j exp(-|i-j| h/eps) x_j,  i = 0..n-1.
 * x, y: device arrays of n elements of dtype dt (double for FS1_F64, float for
 * FS1_F32); any finite sign; must not overlap.  n >= 1; h > 0, eps > 0 finite;
 * n h / eps <= 1e8.  A non-finite entry of x (inf or NaN) makes the outputs it
 * reaches non-finite (inf or NaN; which one is unspecified).  Asynchronous on
 * the context stream. */
int fs1_kv_apply(fs1_ctx *ctx, const void *x, void *y, int64_t n, double h, double eps,
                 int dt);

/* ly_i = ln sum_j exp(lx_j - |i-j| h/eps): the recursions of eq. (recursion)
 * on logarithms (log-sum-exp semiring), as used by the log-domain stabilised
 * method.  lx, ly: device arrays of n elements of dtype dt; must not overlap.
 * lx may hold -inf (a zero of x); all -inf gives all -inf, never NaN.  Every
 * kernel entry is positive, so a NaN entry makes every output NaN, and
 * otherwise a +inf entry makes every output +inf.  Finite entries must satisfy
 * |lx_j| < 1e8; n h / eps <= 1e8.  Asynchronous on the context stream. */
int fs1_kv_apply_log(fs1_ctx *ctx, const void *lx, void *ly, int64_t n, double h,
                     double eps, int dt);

/* ------------------------------------------------------------------------ */
/* Solve (Algorithm 1, FS-1): psi = nu / (K^T phi), phi = mu / (K psi)       */
/* (Sec. 2, Sinkhorn update, psi first), starting from phi = psi = 1/n,      */
/* while iterations < itr_max and the nu-side marginal error                 */
/*   err = sum_i | psi_i (K^T phi)_i - nu_i |                                */
/* exceeds tol; returns the transport cost                                   */
/*   w1 = sum_{i,j} phi_i psi_j lambda^{|i-j|} |i-j| h.                      */
/* ------------------------------------------------------------------------ */

#define FS1_FLAG_POTENTIALS 1
#define FS1_FLAG_GENERAL 2
#define FS1_FLAG_PERSISTENT 4
#define FS1_FLAG_NO_GRAPH 8
#define FS1_FLAG_NO_RESIDENT 16
#define FS1_FLAG_DEVICE_PARAMS 32
#define FS1_FLAG_SERVER_OVERLAP 64

typedef struct {
    double h;             /* grid spacing; <= 0 selects 1/n                         */
    int32_t itr_max;      /* iteration cap; < 0 selects 10000                       */
    int32_t dtype;        /* fs1_dtype of storage and scans                          */
    int32_t domain;       /* fs1_domain                                              */
    int32_t check_every;  /* evaluate the stopping test every k iterations (k >= 1;
                             1 = Algorithm 1; k > 1 may run up to k-1 iterations
                             past the first point where err <= tol)               */
    int32_t sync_every;   /* host polls the device stop flag every s iterations
                             (performance only; results do not depend on it)      */
    int32_t flags;        /* bit 0 (FS1_FLAG_POTENTIALS): return potentials (see
                             potentials_out).  Solver selection (results agree to
                             rounding): by default a grid of at most 8192
                             entries (fewer where h/eps limits the run length R
                             in the log domain: n <= 1024 R) runs the whole
                             solve in one workgroup and one launch (runs of 8 or
                             16 entries per thread; all domains); otherwise, in
                             FS1_LOG, a
                             grid of at most 1024 chunks whose chunk frame fits
                             the working precision runs one fused kernel per
                             half-iteration; bit 1 (FS1_FLAG_GENERAL) forces the
                             general path (extended-range scans, separate carry
                             kernel); bit 2 (FS1_FLAG_PERSISTENT) asks for the
                             single-launch persistent solver when the grid fits
                             in the registers of the co-resident workgroups;
                             bit 4 (FS1_FLAG_NO_RESIDENT) skips the one-workgroup
                             solver; bit 5 (FS1_FLAG_DEVICE_PARAMS): the eps and tol
                             arrays of fs1_solve_batched(_config) are device
                             memory (copied to the host before any launch)         */
    double *potentials_out; /* device, 2n doubles: F = ln phi (n), then G = ln psi
                             (n), written when flags bit 0 is set; -inf where the
                             scaling is zero                                        */
    double *err_history;  /* device, itr_max + 1 doubles or NULL: err at every
                             checked iteration l (index l), NaN elsewhere         */
    double tau;           /* FS1_ABSORB: absorption threshold on the scaled
                             vectors (> 0, finite; default 1e3)                   */
    /* Scalings in split form: phi_i = m[i] 2^e[i], psi_j = m[n+j] 2^e[n+j]
     * (m: 2n doubles, e: 2n int32, device arrays, 16-byte aligned).        */
    const double *warm_m;   /* warm start: with warm_e, Algorithm 1 starts from
                               these (phi^0, psi^0) instead of 1/n; NULL: 1/n.
                               m finite and >= 0, |e| <= 2^20 (else
                               FS1_ERR_INVALID_ARG); in FS1_PLAIN every m 2^e
                               must be finite in the working precision.  Not
                               with FS1_ABSORB.                                   */
    const int32_t *warm_e;
    double *state_m;        /* the final (phi, psi) in the same split form, or
                               NULL.  Exact: a solve of k iterations followed by a
                               warm-started solve of j more gives the same bits
                               (W, errors, potentials, state) as one solve of
                               k + j iterations with the same dtype, domain and
                               solver flags.                                      */
    int32_t *state_e;
} fs1_opts;

/* Fill *o with the defaults (h = 1/n, itr_max 10000, FS1_F64, FS1_PLAIN, tau 1e3,
 * check_every 1, sync_every 16, no potentials, no history, no warm start, no
 * state output).  fs1_solve_batched, fs1_solve_2d and the server ignore the
 * warm-start and state fields. */
int fs1_opts_default(fs1_opts *o);

typedef struct {
    double w1;            /* transport cost <C, P> at the final (phi, psi)          */
    double marginal_err;  /* nu-side L1 marginal error at the final (phi, psi),
                             binary64                                              */
    double mu_err;        /* mu-side L1 marginal error at the final (phi, psi)       */
    int32_t iterations;   /* completed (psi, phi) pairs                             */
    int32_t converged;    /* 1 if marginal_err <= tol at the returned state         */
    int32_t status;       /* same value as the return code                           */
    int32_t absorptions;  /* FS1_ABSORB: times the tau test fired (else 0)       */
} fs1_result;

/* mu, nu: device binary64 arrays of n entries, finite, >= 0, not all zero,
 * |sum mu - sum nu| <= 1e-10 * sum mu (else FS1_ERR_INVALID_ARG; nothing is
 * renormalised).  eps > 0, tol >= 0.  Blocks until *out (host memory) is
 * written.  Reaching itr_max is not an error (status FS1_OK, converged 0), as in
 * Algorithm 1.  A non-finite or zero-denominator scaling at a positive marginal
 * returns FS1_ERR_NONFINITE with out->iterations = the completed iterations
 * before the failing one. */
int fs1_solve(fs1_ctx *ctx, const double *mu, const double *nu, int64_t n, double eps,
              double tol, const fs1_opts *opts, fs1_result *out);

/* fs1_solve enqueued without any host synchronisation, for stream capture
 * into a HIP graph and for pipelined callers.  The solve is the same (same
 * kernels, same arithmetic, same results); its fs1_result is written to
 * out_dev (device memory, 16-byte aligned) when the stream reaches the end of
 * the solve.  All launches of itr_max iterations are enqueued -- those after
 * the stopping test is met return at once -- so itr_max bounds the work;
 * opts->sync_every and diagnostic timing do not apply.  The marginals are
 * checked on the device: invalid ones give out_dev->status =
 * FS1_ERR_INVALID_ARG (iterations 0, W NaN), a non-finite scaling
 * FS1_ERR_NONFINITE with iterations = the failing iteration.  FS1_ABSORB and
 * FS1_FLAG_PERSISTENT are FS1_ERR_INVALID_ARG.  The return value reports
 * argument errors found on the host and launch failures only.  Under capture
 * nothing is allocated, set by a memset node or synchronised, provided the
 * context's workspace already fits the solve (an earlier call of the same
 * size on the context, outside the capture, grows it); otherwise the call
 * fails with FS1_ERR_INVALID_ARG.  Inputs and outputs must stay valid until
 * the stream has run the solve. */
int fs1_solve_async(fs1_ctx *ctx, const double *mu, const double *nu, int64_t n, double eps,
                    double tol, const fs1_opts *opts, fs1_result *out_dev);

/* fs1_solve on a fixed device workspace, for callers that cannot allocate
 * device memory during the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Arguments, results and errors as
 * fs1_solve, except: the workspace is a library-owned device array of 64 MiB
 * per GPU (allocated with the code object, held until the process ends), so a
 * grid needing more (above about 1.6e6 entries in binary64, 1.8e6 in binary32,
 * 1.16e6 with FS1_ABSORB) fails with FS1_ERR_INVALID_ARG before any launch
 * (the message states the bytes needed); diagnostic timing
 * (fs1_ctx_set_profiling) is not recorded; the context's device must be the
 * current device.  Every call on one GPU uses the same array: calls that
 * overlap on one GPU (other streams or host threads) race; calls in sequence
 * do not.  Allocates no device or pinned host memory. */
int fs1_solve_noalloc(fs1_ctx *ctx, const double *mu, const double *nu, int64_t n, double eps,
                      double tol, const fs1_opts *opts, fs1_result *out);

/* Ragged batch of independent solves (Algorithm 1 per instance).  Instance b
 * occupies [offsets[b], offsets[b+1]) of mu_packed / nu_packed (device
 * binary64; the arrays themselves 16-byte aligned, instances anywhere in them);
 * offsets: host int64 array of B+1 entries, offsets[0] = 0, every instance
 * length >= 1.  eps, tol: host arrays of B entries, each validated as for
 * fs1_solve.  Instance b uses h = 1 / n_b (opts->h is ignored), opts->dtype,
 * itr_max and check_every; potentials and error history are not returned.
 *  - FS1_LOG: every instance advances in the same launches, one per
 *    half-iteration and run-length class, each with its own lambda, stopping
 *    test and iteration count.  opts->sync_every iterations are captured in a
 *    HIP graph that is replayed until every instance has stopped
 *    (FS1_FLAG_NO_GRAPH in opts->flags launches the same kernels directly).  An
 *    instance's run length, reduction order and result depend only on its own
 *    (n, eps, tol, marginals) and opts, not on the rest of the batch.
 *  - FS1_PLAIN: the instances run one after another through fs1_solve; each
 *    must then start on a 16-byte boundary.
 * out: host array of B results.  Blocks until every result is written.  Returns
 * FS1_OK if the call ran (then per-instance failures, including invalid
 * marginals, are in out[b].status), else an error before any launch. */
int fs1_solve_batched(fs1_ctx *ctx, const double *mu_packed, const double *nu_packed,
                      const int64_t *offsets, int32_t B, const double *eps,
                      const double *tol, const fs1_opts *opts, fs1_result *out);

/* fs1_solve_batched (FS1_LOG only) with the configuration of every instance
 * forced: run_length[b] and, with threads[b] = 256 or 1024, the resident form
 * (one workgroup of threads[b] threads for all of instance b's iterations; the
 * instance must then hold at most threads[b] x run_length[b] entries), or
 * threads[b] = 0 (or threads NULL), the shared chunk launches.  run_length and
 * threads are host arrays of B entries.  For the project's tuner, which times
 * candidate configurations with this call and ships the fastest as the table
 * that fs1_solve_batched and the server use.  FS1_ERR_INVALID_ARG if the
 * batched kernels are not built for a pair, an instance does not fit, or h/eps
 * does not allow the run length. */
int fs1_solve_batched_config(fs1_ctx *ctx, const double *mu_packed, const double *nu_packed,
                             const int64_t *offsets, int32_t B, const double *eps,
                             const double *tol, const fs1_opts *opts, const int32_t *run_length,
                             const int32_t *threads, fs1_result *out);

/* ------------------------------------------------------------------------ */
/* Two dimensions (Sec. 4, Algorithm 2).  A histogram on an n1 x n2 grid is   */
/* an array of n1 n2 entries in column-major order: entry (i, j) at          */
/* i + n1 j, i along the first axis (spacing h1), j along the second (h2).   */
/* The kernel is K_{(i,j),(k,l)} = lambda1^{|i-k|} lambda2^{|j-l|},          */
/* lambda_a = exp(-h_a / eps): the block matrix of Sec. 4, applied by the    */
/* 1-D recursions along every column and then eq. (2d recursion) across the  */
/* columns.  1 <= n1, n2 <= 8192; h1, h2 > 0 and finite; eps > 0 and finite; */
/* n_a h_a / eps <= 1e8 on each axis; in the log domain an axis with h/eps    */
/* beyond the bound of runs of 8 holds at most 1024 entries (else             */
/* FS1_ERR_INVALID_ARG before any launch).                                   */
/* ------------------------------------------------------------------------ */

/* y = K x for device arrays x, y of n1 n2 entries of dtype dt (FS1_F64 or
 * FS1_F32), plain arithmetic; x and y must not overlap.  Asynchronous on the
 * context stream. */
int fs1_kv_apply_2d(fs1_ctx *ctx, const void *x, void *y, int64_t n1, int64_t n2, double h1,
                    double h2, double eps, int dt);

/* Algorithm 2 (2-D FS-1): phi = psi = 1/(n1 n2); while iterations < itr_max
 * and err = sum | psi (K^T phi) - nu | > tol: psi = nu / (K^T phi), then
 * phi = mu / (K psi).  Returns the transport cost
 *   w1 = sum phi_(i,j) psi_(k,l) K_{(i,j),(k,l)} (|i-k| h1 + |j-l| h2).
 * mu, nu: device binary64 arrays of n1 n2 entries (column-major), finite,
 * >= 0, equal mass to 1e-10 relative.  opts as for fs1_solve except:
 * opts->h is ignored (h1, h2 given); domain FS1_PLAIN is Algorithm 2's
 * arithmetic, FS1_LOG its stabilised form (the Sec. 3 remark on log-domain
 * stabilisation carried to Algorithm 2: every scaling entry held as a
 * mantissa and a binary exponent, so no product underflows at small eps; the
 * same iterates in exact arithmetic; 16 bytes more workspace per grid
 * point); FS1_ABSORB is FS1_ERR_INVALID_ARG.  A small grid (n1 n2 <= 4096,
 * or up to 8192 in the plain domain where three n1 x n2 arrays fit in LDS;
 * n1 + n2 <= 384 in the plain domain, <= 80 (binary64) or 128 (binary32) in
 * the log domain) runs the whole solve in one workgroup (the paper's
 * sequential recursions, the two directions of a line on two threads) unless
 * FS1_FLAG_NO_RESIDENT is set; other grids run one workgroup per line and
 * pass;
 * potentials_out receives ln phi then
 * ln psi (2 n1 n2 doubles).  Blocking; error behaviour as fs1_solve. */
int fs1_solve_2d(fs1_ctx *ctx, const double *mu, const double *nu, int64_t n1, int64_t n2,
                 double h1, double h2, double eps, double tol, const fs1_opts *opts,
                 fs1_result *out);

/* ------------------------------------------------------------------------ */
/* D dimensions (Sec. 4: the 2-D construction carried to any number of axes,  */
/* which the paper states extends without writing it out).  A histogram on an */
/* n_0 x ... x n_{D-1} grid, 1 <= D <= 4, is an array of n_0 ... n_{D-1}     */
/* entries with the first axis fastest: entry (i_0, ..., i_{D-1}) at          */
/* sum_a i_a n_0 ... n_{a-1}.  The ground cost is sum_a |i_a - j_a| h_a, so   */
/* K = K_{D-1} (x) ... (x) K_0 and K x is the 1-D recursions of Sec. 3 along  */
/* every line of each axis in turn (D = 2: Algorithm 2).  dims and h are host */
/* arrays of D entries: 1 <= dims[a] <= 8192, h[a] > 0 and finite, eps > 0    */
/* and finite, dims[a] h[a] / eps <= 1e8, at most 2^31 - 1 grid points (else  */
/* FS1_ERR_INVALID_ARG before any launch).                                   */
/* ------------------------------------------------------------------------ */

/* y = K x for device arrays x, y of n_0 ... n_{D-1} entries of dtype dt
 * (FS1_F64 or FS1_F32), plain arithmetic; x and y must not overlap.  No
 * workspace (the first axis writes y, the others update it in place).
 * Asynchronous on the context stream. */
int fs1_kv_apply_nd(fs1_ctx *ctx, const void *x, void *y, int ndim, const int64_t *dims,
                    const double *h, double eps, int dt);

/* Algorithm 2 on D axes: phi = psi = 1/n; while iterations < itr_max and
 * err = sum | psi (K^T phi) - nu | > tol: psi = nu / (K^T phi), then
 * phi = mu / (K psi).  Returns w1 = sum phi_r psi_q K_rq (sum_a |r_a - q_a| h_a),
 * evaluated as one term per axis, h_a <phi, (K .. C_a .. K) psi>, C_a the 1-D
 * kernel lambda_a^{|d|} |d| along axis a.  mu, nu: device binary64 arrays of
 * n entries, finite, >= 0, equal mass to 1e-10 relative.  opts, domains
 * (FS1_PLAIN, FS1_LOG) and errors as fs1_solve_2d; for D = 2 this is
 * fs1_solve_2d (the one-workgroup form included), for other D one workgroup
 * per line and pass.  potentials_out receives ln phi then ln psi (2 n
 * doubles).  Blocking. */
int fs1_solve_nd(fs1_ctx *ctx, const double *mu, const double *nu, int ndim, const int64_t *dims,
                 const double *h, double eps, double tol, const fs1_opts *opts,
                 fs1_result *out);

/* ------------------------------------------------------------------------ */
/* Serving: a request loop with continuous batching (a library addition, not */
/* part of the paper).  Each request is one solve as fs1_solve in the log    */
/* domain (h = 1/n).  Requests wait in a queue and are admitted in           */
/* submission order whenever an instance slot and room in the device memory  */
/* budget are free; every step runs a fixed number of iterations of all      */
/* admitted requests in the same launches (as fs1_solve_batched), then       */
/* finalises and frees the requests that stopped.  Scaling vectors stay on   */
/* the device from admission to completion.  A request's result does not     */
/* depend on the other requests or on the step at which it was admitted.     */
/* A server uses its context's stream and is driven by one host thread.      */
/* ------------------------------------------------------------------------ */

typedef struct fs1_server fs1_server;

typedef struct {
    int64_t hbm_budget;      /* bytes of device memory for requests, allocated once
                                by fs1_server_create (>= 16 MiB)                   */
    int32_t max_active;      /* requests on the device at once (>= 1)              */
    int32_t dtype;           /* fs1_dtype of storage and scans                     */
    int32_t itr_max;         /* per request; < 0 selects 10000                     */
    int32_t check_every;     /* as fs1_opts (>= 1)                                  */
    int32_t iters_per_step;  /* iterations per fs1_server_step (>= 1)              */
    int32_t flags;           /* FS1_FLAG_NO_GRAPH: launch the kernels directly
                                instead of replaying a captured graph;
                                FS1_FLAG_SERVER_OVERLAP: fs1_server_step returns
                                once its iterations are enqueued, and the next
                                call finalises the requests they stopped (so the
                                caller's own work between calls overlaps the
                                device's); every request's result is the same  */
} fs1_server_opts;

typedef struct {
    int64_t ticket;          /* as returned by fs1_server_submit                   */
    fs1_result result;       /* status FS1_OK, FS1_ERR_INVALID_ARG (marginals not
                                finite, negative, zero or unequal in mass) or
                                FS1_ERR_NONFINITE                                  */
    int64_t admitted_step;   /* step that admitted the request                     */
    int64_t completed_step;  /* step that completed it                             */
} fs1_completion;

typedef struct {
    int64_t queued;          /* submitted, not yet admitted                        */
    int64_t active;          /* admitted, not yet completed                        */
    int64_t completed;       /* completions produced so far (polled or not)        */
    int64_t steps;           /* fs1_server_step calls that ran                     */
    int64_t bytes_in_use;    /* budget taken by admitted requests                  */
    int64_t bytes_total;     /* budget usable for requests                         */
} fs1_server_info;

/* Defaults: 1 GiB budget, 4096 slots, FS1_F32, itr_max 10000, check_every 1,
 * 16 iterations per step, graphs on. */
int fs1_server_opts_default(fs1_server_opts *o);
/* Create a server on ctx (which must outlive it).  FS1_ERR_NO_MEMORY if the
 * budget cannot be allocated. */
int fs1_server_create(fs1_ctx *ctx, const fs1_server_opts *o, fs1_server **out);
/* Waits for the server's work on the stream, then frees it; requests still
 * queued or active are dropped. */
int fs1_server_destroy(fs1_server *srv);
/* Queue one request.  mu, nu: device binary64 arrays of n entries (any
 * alignment) that must stay valid and unchanged until the request completes;
 * eps and tol as fs1_solve.  FS1_ERR_INVALID_ARG if an argument is invalid or
 * the request could never fit the budget (nothing is queued then).  The
 * marginals themselves are checked on the device at admission; a bad pair
 * completes with status FS1_ERR_INVALID_ARG.  *ticket (may be NULL) receives
 * the request's number, 0, 1, 2, ... in submission order. */
int fs1_server_submit(fs1_server *srv, const double *mu, const double *nu, int64_t n,
                      double eps, double tol, int64_t *ticket);
/* One step: admit queued requests (in order, stopping at the first that does
 * not fit), run iters_per_step iterations of every admitted request, finalise
 * the ones that stopped.  Blocks until the step's work is done.  *completed (may
 * be NULL) receives the number of completions this step produced.  With
 * FS1_FLAG_SERVER_OVERLAP the step first waits for the previous call's
 * iterations and finalises the requests they stopped (those are this call's
 * completions), then admits and enqueues its own iterations and returns. */
int fs1_server_step(fs1_server *srv, int32_t *completed);
/* Move up to max completions, oldest first, into out (host array); *count
 * receives how many. */
int fs1_server_poll(fs1_server *srv, fs1_completion *out, int32_t max, int32_t *count);
int fs1_server_get_info(fs1_server *srv, fs1_server_info *out);

#ifdef __cplusplus
}
#endif
#endif /* FS1_H */
