/*
 * fs1_oracle.c -- CPU reference for the FS-1 Sinkhorn method (Liao, Chen, Wang,
 * Bai, Jin, Wu: "Fast Sinkhorn I: an O(N) algorithm for the Wasserstein-1
 * metric", arXiv 2202.10042).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or helper with the
 * GPU library, and the GPU library never calls it.
 *
 * Everything is plain IEEE binary64 (no fast-math), written for readability:
 *   - the dense routines follow the definitions (Sec. 2: the discrete entropic
 *     problem, the scaling form gamma_ij = phi_i K_ij psi_j with
 *     K_ij = exp(-|i-j| h / eps), and the Sinkhorn update that refreshes psi
 *     first and then phi), with K formed entry by entry from its definition;
 *   - the sequential routines follow Sec. 3: the split of row k of K psi into
 *     the lower part p_k and the strict upper part q_k and their first-order
 *     recursions (Qin Jiushao / Horner form), driven by Algorithm 1 (FS-1);
 *   - the log-domain routines are the same iterations written on the
 *     logarithms F = ln(phi), G = ln(psi): the limit of the absorption
 *     stabilisation (Sec. 2, remark on log-domain stabilisation; Sec. 3, remark
 *     on the stabilised FS-1) in which the whole of phi and psi is absorbed at
 *     every step.
 *
 * Readings of points the paper leaves open (zero masses, the stopping rule, the
 * returned value) are stated where they are used.
 *
 * Indices are 0..n-1 here (1..N in the paper).  c = h / eps = -ln(lambda).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_INVALID_ARG (-1)
#define OR_ERR_NONFINITE (-2)
#define OR_ERR_NO_MEMORY (-4)

/* Compensated (Neumaier) summation.  Every long sum in this file is a sum of
 * up to ~1e8 terms that the definitions state exactly; accumulating them in
 * plain binary64 would add an O(n u) error, so they are accumulated with a
 * running compensation term instead. */
typedef struct { double s, c; } nsum;
static void nadd(nsum *a, double t) {
    double u = a->s + t;
    if (fabs(a->s) >= fabs(t)) a->c += (a->s - u) + t;
    else a->c += (t - u) + a->s;
    a->s = u;
}
static double nval(const nsum *a) { return a->s + a->c; }

/* log(exp(a) + exp(b)) with exp(-inf) = 0; never produces NaN for -inf inputs. */
static double lse2(double a, double b) {
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    double m = a > b ? a : b;
    return m + log(exp(a - m) + exp(b - m));
}

/* ------------------------------------------------------------------------- */
/* Kernel application, dense form (definition of K in Sec. 2; the full       */
/* Toeplitz expansion of K psi in Sec. 3).                                   */
/* ------------------------------------------------------------------------- */

/* Table of the n distinct kernel entries e^{-d h / eps}, d = |i - j|. */
static double *kernel_table(int64_t n, double c) {
    double *kd = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!kd) return NULL;
    for (int64_t d = 0; d < n; ++d) kd[d] = exp(-(double)d * c);
    return kd;
}

/* y_i = sum_j e^{-|i-j| h/eps} x_j for the rows listed in `rows` (all rows when
 * rows == NULL; then nrows must equal n and y has length n). */
int or_kv_dense_rows(int64_t n, const double *x, double h, double eps,
                     const int64_t *rows, int64_t nrows, double *y) {
    if (n < 1 || !(h > 0) || !(eps > 0)) return OR_ERR_INVALID_ARG;
    double c = h / eps;
    double *kd = kernel_table(n, c);
    if (!kd) return OR_ERR_NO_MEMORY;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows ? rows[r] : r;
        nsum s = {0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            int64_t d = i > j ? i - j : j - i;
            nadd(&s, kd[d] * x[j]);
        }
        y[r] = nval(&s);
    }
    free(kd);
    return OR_OK;
}

int or_kv_dense(int64_t n, const double *x, double h, double eps, double *y) {
    return or_kv_dense_rows(n, x, h, eps, NULL, n, y);
}

/* ly_i = log sum_j exp(lx_j - |i-j| h/eps), max-shifted; -inf entries allowed. */
int or_kv_log_dense_rows(int64_t n, const double *lx, double h, double eps,
                         const int64_t *rows, int64_t nrows, double *ly) {
    if (n < 1 || !(h > 0) || !(eps > 0)) return OR_ERR_INVALID_ARG;
    double c = h / eps;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows ? rows[r] : r;
        double m = -INFINITY;
        for (int64_t j = 0; j < n; ++j) {
            double d = (double)(i > j ? i - j : j - i);
            double t = lx[j] - d * c;
            if (t > m) m = t;
        }
        if (m == -INFINITY) { ly[r] = -INFINITY; continue; }
        nsum s = {0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            double d = (double)(i > j ? i - j : j - i);
            nadd(&s, exp(lx[j] - d * c - m));
        }
        ly[r] = m + log(nval(&s));
    }
    return OR_OK;
}

int or_kv_log_dense(int64_t n, const double *lx, double h, double eps, double *ly) {
    return or_kv_log_dense_rows(n, lx, h, eps, NULL, n, ly);
}

/* ------------------------------------------------------------------------- */
/* Kernel application by the FS-1 recursions (Sec. 3).                       */
/*   p_0 = x_0,      p_{k+1} = lambda p_k + x_{k+1}        (lower part)      */
/*   q_{n-1} = 0,    q_k = lambda (q_{k+1} + x_{k+1})      (strict upper)    */
/*   (K x)_k = p_k + q_k                                                     */
/* ------------------------------------------------------------------------- */

int or_kv_fs1(int64_t n, const double *x, double h, double eps, double *y) {
    if (n < 1 || !(h > 0) || !(eps > 0)) return OR_ERR_INVALID_ARG;
    double lam = exp(-h / eps);
    double *q = (double *)malloc((size_t)n * sizeof(double));
    if (!q) return OR_ERR_NO_MEMORY;
    q[n - 1] = 0.0;
    for (int64_t k = n - 2; k >= 0; --k) q[k] = lam * (q[k + 1] + x[k + 1]);
    double p = x[0];
    y[0] = p + q[0];
    for (int64_t k = 1; k < n; ++k) {
        p = lam * p + x[k];
        y[k] = p + q[k];
    }
    free(q);
    return OR_OK;
}

/* The same recursions on logarithms: with X = ln x,
 *   A_0 = X_0,        A_{k+1} = lse(A_k - c, X_{k+1})
 *   B_{n-1} = -inf,   B_k = lse(B_{k+1}, X_{k+1}) - c
 *   ln (K x)_k = lse(A_k, B_k). */
int or_kv_fs1_log(int64_t n, const double *lx, double h, double eps, double *ly) {
    if (n < 1 || !(h > 0) || !(eps > 0)) return OR_ERR_INVALID_ARG;
    double c = h / eps;
    double *b = (double *)malloc((size_t)n * sizeof(double));
    if (!b) return OR_ERR_NO_MEMORY;
    b[n - 1] = -INFINITY;
    for (int64_t k = n - 2; k >= 0; --k) {
        double t = lse2(b[k + 1], lx[k + 1]);
        b[k] = (t == -INFINITY) ? -INFINITY : t - c;
    }
    double a = lx[0];
    ly[0] = lse2(a, b[0]);
    for (int64_t k = 1; k < n; ++k) {
        a = lse2(a == -INFINITY ? -INFINITY : a - c, lx[k]);
        ly[k] = lse2(a, b[k]);
    }
    free(b);
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Marginal error and transport cost written as the paper writes them        */
/* (double sums in Algorithm 1: the stopping test and the returned value).   */
/* ------------------------------------------------------------------------- */

/* err = sum_i | psi_i * sum_j phi_j e^{-|i-j|c} - nu_i |  (nu-side L1 error) */
double or_marginal_err_dense(int64_t n, const double *phi, const double *psi,
                             const double *nu, double h, double eps) {
    double c = h / eps;
    double *kd = kernel_table(n, c);
    double *row = (double *)malloc((size_t)n * sizeof(double));
    if (!kd || !row) { free(kd); free(row); return NAN; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        nsum s = {0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            int64_t d = i > j ? i - j : j - i;
            nadd(&s, phi[j] * kd[d]);
        }
        row[i] = fabs(psi[i] * nval(&s) - nu[i]);
    }
    nsum err = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) nadd(&err, row[i]);
    free(kd); free(row);
    return nval(&err);
}

/* W = sum_{i,j} phi_i psi_j e^{-|i-j|c} |i-j| h  (the value Algorithm 1 returns) */
double or_cost_dense(int64_t n, const double *phi, const double *psi, double h,
                     double eps) {
    double c = h / eps;
    double *kd = kernel_table(n, c);
    double *row = (double *)malloc((size_t)n * sizeof(double));
    if (!kd || !row) { free(kd); free(row); return NAN; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        nsum s = {0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            int64_t d = i > j ? i - j : j - i;
            nadd(&s, psi[j] * kd[d] * (double)d * h);
        }
        row[i] = phi[i] * nval(&s);
    }
    nsum w = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) nadd(&w, row[i]);
    free(kd); free(row);
    return nval(&w);
}

/* Log-domain versions of the two sums (phi = e^F, psi = e^G). */
double or_marginal_err_log_dense(int64_t n, const double *F, const double *G,
                                 const double *nu, double h, double eps) {
    double c = h / eps;
    double *row = (double *)malloc((size_t)n * sizeof(double));
    if (!row) return NAN;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        nsum s = {0.0, 0.0};
        if (G[i] != -INFINITY) {
            for (int64_t j = 0; j < n; ++j) {
                double d = (double)(i > j ? i - j : j - i);
                if (F[j] != -INFINITY) nadd(&s, exp(F[j] + G[i] - d * c));
            }
        }
        row[i] = fabs(nval(&s) - nu[i]);
    }
    nsum err = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) nadd(&err, row[i]);
    free(row);
    return nval(&err);
}

double or_cost_log_dense(int64_t n, const double *F, const double *G, double h,
                         double eps) {
    double c = h / eps;
    double *row = (double *)malloc((size_t)n * sizeof(double));
    if (!row) return NAN;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        nsum s = {0.0, 0.0};
        if (F[i] != -INFINITY) {
            for (int64_t j = 0; j < n; ++j) {
                if (G[j] == -INFINITY) continue;
                double d = (double)(i > j ? i - j : j - i);
                nadd(&s, exp(F[i] + G[j] - d * c) * d * h);
            }
        }
        row[i] = nval(&s);
    }
    nsum w = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) nadd(&w, row[i]);
    free(row);
    return nval(&w);
}

/* ------------------------------------------------------------------------- */
/* Pointwise division of the Sinkhorn update (psi = nu / (K^T phi),          */
/* phi = mu / (K psi)).  Reading: a zero marginal entry gives a zero scaling */
/* whatever the denominator; a positive entry over a zero or non-finite      */
/* denominator is the failure the paper calls abnormal termination.          */
/* ------------------------------------------------------------------------- */
static int divide_update(int64_t n, const double *marg, const double *den,
                         double *out) {
    int bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (marg[i] == 0.0) { out[i] = 0.0; continue; }
        double v = marg[i] / den[i];
        if (!isfinite(v)) bad = 1;
        out[i] = v;
    }
    return bad;
}

static int divide_update_log(int64_t n, const double *lmarg, const double *lden,
                             double *out) {
    int bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (lmarg[i] == -INFINITY) { out[i] = -INFINITY; continue; }
        double v = lmarg[i] - lden[i];
        if (!isfinite(v)) bad = 1;
        out[i] = v;
    }
    return bad;
}

/* res layout for every solver: [0] = W (the returned transport cost),
 * [1] = final marginal error, [2] = completed iterations, [3] = status,
 * [4] = 1 if the stopping test was met (err <= tol) else 0. */
static void pack_result(double *res, double w, double err, int64_t it, int st,
                        int conv) {
    res[0] = w;
    res[1] = err;
    res[2] = (double)it;
    res[3] = (double)st;
    res[4] = (double)conv;
}

/* ------------------------------------------------------------------------- */
/* Dense Sinkhorn, linear domain (Sec. 2 update; Algorithm 1's loop, stopping */
/* rule and return value, with K applied as a dense matrix).                  */
/* Loop: while it < itr_max and err(phi, psi) > tol:                          */
/*         psi <- nu / (K^T phi); phi <- mu / (K psi); it++                   */
/* phi, psi: outputs (length n); initial value 1/n each (Algorithm 1).        */
/* ------------------------------------------------------------------------- */
int or_sinkhorn_dense(int64_t n, const double *mu, const double *nu, double h,
                      double eps, double tol, int64_t itr_max, double *phi,
                      double *psi, double *res) {
    if (n < 1 || !(h > 0) || !(eps > 0) || itr_max < 0) return OR_ERR_INVALID_ARG;
    double *den = (double *)malloc((size_t)n * sizeof(double));
    if (!den) return OR_ERR_NO_MEMORY;
    for (int64_t i = 0; i < n; ++i) phi[i] = psi[i] = 1.0 / (double)n;
    int64_t it = 0;
    int st = OR_OK, conv = 0;
    double err = or_marginal_err_dense(n, phi, psi, nu, h, eps);
    while (it < itr_max) {
        if (!(err > tol)) { conv = 1; break; }
        or_kv_dense(n, phi, h, eps, den);           /* K^T phi (K symmetric) */
        if (divide_update(n, nu, den, psi)) { st = OR_ERR_NONFINITE; break; }
        or_kv_dense(n, psi, h, eps, den);           /* K psi */
        if (divide_update(n, mu, den, phi)) { st = OR_ERR_NONFINITE; break; }
        ++it;
        err = or_marginal_err_dense(n, phi, psi, nu, h, eps);
    }
    if (st == OR_OK && it == itr_max && !(err > tol)) conv = 1;
    double w = (st == OR_OK) ? or_cost_dense(n, phi, psi, h, eps) : NAN;
    pack_result(res, w, err, it, st, conv);
    free(den);
    return st;
}

/* Dense Sinkhorn on logarithms: G = ln nu - LSE_i(F_i - |i-j| c), then
 * F = ln mu - LSE_j(G_j - |i-j| c); start F = G = -ln n.  In exact arithmetic
 * the iterates are the logarithms of those of or_sinkhorn_dense. */
int or_sinkhorn_log_dense(int64_t n, const double *mu, const double *nu, double h,
                          double eps, double tol, int64_t itr_max, double *F,
                          double *G, double *res) {
    if (n < 1 || !(h > 0) || !(eps > 0) || itr_max < 0) return OR_ERR_INVALID_ARG;
    double *lmu = (double *)malloc((size_t)n * sizeof(double));
    double *lnu = (double *)malloc((size_t)n * sizeof(double));
    double *lden = (double *)malloc((size_t)n * sizeof(double));
    if (!lmu || !lnu || !lden) { free(lmu); free(lnu); free(lden); return OR_ERR_NO_MEMORY; }
    for (int64_t i = 0; i < n; ++i) {
        lmu[i] = mu[i] > 0 ? log(mu[i]) : -INFINITY;
        lnu[i] = nu[i] > 0 ? log(nu[i]) : -INFINITY;
        F[i] = G[i] = -log((double)n);
    }
    int64_t it = 0;
    int st = OR_OK, conv = 0;
    double err = or_marginal_err_log_dense(n, F, G, nu, h, eps);
    while (it < itr_max) {
        if (!(err > tol)) { conv = 1; break; }
        or_kv_log_dense(n, F, h, eps, lden);
        if (divide_update_log(n, lnu, lden, G)) { st = OR_ERR_NONFINITE; break; }
        or_kv_log_dense(n, G, h, eps, lden);
        if (divide_update_log(n, lmu, lden, F)) { st = OR_ERR_NONFINITE; break; }
        ++it;
        err = or_marginal_err_log_dense(n, F, G, nu, h, eps);
    }
    if (st == OR_OK && it == itr_max && !(err > tol)) conv = 1;
    double w = (st == OR_OK) ? or_cost_log_dense(n, F, G, h, eps) : NAN;
    pack_result(res, w, err, it, st, conv);
    free(lmu); free(lnu); free(lden);
    return st;
}

/* ------------------------------------------------------------------------- */
/* Sequential FS-1 (Algorithm 1): the same loop with every K-product done by  */
/* the Sec. 3 recursions, so each iteration costs O(n).  The stopping test's  */
/* inner sum sum_j phi_j lambda^{|i-j|} is the K^T phi of the recursions.     */
/* The returned double sum is evaluated by two further recursions that follow */
/* from the same splitting of |i-j| into j < i and j > i:                     */
/*   L_0 = 0,       L_{i+1} = lambda (L_i + p_i)         (sum over j <= i)    */
/*   U_{n-1} = 0,   U_{i-1} = lambda (U_i + q_i + psi_i) (sum over j >= i)    */
/* with p, q the lower/strict-upper recursions applied to psi; then           */
/*   W = h sum_i phi_i (L_i + U_i).                                           */
/* ------------------------------------------------------------------------- */
double or_cost_fs1(int64_t n, const double *phi, const double *psi, double h,
                   double eps) {
    double lam = exp(-h / eps);
    double *q = (double *)malloc((size_t)n * sizeof(double));
    double *U = (double *)malloc((size_t)n * sizeof(double));
    if (!q || !U) { free(q); free(U); return NAN; }
    q[n - 1] = 0.0;
    for (int64_t k = n - 2; k >= 0; --k) q[k] = lam * (q[k + 1] + psi[k + 1]);
    U[n - 1] = 0.0;
    for (int64_t i = n - 1; i >= 1; --i) U[i - 1] = lam * (U[i] + q[i] + psi[i]);
    nsum w = {0.0, 0.0};
    double p = 0.0, L = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        p = (i == 0) ? psi[0] : lam * p + psi[i];
        nadd(&w, phi[i] * (L + U[i]));
        L = lam * (L + p);
    }
    free(q); free(U);
    return nval(&w) * h;
}

double or_marginal_err_fs1(int64_t n, const double *phi, const double *psi,
                           const double *nu, double h, double eps) {
    double *ktphi = (double *)malloc((size_t)n * sizeof(double));
    if (!ktphi) return NAN;
    or_kv_fs1(n, phi, h, eps, ktphi);
    nsum err = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) nadd(&err, fabs(psi[i] * ktphi[i] - nu[i]));
    free(ktphi);
    return nval(&err);
}

int or_fs1(int64_t n, const double *mu, const double *nu, double h, double eps,
           double tol, int64_t itr_max, double *phi, double *psi, double *res) {
    if (n < 1 || !(h > 0) || !(eps > 0) || itr_max < 0) return OR_ERR_INVALID_ARG;
    double *den = (double *)malloc((size_t)n * sizeof(double));
    if (!den) return OR_ERR_NO_MEMORY;
    for (int64_t i = 0; i < n; ++i) phi[i] = psi[i] = 1.0 / (double)n;
    int64_t it = 0;
    int st = OR_OK, conv = 0;
    double err = or_marginal_err_fs1(n, phi, psi, nu, h, eps);
    while (it < itr_max) {
        if (!(err > tol)) { conv = 1; break; }
        or_kv_fs1(n, phi, h, eps, den);               /* r + s */
        if (divide_update(n, nu, den, psi)) { st = OR_ERR_NONFINITE; break; }
        or_kv_fs1(n, psi, h, eps, den);               /* p + q */
        if (divide_update(n, mu, den, phi)) { st = OR_ERR_NONFINITE; break; }
        ++it;
        err = or_marginal_err_fs1(n, phi, psi, nu, h, eps);
    }
    if (st == OR_OK && it == itr_max && !(err > tol)) conv = 1;
    double w = (st == OR_OK) ? or_cost_fs1(n, phi, psi, h, eps) : NAN;
    pack_result(res, w, err, it, st, conv);
    free(den);
    return st;
}

/* Log-domain sequential FS-1: the recursions of or_kv_fs1_log inside the
 * same loop; the cost recursions run on logarithms as well:
 *   lnL_0 = -inf,  lnL_{i+1} = lse(lnL_i, A_i) - c
 *   lnU_{n-1} = -inf, lnU_{i-1} = lse(lnU_i, B_i, G_i) - c
 *   W = h sum_i exp(F_i + lse(lnL_i, lnU_i)). */
double or_cost_fs1_log(int64_t n, const double *F, const double *G, double h,
                       double eps) {
    double c = h / eps;
    double *B = (double *)malloc((size_t)n * sizeof(double));
    double *lU = (double *)malloc((size_t)n * sizeof(double));
    if (!B || !lU) { free(B); free(lU); return NAN; }
    B[n - 1] = -INFINITY;
    for (int64_t k = n - 2; k >= 0; --k) {
        double t = lse2(B[k + 1], G[k + 1]);
        B[k] = (t == -INFINITY) ? -INFINITY : t - c;
    }
    lU[n - 1] = -INFINITY;
    for (int64_t i = n - 1; i >= 1; --i) {
        double t = lse2(lse2(lU[i], B[i]), G[i]);
        lU[i - 1] = (t == -INFINITY) ? -INFINITY : t - c;
    }
    nsum w = {0.0, 0.0};
    double A = -INFINITY, lL = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        A = (i == 0) ? G[0] : lse2(A == -INFINITY ? -INFINITY : A - c, G[i]);
        double t = lse2(lL, lU[i]);
        if (F[i] != -INFINITY && t != -INFINITY) nadd(&w, exp(F[i] + t));
        double u = lse2(lL, A);
        lL = (u == -INFINITY) ? -INFINITY : u - c;
    }
    free(B); free(lU);
    return nval(&w) * h;
}

double or_marginal_err_fs1_log(int64_t n, const double *F, const double *G,
                               const double *nu, double h, double eps) {
    double *lk = (double *)malloc((size_t)n * sizeof(double));
    if (!lk) return NAN;
    or_kv_fs1_log(n, F, h, eps, lk);
    nsum err = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        double v = (G[i] == -INFINITY || lk[i] == -INFINITY) ? 0.0 : exp(G[i] + lk[i]);
        nadd(&err, fabs(v - nu[i]));
    }
    free(lk);
    return nval(&err);
}

int or_fs1_log(int64_t n, const double *mu, const double *nu, double h, double eps,
               double tol, int64_t itr_max, double *F, double *G, double *res) {
    if (n < 1 || !(h > 0) || !(eps > 0) || itr_max < 0) return OR_ERR_INVALID_ARG;
    double *lmu = (double *)malloc((size_t)n * sizeof(double));
    double *lnu = (double *)malloc((size_t)n * sizeof(double));
    double *lden = (double *)malloc((size_t)n * sizeof(double));
    if (!lmu || !lnu || !lden) { free(lmu); free(lnu); free(lden); return OR_ERR_NO_MEMORY; }
    for (int64_t i = 0; i < n; ++i) {
        lmu[i] = mu[i] > 0 ? log(mu[i]) : -INFINITY;
        lnu[i] = nu[i] > 0 ? log(nu[i]) : -INFINITY;
        F[i] = G[i] = -log((double)n);
    }
    int64_t it = 0;
    int st = OR_OK, conv = 0;
    double err = or_marginal_err_fs1_log(n, F, G, nu, h, eps);
    while (it < itr_max) {
        if (!(err > tol)) { conv = 1; break; }
        or_kv_fs1_log(n, F, h, eps, lden);
        if (divide_update_log(n, lnu, lden, G)) { st = OR_ERR_NONFINITE; break; }
        or_kv_fs1_log(n, G, h, eps, lden);
        if (divide_update_log(n, lmu, lden, F)) { st = OR_ERR_NONFINITE; break; }
        ++it;
        err = or_marginal_err_fs1_log(n, F, G, nu, h, eps);
    }
    if (st == OR_OK && it == itr_max && !(err > tol)) conv = 1;
    double w = (st == OR_OK) ? or_cost_fs1_log(n, F, G, h, eps) : NAN;
    pack_result(res, w, err, it, st, conv);
    free(lmu); free(lnu); free(lden);
    return st;
}

/* ------------------------------------------------------------------------- */
/* Stabilised FS-1 (Sec. 2 and Sec. 3 remarks on log-domain stabilisation).   */
/* The scalings are kept as phi_i = e^{alpha_i/eps} phit_i and                 */
/* psi_j = e^{beta_j/eps} psit_j, i.e. the kernel is rescaled to               */
/*   Kt = diag(e^{alpha/eps}) K diag(e^{beta/eps})                            */
/* and the iteration runs on (phit, psit).  Whenever the largest entry of     */
/* phit or psit exceeds tau, both are absorbed:                               */
/*   alpha += eps ln phit, beta += eps ln psit, phit = psit = 1                */
/* (the remark writes alpha += ln phi; with K rescaled by e^{alpha/eps} the   */
/* consistent update carries the factor eps).  Entries that are exactly zero  */
/* (zero marginal) stay zero and keep their potential.  The products with Kt  */
/* use the recursions that replace those of Algorithm 1's two products:      */
/*   r_{i+1} = lambda e^{(beta_{i+1}-beta_i)/eps} r_i                          */
/*             + e^{(alpha_{i+1}+beta_{i+1})/eps} phit_{i+1}                   */
/*   s_i     = lambda e^{(beta_i-beta_{i+1})/eps}                              */
/*             (s_{i+1} + e^{(alpha_{i+1}+beta_{i+1})/eps} phit_{i+1})         */
/* and the same with alpha and beta exchanged for p, q (Kt psit).  The        */
/* absorption test runs at the top of every iteration.                         */
/* ------------------------------------------------------------------------- */

/* y = Kt^T x (side = 0: coefficients from beta, the K^T phi of the psi-half)
 * or y = Kt x (side = 1: from alpha).  `own` are the potentials of the
 * output side, `oth` those of the input side: the diagonal factor is
 * e^{(own_k + oth_k)/eps}. */
static void kv_absorbed(int64_t n, const double *x, const double *own, const double *oth,
                        double lam, double eps, double *y) {
    double *s = (double *)malloc((size_t)n * sizeof(double));
    if (!s) return;
    s[n - 1] = 0.0;
    for (int64_t k = n - 2; k >= 0; --k) {
        const double d = exp((own[k + 1] + oth[k + 1]) / eps) * x[k + 1];
        s[k] = lam * exp((own[k] - own[k + 1]) / eps) * (s[k + 1] + d);
    }
    double r = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        const double d = exp((own[k] + oth[k]) / eps) * x[k];
        r = (k == 0) ? d : lam * exp((own[k] - own[k - 1]) / eps) * r + d;
        y[k] = r + s[k];
    }
    free(s);
}

static double maxabs(int64_t n, const double *v) {
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) m = fabs(v[i]) > m ? fabs(v[i]) : m;
    return m;
}

static void absorb(int64_t n, double *pot, double *v, double eps) {
    for (int64_t i = 0; i < n; ++i) {
        if (v[i] > 0.0) {
            pot[i] += eps * log(v[i]);
            v[i] = 1.0;
        }
    }
}

/* Algorithm 1 with the stabilisation.  Outputs: phit, psit (length n),
 * alpha, beta (length n), res as for the other solvers plus res[5] = the
 * number of absorptions.  The returned W and err are those of the true
 * scalings phi = e^{alpha/eps} phit, psi = e^{beta/eps} psit. */
int or_fs1_absorb(int64_t n, const double *mu, const double *nu, double h, double eps,
                  double tol, int64_t itr_max, double tau, double *phit, double *psit,
                  double *alpha, double *beta, double *res) {
    if (n < 1 || !(h > 0) || !(eps > 0) || itr_max < 0 || !(tau > 0)) return OR_ERR_INVALID_ARG;
    const double lam = exp(-h / eps);
    double *den = (double *)malloc((size_t)n * sizeof(double));
    if (!den) return OR_ERR_NO_MEMORY;
    for (int64_t i = 0; i < n; ++i) {
        phit[i] = psit[i] = 1.0 / (double)n;
        alpha[i] = beta[i] = 0.0;
    }
    int64_t it = 0, nabs = 0;
    int st = OR_OK, conv = 0;
    /* err = sum_j | psit_j (Kt^T phit)_j - nu_j | */
    kv_absorbed(n, phit, beta, alpha, lam, eps, den);
    nsum e0 = {0.0, 0.0};
    for (int64_t j = 0; j < n; ++j) nadd(&e0, fabs(psit[j] * den[j] - nu[j]));
    double err = nval(&e0);
    while (it < itr_max) {
        if (!(err > tol)) { conv = 1; break; }
        if (maxabs(n, phit) > tau || maxabs(n, psit) > tau) {
            absorb(n, alpha, phit, eps);
            absorb(n, beta, psit, eps);
            ++nabs;
        }
        kv_absorbed(n, phit, beta, alpha, lam, eps, den);   /* Kt^T phit: r + s */
        if (divide_update(n, nu, den, psit)) { st = OR_ERR_NONFINITE; break; }
        kv_absorbed(n, psit, alpha, beta, lam, eps, den);   /* Kt psit: p + q */
        if (divide_update(n, mu, den, phit)) { st = OR_ERR_NONFINITE; break; }
        ++it;
        kv_absorbed(n, phit, beta, alpha, lam, eps, den);
        nsum e = {0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) nadd(&e, fabs(psit[j] * den[j] - nu[j]));
        err = nval(&e);
    }
    if (st == OR_OK && it == itr_max && !(err > tol)) conv = 1;
    double w = NAN;
    if (st == OR_OK) {
        /* W = sum_{i,j} phi_i psi_j K_ij |i-j| h, each term formed from its
         * logarithm ln phit_i + ln psit_j + (alpha_i + beta_j - |i-j| h)/eps
         * (the factors alone can overflow where their product does not) */
        nsum acc = {0.0, 0.0};
        for (int64_t i = 0; i < n; ++i) {
            if (phit[i] == 0.0) continue;
            for (int64_t j = 0; j < n; ++j) {
                if (psit[j] == 0.0 || i == j) continue;
                const double d = (double)(i > j ? i - j : j - i);
                nadd(&acc, exp(log(phit[i]) + log(psit[j]) + (alpha[i] + beta[j] - d * h) / eps) *
                               d * h);
            }
        }
        w = nval(&acc);
    }
    pack_result(res, w, err, it, st, conv);
    res[5] = (double)nabs;
    free(den);
    return st;
}

/* ========================================================================= */
/* Two dimensions (Sec. 4, Algorithm 2).                                      */
/* Histograms on an n1 x n2 grid, flattened in column-major order: entry      */
/* (i, j) sits at i + n1 j; i runs along the first axis (spacing h1,           */
/* lambda1 = e^{-h1/eps}), j along the second (h2, lambda2 = e^{-h2/eps}).     */
/* The kernel of the 2-D problem is                                            */
/*   K_{(i,j),(k,l)} = exp(-(|i-k| h1 + |j-l| h2) / eps),                      */
/* i.e. the block matrix of Sec. 4 with blocks lambda2^{|j-l|} K0, K0 the 1-D  */
/* kernel of the first axis.                                                   */
/* ========================================================================= */

/* Table of the distinct entries exp(-(di h1 + dj h2)/eps), di < n1, dj < n2:
 * each entry of K is read from it by its two index distances. */
static double *kernel_table2(int64_t n1, int64_t n2, double h1, double h2, double eps) {
    double *t = (double *)malloc((size_t)(n1 * n2) * sizeof(double));
    if (!t) return NULL;
    for (int64_t dj = 0; dj < n2; ++dj)
        for (int64_t di = 0; di < n1; ++di)
            t[di + n1 * dj] = exp(-((double)di * h1 + (double)dj * h2) / eps);
    return t;
}

/* y = K x with K dense (every one of the (n1 n2)^2 entries used). */
int or_kv2_dense(int64_t n1, int64_t n2, const double *x, double h1, double h2,
                 double eps, double *y) {
    if (n1 < 1 || n2 < 1) return OR_ERR_INVALID_ARG;
    double *t = kernel_table2(n1, n2, h1, h2, eps);
    if (!t) return OR_ERR_NO_MEMORY;
    const int64_t n = n1 * n2;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        const int64_t i = r % n1, j = r / n1;
        nsum acc = {0.0, 0.0};
        for (int64_t l = 0; l < n2; ++l) {
            const int64_t dj = l > j ? l - j : j - l;
            for (int64_t k = 0; k < n1; ++k) {
                const int64_t di = k > i ? k - i : i - k;
                nadd(&acc, t[di + n1 * dj] * x[k + n1 * l]);
            }
        }
        y[r] = nval(&acc);
    }
    free(t);
    return OR_OK;
}

/* y = K x by Algorithm 2: K0 (the 1-D recursions of Sec. 3 with h = h1)
 * applied to every column, then the recursions of eq. (2d recursion) across
 * the columns:
 *   r_1 = K0 x_1,  r_{j+1} = lambda2 r_j + K0 x_{j+1},
 *   s_{n2} = 0,    s_j = lambda2 (s_{j+1} + K0 x_{j+1}),
 *   (K x)_j = r_j + s_j   (columns j = 1..n2 in the paper's numbering). */
int or_kv2_fs1(int64_t n1, int64_t n2, const double *x, double h1, double h2,
               double eps, double *y) {
    if (n1 < 1 || n2 < 1) return OR_ERR_INVALID_ARG;
    const double lam2 = exp(-h2 / eps);
    double *kx = (double *)malloc((size_t)(n1 * n2) * sizeof(double));
    double *r = (double *)malloc((size_t)n1 * sizeof(double));
    double *s = (double *)malloc((size_t)(n1 * n2) * sizeof(double));
    if (!kx || !r || !s) { free(kx); free(r); free(s); return OR_ERR_NO_MEMORY; }
    for (int64_t j = 0; j < n2; ++j) or_kv_fs1(n1, x + n1 * j, h1, eps, kx + n1 * j);
    /* backward part s, last column first */
    for (int64_t i = 0; i < n1; ++i) s[i + n1 * (n2 - 1)] = 0.0;
    for (int64_t j = n2 - 2; j >= 0; --j)
        for (int64_t i = 0; i < n1; ++i)
            s[i + n1 * j] = lam2 * (s[i + n1 * (j + 1)] + kx[i + n1 * (j + 1)]);
    /* forward part r, first column first */
    for (int64_t j = 0; j < n2; ++j)
        for (int64_t i = 0; i < n1; ++i) {
            r[i] = (j == 0) ? kx[i] : lam2 * r[i] + kx[i + n1 * j];
            y[i + n1 * j] = r[i] + s[i + n1 * j];
        }
    free(kx); free(r); free(s);
    return OR_OK;
}

/* Algorithm 2's stopping-test sum with K dense:
 *   err = sum_{(i,j)} | psi_(i,j) sum_{(k,l)} K_{(i,j),(k,l)} phi_(k,l) - nu_(i,j) | */
double or_marginal_err2_dense(int64_t n1, int64_t n2, const double *phi, const double *psi,
                              const double *nu, double h1, double h2, double eps) {
    const int64_t n = n1 * n2;
    double *kt = (double *)malloc((size_t)n * sizeof(double));
    if (!kt || or_kv2_dense(n1, n2, phi, h1, h2, eps, kt) != OR_OK) { free(kt); return NAN; }
    nsum err = {0.0, 0.0};
    for (int64_t r = 0; r < n; ++r) nadd(&err, fabs(psi[r] * kt[r] - nu[r]));
    free(kt);
    return nval(&err);
}

double or_marginal_err2_fs1(int64_t n1, int64_t n2, const double *phi, const double *psi,
                            const double *nu, double h1, double h2, double eps) {
    const int64_t n = n1 * n2;
    double *kt = (double *)malloc((size_t)n * sizeof(double));
    if (!kt || or_kv2_fs1(n1, n2, phi, h1, h2, eps, kt) != OR_OK) { free(kt); return NAN; }
    nsum err = {0.0, 0.0};
    for (int64_t r = 0; r < n; ++r) nadd(&err, fabs(psi[r] * kt[r] - nu[r]));
    free(kt);
    return nval(&err);
}

/* Algorithm 2's returned value, literally:
 *   W = sum_{(i,j),(k,l)} phi_(i,j) psi_(k,l) K_{(i,j),(k,l)} (|i-k| h1 + |j-l| h2) */
double or_cost2_dense(int64_t n1, int64_t n2, const double *phi, const double *psi,
                      double h1, double h2, double eps) {
    double *t = kernel_table2(n1, n2, h1, h2, eps);
    if (!t) return NAN;
    const int64_t n = n1 * n2;
    double w = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : w)
    for (int64_t r = 0; r < n; ++r) {
        const int64_t i = r % n1, j = r / n1;
        nsum acc = {0.0, 0.0};
        for (int64_t l = 0; l < n2; ++l) {
            const int64_t dj = l > j ? l - j : j - l;
            for (int64_t k = 0; k < n1; ++k) {
                const int64_t di = k > i ? k - i : i - k;
                nadd(&acc, t[di + n1 * dj] * psi[k + n1 * l] *
                               ((double)di * h1 + (double)dj * h2));
            }
        }
        w += phi[r] * nval(&acc);
    }
    free(t);
    return w;
}

/* (C x)_i = sum_k lambda^{|i-k|} |i-k| x_k by the recursions of or_cost_fs1:
 *   L_0 = 0, L_{i+1} = lambda (L_i + p_i);  U_{n-1} = 0, U_{i-1} = lambda (U_i + q_i + x_i). */
static int cost_kernel_fs1(int64_t n, const double *x, double lam, double *out) {
    double *q = (double *)malloc((size_t)n * sizeof(double));
    double *U = (double *)malloc((size_t)n * sizeof(double));
    if (!q || !U) { free(q); free(U); return OR_ERR_NO_MEMORY; }
    q[n - 1] = 0.0;
    for (int64_t k = n - 2; k >= 0; --k) q[k] = lam * (q[k + 1] + x[k + 1]);
    U[n - 1] = 0.0;
    for (int64_t i = n - 1; i >= 1; --i) U[i - 1] = lam * (U[i] + q[i] + x[i]);
    double p = 0.0, L = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        p = (i == 0) ? x[0] : lam * p + x[i];
        out[i] = L + U[i];
        L = lam * (L + p);
    }
    free(q); free(U);
    return OR_OK;
}

/* The same W in O(n1 n2): the cost |i-k| h1 + |j-l| h2 splits the sum into
 *   h1 sum phi . (K2 (x) C1) psi  +  h2 sum phi . (C2 (x) K1) psi,
 * with C_a the 1-D kernel lambda_a^{|d|} |d| of axis a and K_a its Gibbs
 * kernel, each applied by its recursions along its own axis. */
double or_cost2_fs1(int64_t n1, int64_t n2, const double *phi, const double *psi,
                    double h1, double h2, double eps) {
    const int64_t n = n1 * n2;
    const double lam1 = exp(-h1 / eps), lam2 = exp(-h2 / eps);
    double *a = (double *)malloc((size_t)n * sizeof(double));
    double *row = (double *)malloc((size_t)n2 * sizeof(double));
    double *row2 = (double *)malloc((size_t)n2 * sizeof(double));
    if (!a || !row || !row2) { free(a); free(row); free(row2); return NAN; }
    nsum w1 = {0.0, 0.0}, w2 = {0.0, 0.0};
    /* term 1: C1 along the first axis, then K2 along the second */
    for (int64_t j = 0; j < n2; ++j) cost_kernel_fs1(n1, psi + n1 * j, lam1, a + n1 * j);
    for (int64_t i = 0; i < n1; ++i) {
        for (int64_t j = 0; j < n2; ++j) row[j] = a[i + n1 * j];
        or_kv_fs1(n2, row, h2, eps, row2);
        for (int64_t j = 0; j < n2; ++j) nadd(&w1, phi[i + n1 * j] * row2[j]);
    }
    /* term 2: K1 along the first axis, then C2 along the second */
    for (int64_t j = 0; j < n2; ++j) or_kv_fs1(n1, psi + n1 * j, h1, eps, a + n1 * j);
    for (int64_t i = 0; i < n1; ++i) {
        for (int64_t j = 0; j < n2; ++j) row[j] = a[i + n1 * j];
        cost_kernel_fs1(n2, row, lam2, row2);
        for (int64_t j = 0; j < n2; ++j) nadd(&w2, phi[i + n1 * j] * row2[j]);
    }
    free(a); free(row); free(row2);
    return h1 * nval(&w1) + h2 * nval(&w2);
}

/* Algorithm 2 (2-D FS-1) with K applied densely (dense = 1) or by the
 * recursions (dense = 0): phi = psi = 1/(n1 n2); while it < itr_max and
 * err > tol: psi <- nu / (K^T phi); phi <- mu / (K psi).  Returns W as above. */
static int solve2(int dense, int64_t n1, int64_t n2, const double *mu, const double *nu,
                  double h1, double h2, double eps, double tol, int64_t itr_max,
                  double *phi, double *psi, double *res) {
    if (n1 < 1 || n2 < 1 || !(h1 > 0) || !(h2 > 0) || !(eps > 0) || itr_max < 0)
        return OR_ERR_INVALID_ARG;
    const int64_t n = n1 * n2;
    double *den = (double *)malloc((size_t)n * sizeof(double));
    if (!den) return OR_ERR_NO_MEMORY;
    for (int64_t r = 0; r < n; ++r) phi[r] = psi[r] = 1.0 / (double)n;
    int64_t it = 0;
    int st = OR_OK, conv = 0;
    double err = dense ? or_marginal_err2_dense(n1, n2, phi, psi, nu, h1, h2, eps)
                       : or_marginal_err2_fs1(n1, n2, phi, psi, nu, h1, h2, eps);
    while (it < itr_max) {
        if (!(err > tol)) { conv = 1; break; }
        if (dense) or_kv2_dense(n1, n2, phi, h1, h2, eps, den);   /* K^T phi (K symmetric) */
        else or_kv2_fs1(n1, n2, phi, h1, h2, eps, den);
        if (divide_update(n, nu, den, psi)) { st = OR_ERR_NONFINITE; break; }
        if (dense) or_kv2_dense(n1, n2, psi, h1, h2, eps, den);   /* K psi */
        else or_kv2_fs1(n1, n2, psi, h1, h2, eps, den);
        if (divide_update(n, mu, den, phi)) { st = OR_ERR_NONFINITE; break; }
        ++it;
        err = dense ? or_marginal_err2_dense(n1, n2, phi, psi, nu, h1, h2, eps)
                    : or_marginal_err2_fs1(n1, n2, phi, psi, nu, h1, h2, eps);
    }
    if (st == OR_OK && it == itr_max && !(err > tol)) conv = 1;
    double w = NAN;
    if (st == OR_OK)
        w = dense ? or_cost2_dense(n1, n2, phi, psi, h1, h2, eps)
                  : or_cost2_fs1(n1, n2, phi, psi, h1, h2, eps);
    pack_result(res, w, err, it, st, conv);
    free(den);
    return st;
}

int or_sinkhorn2_dense(int64_t n1, int64_t n2, const double *mu, const double *nu, double h1,
                       double h2, double eps, double tol, int64_t itr_max, double *phi,
                       double *psi, double *res) {
    return solve2(1, n1, n2, mu, nu, h1, h2, eps, tol, itr_max, phi, psi, res);
}

int or_fs1_2d(int64_t n1, int64_t n2, const double *mu, const double *nu, double h1, double h2,
              double eps, double tol, int64_t itr_max, double *phi, double *psi, double *res) {
    return solve2(0, n1, n2, mu, nu, h1, h2, eps, tol, itr_max, phi, psi, res);
}

/* ========================================================================= */
/* Two dimensions on logarithms: Algorithm 2 written on F = ln phi and        */
/* G = ln psi, the limit of the absorption stabilisation (Sec. 2 and Sec. 3   */
/* remarks) in which the whole of phi and psi is absorbed at every step, as   */
/* in one dimension.  Same grid, kernel and layout as above.                  */
/* ========================================================================= */

/* ly = ln K e^lx with K dense: every one of the (n1 n2)^2 terms, max-shifted. */
int or_kv2_log_dense(int64_t n1, int64_t n2, const double *lx, double h1, double h2,
                     double eps, double *ly) {
    if (n1 < 1 || n2 < 1 || !(h1 > 0) || !(h2 > 0) || !(eps > 0)) return OR_ERR_INVALID_ARG;
    const int64_t n = n1 * n2;
    const double c1 = h1 / eps, c2 = h2 / eps;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        const int64_t i = r % n1, j = r / n1;
        double m = -INFINITY;
        for (int64_t l = 0; l < n2; ++l)
            for (int64_t k = 0; k < n1; ++k) {
                const double d = (double)(k > i ? k - i : i - k) * c1 +
                                 (double)(l > j ? l - j : j - l) * c2;
                const double t = lx[k + n1 * l] - d;
                if (t > m) m = t;
            }
        if (m == -INFINITY) { ly[r] = -INFINITY; continue; }
        nsum acc = {0.0, 0.0};
        for (int64_t l = 0; l < n2; ++l)
            for (int64_t k = 0; k < n1; ++k) {
                const double d = (double)(k > i ? k - i : i - k) * c1 +
                                 (double)(l > j ? l - j : j - l) * c2;
                nadd(&acc, exp(lx[k + n1 * l] - d - m));
            }
        ly[r] = m + log(nval(&acc));
    }
    return OR_OK;
}

/* The same product by Algorithm 2's structure: the 1-D log recursions
 * (or_kv_fs1_log, spacing h1) along every column, then (spacing h2) along
 * every row. */
int or_kv2_fs1_log(int64_t n1, int64_t n2, const double *lx, double h1, double h2,
                   double eps, double *ly) {
    if (n1 < 1 || n2 < 1 || !(h1 > 0) || !(h2 > 0) || !(eps > 0)) return OR_ERR_INVALID_ARG;
    const int64_t n = n1 * n2;
    double *t = (double *)malloc((size_t)n * sizeof(double));
    double *row = (double *)malloc((size_t)n2 * sizeof(double));
    double *out = (double *)malloc((size_t)n2 * sizeof(double));
    if (!t || !row || !out) { free(t); free(row); free(out); return OR_ERR_NO_MEMORY; }
    for (int64_t j = 0; j < n2; ++j) or_kv_fs1_log(n1, lx + n1 * j, h1, eps, t + n1 * j);
    for (int64_t i = 0; i < n1; ++i) {
        for (int64_t j = 0; j < n2; ++j) row[j] = t[i + n1 * j];
        or_kv_fs1_log(n2, row, h2, eps, out);
        for (int64_t j = 0; j < n2; ++j) ly[i + n1 * j] = out[j];
    }
    free(t); free(row); free(out);
    return OR_OK;
}

/* err = sum | exp(G + ln K^T e^F) - nu |, with the product dense (dense = 1)
 * or by the recursions. */
static double marginal_err2_log(int dense, int64_t n1, int64_t n2, const double *F,
                                const double *G, const double *nu, double h1, double h2,
                                double eps) {
    const int64_t n = n1 * n2;
    double *lk = (double *)malloc((size_t)n * sizeof(double));
    if (!lk) return NAN;
    if (dense) or_kv2_log_dense(n1, n2, F, h1, h2, eps, lk);
    else or_kv2_fs1_log(n1, n2, F, h1, h2, eps, lk);
    nsum err = {0.0, 0.0};
    for (int64_t r = 0; r < n; ++r) {
        const double v = (G[r] == -INFINITY || lk[r] == -INFINITY) ? 0.0 : exp(G[r] + lk[r]);
        nadd(&err, fabs(v - nu[r]));
    }
    free(lk);
    return nval(&err);
}

double or_marginal_err2_log_dense(int64_t n1, int64_t n2, const double *F, const double *G,
                                  const double *nu, double h1, double h2, double eps) {
    return marginal_err2_log(1, n1, n2, F, G, nu, h1, h2, eps);
}

double or_marginal_err2_fs1_log(int64_t n1, int64_t n2, const double *F, const double *G,
                                const double *nu, double h1, double h2, double eps) {
    return marginal_err2_log(0, n1, n2, F, G, nu, h1, h2, eps);
}

/* Algorithm 2's returned value on logarithms, literally:
 *   W = sum exp(F_(i,j) + G_(k,l) - (|i-k| h1 + |j-l| h2)/eps) (|i-k| h1 + |j-l| h2). */
double or_cost2_log_dense(int64_t n1, int64_t n2, const double *F, const double *G,
                          double h1, double h2, double eps) {
    const int64_t n = n1 * n2;
    double *row = (double *)malloc((size_t)n * sizeof(double));
    if (!row) return NAN;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        const int64_t i = r % n1, j = r / n1;
        nsum acc = {0.0, 0.0};
        if (F[r] != -INFINITY) {
            for (int64_t l = 0; l < n2; ++l)
                for (int64_t k = 0; k < n1; ++k) {
                    const double g = G[k + n1 * l];
                    if (g == -INFINITY) continue;
                    const double d = (double)(k > i ? k - i : i - k) * h1 +
                                     (double)(l > j ? l - j : j - l) * h2;
                    nadd(&acc, exp(F[r] + g - d / eps) * d);
                }
        }
        row[r] = nval(&acc);
    }
    nsum w = {0.0, 0.0};
    for (int64_t r = 0; r < n; ++r) nadd(&w, row[r]);
    free(row);
    return nval(&w);
}

/* out_i = ln sum_k e^{X_k} lambda^{|i-k|} |i-k| along one line, by the
 * logarithmic form of the cost recursions of or_cost_fs1_log:
 *   lnL_0 = -inf, lnL_{i+1} = lse(lnL_i, A_i) - c;
 *   lnU_{n-1} = -inf, lnU_{i-1} = lse(lnU_i, B_i, X_i) - c;
 *   out_i = lse(lnL_i, lnU_i), with A, B the forward and strict backward
 * log recursions of X. */
static int cost_kernel_fs1_log(int64_t n, const double *X, double c, double *out) {
    double *B = (double *)malloc((size_t)n * sizeof(double));
    double *lU = (double *)malloc((size_t)n * sizeof(double));
    if (!B || !lU) { free(B); free(lU); return OR_ERR_NO_MEMORY; }
    B[n - 1] = -INFINITY;
    for (int64_t k = n - 2; k >= 0; --k) {
        const double t = lse2(B[k + 1], X[k + 1]);
        B[k] = (t == -INFINITY) ? -INFINITY : t - c;
    }
    lU[n - 1] = -INFINITY;
    for (int64_t i = n - 1; i >= 1; --i) {
        const double t = lse2(lse2(lU[i], B[i]), X[i]);
        lU[i - 1] = (t == -INFINITY) ? -INFINITY : t - c;
    }
    double A = -INFINITY, lL = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        A = (i == 0) ? X[0] : lse2(A == -INFINITY ? -INFINITY : A - c, X[i]);
        out[i] = lse2(lL, lU[i]);
        const double u = lse2(lL, A);
        lL = (u == -INFINITY) ? -INFINITY : u - c;
    }
    free(B); free(lU);
    return OR_OK;
}

/* The same W in O(n1 n2 (n1 + n2)) at most: the split of or_cost2_fs1,
 *   h1 sum phi . (K2 (x) C1) psi  +  h2 sum phi . (C2 (x) K1) psi,
 * with every product taken on logarithms along its own axis. */
double or_cost2_fs1_log(int64_t n1, int64_t n2, const double *F, const double *G,
                        double h1, double h2, double eps) {
    const int64_t n = n1 * n2;
    const double c1 = h1 / eps, c2 = h2 / eps;
    double *a = (double *)malloc((size_t)n * sizeof(double));
    double *row = (double *)malloc((size_t)n2 * sizeof(double));
    double *row2 = (double *)malloc((size_t)n2 * sizeof(double));
    if (!a || !row || !row2) { free(a); free(row); free(row2); return NAN; }
    nsum w1 = {0.0, 0.0}, w2 = {0.0, 0.0};
    /* term 1: C1 along the first axis, then K2 along the second */
    for (int64_t j = 0; j < n2; ++j) cost_kernel_fs1_log(n1, G + n1 * j, c1, a + n1 * j);
    for (int64_t i = 0; i < n1; ++i) {
        for (int64_t j = 0; j < n2; ++j) row[j] = a[i + n1 * j];
        or_kv_fs1_log(n2, row, h2, eps, row2);
        for (int64_t j = 0; j < n2; ++j) {
            const double f = F[i + n1 * j];
            if (f != -INFINITY && row2[j] != -INFINITY) nadd(&w1, exp(f + row2[j]));
        }
    }
    /* term 2: K1 along the first axis, then C2 along the second */
    for (int64_t j = 0; j < n2; ++j) or_kv_fs1_log(n1, G + n1 * j, h1, eps, a + n1 * j);
    for (int64_t i = 0; i < n1; ++i) {
        for (int64_t j = 0; j < n2; ++j) row[j] = a[i + n1 * j];
        cost_kernel_fs1_log(n2, row, c2, row2);
        for (int64_t j = 0; j < n2; ++j) {
            const double f = F[i + n1 * j];
            if (f != -INFINITY && row2[j] != -INFINITY) nadd(&w2, exp(f + row2[j]));
        }
    }
    free(a); free(row); free(row2);
    return h1 * nval(&w1) + h2 * nval(&w2);
}

/* Algorithm 2 on logarithms with the products dense (dense = 1) or by the
 * recursions: F = G = -ln(n1 n2); while it < itr_max and err > tol:
 * G <- ln nu - ln K^T e^F; F <- ln mu - ln K e^G.  Returns W as above. */
static int solve2_log(int dense, int64_t n1, int64_t n2, const double *mu, const double *nu,
                      double h1, double h2, double eps, double tol, int64_t itr_max,
                      double *F, double *G, double *res) {
    if (n1 < 1 || n2 < 1 || !(h1 > 0) || !(h2 > 0) || !(eps > 0) || itr_max < 0)
        return OR_ERR_INVALID_ARG;
    const int64_t n = n1 * n2;
    double *lmu = (double *)malloc((size_t)n * sizeof(double));
    double *lnu = (double *)malloc((size_t)n * sizeof(double));
    double *lden = (double *)malloc((size_t)n * sizeof(double));
    if (!lmu || !lnu || !lden) { free(lmu); free(lnu); free(lden); return OR_ERR_NO_MEMORY; }
    for (int64_t r = 0; r < n; ++r) {
        lmu[r] = mu[r] > 0 ? log(mu[r]) : -INFINITY;
        lnu[r] = nu[r] > 0 ? log(nu[r]) : -INFINITY;
        F[r] = G[r] = -log((double)n);
    }
    int64_t it = 0;
    int st = OR_OK, conv = 0;
    double err = marginal_err2_log(dense, n1, n2, F, G, nu, h1, h2, eps);
    while (it < itr_max) {
        if (!(err > tol)) { conv = 1; break; }
        if (dense) or_kv2_log_dense(n1, n2, F, h1, h2, eps, lden);  /* K symmetric */
        else or_kv2_fs1_log(n1, n2, F, h1, h2, eps, lden);
        if (divide_update_log(n, lnu, lden, G)) { st = OR_ERR_NONFINITE; break; }
        if (dense) or_kv2_log_dense(n1, n2, G, h1, h2, eps, lden);
        else or_kv2_fs1_log(n1, n2, G, h1, h2, eps, lden);
        if (divide_update_log(n, lmu, lden, F)) { st = OR_ERR_NONFINITE; break; }
        ++it;
        err = marginal_err2_log(dense, n1, n2, F, G, nu, h1, h2, eps);
    }
    if (st == OR_OK && it == itr_max && !(err > tol)) conv = 1;
    double w = NAN;
    if (st == OR_OK)
        w = dense ? or_cost2_log_dense(n1, n2, F, G, h1, h2, eps)
                  : or_cost2_fs1_log(n1, n2, F, G, h1, h2, eps);
    pack_result(res, w, err, it, st, conv);
    free(lmu); free(lnu); free(lden);
    return st;
}

int or_sinkhorn2_log_dense(int64_t n1, int64_t n2, const double *mu, const double *nu,
                           double h1, double h2, double eps, double tol, int64_t itr_max,
                           double *F, double *G, double *res) {
    return solve2_log(1, n1, n2, mu, nu, h1, h2, eps, tol, itr_max, F, G, res);
}

int or_fs1_2d_log(int64_t n1, int64_t n2, const double *mu, const double *nu, double h1,
                  double h2, double eps, double tol, int64_t itr_max, double *F, double *G,
                  double *res) {
    return solve2_log(0, n1, n2, mu, nu, h1, h2, eps, tol, itr_max, F, G, res);
}

/* ========================================================================= */
/* D dimensions (Sec. 4: the construction of the 2-D case carried to any      */
/* number of axes, which the paper states without writing it out).  A         */
/* histogram on an n_0 x ... x n_{D-1} grid is flattened with the first axis  */
/* fastest: entry (i_0, ..., i_{D-1}) at sum_a i_a s_a, s_a = n_0 ... n_{a-1}. */
/* The ground cost is the L1 distance sum_a |i_a - j_a| h_a, so               */
/*   K = K_{D-1} (x) ... (x) K_0,  K_a the 1-D Gibbs kernel of axis a,         */
/* and K x is the 1-D recursions of Sec. 3 along every line of every axis in  */
/* turn (for D = 2 this is Algorithm 2: columns first, then eq. (2d           */
/* recursion) across them).  The cost splits into one term per axis:          */
/*   W = sum_a h_a <phi, (K_{D-1} (x) .. C_a .. (x) K_0) psi>,                 */
/* C_a the 1-D kernel lambda_a^{|d|} |d| applied along axis a.                */
/* ========================================================================= */

#define OR_MAX_DIM 8

static int dims_ok(int ndim, const int64_t *dims, const double *h, double eps, int64_t *n) {
    if (ndim < 1 || ndim > OR_MAX_DIM || !(eps > 0)) return 0;
    int64_t t = 1;
    for (int a = 0; a < ndim; ++a) {
        if (dims[a] < 1 || !(h[a] > 0)) return 0;
        t *= dims[a];
    }
    *n = t;
    return 1;
}

/* L1 distance (in units of eps) between entries r and q of the grid */
static double grid_dist(int ndim, const int64_t *dims, const double *h, int64_t r, int64_t q) {
    double d = 0.0;
    for (int a = 0; a < ndim; ++a) {
        const int64_t i = r % dims[a], j = q % dims[a];
        d += (double)(i > j ? i - j : j - i) * h[a];
        r /= dims[a];
        q /= dims[a];
    }
    return d;
}

/* A 1-D operator on one line of len entries: y = op(x) with spacing h. */
typedef int (*line_op)(int64_t len, const double *x, double h, double eps, double *y);

static int kv_line(int64_t len, const double *x, double h, double eps, double *y) {
    return or_kv_fs1(len, x, h, eps, y);
}
static int cost_line(int64_t len, const double *x, double h, double eps, double *y) {
    return cost_kernel_fs1(len, x, exp(-h / eps), y);
}
static int kv_line_log(int64_t len, const double *x, double h, double eps, double *y) {
    return or_kv_fs1_log(len, x, h, eps, y);
}
static int cost_line_log(int64_t len, const double *x, double h, double eps, double *y) {
    return cost_kernel_fs1_log(len, x, h / eps, y);
}

/* out = op applied along every line of axis a (in and out may be the same
 * array: each line is read whole before it is written). */
static int along_axis(int ndim, const int64_t *dims, int a, const double *in, double *out,
                      line_op op, double h, double eps) {
    int64_t n = 1, s = 1;
    for (int b = 0; b < ndim; ++b) {
        n *= dims[b];
        if (b < a) s *= dims[b];
    }
    const int64_t len = dims[a], nlines = n / len;
    double *x = (double *)malloc((size_t)len * sizeof(double));
    double *y = (double *)malloc((size_t)len * sizeof(double));
    if (!x || !y) { free(x); free(y); return OR_ERR_NO_MEMORY; }
    int st = OR_OK;
    for (int64_t L = 0; L < nlines && st == OR_OK; ++L) {
        const int64_t base = (L % s) + (L / s) * s * len;
        for (int64_t k = 0; k < len; ++k) x[k] = in[base + k * s];
        st = op(len, x, h, eps, y);
        for (int64_t k = 0; k < len; ++k) out[base + k * s] = y[k];
    }
    free(x); free(y);
    return st;
}

/* y = K x with K dense: every one of the n^2 entries formed from its
 * definition exp(-sum_a |i_a - j_a| h_a / eps). */
int or_kvn_dense(int ndim, const int64_t *dims, const double *x, const double *h, double eps,
                 double *y) {
    int64_t n;
    if (!dims_ok(ndim, dims, h, eps, &n)) return OR_ERR_INVALID_ARG;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        nsum acc = {0.0, 0.0};
        for (int64_t q = 0; q < n; ++q)
            nadd(&acc, exp(-grid_dist(ndim, dims, h, r, q) / eps) * x[q]);
        y[r] = nval(&acc);
    }
    return OR_OK;
}

/* y = K x by the 1-D recursions along axis 0, then axis 1, ... */
int or_kvn_fs1(int ndim, const int64_t *dims, const double *x, const double *h, double eps,
               double *y) {
    int64_t n;
    if (!dims_ok(ndim, dims, h, eps, &n)) return OR_ERR_INVALID_ARG;
    memcpy(y, x, (size_t)n * sizeof(double));
    for (int a = 0; a < ndim; ++a) {
        const int st = along_axis(ndim, dims, a, y, y, kv_line, h[a], eps);
        if (st != OR_OK) return st;
    }
    return OR_OK;
}

/* ly = ln K e^lx, dense (max-shifted) */
int or_kvn_log_dense(int ndim, const int64_t *dims, const double *lx, const double *h,
                     double eps, double *ly) {
    int64_t n;
    if (!dims_ok(ndim, dims, h, eps, &n)) return OR_ERR_INVALID_ARG;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        double m = -INFINITY;
        for (int64_t q = 0; q < n; ++q) {
            const double t = lx[q] - grid_dist(ndim, dims, h, r, q) / eps;
            if (t > m) m = t;
        }
        if (m == -INFINITY) { ly[r] = -INFINITY; continue; }
        nsum acc = {0.0, 0.0};
        for (int64_t q = 0; q < n; ++q)
            nadd(&acc, exp(lx[q] - grid_dist(ndim, dims, h, r, q) / eps - m));
        ly[r] = m + log(nval(&acc));
    }
    return OR_OK;
}

/* the same product by the 1-D log recursions along each axis in turn */
int or_kvn_fs1_log(int ndim, const int64_t *dims, const double *lx, const double *h,
                   double eps, double *ly) {
    int64_t n;
    if (!dims_ok(ndim, dims, h, eps, &n)) return OR_ERR_INVALID_ARG;
    memcpy(ly, lx, (size_t)n * sizeof(double));
    for (int a = 0; a < ndim; ++a) {
        const int st = along_axis(ndim, dims, a, ly, ly, kv_line_log, h[a], eps);
        if (st != OR_OK) return st;
    }
    return OR_OK;
}

/* K x (lg: ln K e^x), dense or by the recursions */
static int kvn(int dense, int lg, int ndim, const int64_t *dims, const double *x,
               const double *h, double eps, double *y) {
    if (lg) return dense ? or_kvn_log_dense(ndim, dims, x, h, eps, y)
                         : or_kvn_fs1_log(ndim, dims, x, h, eps, y);
    return dense ? or_kvn_dense(ndim, dims, x, h, eps, y) : or_kvn_fs1(ndim, dims, x, h, eps, y);
}

/* The stopping-test sum err = sum | psi (K^T phi) - nu | (K symmetric) with
 * the product dense or by the recursions; lg: phi, psi are F = ln phi,
 * G = ln psi. */
static double marginal_errn(int dense, int lg, int ndim, const int64_t *dims, const double *phi,
                            const double *psi, const double *nu, const double *h, double eps) {
    int64_t n;
    if (!dims_ok(ndim, dims, h, eps, &n)) return NAN;
    double *kt = (double *)malloc((size_t)n * sizeof(double));
    if (!kt) return NAN;
    if (kvn(dense, lg, ndim, dims, phi, h, eps, kt) != OR_OK) { free(kt); return NAN; }
    nsum err = {0.0, 0.0};
    for (int64_t r = 0; r < n; ++r) {
        double v;
        if (lg) v = (psi[r] == -INFINITY || kt[r] == -INFINITY) ? 0.0 : exp(psi[r] + kt[r]);
        else v = psi[r] * kt[r];
        nadd(&err, fabs(v - nu[r]));
    }
    free(kt);
    return nval(&err);
}

double or_marginal_errn_dense(int ndim, const int64_t *dims, const double *phi,
                              const double *psi, const double *nu, const double *h, double eps) {
    return marginal_errn(1, 0, ndim, dims, phi, psi, nu, h, eps);
}
double or_marginal_errn_fs1(int ndim, const int64_t *dims, const double *phi, const double *psi,
                            const double *nu, const double *h, double eps) {
    return marginal_errn(0, 0, ndim, dims, phi, psi, nu, h, eps);
}
double or_marginal_errn_log_dense(int ndim, const int64_t *dims, const double *F,
                                  const double *G, const double *nu, const double *h,
                                  double eps) {
    return marginal_errn(1, 1, ndim, dims, F, G, nu, h, eps);
}
double or_marginal_errn_fs1_log(int ndim, const int64_t *dims, const double *F, const double *G,
                                const double *nu, const double *h, double eps) {
    return marginal_errn(0, 1, ndim, dims, F, G, nu, h, eps);
}

/* The returned value, literally: W = sum_{r,q} phi_r psi_q K_rq d(r, q)
 * (lg: on logarithms, exp(F_r + G_q - d/eps) d). */
static double costn_dense(int lg, int ndim, const int64_t *dims, const double *phi,
                          const double *psi, const double *h, double eps) {
    int64_t n;
    if (!dims_ok(ndim, dims, h, eps, &n)) return NAN;
    double *row = (double *)malloc((size_t)n * sizeof(double));
    if (!row) return NAN;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        nsum acc = {0.0, 0.0};
        for (int64_t q = 0; q < n; ++q) {
            const double d = grid_dist(ndim, dims, h, r, q);
            if (lg) {
                if (phi[r] == -INFINITY || psi[q] == -INFINITY) continue;
                nadd(&acc, exp(phi[r] + psi[q] - d / eps) * d);
            } else {
                nadd(&acc, phi[r] * psi[q] * exp(-d / eps) * d);
            }
        }
        row[r] = nval(&acc);
    }
    nsum w = {0.0, 0.0};
    for (int64_t r = 0; r < n; ++r) nadd(&w, row[r]);
    free(row);
    return nval(&w);
}

double or_costn_dense(int ndim, const int64_t *dims, const double *phi, const double *psi,
                      const double *h, double eps) {
    return costn_dense(0, ndim, dims, phi, psi, h, eps);
}
double or_costn_log_dense(int ndim, const int64_t *dims, const double *F, const double *G,
                          const double *h, double eps) {
    return costn_dense(1, ndim, dims, F, G, h, eps);
}

/* The same W by the split over the axes: term a applies C_a along axis a
 * and K_b along every other axis b, then takes h_a <phi, .>. */
static double costn_fs1(int lg, int ndim, const int64_t *dims, const double *phi,
                        const double *psi, const double *h, double eps) {
    int64_t n;
    if (!dims_ok(ndim, dims, h, eps, &n)) return NAN;
    double *t = (double *)malloc((size_t)n * sizeof(double));
    if (!t) return NAN;
    double w = 0.0;
    for (int a = 0; a < ndim; ++a) {
        memcpy(t, psi, (size_t)n * sizeof(double));
        for (int b = 0; b < ndim; ++b) {
            line_op op = lg ? (b == a ? cost_line_log : kv_line_log) : (b == a ? cost_line : kv_line);
            if (along_axis(ndim, dims, b, t, t, op, h[b], eps) != OR_OK) { free(t); return NAN; }
        }
        nsum acc = {0.0, 0.0};
        for (int64_t r = 0; r < n; ++r) {
            if (lg) {
                if (phi[r] != -INFINITY && t[r] != -INFINITY) nadd(&acc, exp(phi[r] + t[r]));
            } else {
                nadd(&acc, phi[r] * t[r]);
            }
        }
        w += h[a] * nval(&acc);
    }
    free(t);
    return w;
}

double or_costn_fs1(int ndim, const int64_t *dims, const double *phi, const double *psi,
                    const double *h, double eps) {
    return costn_fs1(0, ndim, dims, phi, psi, h, eps);
}
double or_costn_fs1_log(int ndim, const int64_t *dims, const double *F, const double *G,
                        const double *h, double eps) {
    return costn_fs1(1, ndim, dims, F, G, h, eps);
}

/* Algorithm 2 on D axes with the products dense (dense = 1) or by the
 * recursions; lg: on logarithms (F, G), as the 2-D log form.  phi = psi =
 * 1/n (F = G = -ln n); while it < itr_max and err > tol: psi <- nu / (K^T
 * phi); phi <- mu / (K psi).  Returns W as above. */
static int solve_n(int dense, int lg, int ndim, const int64_t *dims, const double *mu,
                   const double *nu, const double *h, double eps, double tol, int64_t itr_max,
                   double *phi, double *psi, double *res) {
    int64_t n;
    if (!dims_ok(ndim, dims, h, eps, &n) || itr_max < 0) return OR_ERR_INVALID_ARG;
    double *lmu = (double *)malloc((size_t)n * sizeof(double));
    double *lnu = (double *)malloc((size_t)n * sizeof(double));
    double *den = (double *)malloc((size_t)n * sizeof(double));
    if (!lmu || !lnu || !den) { free(lmu); free(lnu); free(den); return OR_ERR_NO_MEMORY; }
    for (int64_t r = 0; r < n; ++r) {
        lmu[r] = mu[r] > 0 ? log(mu[r]) : -INFINITY;
        lnu[r] = nu[r] > 0 ? log(nu[r]) : -INFINITY;
        phi[r] = psi[r] = lg ? -log((double)n) : 1.0 / (double)n;
    }
    int64_t it = 0;
    int st = OR_OK, conv = 0;
    double err = marginal_errn(dense, lg, ndim, dims, phi, psi, nu, h, eps);
    while (it < itr_max) {
        if (!(err > tol)) { conv = 1; break; }
        /* psi-half: K^T phi (K is symmetric) */
        if (kvn(dense, lg, ndim, dims, phi, h, eps, den) != OR_OK ||
            (lg ? divide_update_log(n, lnu, den, psi) : divide_update(n, nu, den, psi))) {
            st = OR_ERR_NONFINITE;
            break;
        }
        /* phi-half: K psi */
        if (kvn(dense, lg, ndim, dims, psi, h, eps, den) != OR_OK ||
            (lg ? divide_update_log(n, lmu, den, phi) : divide_update(n, mu, den, phi))) {
            st = OR_ERR_NONFINITE;
            break;
        }
        ++it;
        err = marginal_errn(dense, lg, ndim, dims, phi, psi, nu, h, eps);
    }
    if (st == OR_OK && it == itr_max && !(err > tol)) conv = 1;
    double w = NAN;
    if (st == OR_OK)
        w = dense ? costn_dense(lg, ndim, dims, phi, psi, h, eps)
                  : costn_fs1(lg, ndim, dims, phi, psi, h, eps);
    pack_result(res, w, err, it, st, conv);
    free(lmu); free(lnu); free(den);
    return st;
}

int or_sinkhornn_dense(int ndim, const int64_t *dims, const double *mu, const double *nu,
                       const double *h, double eps, double tol, int64_t itr_max, double *phi,
                       double *psi, double *res) {
    return solve_n(1, 0, ndim, dims, mu, nu, h, eps, tol, itr_max, phi, psi, res);
}
int or_fs1_nd(int ndim, const int64_t *dims, const double *mu, const double *nu,
              const double *h, double eps, double tol, int64_t itr_max, double *phi,
              double *psi, double *res) {
    return solve_n(0, 0, ndim, dims, mu, nu, h, eps, tol, itr_max, phi, psi, res);
}
int or_sinkhornn_log_dense(int ndim, const int64_t *dims, const double *mu, const double *nu,
                           const double *h, double eps, double tol, int64_t itr_max, double *F,
                           double *G, double *res) {
    return solve_n(1, 1, ndim, dims, mu, nu, h, eps, tol, itr_max, F, G, res);
}
int or_fs1_nd_log(int ndim, const int64_t *dims, const double *mu, const double *nu,
                  const double *h, double eps, double tol, int64_t itr_max, double *F,
                  double *G, double *res) {
    return solve_n(0, 1, ndim, dims, mu, nu, h, eps, tol, itr_max, F, G, res);
}

/* Thread count of the OpenMP loops (timing on a stated number of cores). */
void or_set_num_threads(int k) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(k > 0 ? k : 1);
#else
    (void)k;
#endif
}

/* Number of OpenMP threads the dense routines use (1 without OpenMP). */
int or_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
