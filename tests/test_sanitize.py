"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): a small driver calls every entry point on grids from 1 to a
few hundred entries, with row lists at both ends, invalid arguments, the 2-D
forms (plain and log), the forms on 1 to 4 axes and the stabilised solver, and compares the O(n) recursions with the
dense definitions on the way.  Any out-of-bounds access, leak, overflow or
other undefined behaviour aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "fs1_oracle.c")

DRIVER = r'''
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int or_kv_dense_rows(int64_t, const double *, double, double, const int64_t *, int64_t, double *);
int or_kv_dense(int64_t, const double *, double, double, double *);
int or_kv_log_dense_rows(int64_t, const double *, double, double, const int64_t *, int64_t,
                         double *);
int or_kv_log_dense(int64_t, const double *, double, double, double *);
int or_kv_fs1(int64_t, const double *, double, double, double *);
int or_kv_fs1_log(int64_t, const double *, double, double, double *);
int or_sinkhorn_dense(int64_t, const double *, const double *, double, double, double, int64_t,
                      double *, double *, double *);
int or_sinkhorn_log_dense(int64_t, const double *, const double *, double, double, double,
                          int64_t, double *, double *, double *);
int or_fs1(int64_t, const double *, const double *, double, double, double, int64_t, double *,
           double *, double *);
int or_fs1_log(int64_t, const double *, const double *, double, double, double, int64_t,
               double *, double *, double *);
int or_fs1_absorb(int64_t, const double *, const double *, double, double, double, int64_t,
                  double, double *, double *, double *, double *, double *);
int or_kv2_dense(int64_t, int64_t, const double *, double, double, double, double *);
int or_kv2_fs1(int64_t, int64_t, const double *, double, double, double, double *);
int or_sinkhorn2_dense(int64_t, int64_t, const double *, const double *, double, double, double,
                       double, int64_t, double *, double *, double *);
int or_fs1_2d(int64_t, int64_t, const double *, const double *, double, double, double, double,
              int64_t, double *, double *, double *);
int or_sinkhorn2_log_dense(int64_t, int64_t, const double *, const double *, double, double,
                           double, double, int64_t, double *, double *, double *);
int or_fs1_2d_log(int64_t, int64_t, const double *, const double *, double, double, double,
                  double, int64_t, double *, double *, double *);
int or_kvn_dense(int, const int64_t *, const double *, const double *, double, double *);
int or_kvn_fs1(int, const int64_t *, const double *, const double *, double, double *);
int or_kvn_log_dense(int, const int64_t *, const double *, const double *, double, double *);
int or_kvn_fs1_log(int, const int64_t *, const double *, const double *, double, double *);
int or_sinkhornn_dense(int, const int64_t *, const double *, const double *, const double *,
                       double, double, int64_t, double *, double *, double *);
int or_fs1_nd(int, const int64_t *, const double *, const double *, const double *, double,
              double, int64_t, double *, double *, double *);
int or_sinkhornn_log_dense(int, const int64_t *, const double *, const double *, const double *,
                           double, double, int64_t, double *, double *, double *);
int or_fs1_nd_log(int, const int64_t *, const double *, const double *, const double *, double,
                  double, int64_t, double *, double *, double *);
void or_set_num_threads(int);

static uint64_t s = 88172645463325252ull;
static double urand(void) {  /* xorshift64 */
  s ^= s << 13; s ^= s >> 7; s ^= s << 17;
  return (double)(s >> 11) * (1.0 / 9007199254740992.0);
}
static void hist(int64_t n, double *p) {
  double t = 0;
  for (int64_t i = 0; i < n; ++i) { p[i] = 0.05 + urand(); t += p[i]; }
  for (int64_t i = 0; i < n; ++i) p[i] /= t;
}
#define CHECK(c) do { if (!(c)) { printf("check failed line %d\n", __LINE__); return 1; } } while (0)

int main(void) {
  or_set_num_threads(2);
  const int64_t ns[] = {1, 2, 3, 17, 64, 257};
  for (size_t k = 0; k < sizeof ns / sizeof ns[0]; ++k) {
    const int64_t n = ns[k];
    const double h = 1.0 / (double)n;
    double *x = malloc(n * sizeof *x), *y = malloc(n * sizeof *y), *z = malloc(n * sizeof *z);
    double *mu = malloc(n * sizeof *mu), *nu = malloc(n * sizeof *nu);
    double *a = malloc(n * sizeof *a), *b = malloc(n * sizeof *b);
    double *al = malloc(n * sizeof *al), *be = malloc(n * sizeof *be);
    double res[6];
    for (int64_t i = 0; i < n; ++i) x[i] = urand() < 0.2 ? 0.0 : urand();
    const double epss[] = {1e-3, 0.05, 2.0};
    for (int e = 0; e < 3; ++e) {
      const double eps = epss[e];
      CHECK(or_kv_dense(n, x, h, eps, y) == 0);
      CHECK(or_kv_fs1(n, x, h, eps, z) == 0);
      for (int64_t i = 0; i < n; ++i) CHECK(fabs(y[i] - z[i]) <= 1e-12 * y[i] + 1e-300);
      int64_t rows[3] = {0, n / 2, n - 1};
      double yr[3];
      CHECK(or_kv_dense_rows(n, x, h, eps, rows, 3, yr) == 0);
      for (int i = 0; i < 3; ++i) CHECK(yr[i] == y[rows[i]]);
      for (int64_t i = 0; i < n; ++i) x[i] = (urand() < 0.2) ? -INFINITY : 3.0 * urand();
      CHECK(or_kv_log_dense(n, x, h, eps, y) == 0);
      CHECK(or_kv_fs1_log(n, x, h, eps, z) == 0);
      CHECK(or_kv_log_dense_rows(n, x, h, eps, rows, 3, yr) == 0);
      for (int64_t i = 0; i < n; ++i) x[i] = urand();
      hist(n, mu);
      hist(n, nu);
      CHECK(or_sinkhorn_dense(n, mu, nu, h, eps, 1e-9, 20, a, b, res) == 0 || eps < 0.01);
      CHECK(or_fs1(n, mu, nu, h, eps, 1e-9, 20, a, b, res) == 0 || eps < 0.01);
      CHECK(or_sinkhorn_log_dense(n, mu, nu, h, eps, 1e-9, 20, a, b, res) == 0);
      CHECK(or_fs1_log(n, mu, nu, h, eps, 1e-9, 20, a, b, res) == 0);
      CHECK(or_fs1_absorb(n, mu, nu, h, eps, 1e-9, 20, 1e3, a, b, al, be, res) == 0);
    }
    CHECK(or_kv_dense(0, x, h, 0.1, y) != 0);
    CHECK(or_fs1_log(n, mu, nu, h, -1.0, 0.0, 5, a, b, res) != 0);
    free(x); free(y); free(z); free(mu); free(nu); free(a); free(b); free(al); free(be);
  }
  {
    const int64_t n1 = 5, n2 = 7, n = n1 * n2;
    double x[35], y[35], z[35], mu[35], nu[35], a[35], b[35], res[6];
    for (int i = 0; i < n; ++i) x[i] = urand();
    CHECK(or_kv2_dense(n1, n2, x, 0.2, 0.1, 0.05, y) == 0);
    CHECK(or_kv2_fs1(n1, n2, x, 0.2, 0.1, 0.05, z) == 0);
    for (int i = 0; i < n; ++i) CHECK(fabs(y[i] - z[i]) <= 1e-12 * y[i]);
    hist(n, mu);
    hist(n, nu);
    CHECK(or_sinkhorn2_dense(n1, n2, mu, nu, 0.2, 0.1, 0.05, 1e-9, 30, a, b, res) == 0);
    CHECK(or_fs1_2d(n1, n2, mu, nu, 0.2, 0.1, 0.05, 1e-9, 30, a, b, res) == 0);
    CHECK(or_sinkhorn2_log_dense(n1, n2, mu, nu, 0.2, 0.1, 0.01, 1e-9, 30, a, b, res) == 0);
    CHECK(or_fs1_2d_log(n1, n2, mu, nu, 0.2, 0.1, 0.01, 1e-9, 30, a, b, res) == 0);
  }
  {
    /* D axes: 1 to 4, with a singleton axis */
    const int64_t dims_all[4][4] = {{7, 0, 0, 0}, {4, 5, 0, 0}, {3, 1, 4, 0}, {2, 3, 2, 3}};
    const double hs[4] = {0.2, 0.1, 0.3, 0.15};
    for (int d = 1; d <= 4; ++d) {
      const int64_t *dims = dims_all[d - 1];
      int64_t n = 1;
      for (int a2 = 0; a2 < d; ++a2) n *= dims[a2];
      double *x = malloc(n * sizeof *x), *y = malloc(n * sizeof *y), *z = malloc(n * sizeof *z);
      double *mu = malloc(n * sizeof *mu), *nu = malloc(n * sizeof *nu);
      double *a = malloc(n * sizeof *a), *b = malloc(n * sizeof *b);
      double res[6];
      for (int64_t i = 0; i < n; ++i) x[i] = 0.1 + urand();
      CHECK(or_kvn_dense(d, dims, x, hs, 0.07, y) == 0);
      CHECK(or_kvn_fs1(d, dims, x, hs, 0.07, z) == 0);
      for (int64_t i = 0; i < n; ++i) CHECK(fabs(y[i] - z[i]) <= 1e-12 * y[i]);
      for (int64_t i = 0; i < n; ++i) x[i] = (urand() < 0.2) ? -INFINITY : 3.0 * urand();
      CHECK(or_kvn_log_dense(d, dims, x, hs, 0.07, y) == 0);
      CHECK(or_kvn_fs1_log(d, dims, x, hs, 0.07, z) == 0);
      hist(n, mu);
      hist(n, nu);
      CHECK(or_sinkhornn_dense(d, dims, mu, nu, hs, 0.07, 1e-9, 20, a, b, res) == 0);
      CHECK(or_fs1_nd(d, dims, mu, nu, hs, 0.07, 1e-9, 20, a, b, res) == 0);
      CHECK(or_sinkhornn_log_dense(d, dims, mu, nu, hs, 0.01, 1e-9, 20, a, b, res) == 0);
      CHECK(or_fs1_nd_log(d, dims, mu, nu, hs, 0.01, 1e-9, 20, a, b, res) == 0);
      CHECK(or_fs1_nd(d, dims, mu, nu, hs, -1.0, 1e-9, 20, a, b, res) != 0);
      free(x); free(y); free(z); free(mu); free(nu); free(a); free(b);
    }
    const int64_t bad[2] = {3, 0};
    double t[3], u[3];
    CHECK(or_kvn_dense(2, bad, t, hs, 0.1, u) != 0);
    CHECK(or_kvn_fs1(0, bad, t, hs, 0.1, u) != 0);
  }
  printf("ok\n");
  return 0;
}
'''


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    drv = tmp_path / "drv.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "drv"
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off",
           SRC, str(drv), "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("ok")
