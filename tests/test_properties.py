"""Property tests of the oracle over random (N, eps, seed): its O(N)
recursions (Sec. 3, eq. (recursion); Algorithm 1) against its dense
definitions (K_ij = lambda^|i-j| written out; Sinkhorn's update of Sec. 2 with
the dense kernel), on small grids.  The two sides share no arithmetic beyond
the marginals, so a wrong index, sign or dropped term in either fails here
for some draw.  Examples are derandomised: every run draws the same cases."""
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_2202_10042_amd import inputs

SETTINGS = settings(max_examples=150, deadline=None, derandomize=True, database=None,
                    suppress_health_check=[HealthCheck.too_slow])

sizes = st.integers(min_value=1, max_value=160)
log_c = st.floats(min_value=math.log(1e-3), max_value=math.log(60.0))
seeds = st.integers(min_value=0, max_value=2 ** 31 - 1)


@SETTINGS
@given(n=sizes, lc=log_c, seed=seeds)
def test_kv_recursion_equals_dense_definition(n, lc, seed):
    c = math.exp(lc)
    h = 1.0 / n
    eps = h / c
    rng = np.random.default_rng(seed)
    x = rng.random(n)
    x[rng.random(n) < 0.2] = 0.0
    y = oracle.kv_fs1(x, h, eps)
    ref = oracle.kv_dense(x, h, eps)
    # non-negative terms: a few ulp per recursion step over at most n steps
    assert np.all(np.abs(y - ref) <= 4 * n * 2.0 ** -53 * ref + 1e-300)


@SETTINGS
@given(n=sizes, lc=st.floats(min_value=math.log(1e-3), max_value=math.log(800.0)), seed=seeds)
def test_log_recursion_equals_dense_logsumexp(n, lc, seed):
    c = math.exp(lc)
    h = 1.0 / n
    eps = h / c
    rng = np.random.default_rng(seed)
    lx = 5.0 * rng.standard_normal(n) + 0.5 * c * np.arange(n) * rng.choice([-1.0, 1.0])
    lx[rng.random(n) < 0.15] = -np.inf
    y = oracle.kv_fs1_log(lx, h, eps)
    ref = oracle.kv_log_dense(lx, h, eps)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(y), fin)
    assert np.all(np.abs(y[fin] - ref[fin]) <= 8 * n * 2.0 ** -53 * (1 + np.abs(ref[fin])))


@SETTINGS
@given(n=st.integers(min_value=2, max_value=64), le=st.floats(min_value=math.log(0.02),
                                                               max_value=math.log(1.0)),
       seed=seeds, its=st.integers(min_value=1, max_value=30))
def test_sequential_fs1_equals_dense_sinkhorn(n, le, seed, its):
    eps = math.exp(le)
    h = 1.0 / n
    mu, nu = inputs.mixture_pair(n, 2, seed % 100000)
    a = oracle.fs1(mu, nu, h, eps, tol=-1.0, itr_max=its)
    b = oracle.sinkhorn_dense(mu, nu, h, eps, tol=-1.0, itr_max=its)
    assert a.iterations == b.iterations
    assert a.w1 == pytest.approx(b.w1, rel=1e-10, abs=1e-300)
    assert a.marginal_err == pytest.approx(b.marginal_err, rel=1e-8, abs=1e-13)
    # the phi-update comes last, so the mu-side marginal holds to rounding
    P = oracle.plan_linear(a.a, a.b, h, eps)
    assert np.max(np.abs(P.sum(axis=1) - mu)) <= 1e-13
    assert a.w1 >= 0.0


@SETTINGS
@given(n=st.integers(min_value=2, max_value=64), le=st.floats(min_value=math.log(1e-3),
                                                               max_value=math.log(0.1)),
       seed=seeds, its=st.integers(min_value=1, max_value=30))
def test_log_fs1_equals_dense_log_sinkhorn(n, le, seed, its):
    eps = math.exp(le)
    h = 1.0 / n
    mu, nu = inputs.mixture_pair(n, 3, seed % 100000)
    a = oracle.fs1_log(mu, nu, h, eps, tol=-1.0, itr_max=its)
    b = oracle.sinkhorn_log_dense(mu, nu, h, eps, tol=-1.0, itr_max=its)
    assert a.iterations == b.iterations
    assert a.w1 == pytest.approx(b.w1, rel=1e-10, abs=1e-300)
    assert a.marginal_err == pytest.approx(b.marginal_err, rel=1e-7, abs=1e-13)


dims_st = st.lists(st.integers(min_value=1, max_value=7), min_size=1, max_size=4)


@settings(max_examples=60, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow])
@given(dims=dims_st, lcs=st.lists(st.floats(min_value=math.log(1e-2), max_value=math.log(40.0)),
                                  min_size=4, max_size=4), seed=seeds)
def test_grid_recursions_equal_dense_definition(dims, lcs, seed):
    # Sec. 4 on D axes: the per-axis recursions against K formed entry by
    # entry, plain and on logarithms, and the split cost against the double sum
    eps = 0.1
    h = [math.exp(lc) * eps for lc in lcs[:len(dims)]]
    rng = np.random.default_rng(seed)
    n = int(np.prod(dims))
    x = rng.random(n) + 0.05
    y = oracle.kvn_fs1(x, dims, h, eps)
    ref = oracle.kvn_dense(x, dims, h, eps)
    assert np.all(np.abs(y - ref) <= 8 * sum(dims) * 2.0 ** -53 * ref + 1e-300)
    ly = oracle.kvn_fs1_log(np.log(x), dims, h, eps)
    lref = oracle.kvn_log_dense(np.log(x), dims, h, eps)
    assert np.all(np.abs(ly - lref) <= 8 * sum(dims) * 2.0 ** -53 * (1 + np.abs(lref)))
    psi = rng.random(n)
    w = oracle.costn_fs1(x, psi, dims, h, eps)
    wd = oracle.costn_dense(x, psi, dims, h, eps)
    assert w == pytest.approx(wd, rel=1e-12, abs=1e-300)
