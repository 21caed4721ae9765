"""Pins for the two-dimensional oracle (Sec. 4, Algorithm 2): facts fixed by
the paper or by the mathematics, independent of the oracle's own code.

Grids are n1 x n2, flattened in column-major order (entry (i, j) at
i + n1 j); the kernel is exp(-(|i-k| h1 + |j-l| h2) / eps).  Every test uses
h1 != h2 and n1 != n2 where it can, so that a swapped axis fails.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

import oracle
from paper_2202_10042_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _k1d(n, h, eps):
    return scipy.linalg.toeplitz(np.exp(-np.arange(n) * (h / eps)))


def _k2d(n1, n2, h1, h2, eps):
    # column-major flattening: the first axis varies fastest, so K = K2 (x) K1
    return np.kron(_k1d(n2, h2, eps), _k1d(n1, h1, eps))


def _dist2d(n1, n2, h1, h2):
    r = np.arange(n1 * n2)
    i, j = r % n1, r // n1
    return np.abs(i[:, None] - i[None, :]) * h1 + np.abs(j[:, None] - j[None, :]) * h2


@pytest.mark.parametrize("n1,n2,h1,h2,eps", [(1, 1, 0.1, 0.2, 0.3), (7, 1, 0.1, 0.2, 0.3),
                                             (1, 6, 0.1, 0.2, 0.3), (9, 5, 0.1, 0.25, 0.2),
                                             (4, 11, 0.3, 0.05, 0.1), (12, 12, 1.0, 1.0, 0.5)])
def test_kv2_against_kronecker_product(n1, n2, h1, h2, eps):
    # Sec. 4: K is the block matrix with blocks lambda2^{|j-l|} K0
    rng = np.random.default_rng(n1 * 31 + n2)
    x = rng.random(n1 * n2)
    ref = _k2d(n1, n2, h1, h2, eps) @ x
    np.testing.assert_allclose(oracle.kv2_dense(x, n1, n2, h1, h2, eps), ref, rtol=1e-13)
    np.testing.assert_allclose(oracle.kv2_fs1(x, n1, n2, h1, h2, eps), ref, rtol=1e-13)


def test_kv2_separable_outer_product():
    # K (a (x) b) = (K1 a) (x) (K2 b): the kernel factorises along the axes
    n1, n2, h1, h2, eps = 17, 6, 0.04, 0.3, 0.15
    rng = np.random.default_rng(3)
    a, b = rng.random(n1), rng.random(n2)
    x = np.outer(b, a).reshape(-1)
    ref = np.outer(_k1d(n2, h2, eps) @ b, _k1d(n1, h1, eps) @ a).reshape(-1)
    np.testing.assert_allclose(oracle.kv2_fs1(x, n1, n2, h1, h2, eps), ref, rtol=1e-13)
    np.testing.assert_allclose(oracle.kv2_dense(x, n1, n2, h1, h2, eps), ref, rtol=1e-13)


@pytest.mark.parametrize("n1,n2", [(1, 1), (6, 1), (1, 5), (7, 4), (5, 9)])
def test_cost2_and_err2_against_numpy(n1, n2):
    h1, h2, eps = 0.2, 0.35, 0.25
    rng = np.random.default_rng(n1 + 7 * n2)
    phi, psi, nu = rng.random(n1 * n2), rng.random(n1 * n2), rng.random(n1 * n2)
    K = _k2d(n1, n2, h1, h2, eps)
    D = _dist2d(n1, n2, h1, h2)
    w = float(phi @ (K * D) @ psi)
    err = float(np.abs(psi * (K.T @ phi) - nu).sum())
    for f in (oracle.cost2_dense, oracle.cost2_fs1):
        assert f(phi, psi, n1, n2, h1, h2, eps) == pytest.approx(w, rel=1e-13, abs=1e-300)
    for f in (oracle.marginal_err2_dense, oracle.marginal_err2_fs1):
        assert f(phi, psi, nu, n1, n2, h1, h2, eps) == pytest.approx(err, rel=1e-13)


@pytest.mark.parametrize("solver", ["sinkhorn2_dense", "fs1_2d"])
def test_2d_reduces_to_1d(solver):
    # a grid with one column (or one row) is the 1-D problem along the other axis
    n = 40
    mu, nu = inputs.mixture_pair(n, 2, 4)
    r1 = oracle.sinkhorn_dense(mu, nu, 0.03, 0.05, tol=0.0, itr_max=15)
    for n1, n2, h1, h2 in ((n, 1, 0.03, 0.7), (1, n, 0.7, 0.03)):
        r = getattr(oracle, solver)(mu, nu, n1, n2, h1, h2, 0.05, tol=0.0, itr_max=15)
        assert r.status == 0 and r.iterations == 15
        assert r.w1 == pytest.approx(r1.w1, rel=1e-12)
        np.testing.assert_allclose(r.a, r1.a, rtol=1e-11)
        np.testing.assert_allclose(r.b, r1.b, rtol=1e-11)


@pytest.mark.parametrize("solver", ["sinkhorn2_dense", "fs1_2d"])
def test_2d_dirac(solver):
    # Dirac marginals: one iteration moves the unit mass exactly, err = 0 and
    # W = |a1 - b1| h1 + |a2 - b2| h2 whatever eps
    n1, n2, h1, h2 = 9, 7, 0.1, 0.15
    mu = np.zeros(n1 * n2)
    nu = np.zeros(n1 * n2)
    a1, a2, b1, b2 = 2, 5, 7, 1
    mu[a1 + n1 * a2] = 1.0
    nu[b1 + n1 * b2] = 1.0
    for eps in (0.5, 0.05):
        r = getattr(oracle, solver)(mu, nu, n1, n2, h1, h2, eps, tol=0.0, itr_max=1)
        assert r.status == 0
        assert r.w1 == pytest.approx(abs(a1 - b1) * h1 + abs(a2 - b2) * h2, rel=1e-12)
        assert r.marginal_err <= 1e-15


@pytest.mark.parametrize("solver", ["sinkhorn2_dense", "fs1_2d"])
def test_2d_product_marginals_split_into_1d(solver):
    # With mu = mu1 (x) mu2 and nu = nu1 (x) nu2 every iterate is a product of
    # the 1-D iterates (the start 1/(n1 n2) = (1/n1)(1/n2) is one, and the
    # update keeps the form because K factorises), so P = P1 (x) P2 and
    # W = W1 sum(P2) + W2 sum(P1) with sum(P_a) = sum(mu_a) = 1 after every
    # phi update: W_2D = W_1D(axis 1) + W_1D(axis 2) at every iteration count.
    n1, n2, h1, h2, eps = 30, 22, 1.0 / 30, 1.0 / 22, 0.02
    m1, v1 = inputs.mixture_pair(n1, 2, 11)
    m2, v2 = inputs.mixture_pair(n2, 3, 13)
    mu = np.outer(m2, m1).reshape(-1)
    nu = np.outer(v2, v1).reshape(-1)
    for its in (1, 4, 25):
        w1 = oracle.sinkhorn_dense(m1, v1, h1, eps, tol=0.0, itr_max=its).w1
        w2 = oracle.sinkhorn_dense(m2, v2, h2, eps, tol=0.0, itr_max=its).w1
        r = getattr(oracle, solver)(mu, nu, n1, n2, h1, h2, eps, tol=0.0, itr_max=its)
        assert r.status == 0
        assert r.w1 == pytest.approx(w1 + w2, rel=1e-11)


def _w1_linprog_2d(mu, nu, n1, n2, h1, h2):
    n = n1 * n2
    D = _dist2d(n1, n2, h1, h2)
    A_eq = np.zeros((2 * n, n * n))
    for r in range(n):
        A_eq[r, r * n:(r + 1) * n] = 1.0
        A_eq[n + r, r::n] = 1.0
    res = scipy.optimize.linprog(D.ravel(), A_eq=A_eq, b_eq=np.concatenate([mu, nu]),
                                 bounds=(0, None), method="highs")
    assert res.status == 0
    return res.fun


def _entropy(p):
    p = p[p > 0]
    return float(-(p * np.log(p)).sum())


@pytest.mark.parametrize("n1,n2,seed", [(3, 3, 0), (4, 2, 1), (3, 4, 2)])
def test_2d_entropic_bound_against_linprog(n1, n2, seed):
    # 0 <= W_eps - W_LP <= eps min(H(mu), H(nu)) at convergence (the 1-D
    # argument carries over: it uses only the marginals and the entropy)
    mu, nu = inputs.paper_uniform_2d(n1, n2, seed)
    h1, h2 = 0.3, 0.2
    w_lp = _w1_linprog_2d(mu, nu, n1, n2, h1, h2)
    for eps in (0.1, 0.03):
        bound = eps * min(_entropy(mu), _entropy(nu))
        for solver in ("sinkhorn2_dense", "fs1_2d"):
            r = getattr(oracle, solver)(mu, nu, n1, n2, h1, h2, eps, tol=1e-14, itr_max=200000)
            assert r.status == 0 and r.converged
            slack = 2 * ((n1 - 1) * h1 + (n2 - 1) * h2) * r.marginal_err
            assert -slack - 1e-14 <= r.w1 - w_lp <= bound + slack + 1e-14


def test_2d_axis_swap_symmetry():
    # transposing both histograms and swapping (h1, h2) is the same problem
    n1, n2, h1, h2, eps = 8, 13, 0.05, 0.12, 0.04
    mu, nu = inputs.paper_uniform_2d(n1, n2, 5)
    muT = mu.reshape(n2, n1).T.reshape(-1)
    nuT = nu.reshape(n2, n1).T.reshape(-1)
    for solver in ("sinkhorn2_dense", "fs1_2d"):
        a = getattr(oracle, solver)(mu, nu, n1, n2, h1, h2, eps, tol=0.0, itr_max=20)
        b = getattr(oracle, solver)(muT, nuT, n2, n1, h2, h1, eps, tol=0.0, itr_max=20)
        assert b.w1 == pytest.approx(a.w1, rel=1e-12)
        np.testing.assert_allclose(b.b, a.b.reshape(n2, n1).T.reshape(-1), rtol=1e-10)


@pytest.mark.parametrize("n", [10, 20])
def test_table3_plan_parity_fs1_vs_dense(n):
    # Sec. 5.3, Table 3: 2-D FS-1 and dense Sinkhorn give plans that differ by
    # binary64 rounding only (the printed ||P_FS1 - P||_F)
    g = json.load(open(os.path.join(GOLDEN, "paper_tables.json")))
    h, eps, its = g["table3_h"], g["table3_eps"], g["table3_iterations"]
    u, v = inputs.paper_uniform_2d(n, n, 0)
    a = oracle.fs1_2d(u, v, n, n, h, h, eps, tol=0.0, itr_max=its)
    b = oracle.sinkhorn2_dense(u, v, n, n, h, h, eps, tol=0.0, itr_max=its)
    assert a.status == 0 and b.status == 0 and a.iterations == its
    diff = np.linalg.norm(oracle.plan2(a.a, a.b, n, n, h, h, eps)
                          - oracle.plan2(b.a, b.b, n, n, h, h, eps))
    assert diff <= 10 * g["table3_plan_diff"][str(n)]
    assert a.w1 == pytest.approx(b.w1, rel=1e-12)


# --------------------------------------------------------------------------
# Algorithm 2 on logarithms (F = ln phi, G = ln psi; the stabilised form)
# --------------------------------------------------------------------------

def _logsumexp_rows(M):
    m = np.max(M, axis=1)
    m = np.where(np.isfinite(m), m, 0.0)
    with np.errstate(divide="ignore"):
        return m + np.log(np.exp(M - m[:, None]).sum(axis=1))


@pytest.mark.parametrize("n1,n2,h1,h2,eps", [(1, 1, 0.1, 0.2, 0.3), (7, 1, 0.1, 0.2, 0.3),
                                             (1, 6, 0.1, 0.2, 0.3), (9, 5, 0.1, 0.25, 0.02),
                                             (4, 11, 0.3, 0.05, 0.001)])
def test_kv2_log_against_logsumexp_of_the_kernel(n1, n2, h1, h2, eps):
    # ln (K e^x) with K_{xy} = exp(-d(x, y)/eps), written as a logsumexp over
    # the distance matrix; -inf entries are zeros of e^x
    rng = np.random.default_rng(n1 * 13 + n2)
    lx = 30.0 * rng.standard_normal(n1 * n2)
    lx[rng.random(n1 * n2) < 0.2] = -np.inf
    D = _dist2d(n1, n2, h1, h2)
    ref = _logsumexp_rows(lx[None, :] - D / eps)
    for f in (oracle.kv2_log_dense, oracle.kv2_fs1_log):
        got = f(lx, n1, n2, h1, h2, eps)
        fin = np.isfinite(ref)
        assert np.array_equal(np.isfinite(got), fin)
        np.testing.assert_allclose(got[fin], ref[fin], rtol=0, atol=1e-12 * (1 + np.abs(ref[fin])).max())


def test_log_2d_equals_plain_2d_where_plain_works():
    # in exact arithmetic the log iterates are the logarithms of the plain ones
    n1, n2, h1, h2, eps = 9, 7, 0.1, 0.15, 0.2
    mu, nu = inputs.paper_uniform_2d(n1, n2, 3)
    for its in (1, 6, 30):
        p = oracle.sinkhorn2_dense(mu, nu, n1, n2, h1, h2, eps, tol=0.0, itr_max=its)
        for solver in ("sinkhorn2_log_dense", "fs1_2d_log"):
            r = getattr(oracle, solver)(mu, nu, n1, n2, h1, h2, eps, tol=0.0, itr_max=its)
            assert r.status == 0 and r.iterations == its
            assert r.w1 == pytest.approx(p.w1, rel=1e-12)
            assert r.marginal_err == pytest.approx(p.marginal_err, rel=1e-9, abs=1e-15)
            np.testing.assert_allclose(r.a, np.log(p.a), rtol=0, atol=1e-12)
            np.testing.assert_allclose(r.b, np.log(p.b), rtol=0, atol=1e-12)


def test_log_2d_small_eps_where_plain_fails():
    # h/eps = 800 along an axis: lambda1 = e^-800 underflows in plain binary64
    # (the plain products lose every transport along that axis); the log
    # forms agree with each other and keep the marginal on the mu side exact
    n1, n2, h1, h2, eps = 12, 5, 0.8, 0.3, 0.001
    mu, nu = inputs.paper_uniform_2d(n1, n2, 7)
    a = oracle.sinkhorn2_log_dense(mu, nu, n1, n2, h1, h2, eps, tol=0.0, itr_max=40)
    b = oracle.fs1_2d_log(mu, nu, n1, n2, h1, h2, eps, tol=0.0, itr_max=40)
    assert a.status == 0 and b.status == 0
    assert b.w1 == pytest.approx(a.w1, rel=1e-11)
    assert b.marginal_err == pytest.approx(a.marginal_err, rel=1e-8, abs=1e-14)
    np.testing.assert_allclose(b.a, a.a, rtol=0, atol=1e-9 * np.abs(a.a).max())
    P = np.exp(a.a[:, None] + a.b[None, :] - _dist2d(n1, n2, h1, h2) / eps)
    np.testing.assert_allclose(P.sum(axis=1), mu, rtol=0, atol=1e-13)


@pytest.mark.parametrize("solver", ["sinkhorn2_log_dense", "fs1_2d_log"])
def test_log_2d_reduces_to_1d(solver):
    n = 40
    mu, nu = inputs.mixture_pair(n, 2, 4)
    r1 = oracle.fs1_log(mu, nu, 0.03, 0.002, tol=0.0, itr_max=15)
    for n1, n2, h1, h2 in ((n, 1, 0.03, 0.7), (1, n, 0.7, 0.03)):
        r = getattr(oracle, solver)(mu, nu, n1, n2, h1, h2, 0.002, tol=0.0, itr_max=15)
        assert r.status == 0 and r.iterations == 15
        assert r.w1 == pytest.approx(r1.w1, rel=1e-11)
        np.testing.assert_allclose(r.a, r1.a, rtol=0, atol=1e-9)


@pytest.mark.parametrize("solver", ["sinkhorn2_log_dense", "fs1_2d_log"])
def test_log_2d_dirac_at_tiny_eps(solver):
    # one iteration moves the unit mass exactly, even where e^{-d/eps} is far
    # below the binary64 range; the potentials then reach d/eps = 1.1e4, whose
    # rounding (d/eps) u = 1.2e-12 bounds the relative accuracy of P
    n1, n2, h1, h2 = 9, 7, 0.1, 0.15
    mu = np.zeros(n1 * n2)
    nu = np.zeros(n1 * n2)
    mu[2 + n1 * 5] = 1.0
    nu[7 + n1 * 1] = 1.0
    for eps in (0.05, 1e-4):
        r = getattr(oracle, solver)(mu, nu, n1, n2, h1, h2, eps, tol=0.0, itr_max=1)
        tol = 16 * (5 * h1 + 4 * h2) / eps * 2.0 ** -53
        assert r.status == 0
        assert r.w1 == pytest.approx(5 * h1 + 4 * h2, rel=max(tol, 1e-14))
        assert r.marginal_err <= max(tol, 1e-15)


@pytest.mark.parametrize("solver", ["sinkhorn2_log_dense", "fs1_2d_log"])
def test_log_2d_product_marginals_split_into_1d(solver):
    # as for the plain form, at an eps where the plain products underflow
    n1, n2, h1, h2, eps = 24, 15, 1.0 / 24, 1.0 / 15, 2e-4
    m1, v1 = inputs.mixture_pair(n1, 2, 11)
    m2, v2 = inputs.mixture_pair(n2, 3, 13)
    mu = np.outer(m2, m1).reshape(-1)
    nu = np.outer(v2, v1).reshape(-1)
    for its in (1, 7):
        w1 = oracle.fs1_log(m1, v1, h1, eps, tol=0.0, itr_max=its).w1
        w2 = oracle.fs1_log(m2, v2, h2, eps, tol=0.0, itr_max=its).w1
        r = getattr(oracle, solver)(mu, nu, n1, n2, h1, h2, eps, tol=0.0, itr_max=its)
        assert r.status == 0
        assert r.w1 == pytest.approx(w1 + w2, rel=1e-10)


def test_log_2d_cost_and_err_against_numpy():
    n1, n2, h1, h2, eps = 6, 8, 0.2, 0.35, 0.01
    rng = np.random.default_rng(5)
    F, G = 3.0 * rng.standard_normal(n1 * n2), 3.0 * rng.standard_normal(n1 * n2)
    F[3] = -np.inf
    G[10] = -np.inf
    nu = rng.random(n1 * n2)
    D = _dist2d(n1, n2, h1, h2)
    P = np.exp(F[:, None] + G[None, :] - D / eps)
    w = float((P * D).sum())
    err = float(np.abs(P.sum(axis=0) - nu).sum())
    for f in (oracle.cost2_log_dense, oracle.cost2_fs1_log):
        assert f(F, G, n1, n2, h1, h2, eps) == pytest.approx(w, rel=1e-12)
    for f in (oracle.marginal_err2_log_dense, oracle.marginal_err2_fs1_log):
        assert f(F, G, nu, n1, n2, h1, h2, eps) == pytest.approx(err, rel=1e-12)
