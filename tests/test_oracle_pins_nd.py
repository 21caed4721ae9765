"""Pins of the D-dimensional oracle (Sec. 4: Algorithm 2's construction on any
number of axes; the paper states that it extends without writing it out).

Grids n_0 x ... x n_{D-1}, first axis fastest, spacings h_a, L1 ground cost.
Each routine is checked against something other than itself:
  * the dense kernel against a numpy Kronecker product of 1-D kernels built
    here from exp(-|i-j| h / eps);
  * the recursions against the dense kernel (plain and log, with zeros and
    h/eps beyond plain range in the log form);
  * the dense cost against an explicit sum over a distance matrix built here
    from numpy index grids, and the split cost against the dense one;
  * the solvers against the dense solvers, against the closed form of product
    marginals (W = sum over axes of the 1-D values, at every iteration count:
    the iterates of a product problem stay products), against the 1-D and 2-D
    oracles when D is 1 or 2, against an axis permutation of the same problem,
    against singleton axes, and against Dirac marginals at small eps (log form).
"""
import numpy as np
import pytest

import oracle
from paper_2202_10042_amd import inputs

pytestmark = pytest.mark.filterwarnings("ignore")


def _kernel_1d(n, h, eps):
    i = np.arange(n)
    return np.exp(-np.abs(i[:, None] - i[None, :]) * h / eps)


def _kron_kernel(dims, h, eps):
    # first axis fastest: K = K_{D-1} (x) ... (x) K_0
    K = np.ones((1, 1))
    for n, hh in zip(dims, h):
        K = np.kron(_kernel_1d(n, hh, eps), K)
    return K


def _dist(dims, h):
    idx = np.indices(dims[::-1]).reshape(len(dims), -1)[::-1]  # idx[a][r] = i_a of entry r
    d = np.zeros((idx.shape[1], idx.shape[1]))
    for a, hh in enumerate(h):
        d += np.abs(idx[a][:, None] - idx[a][None, :]) * hh
    return d


CASES = [((3, 4, 5), (0.2, 0.1, 0.3), 0.07), ((2, 3, 2, 3), (0.5, 0.2, 0.3, 0.1), 0.2),
         ((7, 1, 6), (0.05, 0.4, 0.02), 0.03), ((5,), (0.1,), 0.05), ((4, 9), (0.3, 0.11), 0.1)]


@pytest.mark.parametrize("dims,h,eps", CASES)
def test_kvn_dense_is_the_kronecker_product(dims, h, eps):
    rng = np.random.default_rng(len(dims))
    x = rng.random(int(np.prod(dims)))
    ref = _kron_kernel(dims, h, eps) @ x
    assert np.allclose(oracle.kvn_dense(x, dims, h, eps), ref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("dims,h,eps", CASES + [((6, 5, 4), (1.0, 0.5, 2.0), 0.01)])
def test_kvn_fs1_against_dense(dims, h, eps):
    rng = np.random.default_rng(7)
    x = rng.random(int(np.prod(dims)))
    x[::5] = 0.0
    a = oracle.kvn_dense(x, dims, h, eps)
    b = oracle.kvn_fs1(x, dims, h, eps)
    assert np.max(np.abs(a - b) / np.maximum(a, 1e-300)) <= 1e-13


@pytest.mark.parametrize("dims,h,eps", CASES + [((6, 5, 4), (1.0, 0.5, 2.0), 1e-3)])
def test_kvn_log_against_dense_and_plain(dims, h, eps):
    rng = np.random.default_rng(11)
    n = int(np.prod(dims))
    lx = rng.normal(0.0, 30.0, n)
    lx[::4] = -np.inf
    a = oracle.kvn_log_dense(lx, dims, h, eps)
    b = oracle.kvn_fs1_log(lx, dims, h, eps)
    fin = np.isfinite(a)
    assert np.array_equal(fin, np.isfinite(b))
    assert np.max(np.abs(a[fin] - b[fin]) / (1.0 + np.abs(a[fin]))) <= 1e-13
    # where plain arithmetic holds the product, the log form is its logarithm
    if max(h) / eps < 50:
        x = np.exp(lx / 30.0)
        y = oracle.kvn_dense(x, dims, h, eps)
        assert np.allclose(oracle.kvn_log_dense(np.log(x), dims, h, eps), np.log(y),
                           rtol=0, atol=1e-13)


@pytest.mark.parametrize("dims,h,eps", CASES)
def test_costn_against_distance_matrix(dims, h, eps):
    rng = np.random.default_rng(3)
    n = int(np.prod(dims))
    phi, psi = rng.random(n), rng.random(n)
    d = _dist(dims, h)
    ref = float(np.sum(phi[:, None] * np.exp(-d / eps) * psi[None, :] * d))
    assert oracle.costn_dense(phi, psi, dims, h, eps) == pytest.approx(ref, rel=1e-13)
    assert oracle.costn_fs1(phi, psi, dims, h, eps) == pytest.approx(ref, rel=1e-12)
    F, G = np.log(phi), np.log(psi)
    assert oracle.costn_log_dense(F, G, dims, h, eps) == pytest.approx(ref, rel=1e-13)
    assert oracle.costn_fs1_log(F, G, dims, h, eps) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("dims,h,eps", CASES)
def test_marginal_errn_definition(dims, h, eps):
    rng = np.random.default_rng(5)
    n = int(np.prod(dims))
    phi, psi, nu = rng.random(n), rng.random(n), rng.random(n)
    ref = float(np.sum(np.abs(psi * (_kron_kernel(dims, h, eps).T @ phi) - nu)))
    for f in (oracle.marginal_errn_dense, oracle.marginal_errn_fs1):
        assert f(phi, psi, nu, dims, h, eps) == pytest.approx(ref, rel=1e-12)
    for f in (oracle.marginal_errn_log_dense, oracle.marginal_errn_fs1_log):
        assert f(np.log(phi), np.log(psi), nu, dims, h, eps) == pytest.approx(ref, rel=1e-12)


def _pair(dims, seed):
    rng = np.random.default_rng(seed)
    n = int(np.prod(dims))
    mu, nu = rng.random(n) + 0.05, rng.random(n) + 0.05
    return mu / mu.sum(), nu / nu.sum()


@pytest.mark.parametrize("dims,h,eps,its", [((3, 4, 5), (0.2, 0.1, 0.3), 0.07, 25),
                                            ((2, 3, 2, 3), (0.5, 0.2, 0.3, 0.1), 0.2, 15)])
def test_solvers_against_dense(dims, h, eps, its):
    mu, nu = _pair(dims, 1)
    a = oracle.sinkhornn_dense(mu, nu, dims, h, eps, tol=0.0, itr_max=its)
    b = oracle.fs1_nd(mu, nu, dims, h, eps, tol=0.0, itr_max=its)
    assert a.status == b.status == 0 and a.iterations == b.iterations == its
    assert b.w1 == pytest.approx(a.w1, rel=1e-12)
    assert b.marginal_err == pytest.approx(a.marginal_err, rel=1e-9, abs=1e-15)
    assert np.allclose(b.a, a.a, rtol=1e-11) and np.allclose(b.b, a.b, rtol=1e-11)
    la = oracle.sinkhornn_log_dense(mu, nu, dims, h, eps, tol=0.0, itr_max=its)
    lb = oracle.fs1_nd_log(mu, nu, dims, h, eps, tol=0.0, itr_max=its)
    assert la.w1 == pytest.approx(a.w1, rel=1e-12) and lb.w1 == pytest.approx(a.w1, rel=1e-12)
    assert np.allclose(lb.a, np.log(a.a), rtol=0, atol=1e-10)


@pytest.mark.parametrize("its", [1, 4, 30])
def test_product_marginals_closed_form(its):
    # mu = mu_0 (x) mu_1 (x) mu_2: the iterates stay products and
    # W = sum_a W_1D(mu_a, nu_a) at every iteration count
    dims, h, eps = (12, 7, 9), (1.0 / 12, 1.0 / 7, 1.0 / 9), 0.02
    parts = [inputs.mixture_pair(n, 2, 20 + a) for a, n in enumerate(dims)]
    mu = np.ones(1)
    nu = np.ones(1)
    for m, v in parts:
        mu = np.kron(m, mu)
        nu = np.kron(v, nu)
    w = sum(oracle.fs1(m, v, hh, eps, tol=0.0, itr_max=its).w1 for (m, v), hh in zip(parts, h))
    for f in (oracle.fs1_nd, oracle.fs1_nd_log):
        r = f(mu, nu, dims, h, eps, tol=0.0, itr_max=its)
        assert r.status == 0 and r.w1 == pytest.approx(w, rel=1e-11)


def test_reduces_to_1d_and_2d_oracles():
    m, v = inputs.mixture_pair(40, 3, 2)
    a = oracle.fs1(m, v, 0.025, 0.01, tol=0.0, itr_max=20)
    b = oracle.fs1_nd(m, v, (40,), (0.025,), 0.01, tol=0.0, itr_max=20)
    assert b.w1 == pytest.approx(a.w1, rel=1e-13)
    n1, n2, h1, h2, eps = 9, 13, 0.1, 0.07, 0.03
    mu, nu = _pair((n1, n2), 4)
    a = oracle.fs1_2d(mu, nu, n1, n2, h1, h2, eps, tol=0.0, itr_max=30)
    b = oracle.fs1_nd(mu, nu, (n1, n2), (h1, h2), eps, tol=0.0, itr_max=30)
    assert b.w1 == pytest.approx(a.w1, rel=1e-13)
    assert np.allclose(b.a, a.a, rtol=1e-12)
    a = oracle.fs1_2d_log(mu, nu, n1, n2, h1, h2, eps, tol=0.0, itr_max=30)
    b = oracle.fs1_nd_log(mu, nu, (n1, n2), (h1, h2), eps, tol=0.0, itr_max=30)
    assert b.w1 == pytest.approx(a.w1, rel=1e-13)


def test_singleton_axis_and_axis_permutation():
    dims, h, eps = (5, 6, 7), (0.1, 0.2, 0.15), 0.05
    mu, nu = _pair(dims, 8)
    r = oracle.fs1_nd(mu, nu, dims, h, eps, tol=0.0, itr_max=25)
    # the same grid with its axes reordered (2, 0, 1)
    perm = (2, 0, 1)
    def tr(x):
        return np.transpose(x.reshape(dims[::-1]), [2 - p for p in perm][::-1]).reshape(-1)
    t = oracle.fs1_nd(tr(mu), tr(nu), tuple(dims[p] for p in perm), tuple(h[p] for p in perm),
                      eps, tol=0.0, itr_max=25)
    assert t.w1 == pytest.approx(r.w1, rel=1e-12)
    # a singleton axis changes nothing, whatever its spacing
    s = oracle.fs1_nd(mu, nu, (5, 1, 6, 7), (0.1, 9.0, 0.2, 0.15), eps, tol=0.0, itr_max=25)
    assert s.w1 == pytest.approx(r.w1, rel=1e-13)


def test_dirac_pair_log_form_at_small_eps():
    # all the mass moves from p to q: W = sum_a |p_a - q_a| h_a; the plain
    # products underflow at this eps, the log form does not
    dims, h, eps = (6, 5, 4), (0.2, 0.3, 0.1), 1e-3
    n = int(np.prod(dims))
    mu, nu = np.zeros(n), np.zeros(n)
    p, q = (1, 0, 3), (4, 3, 0)
    mu[p[0] + dims[0] * (p[1] + dims[1] * p[2])] = 1.0
    nu[q[0] + dims[0] * (q[1] + dims[1] * q[2])] = 1.0
    w = sum(abs(a - b) * hh for a, b, hh in zip(p, q, h))
    r = oracle.fs1_nd_log(mu, nu, dims, h, eps, tol=0.0, itr_max=2)
    assert r.status == 0 and r.w1 == pytest.approx(w, rel=1e-12)
    assert oracle.fs1_nd(mu, nu, dims, h, eps, tol=0.0, itr_max=2).status != 0


def test_invalid_arguments():
    with pytest.raises(ValueError):
        oracle.fs1_nd(np.ones(4) / 4, np.ones(4) / 4, (2, 2), (0.1, -1.0), 0.1)
    with pytest.raises(ValueError):
        oracle.kvn_dense(np.ones(4), (2, 2), (0.1, 0.1), 0.0)
