"""The seeded workload generators: determinism, normalisation, recipe."""
import numpy as np
import pytest

from paper_2202_10042_amd import inputs


def test_mixture_deterministic_and_normalised():
    a1, b1 = inputs.mixture_pair(1000, 2, 1)
    a2, b2 = inputs.mixture_pair(1000, 2, 1)
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)
    assert not np.array_equal(a1, b1)
    for v in (a1, b1):
        assert abs(v.sum() - 1.0) < 1e-14 and v.min() > 0
        # the 1e-6 density floor bounds the smallest cell mass from below
        assert v.min() >= 1e-6 / (v.size * (1e-6 + 40.0))


def test_mixture_differs_by_seed():
    a, _ = inputs.mixture_pair(500, 3, 10)
    b, _ = inputs.mixture_pair(500, 3, 12)
    assert np.abs(a - b).max() > 1e-4


def test_shifted_noisy_pair():
    mu, nu = inputs.shifted_noisy_pair(100000, 8, 3)
    x, h = inputs.grid(100000)
    assert abs(mu.sum() - 1) < 1e-12 and abs(nu.sum() - 1) < 1e-12
    shift = (x * nu).sum() - (x * mu).sum()
    assert 0.03 < shift < 0.07


def test_blocked_density_equals_one_pass():
    # grids longer than one block are evaluated on several threads: the values
    # must be those of a single pass, bit for bit
    n = 2 * inputs._BLOCK + 12345
    x, _ = inputs.grid(n)
    prm = inputs._mixture_params(np.random.default_rng(5), 8)
    assert np.array_equal(inputs._mixture_density(x, *prm),
                          inputs._mixture_density_block(x, *prm))


def test_paper_uniform_and_ricker():
    u, v, dx = inputs.paper_uniform_pair(500, 0)
    assert dx == 6.0 / 499 and abs(u.sum() - 1) < 1e-14 and abs(v.sum() - 1) < 1e-14
    u, v, dt = inputs.ricker_pair(500)
    assert abs(u.sum() - 1) < 1e-12 and abs(v.sum() - 1) < 1e-12 and u.min() > 0


def test_batch_spec_ranges():
    s = inputs.batch_spec(4096, 256, 65536, [1e-2, 3e-3, 1e-3], seed=7)
    assert s.sizes.min() >= 256 and s.sizes.max() <= 65536
    assert set(np.unique(s.eps)) <= {1e-2, 3e-3, 1e-3}
    # log-uniform: the median is near the geometric mean 4096
    assert 2500 < np.median(s.sizes) < 6500
    s2 = inputs.batch_spec(4096, 256, 65536, [1e-2, 3e-3, 1e-3], seed=7)
    assert np.array_equal(s.sizes, s2.sizes) and np.array_equal(s.eps, s2.eps)
    mu, nu, offs = inputs.batch_hists(inputs.batch_spec(5, 100, 300, [0.01], seed=1))
    assert offs[0] == 0 and offs.size == 6 and mu.size == offs[-1]
    for b in range(5):
        assert abs(mu[offs[b]:offs[b + 1]].sum() - 1) < 1e-13


def test_poisson_arrivals():
    t = inputs.poisson_arrivals(20000.0, 1.0, 3)
    assert np.all(np.diff(t) > 0) and t[-1] < 1.0
    assert 19000 < t.size < 21000


def test_device_mixture_pairs_follow_the_host_recipe():
    torch = pytest.importorskip("torch")
    sizes, ks, seeds = [128, 1000, 7, 4099], [3, 5, 4, 3], [10, 20, 30, 40]
    mu, nu, offs = inputs.mixture_pairs_device(sizes, ks, seeds, torch, device="cpu")
    assert list(offs) == [0, 128, 1128, 1135, 5234]
    for i, (n, k, s) in enumerate(zip(sizes, ks, seeds)):
        a, b = inputs.mixture_pair(n, k, s)
        np.testing.assert_allclose(mu[offs[i]:offs[i + 1]].numpy(), a, rtol=1e-13)
        np.testing.assert_allclose(nu[offs[i]:offs[i + 1]].numpy(), b, rtol=1e-13)
