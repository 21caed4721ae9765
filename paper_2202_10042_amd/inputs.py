"""Seeded synthetic inputs for FS-1 solves.

This module only draws histograms and request streams; it contains none of the
method's arithmetic, so both the GPU path and the CPU oracle can be fed from it.
Every generator is deterministic in its seed (numpy PCG64 ``default_rng``).

Recipes
-------
* Uniform grid on [0, 1] with n cells, spacing h = 1/n, cell centres
  x_i = (i + 1/2) h.
* Gaussian mixture histogram: K components with means ~ U[0.2, 0.8], standard
  deviations ~ U[0.03, 0.1], weights ~ U[0.3, 0.7] (then normalised); the density
  is evaluated at the cell centres, a floor of 1e-6 is added to the density values,
  and the result is normalised to total mass 1.
* Pair (mu, nu): mu from seed s, nu from seed s + 1.
* Shifted-noisy pair (large single-pair precision study): mu is a K-component
  mixture; nu_i is proportional to p_mu(x_i - shift) * exp(sigma * Z_i),
  Z ~ N(0, 1), plus the floor, normalised.
* The paper's Sec. 5.1 workload ("1-D random distributions"): grid
  x_i = (i-1) dx - 3, dx = 6/(N-1) on [-3, 3]; u_i, v_j ~ U[0, 1]; each divided
  by its sum (L1 norm).
* The paper's Sec. 5.2 workload (Ricker wavelet and its translate), squared and
  normalised as in the paper's eq. (ricker), on a stated time window.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

FLOOR = 1e-6
# Densities of grids longer than this are evaluated in blocks on a few threads
# (elementwise, so the values are the same as in one pass).
_BLOCK = 1 << 22
_THREADS = max(1, min(16, os.cpu_count() or 1))


def grid(n: int) -> tuple[np.ndarray, float]:
    """Cell centres of the uniform grid on [0, 1] and its spacing h = 1/n."""
    h = 1.0 / n
    return (np.arange(n, dtype=np.float64) + 0.5) * h, h


def _mixture_params(rng: np.random.Generator, k: int):
    means = rng.uniform(0.2, 0.8, size=k)
    sds = rng.uniform(0.03, 0.1, size=k)
    w = rng.uniform(0.3, 0.7, size=k)
    return means, sds, w / w.sum()


def _mixture_density_block(x: np.ndarray, means, sds, w) -> np.ndarray:
    p = np.zeros_like(x)
    for m, s, wk in zip(means, sds, w):
        p += wk * np.exp(-0.5 * ((x - m) / s) ** 2) / (s * math.sqrt(2.0 * math.pi))
    return p


def _mixture_density(x: np.ndarray, means, sds, w) -> np.ndarray:
    if x.size <= _BLOCK or _THREADS == 1:
        return _mixture_density_block(x, means, sds, w)
    p = np.empty_like(x)

    def one(lo: int) -> None:
        hi = min(x.size, lo + _BLOCK)
        p[lo:hi] = _mixture_density_block(x[lo:hi], means, sds, w)

    with ThreadPoolExecutor(_THREADS) as ex:
        list(ex.map(one, range(0, x.size, _BLOCK)))
    return p


def mixture_hist(n: int, k: int, seed: int) -> np.ndarray:
    """One K-component Gaussian-mixture histogram on the unit grid (sum 1)."""
    rng = np.random.default_rng(seed)
    x, _ = grid(n)
    p = _mixture_density(x, *_mixture_params(rng, k)) + FLOOR
    return p / p.sum()


def mixture_pair(n: int, k: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """(mu, nu) with mu from ``seed`` and nu from ``seed + 1``."""
    return mixture_hist(n, k, seed), mixture_hist(n, k, seed + 1)


def random_k(seed: int, lo: int = 3, hi: int = 5) -> int:
    """Number of mixture components drawn uniformly from {lo, ..., hi}."""
    return int(np.random.default_rng(seed + 7919).integers(lo, hi + 1))


def shifted_noisy_pair(n: int, k: int, seed: int, shift: float = 0.05,
                       sigma: float = 0.05) -> tuple[np.ndarray, np.ndarray]:
    """mu: K-component mixture; nu ~ mu(x - shift) * lognormal(0, sigma) noise."""
    rng = np.random.default_rng(seed)
    x, _ = grid(n)
    params = _mixture_params(rng, k)
    pm = _mixture_density(x, *params) + FLOOR
    mu = pm / pm.sum()
    z = np.random.default_rng(seed + 1).standard_normal(n)
    pn = _mixture_density(x - shift, *params) * np.exp(sigma * z) + FLOOR
    nu = pn / pn.sum()
    return mu, nu


def paper_uniform_pair(n: int, seed: int) -> tuple[np.ndarray, np.ndarray, float]:
    """Sec. 5.1 workload: u, v ~ U[0,1] on the grid of [-3, 3], L1-normalised.

    Returns (u, v, dx) with dx = 6 / (N - 1)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, size=n)
    v = rng.uniform(0.0, 1.0, size=n)
    return u / u.sum(), v / v.sum(), 6.0 / (n - 1)


def paper_uniform_2d(n1: int, n2: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Sec. 5.3 workload: u, v ~ U[0,1] on an n1 x n2 grid (h1 = h2 = 1 in the
    paper), each L1-normalised; flattened in column-major order (entry (i, j)
    at i + n1 j)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, size=(n2, n1)).reshape(-1)
    v = rng.uniform(0.0, 1.0, size=(n2, n1)).reshape(-1)
    return u / u.sum(), v / v.sum()


def paper_uniform_nd(dims, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """The Sec. 5.3 recipe on a grid of any number of axes: u, v ~ U[0,1] at
    every grid point, each L1-normalised, flattened with the first axis
    fastest."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(dims))
    u = rng.uniform(0.0, 1.0, size=n)
    v = rng.uniform(0.0, 1.0, size=n)
    return u / u.sum(), v / v.sum()


def product_pair_2d(n1: int, n2: int, k: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Product histograms mu = mu1 (x) mu2, nu = nu1 (x) nu2 from the 1-D
    mixtures of n1 (seed s) and n2 (seed s + 2) points, column-major."""
    m1, v1 = mixture_pair(n1, k, seed)
    m2, v2 = mixture_pair(n2, k, seed + 2)
    return np.outer(m2, m1).reshape(-1), np.outer(v2, v1).reshape(-1)


def ricker_pair(n: int, shift: float = -1.2032, delta: float = 1e-3,
                t0: float = -4.0, t1: float = 4.0, f0: float = 1.0, amp: float = 1.0):
    """Sec. 5.2 workload: R(t) and R(t - s), squared and normalised by eq. (ricker).

    The paper does not state the time window nor L; here the window is [t0, t1]
    sampled at n points (dt = (t1 - t0)/(n - 1)), ||f^2|| is the sum of f^2, and
    L = n so that (f^2/||f^2|| + delta) / (1 + L delta) sums to one.
    Returns (u, v, dt)."""
    t = np.linspace(t0, t1, n)
    dt = (t1 - t0) / (n - 1)

    def ricker(tt):
        a = (math.pi * f0 * tt) ** 2
        return amp * (1.0 - 2.0 * a) * np.exp(-a)

    f2 = ricker(t) ** 2
    g2 = ricker(t - shift) ** 2
    L = float(n)
    u = (f2 / f2.sum() + delta) / (1.0 + L * delta)
    v = (g2 / g2.sum() + delta) / (1.0 + L * delta)
    return u, v, dt


def dirac_pair(n: int, a: int, b: int) -> tuple[np.ndarray, np.ndarray]:
    mu = np.zeros(n)
    nu = np.zeros(n)
    mu[a] = 1.0
    nu[b] = 1.0
    return mu, nu


# --------------------------------------------------------------------------
# batched and served workloads
# --------------------------------------------------------------------------

@dataclass
class BatchSpec:
    sizes: np.ndarray     # int64 [B]
    eps: np.ndarray       # float64 [B]
    seeds: np.ndarray     # int64 [B]  (mu from seed, nu from seed + 1)
    ks: np.ndarray        # int64 [B]  mixture components


def batch_spec(b: int, n_lo: int, n_hi: int, eps_choices, seed: int,
               k_lo: int = 3, k_hi: int = 5) -> BatchSpec:
    """B instances with N log-uniform in [n_lo, n_hi], eps uniform over the
    choices, instance i seeded with seed + 2 i."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=b))).astype(np.int64)
    sizes = np.clip(sizes, n_lo, n_hi)
    eps = np.asarray(eps_choices, dtype=np.float64)[rng.integers(0, len(eps_choices), size=b)]
    ks = rng.integers(k_lo, k_hi + 1, size=b).astype(np.int64)
    seeds = seed + 1000 + 2 * np.arange(b, dtype=np.int64)
    return BatchSpec(sizes, eps, seeds, ks)


def batch_hists(spec: BatchSpec):
    """Packed (mu, nu, offsets) for a BatchSpec: instance b lives in
    [offsets[b], offsets[b+1])."""
    offs = np.zeros(spec.sizes.size + 1, dtype=np.int64)
    np.cumsum(spec.sizes, out=offs[1:])
    mu = np.empty(int(offs[-1]))
    nu = np.empty(int(offs[-1]))
    for i, (n, s, k) in enumerate(zip(spec.sizes, spec.seeds, spec.ks)):
        a, b = mixture_pair(int(n), int(k), int(s))
        mu[offs[i]:offs[i + 1]] = a
        nu[offs[i]:offs[i + 1]] = b
    return mu, nu, offs


def mixture_pairs_device(sizes, ks, seeds, torch, device="cuda"):
    """Many (mu, nu) pairs at once on a GPU, by the recipe of mixture_pair:
    pair i has sizes[i] cells, ks[i] components, mu from seeds[i] and nu from
    seeds[i] + 1 (the same mixture parameters as mixture_pair draws); the
    densities are evaluated in binary64 on the device (so the values equal
    mixture_pair's to rounding).  Returns (mu, nu, offsets): packed device
    tensors and the host offsets of the pairs."""
    sizes = np.asarray(sizes, dtype=np.int64)
    B = sizes.size
    kmax = int(max(ks)) if B else 1
    offs = np.zeros(B + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    total = int(offs[-1])
    out = []
    for side in (0, 1):
        prm = np.zeros((B, kmax, 3))  # means, sds, weights (weight 0 pads)
        prm[:, :, 1] = 1.0
        for i in range(B):
            m, sd, w = _mixture_params(np.random.default_rng(int(seeds[i]) + side), int(ks[i]))
            prm[i, :len(m), 0] = m
            prm[i, :len(m), 1] = sd
            prm[i, :len(m), 2] = w
        p = torch.tensor(prm, dtype=torch.float64, device=device)
        szt = torch.tensor(sizes, device=device)
        owner = torch.repeat_interleave(torch.arange(B, device=device), szt)
        start = torch.tensor(offs[:-1], device=device)
        idx = torch.arange(total, device=device, dtype=torch.int64) - start[owner]
        x = (idx.double() + 0.5) / szt[owner].double()
        dens = torch.zeros(total, dtype=torch.float64, device=device)
        for k in range(kmax):
            mk, sk, wk = p[owner, k, 0], p[owner, k, 1], p[owner, k, 2]
            dens += wk * torch.exp(-0.5 * ((x - mk) / sk) ** 2) / (sk * math.sqrt(2.0 * math.pi))
        dens += FLOOR
        # one reduction per pair (a scatter-add into B sums would contend on
        # B addresses)
        sums = torch.stack([dens[int(offs[i]):int(offs[i + 1])].sum() for i in range(B)])
        out.append(dens / sums[owner])
    return out[0], out[1], offs


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate on [0, duration)."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    chunk = max(16, int(rate * duration * 1.2) + 16)
    while t < duration:
        gaps = rng.exponential(1.0 / rate, size=chunk)
        ts = t + np.cumsum(gaps)
        out.append(ts[ts < duration])
        t = float(ts[-1])
    return np.concatenate(out) if out else np.zeros(0)
