"""fs1_solve_noalloc (the solve on the library's fixed per-GPU workspace)
against fs1_solve (the context's workspace): the same kernels on the same
inputs, so the same bits -- W, the marginal errors, the iteration count and
both potentials -- on two calls in a row, the second on a smaller grid, and a
grid too large for the fixed workspace is refused before any launch."""
import sys

import numpy as np
import pytest

from paper_2202_10042_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


def _same(a, b):
    assert a.status == b.status == 0
    assert a.iterations == b.iterations and a.converged == b.converged
    assert a.w1 == b.w1 and a.marginal_err == b.marginal_err and a.mu_err == b.mu_err
    assert torch.equal(a.F, b.F) and torch.equal(a.G, b.G)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("domain", ["log", "plain"])
def test_noalloc_equals_solve_twice(dtype, domain):
    from paper_2202_10042_amd import fs1
    # the second call is smaller: the fixed workspace keeps the first call's
    # contents, which must not leak into the second result
    for n, eps, tol, seed in ((1_500_007, 1e-3, 1e-6, 41), (300_001, 1e-2, 1e-8, 43)):
        if domain == "plain":
            eps *= 30.0
        mu_np, nu_np = inputs.mixture_pair(n, 3, seed)
        mu, nu = dev(mu_np), dev(nu_np)
        _say(f"noalloc {dtype} {domain} n={n}")
        ref = fs1.fs1_solve(mu, nu, eps, tol, itr_max=300, dtype=dtype, domain=domain,
                            potentials=True, sync_every=16)
        got = fs1.fs1_solve(mu, nu, eps, tol, itr_max=300, dtype=dtype, domain=domain,
                            potentials=True, sync_every=16, noalloc=True)
        _same(got, ref)


def test_noalloc_small_grid_paths_and_too_large():
    from paper_2202_10042_amd import fs1
    # one-workgroup solver and the threshold variant on the fixed workspace
    mu_np, nu_np = inputs.mixture_pair(5000, 2, 3)
    mu, nu = dev(mu_np), dev(nu_np)
    for domain in ("log", "absorb"):
        _say(f"noalloc small {domain}")
        ref = fs1.fs1_solve(mu, nu, 1e-3, 0.0, itr_max=200, domain=domain, potentials=True)
        got = fs1.fs1_solve(mu, nu, 1e-3, 0.0, itr_max=200, domain=domain, potentials=True,
                            noalloc=True)
        _same(got, ref)
    _say("noalloc too large")
    n = 2_000_000
    mu_np, nu_np = inputs.mixture_pair(n, 3, 5)
    with pytest.raises(fs1.Fs1Error) as ei:
        fs1.fs1_solve(dev(mu_np), dev(nu_np), 1e-3, 0.0, itr_max=10, dtype="f64", domain="log",
                      noalloc=True)
    assert ei.value.status == fs1.FS1_ERR_INVALID_ARG and "workspace" in str(ei.value)
