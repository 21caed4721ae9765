"""fs1_solve_async: the solve enqueued without host synchronisation, its
result written to device memory.  Eagerly it gives the same bits as fs1_solve
on every solver path; captured once into a HIP graph (torch.cuda.graph) and
replayed on new marginals written into the same tensors, every replay gives
the bits of an eager fs1_solve on that replay's marginals, with the program's
own eager work and synchronisations between the replays; bad marginals come
back as a status in the device result."""
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


# (n, eps, domain, solver): one workgroup, fused, large-grid, general (log and
# plain)
CASES = [(5000, 1e-2, "log", "auto"), (300007, 1e-2, "log", "auto"),
         (2 * 1024 * 2048 + 3, 1e-2, "log", "auto"), (300007, 1e-2, "log", "general"),
         (100003, 1e-1, "plain", "auto")]


def _same(got, ref):
    assert got.status == ref.status == 0, (got, ref)
    assert got.iterations == ref.iterations and got.converged == ref.converged
    assert got.w1 == ref.w1 and got.marginal_err == ref.marginal_err and got.mu_err == ref.mu_err


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,eps,domain,solver", CASES)
def test_async_equals_solve(n, eps, domain, solver, dtype):
    from paper_2202_10042_amd import fs1
    mu, nu = (dev(a) for a in inputs.mixture_pair(n, 3, 7))
    _say(f"async n={n} {domain} {solver} {dtype}")
    for tol, itr_max in ((1e-7, 600), (0.0, 37)):
        ref = fs1.fs1_solve(mu, nu, eps, tol, itr_max=itr_max, dtype=dtype, domain=domain,
                            solver=solver, potentials=True, err_history=True)
        pot = torch.empty(2 * n, dtype=torch.float64, device="cuda")
        hist = torch.empty(itr_max + 1, dtype=torch.float64, device="cuda")
        out = fs1.fs1_solve_async(mu, nu, eps, tol, itr_max=itr_max, dtype=dtype, domain=domain,
                                  solver=solver, potentials_out=pot, err_history_out=hist)
        got = fs1.read_result(out)
        _same(got, ref)
        assert torch.equal(pot[:n], ref.F) and torch.equal(pot[n:], ref.G)
        assert torch.equal(torch.nan_to_num(hist, nan=-1.0),
                           torch.nan_to_num(ref.err_history, nan=-1.0))


@pytest.mark.parametrize("n,eps,domain,solver", CASES)
def test_async_graph_replays(n, eps, domain, solver):
    from paper_2202_10042_amd import fs1
    tol, itr_max = 1e-6, 300
    pairs = [inputs.mixture_pair(n, 3, s) for s in (11, 13, 15)]
    ctx = fs1.Context()
    mu, nu = dev(pairs[0][0]), dev(pairs[0][1])
    out = torch.empty(fs1.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    pot = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    kw = dict(itr_max=itr_max, domain=domain, solver=solver, ctx=ctx)
    # a first call outside the capture sizes the context's workspace
    fs1.fs1_solve_async(mu, nu, eps, tol, out=out, potentials_out=pot, **kw)
    torch.cuda.synchronize()
    _say(f"capture n={n} {domain} {solver}")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.set_stream(torch.cuda.current_stream())
        fs1.fs1_solve_async(mu, nu, eps, tol, out=out, potentials_out=pot, **kw)
    ctx.set_stream(torch.cuda.current_stream())
    ref_ctx = fs1.Context()
    for rep, (a, b) in enumerate(pairs + pairs[:1]):
        mu.copy_(dev(a))
        nu.copy_(dev(b))
        g.replay()
        torch.cuda.synchronize()
        got = fs1.read_result(out)
        gp = pot.clone()
        ref = fs1.fs1_solve(mu, nu, eps, tol, itr_max=itr_max, domain=domain, solver=solver,
                            potentials=True, ctx=ref_ctx)
        _say(f"  replay {rep}: {got.iterations} iterations, W {got.w1:.15g}")
        _same(got, ref)
        assert torch.equal(gp[:n], ref.F) and torch.equal(gp[n:], ref.G)


def test_async_bad_marginals_and_arguments():
    from paper_2202_10042_amd import fs1
    n = 20000
    a, b = inputs.mixture_pair(n, 3, 17)
    a[5] = -1e-3
    got = fs1.read_result(fs1.fs1_solve_async(dev(a), dev(b), 1e-2, 1e-6, itr_max=50))
    assert got.status == fs1.FS1_ERR_INVALID_ARG and got.iterations == 0
    a[5] = 0.0
    b = b / b.sum() * a.sum() * (1 + 1e-6)  # unequal masses
    got = fs1.read_result(fs1.fs1_solve_async(dev(a), dev(b), 1e-2, 1e-6, itr_max=50))
    assert got.status == fs1.FS1_ERR_INVALID_ARG
    mu, nu = (dev(v) for v in inputs.mixture_pair(n, 3, 19))
    with pytest.raises(fs1.Fs1Error):
        fs1.fs1_solve_async(mu, nu, 1e-2, 1e-6, itr_max=50, domain="absorb")
    # plain domain overflow: a non-finite scaling comes back as a status
    d_mu, d_nu = inputs.dirac_pair(4000, 10, 3900)
    got = fs1.read_result(fs1.fs1_solve_async(dev(d_mu), dev(d_nu), 1e-3, 0.0, itr_max=5,
                                              domain="plain", solver="general"))
    assert got.status == fs1.FS1_ERR_NONFINITE
