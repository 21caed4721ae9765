"""Contexts whose device memory comes from the caller's allocator
(fs1_ctx_create_with_allocator, here PyTorch's caching allocator through the
binding): the workspace and a server's pool are taken from it and given back,
and the results are the same bits as with the library's own allocations."""
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


def test_torch_allocator_workspace_and_pool():
    from paper_2202_10042_amd import fs1
    n = 1_000_003
    mu, nu = (dev(a) for a in inputs.mixture_pair(n, 3, 71))
    torch.cuda.synchronize()
    ctx = fs1.Context(allocator="torch")
    base = torch.cuda.memory_allocated()
    _say("solve on a torch-allocated workspace")
    r = fs1.fs1_solve(mu, nu, 1e-3, 0.0, itr_max=40, domain="log", ctx=ctx)
    grown = torch.cuda.memory_allocated() - base
    # vF, vG x 2, the binary64 marginal copies: > 5 n doubles
    assert grown >= 5 * 8 * n, grown
    ref_ctx = fs1.Context()
    ref = fs1.fs1_solve(mu, nu, 1e-3, 0.0, itr_max=40, domain="log", ctx=ref_ctx)
    assert r.status == ref.status == 0 and r.w1 == ref.w1 and r.marginal_err == ref.marginal_err
    # a larger solve regrows the workspace through the same allocator
    m2, v2 = (dev(a) for a in inputs.mixture_pair(3 * n, 3, 73))
    r2 = fs1.fs1_solve(m2, v2, 1e-3, 0.0, itr_max=5, domain="log", ctx=ctx)
    assert r2.status == 0
    assert torch.cuda.memory_allocated() - base >= 3 * grown - (1 << 20)
    _say("server pool from the torch allocator")
    before = torch.cuda.memory_allocated()
    srv = fs1.Server(hbm_budget=256 << 20, max_active=64, ctx=ctx)
    assert torch.cuda.memory_allocated() - before >= 200 << 20
    m3, v3 = (dev(a) for a in inputs.mixture_pair(5000, 3, 75))
    srv.submit(m3, v3, 1e-2, 1e-6)
    while srv.info()["active"] or srv.info()["queued"]:
        srv.step()
    (t, res, _, _), = srv.poll()
    assert res.status == 0 and res.converged
    srv.close()
    del m3, v3
    assert torch.cuda.memory_allocated() - before < (1 << 20)
    del m2, v2
    torch.cuda.synchronize()
    ctx.close()
    ref_ctx.close()
    assert torch.cuda.memory_allocated() - base < (1 << 20)
