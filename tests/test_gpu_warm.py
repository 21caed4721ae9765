"""Warm start and state output of fs1_solve (Algorithm 1's loop resumed from a
given (phi, psi)): k iterations, then j more from the returned state, give the
same bits as k + j iterations in one solve -- W, both marginal errors, the
potentials and the state -- on every solver path, in both precisions and both
domains; a tolerance-driven solve resumed mid-way stops where the single
solve stops; bad warm-start input is refused."""
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
    assert a.status == b.status == 0, (a, b)
    assert a.w1 == b.w1 and a.marginal_err == b.marginal_err and a.mu_err == b.mu_err
    assert torch.equal(a.F, b.F) and torch.equal(a.G, b.G)
    assert torch.equal(a.state[0], b.state[0]) and torch.equal(a.state[1], b.state[1])


# (n, eps, domain, solver): one workgroup, fused, large-grid, general (log and
# plain), persistent
CASES = [(5000, 1e-3, "log", "auto"), (300007, 1e-3, "log", "auto"),
         (2 * 1024 * 2048 + 3, 1e-3, "log", "auto"), (300007, 1e-3, "log", "general"),
         (100003, 3e-2, "plain", "auto"), (300007, 1e-3, "log", "persistent"),
         (7000, 2e-2, "plain", "auto")]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,eps,domain,solver", CASES)
def test_resume_equals_one_solve(n, eps, domain, solver, dtype):
    from paper_2202_10042_amd import fs1
    if solver == "persistent" and dtype == "f32":
        pytest.skip("covered in binary64")
    mu, nu = (dev(a) for a in inputs.mixture_pair(n, 3, 97))
    kw = dict(dtype=dtype, domain=domain, solver=solver, potentials=True, state=True,
              sync_every=8)
    _say(f"resume n={n} {domain} {solver} {dtype}")
    whole = fs1.fs1_solve(mu, nu, eps, 0.0, itr_max=30, **kw)
    first = fs1.fs1_solve(mu, nu, eps, 0.0, itr_max=11, **kw)
    rest = fs1.fs1_solve(mu, nu, eps, 0.0, itr_max=19, warm=first.state, **kw)
    assert rest.iterations == 19
    _same(rest, whole)


def test_resume_to_tolerance_stops_where_one_solve_stops():
    from paper_2202_10042_amd import fs1
    mu, nu = (dev(a) for a in inputs.mixture_pair(200003, 4, 99))
    whole = fs1.fs1_solve(mu, nu, 1e-2, 1e-8, itr_max=2000, domain="log", state=True,
                          potentials=True)
    assert whole.converged and whole.iterations > 60
    first = fs1.fs1_solve(mu, nu, 1e-2, 0.0, itr_max=40, domain="log", state=True)
    rest = fs1.fs1_solve(mu, nu, 1e-2, 1e-8, itr_max=2000, domain="log", warm=first.state,
                         state=True, potentials=True)
    assert rest.iterations + 40 == whole.iterations
    _same(rest, whole)


def test_warm_start_from_potentials_and_bad_input():
    from paper_2202_10042_amd import fs1
    n = 4097
    mu, nu = (dev(a) for a in inputs.mixture_pair(n, 3, 101))
    cold = fs1.fs1_solve(mu, nu, 1e-2, 1e-9, itr_max=3000, domain="log", potentials=True)
    assert cold.converged
    # a warm start near the solution (from the converged potentials, as
    # mantissa 1 and a binary exponent per entry: ln 2 steps) converges sooner
    e = torch.round(torch.cat([cold.F, cold.G]) / np.log(2.0)).to(torch.int32)
    m = torch.exp(torch.cat([cold.F, cold.G]) - e.double() * np.log(2.0))
    hot = fs1.fs1_solve(mu, nu, 1e-2, 1e-9, itr_max=3000, domain="log", warm=(m, e))
    assert hot.converged and hot.iterations < cold.iterations / 2
    assert hot.w1 == pytest.approx(cold.w1, rel=1e-7)
    for bad_m, bad_e in ((m * float("nan"), e), (-m, e), (m, e + (1 << 21))):
        with pytest.raises(fs1.Fs1Error) as ei:
            fs1.fs1_solve(mu, nu, 1e-2, 1e-9, itr_max=10, domain="log", warm=(bad_m, bad_e))
        assert ei.value.status == fs1.FS1_ERR_INVALID_ARG and "warm" in str(ei.value)
    with pytest.raises(fs1.Fs1Error):
        fs1.fs1_solve(mu, nu, 1e-2, 0.0, itr_max=10, domain="absorb", warm=(m, e))
