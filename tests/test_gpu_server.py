"""GPU tests of the serving loop (fs1_server_*): continuous batching gives each
request the result it gets alone (bitwise), admission follows submission order
under the memory budget, and results match the CPU oracle (binary32 scans:
|dW|/W <= 1e-5 against the binary64 oracle at the same iteration count;
binary64: 1e-10)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2202_10042_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _fs1():
    from paper_2202_10042_amd import fs1
    return fs1


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


def _requests(k, seed, n_lo=128, n_hi=30000, eps=(1e-2, 1e-3)):
    spec = inputs.batch_spec(k, n_lo, n_hi, list(eps), seed)
    mu, nu, offs = inputs.batch_hists(spec)
    return [(mu[offs[i]:offs[i + 1]], nu[offs[i]:offs[i + 1]], float(spec.eps[i]))
            for i in range(k)]


def _drain(srv, limit=100000):
    out = {}
    for _ in range(limit):
        srv.step()
        for t, r, a, c in srv.poll():
            out[t] = (r, a, c)
        info = srv.info()
        if info["queued"] == 0 and info["active"] == 0:
            return out
    raise AssertionError("server did not drain")


def _eq(x, y):
    return x == y or (np.isnan(x) and np.isnan(y))


def _same(a, b):
    return (a.status == b.status and a.iterations == b.iterations and a.converged == b.converged
            and _eq(a.w1, b.w1) and _eq(a.marginal_err, b.marginal_err)
            and _eq(a.mu_err, b.mu_err))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_server_results_equal_alone_and_in_the_mix(dtype):
    fs1 = _fs1()
    reqs = _requests(12, 31)
    tol = 1e-6
    _say(f"server mix {dtype}")
    srv = fs1.Server(hbm_budget=256 << 20, max_active=64, dtype=dtype, itr_max=3000,
                     iters_per_step=16)
    held = [(dev(m), dev(v), e) for m, v, e in reqs]
    tickets = []
    # staggered arrivals: requests join while others are part-way through
    for i, (m, v, e) in enumerate(held):
        tickets.append(srv.submit(m, v, e, tol))
        if i % 3 == 2:
            srv.step()
    mix = _drain(srv)
    srv.close()
    assert sorted(mix) == tickets
    admitted = [mix[t][1] for t in tickets]
    assert len(set(admitted)) > 1  # requests really were admitted at different steps
    for i in (0, 5, 11):
        m, v, e = held[i]
        alone_srv = fs1.Server(hbm_budget=64 << 20, max_active=4, dtype=dtype, itr_max=3000,
                               iters_per_step=7)
        alone_srv.submit(m, v, e, tol)
        alone = _drain(alone_srv)
        alone_srv.close()
        (r_alone, _, _), = alone.values()
        assert _same(r_alone, mix[tickets[i]][0]), (i, r_alone, mix[tickets[i]][0])
        # the batched entry point runs the same arithmetic
        b = fs1.fs1_solve_batched(m, v, [0, m.numel()], [e], [tol], itr_max=3000, dtype=dtype)[0]
        assert _same(b, r_alone), (i, b, r_alone)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_server_overlapped_steps_same_results(dtype):
    # FS1_FLAG_SERVER_OVERLAP: a step returns with its iterations enqueued and
    # the next call reports what they stopped; every request's result is the
    # blocking server's, bit for bit, and each completes at the same step
    fs1 = _fs1()
    reqs = _requests(10, 47)
    held = [(dev(m), dev(v), e) for m, v, e in reqs]
    out = {}
    for overlap in (False, True):
        _say(f"server overlap={overlap} {dtype}")
        srv = fs1.Server(hbm_budget=256 << 20, max_active=64, dtype=dtype, itr_max=3000,
                         iters_per_step=16, overlap=overlap)
        tickets = []
        for i, (m, v, e) in enumerate(held):
            tickets.append(srv.submit(m, v, e, 1e-6))
            if i % 3 == 2:
                srv.step()
        out[overlap] = (tickets, _drain(srv))
        srv.close()
    (tb, blocking), (to, overlapped) = out[False], out[True]
    assert tb == to and sorted(overlapped) == to
    for t in to:
        (rb, ab, cb), (ro, ao, co) = blocking[t], overlapped[t]
        assert _same(rb, ro), (t, rb, ro)
        assert ao == ab and co == cb


def test_server_matches_oracle_and_converges():
    fs1 = _fs1()
    reqs = _requests(8, 5, n_hi=8000)
    srv = fs1.Server(hbm_budget=128 << 20, max_active=16, dtype="f64", itr_max=4000,
                     iters_per_step=32)
    held = [(dev(m), dev(v), e) for m, v, e in reqs]
    tickets = [srv.submit(m, v, e, 1e-8) for m, v, e in held]
    res = _drain(srv)
    srv.close()
    for t, (m, v, e) in zip(tickets, reqs):
        r = res[t][0]
        assert r.status == 0
        ref = oracle.fs1_log(m, v, 1.0 / len(m), e, tol=0.0, itr_max=r.iterations)
        assert r.w1 == pytest.approx(ref.w1, rel=1e-10)
        if r.converged:
            assert r.marginal_err <= 1e-8


def test_server_budget_admission_order_and_reuse():
    fs1 = _fs1()
    # a budget that holds only a few of these requests at once
    reqs = _requests(10, 9, n_lo=60000, n_hi=65536, eps=(1e-2,))
    srv = fs1.Server(hbm_budget=24 << 20, max_active=16, dtype="f32", itr_max=2000,
                     iters_per_step=16)
    held = [(dev(m), dev(v), e) for m, v, e in reqs]
    tickets = [srv.submit(m, v, e, 1e-6) for m, v, e in held]
    srv.step()
    info = srv.info()
    assert 0 < info["active"] < len(reqs) and info["queued"] > 0
    assert info["bytes_in_use"] <= info["bytes_total"]
    res = _drain(srv)
    assert srv.info()["bytes_in_use"] == 0
    srv.close()
    admitted = [res[t][1] for t in tickets]
    assert admitted == sorted(admitted)  # first come, first admitted
    assert all(res[t][0].status == 0 and res[t][0].converged for t in tickets)


def test_server_invalid_requests_and_graph_option():
    fs1 = _fs1()
    good = _requests(3, 17, n_hi=5000)
    bad = (np.full(100, 0.01), np.full(100, 0.02), 0.01)  # unequal masses
    items = [good[0], bad, good[1], good[2]]
    results = []
    for graph in (True, False):
        srv = fs1.Server(hbm_budget=64 << 20, max_active=8, dtype="f32", itr_max=1000,
                         iters_per_step=8, graph=graph)
        held = [(dev(m), dev(v), e) for m, v, e in items]
        tickets = [srv.submit(m, v, e, 1e-6) for m, v, e in held]
        res = _drain(srv)
        srv.close()
        results.append([res[t][0] for t in tickets])
    a, b = results
    assert [r.status for r in a] == [0, -1, 0, 0]
    assert all(_same(x, y) for x, y in zip(a, b))
    srv = fs1.Server(hbm_budget=16 << 20, max_active=2)
    x = dev(np.ones(10) / 10)
    with pytest.raises(fs1.Fs1Error):
        srv.submit(x, x, -1.0, 0.0)
    with pytest.raises(fs1.Fs1Error):
        srv.submit(x, x, 0.1, -1.0)
    big = torch.ones(1 << 22, dtype=torch.float64, device="cuda")
    with pytest.raises(fs1.Fs1Error):  # never fits the 16 MiB budget
        srv.submit(big, big, 0.1, 0.0)
    srv.close()
