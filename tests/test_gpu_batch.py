"""GPU parity of fs1_solve_batched (ragged batches, one launch per half) against
the CPU oracle, and invariance of each instance's result to the batch around it.

Tolerances (as for single solves):
  * binary64: |dW|/W <= 1e-10 at a fixed iteration count, marginal error within
    1e-6 relative plus 1e-12 absolute of the oracle's;
  * binary32 scans against the binary64 oracle: |dW|/W <= 1e-5;
  * an instance alone and in a mix, with or without graph replay and for any
    polling interval: bitwise identical results.
"""
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


def _pack(pairs):
    offs = np.zeros(len(pairs) + 1, dtype=np.int64)
    np.cumsum([len(m) for m, _ in pairs], out=offs[1:])
    mu = np.concatenate([m for m, _ in pairs])
    nu = np.concatenate([v for _, v in pairs])
    return mu, nu, offs


def _pair(n, seed):
    if n == 1:
        return np.array([1.0]), np.array([1.0])
    if n == 2:
        return np.array([0.3, 0.7]), np.array([0.6, 0.4])
    return inputs.mixture_pair(n, 3, seed)


def _ref(mu, nu, eps, tol, its):
    # the log-domain oracles: plain scalings overflow at the largest h/eps here
    n = len(mu)
    if n <= 3000 and its <= 100:
        return oracle.sinkhorn_log_dense(mu, nu, 1.0 / n, eps, tol=tol, itr_max=its)
    return oracle.fs1_log(mu, nu, 1.0 / n, eps, tol=tol, itr_max=its)


# sizes span one run, one chunk, several chunks with a ragged tail, and more
# than one run-length class (h/eps = 100 at n = 500, eps = 2e-5 needs R = 1)
RAGGED = [(1, 0.01), (2, 0.05), (7, 0.01), (300, 0.003), (2048, 0.01), (2049, 0.001),
          (5000, 0.01), (20000, 0.001), (500, 2e-5), (700, 2e-5)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batched_fixed_iterations_vs_oracle(dtype):
    fs1 = _fs1()
    its = 30
    pairs = [_pair(n, 10 + i) for i, (n, _) in enumerate(RAGGED)]
    eps = [e for _, e in RAGGED]
    mu, nu, offs = _pack(pairs)
    _say(f"batched {dtype} B={len(pairs)} its={its}")
    res = fs1.fs1_solve_batched(dev(mu), dev(nu), offs, eps, [0.0] * len(pairs), itr_max=its,
                                dtype=dtype)
    for i, ((m, v), e) in enumerate(zip(pairs, eps)):
        ref = _ref(m, v, e, 0.0, its)
        r = res[i]
        assert r.status == 0, (i, r)
        assert r.iterations == ref.iterations, (i, r.iterations, ref.iterations)
        if dtype == "f64":
            assert r.w1 == pytest.approx(ref.w1, rel=1e-10, abs=1e-300), i
            assert r.marginal_err == pytest.approx(ref.marginal_err, rel=1e-6, abs=1e-12), i
            assert r.mu_err <= 1e-12, i
        else:
            assert r.w1 == pytest.approx(ref.w1, rel=1e-5, abs=1e-300), i
            assert r.marginal_err == pytest.approx(ref.marginal_err, rel=1e-3, abs=1e-6), i


def test_batched_to_tolerance_vs_oracle():
    fs1 = _fs1()
    spec = inputs.batch_spec(12, 256, 4096, [1e-2, 3e-3, 1e-3], seed=7)
    mu, nu, offs = inputs.batch_hists(spec)
    tol = 1e-9
    its = 3000
    _say("batched to tolerance B=12")
    res = fs1.fs1_solve_batched(dev(mu), dev(nu), offs, spec.eps, [tol] * 12, itr_max=its,
                                dtype="f64")
    assert sum(r.converged for r in res) >= 6
    for i in range(12):
        m, v = mu[offs[i]:offs[i + 1]], nu[offs[i]:offs[i + 1]]
        ref = _ref(m, v, spec.eps[i], tol, its)
        r = res[i]
        assert r.status == 0 and r.converged == ref.converged
        # the stopping iteration may move by one when err(l) sits at tol
        assert abs(r.iterations - ref.iterations) <= 1, (i, r.iterations, ref.iterations)
        if r.iterations == ref.iterations:
            assert r.w1 == pytest.approx(ref.w1, rel=1e-10)
        if r.converged:
            assert r.marginal_err <= tol
        else:
            assert r.iterations == its and r.marginal_err > tol


def _same(a, b):
    return (a.status == b.status and a.iterations == b.iterations and a.converged == b.converged
            and (a.w1 == b.w1 or (np.isnan(a.w1) and np.isnan(b.w1)))
            and (a.marginal_err == b.marginal_err
                 or (np.isnan(a.marginal_err) and np.isnan(b.marginal_err)))
            and (a.mu_err == b.mu_err or (np.isnan(a.mu_err) and np.isnan(b.mu_err))))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batched_instance_alone_equals_in_mix(dtype):
    fs1 = _fs1()
    spec = inputs.batch_spec(10, 128, 20000, [1e-2, 1e-3, 3e-4], seed=3)
    mu, nu, offs = inputs.batch_hists(spec)
    tol = [1e-6] * 10
    _say(f"batched invariance {dtype}")
    mix = fs1.fs1_solve_batched(dev(mu), dev(nu), offs, spec.eps, tol, itr_max=800,
                                dtype=dtype)
    for i in (0, 3, 9):
        m, v = mu[offs[i]:offs[i + 1]], nu[offs[i]:offs[i + 1]]
        alone = fs1.fs1_solve_batched(dev(m), dev(v), [0, len(m)], [spec.eps[i]], [tol[i]],
                                      itr_max=800, dtype=dtype)[0]
        assert _same(alone, mix[i]), (i, alone, mix[i])
    # reversed order: every instance at another place in the packed arrays
    order = list(range(9, -1, -1))
    pairs = [(mu[offs[i]:offs[i + 1]], nu[offs[i]:offs[i + 1]]) for i in order]
    rm, rn, ro = _pack(pairs)
    rev = fs1.fs1_solve_batched(dev(rm), dev(rn), ro, [spec.eps[i] for i in order], tol,
                                itr_max=800, dtype=dtype)
    for k, i in enumerate(order):
        assert _same(rev[k], mix[i]), (i, rev[k], mix[i])


def test_batched_graph_and_polling_do_not_change_results():
    fs1 = _fs1()
    spec = inputs.batch_spec(8, 256, 8192, [1e-2, 3e-3, 1e-3], seed=5)
    mu, nu, offs = inputs.batch_hists(spec)
    args = (dev(mu), dev(nu), offs, spec.eps, [1e-7] * 8)
    base = fs1.fs1_solve_batched(*args, itr_max=1500, dtype="f32", sync_every=16)
    for kw in ({"graph": False}, {"sync_every": 1}, {"sync_every": 97},
               {"sync_every": 5, "graph": False}):
        _say(f"batched variant {kw}")
        other = fs1.fs1_solve_batched(*args, itr_max=1500, dtype="f32", **kw)
        for a, b in zip(base, other):
            assert _same(a, b), (kw, a, b)


def test_batched_matches_single_solve():
    fs1 = _fs1()
    spec = inputs.batch_spec(6, 300, 30000, [1e-2, 1e-3], seed=11)
    mu, nu, offs = inputs.batch_hists(spec)
    res = fs1.fs1_solve_batched(dev(mu), dev(nu), offs, spec.eps, [0.0] * 6, itr_max=50,
                                dtype="f64")
    for i in range(6):
        m, v = dev(mu[offs[i]:offs[i + 1]]), dev(nu[offs[i]:offs[i + 1]])
        s = fs1.fs1_solve(m, v, spec.eps[i], 0.0, itr_max=50, dtype="f64", domain="log")
        assert s.iterations == res[i].iterations == 50
        assert res[i].w1 == pytest.approx(s.w1, rel=1e-11)
        assert res[i].marginal_err == pytest.approx(s.marginal_err, rel=1e-7, abs=1e-13)


def test_batched_invalid_instances_do_not_disturb_others():
    fs1 = _fs1()
    good = [_pair(500, 1), _pair(3000, 2)]
    bad_neg = (np.full(40, 1 / 40), np.full(40, 1 / 40))
    bad_neg[0][3] = -1e-3
    bad_mass = (np.full(50, 1 / 50), np.full(50, 1.5 / 50))
    zero = (np.zeros(60), np.zeros(60))
    nan = (np.full(30, 1 / 30), np.full(30, 1 / 30))
    nan[1][5] = np.nan
    pairs = [good[0], bad_neg, good[1], bad_mass, zero, nan]
    eps = [0.01] * len(pairs)
    mu, nu, offs = _pack(pairs)
    res = fs1.fs1_solve_batched(dev(mu), dev(nu), offs, eps, [1e-9] * len(pairs), itr_max=2000)
    assert [r.status for r in res] == [0, -1, 0, -1, -1, -1]
    mu2, nu2, offs2 = _pack(good)
    ref = fs1.fs1_solve_batched(dev(mu2), dev(nu2), offs2, eps[:2], [1e-9] * 2, itr_max=2000)
    assert _same(res[0], ref[0]) and _same(res[2], ref[1])


def test_batched_itr_max_and_check_every():
    fs1 = _fs1()
    pairs = [_pair(1000, 3), _pair(4000, 4)]
    mu, nu, offs = _pack(pairs)
    res = fs1.fs1_solve_batched(dev(mu), dev(nu), offs, [1e-3, 1e-3], [1e-14, 1e-14],
                                itr_max=7)
    for r in res:
        assert r.status == 0 and r.iterations == 7 and not r.converged
    # check_every = 5: the stop lands on a multiple of 5 at or after the first hit
    res1 = fs1.fs1_solve_batched(dev(mu), dev(nu), offs, [1e-2, 1e-2], [1e-8, 1e-8],
                                 itr_max=5000)
    res5 = fs1.fs1_solve_batched(dev(mu), dev(nu), offs, [1e-2, 1e-2], [1e-8, 1e-8],
                                 itr_max=5000, check_every=5)
    for a, b in zip(res1, res5):
        assert a.converged and b.converged
        assert b.iterations % 5 == 0 and a.iterations <= b.iterations < a.iterations + 5


def test_batched_empty_and_argument_errors():
    fs1 = _fs1()
    x = dev(np.ones(8) / 8)
    assert fs1.fs1_solve_batched(x, x, [0], [], []) == []
    with pytest.raises(fs1.Fs1Error):
        fs1.fs1_solve_batched(x, x, [0, 0, 8], [0.1, 0.1], [0.0, 0.0])  # empty instance
    with pytest.raises(fs1.Fs1Error):
        fs1.fs1_solve_batched(x, x, [0, 8], [-1.0], [0.0])
    with pytest.raises(fs1.Fs1Error):
        fs1.fs1_solve_batched(x, x, [0, 8], [0.1], [-1.0])


def test_batched_plain_domain_runs_single_solves():
    fs1 = _fs1()
    pairs = [_pair(1000, 1), _pair(512, 2)]
    mu, nu, offs = _pack(pairs)
    res = fs1.fs1_solve_batched(dev(mu), dev(nu), offs, [0.01, 0.01], [0.0, 0.0], itr_max=20,
                                domain="plain")
    for (m, v), r in zip(pairs, res):
        s = fs1.fs1_solve(dev(m), dev(v), 0.01, 0.0, itr_max=20, domain="plain")
        assert _same(r, s)


def test_batched_c3_sample_fp32():
    """The uneven-batch workload at reduced count (N log-uniform in [256, 65536],
    eps in {1e-2, 3e-3, 1e-3}, tol 1e-6): binary32 scans against binary64 scans
    of the same batch and against the oracle.  A few eps = 1e-3 instances need
    more than itr_max iterations in either precision."""
    fs1 = _fs1()
    B = 96
    spec = inputs.batch_spec(B, 256, 65536, [1e-2, 3e-3, 1e-3], seed=2024)
    mu, nu, offs = inputs.batch_hists(spec)
    _say(f"batched C3 sample B={B} sum N={int(offs[-1])}")
    args = (dev(mu), dev(nu), offs, spec.eps, [1e-6] * B)
    r32 = fs1.fs1_solve_batched(*args, itr_max=5000, dtype="f32")
    r64 = fs1.fs1_solve_batched(*args, itr_max=5000, dtype="f64")
    assert all(r.status == 0 for r in r32 + r64)
    assert sum(r.converged for r in r32) >= 0.9 * B
    for a, b in zip(r32, r64):
        assert a.converged == b.converged
        if a.converged:
            assert a.marginal_err <= 1e-6
            # the binary32 error curve tracks the binary64 one closely
            assert abs(a.iterations - b.iterations) <= max(5, b.iterations // 100)
        assert a.w1 == pytest.approx(b.w1, rel=1e-6)
    for i in range(0, B, 12):
        m, v = mu[offs[i]:offs[i + 1]], nu[offs[i]:offs[i + 1]]
        ref = oracle.fs1_log(m, v, 1.0 / len(m), spec.eps[i], tol=0.0,
                             itr_max=r32[i].iterations)
        assert r32[i].w1 == pytest.approx(ref.w1, rel=1e-5), i
        if r64[i].iterations == r32[i].iterations:
            assert r64[i].w1 == pytest.approx(ref.w1, rel=1e-10), i


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batched_forced_configurations(dtype):
    # fs1_solve_batched_config: per-instance configurations forced by the
    # caller.  The tuner's mirror of the library's choice reproduces the
    # default call bit for bit; other configurations stay within the stated
    # tolerance of the oracle; invalid ones are refused before any launch.
    from paper_2202_10042_amd import tune
    fs1 = _fs1()
    spec = inputs.batch_spec(24, 128, 20000, [1e-2, 3e-3, 1e-3], seed=11)
    mu, nu, offs = inputs.batch_hists(spec)
    sizes = np.diff(offs).astype(int)
    tol = [0.0] * 24
    args = (dev(mu), dev(nu), offs, spec.eps, tol)
    _say(f"batched forced configurations {dtype}")
    base = fs1.fs1_solve_batched(*args, itr_max=60, dtype=dtype)
    rows = tune.read_table()
    mirror = [tune.instance_config(rows, dtype, int(n), float(e)) for n, e in zip(sizes, spec.eps)]
    forced = fs1.fs1_solve_batched(*args, itr_max=60, dtype=dtype, config=mirror)
    for a, b in zip(base, forced):
        assert _same(a, b), (a, b)
    shared8 = fs1.fs1_solve_batched(*args, itr_max=60, dtype=dtype, config=(8, 0))
    for i in (0, 7, 23):
        m, v = mu[offs[i]:offs[i + 1]], nu[offs[i]:offs[i + 1]]
        ref = oracle.fs1_log(m, v, 1.0 / len(m), float(spec.eps[i]), tol=0.0, itr_max=60)
        r = shared8[i]
        assert r.status == 0 and r.iterations == ref.iterations
        assert r.w1 == pytest.approx(ref.w1, rel=1e-10 if dtype == "f64" else 1e-5)
    with pytest.raises(RuntimeError):
        fs1.fs1_solve_batched(*args, itr_max=60, dtype=dtype, config=(3, 0))
    with pytest.raises(RuntimeError):  # the largest instance does not fit one workgroup
        fs1.fs1_solve_batched(*args, itr_max=60, dtype=dtype, config=(8, 256))


def test_batched_device_eps_and_tol():
    # FS1_FLAG_DEVICE_PARAMS: eps and tol handed over as device arrays give the
    # results of the host arrays bit for bit
    fs1 = _fs1()
    spec = inputs.batch_spec(9, 128, 9000, [1e-2, 3e-3], seed=17)
    mu, nu, offs = inputs.batch_hists(spec)
    tol = [1e-6] * 9
    _say("batched device eps/tol")
    host = fs1.fs1_solve_batched(dev(mu), dev(nu), offs, spec.eps, tol, itr_max=400,
                                 dtype="f32")
    on_dev = fs1.fs1_solve_batched(dev(mu), dev(nu), offs, dev(spec.eps), dev(tol),
                                   itr_max=400, dtype="f32")
    for a, b in zip(host, on_dev):
        assert _same(a, b), (a, b)
    with pytest.raises(ValueError):
        fs1.fs1_solve_batched(dev(mu), dev(nu), offs, dev(spec.eps), tol, itr_max=10)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batched_instance_beyond_prefetch_carries(dtype):
    # an instance of more than 1024 chunks (runs of 8 in binary64: 2048 entries
    # per chunk; runs of 16 in binary32: 4096) takes its carries from the
    # instance's aggregates by the whole-wavefront sums, beside a small one
    fs1 = _fs1()
    n_big = 2_500_000 if dtype == "f64" else 4_300_000
    m1, v1 = inputs.mixture_pair(n_big, 4, 31)
    m2, v2 = inputs.mixture_pair(3000, 3, 32)
    mu, nu, offs = _pack([(m1, v1), (m2, v2)])
    eps = [1e-3, 1e-2]
    its = 6
    _say(f"batched large instance {dtype} n={n_big}")
    res = fs1.fs1_solve_batched(dev(mu), dev(nu), offs, eps, [0.0, 0.0], itr_max=its,
                                dtype=dtype)
    for (m, v), e, r in zip([(m1, v1), (m2, v2)], eps, res):
        ref = oracle.fs1_log(m, v, 1.0 / len(m), e, tol=0.0, itr_max=its)
        assert r.status == 0 and r.iterations == its
        assert r.w1 == pytest.approx(ref.w1, rel=1e-9 if dtype == "f64" else 1e-5)
        assert r.marginal_err == pytest.approx(ref.marginal_err, rel=1e-5 if dtype == "f64" else 1e-3)
