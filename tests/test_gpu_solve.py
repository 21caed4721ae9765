"""GPU parity of fs1_solve against the CPU oracle.

Tolerances:
  * binary64 (plain or log) at a fixed iteration count: |dW|/W <= 1e-10 and
    potentials ln phi, ln psi within 1e-9 (absolute, on entries with positive
    marginal) of the oracle's;
  * binary32 scans (log domain) against the binary64 oracle: |dW|/W <= 1e-5;
  * the marginal error is reported in binary64 in every mode and is compared to
    the oracle's at 1e-6 relative plus 1e-12 absolute (binary64).
"""
import math
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


def _pot_close(got, ref_lin, mask, atol):
    ref = np.log(ref_lin[mask])
    g = got[mask]
    assert np.max(np.abs(g - ref)) <= atol, float(np.max(np.abs(g - ref)))


# solver paths: "auto" (one resident workgroup for n <= 1024 R, else fused
# one-launch-per-half kernels where they apply), "fused" (auto without the
# resident workgroup), "general" (extended-range scans + carry kernel),
# "persistent" (one cooperative launch)
PATHS = ["auto", "fused", "general", "persistent"]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("domain", ["plain", "log"])
@pytest.mark.parametrize("n,seed,its", [(1000, 1, 5), (1000, 2, 60), (1, 0, 3), (2, 0, 4),
                                        (2049, 3, 25), (4097, 4, 25), (10001, 5, 12)])
def test_solve_f64_fixed_iterations(domain, n, seed, its, path):
    fs1 = _fs1()
    _say(f"solve f64 {domain} n={n} seed={seed} its={its} {path}")
    mu, nu = inputs.mixture_pair(n, 2, seed) if n > 2 else (np.array([0.3, 0.7][:n]) / sum([0.3, 0.7][:n]), np.array([0.6, 0.4][:n]) / sum([0.6, 0.4][:n]))
    h = 1.0 / n
    eps = 0.01
    ref = oracle.fs1(mu, nu, h, eps, tol=0.0, itr_max=its) if n > 2000 else \
        oracle.sinkhorn_dense(mu, nu, h, eps, tol=0.0, itr_max=its)
    r = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=its, dtype="f64", domain=domain,
                      potentials=True, solver=path)
    # (for n = 1 the initial error is exactly 0 and Algorithm 1 stops at once)
    assert r.status == 0 and r.iterations == ref.iterations
    assert r.w1 == pytest.approx(ref.w1, rel=1e-10, abs=1e-300)
    assert r.marginal_err == pytest.approx(ref.marginal_err, rel=1e-6, abs=1e-12)
    assert r.mu_err <= 1e-12
    F = r.F.cpu().numpy()
    G = r.G.cpu().numpy()
    _pot_close(F, ref.a, mu > 0, 1e-9)
    _pot_close(G, ref.b, nu > 0, 1e-9)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("domain", ["plain", "log"])
def test_solve_c1_to_tolerance(domain, path):
    # single pair, N = 1000, eps = 0.01, tol 1e-9 (stop on the nu-side L1 error)
    fs1 = _fs1()
    n = 1000
    h = 1.0 / n
    for seed in (1, 2, 4):
        _say(f"solve C1 to tol {domain} seed={seed} {path}")
        mu, nu = inputs.mixture_pair(n, 2, seed)
        ref = oracle.sinkhorn_dense(mu, nu, h, 0.01, tol=1e-9, itr_max=2000)
        r = fs1.fs1_solve(dev(mu), dev(nu), 0.01, 1e-9, itr_max=2000, domain=domain,
                          solver=path)
        assert r.status == 0 and r.converged and ref.converged
        # the stopping iteration may differ by one where err(l) is within rounding of tol
        assert abs(r.iterations - ref.iterations) <= 1
        if r.iterations == ref.iterations:
            assert r.w1 == pytest.approx(ref.w1, rel=1e-10)
        else:
            assert r.w1 == pytest.approx(ref.w1, rel=1e-8)
        assert r.marginal_err <= 1e-9


@pytest.mark.parametrize("path", PATHS)
def test_solve_log_f32_against_f64_oracle(path):
    fs1 = _fs1()
    for n, eps, its in [(1000, 0.01, 80), (20000, 1e-3, 40), (4099, 3e-3, 30)]:
        _say(f"solve f32 log n={n} eps={eps} its={its} {path}")
        mu, nu = inputs.mixture_pair(n, 3, 21)
        h = 1.0 / n
        ref = oracle.fs1_log(mu, nu, h, eps, tol=0.0, itr_max=its)
        r = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=its, dtype="f32", domain="log",
                          potentials=True, solver=path)
        assert r.status == 0
        assert r.w1 == pytest.approx(ref.w1, rel=1e-5)
        m = nu > 0
        assert np.max(np.abs(r.G.cpu().numpy()[m] - ref.b[m])) <= 1e-4


@pytest.mark.parametrize("dtype,domain", [("f64", "plain"), ("f64", "log"), ("f32", "log")])
def test_solve_dirac(dtype, domain):
    fs1 = _fs1()
    for n, a, b in [(20, 3, 11), (5000, 4999, 0), (3000, 1200, 1200)]:
        _say(f"dirac {dtype} {domain} n={n}")
        mu, nu = inputs.dirac_pair(n, a, b)
        h = 1.0 / n
        eps = 0.1 if domain == "plain" else 0.01
        if domain == "plain" and abs(a - b) * h / eps > 600:
            eps = abs(a - b) * h / 600
        r = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=1, dtype=dtype, domain=domain)
        assert r.status == 0
        assert r.marginal_err <= (1e-15 if dtype == "f64" else 1e-6)
        assert r.w1 == pytest.approx(abs(a - b) * h, rel=1e-14 if dtype == "f64" else 1e-6,
                                     abs=1e-300)


def test_plain_fails_log_succeeds():
    # far-apart Dirac masses (|a-b| h/eps = 900): K_ab underflows in binary64;
    # the plain iteration must report abnormal termination, the log one is exact
    fs1 = _fs1()
    n, a, b = 100, 0, 90
    h = 1.0 / n
    eps = h / 10.0
    mu, nu = inputs.dirac_pair(n, a, b)
    _say("plain failure")
    r = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=3, domain="plain")
    assert r.status == fs1.FS1_ERR_NONFINITE and r.iterations == 0
    _say("log success")
    r = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=3, domain="log")
    assert r.status == 0 and r.w1 == pytest.approx(90 * h, rel=1e-13)
    # the Ricker workload of Sec. 5.2 at eps = 1e-3: plain terminates abnormally
    u, v, dt = inputs.ricker_pair(500)
    o = oracle.fs1(u, v, dt, 1e-3, tol=0.0, itr_max=500)
    _say("ricker plain / log")
    r = fs1.fs1_solve(dev(u), dev(v), 1e-3, 0.0, h=dt, itr_max=500, domain="plain")
    # the failing iteration depends on underflow details: the dense and the
    # sequential oracles already disagree on it, so only the outcome is pinned
    assert o.status == -2
    assert r.status == fs1.FS1_ERR_NONFINITE and r.iterations < 500
    rl = fs1.fs1_solve(dev(u), dev(v), 1e-3, 0.0, h=dt, itr_max=500, domain="log")
    ol = oracle.fs1_log(u, v, dt, 1e-3, tol=0.0, itr_max=500)
    assert rl.status == 0 and rl.w1 == pytest.approx(ol.w1, rel=1e-9)


def test_solve_invalid_marginals():
    fs1 = _fs1()
    n = 300
    mu, nu = inputs.mixture_pair(n, 2, 1)
    _say("invalid marginals")
    with pytest.raises(fs1.Fs1Error):
        fs1.fs1_solve(dev(mu), dev(nu * 1.01), 0.01, 0.0, itr_max=2)
    bad = mu.copy()
    bad[5] = -bad[5]
    with pytest.raises(fs1.Fs1Error):
        fs1.fs1_solve(dev(bad), dev(nu), 0.01, 0.0, itr_max=2)
    bad = mu.copy()
    bad[7] = np.nan
    with pytest.raises(fs1.Fs1Error):
        fs1.fs1_solve(dev(bad), dev(nu), 0.01, 0.0, itr_max=2)
    with pytest.raises(fs1.Fs1Error):
        fs1.fs1_solve(dev(np.zeros(n)), dev(np.zeros(n)), 0.01, 0.0, itr_max=2)
    # an empty grid is an argument error, not a launch
    empty = dev(np.zeros(0))
    for domain in ("plain", "log", "absorb"):
        with pytest.raises(fs1.Fs1Error):
            fs1.fs1_solve(empty, empty, 0.01, 0.0, itr_max=2, domain=domain)


@pytest.mark.parametrize("path", PATHS)
def test_error_history_and_check_interval(path):
    fs1 = _fs1()
    n = 400
    mu, nu = inputs.mixture_pair(n, 2, 7)
    h = 1.0 / n
    _say(f"error history {path}")
    r = fs1.fs1_solve(dev(mu), dev(nu), 0.01, 0.0, itr_max=12, domain="log", err_history=True,
                      solver=path)
    hist = r.err_history.cpu().numpy()
    for l in range(12):
        ref = oracle.fs1(mu, nu, h, 0.01, tol=0.0, itr_max=l).marginal_err
        assert hist[l] == pytest.approx(ref, rel=1e-9, abs=1e-14)
    assert np.isnan(hist[12])
    # the result does not depend on the host polling interval; with check_every
    # k the stop happens at the first multiple of k with err <= tol
    base = fs1.fs1_solve(dev(mu), dev(nu), 0.01, 1e-8, itr_max=3000, domain="log", solver=path)
    for se in (1, 5, 64):
        r = fs1.fs1_solve(dev(mu), dev(nu), 0.01, 1e-8, itr_max=3000, domain="log", sync_every=se,
                          solver=path)
        assert r.iterations == base.iterations and r.w1 == base.w1
    r = fs1.fs1_solve(dev(mu), dev(nu), 0.01, 1e-8, itr_max=3000, domain="log", check_every=7,
                      solver=path)
    assert r.iterations % 7 == 0 and base.iterations <= r.iterations < base.iterations + 7


@pytest.mark.parametrize("path", PATHS)
def test_solve_deterministic(path):
    fs1 = _fs1()
    n = 70001
    mu, nu = inputs.mixture_pair(n, 4, 3)
    _say(f"determinism {path}")
    a = fs1.fs1_solve(dev(mu), dev(nu), 1e-3, 0.0, itr_max=30, domain="log", potentials=True,
                      solver=path)
    b = fs1.fs1_solve(dev(mu), dev(nu), 1e-3, 0.0, itr_max=30, domain="log", potentials=True,
                      solver=path)
    assert a.w1 == b.w1 and a.marginal_err == b.marginal_err
    assert torch.equal(a.F, b.F) and torch.equal(a.G, b.G)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_solver_paths_agree(dtype):
    # the solvers differ only in the in-chunk arithmetic (frame vs extended
    # range) and the launch structure, so they agree to rounding
    fs1 = _fs1()
    n = 300007
    mu, nu = inputs.mixture_pair(n, 5, 8)
    _say(f"solver paths agree {dtype}")
    rs = [fs1.fs1_solve(dev(mu), dev(nu), 1e-3, 1e-7, itr_max=800, domain="log", dtype=dtype,
                        solver=p) for p in PATHS]
    for r in rs[1:]:
        assert abs(r.iterations - rs[0].iterations) <= 1
        assert r.w1 == pytest.approx(rs[0].w1, rel=1e-11 if dtype == "f64" else 1e-5)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("eps", [1e-3, 1e-4])
def test_solve_full_size_f64_log(eps, path):
    # N = 2^20 (the single-pair workload), 6 iterations against the sequential
    # FS-1 oracle in the log domain, at the binary64 bar (W 1e-10, potentials
    # 1e-9); 50 iterations and per-step checks in test_gpu_fullsize.py
    fs1 = _fs1()
    n = 1 << 20
    its = 6
    mu, nu = inputs.mixture_pair(n, 4, 5)
    h = 1.0 / n
    _say(f"full size f64 log eps={eps}")
    ref = oracle.fs1_log(mu, nu, h, eps, tol=0.0, itr_max=its)
    r = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=its, domain="log", potentials=True,
                      solver=path)
    assert r.status == 0
    assert r.w1 == pytest.approx(ref.w1, rel=1e-10)
    assert r.marginal_err == pytest.approx(ref.marginal_err, rel=1e-6)
    G = r.G.cpu().numpy()
    F = r.F.cpu().numpy()
    assert np.max(np.abs(G - ref.b)) <= 1e-9 and np.max(np.abs(F - ref.a)) <= 1e-9
    _say(f"full size f32 log eps={eps}")
    r32 = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=its, dtype="f32", domain="log",
                        solver=path)
    assert r32.status == 0 and r32.w1 == pytest.approx(ref.w1, rel=1e-5)


@pytest.mark.parametrize("dtype,c", [("f64", 0.5), ("f64", 0.05), ("f32", 0.02), ("f32", 0.005)])
def test_fused_run_lengths(dtype, c):
    # the fused path's run length follows h/eps = c (binary64: 8 entries while
    # a chunk frame of 2048 entries fits, else 4; binary32: 16, else 8), on a
    # ragged grid of several chunks, against the log-domain oracle
    fs1 = _fs1()
    n = 30011
    h = 1.0 / n
    eps = h / c
    mu, nu = inputs.mixture_pair(n, 3, 77)
    _say(f"fused run lengths {dtype} c={c}")
    its = 25
    ref = oracle.fs1_log(mu, nu, h, eps, tol=0.0, itr_max=its)
    r = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=its, dtype=dtype, domain="log",
                      potentials=True, solver="fused")
    g = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=its, dtype=dtype, domain="log",
                      solver="general")
    assert r.status == 0 and r.iterations == its
    rel = 1e-10 if dtype == "f64" else 1e-5
    assert r.w1 == pytest.approx(ref.w1, rel=rel)
    assert r.w1 == pytest.approx(g.w1, rel=1e-12 if dtype == "f64" else 1e-5)
    m = nu > 0
    assert np.max(np.abs(r.G.cpu().numpy()[m] - ref.b[m])) <= (1e-9 if dtype == "f64" else 1e-4)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_persistent_single_launch_full_size(dtype):
    # N = 2^20 at eps 1e-3 to tol 1e-8 (1e-6 in binary32, whose rounding
    # floor is near 1e-7): the persistent solver must take its one cooperative
    # launch (512 chunks in binary64, 256 in binary32) and agree with the
    # fused per-half kernels; only the summation order of the stopping error
    # differs, so the stop may move by one iteration
    fs1 = _fs1()
    n = 1 << 20
    tol = 1e-8 if dtype == "f64" else 1e-6
    mu, nu = inputs.mixture_pair(n, inputs.random_k(1), 1)
    ctx = fs1.Context()
    ctx.set_profiling(1)
    _say(f"persistent full size {dtype}")
    r = fs1.fs1_solve(dev(mu), dev(nu), 1e-3, tol, itr_max=5000, dtype=dtype, domain="log",
                      solver="persistent", sync_every=64, ctx=ctx)
    _, launches, _ = ctx.kernel_stats()
    assert launches == 1
    f = fs1.fs1_solve(dev(mu), dev(nu), 1e-3, tol, itr_max=5000, dtype=dtype, domain="log",
                      solver="fused", sync_every=64)
    assert r.status == 0 and f.status == 0
    assert r.iterations < 5000 and abs(r.iterations - f.iterations) <= 1
    rel = 1e-11 if dtype == "f64" else 1e-5
    if r.iterations == f.iterations:
        assert r.w1 == pytest.approx(f.w1, rel=rel)
    # the stop test runs in the working precision, the reported error in
    # binary64: in binary32 the two differ by a few per cent
    assert r.marginal_err <= (tol if dtype == "f64" else 1.1 * tol)
    # a fixed iteration count: same iterates, agreement to rounding
    r = fs1.fs1_solve(dev(mu), dev(nu), 1e-3, 0.0, itr_max=37, dtype=dtype, domain="log",
                      solver="persistent", potentials=True)
    f = fs1.fs1_solve(dev(mu), dev(nu), 1e-3, 0.0, itr_max=37, dtype=dtype, domain="log",
                      solver="fused", potentials=True)
    assert r.iterations == f.iterations == 37
    assert r.w1 == pytest.approx(f.w1, rel=rel)
    assert r.marginal_err == pytest.approx(f.marginal_err, rel=1e-6 if dtype == "f64" else 1e-2)
    m = nu > 0
    tol_pot = 1e-9 if dtype == "f64" else 1e-3
    assert np.max(np.abs(r.G.cpu().numpy()[m] - f.G.cpu().numpy()[m])) <= tol_pot


@pytest.mark.parametrize("domain", ["plain", "log"])
@pytest.mark.parametrize("dtype,n", [("f64", 511), ("f64", 512), ("f64", 513), ("f32", 1024),
                                     ("f32", 1025), ("f64", 2047), ("f64", 2048), ("f64", 2049),
                                     ("f64", 4096), ("f64", 4097), ("f64", 5000), ("f64", 8192),
                                     ("f64", 8193), ("f32", 4096), ("f32", 4097), ("f32", 8192)])
def test_resident_workgroup_sizes(dtype, n, domain):
    """The one-workgroup solver at the edges of its workgroup sizes (one
    wavefront up to 64 R entries, 256 threads up to 256 R, 1024 threads up to
    1024 R with R <= 8; binary64 grids of 2049 to 8192 entries and binary32
    grids of 4097 to 8192 take runs of 16 on 256 or 512 threads) against the oracle at a fixed iteration count and
    against the general path (same arithmetic, other association order).  A
    grid of 8193 binary64 entries is past the one-workgroup limit."""
    fs1 = _fs1()
    mu, nu = inputs.mixture_pair(n, 3, n)
    h = 1.0 / n
    # plain binary32 overflows at small eps (scalings reach e^(1/eps)), as the
    # paper's unstabilised iteration does: a larger eps there
    eps = 5e-2 if (dtype == "f32" and domain == "plain") else 2e-3
    its = 40
    _say(f"resident {dtype} {domain} n={n}")
    ref = oracle.fs1_log(mu, nu, h, eps, tol=0.0, itr_max=its)
    r = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=its, dtype=dtype, domain=domain,
                      potentials=True)
    g = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=its, dtype=dtype, domain=domain,
                      solver="general")
    assert r.status == 0 and g.status == 0 and r.iterations == its
    rel = 1e-10 if dtype == "f64" else 1e-5
    assert r.w1 == pytest.approx(ref.w1, rel=rel)
    assert r.w1 == pytest.approx(g.w1, rel=1e-12 if dtype == "f64" else 1e-5)
    assert r.marginal_err == pytest.approx(ref.marginal_err, rel=1e-6 if dtype == "f64" else 1e-2,
                                           abs=1e-12 if dtype == "f64" else 1e-6)
    m = nu > 0
    assert np.max(np.abs(r.G.cpu().numpy()[m] - ref.b[m])) <= (1e-9 if dtype == "f64" else 1e-4)
    # to tolerance: the stop decision of Algorithm 1 inside the launch
    t = fs1.fs1_solve(dev(mu), dev(nu), eps, 1e-6, itr_max=5000, dtype=dtype, domain=domain)
    tg = fs1.fs1_solve(dev(mu), dev(nu), eps, 1e-6, itr_max=5000, dtype=dtype, domain=domain,
                       solver="general")
    assert t.status == 0 and t.converged == tg.converged
    # binary64: the stop may move by one where err(l) is within rounding of
    # tol; binary32: its rounding noise on err (~1e-8 here) spans a few
    # iterations of the slow final decrease
    slack = 1 if dtype == "f64" else max(1, tg.iterations // 50)
    assert abs(t.iterations - tg.iterations) <= slack


@pytest.mark.parametrize("c", [39.0, 41.0])
def test_resident_runs_of_16_exponent_bound(c):
    """Binary64 log-domain grids of 2049 to 8192 entries take runs of 16 only
    while 15 h/eps stays inside the scaled arithmetic's exponent range (h/eps
    <= 40); beyond it they keep runs of 8 on 1024 threads.  Both sides of the
    bound against the oracle and the general path."""
    fs1 = _fs1()
    n, its = 3000, 20
    mu, nu = inputs.mixture_pair(n, 3, 7)
    h = 1.0 / n
    eps = h / c
    _say(f"resident runs of 16 bound c={c}")
    ref = oracle.fs1_log(mu, nu, h, eps, tol=0.0, itr_max=its)
    r = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=its, dtype="f64", domain="log",
                      potentials=True)
    g = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=its, dtype="f64", domain="log",
                      solver="general")
    assert r.status == 0 and g.status == 0 and r.iterations == its
    assert r.w1 == pytest.approx(ref.w1, rel=1e-10)
    assert r.w1 == pytest.approx(g.w1, rel=1e-12)
    assert r.marginal_err == pytest.approx(ref.marginal_err, rel=1e-6, abs=1e-12)
    m = nu > 0
    # at eps = h / 40 the potentials reach a few hundred: the bound is relative
    scale = max(1.0, float(np.max(np.abs(ref.b[m]))))
    assert np.max(np.abs(r.G.cpu().numpy()[m] - ref.b[m])) <= 1e-11 * scale


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_solve_two_level_carries_general_path(dtype):
    """A grid of more than 1024 chunks on the general path (two-level carries)
    against the sequential oracle at a fixed iteration count."""
    fs1 = _fs1()
    n = 2_500_003
    mu, nu = inputs.mixture_pair(n, 4, 21)
    eps = 1e-3
    its = 12
    _say(f"two-level solve {dtype} n={n}")
    ref = oracle.fs1_log(mu, nu, 1.0 / n, eps, tol=0.0, itr_max=its)
    r = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=its, dtype=dtype, domain="log",
                      solver="general")
    assert r.status == 0 and r.iterations == its
    assert r.w1 == pytest.approx(ref.w1, rel=1e-10 if dtype == "f64" else 1e-5)
    assert r.marginal_err == pytest.approx(ref.marginal_err, rel=1e-6 if dtype == "f64" else 1e-3)
    # and the same grid through the default solver selection
    r2 = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=its, dtype=dtype, domain="log")
    assert r2.w1 == pytest.approx(ref.w1, rel=1e-10 if dtype == "f64" else 1e-5)



# ---------------------------------------------------------------------------
# The threshold form of the stabilisation (domain "absorb": scaled vectors
# with binary64 potentials, absorption when the largest scaled entry exceeds
# tau) against the oracle's stabilised FS-1 with the same tau.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,eps,its,tau", [(300, 1e-2, 60, 1e3), (300, 1e-3, 200, 10.0),
                                          (2049, 1e-3, 120, 1e3), (5000, 5e-4, 80, 1e3)])
def test_absorb_domain_against_oracle(dtype, n, eps, its, tau):
    fs1 = _fs1()
    mu, nu = inputs.mixture_pair(n, 3, n + 1)
    h = 1.0 / n
    _say(f"absorb {dtype} n={n} eps={eps} tau={tau}")
    ref = oracle.fs1_absorb(mu, nu, h, eps, tol=0.0, itr_max=its, tau=tau)
    assert ref.status == 0
    r = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=its, dtype=dtype, domain="absorb",
                      tau=tau, potentials=True)
    assert r.status == 0 and r.iterations == its
    m = nu > 0
    if dtype == "f64":
        assert r.w1 == pytest.approx(ref.w1, rel=1e-10)
        assert r.marginal_err == pytest.approx(ref.marginal_err, rel=1e-6, abs=1e-12)
        assert np.max(np.abs(r.G.cpu().numpy()[m] - ref.G[m])) <= 1e-9
        # the test max > tau is taken on values equal to rounding
        assert abs(r.absorptions - ref.absorptions) <= 1
    else:
        assert r.w1 == pytest.approx(ref.w1, rel=1e-5)
        assert np.max(np.abs(r.G.cpu().numpy()[m] - ref.G[m])) <= 1e-4
    assert ref.absorptions > 0


def test_absorb_domain_ricker_and_stop():
    # Sec. 5.2: at eps = 1e-3 the unstabilised iteration terminates abnormally
    # and the stabilised one does not
    fs1 = _fs1()
    u, v, dt = inputs.ricker_pair(500)
    p = fs1.fs1_solve(dev(u), dev(v), 1e-3, 0.0, h=dt, itr_max=500, domain="plain")
    assert p.status == fs1.FS1_ERR_NONFINITE
    ref = oracle.fs1_absorb(u, v, dt, 1e-3, tol=0.0, itr_max=500, tau=1e3)
    r = fs1.fs1_solve(dev(u), dev(v), 1e-3, 0.0, h=dt, itr_max=500, domain="absorb", tau=1e3)
    assert r.status == 0 and r.absorptions > 0
    assert r.w1 == pytest.approx(ref.w1, rel=1e-9)
    # to tolerance
    n = 400
    mu, nu = inputs.mixture_pair(n, 2, 3)
    ref = oracle.fs1_absorb(mu, nu, 1.0 / n, 0.01, tol=1e-9, itr_max=5000, tau=100.0)
    r = fs1.fs1_solve(dev(mu), dev(nu), 0.01, 1e-9, itr_max=5000, domain="absorb", tau=100.0)
    assert r.status == 0 and r.converged and abs(r.iterations - ref.iterations) <= 1


def test_absorb_domain_arguments():
    fs1 = _fs1()
    x = dev(np.full(100, 0.01))
    with pytest.raises(fs1.Fs1Error):
        fs1.fs1_solve(x, x, 0.01, 0.0, itr_max=5, domain="absorb", tau=0.0)
    with pytest.raises(fs1.Fs1Error):
        fs1.fs1_solve(x, x, 0.01, 0.0, itr_max=5, domain="absorb", tau=float("inf"))
    with pytest.raises(fs1.Fs1Error):
        fs1.fs1_solve(x, x, 0.01, 0.0, itr_max=5, domain="absorb", solver="persistent")


# The threshold form on the multi-workgroup (general) path.  One chunk carries
# 256 R entries (R = 8 in binary64, 16 in binary32).  Grids that fit one
# workgroup are sent to the general path by the solver choice and compared
# with the stabilised oracle (absorption counts included); larger grids
# (n = 20011, 300007, and 2^21 + 3, which has more than 1024 chunks in
# binary64 and takes the two-level carry scan) are compared with the
# log-domain oracle, whose iterates are the same in exact arithmetic (the
# stabilised oracle's transport cost is a literal double sum, too slow there).
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,eps,its,tau", [(5000, 5e-4, 80, 1e3), (6007, 2e-4, 60, 10.0)])
def test_absorb_general_path_against_oracle(dtype, n, eps, its, tau):
    fs1 = _fs1()
    mu, nu = inputs.mixture_pair(n, 4, n + 5)
    h = 1.0 / n
    _say(f"absorb general {dtype} n={n} eps={eps} tau={tau}")
    ref = oracle.fs1_absorb(mu, nu, h, eps, tol=0.0, itr_max=its, tau=tau)
    assert ref.status == 0 and ref.absorptions > 0
    r = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=its, dtype=dtype, domain="absorb",
                      tau=tau, potentials=True, solver="general")
    assert r.status == 0 and r.iterations == its
    m = nu > 0
    if dtype == "f64":
        assert r.w1 == pytest.approx(ref.w1, rel=1e-10)
        assert r.marginal_err == pytest.approx(ref.marginal_err, rel=1e-6, abs=1e-12)
        assert np.max(np.abs(r.G.cpu().numpy()[m] - ref.G[m])) <= 1e-8
        assert np.max(np.abs(r.F.cpu().numpy()[mu > 0] - ref.F[mu > 0])) <= 1e-8
        # the test max > tau is taken on values equal to rounding
        assert abs(r.absorptions - ref.absorptions) <= 1
    else:
        assert r.w1 == pytest.approx(ref.w1, rel=1e-5)
        assert np.max(np.abs(r.G.cpu().numpy()[m] - ref.G[m])) <= 1e-3
        assert r.absorptions > 0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,eps,its,tau", [(20011, 1e-4, 60, 1e3), (20011, 1e-4, 60, 10.0),
                                          (300007, 2e-5, 40, 1e3), ((1 << 21) + 3, 1e-5, 8, 10.0)])
def test_absorb_general_path_large(dtype, n, eps, its, tau):
    fs1 = _fs1()
    mu, nu = inputs.mixture_pair(n, 4, n + 5)
    h = 1.0 / n
    _say(f"absorb general large {dtype} n={n} eps={eps} tau={tau}")
    ref = oracle.fs1_log(mu, nu, h, eps, tol=0.0, itr_max=its)
    r = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=its, dtype=dtype, domain="absorb",
                      tau=tau, potentials=True)
    assert r.status == 0 and r.iterations == its and r.absorptions > 0
    m = nu > 0
    if dtype == "f64":
        assert r.w1 == pytest.approx(ref.w1, rel=1e-9)
        assert r.marginal_err == pytest.approx(ref.marginal_err, rel=1e-6)
        assert np.max(np.abs(r.G.cpu().numpy()[m] - ref.b[m])) <= 1e-8
    else:
        assert r.w1 == pytest.approx(ref.w1, rel=1e-5)
        assert np.max(np.abs(r.G.cpu().numpy()[m] - ref.b[m])) <= 1e-3


def test_absorb_general_path_matches_one_workgroup():
    # n = 4096 fits one workgroup; the general path must give the same
    # iterates up to rounding and the same absorption count
    fs1 = _fs1()
    n = 4096
    mu, nu = inputs.mixture_pair(n, 3, 17)
    _say("absorb general vs one workgroup")
    a = fs1.fs1_solve(dev(mu), dev(nu), 1e-3, 0.0, itr_max=150, domain="absorb", tau=50.0,
                      potentials=True)
    b = fs1.fs1_solve(dev(mu), dev(nu), 1e-3, 0.0, itr_max=150, domain="absorb", tau=50.0,
                      potentials=True, solver="general")
    assert a.status == 0 and b.status == 0 and a.absorptions > 2
    assert abs(a.absorptions - b.absorptions) <= 1
    assert b.w1 == pytest.approx(a.w1, rel=1e-11)
    m = nu > 0
    assert np.max(np.abs(a.G.cpu().numpy()[m] - b.G.cpu().numpy()[m])) <= 1e-9


def test_absorb_general_path_to_tolerance():
    # to tolerance with frequent absorptions (tau = 2): the state returned at
    # the stop must be consistent (absorbed vectors with their new
    # potentials), and W, err and the stop iteration match the oracle's
    fs1 = _fs1()
    n = 12001
    mu, nu = inputs.mixture_pair(n, 3, 9)
    _say("absorb general to tolerance")
    ref = oracle.fs1_log(mu, nu, 1.0 / n, 1e-2, tol=1e-8, itr_max=4000)
    r = fs1.fs1_solve(dev(mu), dev(nu), 1e-2, 1e-8, itr_max=4000, domain="absorb", tau=2.0,
                      potentials=True)
    assert ref.converged and r.status == 0 and r.converged and r.absorptions > 10
    assert abs(r.iterations - ref.iterations) <= 1
    assert r.w1 == pytest.approx(ref.w1, rel=1e-9)
    assert r.marginal_err <= 1e-8
    if r.iterations == ref.iterations:
        m = nu > 0
        assert np.max(np.abs(r.G.cpu().numpy()[m] - ref.b[m])) <= 1e-8
