"""Property tests of the GPU path over random (N, eps, seed, dtype, solver) on
grids of at most 512 entries, against the dense oracle: the kernel product
(Sec. 3, eq. (recursion)) element by element, and Algorithm 1 in the
log-domain after a drawn number of iterations (W, potentials, marginal
error).  Examples are derandomised and few, so every run draws the same
cases and the whole file takes seconds.  Bounds as in test_gpu_kv.py and
test_gpu_solve.py: 64 u (binary64) and 256 u (binary32) of K|x| for the
product, plus the output format's underflow floor; W to 1e-10 relative and potentials to 1e-9 in binary64, W to 1e-5
in binary32 scans against the binary64 oracle."""
import math
import sys

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_2202_10042_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SETTINGS = settings(max_examples=40, deadline=None, derandomize=True, database=None,
                    suppress_health_check=[HealthCheck.too_slow])
U64 = 2.0 ** -53
U32 = 2.0 ** -24


def _fs1():
    from paper_2202_10042_amd import fs1
    return fs1


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a, dt=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dt, device="cuda")


@SETTINGS
@given(n=st.integers(min_value=1, max_value=512),
       lc=st.floats(min_value=math.log(1e-4), max_value=math.log(100.0)),
       seed=st.integers(min_value=0, max_value=2 ** 31 - 1), f32=st.booleans())
def test_kv_apply_property(n, lc, seed, f32):
    fs1 = _fs1()
    c = math.exp(lc)
    h = 1.0 / n
    eps = h / c
    _say(f"kv property n={n} c={c:.4g} seed={seed} f32={f32}")
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n)
    x[rng.random(n) < 0.1] = 0.0
    tdt = torch.float32 if f32 else torch.float64
    if f32:
        x = x.astype(np.float32).astype(np.float64)
    y = fs1.fs1_kv_apply(dev(x, tdt), h, eps).double().cpu().numpy()
    ref = oracle.kv_dense(x, h, eps)
    scale = oracle.kv_dense(np.abs(x), h, eps)
    # plus the output format's underflow floor: a true value below the smallest
    # denormal (2^-149 in binary32, 2^-1074 in binary64) cannot be returned
    floor = 4.0 * (2.0 ** -149 if f32 else 2.0 ** -1074)
    tol = (256 * U32 if f32 else 64 * U64) * scale
    assert np.all(np.abs(y - ref) <= tol + floor)


@SETTINGS
@given(n=st.integers(min_value=2, max_value=512),
       le=st.floats(min_value=math.log(1e-3), max_value=math.log(0.3)),
       seed=st.integers(min_value=0, max_value=99999), its=st.integers(min_value=1, max_value=40),
       f32=st.booleans(), solver=st.sampled_from(["auto", "fused", "general", "persistent"]))
def test_log_solve_property(n, le, seed, its, f32, solver):
    fs1 = _fs1()
    eps = math.exp(le)
    h = 1.0 / n
    _say(f"solve property n={n} eps={eps:.4g} seed={seed} its={its} f32={f32} {solver}")
    mu, nu = inputs.mixture_pair(n, inputs.random_k(seed), seed)
    # tol 0: the drawn count of iterations, unless the error reaches exactly 0
    # first, which happens only at the rounding level and may then differ
    # by an iteration between the two sides
    ref = oracle.sinkhorn_log_dense(mu, nu, h, eps, tol=0.0, itr_max=its)
    r = fs1.fs1_solve(dev(mu), dev(nu), eps, 0.0, itr_max=its, dtype="f32" if f32 else "f64",
                      domain="log", potentials=True, solver=solver)
    assert r.status == 0
    if r.iterations != ref.iterations:
        assert max(r.marginal_err, ref.marginal_err) <= (1e-6 if f32 else 1e-15)
        assert r.w1 == pytest.approx(ref.w1, rel=1e-5 if f32 else 1e-9)
        return
    if f32:
        assert r.w1 == pytest.approx(ref.w1, rel=1e-5, abs=1e-300)
        return
    assert r.w1 == pytest.approx(ref.w1, rel=1e-10, abs=1e-300)
    assert r.marginal_err == pytest.approx(ref.marginal_err, rel=1e-6, abs=1e-12)
    F = r.F.cpu().numpy()
    G = r.G.cpu().numpy()
    m, v = mu > 0, nu > 0
    assert np.max(np.abs(F[m] - ref.a[m])) <= 1e-9
    assert np.max(np.abs(G[v] - ref.b[v])) <= 1e-9


@settings(max_examples=12, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow])
@given(sizes=st.lists(st.integers(min_value=1, max_value=6000), min_size=1, max_size=6),
       les=st.lists(st.floats(min_value=math.log(1e-3), max_value=math.log(0.1)), min_size=6,
                    max_size=6),
       seed=st.integers(min_value=0, max_value=99999), its=st.integers(min_value=1, max_value=30),
       f32=st.booleans())
def test_batched_property(sizes, les, seed, its, f32):
    # a random ragged batch at a fixed iteration count: every instance against
    # the log-domain oracle (sequential for n > 600, dense below)
    fs1 = _fs1()
    B = len(sizes)
    eps = [math.exp(v) for v in les[:B]]
    _say(f"batched property sizes={sizes} its={its} f32={f32}")
    pairs = [inputs.mixture_pair(n, 3, seed + 7 * i) if n > 2 else
             (np.full(n, 1.0 / n), np.full(n, 1.0 / n)) for i, n in enumerate(sizes)]
    offs = np.zeros(B + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    mu = np.concatenate([m for m, _ in pairs])
    nu = np.concatenate([v for _, v in pairs])
    res = fs1.fs1_solve_batched(dev(mu), dev(nu), offs, eps, [0.0] * B, itr_max=its,
                                dtype="f32" if f32 else "f64")
    for (m, v), e, r in zip(pairs, eps, res):
        n = len(m)
        ref = (oracle.fs1_log if n > 600 else oracle.sinkhorn_log_dense)(
            m, v, 1.0 / n, e, tol=0.0, itr_max=its)
        assert r.status == 0
        if r.iterations != ref.iterations:
            # the error reached exactly 0 on one side (rounding level)
            assert max(r.marginal_err, ref.marginal_err) <= (1e-6 if f32 else 1e-15)
            continue
        assert r.w1 == pytest.approx(ref.w1, rel=1e-5 if f32 else 1e-10, abs=1e-300)


@settings(max_examples=20, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow])
@given(dims=st.lists(st.integers(min_value=1, max_value=40), min_size=1, max_size=4),
       lcs=st.lists(st.floats(min_value=math.log(1e-3), max_value=math.log(50.0)),
                    min_size=4, max_size=4),
       seed=st.integers(min_value=0, max_value=2 ** 31 - 1), f32=st.booleans())
def test_kv_apply_nd_property(dims, lcs, seed, f32):
    # the product on up to four axes against the D-axis oracle's recursions
    # (positive inputs): 64 u per axis plus summation order, 128 u D
    fs1 = _fs1()
    eps = 0.05
    h = [math.exp(lc) * eps for lc in lcs[:len(dims)]]
    n = int(np.prod(dims))
    _say(f"kv_nd property dims={dims} seed={seed} f32={f32}")
    rng = np.random.default_rng(seed)
    x = rng.random(n) + 0.1
    tdt = torch.float32 if f32 else torch.float64
    if f32:
        x = x.astype(np.float32).astype(np.float64)
    y = fs1.fs1_kv_apply_nd(dev(x, tdt), dims, h, eps).double().cpu().numpy()
    ref = oracle.kvn_fs1(x, dims, h, eps)
    u = U32 if f32 else U64
    tiny = (2.0 ** -149 if f32 else 2.0 ** -1074) * 4
    assert np.all(np.abs(y - ref) <= 128 * u * len(dims) * ref + tiny)
