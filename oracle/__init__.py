"""CPU oracle for the FS-1 Sinkhorn method (arXiv 2202.10042).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline leg of
the benchmark use this package to check the GPU library; the library itself never
imports it.  The arithmetic lives in ``fs1_oracle.c`` (plain binary64 C, no code
shared with the GPU path); this module only marshals numpy arrays.

What each routine follows in the paper:

* ``kv_dense`` / ``kv_log_dense``: K x and ln K e^x with K_ij = exp(-|i-j| h/eps)
  formed entry by entry (Sec. 2, the kernel of the scaling form; Sec. 3, the full
  Toeplitz expansion of K psi).
* ``kv_fs1`` / ``kv_fs1_log``: the Sec. 3 recursions for the lower part p and the
  strict upper part q (Qin Jiushao / Horner form), and the same recursions on
  logarithms.
* ``sinkhorn_dense`` / ``sinkhorn_log_dense``: the Sinkhorn update of Sec. 2 (psi
  first, then phi) inside Algorithm 1's loop, stopping rule and return value, with
  K dense.
* ``fs1`` / ``fs1_log``: Algorithm 1 (FS-1) with the recursions; the log variant
  is the limit of the log-domain absorption (Sec. 2 and Sec. 3 remarks) where
  all of phi and psi is absorbed at every step.
* ``cost_*`` / ``marginal_err_*``: the returned double sum and the stopping-test
  double sum of Algorithm 1, literally (``*_dense``) and by recursions (``*_fs1``).
* ``kv2_*``, ``sinkhorn2_dense``, ``fs1_2d``, ``cost2_*``, ``marginal_err2_*``:
  the two-dimensional problem of Sec. 4 on an n1 x n2 grid in column-major order
  (entry (i, j) at i + n1 j): K dense from its definition, or Algorithm 2 (the
  1-D recursions along the first axis, then eq. (2d recursion) across columns);
  the cost as the literal double sum or split along the two axes.
* ``kvn_*``, ``sinkhornn_*``, ``fs1_nd*``, ``costn_*``, ``marginal_errn_*``: the
  same on D axes (first axis fastest; Sec. 4 says the construction extends to
  higher dimensions without writing it out): K = K_{D-1} (x) ... (x) K_0 by the
  1-D recursions along each axis in turn, the cost split into one term per axis.

Pins: every routine is checked in ``tests/test_oracle_pins.py`` against facts the
paper or the mathematics fixes (closed form of K 1 from the stability analysis of
Sec. 3, library products, Dirac marginals, the N = 2 closed form, the 1-D linear
programme / CDF formula, the entropic bound, the smooth-dual Newton solve, the
invariants and the plan differences of Tables 1 and 2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fs1_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libfs1_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile fs1_oracle.c with gcc (-O2, IEEE semantics, OpenMP)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    d = ctypes.c_double
    i64 = ctypes.c_int64
    p = ctypes.c_void_p
    sig = {
        "or_kv_dense": (ctypes.c_int, [i64, p, d, d, p]),
        "or_kv_dense_rows": (ctypes.c_int, [i64, p, d, d, p, i64, p]),
        "or_kv_log_dense": (ctypes.c_int, [i64, p, d, d, p]),
        "or_kv_log_dense_rows": (ctypes.c_int, [i64, p, d, d, p, i64, p]),
        "or_kv_fs1": (ctypes.c_int, [i64, p, d, d, p]),
        "or_kv_fs1_log": (ctypes.c_int, [i64, p, d, d, p]),
        "or_marginal_err_dense": (d, [i64, p, p, p, d, d]),
        "or_cost_dense": (d, [i64, p, p, d, d]),
        "or_marginal_err_log_dense": (d, [i64, p, p, p, d, d]),
        "or_cost_log_dense": (d, [i64, p, p, d, d]),
        "or_marginal_err_fs1": (d, [i64, p, p, p, d, d]),
        "or_cost_fs1": (d, [i64, p, p, d, d]),
        "or_marginal_err_fs1_log": (d, [i64, p, p, p, d, d]),
        "or_cost_fs1_log": (d, [i64, p, p, d, d]),
        "or_sinkhorn_dense": (ctypes.c_int, [i64, p, p, d, d, d, i64, p, p, p]),
        "or_sinkhorn_log_dense": (ctypes.c_int, [i64, p, p, d, d, d, i64, p, p, p]),
        "or_fs1": (ctypes.c_int, [i64, p, p, d, d, d, i64, p, p, p]),
        "or_fs1_log": (ctypes.c_int, [i64, p, p, d, d, d, i64, p, p, p]),
        "or_num_threads": (ctypes.c_int, []),
        "or_set_num_threads": (None, [ctypes.c_int]),
        "or_fs1_absorb": (ctypes.c_int, [i64, p, p, d, d, d, i64, d, p, p, p, p, p]),
        "or_kv2_dense": (ctypes.c_int, [i64, i64, p, d, d, d, p]),
        "or_kv2_fs1": (ctypes.c_int, [i64, i64, p, d, d, d, p]),
        "or_marginal_err2_dense": (d, [i64, i64, p, p, p, d, d, d]),
        "or_marginal_err2_fs1": (d, [i64, i64, p, p, p, d, d, d]),
        "or_cost2_dense": (d, [i64, i64, p, p, d, d, d]),
        "or_cost2_fs1": (d, [i64, i64, p, p, d, d, d]),
        "or_sinkhorn2_dense": (ctypes.c_int, [i64, i64, p, p, d, d, d, d, i64, p, p, p]),
        "or_fs1_2d": (ctypes.c_int, [i64, i64, p, p, d, d, d, d, i64, p, p, p]),
        "or_kv2_log_dense": (ctypes.c_int, [i64, i64, p, d, d, d, p]),
        "or_kv2_fs1_log": (ctypes.c_int, [i64, i64, p, d, d, d, p]),
        "or_marginal_err2_log_dense": (d, [i64, i64, p, p, p, d, d, d]),
        "or_marginal_err2_fs1_log": (d, [i64, i64, p, p, p, d, d, d]),
        "or_cost2_log_dense": (d, [i64, i64, p, p, d, d, d]),
        "or_cost2_fs1_log": (d, [i64, i64, p, p, d, d, d]),
        "or_sinkhorn2_log_dense": (ctypes.c_int, [i64, i64, p, p, d, d, d, d, i64, p, p, p]),
        "or_fs1_2d_log": (ctypes.c_int, [i64, i64, p, p, d, d, d, d, i64, p, p, p]),
        "or_kvn_dense": (ctypes.c_int, [ctypes.c_int, p, p, p, d, p]),
        "or_kvn_fs1": (ctypes.c_int, [ctypes.c_int, p, p, p, d, p]),
        "or_kvn_log_dense": (ctypes.c_int, [ctypes.c_int, p, p, p, d, p]),
        "or_kvn_fs1_log": (ctypes.c_int, [ctypes.c_int, p, p, p, d, p]),
        "or_marginal_errn_dense": (d, [ctypes.c_int, p, p, p, p, p, d]),
        "or_marginal_errn_fs1": (d, [ctypes.c_int, p, p, p, p, p, d]),
        "or_marginal_errn_log_dense": (d, [ctypes.c_int, p, p, p, p, p, d]),
        "or_marginal_errn_fs1_log": (d, [ctypes.c_int, p, p, p, p, p, d]),
        "or_costn_dense": (d, [ctypes.c_int, p, p, p, p, d]),
        "or_costn_fs1": (d, [ctypes.c_int, p, p, p, p, d]),
        "or_costn_log_dense": (d, [ctypes.c_int, p, p, p, p, d]),
        "or_costn_fs1_log": (d, [ctypes.c_int, p, p, p, p, d]),
        "or_sinkhornn_dense": (ctypes.c_int, [ctypes.c_int, p, p, p, p, d, d, i64, p, p, p]),
        "or_fs1_nd": (ctypes.c_int, [ctypes.c_int, p, p, p, p, d, d, i64, p, p, p]),
        "or_sinkhornn_log_dense": (ctypes.c_int, [ctypes.c_int, p, p, p, p, d, d, i64, p, p, p]),
        "or_fs1_nd_log": (ctypes.c_int, [ctypes.c_int, p, p, p, p, d, d, i64, p, p, p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_num_threads(k: int) -> None:
    """Thread count of the OpenMP loops of the dense routines."""
    _load().or_set_num_threads(int(k))


# --------------------------------------------------------------------------
# kernel application
# --------------------------------------------------------------------------

def kv_dense(x, h: float, eps: float, rows=None) -> np.ndarray:
    """(K x)_i for all i (or the listed rows), K_ij = exp(-|i-j| h/eps)."""
    x = _f64(x)
    n = x.size
    lib = _load()
    if rows is None:
        y = np.empty(n)
        st = lib.or_kv_dense(n, _ptr(x), h, eps, _ptr(y))
    else:
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        y = np.empty(r.size)
        st = lib.or_kv_dense_rows(n, _ptr(x), h, eps, _ptr(r), r.size, _ptr(y))
    if st != 0:
        raise ValueError(f"or_kv_dense: status {st}")
    return y


def kv_log_dense(lx, h: float, eps: float, rows=None) -> np.ndarray:
    """ln (K e^{lx})_i, max-shifted; -inf entries allowed."""
    lx = _f64(lx)
    n = lx.size
    lib = _load()
    if rows is None:
        y = np.empty(n)
        st = lib.or_kv_log_dense(n, _ptr(lx), h, eps, _ptr(y))
    else:
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        y = np.empty(r.size)
        st = lib.or_kv_log_dense_rows(n, _ptr(lx), h, eps, _ptr(r), r.size, _ptr(y))
    if st != 0:
        raise ValueError(f"or_kv_log_dense: status {st}")
    return y


def kv_fs1(x, h: float, eps: float) -> np.ndarray:
    x = _f64(x)
    y = np.empty(x.size)
    st = _load().or_kv_fs1(x.size, _ptr(x), h, eps, _ptr(y))
    if st != 0:
        raise ValueError(f"or_kv_fs1: status {st}")
    return y


def kv_fs1_log(lx, h: float, eps: float) -> np.ndarray:
    lx = _f64(lx)
    y = np.empty(lx.size)
    st = _load().or_kv_fs1_log(lx.size, _ptr(lx), h, eps, _ptr(y))
    if st != 0:
        raise ValueError(f"or_kv_fs1_log: status {st}")
    return y


# --------------------------------------------------------------------------
# the two double sums of Algorithm 1
# --------------------------------------------------------------------------

def marginal_err_dense(phi, psi, nu, h, eps) -> float:
    phi, psi, nu = _f64(phi), _f64(psi), _f64(nu)
    return float(_load().or_marginal_err_dense(phi.size, _ptr(phi), _ptr(psi), _ptr(nu), h, eps))


def cost_dense(phi, psi, h, eps) -> float:
    phi, psi = _f64(phi), _f64(psi)
    return float(_load().or_cost_dense(phi.size, _ptr(phi), _ptr(psi), h, eps))


def marginal_err_log_dense(F, G, nu, h, eps) -> float:
    F, G, nu = _f64(F), _f64(G), _f64(nu)
    return float(_load().or_marginal_err_log_dense(F.size, _ptr(F), _ptr(G), _ptr(nu), h, eps))


def cost_log_dense(F, G, h, eps) -> float:
    F, G = _f64(F), _f64(G)
    return float(_load().or_cost_log_dense(F.size, _ptr(F), _ptr(G), h, eps))


def marginal_err_fs1(phi, psi, nu, h, eps) -> float:
    phi, psi, nu = _f64(phi), _f64(psi), _f64(nu)
    return float(_load().or_marginal_err_fs1(phi.size, _ptr(phi), _ptr(psi), _ptr(nu), h, eps))


def cost_fs1(phi, psi, h, eps) -> float:
    phi, psi = _f64(phi), _f64(psi)
    return float(_load().or_cost_fs1(phi.size, _ptr(phi), _ptr(psi), h, eps))


def marginal_err_fs1_log(F, G, nu, h, eps) -> float:
    F, G, nu = _f64(F), _f64(G), _f64(nu)
    return float(_load().or_marginal_err_fs1_log(F.size, _ptr(F), _ptr(G), _ptr(nu), h, eps))


def cost_fs1_log(F, G, h, eps) -> float:
    F, G = _f64(F), _f64(G)
    return float(_load().or_cost_fs1_log(F.size, _ptr(F), _ptr(G), h, eps))


# --------------------------------------------------------------------------
# solvers
# --------------------------------------------------------------------------

@dataclass
class OracleResult:
    w1: float            # the value Algorithm 1 returns: sum phi_i psi_j K_ij |i-j| h
    marginal_err: float  # final nu-side L1 marginal error
    iterations: int      # completed (psi, phi) pairs
    status: int          # 0 ok, -2 non-finite scaling (abnormal termination)
    converged: bool      # stopping test met (err <= tol)
    a: np.ndarray        # phi (linear solvers) or F = ln phi (log solvers)
    b: np.ndarray        # psi (linear solvers) or G = ln psi (log solvers)


def _solve(fname, mu, nu, h, eps, tol, itr_max) -> OracleResult:
    mu, nu = _f64(mu), _f64(nu)
    n = mu.size
    if nu.size != n:
        raise ValueError("mu and nu must have the same length")
    a = np.empty(n)
    b = np.empty(n)
    res = np.zeros(5)
    st = getattr(_load(), fname)(n, _ptr(mu), _ptr(nu), h, eps, tol, int(itr_max),
                                 _ptr(a), _ptr(b), _ptr(res))
    if st == -1:
        raise ValueError(f"{fname}: invalid argument")
    if st == -4:
        raise MemoryError(fname)
    return OracleResult(float(res[0]), float(res[1]), int(res[2]), int(res[3]),
                        bool(res[4]), a, b)


def sinkhorn_dense(mu, nu, h, eps, tol=0.0, itr_max=1000) -> OracleResult:
    return _solve("or_sinkhorn_dense", mu, nu, h, eps, tol, itr_max)


def sinkhorn_log_dense(mu, nu, h, eps, tol=0.0, itr_max=1000) -> OracleResult:
    return _solve("or_sinkhorn_log_dense", mu, nu, h, eps, tol, itr_max)


def fs1(mu, nu, h, eps, tol=0.0, itr_max=1000) -> OracleResult:
    return _solve("or_fs1", mu, nu, h, eps, tol, itr_max)


def fs1_log(mu, nu, h, eps, tol=0.0, itr_max=1000) -> OracleResult:
    return _solve("or_fs1_log", mu, nu, h, eps, tol, itr_max)


@dataclass
class AbsorbResult:
    w1: float
    marginal_err: float
    iterations: int
    status: int
    converged: bool
    absorptions: int     # how many times the tau test fired
    phit: np.ndarray     # scaled vectors and absorbed potentials:
    psit: np.ndarray     #   phi = e^{alpha/eps} phit, psi = e^{beta/eps} psit
    alpha: np.ndarray
    beta: np.ndarray

    @property
    def F(self) -> np.ndarray:
        """ln phi = alpha/eps + ln phit."""
        with np.errstate(divide="ignore"):
            return self.alpha / self._eps + np.log(self.phit)

    @property
    def G(self) -> np.ndarray:
        with np.errstate(divide="ignore"):
            return self.beta / self._eps + np.log(self.psit)


def fs1_absorb(mu, nu, h, eps, tol=0.0, itr_max=1000, tau=1e3) -> AbsorbResult:
    """Stabilised FS-1 (Sec. 2 and Sec. 3 remarks): absorbed potentials alpha,
    beta and scaled vectors, absorption whenever max(phit) or max(psit) > tau,
    the products with the rescaled kernel by the recursions with per-element
    coefficients that replace the recursions of the two kernel products of
    Algorithm 1."""
    mu, nu = _f64(mu), _f64(nu)
    n = mu.size
    phit, psit, alpha, beta = (np.empty(n) for _ in range(4))
    res = np.zeros(6)
    st = _load().or_fs1_absorb(n, _ptr(mu), _ptr(nu), h, eps, tol, int(itr_max), tau,
                               _ptr(phit), _ptr(psit), _ptr(alpha), _ptr(beta), _ptr(res))
    if st == -1:
        raise ValueError("or_fs1_absorb: invalid argument")
    if st == -4:
        raise MemoryError("or_fs1_absorb")
    r = AbsorbResult(float(res[0]), float(res[1]), int(res[2]), int(res[3]), bool(res[4]),
                     int(res[5]), phit, psit, alpha, beta)
    r._eps = eps
    return r


def plan_linear(phi, psi, h, eps) -> np.ndarray:
    """P_ij = phi_i exp(-|i-j| h/eps) psi_j (the scaling form of Sec. 2)."""
    phi, psi = _f64(phi), _f64(psi)
    n = phi.size
    d = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :]).astype(np.float64)
    return phi[:, None] * np.exp(-d * (h / eps)) * psi[None, :]


def plan_log(F, G, h, eps) -> np.ndarray:
    """P_ij = exp(F_i + G_j - |i-j| h/eps)."""
    F, G = _f64(F), _f64(G)
    n = F.size
    d = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :]).astype(np.float64)
    with np.errstate(invalid="ignore"):
        t = F[:, None] + G[None, :] - d * (h / eps)
    t = np.where(np.isnan(t), -np.inf, t)
    return np.exp(t)


# --------------------------------------------------------------------------
# two dimensions (Sec. 4, Algorithm 2); arrays are n1 x n2 in column-major
# order, flattened: entry (i, j) at i + n1 j
# --------------------------------------------------------------------------

def _grid2(x, n1, n2) -> np.ndarray:
    x = _f64(x).reshape(-1)
    if x.size != n1 * n2:
        raise ValueError("array size must be n1 * n2")
    return x


def kv2_dense(x, n1: int, n2: int, h1: float, h2: float, eps: float) -> np.ndarray:
    x = _grid2(x, n1, n2)
    y = np.empty_like(x)
    _load().or_kv2_dense(n1, n2, _ptr(x), h1, h2, eps, _ptr(y))
    return y


def kv2_fs1(x, n1: int, n2: int, h1: float, h2: float, eps: float) -> np.ndarray:
    x = _grid2(x, n1, n2)
    y = np.empty_like(x)
    _load().or_kv2_fs1(n1, n2, _ptr(x), h1, h2, eps, _ptr(y))
    return y


def marginal_err2_dense(phi, psi, nu, n1, n2, h1, h2, eps) -> float:
    phi, psi, nu = _grid2(phi, n1, n2), _grid2(psi, n1, n2), _grid2(nu, n1, n2)
    return float(_load().or_marginal_err2_dense(n1, n2, _ptr(phi), _ptr(psi), _ptr(nu),
                                                h1, h2, eps))


def marginal_err2_fs1(phi, psi, nu, n1, n2, h1, h2, eps) -> float:
    phi, psi, nu = _grid2(phi, n1, n2), _grid2(psi, n1, n2), _grid2(nu, n1, n2)
    return float(_load().or_marginal_err2_fs1(n1, n2, _ptr(phi), _ptr(psi), _ptr(nu),
                                              h1, h2, eps))


def cost2_dense(phi, psi, n1, n2, h1, h2, eps) -> float:
    phi, psi = _grid2(phi, n1, n2), _grid2(psi, n1, n2)
    return float(_load().or_cost2_dense(n1, n2, _ptr(phi), _ptr(psi), h1, h2, eps))


def cost2_fs1(phi, psi, n1, n2, h1, h2, eps) -> float:
    phi, psi = _grid2(phi, n1, n2), _grid2(psi, n1, n2)
    return float(_load().or_cost2_fs1(n1, n2, _ptr(phi), _ptr(psi), h1, h2, eps))


def _solve2(fname, mu, nu, n1, n2, h1, h2, eps, tol, itr_max) -> OracleResult:
    mu, nu = _grid2(mu, n1, n2), _grid2(nu, n1, n2)
    a = np.empty(n1 * n2)
    b = np.empty(n1 * n2)
    res = np.zeros(5)
    st = getattr(_load(), fname)(n1, n2, _ptr(mu), _ptr(nu), h1, h2, eps, tol, int(itr_max),
                                 _ptr(a), _ptr(b), _ptr(res))
    if st == -1:
        raise ValueError(f"{fname}: invalid argument")
    if st == -4:
        raise MemoryError(fname)
    return OracleResult(float(res[0]), float(res[1]), int(res[2]), int(res[3]),
                        bool(res[4]), a, b)


def sinkhorn2_dense(mu, nu, n1, n2, h1, h2, eps, tol=0.0, itr_max=1000) -> OracleResult:
    return _solve2("or_sinkhorn2_dense", mu, nu, n1, n2, h1, h2, eps, tol, itr_max)


def fs1_2d(mu, nu, n1, n2, h1, h2, eps, tol=0.0, itr_max=1000) -> OracleResult:
    return _solve2("or_fs1_2d", mu, nu, n1, n2, h1, h2, eps, tol, itr_max)


def kv2_log_dense(lx, n1: int, n2: int, h1: float, h2: float, eps: float) -> np.ndarray:
    """ln K e^lx on the 2-D grid, every term of the sum (max-shifted)."""
    lx = _grid2(lx, n1, n2)
    y = np.empty_like(lx)
    _load().or_kv2_log_dense(n1, n2, _ptr(lx), h1, h2, eps, _ptr(y))
    return y


def kv2_fs1_log(lx, n1: int, n2: int, h1: float, h2: float, eps: float) -> np.ndarray:
    """ln K e^lx by the 1-D log recursions along the columns, then the rows."""
    lx = _grid2(lx, n1, n2)
    y = np.empty_like(lx)
    _load().or_kv2_fs1_log(n1, n2, _ptr(lx), h1, h2, eps, _ptr(y))
    return y


def marginal_err2_log_dense(F, G, nu, n1, n2, h1, h2, eps) -> float:
    F, G, nu = _grid2(F, n1, n2), _grid2(G, n1, n2), _grid2(nu, n1, n2)
    return float(_load().or_marginal_err2_log_dense(n1, n2, _ptr(F), _ptr(G), _ptr(nu),
                                                    h1, h2, eps))


def marginal_err2_fs1_log(F, G, nu, n1, n2, h1, h2, eps) -> float:
    F, G, nu = _grid2(F, n1, n2), _grid2(G, n1, n2), _grid2(nu, n1, n2)
    return float(_load().or_marginal_err2_fs1_log(n1, n2, _ptr(F), _ptr(G), _ptr(nu),
                                                  h1, h2, eps))


def cost2_log_dense(F, G, n1, n2, h1, h2, eps) -> float:
    F, G = _grid2(F, n1, n2), _grid2(G, n1, n2)
    return float(_load().or_cost2_log_dense(n1, n2, _ptr(F), _ptr(G), h1, h2, eps))


def cost2_fs1_log(F, G, n1, n2, h1, h2, eps) -> float:
    F, G = _grid2(F, n1, n2), _grid2(G, n1, n2)
    return float(_load().or_cost2_fs1_log(n1, n2, _ptr(F), _ptr(G), h1, h2, eps))


def sinkhorn2_log_dense(mu, nu, n1, n2, h1, h2, eps, tol=0.0, itr_max=1000) -> OracleResult:
    """Algorithm 2 on logarithms with dense products; .a = F = ln phi, .b = G = ln psi."""
    return _solve2("or_sinkhorn2_log_dense", mu, nu, n1, n2, h1, h2, eps, tol, itr_max)


def fs1_2d_log(mu, nu, n1, n2, h1, h2, eps, tol=0.0, itr_max=1000) -> OracleResult:
    """Algorithm 2 on logarithms by the recursions; .a = F = ln phi, .b = G = ln psi."""
    return _solve2("or_fs1_2d_log", mu, nu, n1, n2, h1, h2, eps, tol, itr_max)


def plan2(phi, psi, n1, n2, h1, h2, eps) -> np.ndarray:
    """P_{(i,j),(k,l)} = phi_(i,j) exp(-(|i-k| h1 + |j-l| h2)/eps) psi_(k,l), as an
    (n1 n2) x (n1 n2) matrix over the column-major flattening."""
    phi, psi = _grid2(phi, n1, n2), _grid2(psi, n1, n2)
    r = np.arange(n1 * n2)
    i, j = r % n1, r // n1
    d = (np.abs(i[:, None] - i[None, :]) * h1 + np.abs(j[:, None] - j[None, :]) * h2)
    return phi[:, None] * np.exp(-d / eps) * psi[None, :]


# ---------------------------------------------------------------------------
# D dimensions (Sec. 4 carried to any number of axes): grids n_0 x ... x
# n_{D-1} with the first axis fastest, spacings h_a, the L1 ground cost.
# ---------------------------------------------------------------------------

def _gridn(x, dims):
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    if x.size != int(np.prod(dims)):
        raise ValueError("array size must be the product of dims")
    return x


def _dimsh(dims, h):
    dims = np.ascontiguousarray(dims, dtype=np.int64).reshape(-1)
    h = np.ascontiguousarray(h, dtype=np.float64).reshape(-1)
    if dims.size != h.size or dims.size < 1:
        raise ValueError("dims and h must have the same length >= 1")
    return dims, h


def _kvn(fname, x, dims, h, eps):
    dims, h = _dimsh(dims, h)
    x = _gridn(x, dims)
    y = np.empty_like(x)
    st = getattr(_load(), fname)(int(dims.size), _ptr(dims), _ptr(x), _ptr(h), eps, _ptr(y))
    if st != 0:
        raise ValueError(f"{fname}: status {st}")
    return y


def kvn_dense(x, dims, h, eps: float) -> np.ndarray:
    """K x on the D-dimensional grid, K formed entry by entry."""
    return _kvn("or_kvn_dense", x, dims, h, eps)


def kvn_fs1(x, dims, h, eps: float) -> np.ndarray:
    """K x by the 1-D recursions along axis 0, then 1, ..."""
    return _kvn("or_kvn_fs1", x, dims, h, eps)


def kvn_log_dense(lx, dims, h, eps: float) -> np.ndarray:
    """ln K e^lx, every term (max-shifted)."""
    return _kvn("or_kvn_log_dense", lx, dims, h, eps)


def kvn_fs1_log(lx, dims, h, eps: float) -> np.ndarray:
    """ln K e^lx by the 1-D log recursions along each axis in turn."""
    return _kvn("or_kvn_fs1_log", lx, dims, h, eps)


def _errn(fname, a, b, nu, dims, h, eps) -> float:
    dims, h = _dimsh(dims, h)
    a, b, nu = _gridn(a, dims), _gridn(b, dims), _gridn(nu, dims)
    return float(getattr(_load(), fname)(int(dims.size), _ptr(dims), _ptr(a), _ptr(b), _ptr(nu),
                                          _ptr(h), eps))


def marginal_errn_dense(phi, psi, nu, dims, h, eps) -> float:
    return _errn("or_marginal_errn_dense", phi, psi, nu, dims, h, eps)


def marginal_errn_fs1(phi, psi, nu, dims, h, eps) -> float:
    return _errn("or_marginal_errn_fs1", phi, psi, nu, dims, h, eps)


def marginal_errn_log_dense(F, G, nu, dims, h, eps) -> float:
    return _errn("or_marginal_errn_log_dense", F, G, nu, dims, h, eps)


def marginal_errn_fs1_log(F, G, nu, dims, h, eps) -> float:
    return _errn("or_marginal_errn_fs1_log", F, G, nu, dims, h, eps)


def _costn(fname, a, b, dims, h, eps) -> float:
    dims, h = _dimsh(dims, h)
    a, b = _gridn(a, dims), _gridn(b, dims)
    return float(getattr(_load(), fname)(int(dims.size), _ptr(dims), _ptr(a), _ptr(b), _ptr(h),
                                          eps))


def costn_dense(phi, psi, dims, h, eps) -> float:
    return _costn("or_costn_dense", phi, psi, dims, h, eps)


def costn_fs1(phi, psi, dims, h, eps) -> float:
    return _costn("or_costn_fs1", phi, psi, dims, h, eps)


def costn_log_dense(F, G, dims, h, eps) -> float:
    return _costn("or_costn_log_dense", F, G, dims, h, eps)


def costn_fs1_log(F, G, dims, h, eps) -> float:
    return _costn("or_costn_fs1_log", F, G, dims, h, eps)


def _solven(fname, mu, nu, dims, h, eps, tol, itr_max) -> OracleResult:
    dims, h = _dimsh(dims, h)
    mu, nu = _gridn(mu, dims), _gridn(nu, dims)
    n = mu.size
    a = np.empty(n)
    b = np.empty(n)
    res = np.zeros(5)
    st = getattr(_load(), fname)(int(dims.size), _ptr(dims), _ptr(mu), _ptr(nu), _ptr(h), eps,
                                 tol, int(itr_max), _ptr(a), _ptr(b), _ptr(res))
    if st == -1:
        raise ValueError(f"{fname}: invalid argument")
    if st == -4:
        raise MemoryError(fname)
    return OracleResult(float(res[0]), float(res[1]), int(res[2]), int(res[3]),
                        bool(res[4]), a, b)


def sinkhornn_dense(mu, nu, dims, h, eps, tol=0.0, itr_max=1000) -> OracleResult:
    """Algorithm 2 on D axes with dense products."""
    return _solven("or_sinkhornn_dense", mu, nu, dims, h, eps, tol, itr_max)


def fs1_nd(mu, nu, dims, h, eps, tol=0.0, itr_max=1000) -> OracleResult:
    """Algorithm 2 on D axes by the recursions along each axis."""
    return _solven("or_fs1_nd", mu, nu, dims, h, eps, tol, itr_max)


def sinkhornn_log_dense(mu, nu, dims, h, eps, tol=0.0, itr_max=1000) -> OracleResult:
    """The log form with dense products; .a = F = ln phi, .b = G = ln psi."""
    return _solven("or_sinkhornn_log_dense", mu, nu, dims, h, eps, tol, itr_max)


def fs1_nd_log(mu, nu, dims, h, eps, tol=0.0, itr_max=1000) -> OracleResult:
    """The log form by the recursions; .a = F = ln phi, .b = G = ln psi."""
    return _solven("or_fs1_nd_log", mu, nu, dims, h, eps, tol, itr_max)

