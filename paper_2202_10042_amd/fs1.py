"""Thin ctypes binding of libfs1 (include/fs1.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libfs1.so.  Torch tensors supply device memory and the stream.  There
is no CPU fallback: if the library or a GPU is missing, calls raise.

The functions keep the C names:
  fs1_kv_apply(x, h, eps)            -> K x
  fs1_kv_apply_log(lx, h, eps)       -> ln K e^lx
  fs1_solve(mu, nu, eps, tol, ...)   -> Result (Algorithm 1, FS-1)
  fs1_solve_batched(mu, nu, offsets, eps, tol, ...) -> list[Result]
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfs1.so")

FS1_OK = 0
FS1_ERR_INVALID_ARG = -1
FS1_ERR_NONFINITE = -2
FS1_ERR_HIP = -3
FS1_ERR_NO_MEMORY = -4
FS1_ERR_INTERNAL = -5

FS1_F64 = 0
FS1_F32 = 1
FS1_PLAIN = 0
FS1_LOG = 1
FS1_ABSORB = 2
FS1_FLAG_POTENTIALS = 1
FS1_FLAG_GENERAL = 2
FS1_FLAG_PERSISTENT = 4
FS1_FLAG_NO_GRAPH = 8
FS1_FLAG_NO_RESIDENT = 16
FS1_FLAG_DEVICE_PARAMS = 32
FS1_FLAG_SERVER_OVERLAP = 64

# every symbol include/fs1.h declares
EXPORTS = (
    "fs1_ctx_create", "fs1_ctx_destroy", "fs1_ctx_set_stream", "fs1_ctx_set_profiling",
    "fs1_ctx_kernel_stats", "fs1_last_error", "fs1_version", "fs1_kv_apply",
    "fs1_kv_apply_log", "fs1_opts_default", "fs1_solve", "fs1_solve_batched",
    "fs1_server_opts_default", "fs1_server_create", "fs1_server_destroy", "fs1_server_submit",
    "fs1_server_step", "fs1_server_poll", "fs1_server_get_info", "fs1_kv_apply_2d",
    "fs1_solve_2d", "fs1_stream_copy", "fs1_solve_noalloc", "fs1_ctx_create_with_allocator",
    "fs1_solve_async", "fs1_solve_batched_config", "fs1_kv_apply_nd", "fs1_solve_nd",
)

# fs1_alloc_fn / fs1_free_fn
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Fs1Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libfs1 status {status}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [
        ("h", ctypes.c_double),
        ("itr_max", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("domain", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("sync_every", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("potentials_out", ctypes.c_void_p),
        ("err_history", ctypes.c_void_p),
        ("tau", ctypes.c_double),
        ("warm_m", ctypes.c_void_p),
        ("warm_e", ctypes.c_void_p),
        ("state_m", ctypes.c_void_p),
        ("state_e", ctypes.c_void_p),
    ]


class CResult(ctypes.Structure):
    _fields_ = [
        ("w1", ctypes.c_double),
        ("marginal_err", ctypes.c_double),
        ("mu_err", ctypes.c_double),
        ("iterations", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("absorptions", ctypes.c_int32),
    ]


class ServerOpts(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_int64),
        ("max_active", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("itr_max", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("iters_per_step", ctypes.c_int32),
        ("flags", ctypes.c_int32),
    ]


class Completion(ctypes.Structure):
    _fields_ = [
        ("ticket", ctypes.c_int64),
        ("result", CResult),
        ("admitted_step", ctypes.c_int64),
        ("completed_step", ctypes.c_int64),
    ]


class ServerInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("queued", "active", "completed", "steps",
                                              "bytes_in_use", "bytes_total")]


@dataclass
class Result:
    w1: float
    marginal_err: float
    mu_err: float
    iterations: int
    converged: bool
    status: int
    F: Optional[object] = None        # torch tensor ln(phi) when requested
    G: Optional[object] = None        # torch tensor ln(psi) when requested
    err_history: Optional[object] = None
    absorptions: int = 0              # domain "absorb": times the tau test fired
    state: Optional[tuple] = None     # (m, e): final phi, psi in split form when requested


_lib = None


def load(path: str = LIB_PATH):
    """Load libfs1.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libfs1.so not found at {path}; build it with "
                           "`python -m paper_2202_10042_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64, d, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int32
    lib.fs1_ctx_create.argtypes = [vp, ctypes.POINTER(vp)]
    lib.fs1_ctx_create.restype = ctypes.c_int
    lib.fs1_ctx_create_with_allocator.argtypes = [vp, ALLOC_FN, FREE_FN, vp, ctypes.POINTER(vp)]
    lib.fs1_ctx_create_with_allocator.restype = ctypes.c_int
    lib.fs1_ctx_destroy.argtypes = [vp]
    lib.fs1_ctx_destroy.restype = ctypes.c_int
    lib.fs1_ctx_set_stream.argtypes = [vp, vp]
    lib.fs1_ctx_set_stream.restype = ctypes.c_int
    lib.fs1_ctx_set_profiling.argtypes = [vp, ctypes.c_int]
    lib.fs1_ctx_set_profiling.restype = ctypes.c_int
    lib.fs1_ctx_kernel_stats.argtypes = [vp, ctypes.POINTER(d), ctypes.POINTER(i64),
                                         ctypes.POINTER(d)]
    lib.fs1_ctx_kernel_stats.restype = ctypes.c_int
    lib.fs1_last_error.argtypes = []
    lib.fs1_last_error.restype = ctypes.c_char_p
    lib.fs1_version.argtypes = []
    lib.fs1_version.restype = ctypes.c_char_p
    lib.fs1_kv_apply.argtypes = [vp, vp, vp, i64, d, d, ctypes.c_int]
    lib.fs1_kv_apply.restype = ctypes.c_int
    lib.fs1_kv_apply_log.argtypes = [vp, vp, vp, i64, d, d, ctypes.c_int]
    lib.fs1_kv_apply_log.restype = ctypes.c_int
    lib.fs1_opts_default.argtypes = [ctypes.POINTER(Opts)]
    lib.fs1_opts_default.restype = ctypes.c_int
    lib.fs1_solve.argtypes = [vp, vp, vp, i64, d, d, ctypes.POINTER(Opts), ctypes.POINTER(CResult)]
    lib.fs1_solve.restype = ctypes.c_int
    # eps and tol: host arrays, or device memory with FS1_FLAG_DEVICE_PARAMS
    lib.fs1_solve_batched.argtypes = [vp, vp, vp, ctypes.POINTER(i64), i32, vp, vp,
                                      ctypes.POINTER(Opts), ctypes.POINTER(CResult)]
    lib.fs1_solve_batched.restype = ctypes.c_int
    lib.fs1_server_opts_default.argtypes = [ctypes.POINTER(ServerOpts)]
    lib.fs1_server_opts_default.restype = ctypes.c_int
    lib.fs1_server_create.argtypes = [vp, ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
    lib.fs1_server_create.restype = ctypes.c_int
    lib.fs1_server_destroy.argtypes = [vp]
    lib.fs1_server_destroy.restype = ctypes.c_int
    lib.fs1_server_submit.argtypes = [vp, vp, vp, i64, d, d, ctypes.POINTER(i64)]
    lib.fs1_server_submit.restype = ctypes.c_int
    lib.fs1_server_step.argtypes = [vp, ctypes.POINTER(i32)]
    lib.fs1_server_step.restype = ctypes.c_int
    lib.fs1_server_poll.argtypes = [vp, ctypes.POINTER(Completion), i32, ctypes.POINTER(i32)]
    lib.fs1_server_poll.restype = ctypes.c_int
    lib.fs1_server_get_info.argtypes = [vp, ctypes.POINTER(ServerInfo)]
    lib.fs1_server_get_info.restype = ctypes.c_int
    lib.fs1_kv_apply_2d.argtypes = [vp, vp, vp, i64, i64, d, d, d, ctypes.c_int]
    lib.fs1_kv_apply_2d.restype = ctypes.c_int
    lib.fs1_solve_2d.argtypes = [vp, vp, vp, i64, i64, d, d, d, d, ctypes.POINTER(Opts),
                                 ctypes.POINTER(CResult)]
    lib.fs1_solve_2d.restype = ctypes.c_int
    lib.fs1_kv_apply_nd.argtypes = [vp, vp, vp, ctypes.c_int, vp, vp, d, ctypes.c_int]
    lib.fs1_kv_apply_nd.restype = ctypes.c_int
    lib.fs1_solve_nd.argtypes = [vp, vp, vp, ctypes.c_int, vp, vp, d, d, ctypes.POINTER(Opts),
                                 ctypes.POINTER(CResult)]
    lib.fs1_solve_nd.restype = ctypes.c_int
    lib.fs1_solve_batched_config.argtypes = [vp, vp, vp, ctypes.POINTER(i64), i32, vp, vp,
                                             ctypes.POINTER(Opts), ctypes.POINTER(i32),
                                             ctypes.POINTER(i32), ctypes.POINTER(CResult)]
    lib.fs1_solve_batched_config.restype = ctypes.c_int
    lib.fs1_solve_async.argtypes = lib.fs1_solve.argtypes
    lib.fs1_solve_async.restype = ctypes.c_int
    lib.fs1_solve_noalloc.argtypes = lib.fs1_solve.argtypes
    lib.fs1_solve_noalloc.restype = ctypes.c_int
    lib.fs1_stream_copy.argtypes = [vp, vp, vp, i64, ctypes.c_int]
    lib.fs1_stream_copy.restype = ctypes.c_int
    _lib = lib
    return lib


def last_error() -> str:
    return load().fs1_last_error().decode()


def _check(st: int):
    if st != FS1_OK:
        raise Fs1Error(st, last_error())


class Context:
    """A libfs1 context bound to a HIP stream (default: torch's current stream).

    allocator="torch": the context's device memory (solve workspace, server
    pools) comes from PyTorch's caching allocator through the library's
    allocator callbacks, on the context's current stream."""

    def __init__(self, stream=None, allocator: Optional[str] = None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libfs1 needs a ROCm GPU; none is visible")
        lib = load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream_obj = stream
        h = ctypes.c_void_p()
        if allocator is None:
            _check(lib.fs1_ctx_create(ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        elif allocator == "torch":
            device = torch.cuda.current_device()

            def _alloc(nbytes, _user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), device,
                                                              self._stream_obj)
                except RuntimeError:
                    return None

            def _free(ptr, _user):
                torch.cuda.caching_allocator_delete(ptr)

            self._callbacks = (ALLOC_FN(_alloc), FREE_FN(_free))  # kept alive with the context
            _check(lib.fs1_ctx_create_with_allocator(ctypes.c_void_p(stream.cuda_stream),
                                                     self._callbacks[0], self._callbacks[1],
                                                     None, ctypes.byref(h)))
        else:
            raise ValueError(f"unknown allocator {allocator!r}")
        self.handle = h

    def set_stream(self, stream):
        self._stream_obj = stream
        _check(load().fs1_ctx_set_stream(self.handle, ctypes.c_void_p(stream.cuda_stream)))

    def set_profiling(self, stride: int):
        """Time the half-iteration kernels of every `stride`-th iteration (0: off)."""
        _check(load().fs1_ctx_set_profiling(self.handle, int(stride)))

    def kernel_stats(self):
        """(total ms, launches, algorithmic bytes) of timed half-iteration kernels."""
        ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _check(load().fs1_ctx_kernel_stats(self.handle, ctypes.byref(ms), ctypes.byref(n),
                                           ctypes.byref(b)))
        return ms.value, n.value, b.value

    def close(self):
        if getattr(self, "handle", None):
            load().fs1_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx: Optional[Context] = None


def default_context() -> Context:
    global _default_ctx
    import torch
    if _default_ctx is None:
        _default_ctx = Context()
    _default_ctx.set_stream(torch.cuda.current_stream())
    return _default_ctx


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return FS1_F64
    if t.dtype == torch.float32:
        return FS1_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def fs1_kv_apply(x, h: float, eps: float, out=None, ctx: Optional[Context] = None):
    """y = K x, K_ij = exp(-|i-j| h/eps)  (float64 or float32 tensor)."""
    import torch
    ctx = ctx or default_context()
    if out is None:
        out = torch.empty_like(x)
    _check(load().fs1_kv_apply(ctx.handle, _dev(x, "x"), _dev(out, "out"), x.numel(),
                               float(h), float(eps), _dtype_code(x)))
    return out


def fs1_kv_apply_log(lx, h: float, eps: float, out=None, ctx: Optional[Context] = None):
    """ly = ln K e^lx (log-sum-exp semiring)."""
    import torch
    ctx = ctx or default_context()
    if out is None:
        out = torch.empty_like(lx)
    _check(load().fs1_kv_apply_log(ctx.handle, _dev(lx, "lx"), _dev(out, "out"), lx.numel(),
                                   float(h), float(eps), _dtype_code(lx)))
    return out


def fs1_stream_copy(src, dst, nontemporal: bool = False, ctx: Optional[Context] = None):
    """Diagnostic device copy of src into dst (same number of bytes), the
    attainable-bandwidth reference of the benchmark."""
    ctx = ctx or default_context()
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("src and dst must have the same size in bytes")
    _check(load().fs1_stream_copy(ctx.handle, _dev(src, "src"), _dev(dst, "dst"), nb,
                                  1 if nontemporal else 0))
    return dst


def make_opts(h: Optional[float] = None, itr_max: int = 10000, dtype: str = "f64",
              domain: str = "plain", check_every: int = 1, sync_every: int = 16) -> Opts:
    o = Opts()
    load().fs1_opts_default(ctypes.byref(o))
    o.h = float(h) if h else 0.0
    o.itr_max = int(itr_max)
    o.dtype = {"f64": FS1_F64, "f32": FS1_F32}[dtype]
    o.domain = {"plain": FS1_PLAIN, "log": FS1_LOG, "absorb": FS1_ABSORB}[domain]
    o.check_every = int(check_every)
    o.sync_every = int(sync_every)
    return o


def fs1_solve(mu, nu, eps: float, tol: float, h: Optional[float] = None, itr_max: int = 10000,
              dtype: str = "f64", domain: str = "plain", check_every: int = 1,
              sync_every: int = 16, potentials: bool = False, err_history: bool = False,
              solver: str = "auto", ctx: Optional[Context] = None,
              raise_on_error: bool = False, tau: float = 1e3, noalloc: bool = False,
              warm=None, state: bool = False) -> Result:
    """Algorithm 1 (FS-1) on device marginals mu, nu (float64 tensors).

    warm: (m, e) device tensors (float64 and int32, 2n entries each, phi then
    psi): start from phi_i = m[i] 2^e[i], psi_j = m[n+j] 2^e[n+j] instead of
    1/n.  state: return the final (phi, psi) in that split form as
    Result.state (a later solve warm-started from it continues bit for bit).

    noalloc: call fs1_solve_noalloc (the library's fixed 64 MiB workspace per
    GPU instead of the context's; the output tensors are still allocated here).

    domain: "plain" (Algorithm 1 as printed), "log" (stabilised, absorption
    at every half-iteration) or "absorb" (the stabilisation with threshold
    tau: one workgroup for n <= 1024 R, else the general path; no persistent
    solver).
    solver: "auto" (the whole solve in one workgroup and one launch when
    n <= 1024 R, else fused one-launch-per-half kernels when they apply),
    "fused" (as "auto" without the one-workgroup solver), "general"
    (extended-range scans with a separate carry kernel) or "persistent"
    (single cooperative launch when the grid fits)."""
    import torch
    ctx = ctx or default_context()
    n = mu.numel()
    if nu.numel() != n:
        raise ValueError("mu and nu must have the same length")
    o = make_opts(h, itr_max, dtype, domain, check_every, sync_every)
    o.tau = float(tau)
    o.flags |= {"auto": 0, "fused": FS1_FLAG_NO_RESIDENT, "general": FS1_FLAG_GENERAL,
                "persistent": FS1_FLAG_PERSISTENT}[solver]
    pot = hist = None
    if potentials:
        pot = torch.empty(2 * n, dtype=torch.float64, device=mu.device)
        o.flags |= FS1_FLAG_POTENTIALS
        o.potentials_out = pot.data_ptr()
    if err_history:
        hist = torch.empty(itr_max + 1, dtype=torch.float64, device=mu.device)
        o.err_history = hist.data_ptr()
    if warm is not None:
        wm, we = warm
        if wm.numel() != 2 * n or we.numel() != 2 * n or wm.dtype != torch.float64 or \
                we.dtype != torch.int32:
            raise ValueError("warm start: (float64, int32) tensors of 2n entries")
        o.warm_m = _dev(wm, "warm_m").value
        o.warm_e = _dev(we, "warm_e").value
    st_m = st_e = None
    if state:
        st_m = torch.empty(2 * n, dtype=torch.float64, device=mu.device)
        st_e = torch.empty(2 * n, dtype=torch.int32, device=mu.device)
        o.state_m = st_m.data_ptr()
        o.state_e = st_e.data_ptr()
    r = CResult()
    call = load().fs1_solve_noalloc if noalloc else load().fs1_solve
    st = call(ctx.handle, _dev(mu, "mu"), _dev(nu, "nu"), n, float(eps), float(tol),
              ctypes.byref(o), ctypes.byref(r))
    if st == FS1_ERR_INVALID_ARG or st == FS1_ERR_HIP or st == FS1_ERR_NO_MEMORY or (
            raise_on_error and st != FS1_OK):
        raise Fs1Error(st, last_error())
    res = Result(r.w1, r.marginal_err, r.mu_err, r.iterations, bool(r.converged), st)
    res.absorptions = int(r.absorptions)
    if pot is not None and st == FS1_OK:
        res.F, res.G = pot[:n], pot[n:]
    if hist is not None:
        res.err_history = hist
    if st_m is not None and st == FS1_OK:
        res.state = (st_m, st_e)
    return res


def fs1_solve_async(mu, nu, eps: float, tol: float, out=None, h: Optional[float] = None,
                    itr_max: int = 10000, dtype: str = "f64", domain: str = "log",
                    check_every: int = 1, solver: str = "auto", potentials_out=None,
                    err_history_out=None, ctx: Optional[Context] = None):
    """Enqueue Algorithm 1 on the context stream with no host synchronisation
    (fs1_solve_async; capturable in a graph).  out: a device uint8 tensor of
    at least RESULT_BYTES bytes that receives the fs1_result (allocated here
    when None); potentials_out / err_history_out: optional device float64
    tensors of 2n / itr_max + 1 entries.  Returns `out`; read_result(out)
    gives the Result once the stream has run."""
    import torch
    ctx = ctx or default_context()
    n = mu.numel()
    if nu.numel() != n:
        raise ValueError("mu and nu must have the same length")
    if out is None:
        out = torch.empty(RESULT_BYTES, dtype=torch.uint8, device=mu.device)
    elif out.numel() * out.element_size() < RESULT_BYTES:
        raise ValueError("out is too small for an fs1_result")
    o = make_opts(h, itr_max, dtype, domain, check_every, 16)
    o.flags |= {"auto": 0, "fused": FS1_FLAG_NO_RESIDENT, "general": FS1_FLAG_GENERAL}[solver]
    if potentials_out is not None:
        if potentials_out.numel() != 2 * n or potentials_out.dtype != torch.float64:
            raise ValueError("potentials_out: 2n float64 entries")
        o.flags |= FS1_FLAG_POTENTIALS
        o.potentials_out = _dev(potentials_out, "potentials_out").value
    if err_history_out is not None:
        if err_history_out.numel() < itr_max + 1 or err_history_out.dtype != torch.float64:
            raise ValueError("err_history_out: itr_max + 1 float64 entries")
        o.err_history = _dev(err_history_out, "err_history_out").value
    _check(load().fs1_solve_async(ctx.handle, _dev(mu, "mu"), _dev(nu, "nu"), n, float(eps),
                                  float(tol), ctypes.byref(o),
                                  ctypes.cast(ctypes.c_void_p(out.data_ptr()),
                                              ctypes.POINTER(CResult))))
    return out


RESULT_BYTES = ctypes.sizeof(CResult)


def read_result(out) -> Result:
    """The Result an fs1_solve_async call wrote to the device tensor `out`
    (copies it to the host: synchronises with the tensor's stream)."""
    raw = bytes(out[:RESULT_BYTES].cpu().numpy().tobytes())
    r = CResult.from_buffer_copy(raw)
    return Result(r.w1, r.marginal_err, r.mu_err, r.iterations, bool(r.converged), r.status)


def fs1_kv_apply_2d(x, n1: int, n2: int, h1: float, h2: float, eps: float, out=None,
                    ctx: Optional[Context] = None):
    """y = K x on an n1 x n2 grid (column-major flattening, entry (i, j) at
    i + n1 j), K = exp(-(|i-k| h1 + |j-l| h2)/eps)  (float64 or float32)."""
    import torch
    ctx = ctx or default_context()
    if x.numel() != n1 * n2:
        raise ValueError("x must hold n1 * n2 entries")
    if out is None:
        out = torch.empty_like(x)
    _check(load().fs1_kv_apply_2d(ctx.handle, _dev(x, "x"), _dev(out, "out"), int(n1), int(n2),
                                  float(h1), float(h2), float(eps), _dtype_code(x)))
    return out


def fs1_solve_2d(mu, nu, n1: int, n2: int, h1: float, h2: float, eps: float, tol: float,
                 itr_max: int = 10000, dtype: str = "f64", check_every: int = 1,
                 sync_every: int = 16, potentials: bool = False, err_history: bool = False,
                 solver: str = "auto", ctx: Optional[Context] = None,
                 raise_on_error: bool = False, domain: str = "plain") -> Result:
    """Algorithm 2 (2-D FS-1) on device float64 marginals of n1 * n2 entries
    (column-major).  domain: "plain" (Algorithm 2's arithmetic) or "log" (its
    stabilised form: scalings as mantissas with per-entry binary exponents).
    solver: "auto" (one workgroup for small grids: n1 n2 <= 4096, or up to
    8192 in the plain domain where the grid's three LDS arrays fit, and n1 + n2
    <= 384 in the plain domain, <= 80 (binary64) or 128 (binary32) in the log
    domain; else one launch per line pass) or "lines" (always the per-line
    launches)."""
    import torch
    ctx = ctx or default_context()
    n = n1 * n2
    if mu.numel() != n or nu.numel() != n:
        raise ValueError("mu and nu must hold n1 * n2 entries")
    o = make_opts(None, itr_max, dtype, domain, check_every, sync_every)
    o.flags |= {"auto": 0, "lines": FS1_FLAG_NO_RESIDENT}[solver]
    pot = hist = None
    if potentials:
        pot = torch.empty(2 * n, dtype=torch.float64, device=mu.device)
        o.flags |= FS1_FLAG_POTENTIALS
        o.potentials_out = pot.data_ptr()
    if err_history:
        hist = torch.empty(itr_max + 1, dtype=torch.float64, device=mu.device)
        o.err_history = hist.data_ptr()
    r = CResult()
    st = load().fs1_solve_2d(ctx.handle, _dev(mu, "mu"), _dev(nu, "nu"), int(n1), int(n2),
                             float(h1), float(h2), float(eps), float(tol), ctypes.byref(o),
                             ctypes.byref(r))
    if st == FS1_ERR_INVALID_ARG or st == FS1_ERR_HIP or st == FS1_ERR_NO_MEMORY or (
            raise_on_error and st != FS1_OK):
        raise Fs1Error(st, last_error())
    res = Result(r.w1, r.marginal_err, r.mu_err, r.iterations, bool(r.converged), st)
    if pot is not None and st == FS1_OK:
        res.F, res.G = pot[:n], pot[n:]
    if hist is not None:
        res.err_history = hist
    return res


def _dims_h(dims, h):
    if len(dims) != len(h):
        raise ValueError("dims and h must have the same length")
    cd = (ctypes.c_int64 * max(1, len(dims)))(*[int(v) for v in dims])
    ch = (ctypes.c_double * max(1, len(h)))(*[float(v) for v in h])
    n = 1
    for v in dims:
        n *= int(v)
    return cd, ch, n


def fs1_kv_apply_nd(x, dims: Sequence[int], h: Sequence[float], eps: float, out=None,
                    ctx: Optional[Context] = None):
    """y = K x on an n_0 x ... x n_{D-1} grid (first axis fastest),
    K = exp(-sum_a |i_a - j_a| h_a / eps)  (float64 or float32)."""
    import torch
    ctx = ctx or default_context()
    cd, ch, n = _dims_h(dims, h)
    if x.numel() != n:
        raise ValueError("x must hold prod(dims) entries")
    if out is None:
        out = torch.empty_like(x)
    _check(load().fs1_kv_apply_nd(ctx.handle, _dev(x, "x"), _dev(out, "out"), len(dims),
                                  ctypes.addressof(cd), ctypes.addressof(ch), float(eps),
                                  _dtype_code(x)))
    return out


def fs1_solve_nd(mu, nu, dims: Sequence[int], h: Sequence[float], eps: float, tol: float,
                 itr_max: int = 10000, dtype: str = "f64", check_every: int = 1,
                 sync_every: int = 16, potentials: bool = False, err_history: bool = False,
                 solver: str = "auto", ctx: Optional[Context] = None,
                 raise_on_error: bool = False, domain: str = "plain") -> Result:
    """Algorithm 2 on D axes (first axis fastest) on device float64 marginals
    of prod(dims) entries; arguments as fs1_solve_2d (solver "auto" takes the
    one-workgroup form only for D = 2)."""
    import torch
    ctx = ctx or default_context()
    cd, ch, n = _dims_h(dims, h)
    if mu.numel() != n or nu.numel() != n:
        raise ValueError("mu and nu must hold prod(dims) entries")
    o = make_opts(None, itr_max, dtype, domain, check_every, sync_every)
    o.flags |= {"auto": 0, "lines": FS1_FLAG_NO_RESIDENT}[solver]
    pot = hist = None
    if potentials:
        pot = torch.empty(2 * n, dtype=torch.float64, device=mu.device)
        o.flags |= FS1_FLAG_POTENTIALS
        o.potentials_out = pot.data_ptr()
    if err_history:
        hist = torch.empty(itr_max + 1, dtype=torch.float64, device=mu.device)
        o.err_history = hist.data_ptr()
    r = CResult()
    st = load().fs1_solve_nd(ctx.handle, _dev(mu, "mu"), _dev(nu, "nu"), len(dims),
                             ctypes.addressof(cd), ctypes.addressof(ch), float(eps), float(tol),
                             ctypes.byref(o), ctypes.byref(r))
    if st == FS1_ERR_INVALID_ARG or st == FS1_ERR_HIP or st == FS1_ERR_NO_MEMORY or (
            raise_on_error and st != FS1_OK):
        raise Fs1Error(st, last_error())
    res = Result(r.w1, r.marginal_err, r.mu_err, r.iterations, bool(r.converged), st)
    if pot is not None and st == FS1_OK:
        res.F, res.G = pot[:n], pot[n:]
    if hist is not None:
        res.err_history = hist
    return res


def fs1_solve_batched(mu_packed, nu_packed, offsets: Sequence[int], eps: Sequence[float],
                      tol: Sequence[float], itr_max: int = 10000, dtype: str = "f64",
                      domain: str = "log", check_every: int = 1, sync_every: int = 16,
                      graph: bool = True, ctx: Optional[Context] = None,
                      config: Optional[tuple] = None) -> list:
    """Ragged batch: instance b is [offsets[b], offsets[b+1]) of the packed
    float64 device tensors; eps and tol per instance.  Returns one Result per
    instance (per-instance failures in Result.status).  With domain="log" all
    instances advance in the same launches, `sync_every` iterations per
    replayed HIP graph (graph=False launches the kernels directly).
    config: (run length, threads) forced on every instance, or a list of such
    pairs, one per instance (threads 0: shared chunk launches; 256 or 1024:
    resident), through fs1_solve_batched_config."""
    ctx = ctx or default_context()
    B = len(offsets) - 1
    if len(eps) != B or len(tol) != B:
        raise ValueError("eps and tol need one entry per instance")
    if B > 0 and (int(offsets[-1]) > mu_packed.numel() or int(offsets[-1]) > nu_packed.numel()):
        raise ValueError("offsets run past the packed marginals")
    offs = (ctypes.c_int64 * (B + 1))(*[int(v) for v in offsets])
    o = make_opts(None, itr_max, dtype, domain, check_every, sync_every)
    on_device = [getattr(v, "is_cuda", False) for v in (eps, tol)]
    if any(on_device):
        # device tensors of eps and tol: passed as they are (FS1_FLAG_DEVICE_PARAMS)
        if not all(on_device):
            raise ValueError("eps and tol must both be device tensors or both host sequences")
        import torch
        if eps.dtype != torch.float64 or tol.dtype != torch.float64:
            raise TypeError("device eps and tol must be float64")
        if eps.numel() != B or tol.numel() != B:
            raise ValueError("eps and tol need one entry per instance")
        e, t = _dev(eps, "eps"), _dev(tol, "tol")
        o.flags |= FS1_FLAG_DEVICE_PARAMS
    else:
        e = (ctypes.c_double * max(B, 1))(*[float(v) for v in eps])
        t = (ctypes.c_double * max(B, 1))(*[float(v) for v in tol])
    if not graph:
        o.flags |= FS1_FLAG_NO_GRAPH
    res = (CResult * max(B, 1))()
    if config is None:
        _check(load().fs1_solve_batched(ctx.handle, _dev(mu_packed, "mu"), _dev(nu_packed, "nu"),
                                        offs, B, e, t, ctypes.byref(o), res))
    else:  # fs1_solve_batched_config
        if len(config) == 2 and not isinstance(config[0], (tuple, list)):
            config = [config] * B
        if len(config) != B:
            raise ValueError("config: one (run length, threads) pair, or one per instance")
        rl = (ctypes.c_int32 * max(B, 1))(*[int(c[0]) for c in config])
        th = (ctypes.c_int32 * max(B, 1))(*[int(c[1]) for c in config])
        _check(load().fs1_solve_batched_config(ctx.handle, _dev(mu_packed, "mu"),
                                               _dev(nu_packed, "nu"), offs, B, e, t,
                                               ctypes.byref(o), rl, th, res))
    return [Result(r.w1, r.marginal_err, r.mu_err, r.iterations, bool(r.converged), r.status)
            for r in res[:B]]


class Server:
    """Request loop with continuous batching (fs1_server_*): submit device
    marginal pairs, call step() repeatedly, poll() completions.  The binding
    keeps each request's tensors alive until its completion is polled.
    overlap: step() returns once its iterations are enqueued and the next
    call reports the completions they produce (FS1_FLAG_SERVER_OVERLAP)."""

    def __init__(self, hbm_budget: int = 1 << 30, max_active: int = 4096, dtype: str = "f32",
                 itr_max: int = 10000, check_every: int = 1, iters_per_step: int = 16,
                 graph: bool = True, overlap: bool = False, ctx: Optional[Context] = None):
        lib = load()
        self.ctx = ctx or default_context()
        o = ServerOpts()
        _check(lib.fs1_server_opts_default(ctypes.byref(o)))
        o.hbm_budget = int(hbm_budget)
        o.max_active = int(max_active)
        o.dtype = {"f64": FS1_F64, "f32": FS1_F32}[dtype]
        o.itr_max = int(itr_max)
        o.check_every = int(check_every)
        o.iters_per_step = int(iters_per_step)
        o.flags = (0 if graph else FS1_FLAG_NO_GRAPH) | (FS1_FLAG_SERVER_OVERLAP if overlap else 0)
        h = ctypes.c_void_p()
        _check(lib.fs1_server_create(self.ctx.handle, ctypes.byref(o), ctypes.byref(h)))
        self.handle = h
        self._held = {}
        self._buf = (Completion * 1024)()

    def submit(self, mu, nu, eps: float, tol: float) -> int:
        if mu.numel() != nu.numel():
            raise ValueError("mu and nu must have the same length")
        t = ctypes.c_int64()
        _check(load().fs1_server_submit(self.handle, _dev(mu, "mu"), _dev(nu, "nu"), mu.numel(),
                                        float(eps), float(tol), ctypes.byref(t)))
        self._held[t.value] = (mu, nu)
        return t.value

    def step(self) -> int:
        n = ctypes.c_int32()
        _check(load().fs1_server_step(self.handle, ctypes.byref(n)))
        return n.value

    def poll(self) -> list:
        """[(ticket, Result, admitted_step, completed_step), ...], oldest first."""
        out = []
        while True:
            k = ctypes.c_int32()
            _check(load().fs1_server_poll(self.handle, self._buf, len(self._buf),
                                          ctypes.byref(k)))
            for c in self._buf[:k.value]:
                r = c.result
                out.append((c.ticket, Result(r.w1, r.marginal_err, r.mu_err, r.iterations,
                                             bool(r.converged), r.status),
                            c.admitted_step, c.completed_step))
                self._held.pop(c.ticket, None)
            if k.value < len(self._buf):
                return out

    def info(self) -> dict:
        i = ServerInfo()
        _check(load().fs1_server_get_info(self.handle, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in ServerInfo._fields_}

    def close(self):
        if getattr(self, "handle", None):
            load().fs1_server_destroy(self.handle)
            self.handle = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
