"""The C ABI without a GPU: the library loads, exports every declared symbol,
the binding's struct layouts match the header, and validation fails fast."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2202_10042_amd import fs1

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fs1.h")


def _lib():
    if not os.path.exists(fs1.LIB_PATH):
        from paper_2202_10042_amd import build
        build.build()
    return fs1.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fs1_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = _lib()
    names = declared_functions()
    assert len(names) >= 10
    assert set(names) == set(fs1.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", fs1.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (fs1_\w+)", out))
    assert set(names) <= exported


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "fs1.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(fs1_opts),
         offsetof(fs1_opts, itr_max), offsetof(fs1_opts, check_every),
         offsetof(fs1_opts, flags), offsetof(fs1_opts, potentials_out),
         offsetof(fs1_opts, err_history), sizeof(fs1_result),
         offsetof(fs1_result, iterations), offsetof(fs1_result, status),
         offsetof(fs1_result, mu_err), offsetof(fs1_opts, warm_m), offsetof(fs1_opts, warm_e),
         offsetof(fs1_opts, state_m), offsetof(fs1_opts, state_e));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    O, R = fs1.Opts, fs1.CResult
    want = [ctypes.sizeof(O), O.itr_max.offset, O.check_every.offset, O.flags.offset,
            O.potentials_out.offset, O.err_history.offset, ctypes.sizeof(R),
            R.iterations.offset, R.status.offset, R.mu_err.offset, O.warm_m.offset,
            O.warm_e.offset, O.state_m.offset, O.state_e.offset]
    assert got == want


def test_validation_before_any_launch():
    lib = _lib()
    # no context -> invalid argument, no device call
    st = lib.fs1_kv_apply(None, ctypes.c_void_p(16), ctypes.c_void_p(4096), 10, 0.1, 0.1, 0)
    assert st == fs1.FS1_ERR_INVALID_ARG
    assert "context" in fs1.last_error()
    r = fs1.CResult()
    st = lib.fs1_solve(None, None, None, 10, 0.1, 0.0, None, ctypes.byref(r))
    assert st == fs1.FS1_ERR_INVALID_ARG
    o = fs1.Opts()
    assert lib.fs1_opts_default(ctypes.byref(o)) == 0
    assert o.itr_max == 10000 and o.check_every == 1 and o.dtype == 0 and o.domain == 0
    assert lib.fs1_version().decode().startswith("fs1")
    # allocator callbacks come in pairs (checked before any device call)
    h = ctypes.c_void_p()
    alloc = fs1.ALLOC_FN(lambda n, u: None)
    st = lib.fs1_ctx_create_with_allocator(None, alloc, fs1.FREE_FN(), None, ctypes.byref(h))
    assert st == fs1.FS1_ERR_INVALID_ARG and "callbacks" in fs1.last_error()
    # the no-allocation solve validates its context first
    st = lib.fs1_solve_noalloc(None, None, None, 10, 0.1, 0.0, None, ctypes.byref(r))
    assert st == fs1.FS1_ERR_INVALID_ARG


def test_no_cpu_fallback_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(fs1, "_lib", None)
    with pytest.raises(RuntimeError):
        fs1.load(str(tmp_path / "missing.so"))


def test_flag_and_enum_values_match_header():
    text = open(HEADER).read()
    flags = dict((k, int(v)) for k, v in re.findall(r"#define (FS1_FLAG_\w+) (\d+)", text))
    assert flags and all(getattr(fs1, k) == v for k, v in flags.items())
    for name in ("FS1_OK", "FS1_ERR_INVALID_ARG", "FS1_ERR_NONFINITE", "FS1_F64", "FS1_F32",
                 "FS1_PLAIN", "FS1_LOG"):
        m = re.search(name + r"\s*=\s*(-?\d+)", text)
        assert m and getattr(fs1, name) == int(m.group(1)), name


def test_batched_validation_without_context():
    lib = _lib()
    r = (fs1.CResult * 1)()
    offs = (ctypes.c_int64 * 2)(0, 4)
    e = (ctypes.c_double * 1)(0.1)
    st = lib.fs1_solve_batched(None, None, None, offs, 1, e, e, None, r)
    assert st == fs1.FS1_ERR_INVALID_ARG and "context" in fs1.last_error()


def test_server_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout2.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "fs1.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(fs1_server_opts),
         offsetof(fs1_server_opts, max_active), offsetof(fs1_server_opts, iters_per_step),
         offsetof(fs1_server_opts, flags), sizeof(fs1_completion),
         offsetof(fs1_completion, result), offsetof(fs1_completion, admitted_step),
         offsetof(fs1_completion, completed_step), sizeof(fs1_server_info),
         offsetof(fs1_server_info, bytes_total));
  return 0;
}
''')
    exe = tmp_path / "layout2"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    S, C, I = fs1.ServerOpts, fs1.Completion, fs1.ServerInfo
    want = [ctypes.sizeof(S), S.max_active.offset, S.iters_per_step.offset, S.flags.offset,
            ctypes.sizeof(C), C.result.offset, C.admitted_step.offset, C.completed_step.offset,
            ctypes.sizeof(I), I.bytes_total.offset]
    assert got == want


def test_server_validation_without_gpu():
    lib = _lib()
    o = fs1.ServerOpts()
    assert lib.fs1_server_opts_default(ctypes.byref(o)) == 0
    assert o.dtype == fs1.FS1_F32 and o.iters_per_step == 16 and o.max_active == 4096
    h = ctypes.c_void_p()
    assert lib.fs1_server_create(None, ctypes.byref(o), ctypes.byref(h)) == fs1.FS1_ERR_INVALID_ARG
    assert lib.fs1_server_step(None, None) == fs1.FS1_ERR_INVALID_ARG
    t = ctypes.c_int64()
    assert lib.fs1_server_submit(None, None, None, 4, 0.1, 0.0,
                                 ctypes.byref(t)) == fs1.FS1_ERR_INVALID_ARG
    assert lib.fs1_server_destroy(None) == 0

