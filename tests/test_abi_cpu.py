"""The C ABI library loads and exports every function include/hawkes.h declares; host-side argument
checks that touch no device.  CPU only."""
import ctypes
import os
import subprocess

import pytest

from paper_2005_10123_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_function():
    lib = binding.load()
    names = binding.exported_names()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIBRARY], capture_output=True, text=True).stdout
    for name in names:
        assert f" T {name}\n" in out, name


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include "hawkes.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(hawkes_params), sizeof(hawkes_request),'
                   ' sizeof(hawkes_result), offsetof(hawkes_result, loglik), offsetof(hawkes_request, tag));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert got == [ctypes.sizeof(binding.Params), ctypes.sizeof(binding.Request), ctypes.sizeof(binding.Result),
                   binding.Result.loglik.offset, binding.Request.tag.offset]


def test_null_context_is_rejected_without_device():
    lib = binding.load()
    out = ctypes.c_double()
    p = binding.params([1, 0.5, 20, 0.3, 0.5, 0.1])
    assert lib.hawkes_loglik(None, 0, ctypes.byref(p), 1, ctypes.byref(out)) == binding.HAWKES_EINVAL
    assert b"NULL" in lib.hawkes_last_error()
    assert lib.hawkes_submit(None, None, 0) == binding.HAWKES_EINVAL
    n = ctypes.c_int32()
    assert lib.hawkes_poll(None, None, 0, ctypes.byref(n), 0) == binding.HAWKES_EINVAL
    sums = (ctypes.c_double * 6)()
    assert lib.hawkes_shard_sums(None, 0, ctypes.byref(p), 1, 0, 1, sums) == binding.HAWKES_EINVAL
    assert lib.hawkes_finish(None, 0, ctypes.byref(p), sums, ctypes.byref(out), None) == binding.HAWKES_EINVAL
    assert lib.hawkes_set_zero_tile_skipping(None, 1) == binding.HAWKES_EINVAL
    assert lib.hawkes_destroy(None) == binding.HAWKES_OK
    assert lib.hawkes_create(0, 0, None, None) == binding.HAWKES_EINVAL


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(ImportError):
        binding.load(str(tmp_path / "nope.so"))


def test_failures_are_logged_when_asked(tmp_path):
    """HAWKES_LOG=1 prints each recorded failure message to stderr (read once per process)."""
    import sys

    code = ("import ctypes; from paper_2005_10123_amd import binding; lib = binding.load(); "
            "out = ctypes.c_double(); p = binding.params([1, 0.5, 20, 0.3, 0.5, 0.1]); "
            "lib.hawkes_loglik(None, 0, ctypes.byref(p), 1, ctypes.byref(out))")
    env = dict(os.environ, HAWKES_LOG="1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    assert "libhawkes: status -1: ctx is NULL" in r.stderr
    env["HAWKES_LOG"] = "0"
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT)
    assert "libhawkes" not in r.stderr


def test_package_star_import_names_real_modules():
    """Every name the package lists in __all__ is a module of the package."""
    import importlib

    import paper_2005_10123_amd as pkg

    for name in pkg.__all__:
        importlib.import_module(f"paper_2005_10123_amd.{name}")
    ns = {}
    exec("from paper_2005_10123_amd import *", ns)
    assert set(pkg.__all__) <= set(ns)
