"""FP64 CPU oracle of the spatiotemporal Hawkes log-likelihood (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg import this
package.  The product library never does, and this package imports nothing from it.

The arithmetic lives in ``hawkes_oracle.c`` (plain nested loops, binary64, libm); this module only
compiles it with gcc and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "hawkes_oracle.c")
LIBRARY = os.path.join(_HERE, "libhawkes_oracle.so")
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-shared", "-fPIC"]

_lib = None


def build(source: str = SOURCE, output: str = LIBRARY) -> str:
    """Compile the oracle (or a planted-mistake copy of it) into a shared library."""
    cmd = ["gcc", *CFLAGS, source, "-lm", "-o", output]
    subprocess.run(cmd, check=True)
    return output


def load(path: str | None = None):
    """Load a compiled oracle library; builds the default one if it is missing."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    target = path or LIBRARY
    if not os.path.exists(target):
        if path is not None:
            raise FileNotFoundError(target)
        build()
    lib = ctypes.CDLL(target)
    dp = ctypes.POINTER(ctypes.c_double)
    lp = ctypes.POINTER(ctypes.c_long)
    lib.hawkes_oracle_eval.argtypes = [dp, dp, dp, ctypes.c_long, dp, dp, dp, dp, dp, dp]
    lib.hawkes_oracle_eval.restype = ctypes.c_int
    lib.hawkes_oracle_rows.argtypes = [dp, dp, dp, ctypes.c_long, dp, lp, ctypes.c_long, dp]
    lib.hawkes_oracle_rows.restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _events(x, y, t):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    if not (x.shape == y.shape == t.shape and x.ndim == 1):
        raise ValueError("x, y, t must be 1-D arrays of equal length")
    return x, y, t


def evaluate(x, y, t, theta, lib=None, rows: bool = False):
    """Log-likelihood and gradient of all events.

    Returns ``(ell, grad[6])``, or with ``rows=True`` a dict that also holds the per-event
    ``row_ell``, ``row_Lambda``, ``row_pi`` and ``row_grad`` (n x 6).
    """
    lib = lib or load()
    x, y, t = _events(x, y, t)
    n = x.size
    th = np.ascontiguousarray(theta, dtype=np.float64)
    assert th.shape == (6,)
    out = np.zeros(7)
    r_ell = np.zeros(n) if rows else None
    r_Lam = np.zeros(n) if rows else None
    r_pi = np.zeros(n) if rows else None
    r_grad = np.zeros((n, 6)) if rows else None
    rc = lib.hawkes_oracle_eval(_dptr(x), _dptr(y), _dptr(t), n, _dptr(th), _dptr(out),
                                _dptr(r_ell), _dptr(r_Lam), _dptr(r_pi), _dptr(r_grad))
    if rc != 0:
        raise ValueError("oracle rejected its input")
    if not rows:
        return out[0], out[1:].copy()
    return {"ell": out[0], "grad": out[1:].copy(), "row_ell": r_ell, "row_Lambda": r_Lam,
            "row_pi": r_pi, "row_grad": r_grad}


ROW_FIELDS = ("lambda", "Lambda", "ell", "pi", "grad", "sums")


def rows(x, y, t, theta, row_index, lib=None):
    """Per-row results for the selected events (each row against all n events).

    Returns a dict of arrays: lambda, Lambda, ell, pi (m,), grad (m, 6) and sums (m, 6) with
    sums = (Sb, Sbr, Sbt, Se, Set, Ser).
    """
    lib = lib or load()
    x, y, t = _events(x, y, t)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    idx = np.ascontiguousarray(row_index, dtype=np.int64)
    out = np.zeros((idx.size, 16))
    rc = lib.hawkes_oracle_rows(_dptr(x), _dptr(y), _dptr(t), x.size, _dptr(th),
                                idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), idx.size,
                                _dptr(out))
    if rc != 0:
        raise ValueError("oracle rejected its input")
    return {"lambda": out[:, 0].copy(), "Lambda": out[:, 1].copy(), "ell": out[:, 2].copy(),
            "pi": out[:, 3].copy(), "grad": out[:, 4:10].copy(), "sums": out[:, 10:16].copy()}


def evaluate_parallel(x, y, t, theta, threads: int | None = None, lib=None):
    """The whole evaluation (``evaluate(..., rows=True)``) with the rows split into contiguous
    ranges run on host threads (the C loop releases the interpreter lock): each range goes
    through ``hawkes_oracle_rows``, which evaluates every row exactly as ``evaluate`` does.  The
    totals are the exactly rounded sums (``math.fsum``) of the per-event values, so they do not
    depend on the split.  Returns the same dict as ``evaluate(rows=True)`` plus ``row_lambda``
    and ``row_sums`` (n x 6)."""
    from concurrent.futures import ThreadPoolExecutor

    lib = lib or load()
    x, y, t = _events(x, y, t)
    n = x.size
    if threads is None:
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
    parts = [p for p in np.array_split(np.arange(n, dtype=np.int64), threads) if p.size]
    with ThreadPoolExecutor(len(parts)) as pool:
        res = list(pool.map(lambda idx: rows(x, y, t, theta, idx, lib=lib), parts))
    cat = {k: np.concatenate([r[k] for r in res]) for k in res[0]}
    return {"ell": math.fsum(cat["ell"]), "grad": np.array([math.fsum(cat["grad"][:, p]) for p in range(6)]),
            "row_ell": cat["ell"], "row_Lambda": cat["Lambda"], "row_pi": cat["pi"], "row_grad": cat["grad"],
            "row_lambda": cat["lambda"], "row_sums": cat["sums"]}
