"""ctypes binding of libhawkes (include/hawkes.h): argument marshalling only.

Every evaluation runs in the library's HIP kernels on the GPU; nothing here computes any part of
the likelihood, and there is no fallback: if ``libhawkes.so`` is missing or cannot be loaded the
import of this module's entry points raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(HERE, "libhawkes.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hawkes.h")

HAWKES_OK = 0
HAWKES_EINVAL = -1
HAWKES_ENOMEM = -2
HAWKES_EBUSY = -3
HAWKES_EAGAIN = -4
HAWKES_EDEVICE = -5
HAWKES_ENOTFOUND = -6
HAWKES_ECANCELED = -7
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EBUSY", -4: "EAGAIN", -5: "EDEVICE",
                -6: "ENOTFOUND", -7: "ECANCELED"}
FP64 = 0
FP32C = 1
PAIRS_SYMMETRIC = 0
PAIRS_DIRECT = 1
SCHEMES = {"symmetric": PAIRS_SYMMETRIC, "direct": PAIRS_DIRECT}
PRECISIONS = {"fp64": FP64, "fp32c": FP32C}
ROW_FIELDS = 10
PARAM_NAMES = ("mu0", "tau_x", "tau_t", "theta", "omega", "h")


class HawkesError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in PARAM_NAMES]


class Request(ctypes.Structure):
    _fields_ = [("dataset", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("want_grad", ctypes.c_int32), ("_pad", ctypes.c_int32), ("p", Params),
                ("tag", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("_pad", ctypes.c_int32),
                ("loglik", ctypes.c_double), ("grad", ctypes.c_double * 6),
                ("t_submit_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def exported_names():
    """Function names declared in include/hawkes.h."""
    import re

    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hawkes_[a-z_0-9]+)\s*\(", text)))


def load(path: str | None = None):
    """Load libhawkes.so (built in-tree by paper_2005_10123_amd.build); raises if it is missing."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    target = path or LIBRARY
    if not os.path.exists(target):
        raise ImportError(f"{target} is not built; run paper_2005_10123_amd.build.build() first")
    # torch ships a HIP runtime with the same soname as the system one; loading torch first makes
    # the library bind to that single runtime, so torch tensors and library calls share one.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(target)
    vp = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    sig = {
        "hawkes_create": ([ctypes.c_int, ctypes.c_size_t, vp, ctypes.POINTER(vp)], i32),
        "hawkes_destroy": ([vp], i32),
        "hawkes_dataset_create": ([vp, _dp, _dp, _dp, i64, ctypes.POINTER(i32)], i32),
        "hawkes_dataset_destroy": ([vp, i32], i32),
        "hawkes_dataset_info": ([vp, i32, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_size_t)], i32),
        "hawkes_loglik": ([vp, i32, ctypes.POINTER(Params), ctypes.c_int, _dp], i32),
        "hawkes_grad": ([vp, i32, ctypes.POINTER(Params), ctypes.c_int, _dp, _dp], i32),
        "hawkes_grad_device": ([vp, i32, ctypes.POINTER(Params), ctypes.c_int, vp, vp], i32),
        "hawkes_grad_device_noalloc": ([vp, i32, ctypes.POINTER(Params), ctypes.c_int, vp, vp], i32),
        "hawkes_rows": ([vp, i32, ctypes.POINTER(Params), ctypes.c_int, _dp], i32),
        "hawkes_submit": ([vp, ctypes.POINTER(Request), i32], i32),
        "hawkes_poll": ([vp, ctypes.POINTER(Result), i32, ctypes.POINTER(i32), i64], i32),
        "hawkes_outstanding": ([vp, ctypes.POINTER(i64)], i32),
        "hawkes_last_error": ([], ctypes.c_char_p),
        "hawkes_profile": ([vp, ctypes.c_int], i32),
        "hawkes_set_pair_scheme": ([vp, ctypes.c_int], i32),
        "hawkes_set_zero_tile_skipping": ([vp, ctypes.c_int], i32),
        "hawkes_set_shared_passes": ([vp, ctypes.c_int], i32),
        "hawkes_loglik_multi": ([vp, i32, ctypes.POINTER(Params), i32, ctypes.c_int, _dp, _dp], i32),
        "hawkes_kernel_time": ([vp, _dp, ctypes.POINTER(i64), ctypes.c_int], i32),
        "hawkes_host_eval": ([_dp, _dp, _dp, i64, ctypes.POINTER(Params), ctypes.c_int, _dp, _dp], i32),
        "hawkes_shard_sums": ([vp, i32, ctypes.POINTER(Params), ctypes.c_int, i32, i32, _dp], i32),
        "hawkes_finish": ([vp, i32, ctypes.POINTER(Params), _dp, _dp, _dp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    if path is None:
        _lib = lib
    return lib


def _check(status):
    if status != HAWKES_OK:
        raise HawkesError(status, load().hawkes_last_error().decode())


def params(theta) -> Params:
    if isinstance(theta, Params):
        return theta
    v = [float(a) for a in theta]
    if len(v) != 6:
        raise ValueError("theta must hold (mu0, tau_x, tau_t, theta, omega, h)")
    return Params(*v)


def _prec(precision):
    return PRECISIONS[precision] if isinstance(precision, str) else int(precision)


class Context:
    """A libhawkes context on one GPU (hawkes_create / hawkes_destroy)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, stream=None):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.hawkes_create(int(device), int(hbm_budget), stream, ctypes.byref(h)))
        self._h = h
        self.lib = lib

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            self.lib.hawkes_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- datasets ----------------------------------------------------------------------------
    def dataset(self, x, y, t) -> "Dataset":
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        t = np.ascontiguousarray(t, dtype=np.float64)
        if not (x.shape == y.shape == t.shape and x.ndim == 1):
            raise ValueError("x, y, t must be 1-D arrays of equal length")
        out = ctypes.c_int32()
        _check(self.lib.hawkes_dataset_create(self._h, x.ctypes.data_as(_dp), y.ctypes.data_as(_dp),
                                              t.ctypes.data_as(_dp), x.size, ctypes.byref(out)))
        return Dataset(self, out.value, x.size)

    # -- blocking evaluation -----------------------------------------------------------------
    def loglik(self, ds, theta, precision="fp32c") -> float:
        out = ctypes.c_double()
        _check(self.lib.hawkes_loglik(self._h, _id(ds), ctypes.byref(params(theta)), _prec(precision),
                                      ctypes.byref(out)))
        return out.value

    def grad(self, ds, theta, precision="fp32c"):
        ell = ctypes.c_double()
        g = np.zeros(6)
        _check(self.lib.hawkes_grad(self._h, _id(ds), ctypes.byref(params(theta)), _prec(precision),
                                    ctypes.byref(ell), g.ctypes.data_as(_dp)))
        return ell.value, g

    def rows(self, ds, theta, precision="fp32c"):
        """Per-event results in caller order: dict of lambda, Lambda, ell, pi (n,), grad (n, 6)."""
        n = ds.n if isinstance(ds, Dataset) else int(self.info(ds)[0])
        out = np.zeros((n, ROW_FIELDS))
        _check(self.lib.hawkes_rows(self._h, _id(ds), ctypes.byref(params(theta)), _prec(precision),
                                    out.ctypes.data_as(_dp)))
        return {"lambda": out[:, 0].copy(), "Lambda": out[:, 1].copy(), "ell": out[:, 2].copy(),
                "pi": out[:, 3].copy(), "grad": out[:, 4:10].copy()}

    def shard_sums(self, ds, theta, shard, nshards, precision="fp32c"):
        """Per-event sums (n, 6) = (S_b, S_br, S_bt, S_e, S_et, S_er) of one shard of the pairwise
        pass, caller order; the sums of all shards added together go to finish()."""
        n = ds.n if isinstance(ds, Dataset) else int(self.info(ds)[0])
        out = np.zeros((n, 6))
        _check(self.lib.hawkes_shard_sums(self._h, _id(ds), ctypes.byref(params(theta)), _prec(precision),
                                          int(shard), int(nshards), out.ctypes.data_as(_dp)))
        return out

    def finish(self, ds, theta, sums):
        """(ell, gradient) from per-event sums (n, 6) added over all shards."""
        sums = np.ascontiguousarray(sums, dtype=np.float64)
        ell = ctypes.c_double()
        g = np.zeros(6)
        _check(self.lib.hawkes_finish(self._h, _id(ds), ctypes.byref(params(theta)), sums.ctypes.data_as(_dp),
                                      ctypes.byref(ell), g.ctypes.data_as(_dp)))
        return ell.value, g

    def loglik_multi(self, ds, thetas, precision="fp32c", want_pi=True):
        """Log-likelihoods (S,) and, with want_pi, self-excitation probabilities (S, n) for S
        parameter vectors (rows of `thetas`)."""
        th = np.ascontiguousarray(thetas, dtype=np.float64).reshape(-1, 6)
        S = th.shape[0]
        n = ds.n if isinstance(ds, Dataset) else int(self.info(ds)[0])
        arr = (Params * S)(*[params(row) for row in th])
        ll = np.zeros(S)
        pi = np.zeros((S, n)) if want_pi else None
        _check(self.lib.hawkes_loglik_multi(self._h, _id(ds), arr, S, _prec(precision), ll.ctypes.data_as(_dp),
                                            pi.ctypes.data_as(_dp) if want_pi else None))
        return (ll, pi) if want_pi else ll

    def grad_device(self, ds, theta, precision, d_out7_ptr: int, stream_ptr=0):
        """Enqueue on the hipStream_t `stream_ptr` (0: the null stream)."""
        _check(self.lib.hawkes_grad_device(self._h, _id(ds), ctypes.byref(params(theta)), _prec(precision),
                                           ctypes.c_void_p(d_out7_ptr), ctypes.c_void_p(stream_ptr or None)))

    def grad_device_noalloc(self, ds, theta, precision, d_out7_ptr: int, stream_ptr=0):
        """hawkes_grad_device with the library's fixed device scratch (no allocation); enqueued on
        the hipStream_t `stream_ptr` (0: the null stream)."""
        _check(self.lib.hawkes_grad_device_noalloc(self._h, _id(ds), ctypes.byref(params(theta)), _prec(precision),
                                                   ctypes.c_void_p(d_out7_ptr), ctypes.c_void_p(stream_ptr or None)))

    def info(self, ds):
        n = ctypes.c_int64()
        b = ctypes.c_size_t()
        _check(self.lib.hawkes_dataset_info(self._h, _id(ds), ctypes.byref(n), ctypes.byref(b)))
        return n.value, b.value

    # -- serving -------------------------------------------------------------------------------
    def submit(self, requests):
        arr = (Request * len(requests))()
        for k, r in enumerate(requests):
            arr[k] = r
        _check(self.lib.hawkes_submit(self._h, arr, len(requests)))

    def poll(self, cap=256, timeout_us=0):
        buf = (Result * cap)()
        n = ctypes.c_int32()
        st = self.lib.hawkes_poll(self._h, buf, cap, ctypes.byref(n), int(timeout_us))
        if st not in (HAWKES_OK, HAWKES_EAGAIN):
            _check(st)
        return [buf[k] for k in range(n.value)]

    def outstanding(self):
        n = ctypes.c_int64()
        _check(self.lib.hawkes_outstanding(self._h, ctypes.byref(n)))
        return n.value

    def set_pair_scheme(self, scheme="symmetric"):
        """"symmetric" (default: each unordered pair once) or "direct" (every ordered pair)."""
        _check(self.lib.hawkes_set_pair_scheme(self._h, SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)))

    def set_zero_tile_skipping(self, enable=True):
        """Leave out the column tiles whose pair terms are all exactly zero (see include/hawkes.h)."""
        _check(self.lib.hawkes_set_zero_tile_skipping(self._h, 1 if enable else 0))

    def set_shared_passes(self, enable=True):
        """Served FP32C log-likelihoods in shared multi-parameter passes (see include/hawkes.h)."""
        _check(self.lib.hawkes_set_shared_passes(self._h, 1 if enable else 0))

    # -- diagnostics ---------------------------------------------------------------------------
    def profile(self, enable=True):
        _check(self.lib.hawkes_profile(self._h, 1 if enable else 0))

    def kernel_time(self, reset=False):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(self.lib.hawkes_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0))
        return ms.value, n.value


def host_eval(x, y, t, theta, threads=0, want_pi=False):
    """hawkes_host_eval: (ell, gradient[6]) and, with want_pi, pi (n,) in the caller's order, on the
    host's CPU cores (binary64, SIMD); needs no GPU."""
    lib = load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    if not (x.shape == y.shape == t.shape and x.ndim == 1):
        raise ValueError("x, y, t must be 1-D arrays of equal length")
    out = np.zeros(7)
    pi = np.zeros(x.size) if want_pi else None
    _check(lib.hawkes_host_eval(x.ctypes.data_as(_dp), y.ctypes.data_as(_dp), t.ctypes.data_as(_dp), x.size,
                                ctypes.byref(params(theta)), int(threads), out.ctypes.data_as(_dp),
                                pi.ctypes.data_as(_dp) if want_pi else None))
    return (out[0], out[1:].copy(), pi) if want_pi else (out[0], out[1:].copy())


def request(dataset, theta, precision="fp32c", want_grad=True, tag=0) -> Request:
    return Request(_id(dataset), _prec(precision), 1 if want_grad else 0, 0, params(theta), tag)


class Dataset:
    """A device-resident event set (hawkes_dataset_create / hawkes_dataset_destroy)."""

    def __init__(self, ctx: Context, ident: int, n: int):
        self.ctx = ctx
        self.id = ident
        self.n = n

    def close(self):
        if self.id >= 0 and self.ctx._h:
            _check(self.ctx.lib.hawkes_dataset_destroy(self.ctx._h, self.id))
        self.id = -1


def _id(ds):
    return ds.id if isinstance(ds, Dataset) else int(ds)
