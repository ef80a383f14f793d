"""Shared helpers of the GPU tests: one context per session and the error metrics used for every
comparison with the oracle."""
import numpy as np
import pytest

# Tolerances: relative error of ell and of each gradient component against the FP64 oracle.
TOL = {"fp64": 1e-10, "fp32c": 1e-5}


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def floor_scale(ell_ref, theta):
    return abs(ell_ref) / np.maximum(np.abs(np.asarray(theta, float)), 1.0)


def row_ell_error(ell_rows, ell_rows_ref):
    """Per-event ell_i = log lambda_i - Lambda_i may cancel to near 0; its error is measured
    against max(|ell_i|, 1) (the absolute error of log lambda_i is the relative error of lambda_i)."""
    return np.max(np.abs(ell_rows - ell_rows_ref) / np.maximum(np.abs(ell_rows_ref), 1.0))


def grad_errors(g, g_ref, row_grad_ref, ell_ref, theta):
    """Per component p: the plain relative error, and the normalised error
    |dg_p| / max(sum_i |g_{i,p}|, |ell| / |theta_p|).  The first scale is the l1 norm of the
    per-event terms the component is summed from (it may cancel); the floor |ell| / |theta_p| is
    the gradient at which changing theta_p by max(|theta_p|, 1) would change ell by its own size --
    below it a component is negligible (e.g. trigger terms underflowing binary32 at
    omega = 1440 / day)."""
    l1 = np.abs(row_grad_ref).sum(axis=0)
    scale = np.maximum(l1, floor_scale(ell_ref, theta))
    plain = np.abs(g - g_ref) / np.maximum(np.abs(g_ref), 1e-300)
    normed = np.abs(g - g_ref) / np.maximum(scale, 1e-300)
    return plain, normed


def kappa(ref):
    """Cancellation factor of each gradient component: sum_i |g_{i,p}| / |g_p|."""
    return np.abs(ref["row_grad"]).sum(axis=0) / np.maximum(np.abs(ref["grad"]), 1e-300)


def assert_close(ell, g, ref, prec, what="", theta=None):
    tol = TOL[prec]
    assert rel(ell, ref["ell"]) <= tol, (what, prec, "ell", ell, ref["ell"], rel(ell, ref["ell"]))
    if g is None:
        return
    plain, normed = grad_errors(g, ref["grad"], ref["row_grad"], ref["ell"], theta)
    assert np.all(normed <= tol), (what, prec, "grad l1-normalised", normed)
    # The plain relative error is gated at the same tolerance on every component that is not
    # negligible (at or above the floor), however much it cancels between events.
    meaningful = np.abs(ref["grad"]) >= floor_scale(ref["ell"], theta)
    assert np.all(plain[meaningful] <= tol), (what, prec, "grad plain", plain, "kappa", kappa(ref))
