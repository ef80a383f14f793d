"""Large-N workload: N = 1,000,000 events on a 40 x 40 km square over 20,000 days (exact O(N^2),
FP32C and FP64 symmetric passes), compared with each other at full size and, on a seeded
20,000-event subsample evaluated as its own dataset, with the FP64 oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import TOL, assert_close, grad_errors, rel
from paper_2005_10123_amd import binding, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stress():
    (x, y, t), th = synth.config_events("stress_1m")
    return x, y, t, th


def test_subsample_against_oracle(stress):
    x, y, t, th = stress
    xs, ys, ts = synth.subsample(x, y, t, 20000)
    ref = oracle.evaluate(xs, ys, ts, th, rows=True)
    ctx = binding.Context(0)
    ds = ctx.dataset(xs, ys, ts)
    for prec in ("fp64", "fp32c"):
        ell, g = ctx.grad(ds, th, prec)
        assert_close(ell, g, ref, prec, "stress subsample", th)
    ds.close()
    ctx.close()


def test_full_size_fp32c_against_fp64(stress):
    x, y, t, th = stress
    ctx = binding.Context(0)
    ds = ctx.dataset(x, y, t)
    e64, g64 = ctx.grad(ds, th, "fp64")
    e32, g32 = ctx.grad(ds, th, "fp32c")
    r64 = ctx.rows(ds, th, "fp64")
    assert rel(e32, e64) <= TOL["fp32c"], (e32, e64)
    assert abs(e64 - r64["ell"].sum()) <= 1e-9 * np.abs(r64["ell"]).sum()
    plain, normed = grad_errors(g32, g64, r64["grad"], e64, th)
    assert np.all(normed <= TOL["fp32c"]), normed
    assert np.all(plain <= TOL["fp32c"]), plain
    # mu0 dl/dmu0 + theta dl/dtheta = N - Lambda holds at any size
    lhs = th[0] * g64[0] + th[3] * g64[3]
    assert abs(lhs - (x.size - r64["Lambda"].sum())) <= 1e-9 * x.size
    # a few rows against the oracle at full size
    idx = np.array([0, 1, 250000, 500000, 999998, 999999])
    ref = oracle.rows(x, y, t, th, idx)
    r32 = ctx.rows(ds, th, "fp32c")
    assert np.max(np.abs(r32["lambda"][idx] - ref["lambda"]) / ref["lambda"]) <= TOL["fp32c"]
    assert np.max(np.abs(r64["lambda"][idx] - ref["lambda"]) / ref["lambda"]) <= TOL["fp64"]
    ds.close()
    ctx.close()


def test_full_size_zero_tile_skipping(stress):
    """At 10^6 events over 20,000 days most tiles are skipped; the per-event results agree with the
    full pass to rounding and sampled rows with the oracle."""
    x, y, t, th = stress
    ctx = binding.Context(0)
    ds = ctx.dataset(x, y, t)
    e0, g0 = ctx.grad(ds, th, "fp32c")
    ctx.set_zero_tile_skipping(True)
    e1, g1 = ctx.grad(ds, th, "fp32c")
    r1 = ctx.rows(ds, th, "fp32c")
    ctx.set_zero_tile_skipping(False)
    assert rel(e1, e0) <= 1e-12, (e1, e0)
    assert np.all(np.abs(g1 - g0) <= 1e-12 * np.abs(r1["grad"]).sum(axis=0)), (g1, g0)
    idx = np.array([0, 1, 250000, 500000, 999998, 999999])
    ref = oracle.rows(x, y, t, th, idx)
    assert np.max(np.abs(r1["lambda"][idx] - ref["lambda"]) / ref["lambda"]) <= TOL["fp32c"]
    ds.close()
    ctx.close()
