"""torch.autograd.Function over the fused pass: forward equals the blocking call, backward returns
grad_output times the adjoint gradient, checked against central finite differences of the FP64
log-likelihood and against the oracle's gradient."""
import numpy as np
import pytest

import oracle
from paper_2005_10123_amd import binding, synth

pytestmark = pytest.mark.gpu


def test_autograd_matches_blocking_and_fd():
    import torch

    from paper_2005_10123_amd.autograd import HawkesLogLik

    (x, y, t), th = synth.config_events("small_2k")
    ctx = binding.Context(0)
    ds = ctx.dataset(x, y, t)
    ref_ell, ref_g = oracle.evaluate(x, y, t, th)
    rows = oracle.evaluate(x, y, t, th, rows=True)
    l1 = np.abs(rows["row_grad"]).sum(axis=0)
    for prec, tol in (("fp64", 1e-10), ("fp32c", 1e-5)):
        theta = torch.tensor(th, dtype=torch.float64, requires_grad=True)
        ell = HawkesLogLik.apply(theta, ctx, ds, prec)
        (2.0 * ell).backward()
        ell_b, g_b = ctx.grad(ds, th, prec)
        assert ell.item() == ell_b
        assert np.array_equal(theta.grad.numpy(), 2.0 * g_b)
        assert abs(ell.item() - ref_ell) <= tol * abs(ref_ell)
        assert np.all(np.abs(theta.grad.numpy() / 2.0 - ref_g) <= tol * l1)
    # Central differences of the FP64 path (step 1e-6 relative).
    thv = np.array(th)
    _, g64 = ctx.grad(ds, thv, "fp64")
    for p in range(6):
        step = 1e-6 * thv[p]
        tp, tm = thv.copy(), thv.copy()
        tp[p] += step
        tm[p] -= step
        fd = (ctx.loglik(ds, tp, "fp64") - ctx.loglik(ds, tm, "fp64")) / (2 * step)
        assert abs(fd - g64[p]) <= 1e-6 * l1[p], (p, fd, g64[p])
    ds.close()
    ctx.close()


def test_autograd_on_side_stream():
    import torch

    from paper_2005_10123_amd.autograd import loglik

    (x, y, t), th = synth.config_events("small_2k", n=3000)
    ctx = binding.Context(0)
    ds = ctx.dataset(x, y, t)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        theta = torch.tensor(th, dtype=torch.float64, requires_grad=True)
        ell = loglik(theta, ctx, ds, "fp32c")
        ell.backward()
    torch.cuda.synchronize()
    e, g = ctx.grad(ds, th, "fp32c")
    assert ell.item() == e and np.array_equal(theta.grad.numpy(), g)
    ds.close()
    ctx.close()
