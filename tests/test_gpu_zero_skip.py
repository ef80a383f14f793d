"""Zero-tile skipping: on data spanning many multiples of tau_t and 1/omega most column tiles hold
only pairs whose background and trigger exponentials are exactly zero; leaving them out keeps the
same sum of the same non-zero terms, so the result matches the oracle as before and the unskipped
evaluation to the rounding of the regrouped partial sums."""
import time

import numpy as np
import pytest

import oracle
from gpu_util import TOL, assert_close, rel
from paper_2005_10123_amd import binding, synth

pytestmark = pytest.mark.gpu
THETA = synth.THETA_CFG1  # tau_t = 20 days, omega = 0.5 / day


@pytest.fixture(scope="module")
def ctx():
    c = binding.Context(0)
    yield c
    c.close()


def long_window(n, days, seed):
    return synth.simulate(synth.SimSpec(n, 10.0, days, 3, 0.5, 0.1, 0.3, (10123, 90, seed)))


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_skipping_matches_oracle_and_unskipped(ctx, prec):
    """6,000 events over 5,000 days: about 88 % (FP32C) and 48 % (FP64) of the pairs are skipped."""
    x, y, t = long_window(6000, 5000.0, 1)
    ref = oracle.evaluate(x, y, t, THETA, rows=True)
    ds = ctx.dataset(x, y, t)
    try:
        ell0, g0 = ctx.grad(ds, THETA, prec)
        rows0 = ctx.rows(ds, THETA, prec)
        ctx.set_zero_tile_skipping(True)
        ell1, g1 = ctx.grad(ds, THETA, prec)
        ll1 = ctx.loglik(ds, THETA, prec)
        rows1 = ctx.rows(ds, THETA, prec)
        sums_skip = ctx.shard_sums(ds, THETA, 0, 1, prec)
        ctx.set_zero_tile_skipping(False)
        sums = ctx.shard_sums(ds, THETA, 0, 1, prec)
    finally:
        ctx.set_zero_tile_skipping(False)
        ds.close()
    assert_close(ell1, g1, ref, prec, "zero-tile skipping", THETA)
    assert rel(ll1, ref["ell"]) <= TOL[prec]
    # Against the unskipped evaluation: only the grouping of the row partial sums differs
    # (binary64 partials for FP64, compensated binary32 partials for FP32C).
    tol = 1e-13 if prec == "fp64" else 1e-10
    assert rel(ell1, ell0) <= tol, (ell1, ell0)
    l1 = np.abs(ref["row_grad"]).sum(axis=0)
    assert np.all(np.abs(g1 - g0) <= tol * l1), (g1, g0)
    lam0, lam1 = rows0["lambda"], rows1["lambda"]
    assert np.max(np.abs(lam1 - lam0) / lam0) <= tol
    # The shard interface does not skip: identical with the setting on or off.
    assert np.array_equal(sums_skip, sums)


def test_nothing_to_skip(ctx):
    """Over 150 days no pair is 236 days apart: every tile is walked (in another order) and every
    term formed, so the result is the unskipped one up to the order of the row sums."""
    x, y, t = long_window(3000, 150.0, 2)
    ds = ctx.dataset(x, y, t)
    try:
        for prec in ("fp64", "fp32c"):
            ell0, g0 = ctx.grad(ds, THETA, prec)
            l1 = np.abs(ctx.rows(ds, THETA, prec)["grad"]).sum(axis=0)
            ctx.set_zero_tile_skipping(True)
            ell1, g1 = ctx.grad(ds, THETA, prec)
            ctx.set_zero_tile_skipping(False)
            tol = 1e-13 if prec == "fp64" else 1e-10
            assert rel(ell1, ell0) <= tol, (prec, ell1, ell0)
            assert np.all(np.abs(g1 - g0) <= tol * l1), (prec, g1, g0)
    finally:
        ctx.set_zero_tile_skipping(False)
        ds.close()


def test_served_requests_skip_and_match_blocking(ctx):
    """Requests submitted with skipping on run the same plan as the blocking call."""
    x, y, t = long_window(8000, 5000.0, 3)
    ds = ctx.dataset(x, y, t)
    rng = np.random.default_rng(5)
    thetas = [np.array(THETA) * np.exp(0.1 * rng.standard_normal(6)) for _ in range(6)]
    try:
        ctx.set_zero_tile_skipping(True)
        want = [ctx.grad(ds, th, "fp32c") for th in thetas]
        ctx.submit([binding.request(ds, th, "fp32c", True, k) for k, th in enumerate(thetas)])
        got = {}
        deadline = time.time() + 60
        while len(got) < len(thetas) and time.time() < deadline:
            for r in ctx.poll(cap=64, timeout_us=100000):
                assert r.status == 0
                got[r.tag] = (r.loglik, np.array(r.grad[:]))
        assert len(got) == len(thetas)
        for k, (ell, g) in enumerate(want):
            assert got[k][0] == ell and np.array_equal(got[k][1], g), k
    finally:
        ctx.set_zero_tile_skipping(False)
        ds.close()


def test_skipping_is_faster_on_long_windows(ctx):
    """40,000 events over 5,000 days: most FP32C tiles are skipped, the pass runs several times
    faster (timed with device events; the table kernel is included)."""
    x, y, t = long_window(40000, 5000.0, 4)
    ds = ctx.dataset(x, y, t)
    times = {}
    try:
        for skip in (False, True):
            ctx.set_zero_tile_skipping(skip)
            ctx.grad(ds, THETA, "fp32c")
            ctx.kernel_time(reset=True)
            ctx.profile(True)
            for _ in range(3):
                ctx.grad(ds, THETA, "fp32c")
            ms, k = ctx.kernel_time(reset=True)
            ctx.profile(False)
            times[skip] = ms / k
    finally:
        ctx.set_zero_tile_skipping(False)
        ds.close()
    print("pairwise pass ms without / with skipping:", times[False], times[True])
    assert times[True] <= 0.5 * times[False], times


def test_multi_with_skipping_matches_unskipped(ctx):
    """pi_n and ell for several parameter vectors per pass: a tile is left out only where the
    terms of every vector of the pass vanish."""
    x, y, t = long_window(6000, 5000.0, 5)
    rng = np.random.default_rng(6)
    th = np.array(THETA) * np.exp(0.1 * rng.standard_normal((6, 6)))
    ds = ctx.dataset(x, y, t)
    try:
        ll0, pi0 = ctx.loglik_multi(ds, th, "fp32c")
        ctx.set_zero_tile_skipping(True)
        ll1, pi1 = ctx.loglik_multi(ds, th, "fp32c")
    finally:
        ctx.set_zero_tile_skipping(False)
        ds.close()
    assert np.max(np.abs(ll1 - ll0) / np.abs(ll0)) <= 1e-10, (ll1, ll0)
    assert np.max(np.abs(pi1 - pi0)) <= 1e-9
    ref = oracle.evaluate(x, y, t, th[0], rows=True)
    assert rel(ll1[0], ref["ell"]) <= TOL["fp32c"]
    assert np.max(np.abs(pi1[0] - ref["row_pi"])) <= TOL["fp32c"]


def test_direct_enumeration_skips_outside_the_window(ctx):
    """The direct enumeration walks, per row block, only the tiles within the separation on either
    side: same result to rounding, matching the oracle, and a faster pass."""
    x, y, t = long_window(6000, 5000.0, 7)
    ref = oracle.evaluate(x, y, t, THETA, rows=True)
    ds = ctx.dataset(x, y, t)
    try:
        ctx.set_pair_scheme("direct")
        for prec in ("fp64", "fp32c"):
            ell0, g0 = ctx.grad(ds, THETA, prec)
            ctx.set_zero_tile_skipping(True)
            ell1, g1 = ctx.grad(ds, THETA, prec)
            ctx.set_zero_tile_skipping(False)
            assert_close(ell1, g1, ref, prec, "direct, zero-tile skipping", THETA)
            tol = 1e-13 if prec == "fp64" else 1e-10
            assert rel(ell1, ell0) <= tol, (prec, ell1, ell0)
            assert np.all(np.abs(g1 - g0) <= tol * np.abs(ref["row_grad"]).sum(axis=0)), (prec, g1, g0)
    finally:
        ctx.set_zero_tile_skipping(False)
        ctx.set_pair_scheme("symmetric")
        ds.close()
    x, y, t = long_window(40000, 5000.0, 9)
    ds = ctx.dataset(x, y, t)
    times = {}
    try:
        ctx.set_pair_scheme("direct")
        for skip in (False, True):
            ctx.set_zero_tile_skipping(skip)
            ctx.grad(ds, THETA, "fp32c")
            ctx.kernel_time(reset=True)
            ctx.profile(True)
            for _ in range(3):
                ctx.grad(ds, THETA, "fp32c")
            ms, k = ctx.kernel_time(reset=True)
            ctx.profile(False)
            times[skip] = ms / k
    finally:
        ctx.set_zero_tile_skipping(False)
        ctx.set_pair_scheme("symmetric")
        ds.close()
    print("direct pass ms without / with skipping:", times[False], times[True])
    assert times[True] <= 0.5 * times[False], times


def test_autograd_with_skipping_matches_blocking(ctx):
    """The device entry point behind torch.autograd runs the same skipping plan as the blocking call."""
    import torch

    from paper_2005_10123_amd.autograd import HawkesLogLik

    x, y, t = long_window(6000, 5000.0, 8)
    ds = ctx.dataset(x, y, t)
    try:
        ctx.set_zero_tile_skipping(True)
        for prec in ("fp64", "fp32c"):
            theta = torch.tensor(THETA, dtype=torch.float64, requires_grad=True)
            ell = HawkesLogLik.apply(theta, ctx, ds, prec)
            ell.backward()
            ell_b, g_b = ctx.grad(ds, THETA, prec)
            assert ell.item() == ell_b and np.array_equal(theta.grad.numpy(), g_b), prec
    finally:
        ctx.set_zero_tile_skipping(False)
        ds.close()
