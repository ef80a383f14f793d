"""One dataset over several devices, shown on one: the per-event sums of every shard of the
pairwise pass (hawkes_shard_sums) add up to the oracle's per-event sums, and hawkes_finish turns
them into the log-likelihood and gradient of the whole evaluation."""
import numpy as np
import pytest

import oracle
from gpu_util import TOL, assert_close, rel
from paper_2005_10123_amd import binding, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = binding.Context(0)
    yield c
    c.close()


def shard_total(ctx, ds, th, nshards, prec):
    total = np.zeros((ds.n, 6))
    for k in range(nshards):  # added in shard order, as an all-reduce in rank order would
        total += ctx.shard_sums(ds, th, k, nshards, prec)
    return total


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("nshards", [1, 2, 3, 8])
def test_shards_add_up_to_the_whole(ctx, prec, nshards):
    (x, y, t), th = synth.config_events("small_2k", n=5000)
    ds = ctx.dataset(x, y, t)
    try:
        sums = shard_total(ctx, ds, th, nshards, prec)
        ell, g = ctx.finish(ds, th, sums)
        ell_w, g_w = ctx.grad(ds, th, prec)
    finally:
        ds.close()
    ref = oracle.evaluate(x, y, t, th, rows=True)
    assert_close(ell, g, ref, prec, ("shards", nshards), th)
    # The same pair terms regrouped into other partial sums: agreement with the one-shot evaluation
    # to rounding of the regrouping (binary64 partials for FP64; compensated binary32 partials
    # merged at other boundaries for FP32C).
    tol = 1e-12 if prec == "fp64" else 1e-7
    assert rel(ell, ell_w) <= tol, (ell, ell_w)
    assert np.all(np.abs(g - g_w) <= tol * np.abs(ref["row_grad"]).sum(axis=0)), (g, g_w)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_shard_sums_match_the_oracle_per_event(ctx, prec):
    (x, y, t), th = synth.config_events("small_2k", n=3000)
    ds = ctx.dataset(x, y, t)
    try:
        sums = shard_total(ctx, ds, th, 4, prec)
    finally:
        ds.close()
    idx = np.arange(0, 3000, 7)
    ref = oracle.rows(x, y, t, th, idx)["sums"]
    # Background sums include the diagonal (>= 1); trigger sums may be 0 (no earlier event near).
    scale = np.maximum(np.abs(ref), np.abs(ref).max(axis=0) * 1e-12)
    err = (np.abs(sums[idx] - ref) / scale).max(axis=0)
    if prec == "fp64":
        assert err.max() <= 1e-11, err
    else:
        # Every sum, the moments (r^2, dt^2, dt times a term) included, to the FP32C tolerance:
        # pairs close in time take dt from the hi/lo parts of both events, so a close pair's dt
        # carries one binary32 rounding rather than the rounding of a time origin days away.
        print("per-event sums, max relative error", err)
        assert err.max() <= 1e-5, err


def test_more_shards_than_work(ctx):
    """300 events are one row block of four work units: most of 16 shards are empty."""
    (x, y, t), th = synth.config_events("small_2k", n=300)
    ds = ctx.dataset(x, y, t)
    try:
        parts = [ctx.shard_sums(ds, th, k, 16, "fp64") for k in range(16)]
        ell, g = ctx.finish(ds, th, sum(parts))
    finally:
        ds.close()
    assert sum(int(np.any(p != 0)) for p in parts) <= 5
    assert_close(ell, g, oracle.evaluate(x, y, t, th, rows=True), "fp64", "16 shards of 300 events", th)


def test_bad_shard_arguments(ctx):
    (x, y, t), th = synth.config_events("small_2k", n=100)
    ds = ctx.dataset(x, y, t)
    try:
        for k, m in [(-1, 2), (2, 2), (0, 0)]:
            with pytest.raises(binding.HawkesError):
                ctx.shard_sums(ds, th, k, m, "fp64")
    finally:
        ds.close()


def test_shards_ignore_the_context_scheme(ctx):
    """Shards always walk the symmetric enumeration, whatever the context's pair scheme."""
    (x, y, t), th = synth.config_events("small_2k", n=2500)
    ds = ctx.dataset(x, y, t)
    try:
        ref = shard_total(ctx, ds, th, 3, "fp64")
        ctx.set_pair_scheme("direct")
        try:
            got = shard_total(ctx, ds, th, 3, "fp64")
        finally:
            ctx.set_pair_scheme("symmetric")
    finally:
        ds.close()
    assert np.array_equal(got, ref)
